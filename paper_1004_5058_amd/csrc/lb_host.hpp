// Host-only logic of the library that touches no device: validation of the
// model parameters, the tuning cache's text format and the checks of a
// checkpoint header.  Plain C++ (no HIP): it is linked into liblbmi.so and,
// on its own, into a sanitizer harness that feeds it malformed inputs.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/lb.h"

namespace lbh {

// Bytes of one stored value of a storage format; 0 for an unknown format.
size_t storage_size(int storage);
// The tau = 1 moment form (six moments per site instead of 18 populations).
inline bool is_mom(int storage) { return storage >= LB_MOM32; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
// Row pitch (elements) and plane stride (elements) of a lattice's storage
// planes.  The pitch is nx rounded up to 64 elements (every wave's row access
// starts on a 256-byte boundary in FP32).  A plane starts one row and 64
// elements past the previous plane's end: planes a power of two apart
// (64 MiB for 4096^2 FP32) put the concurrent row streams of a step on few
// HBM channels, and the fused FP32 step ran 7-10 % slower at 4096^2.
inline size_t row_pitch(int nx) { return align_up((size_t)nx, 64); }
inline size_t plane_stride(int nx, int ny) { return row_pitch(nx) * ((size_t)ny + 1) + 64; }

// Number of row segments of the fused two-step kernel's tiles for a lattice
// of ny rows and tiles of at most ly2 rows (ly2 >= 1): ceil(ny / ly2) segments
// of near-equal height, one more while they would all be the same multiple of
// 16 rows.  Tiles whose first rows lie a power-of-two-rich number of row
// pitches apart put the rows the resident tiles touch in one tick on few HBM
// channels (128- and 192-row tiles measured up to 40 % slower at 4096^2).
// Always 1 <= result <= ny.
inline int fused_nseg(int ny, int ly2)
{
    const int lh = ly2 < ny ? (ly2 < 1 ? 1 : ly2) : ny;
    int n = (ny + lh - 1) / lh;
    while (n < ny && ny % n == 0 && (ny / n) % 16 == 0) ++n;
    return n;
}

// Checks one lattice's parameters (sizes, tau > 1/2, rho0 > 0, finite
// couplings and wall speeds, the moment form only at tau = 1, the 32-bit
// buffer offsets of one species' planes); storage0 >= 0 additionally requires
// that storage (all lattices of a batch share one).  LB_OK, or LB_EINVAL with
// the reason in *msg.
lb_status validate(const lb_params* p, int storage0, std::string* msg);

// One lattice's initial fields, checked.
struct FieldCheck {
    int what = 0;             // 0: valid; 1: a density not finite and > 0; 2: a non-finite u_x; 3: a non-finite u_y
    size_t site = 0;          // the first offending site (row-major), where what != 0
    double sum[2] = {0, 0};   // sums of rho_A and of rho_B over the sites, in site order
};
// Checks the initial fields of n lattices (ns[k] sites each; ux, uy and any of
// their entries may be null) and sums each lattice's densities in site order,
// one sequential pass per lattice that stops at its first offending site (at a
// site: the densities, then u_x, then u_y).  The lattices are spread over up
// to `threads` host threads (<= 0: the hardware's, at most 16), the largest
// first; the results do not depend on the thread count.
void check_fields(int n, const size_t* ns, const double* const* ra, const double* const* rb,
                  const double* const* ux, const double* const* uy, FieldCheck* out, int threads);

// One autotuner result.
struct TuneEntry {
    int bx = 0, ly = 0, grid = 0;
    int fusion = 1, ly2 = 0;   // time steps per pass and fused tile height (0: automatic)
    int fw = 0;                // fused kernel's lanes per step: 128, 192, 256 (0: automatic)
    double ms = 0;
};
using TuneCache = std::vector<std::pair<std::string, TuneEntry>>;

// Parses the cache text: one entry per line,
//   "key": {"bx": 512, "ly": 128, "grid": 0, "fusion": 2, "ly2": 0, "fw": 128, "ms": 0.35},
// Lines that are not of that form, keys with a quote or control character,
// and entries whose numbers are missing, malformed or out of range (bx not in
// {64, 128, 256, 512}, negative ly / grid / ly2, fusion not 1 or 2, fw not in
// {0, 128, 192, 256}, ms not finite) are skipped; an entry without "fusion"
// runs one step per pass, one without "fw" the automatic fused width.
TuneCache parse_cache(const char* text, size_t len);
// Reads and parses a cache file (missing or unreadable: empty).
TuneCache read_cache(const char* path);
// The text parse_cache reads back.
std::string format_cache(const TuneCache& ents);

// Checkpoint: this header, then the population buffer in its storage
// format, then the FP64 stress and profile accumulators.
struct CkptHeader {
    char magic[8];
    int32_t version, storage, nx, ny, pitch, profile;
    int64_t t, nsamples;
    uint64_t fbytes, sbytes, pbytes;
};
constexpr int32_t CKPT_VERSION = 2;   // 2: planes stored shifted in x by c_ix
// The header of a checkpoint of a lattice with these properties and section sizes.
CkptHeader make_header(int storage, int nx, int ny, int pitch, int profile, int64_t t, int64_t nsamples,
                       uint64_t fbytes, uint64_t sbytes, uint64_t pbytes);
// Whether buf (bytes long) is a complete checkpoint of the lattice `want`
// describes (same magic, version, storage, shape, profile setting and section
// sizes, and long enough for all sections); on success *out is its header.
// LB_EINVAL (buffer too short) or LB_ESTATE (another lattice), reason in *msg.
lb_status check_checkpoint(const void* buf, size_t bytes, const CkptHeader& want, CkptHeader* out,
                           std::string* msg);

}  // namespace lbh
