// Host runtime and C ABI (include/lb.h) of the multirange lattice Boltzmann
// library: parameter validation, the layout of the caller's device state,
// work decomposition, HIP-graph replay of the step kernel, reductions and
// checkpoints.  No compute happens on the host; every array operation is a
// kernel in lb_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <queue>
#include <vector>

#include "../../include/lb.h"
#include "lb_device.hpp"
#include "lb_host.hpp"
#include "lb_kernels.hpp"

namespace {

thread_local std::string g_err;

lb_status fail(lb_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(LB_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));         \
    } while (0)

constexpr size_t ALIGN = 256;

// Owners that release a HIP event pair or a temporary device buffer on every
// return path (HIP_TRY returns early).
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};
struct TempDeviceBuffer {
    char* p = nullptr;
    ~TempDeviceBuffer()
    {
        if (p) (void)hipFree(p);
    }
};


using lbh::align_up;
using lbh::is_mom;
using lbh::storage_size;

// Bytes per site of FP64 staging a state buffer must hold (four arrays).
constexpr size_t STAGE_BYTES_PER_SITE = 4 * sizeof(double);

// Values stored per site: 18 populations, or the 6 moments of the tau = 1 form.
size_t planes_of(int storage) { return storage >= LB_MOM32 ? 6 : 18; }
// Storages with a fused two-steps-per-pass kernel: FP32 and the 16-bit forms.
bool fusion_storage(int storage) { return storage == LB_F32 || storage == LB_F16DEV || storage == LB_BF16DEV; }

// Two-belt weights on |c|^2 = 1, 2, 4, 5, 8 and D2Q9 belt-1 weights.
const double P12[5] = {4.0 / 63.0, 4.0 / 135.0, 1.0 / 180.0, 2.0 / 945.0, 1.0 / 15120.0};
const double W1[2] = {1.0 / 9.0, 1.0 / 36.0};
const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

lb_status validate(const lb_params* p, int storage0)
{
    std::string msg;
    const lb_status st = lbh::validate(p, storage0, &msg);
    if (st != LB_OK) return fail(st, "%s", msg.c_str());
    return LB_OK;
}

struct Lat {
    lb_params p;
    int pitch = 0, ngroups = 0, ngroups2 = 0;   // profile partial rows: single-step, fused
    long long plane = 0;
    size_t off_f[2] = {0, 0}, off_stress = 0, off_prof = 0, off_body = 0, end = 0;
    double rho_ref[2] = {0, 0};
};

// FP64 entries of a lattice's profile accumulators (when enabled).
size_t prof_entries(const Lat& a) { return (size_t)(a.ngroups + a.ngroups2) * (size_t)a.p.ny; }

// Layout: [descs][partials][results][item table] then per lattice
// [f0][f1][stress][prof][body force per row].
struct Layout {
    size_t off_desc = 0, off_part = 0, off_res = 0, off_tiles = 0, off_tiles2 = 0, total = 0;
    int max_items = 0;   // capacity of the item -> lattice table (any launch shape)
    int max_items2 = 0;  // the same for the fused two-step kernel's tiles
};

Layout plan(std::vector<Lat>& lats)
{
    Layout L;
    const int n = (int)lats.size();
    L.off_desc = 0;
    L.off_part = align_up(sizeof(lbk::LatDesc) * n, ALIGN);
    L.off_res = L.off_part + align_up(sizeof(double) * 5 * lbk::sums_blocks(), ALIGN);
    // results: 5 sums + flag slot + 2 per lattice stress + profile staging handled in f buffers
    // Item -> lattice table: at most ceil(nx/60) * ny items per lattice (the
    // narrowest tile collides 60 columns: 64 lanes of the moment form, whose
    // tiles overlap by four; one row per segment) plus 7 alignment slots each.
    long long items = 0;
    for (const auto& a : lats) items += (long long)((a.p.nx + 59) / 60) * a.p.ny + 7;
    L.max_items = (int)std::min<long long>(items, INT32_MAX);
    // Fused two-step tiles: strips of at least the narrowest width's output
    // columns, at most one row per segment.
    long long items2 = 0;
    for (const auto& a : lats) {
        const int tw = lbk::fuse2_tw(a.p.storage, lbk::FUSE2_NW_MIN);
        items2 += (long long)((a.p.nx + tw - 1) / tw) * a.p.ny + 7;
    }
    L.max_items2 = (int)std::min<long long>(items2, INT32_MAX);
    L.off_tiles = L.off_res + align_up(sizeof(double) * (8 + 2 * n), ALIGN);
    L.off_tiles2 = L.off_tiles + align_up(sizeof(int32_t) * (size_t)L.max_items, ALIGN);
    size_t off = L.off_tiles2 + align_up(sizeof(int32_t) * (size_t)L.max_items2, ALIGN);
    for (auto& a : lats) {
        const size_t es = storage_size(a.p.storage);
        a.pitch = (int)lbh::row_pitch(a.p.nx);
        a.plane = (long long)lbh::plane_stride(a.p.nx, a.p.ny);
        // profile accumulator rows: one per 64 columns, or for the moment form
        // one per tile of the narrowest launch shape (60 collided columns)
        a.ngroups = is_mom(a.p.storage) ? (a.p.nx + 59) / 60 : (a.p.nx + 63) / 64;
        // and, for the storages with a fused two-step kernel, its partials:
        // two steps x strips x waves per step, for the widest of its layouts
        a.ngroups2 = 0;
        if (fusion_storage(a.p.storage))
            for (int nw = lbk::FUSE2_NW_MIN; nw <= lbk::FUSE2_NW_MAX; ++nw) {
                const int tw = lbk::fuse2_tw(a.p.storage, nw);
                a.ngroups2 = std::max(a.ngroups2, 2 * nw * ((a.p.nx + tw - 1) / tw));
            }
        // Each state buffer also serves as staging for four FP64 arrays of
        // nx*ny values (initial fields, field reads): at least 32 bytes per
        // site, whatever the storage needs (6 FP32 moments need only 24).
        const size_t per_site = std::max<size_t>(planes_of(a.p.storage) * es, STAGE_BYTES_PER_SITE);
        const size_t fbytes = align_up(per_site * a.plane, ALIGN);
        a.off_f[0] = off;
        a.off_f[1] = off + fbytes;
        a.off_stress = off + 2 * fbytes;
        a.off_prof = a.off_stress + align_up(sizeof(double) * 2 * a.p.nx, ALIGN);
        const size_t pbytes = a.p.profile ? align_up(sizeof(double) * prof_entries(a), ALIGN) : 0;
        a.off_body = a.off_prof + pbytes;
        const size_t bbytes = a.p.fx_amp != 0.0 ? align_up(sizeof(double) * (size_t)a.p.ny, ALIGN) : 0;
        a.end = a.off_body + bbytes;
        off = a.end;
    }
    L.total = off;
    return L;
}

void fill_desc(const Lat& a, lbk::LatDesc& d)
{
    std::memset(&d, 0, sizeof d);
    const lb_params& p = a.p;
    d.off_f[0] = (long long)a.off_f[0];
    d.off_f[1] = (long long)a.off_f[1];
    d.off_stress = (long long)a.off_stress;
    d.off_prof = p.profile ? (long long)a.off_prof : -1;
    d.off_body = p.fx_amp != 0.0 ? (long long)a.off_body : -1;
    d.plane = a.plane;
    d.nx = p.nx;
    d.ny = p.ny;
    d.pitch = a.pitch;
    d.walls = p.walls_y;
    d.ngroups = a.ngroups;
    d.ngroups2 = a.ngroups2;
    d.tau = p.tau;
    d.omega = 1.0 / p.tau;
    d.rho0 = p.rho0;
    d.inv_rho0 = 1.0 / p.rho0;
    const double ga[2] = {p.g_aa1, p.g_bb1}, gr[2] = {p.g_aa2, p.g_bb2};
    for (int s = 0; s < 2; ++s) {
        d.ks[s][0] = ga[s] * W1[0] + gr[s] * P12[0];
        d.ks[s][1] = ga[s] * W1[1] + gr[s] * P12[1];
        for (int k = 2; k < 5; ++k) d.ks[s][k] = gr[s] * P12[k];
    }
    d.kx[0] = p.g_ab / p.rho0 * W1[0];
    d.kx[1] = p.g_ab / p.rho0 * W1[1];
    d.u_top = p.u_top;
    d.u_bot = p.u_bot;
    for (int s = 0; s < 2; ++s) {
        for (int i = 0; i < 9; ++i) d.wref[9 * s + i] = W9[i] * a.rho_ref[s];
        d.rref[s] = a.rho_ref[s];
        d.psiref[s] = -p.rho0 * std::expm1(-a.rho_ref[s] / p.rho0);
        d.epsi[s] = p.rho0 * std::exp(-a.rho_ref[s] / p.rho0);
        d.frref[s] = (float)d.rref[s];
        d.fpsiref[s] = (float)d.psiref[s];
        d.fepsi[s] = (float)d.epsi[s];
    }
    d.ftau = (float)d.tau;
    d.fomega = (float)d.omega;
    d.frho0 = (float)d.rho0;
    d.finv_rho0 = (float)d.inv_rho0;
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < 5; ++k) d.fks[s][k] = (float)d.ks[s][k];
    d.fkx[0] = (float)d.kx[0];
    d.fkx[1] = (float)d.kx[1];
    d.fu_top = (float)d.u_top;
    d.fu_bot = (float)d.u_bot;
}

}  // namespace

// Shared with the surrogate network's C ABI: sets lb_last_error()'s message.
void lbi_set_error(const char* msg) { g_err = msg; }

// ---------------------------------------------------------------- the batch --

struct lbb_handle {
    std::vector<Lat> lats;
    std::vector<lbk::LatDesc> descs;
    Layout lay;
    int storage = 1;
    char* base = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;   // private stream used only to record graphs
    int cur = 0;                     // buffer holding f(t)
    int64_t t = 0, nsamples = 0;
    int bx = 256, ly = 64, grid = 0; // grid 0: one block per tile
    int ntot = 0;
    int ly_max = 1;                  // largest rows-per-tile over the lattices
    int graph_steps = 32;
    int fusion = 1;                  // time steps per step-kernel pass: 1, or 2 (k_step2)
    int ly2 = 0;                     // rows per fused tile as set (0: automatic)
    int ly2_eff = 0;                 // rows per fused tile in effect (the automatic choice resolved)
    int fnw = 0;                     // waves per step of the fused kernel as set (0: automatic)
    int fnw_eff = 2;                 // the same in effect
    int ntot2 = 0;
    hipGraphExec_t exec[2] = {nullptr, nullptr};   // graph starting from buffer 0 / 1
    int watchdog = 0;
    int flag_host = 0;
    double* d_part() { return (double*)(base + lay.off_part); }
    double* d_res() { return (double*)(base + lay.off_res); }
    int* d_flag() { return (int*)(base + lay.off_res + 6 * sizeof(double)); }
    lbk::LatDesc* d_desc() { return (lbk::LatDesc*)(base + lay.off_desc); }
    int32_t* d_tiles() { return (int32_t*)(base + lay.off_tiles); }
    int32_t* d_tiles2() { return (int32_t*)(base + lay.off_tiles2); }
    std::vector<int32_t> tiles;      // host copy of the item -> lattice table
    std::vector<int32_t> tiles2;     // the same for the fused two-step tiles
};

struct lb_handle {
    lbb_handle b;
};

// The state is still the initial one (moment storage: not yet a streamed state).
int first_state(const lbb_handle* h) { return (is_mom(h->storage) && h->t == 0) ? 1 : 0; }

namespace {

void drop_graphs(lbb_handle* h)
{
    for (auto& e : h->exec)
        if (e) { (void)hipGraphExecDestroy(e); e = nullptr; }
}

// Rows of the tallest fused segment of a lattice of ny rows at tile height ly2.
int fused_height(int ny, int ly2)
{
    const int n = lbh::fused_nseg(ny, ly2);
    return (ny + n - 1) / n;
}

// Order in which the lattices' fused tiles are handed out: by segment height,
// tallest first (stable), so the short tiles of shallow lattices fill the end
// of the schedule (longest processing time first; every tile of a lattice has
// the same height to a row).
std::vector<int> fused_order(const lbb_handle* h, int ly2)
{
    std::vector<int> ord(h->lats.size());
    for (size_t k = 0; k < ord.size(); ++k) ord[k] = (int)k;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        return fused_height(h->lats[a].p.ny, ly2) > fused_height(h->lats[b].p.ny, ly2);
    });
    return ord;
}

// Makespan, in ticks, of the fused tiles of height at most ly2 (each lattice's
// rows split into fused_nseg near-equal segments, as the kernel does), handed
// out in fused_order and scheduled greedily on `slots` concurrent blocks; a
// tile of h rows costs h + 8 ticks (the overlap rows of the two steps).
long long fused_makespan(const lbb_handle* h, int ly2, int slots)
{
    std::priority_queue<long long, std::vector<long long>, std::greater<long long>> free_at;
    for (int c = 0; c < slots; ++c) free_at.push(0);
    long long end = 0;
    const int tw = lbk::fuse2_tw(h->storage, h->fnw_eff);
    for (int k : fused_order(h, ly2)) {
        const Lat& a = h->lats[k];
        const int strips = (a.p.nx + tw - 1) / tw;
        const int nseg = lbh::fused_nseg(a.p.ny, ly2), sb = a.p.ny / nseg, sx = a.p.ny - sb * nseg;
        for (int st = 0; st < strips; ++st)
            for (int g = 0; g < nseg; ++g) {
                const long long t = free_at.top() + sb + (g < sx ? 1 : 0) + 8;
                free_at.pop();
                free_at.push(t);
                end = std::max(end, t);
            }
    }
    return end;
}

int device_cus()
{
    int dev = 0, ncu = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        ncu = prop.multiProcessorCount;
    return ncu;
}

// Fused tile heights tried by the automatic choice and the tuner: odd
// multiples of 4.  Segments of a power-of-two number of rows put the rows the
// resident tiles touch in each tick a power-of-two number of row pitches
// apart, and such heights measured up to 40 % slower at 4096^2 (128 or 192
// rows of FP32, 128 of FP16), the signature of accesses piling onto a few
// HBM channels.
const int FUSED_HEIGHTS[] = {20, 28, 36, 44, 52, 60, 68, 76, 84, 92, 100, 108, 124, 140, 156, 172, 204, 252, 300,
                             380, 508};

// Automatic fused tile height: the height with the smallest makespan (ties:
// the taller tiles, fewer of them) on the blocks the device runs at once.
// Candidates: every height up to 64 rows, then heights about 1.5 % apart up to
// the tallest lattice, among those whose tiles fill at most 16 rounds of the
// device's blocks (more rounds leave a negligible tail; the tallest candidate
// is always kept).
int auto_ly2(const lbb_handle* h)
{
    int maxny = 1;
    const int slots = device_cus() * std::max(1, lbk::step2_blocks_per_cu(h->storage, h->fnw_eff));
    const int tw = lbk::fuse2_tw(h->storage, h->fnw_eff);
    for (const Lat& a : h->lats) maxny = std::max(maxny, a.p.ny);
    int best = maxny;
    long long best_t = -1;
    for (int c = maxny; c >= 1; c -= (c > 64 ? std::max(1, c / 64) : 1)) {
        long long tiles = 0;
        for (const Lat& a : h->lats)
            tiles += (long long)((a.p.nx + tw - 1) / tw) * lbh::fused_nseg(a.p.ny, c);
        if (c < maxny && tiles > 16LL * slots) break;   // shorter heights only add tiles
        const long long t = fused_makespan(h, c, slots);
        if (best_t < 0 || t < best_t) { best_t = t; best = c; }
    }
    return best;
}

// Automatic waves per step of the fused kernel: the most waves the device
// keeps on one compute unit (blocks per CU x waves per block); ties go to the
// wider tiles (less overlap).  Only blocks whose waves spread evenly over a
// CU's four SIMDs (4 or 8 waves) are candidates: six-wave blocks leave two
// SIMDs with one step's waves only and measured 20-35 % slower.  2 where no
// fused kernel exists for the storage.
int auto_fnw(const lbb_handle* h)
{
    int best = 2, best_w = -1;
    if (!fusion_storage(h->storage)) return best;
    for (int nw : {2, 4}) {
        const int w = lbk::step2_blocks_per_cu(h->storage, nw) * 2 * nw;
        if (w >= best_w) { best_w = w; best = nw; }
    }
    return best;
}

// Work decomposition for launch shape (bx, ly): tiles per lattice, each
// lattice's first item rounded up to a multiple of 8 (one tile per XCD slot),
// and the item -> lattice table the step kernel reads (-1: padding).
lb_status decompose(lbb_handle* h)
{
    int item = 0;
    h->ly_max = 1;
    h->tiles.clear();
    for (size_t k = 0; k < h->lats.size(); ++k) {
        const Lat& a = h->lats[k];
        lbk::LatDesc& d = h->descs[k];
        // the moment form's tiles overlap by four columns: bx - 4 collided per tile
        const int wt = is_mom(h->storage) ? h->bx - 4 : h->bx;
        d.nstrip = (a.p.nx + wt - 1) / wt;
        d.ly = std::min(std::min(h->ly, a.p.ny), 256);   // the kernel's halo buffer holds 256 rows
        d.nseg = (a.p.ny + d.ly - 1) / d.ly;
        h->ly_max = std::max(h->ly_max, d.ly);
        d.nitems = d.nstrip * d.nseg;
        item = (item + 7) / 8 * 8;
        d.item_begin = item;
        item += (d.nitems + 7) / 8 * 8;   // padding items keep the XCD-banded order (xcd_tile)
        h->tiles.resize(d.item_begin, -1);
        h->tiles.resize(item, (int32_t)k);
    }
    if (item > h->lay.max_items) return fail(LB_EINVAL, "launch shape gives more work items than planned");
    h->ntot = item;
    // Fused two-step tiles: fuse2_tw columns x ly2 rows.  ly2 = 0 picks the height
    // whose tiles, handed to the compute units in table order (each takes the
    // next tile when it finishes one), finish first; a tile of h rows costs
    // h + 8 ticks (the overlap rows of the two steps), whatever its width.
    h->fnw_eff = h->fnw > 0 ? h->fnw : auto_fnw(h);
    int ly2 = h->ly2;
    if (ly2 <= 0) ly2 = auto_ly2(h);
    h->ly2_eff = ly2;
    const int tw = lbk::fuse2_tw(h->storage, h->fnw_eff);
    int item2 = 0;
    h->tiles2.clear();
    for (int k : fused_order(h, ly2)) {
        const Lat& a = h->lats[k];
        lbk::LatDesc& d = h->descs[k];
        d.nstrip2 = (a.p.nx + tw - 1) / tw;
        d.nseg2 = lbh::fused_nseg(a.p.ny, ly2);
        d.ly2 = (a.p.ny + d.nseg2 - 1) / d.nseg2;   // the tallest segment
        d.nitems2 = d.nstrip2 * d.nseg2;
        item2 = (item2 + 7) / 8 * 8;
        d.item_begin2 = item2;
        item2 += (d.nitems2 + 7) / 8 * 8;
        h->tiles2.resize(d.item_begin2, -1);
        h->tiles2.resize(item2, (int32_t)k);
    }
    if (item2 > h->lay.max_items2) return fail(LB_EINVAL, "fused tile height gives more work items than planned");
    h->ntot2 = item2;
    HIP_TRY(hipMemcpyAsync(h->d_desc(), h->descs.data(), sizeof(lbk::LatDesc) * h->descs.size(),
                           hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->d_tiles(), h->tiles.data(), sizeof(int32_t) * h->tiles.size(),
                           hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->d_tiles2(), h->tiles2.data(), sizeof(int32_t) * h->tiles2.size(),
                           hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    return LB_OK;
}

int launch_grid(const lbb_handle* h)
{
    if (h->grid > 0) return h->grid;
    return std::max(1, h->ntot);
}

lb_status launch_one(lbb_handle* h, hipStream_t s, int src, int first = 0)
{
    hipError_t e = lbk::launch_step(h->storage, h->bx, h->base, h->d_desc(), h->d_tiles(),
                                    h->ntot, src, first, launch_grid(h), h->ly_max, s);
    if (e != hipSuccess) return fail(LB_EDEVICE, "step launch failed: %s", hipGetErrorString(e));
    return LB_OK;
}

// Steps t and t+1 in one launch: reads buffer src, writes buffer src ^ 1.
lb_status launch_two(lbb_handle* h, hipStream_t s, int src)
{
    hipError_t e = lbk::launch_step2(h->storage, h->fnw_eff, h->base, h->d_desc(), h->d_tiles2(), h->ntot2, src,
                                     std::max(1, h->ntot2), s);
    if (e != hipSuccess) return fail(LB_EDEVICE, "fused step launch failed: %s", hipGetErrorString(e));
    return LB_OK;
}

lb_status build_graph(lbb_handle* h, int start)
{
    if (!h->capture) HIP_TRY(hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal));
    lb_status st = LB_OK;
    int src = start;
    if (h->fusion == 2) {
        for (int k = 0; k < h->graph_steps / 2 && st == LB_OK; ++k) {
            st = launch_two(h, h->capture, src);
            src ^= 1;
        }
    } else {
        for (int k = 0; k < h->graph_steps && st == LB_OK; ++k) {
            st = launch_one(h, h->capture, src);
            src ^= 1;
        }
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->capture, &g);
    if (st != LB_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return fail(LB_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&h->exec[start], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LB_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    return LB_OK;
}

lb_status run_sums(lbb_handle* h, int k, int* flag)
{
    const Lat& a = h->lats[k];
    (void)a;
    hipError_t e = lbk::launch_sums(h->storage, h->base, h->d_desc() + k, h->cur, first_state(h), lbk::sums_blocks(),
                                    h->d_part(), h->d_res(), flag, h->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "sums launch failed: %s", hipGetErrorString(e));
    return LB_OK;
}

lb_status steps(lbb_handle* h, int32_t n)
{
    if (n < 0) return fail(LB_EINVAL, "negative step count");
    if (n > 0 && first_state(h)) {
        // the moment form's first step reads the initial local equilibria in
        // place; it is launched on its own, never inside a graph
        lb_status st = launch_one(h, h->stream, h->cur, 1);
        if (st != LB_OK) return st;
        h->cur ^= 1;
        h->t += 1;
        h->nsamples += 1;
        n -= 1;
        if (h->watchdog > 0 && h->t % h->watchdog == 0)
            for (size_t k = 0; k < h->lats.size(); ++k) {
                st = run_sums(h, (int)k, h->d_flag());
                if (st != LB_OK) return st;
            }
    }
    while (n > 0) {
        int chunk = n;
        if (h->watchdog > 0) {
            const int64_t to_next = h->watchdog - (h->t % h->watchdog);
            chunk = (int)std::min<int64_t>(chunk, to_next);
        }
        if (h->graph_steps > 0 && chunk >= h->graph_steps) {
            const int reps = chunk / h->graph_steps;
            if (!h->exec[h->cur]) {
                lb_status st = build_graph(h, h->cur);
                if (st != LB_OK) return st;
            }
            for (int r = 0; r < reps; ++r) {
                HIP_TRY(hipGraphLaunch(h->exec[h->cur], h->stream));
                // graph_steps is even: single steps leave the buffer parity
                // unchanged, fused pairs flip it once per pair
                if (h->fusion == 2 && ((h->graph_steps / 2) & 1)) {
                    h->cur ^= 1;
                    if (r + 1 < reps && !h->exec[h->cur]) {
                        lb_status st = build_graph(h, h->cur);
                        if (st != LB_OK) return st;
                    }
                }
            }
            const int done = reps * h->graph_steps;
            h->t += done;
            h->nsamples += done;
            n -= done;
            chunk -= done;
        }
        if (h->fusion == 2) {
            for (; chunk >= 2; chunk -= 2, n -= 2) {
                lb_status st = launch_two(h, h->stream, h->cur);
                if (st != LB_OK) return st;
                h->cur ^= 1;
                h->t += 2;
                h->nsamples += 2;
            }
        }
        for (int k = 0; k < chunk; ++k) {
            lb_status st = launch_one(h, h->stream, h->cur);
            if (st != LB_OK) return st;
            h->cur ^= 1;
            h->t += 1;
            h->nsamples += 1;
        }
        n -= chunk;
        if (h->watchdog > 0 && h->t % h->watchdog == 0)
            for (size_t k = 0; k < h->lats.size(); ++k) {
                lb_status st = run_sums(h, (int)k, h->d_flag());
                if (st != LB_OK) return st;
            }
    }
    return LB_OK;
}

lb_status check_flag(lbb_handle* h)
{
    int f = 0;
    HIP_TRY(hipMemcpyAsync(&f, h->d_flag(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (f) return fail(LB_ENONFINITE, "watchdog: non-finite or non-positive density in the lattice");
    return LB_OK;
}

lb_status reset_acc(lbb_handle* h)
{
    for (const Lat& a : h->lats) {
        HIP_TRY(lbk::launch_fill((double*)(h->base + a.off_stress), 2ll * a.p.nx, 0.0, h->stream));
        if (a.p.profile)
            HIP_TRY(lbk::launch_fill((double*)(h->base + a.off_prof), (long long)prof_entries(a), 0.0,
                                     h->stream));
    }
    h->nsamples = 0;
    return LB_OK;
}

void default_shape(lbb_handle* h);

lb_status batch_init(const lb_params* params, int32_t n, void* dev_state, size_t bytes, void* stream,
                     const double* const* ra, const double* const* rb, const double* const* ux,
                     const double* const* uy, lbb_handle** out)
{
    if (!out) return fail(LB_EINVAL, "null output handle");
    *out = nullptr;
    if (n < 1 || !params) return fail(LB_EINVAL, "need at least one lattice");
    if (!dev_state) return fail(LB_EINVAL, "null device state");
    if (((uintptr_t)dev_state) % ALIGN) return fail(LB_EINVAL, "device state must be 256-byte aligned");
    if (!ra || !rb) return fail(LB_EINVAL, "null initial density arrays");
    std::vector<Lat> lats(n);
    std::vector<size_t> nsites(n);
    for (int k = 0; k < n; ++k) {
        lb_status st = validate(&params[k], params[0].storage);
        if (st != LB_OK) return st;
        lats[k].p = params[k];
        if (!ra[k] || !rb[k]) return fail(LB_EINVAL, "null initial density of lattice %d", k);
        nsites[k] = (size_t)params[k].nx * params[k].ny;
    }
    // the fields of all lattices checked and summed on the host threads (each
    // lattice's sums in site order, whatever the thread count)
    std::vector<lbh::FieldCheck> chk(n);
    lbh::check_fields(n, nsites.data(), ra, rb, ux, uy, chk.data(), 0);
    for (int k = 0; k < n; ++k) {
        const lbh::FieldCheck& c = chk[k];
        if (c.what == 1)
            return fail(LB_EINVAL, "lattice %d: initial density must be finite and > 0 (site %zu)", k, c.site);
        if (c.what == 2) return fail(LB_EINVAL, "lattice %d: non-finite initial ux (site %zu)", k, c.site);
        if (c.what == 3) return fail(LB_EINVAL, "lattice %d: non-finite initial uy (site %zu)", k, c.site);
        const double ns = (double)nsites[k];
        lats[k].rho_ref[0] = params[k].rho_ref_a > 0 ? params[k].rho_ref_a : c.sum[0] / ns;
        lats[k].rho_ref[1] = params[k].rho_ref_b > 0 ? params[k].rho_ref_b : c.sum[1] / ns;
    }
    Layout lay = plan(lats);
    if (bytes < lay.total)
        return fail(LB_ENOMEM, "device state of %zu bytes is smaller than the %zu required", bytes, lay.total);

    lbb_handle* h = new (std::nothrow) lbb_handle();
    if (!h) return fail(LB_ENOMEM, "host allocation failed");
    h->lats = lats;
    h->lay = lay;
    h->storage = params[0].storage;
    h->base = (char*)dev_state;
    h->bytes = bytes;
    h->stream = (hipStream_t)stream;
    h->descs.resize(n);
    for (int k = 0; k < n; ++k) fill_desc(lats[k], h->descs[k]);
    default_shape(h);
    lb_status st = decompose(h);
    if (st != LB_OK) { delete h; return st; }

    // Stage each lattice's initial fields in its second population buffer
    // (at least 32 bytes per site in every storage format), then write f(0).
    for (int k = 0; k < n; ++k) {
        const Lat& a = h->lats[k];
        const size_t ns = (size_t)a.p.nx * a.p.ny;
        if (ns * STAGE_BYTES_PER_SITE > a.off_f[1] - a.off_f[0]) {
            delete h;
            return fail(LB_EINVAL, "internal: staging does not fit the state buffer");
        }
        double* stg = (double*)(h->base + a.off_f[1]);
        const double* src[4] = {ra[k], rb[k], ux ? ux[k] : nullptr, uy ? uy[k] : nullptr};
        double* dst[4] = {nullptr, nullptr, nullptr, nullptr};
        for (int m = 0; m < 4; ++m)
            if (src[m]) {
                dst[m] = stg + m * ns;
                hipError_t e = hipMemcpyAsync(dst[m], src[m], ns * sizeof(double), hipMemcpyHostToDevice, h->stream);
                if (e != hipSuccess) { delete h; return fail(LB_EDEVICE, "upload failed: %s", hipGetErrorString(e)); }
            }
        hipError_t e = lbk::launch_init(h->storage, h->base, h->d_desc() + k, (long long)ns, 0, dst[0], dst[1],
                                        dst[2], dst[3], h->stream);
        if (e != hipSuccess) { delete h; return fail(LB_EDEVICE, "init launch failed: %s", hipGetErrorString(e)); }
    }
    // body force of each row, F_x(y) = fx_amp sin(fx_k y), evaluated in FP64 on the host
    std::vector<std::vector<double>> body(n);
    for (int k = 0; k < n; ++k) {
        const Lat& a = h->lats[k];
        if (a.p.fx_amp == 0.0) continue;
        body[k].resize(a.p.ny);
        for (int y = 0; y < a.p.ny; ++y) body[k][y] = a.p.fx_amp * std::sin(a.p.fx_k * (double)y);
        hipError_t e = hipMemcpyAsync(h->base + a.off_body, body[k].data(), sizeof(double) * a.p.ny,
                                      hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) { delete h; return fail(LB_EDEVICE, "upload failed: %s", hipGetErrorString(e)); }
    }
    hipError_t ef = lbk::launch_fill((double*)(h->base + lay.off_res), 8 + 2 * n, 0.0, h->stream);
    if (ef != hipSuccess) { delete h; return fail(LB_EDEVICE, "fill launch failed: %s", hipGetErrorString(ef)); }
    st = reset_acc(h);
    if (st != LB_OK) { delete h; return st; }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) { delete h; return fail(LB_EDEVICE, "init failed: %s", hipGetErrorString(e)); }
    *out = h;
    return LB_OK;
}

lb_status lattice_fields(lbb_handle* h, int k, double* ra, double* rb, double* ux, double* uy, bool host)
{
    if (k < 0 || k >= (int)h->lats.size()) return fail(LB_EINVAL, "lattice index out of range");
    const Lat& a = h->lats[k];
    const size_t ns = (size_t)a.p.nx * a.p.ny;
    if (!host) {
        HIP_TRY(lbk::launch_fields(h->storage, h->base, h->d_desc() + k, (long long)ns, h->cur, first_state(h), ra,
                                   rb, ux, uy, h->stream));
        return LB_OK;
    }
    // compute into the idle state buffer, then copy out
    if (ns * STAGE_BYTES_PER_SITE > a.off_f[1] - a.off_f[0])
        return fail(LB_EINVAL, "internal: staging does not fit the state buffer");
    double* stg = (double*)(h->base + a.off_f[h->cur ^ 1]);
    double* outs[4] = {ra, rb, ux, uy};
    double* dev[4];
    for (int m = 0; m < 4; ++m) dev[m] = outs[m] ? stg + m * ns : nullptr;
    HIP_TRY(lbk::launch_fields(h->storage, h->base, h->d_desc() + k, (long long)ns, h->cur, first_state(h), dev[0],
                               dev[1], dev[2], dev[3], h->stream));
    for (int m = 0; m < 4; ++m)
        if (outs[m]) HIP_TRY(hipMemcpyAsync(outs[m], dev[m], ns * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LB_OK;
}

lb_status stress_all(lbb_handle* h, double* sb, double* stp, int64_t* ns)
{
    const int n = (int)h->lats.size();
    double* dres = h->d_res() + 8;
    HIP_TRY(lbk::launch_stress_reduce(h->base, h->d_desc(), n, dres, h->stream));
    std::vector<double> r(2 * n);
    HIP_TRY(hipMemcpyAsync(r.data(), dres, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int k = 0; k < n; ++k) {
        const double nx = h->lats[k].p.nx;
        const double m = h->nsamples > 0 ? (double)h->nsamples : 1.0;
        const double vb = h->nsamples > 0 ? r[2 * k] / nx / m : 0.0;
        const double vt = h->nsamples > 0 ? -r[2 * k + 1] / nx / m : 0.0;
        if (sb) sb[k] = vb;
        if (stp) stp[k] = vt;
    }
    if (ns) *ns = h->nsamples;
    return LB_OK;
}

lb_status profile_one(lbb_handle* h, int k, double* prof, int64_t* ns)
{
    if (k < 0 || k >= (int)h->lats.size()) return fail(LB_EINVAL, "lattice index out of range");
    const Lat& a = h->lats[k];
    if (!a.p.profile) return fail(LB_ESTATE, "profile accumulation was not enabled (lb_params.profile)");
    if (!prof) return fail(LB_EINVAL, "null profile array");
    double* stg = (double*)(h->base + a.off_f[h->cur ^ 1]);
    HIP_TRY(lbk::launch_profile_reduce(h->base, h->d_desc() + k, a.p.ny, stg, h->stream));
    HIP_TRY(hipMemcpyAsync(prof, stg, sizeof(double) * a.p.ny, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const double m = h->nsamples > 0 ? (double)h->nsamples * a.p.nx : 1.0;
    for (int y = 0; y < a.p.ny; ++y) prof[y] = h->nsamples > 0 ? prof[y] / m : 0.0;
    if (ns) *ns = h->nsamples;
    return LB_OK;
}

// Instantaneous line-averaged u_x of lattice k, staged in its idle population buffer.
lb_status line_profile(lbb_handle* h, int k, double* prof)
{
    if (k < 0 || k >= (int)h->lats.size()) return fail(LB_EINVAL, "lattice index out of range");
    if (!prof) return fail(LB_EINVAL, "null profile array");
    const Lat& a = h->lats[k];
    double* stg = (double*)(h->base + a.off_f[h->cur ^ 1]);
    HIP_TRY(lbk::launch_line_profile(h->storage, h->base, h->d_desc() + k, a.p.ny, h->cur, first_state(h), stg,
                                     h->stream));
    HIP_TRY(hipMemcpyAsync(prof, stg, sizeof(double) * a.p.ny, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LB_OK;
}

// Default launch shape: the widest tile and tallest row segment that still
// give about sixteen work items per compute unit.  A block marches its segment
// row by row and each row waits on memory, so small lattices and small
// batches split into a few tall items leave the chip idle; big lattices keep
// wide, tall items (fewer segment prologues and halo columns).
void default_shape(lbb_handle* h)
{
    int dev = 0, ncu = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        ncu = prop.multiProcessorCount;
    int maxnx = 0;
    for (const Lat& a : h->lats) maxnx = std::max(maxnx, a.p.nx);
    const int bxmax = maxnx >= 256 ? 256 : (maxnx >= 128 ? 128 : 64);
    static const int cand[][2] = {{256, 64}, {256, 32}, {256, 16}, {128, 16}, {64, 16}, {64, 8}};
    for (const auto& c : cand) {
        if (c[0] > bxmax) continue;
        long long items = 0;
        for (const Lat& a : h->lats)
            items += (long long)((a.p.nx + c[0] - 1) / c[0]) * ((a.p.ny + c[1] - 1) / c[1]);
        h->bx = c[0];
        h->ly = c[1];
        if (items >= 16ll * ncu) return;
    }
}

// Tile widths with a step kernel: 64, 128, 256, and 512 for the FP32 and
// 16-bit population forms.
bool bx_supported(int storage, int bx)
{
    return bx == 64 || bx == 128 || bx == 256 || (bx == 512 && storage >= 1 && storage <= 3);
}

// LDS one step block needs for shape (bx, ly) on this batch, and whether the
// current device grants it.
size_t shape_lds(const lbb_handle* h, int bx, int ly)
{
    int maxny = 1;
    for (const Lat& a : h->lats) maxny = std::max(maxny, a.p.ny);
    return lbk::step_lds_bytes(h->storage, bx, std::min(std::min(ly, maxny), 256));
}
int device_lds_limit()
{
    int dev = 0, lim = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 65536;
    return lim;
}
bool shape_fits(const lbb_handle* h, int bx, int ly)
{
    const size_t need = shape_lds(h, bx, ly);
    return need > 0 && need <= (size_t)device_lds_limit();
}

lb_status set_launch(lbb_handle* h, int bx, int ly, int grid)
{
    if (bx != 0 && !bx_supported(h->storage, bx))
        return fail(LB_EINVAL, "bx must be 64, 128 or 256 (or 512 for FP32 and 16-bit population storage)");
    if (ly < 0) return fail(LB_EINVAL, "ly must be >= 0");
    if (grid < 0) return fail(LB_EINVAL, "grid must be >= 0");
    {
        const int nbx = bx ? bx : h->bx, nly = ly ? ly : h->ly;
        if (!shape_fits(h, nbx, nly))
            return fail(LB_EINVAL, "launch shape bx %d ly %d needs %zu bytes of LDS per block, the device allows %d",
                        nbx, nly, shape_lds(h, nbx, nly), device_lds_limit());
    }
    if (bx) h->bx = bx;
    if (ly) h->ly = ly;
    h->grid = grid;
    return decompose(h);
}

// Whether the handle may run two steps per pass: FP32 or 16-bit population
// storage.
bool fusion_allowed(const lbb_handle* h)
{
    return fusion_storage(h->storage);
}

// The fused kernel's LDS for nw waves per step, checked against the device.
lb_status check_fused_lds(const lbb_handle* h, int nw)
{
    int dev = 0, lim = 65536;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    const size_t need = lbk::step2_lds_bytes(h->storage, nw);
    if (need == 0 || need > (size_t)lim)
        return fail(LB_EINVAL, "two steps per pass with %d lanes per step need %zu bytes of LDS per block, the device "
                    "allows %d", 64 * nw, need, lim);
    return LB_OK;
}

// Two time steps per pass (k_step2): FP32 or 16-bit population storage.
// ly2 = 0 picks the tile height.
lb_status set_fusion(lbb_handle* h, int k, int ly2)
{
    if (k != 1 && k != 2) return fail(LB_EINVAL, "steps per pass must be 1 or 2");
    if (ly2 < 0) return fail(LB_EINVAL, "ly2 must be >= 0");
    if (k == 2) {
        if (!fusion_allowed(h))
            return fail(LB_EINVAL, "two steps per pass need FP32 or 16-bit population storage");
        const int nw = h->fnw > 0 ? h->fnw : auto_fnw(h);
        lb_status st = check_fused_lds(h, nw);
        if (st != LB_OK) return st;
    }
    h->fusion = k;
    h->ly2 = ly2;
    return decompose(h);
}

// Lanes per step of the fused kernel's blocks: 128, 192 or 256 (0: automatic).
lb_status set_fusion_tile(lbb_handle* h, int lanes)
{
    if (lanes != 0 && lanes != 128 && lanes != 192 && lanes != 256)
        return fail(LB_EINVAL, "fused tile lanes must be 0, 128, 192 or 256 (got %d)", lanes);
    const int nw = lanes / 64;
    if (nw && fusion_storage(h->storage)) {
        lb_status st = check_fused_lds(h, nw);
        if (st != LB_OK) return st;
    }
    h->fnw = nw;
    return decompose(h);
}

lb_status steps_direct_warm(lbb_handle* h, int n)
{
    for (int k = 0; k < n; ++k) {
        lb_status st = launch_one(h, h->stream, h->cur);
        if (st != LB_OK) return st;
        h->cur ^= 1;
    }
    return LB_OK;
}

lb_status time_steps(lbb_handle* h, int32_t n, double* ms)
{
    if (n < 1 || !ms) return fail(LB_EINVAL, "need n >= 1 and an output");
    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    HIP_TRY(hipEventRecord(ev.a, h->stream));
    lb_status st = steps(h, n);
    HIP_TRY(hipEventRecord(ev.b, h->stream));
    HIP_TRY(hipEventSynchronize(ev.b));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, ev.a, ev.b));
    if (st != LB_OK) return st;
    *ms = (double)t / n;
    return LB_OK;
}

// ------------------------------------------------------------- autotuner --
//
// Times the step kernel over candidate launch shapes on the handle's own
// lattices, keeps the fastest and leaves the simulation state exactly as it
// was (populations, accumulators and counters are copied aside on the device
// and restored).  Results are cached in a small JSON file keyed by
// "<arch>/<storage>/<lattice shape>".

using lbh::TuneEntry;


std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

const char* storage_name(int s)
{
    static const char* n[] = {"f64", "f32", "f16dev", "bf16dev", "mom32", "mom64"};
    return (s >= 0 && s < 6) ? n[s] : "unknown";
}

std::string tune_key(const lbb_handle* h)
{
    char buf[160];
    if (h->lats.size() == 1) {
        snprintf(buf, sizeof buf, "%s/%s/%dx%d", arch_name().c_str(), storage_name(h->storage),
                 h->lats[0].p.nx, h->lats[0].p.ny);
    } else {
        long long sites = 0;
        for (const Lat& a : h->lats) sites += (long long)a.p.nx * a.p.ny;
        snprintf(buf, sizeof buf, "%s/%s/batch%zu_%lld", arch_name().c_str(), storage_name(h->storage),
                 h->lats.size(), sites);
    }
    return buf;
}

lb_status write_cache(const char* path, const lbh::TuneCache& ents)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return fail(LB_EINVAL, "cannot write tuning cache %s", path);
    const std::string text = lbh::format_cache(ents);
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    if (fclose(f) != 0 || !ok) return fail(LB_EINVAL, "cannot write tuning cache %s", path);
    if (rename(tmp.c_str(), path) != 0) return fail(LB_EINVAL, "cannot replace tuning cache %s", path);
    return LB_OK;
}

lb_status autotune(lbb_handle* h, const char* cache_path, int steps, bool batch, TuneEntry* best_out)
{
    if (steps < 1) return fail(LB_EINVAL, "need steps >= 1");
    const std::string key = tune_key(h);
    auto cache = lbh::read_cache(cache_path);
    for (auto& kv : cache)
        if (kv.first == key && kv.second.bx) {
            lb_status st = set_launch(h, kv.second.bx, kv.second.ly, kv.second.grid);
            if (st != LB_OK) return st;
            const bool fuse = kv.second.fusion == 2 && fusion_allowed(h);
            if (fuse) {
                st = set_fusion_tile(h, kv.second.fw);
                if (st != LB_OK) return st;
            }
            st = set_fusion(h, fuse ? 2 : 1, fuse ? kv.second.ly2 : 0);
            if (st != LB_OK) return st;
            if (best_out) *best_out = kv.second;
            return LB_OK;
        }
    // save the state
    size_t total = 0;
    std::vector<size_t> fb(h->lats.size()), ab(h->lats.size());
    for (size_t k = 0; k < h->lats.size(); ++k) {
        const Lat& a = h->lats[k];
        fb[k] = planes_of(h->storage) * a.plane * storage_size(h->storage);
        ab[k] = a.end - a.off_stress;
        total += fb[k] + ab[k];
    }
    TempDeviceBuffer saved;
    HIP_TRY(hipMalloc(&saved.p, total));
    char* const save = saved.p;
    size_t o = 0;
    for (size_t k = 0; k < h->lats.size(); ++k) {
        const Lat& a = h->lats[k];
        HIP_TRY(hipMemcpyAsync(save + o, h->base + a.off_f[h->cur], fb[k], hipMemcpyDeviceToDevice, h->stream));
        HIP_TRY(hipMemcpyAsync(save + o + fb[k], h->base + a.off_stress, ab[k], hipMemcpyDeviceToDevice, h->stream));
        o += fb[k] + ab[k];
    }
    const int cur = h->cur;
    const int64_t t = h->t, ns = h->nsamples;
    const int bx0 = h->bx, ly0 = h->ly, grid0 = h->grid, gs0 = h->graph_steps, wd0 = h->watchdog;
    const int fu0 = h->fusion, ly20 = h->ly2, fnw0 = h->fnw;
    h->graph_steps = 0;
    h->watchdog = 0;
    h->fusion = 1;          // the single-step kernel's shapes are what is tuned

    int maxnx = 0, maxny = 0;
    for (const Lat& a : h->lats) { maxnx = std::max(maxnx, a.p.nx); maxny = std::max(maxny, a.p.ny); }
    int dev = 0, ncu = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        ncu = prop.multiProcessorCount;
    // Candidates are timed in two rounds: every shape once over `steps`
    // steps, then the fastest few again, twice, over 4 x steps (the best time
    // of those runs decides).  A single short timing is noisy: the first tens
    // of launches after an idle GPU run 3-15 % slow, so the device is first
    // kept busy for about 0.3 s with the default shape.
    std::vector<TuneEntry> cands;
    lb_status st = LB_OK;
    {
        double ms1 = 0;
        st = steps_direct_warm(h, 2);
        if (st == LB_OK) st = time_steps(h, 2, &ms1);
        if (st == LB_OK && ms1 > 0) {
            const int warm = (int)std::min(20000.0, 300.0 / ms1);
            for (int done = 0; st == LB_OK && done < warm; done += 256)
                st = steps_direct_warm(h, std::min(256, warm - done));
        }
    }
    auto time_entry = [&](TuneEntry& e, int n) -> lb_status {
        lb_status s2 = set_launch(h, e.bx, e.ly, e.grid);
        if (s2 == LB_OK && e.fusion == 2) s2 = set_fusion_tile(h, e.fw);
        if (s2 == LB_OK) s2 = set_fusion(h, e.fusion, e.fusion == 2 ? e.ly2 : 0);
        if (s2 == LB_OK) s2 = steps_direct_warm(h, 2);
        double ms = 0;
        const int nn = n + (e.fusion == 2 ? (n & 1) : 0);
        // one untimed pass through the timed path first: the first replay of
        // a new configuration's graph carries one-time costs (up to 5 % of a
        // 40-step timing after a change of block width, enough to reorder
        // shapes a few per cent apart)
        if (s2 == LB_OK) s2 = time_steps(h, nn, &ms);
        if (s2 == LB_OK) s2 = time_steps(h, nn, &ms);
        if (s2 == LB_OK) e.ms = ms;
        return s2;
    };
    for (int bx : {64, 128, 256, 512}) {
        if (st != LB_OK) break;
        if (!bx_supported(h->storage, bx) || (bx > 64 && bx / 2 >= maxnx)) continue;
        for (int ly : {8, 16, 32, 48, 64, 80, 96, 128, 160, 192, 256}) {
            if (ly > 16 && ly / 2 >= maxny) continue;
            if (!shape_fits(h, bx, ly)) continue;
            std::vector<int> grids = {0};
            if (batch)
                for (int per : {1, 2, 4}) grids.push_back(ncu * per);
            for (int grid : grids) {
                TuneEntry e;
                e.bx = bx; e.ly = ly; e.grid = grid;
                st = time_entry(e, steps);
                if (st != LB_OK) break;
                cands.push_back(e);
            }
            if (st != LB_OK) break;
        }
    }
    // two steps per pass behind the best single-step shape (which any odd
    // remaining step uses): each block width the device grants, at the
    // automatic tile height (the smallest modelled makespan) and the other
    // FUSED_HEIGHTS up to 300 rows (the model is approximate: measured times
    // differ from it by several per cent)
    TuneEntry best1;
    for (const TuneEntry& e : cands)
        if (!best1.bx || e.ms < best1.ms) best1 = e;
    if (st == LB_OK && best1.bx && fusion_allowed(h)) {
        for (int lanes : {128, 192, 256}) {
            if (st != LB_OK) break;
            if (lbk::step2_blocks_per_cu(h->storage, lanes / 64) < 1) continue;
            std::vector<int> heights = {0};
            for (int c : FUSED_HEIGHTS)
                if (c <= 300) heights.push_back(c);
            for (int ly2 : heights) {
                if (st != LB_OK) break;
                if (ly2 && ly2 >= maxny) continue;
                TuneEntry e = best1;
                e.fusion = 2; e.ly2 = ly2; e.fw = lanes;
                st = time_entry(e, steps);
                if (st == LB_OK) cands.push_back(e);
            }
        }
    }
    TuneEntry best;
    if (st == LB_OK && !cands.empty()) {
        std::stable_sort(cands.begin(), cands.end(), [](const TuneEntry& x, const TuneEntry& y) { return x.ms < y.ms; });
        const size_t nf = std::min<size_t>(cands.size(), 4);
        for (size_t i = 0; i < nf && st == LB_OK; ++i) {
            TuneEntry e = cands[i];
            double m = 1e300;
            for (int r = 0; r < 2 && st == LB_OK; ++r) {
                st = time_entry(e, 4 * steps);
                m = std::min(m, e.ms);
            }
            e.ms = m;
            if (st == LB_OK && (!best.bx || e.ms < best.ms)) best = e;
        }
    }
    h->fusion = 1;
    // restore the state
    o = 0;
    h->cur = cur;
    for (size_t k = 0; k < h->lats.size(); ++k) {
        const Lat& a = h->lats[k];
        (void)hipMemcpyAsync(h->base + a.off_f[cur], save + o, fb[k], hipMemcpyDeviceToDevice, h->stream);
        (void)hipMemcpyAsync(h->base + a.off_stress, save + o + fb[k], ab[k], hipMemcpyDeviceToDevice, h->stream);
        o += fb[k] + ab[k];
    }
    (void)hipStreamSynchronize(h->stream);
    h->t = t;
    h->nsamples = ns;
    h->graph_steps = gs0;
    h->fusion = fu0;
    h->ly2 = ly20;
    h->fnw = fnw0;
    h->watchdog = wd0;
    if (st != LB_OK) {
        (void)set_launch(h, bx0, ly0, grid0);
        return st;
    }
    st = set_launch(h, best.bx, best.ly, best.grid);
    if (st != LB_OK) return st;
    if (best.fusion == 2) {
        st = set_fusion_tile(h, best.fw);
        if (st != LB_OK) return st;
    }
    st = set_fusion(h, best.fusion, best.ly2);
    if (st != LB_OK) return st;
    if (best_out) *best_out = best;
    if (cache_path) {
        bool found = false;
        for (auto& kv : cache)
            if (kv.first == key) { kv.second = best; found = true; }
        if (!found) cache.emplace_back(key, best);
        return write_cache(cache_path, cache);
    }
    return LB_OK;
}

void destroy_batch(lbb_handle* h)
{
    drop_graphs(h);
    if (h->capture) (void)hipStreamDestroy(h->capture);
    delete h;
}

}  // namespace

// ------------------------------------------------- allocation-free stress ---
//
// lbb_stress_noalloc keeps the per-lattice wall-momentum sums (bottom, top of
// each lattice, interleaved) in this file-scope device array instead of the
// results region of the caller's state.  Every GPU the library runs on holds
// its own copy until the process ends.  Host code uses the address
// hipGetSymbolAddress returns for the current device, never the array's name
// (which is a host-side stand-in).
constexpr int NOALLOC_MAX_LATTICES = 4096;
static __device__ __align__(256) double scratch[2 * NOALLOC_MAX_LATTICES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, resolved once per device.
lb_status scratch_ptr(double** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(LB_EDEVICE, "device %d beyond the %d supported", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LB_EDEVICE, "no device address for the stress scratch array");
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return LB_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI ---

extern "C" {

const char* lb_last_error(void) { return g_err.c_str(); }

lb_status lb_state_bytes(const lb_params* p, size_t* bytes) { return lbb_state_bytes(p, 1, bytes); }

lb_status lbb_state_bytes(const lb_params* params, int32_t n, size_t* bytes)
{
    if (!bytes || !params || n < 1) return fail(LB_EINVAL, "bad arguments");
    std::vector<Lat> lats(n);
    for (int k = 0; k < n; ++k) {
        lb_status st = validate(&params[k], params[0].storage);
        if (st != LB_OK) return st;
        lats[k].p = params[k];
    }
    *bytes = plan(lats).total;
    return LB_OK;
}

lb_status lb_init(const lb_params* p, void* dev_state, size_t bytes, void* hip_stream, const double* rho_a,
                  const double* rho_b, const double* ux, const double* uy, lb_handle** out)
{
    if (!out) return fail(LB_EINVAL, "null output handle");
    *out = nullptr;
    const double* ra[1] = {rho_a};
    const double* rb[1] = {rho_b};
    const double* u[1] = {ux};
    const double* v[1] = {uy};
    lbb_handle* b = nullptr;
    lb_status st = batch_init(p, 1, dev_state, bytes, hip_stream, ra, rb, u, v, &b);
    if (st != LB_OK) return st;
    lb_handle* h = new (std::nothrow) lb_handle();
    if (!h) { destroy_batch(b); return fail(LB_ENOMEM, "host allocation failed"); }
    h->b = std::move(*b);
    b->exec[0] = b->exec[1] = nullptr;
    b->capture = nullptr;
    delete b;
    *out = h;
    return LB_OK;
}

#define CHECK_H(h) \
    if (!(h)) return fail(LB_EINVAL, "null handle")

lb_status lb_step(lb_handle* h, int32_t n)
{
    CHECK_H(h);
    return steps(&h->b, n);
}

lb_status lb_fields(lb_handle* h, double* ra, double* rb, double* ux, double* uy)
{
    CHECK_H(h);
    lb_status st = lattice_fields(&h->b, 0, ra, rb, ux, uy, true);
    if (st != LB_OK) return st;
    return check_flag(&h->b);
}

lb_status lb_fields_device(lb_handle* h, double* ra, double* rb, double* ux, double* uy)
{
    CHECK_H(h);
    return lattice_fields(&h->b, 0, ra, rb, ux, uy, false);
}

lb_status lb_populations(lb_handle* h, double* f)
{
    CHECK_H(h);
    if (!f) return fail(LB_EINVAL, "null output");
    lbb_handle* b = &h->b;
    const Lat& a = b->lats[0];
    const size_t ns = (size_t)a.p.nx * a.p.ny;
    double* stg = (double*)(b->base + a.off_f[b->cur ^ 1]);
    for (int q = 0; q < 18; ++q) {
        HIP_TRY(lbk::launch_export(b->storage, b->base, b->d_desc(), (long long)ns, b->cur, first_state(b), q, stg,
                                   b->stream));
        HIP_TRY(hipMemcpyAsync(f + q * ns, stg, ns * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    return LB_OK;
}

lb_status lb_stress(lb_handle* h, double* sb, double* stp, int64_t* ns)
{
    CHECK_H(h);
    lb_status st = stress_all(&h->b, sb, stp, ns);
    if (st != LB_OK) return st;
    return check_flag(&h->b);
}

lb_status lb_stress_reset(lb_handle* h)
{
    CHECK_H(h);
    return reset_acc(&h->b);
}

lb_status lb_profile(lb_handle* h, double* prof, int64_t* ns)
{
    CHECK_H(h);
    return profile_one(&h->b, 0, prof, ns);
}

lb_status lb_line_profile(lb_handle* h, double* prof)
{
    CHECK_H(h);
    return line_profile(&h->b, 0, prof);
}

lb_status lb_sums(lb_handle* h, double out[5])
{
    CHECK_H(h);
    if (!out) return fail(LB_EINVAL, "null output");
    lbb_handle* b = &h->b;
    lb_status st = run_sums(b, 0, b->d_flag());
    if (st != LB_OK) return st;
    HIP_TRY(hipMemcpyAsync(out, b->d_res(), 5 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (out[4] > 0) return fail(LB_ENONFINITE, "%g sites with a non-finite or non-positive density", out[4]);
    return check_flag(b);
}

lb_status lb_set_watchdog(lb_handle* h, int32_t every)
{
    CHECK_H(h);
    if (every < 0) return fail(LB_EINVAL, "watchdog interval must be >= 0");
    h->b.watchdog = every;
    return LB_OK;
}

lb_status lb_set_launch(lb_handle* h, int32_t bx, int32_t ly)
{
    CHECK_H(h);
    return set_launch(&h->b, bx, ly, 0);
}

lb_status lb_set_fusion(lb_handle* h, int32_t steps_per_pass, int32_t ly2)
{
    CHECK_H(h);
    return set_fusion(&h->b, steps_per_pass, ly2);
}

lb_status lb_set_fusion_tile(lb_handle* h, int32_t lanes)
{
    CHECK_H(h);
    return set_fusion_tile(&h->b, lanes);
}

lb_status lb_get_fusion_tile(lb_handle* h, int32_t* lanes, int32_t* columns)
{
    CHECK_H(h);
    return lbb_get_fusion_tile(&h->b, lanes, columns);
}

lb_status lb_get_launch(lb_handle* h, int32_t* bx, int32_t* ly, int32_t* steps_per_pass, int32_t* ly2)
{
    CHECK_H(h);
    return lbb_get_launch(&h->b, bx, ly, nullptr, steps_per_pass, ly2);
}

lb_status lb_set_graph(lb_handle* h, int32_t k)
{
    CHECK_H(h);
    if (k < 0 || (k % 2)) return fail(LB_EINVAL, "steps per graph must be 0 or a positive even number");
    h->b.graph_steps = k;
    drop_graphs(&h->b);
    return LB_OK;
}

// Checkpoint: lbh::CkptHeader, then the current population buffer in its
// storage format, then the FP64 stress and profile accumulators.
lbh::CkptHeader ckpt_header_of(const lbb_handle* b)
{
    const Lat& a = b->lats[0];
    const size_t fb = planes_of(b->storage) * a.plane * storage_size(b->storage);
    const size_t sbb = 2ull * a.p.nx * sizeof(double);
    const size_t pb = a.p.profile ? prof_entries(a) * sizeof(double) : 0;
    return lbh::make_header(b->storage, a.p.nx, a.p.ny, a.pitch, a.p.profile, b->t, b->nsamples, fb, sbb, pb);
}

lb_status lb_save(lb_handle* h, void* buf, size_t* bytes)
{
    CHECK_H(h);
    if (!bytes) return fail(LB_EINVAL, "null size");
    lbb_handle* b = &h->b;
    const Lat& a = b->lats[0];
    const lbh::CkptHeader hd = ckpt_header_of(b);
    const size_t need = sizeof hd + hd.fbytes + hd.sbytes + hd.pbytes;
    if (!buf) { *bytes = need; return LB_OK; }
    if (*bytes < need) return fail(LB_EINVAL, "checkpoint buffer too small (%zu < %zu)", *bytes, need);
    char* p = (char*)buf;
    std::memcpy(p, &hd, sizeof hd);
    HIP_TRY(hipMemcpyAsync(p + sizeof hd, b->base + a.off_f[b->cur], hd.fbytes, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipMemcpyAsync(p + sizeof hd + hd.fbytes, b->base + a.off_stress, hd.sbytes, hipMemcpyDeviceToHost,
                           b->stream));
    if (hd.pbytes)
        HIP_TRY(hipMemcpyAsync(p + sizeof hd + hd.fbytes + hd.sbytes, b->base + a.off_prof, hd.pbytes,
                               hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    *bytes = need;
    return LB_OK;
}

lb_status lb_load(lb_handle* h, const void* buf, size_t bytes)
{
    CHECK_H(h);
    lbb_handle* b = &h->b;
    const Lat& a = b->lats[0];
    lbh::CkptHeader hd;
    std::string msg;
    const lb_status st = lbh::check_checkpoint(buf, bytes, ckpt_header_of(b), &hd, &msg);
    if (st != LB_OK) return fail(st, "%s", msg.c_str());
    const char* p = (const char*)buf;
    b->cur = 0;
    HIP_TRY(hipMemcpyAsync(b->base + a.off_f[0], p + sizeof hd, hd.fbytes, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->base + a.off_stress, p + sizeof hd + hd.fbytes, hd.sbytes, hipMemcpyHostToDevice,
                           b->stream));
    if (hd.pbytes)
        HIP_TRY(hipMemcpyAsync(b->base + a.off_prof, p + sizeof hd + hd.fbytes + hd.sbytes, hd.pbytes,
                               hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->t = hd.t;
    b->nsamples = hd.nsamples;
    return LB_OK;
}

lb_status lb_time(lb_handle* h, int64_t* t)
{
    CHECK_H(h);
    if (!t) return fail(LB_EINVAL, "null output");
    *t = h->b.t;
    return LB_OK;
}

lb_status lb_time_steps(lb_handle* h, int32_t n, double* ms)
{
    CHECK_H(h);
    return time_steps(&h->b, n, ms);
}

lb_status lb_autotune(lb_handle* h, const char* cache_path, int32_t steps, int32_t* bx, int32_t* ly, double* ms)
{
    CHECK_H(h);
    TuneEntry e;
    lb_status st = autotune(&h->b, cache_path, steps, false, &e);
    if (st != LB_OK) return st;
    if (bx) *bx = e.bx;
    if (ly) *ly = e.ly;
    if (ms) *ms = e.ms;
    return LB_OK;
}

lb_status lb_destroy(lb_handle* h)
{
    if (!h) return LB_OK;
    drop_graphs(&h->b);
    if (h->b.capture) (void)hipStreamDestroy(h->b.capture);
    delete h;
    return LB_OK;
}

// ----------------------------------------------------------------- batch ---

lb_status lbb_init(const lb_params* params, int32_t n, void* dev_state, size_t bytes, void* hip_stream,
                   const double* const* rho_a, const double* const* rho_b, const double* const* ux,
                   const double* const* uy, lbb_handle** out)
{
    return batch_init(params, n, dev_state, bytes, hip_stream, rho_a, rho_b, ux, uy, out);
}

lb_status lbb_step(lbb_handle* h, int32_t n)
{
    CHECK_H(h);
    return steps(h, n);
}

lb_status lbb_stress(lbb_handle* h, double* sb, double* stp, int64_t* ns)
{
    CHECK_H(h);
    lb_status st = stress_all(h, sb, stp, ns);
    if (st != LB_OK) return st;
    return check_flag(h);
}

lb_status lbb_stress_noalloc(lbb_handle* h, double* sb, double* stp, int64_t* ns)
{
    CHECK_H(h);
    const int n = (int)h->lats.size();
    if (n > NOALLOC_MAX_LATTICES)
        return fail(LB_EINVAL, "lbb_stress_noalloc handles at most %d lattices (batch of %d)", NOALLOC_MAX_LATTICES, n);
    double* dres = nullptr;
    lb_status st = scratch_ptr(&dres);
    if (st != LB_OK) return st;
    HIP_TRY(lbk::launch_stress_reduce(h->base, h->d_desc(), n, dres, h->stream));
    // (bottom, top) pairs per lattice -> the caller's two arrays, strided copies
    if (sb)
        HIP_TRY(hipMemcpy2DAsync(sb, sizeof(double), dres, 2 * sizeof(double), sizeof(double), (size_t)n,
                                 hipMemcpyDeviceToHost, h->stream));
    if (stp)
        HIP_TRY(hipMemcpy2DAsync(stp, sizeof(double), dres + 1, 2 * sizeof(double), sizeof(double), (size_t)n,
                                 hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    // the scaling of stress_all, in place
    const double m = h->nsamples > 0 ? (double)h->nsamples : 1.0;
    for (int k = 0; k < n; ++k) {
        const double nx = h->lats[k].p.nx;
        if (sb) sb[k] = h->nsamples > 0 ? sb[k] / nx / m : 0.0;
        if (stp) stp[k] = h->nsamples > 0 ? -stp[k] / nx / m : 0.0;
    }
    if (ns) *ns = h->nsamples;
    return check_flag(h);
}

lb_status lbb_stress_reset(lbb_handle* h)
{
    CHECK_H(h);
    return reset_acc(h);
}

lb_status lbb_fields(lbb_handle* h, int32_t k, double* ra, double* rb, double* ux, double* uy)
{
    CHECK_H(h);
    return lattice_fields(h, k, ra, rb, ux, uy, true);
}

lb_status lbb_profile(lbb_handle* h, int32_t k, double* prof, int64_t* ns)
{
    CHECK_H(h);
    return profile_one(h, k, prof, ns);
}

lb_status lbb_line_profile(lbb_handle* h, int32_t k, double* prof)
{
    CHECK_H(h);
    return line_profile(h, k, prof);
}

lb_status lbb_set_launch(lbb_handle* h, int32_t bx, int32_t ly, int32_t grid)
{
    CHECK_H(h);
    return set_launch(h, bx, ly, grid);
}

lb_status lbb_set_fusion(lbb_handle* h, int32_t steps_per_pass, int32_t ly2)
{
    CHECK_H(h);
    return set_fusion(h, steps_per_pass, ly2);
}

lb_status lbb_set_fusion_tile(lbb_handle* h, int32_t lanes)
{
    CHECK_H(h);
    return set_fusion_tile(h, lanes);
}

lb_status lbb_get_fusion_tile(lbb_handle* h, int32_t* lanes, int32_t* columns)
{
    CHECK_H(h);
    if (lanes) *lanes = 64 * h->fnw_eff;
    if (columns) *columns = lbk::fuse2_tw(h->storage, h->fnw_eff);
    return LB_OK;
}

lb_status lbb_get_launch(lbb_handle* h, int32_t* bx, int32_t* ly, int32_t* grid, int32_t* steps_per_pass,
                         int32_t* ly2)
{
    CHECK_H(h);
    if (bx) *bx = h->bx;
    if (ly) *ly = h->ly;
    if (grid) *grid = h->grid;
    if (steps_per_pass) *steps_per_pass = h->fusion;
    if (ly2) *ly2 = h->ly2_eff;
    return LB_OK;
}

lb_status lbb_set_graph(lbb_handle* h, int32_t k)
{
    CHECK_H(h);
    if (k < 0 || (k % 2)) return fail(LB_EINVAL, "steps per graph must be 0 or a positive even number");
    h->graph_steps = k;
    drop_graphs(h);
    return LB_OK;
}

lb_status lbb_time_steps(lbb_handle* h, int32_t n, double* ms)
{
    CHECK_H(h);
    return time_steps(h, n, ms);
}

lb_status lb_copy_peak(void* dst, const void* src, size_t bytes, void* hip_stream, int32_t reps, double* gbs)
{
    if (!dst || !src || !gbs || reps < 1 || bytes < 16 || (bytes % 16) || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16))
        return fail(LB_EINVAL, "copy needs 16-byte aligned buffers, a size multiple of 16 and reps >= 1");
    hipStream_t s = (hipStream_t)hip_stream;
    // full grid, one 16-byte element per thread: the fastest plain copy on
    // this GPU (a grid-stride loop over a few blocks per CU is slower)
    const long long n16 = (long long)(bytes / 16);
    const int blocks = (int)std::min<long long>((n16 + 255) / 256, 0x7fffffffLL);
    HIP_TRY(lbk::launch_copy(src, dst, n16, blocks, s));   // warm-up
    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    HIP_TRY(hipEventRecord(ev.a, s));
    for (int r = 0; r < reps; ++r) HIP_TRY(lbk::launch_copy(src, dst, n16, blocks, s));
    HIP_TRY(hipEventRecord(ev.b, s));
    HIP_TRY(hipEventSynchronize(ev.b));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
    *gbs = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return LB_OK;
}

lb_status lbb_autotune(lbb_handle* h, const char* cache_path, int32_t steps, int32_t* bx, int32_t* ly,
                       int32_t* grid, double* ms)
{
    CHECK_H(h);
    TuneEntry e;
    lb_status st = autotune(h, cache_path, steps, true, &e);
    if (st != LB_OK) return st;
    if (bx) *bx = e.bx;
    if (ly) *ly = e.ly;
    if (grid) *grid = e.grid;
    if (ms) *ms = e.ms;
    return LB_OK;
}

lb_status lbb_destroy(lbb_handle* h)
{
    if (!h) return LB_OK;
    destroy_batch(h);
    return LB_OK;
}

}  // extern "C"
