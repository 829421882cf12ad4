// Host-only logic of the library (see lb_host.hpp).  No HIP, no device.
#include "lb_host.hpp"

#include <cerrno>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include <algorithm>
#include <atomic>
#include <thread>

namespace lbh {

size_t storage_size(int storage)
{
    switch (storage) {
    case LB_F64: return 8;
    case LB_F32: return 4;
    case LB_F16DEV: return 2;
    case LB_BF16DEV: return 2;
    case LB_MOM32: return 4;
    case LB_MOM64: return 8;
    default: return 0;
    }
}

namespace {

lb_status bad(std::string* msg, lb_status code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
lb_status bad(std::string* msg, lb_status code, const char* fmt, ...)
{
    if (msg) {
        char buf[256];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        *msg = buf;
    }
    return code;
}

}  // namespace

lb_status validate(const lb_params* p, int storage0, std::string* msg)
{
    if (!p) return bad(msg, LB_EINVAL, "null parameters");
    if (p->nx < 1 || p->ny < 2) return bad(msg, LB_EINVAL, "need nx >= 1 and ny >= 2 (got %d x %d)", p->nx, p->ny);
    if (p->nx > 65536 || p->ny > 65536) return bad(msg, LB_EINVAL, "lattice side above 65536");
    if (p->storage < 0 || p->storage > 5) return bad(msg, LB_EINVAL, "unknown storage %d", p->storage);
    if (is_mom(p->storage) && p->tau != 1.0)
        return bad(msg, LB_EINVAL, "moment storage holds the post-collision state only at tau = 1 (got %g)", p->tau);
    if (storage0 >= 0 && p->storage != storage0)
        return bad(msg, LB_EINVAL, "all lattices of a batch share one storage precision");
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return bad(msg, LB_EINVAL, "tau must be > 1/2 (got %g)", p->tau);
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return bad(msg, LB_EINVAL, "rho0 must be > 0");
    const double g[] = {p->g_aa1, p->g_aa2, p->g_bb1, p->g_bb2, p->g_ab, p->u_top, p->u_bot,
                        p->rho_ref_a, p->rho_ref_b, p->fx_amp, p->fx_k};
    for (double v : g)
        if (!std::isfinite(v))
            return bad(msg, LB_EINVAL, "non-finite coupling, wall speed, reference density or body force");
    if (p->walls_y != 0 && p->walls_y != 1) return bad(msg, LB_EINVAL, "walls_y must be 0 or 1");
    if (p->profile != 0 && p->profile != 1) return bad(msg, LB_EINVAL, "profile must be 0 or 1");
    // byte offsets inside one species' planes must fit the 32-bit buffer offset
    const size_t es = storage_size(p->storage);
    const size_t per = is_mom(p->storage) ? 6 : 9;   // values addressed through one buffer resource
    if (per * plane_stride(p->nx, p->ny) * es >= (1ull << 32))
        return bad(msg, LB_EINVAL, "lattice too large: one buffer resource would exceed 4 GiB");
    return LB_OK;
}

namespace {

// The integer after `"name":` in s (leading spaces allowed), if present and
// inside [lo, hi].  0: absent; 1: read into *out; -1: present but malformed
// or out of range.
int get_int(const std::string& s, const char* name, long lo, long hi, int* out)
{
    const std::string pat = std::string("\"") + name + "\":";
    const size_t at = s.find(pat);
    if (at == std::string::npos) return 0;
    const char* b = s.c_str() + at + pat.size();
    char* e = nullptr;
    errno = 0;
    const long v = std::strtol(b, &e, 10);
    if (e == b || errno == ERANGE || v < lo || v > hi) return -1;
    *out = (int)v;
    return 1;
}

int get_double(const std::string& s, const char* name, double* out)
{
    const std::string pat = std::string("\"") + name + "\":";
    const size_t at = s.find(pat);
    if (at == std::string::npos) return 0;
    const char* b = s.c_str() + at + pat.size();
    char* e = nullptr;
    errno = 0;
    const double v = std::strtod(b, &e);
    if (e == b || errno == ERANGE || !std::isfinite(v) || v < 0) return -1;
    *out = v;
    return 1;
}

// One line: the key between the first two quotes, then a '{' and the fields.
bool parse_line(const std::string& line, std::pair<std::string, TuneEntry>* out)
{
    const size_t q1 = line.find('"');
    if (q1 == std::string::npos) return false;
    const size_t q2 = line.find('"', q1 + 1);
    if (q2 == std::string::npos || q2 == q1 + 1) return false;
    const std::string key = line.substr(q1 + 1, q2 - q1 - 1);
    for (unsigned char c : key)
        if (c < 0x20 || c == 0x7f || c == '\\') return false;
    const size_t br = line.find('{', q2 + 1);
    if (br == std::string::npos) return false;
    const std::string body = line.substr(br);
    TuneEntry e;
    if (get_int(body, "bx", 64, 512, &e.bx) != 1) return false;
    if (e.bx != 64 && e.bx != 128 && e.bx != 256 && e.bx != 512) return false;
    if (get_int(body, "ly", 0, 1 << 20, &e.ly) != 1) return false;
    if (get_int(body, "grid", 0, 1 << 24, &e.grid) < 0) return false;
    const int fu = get_int(body, "fusion", 1, 2, &e.fusion);
    if (fu < 0) return false;
    if (fu == 0) e.fusion = 1;
    if (get_int(body, "ly2", 0, 1 << 20, &e.ly2) < 0) return false;
    if (get_int(body, "fw", 0, 256, &e.fw) < 0) return false;
    if (e.fw != 0 && e.fw != 128 && e.fw != 192 && e.fw != 256) return false;
    if (get_double(body, "ms", &e.ms) < 0) return false;
    out->first = key;
    out->second = e;
    return true;
}

}  // namespace

namespace {

void check_one(size_t ns, const double* ra, const double* rb, const double* ux, const double* uy, FieldCheck* c)
{
    double s0 = 0, s1 = 0;
    for (size_t i = 0; i < ns; ++i) {
        const double a = ra[i], b = rb[i];
        if (!(a > 0.0) || !(b > 0.0) || !std::isfinite(a) || !std::isfinite(b)) { c->what = 1; c->site = i; return; }
        s0 += a;
        s1 += b;
        if (ux && !std::isfinite(ux[i])) { c->what = 2; c->site = i; return; }
        if (uy && !std::isfinite(uy[i])) { c->what = 3; c->site = i; return; }
    }
    c->sum[0] = s0;
    c->sum[1] = s1;
}

}  // namespace

void check_fields(int n, const size_t* ns, const double* const* ra, const double* const* rb,
                  const double* const* ux, const double* const* uy, FieldCheck* out, int threads)
{
    if (n < 1) return;
    for (int k = 0; k < n; ++k) out[k] = FieldCheck();
    // the largest lattices first, so that the last one a thread takes is short
    std::vector<int> order(n);
    for (int k = 0; k < n; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ns[a] > ns[b]; });
    std::atomic<int> next(0);
    auto work = [&]() {
        for (int i = next.fetch_add(1); i < n; i = next.fetch_add(1)) {
            const int k = order[i];
            check_one(ns[k], ra[k], rb[k], ux ? ux[k] : nullptr, uy ? uy[k] : nullptr, &out[k]);
        }
    };
    if (threads <= 0) threads = std::min(16, (int)std::max(1u, std::thread::hardware_concurrency()));
    threads = std::min(threads, n);
    std::vector<std::thread> pool;
    for (int t = 1; t < threads; ++t) {
        try {
            pool.emplace_back(work);
        } catch (...) {
            break;   // fewer threads: the calling thread takes the rest
        }
    }
    work();
    for (std::thread& t : pool) t.join();
}

TuneCache parse_cache(const char* text, size_t len)
{
    TuneCache out;
    if (!text) return out;
    const std::string all(text, len);
    size_t b = 0;
    while (b < all.size()) {
        size_t e = all.find('\n', b);
        if (e == std::string::npos) e = all.size();
        std::pair<std::string, TuneEntry> kv;
        if (parse_line(all.substr(b, e - b), &kv)) out.push_back(kv);
        b = e + 1;
    }
    return out;
}

TuneCache read_cache(const char* path)
{
    TuneCache out;
    FILE* f = path ? std::fopen(path, "rb") : nullptr;
    if (!f) return out;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    return parse_cache(text.data(), text.size());
}

std::string format_cache(const TuneCache& ents)
{
    std::string s = "{\n";
    for (size_t i = 0; i < ents.size(); ++i) {
        char buf[256];
        const TuneEntry& e = ents[i].second;
        snprintf(buf, sizeof buf,
                 "{\"bx\": %d, \"ly\": %d, \"grid\": %d, \"fusion\": %d, \"ly2\": %d, \"fw\": %d, \"ms\": %.6f}%s\n",
                 e.bx, e.ly, e.grid, e.fusion, e.ly2, e.fw, e.ms, i + 1 < ents.size() ? "," : "");
        s += "\"" + ents[i].first + "\": " + buf;
    }
    s += "}\n";
    return s;
}

CkptHeader make_header(int storage, int nx, int ny, int pitch, int profile, int64_t t, int64_t nsamples,
                       uint64_t fbytes, uint64_t sbytes, uint64_t pbytes)
{
    CkptHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "LBMI355", 8);
    h.version = CKPT_VERSION;
    h.storage = storage;
    h.nx = nx;
    h.ny = ny;
    h.pitch = pitch;
    h.profile = profile;
    h.t = t;
    h.nsamples = nsamples;
    h.fbytes = fbytes;
    h.sbytes = sbytes;
    h.pbytes = pbytes;
    return h;
}

lb_status check_checkpoint(const void* buf, size_t bytes, const CkptHeader& want, CkptHeader* out, std::string* msg)
{
    if (!buf || bytes < sizeof(CkptHeader)) return bad(msg, LB_EINVAL, "checkpoint buffer too small");
    CkptHeader h;
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, "LBMI355", 8) != 0 || h.version != CKPT_VERSION)
        return bad(msg, LB_ESTATE, "not a checkpoint");
    if (h.storage != want.storage || h.nx != want.nx || h.ny != want.ny || h.pitch != want.pitch ||
        h.profile != want.profile)
        return bad(msg, LB_ESTATE, "checkpoint of another lattice shape, storage or profile setting");
    // the section sizes must be exactly this lattice's (they bound the copies)
    if (h.fbytes != want.fbytes || h.sbytes != want.sbytes || h.pbytes != want.pbytes)
        return bad(msg, LB_ESTATE, "checkpoint section sizes do not match this lattice");
    const size_t need = sizeof h + (size_t)want.fbytes + (size_t)want.sbytes + (size_t)want.pbytes;
    if (bytes < need) return bad(msg, LB_EINVAL, "truncated checkpoint (%zu < %zu bytes)", bytes, need);
    if (h.t < 0 || h.nsamples < 0 || h.nsamples > h.t)
        return bad(msg, LB_ESTATE, "checkpoint with an invalid step count");
    if (out) *out = h;
    return LB_OK;
}

}  // namespace lbh
