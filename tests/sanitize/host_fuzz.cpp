// Sanitizer harness of the library's host-only logic (csrc/lb_host.cpp):
// parameter validation, the initial-field checks, the tuning-cache parser and
// the checkpoint header checks, fed valid and malformed inputs.  Built with
// -fsanitize=address,undefined by tests/test_host_sanitize.py; any invalid
// memory access, leak or undefined behaviour aborts it, and every expected
// result is checked here.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <random>
#include <string>
#include <vector>

#include "lb_host.hpp"

static int failures = 0;
#define EXPECT(c)                                                              \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

static lb_params good()
{
    lb_params p;
    std::memset(&p, 0, sizeof p);
    p.nx = 128;
    p.ny = 96;
    p.walls_y = 1;
    p.storage = LB_F32;
    p.tau = 1.0;
    p.rho0 = 0.83;
    p.g_aa1 = p.g_bb1 = -9.0;
    p.g_aa2 = p.g_bb2 = 8.1;
    p.g_ab = 0.405;
    p.u_top = 0.02;
    p.u_bot = -0.02;
    return p;
}

static void test_validate()
{
    std::string msg;
    lb_params p = good();
    EXPECT(lbh::validate(&p, -1, &msg) == LB_OK);
    EXPECT(lbh::validate(nullptr, -1, &msg) == LB_EINVAL);
    const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();
    double lb_params::*dfield[] = {&lb_params::tau, &lb_params::rho0, &lb_params::g_aa1, &lb_params::g_aa2,
                                   &lb_params::g_bb1, &lb_params::g_bb2, &lb_params::g_ab, &lb_params::u_top,
                                   &lb_params::u_bot, &lb_params::rho_ref_a, &lb_params::rho_ref_b,
                                   &lb_params::fx_amp, &lb_params::fx_k};
    for (auto f : dfield)
        for (double v : {nan, inf, -inf}) {
            p = good();
            p.*f = v;
            msg.clear();
            EXPECT(lbh::validate(&p, -1, &msg) == LB_EINVAL && !msg.empty());
        }
    for (double t : {0.5, 0.4999, 0.0, -1.0}) { p = good(); p.tau = t; EXPECT(lbh::validate(&p, -1, &msg) == LB_EINVAL); }
    for (double r : {0.0, -0.1}) { p = good(); p.rho0 = r; EXPECT(lbh::validate(&p, -1, &msg) == LB_EINVAL); }
    const int32_t sizes[][2] = {{0, 10}, {10, 1}, {-5, 10}, {65537, 4}, {4, 65537}, {INT32_MIN, INT32_MIN},
                                {INT32_MAX, INT32_MAX}};
    for (auto& s : sizes) { p = good(); p.nx = s[0]; p.ny = s[1]; EXPECT(lbh::validate(&p, -1, &msg) == LB_EINVAL); }
    for (int s : {-1, 6, 1000, INT32_MIN}) { p = good(); p.storage = s; EXPECT(lbh::validate(&p, -1, &msg) == LB_EINVAL); }
    for (int w : {-1, 2, INT32_MAX}) { p = good(); p.walls_y = w; EXPECT(lbh::validate(&p, -1, &msg) == LB_EINVAL); }
    for (int w : {-1, 2}) { p = good(); p.profile = w; EXPECT(lbh::validate(&p, -1, &msg) == LB_EINVAL); }
    // moment storage only at tau = 1; a batch shares one storage
    p = good(); p.storage = LB_MOM32; p.tau = 0.9; EXPECT(lbh::validate(&p, -1, &msg) == LB_EINVAL);
    p = good(); p.storage = LB_MOM32; EXPECT(lbh::validate(&p, -1, &msg) == LB_OK);
    p = good(); EXPECT(lbh::validate(&p, LB_F16DEV, &msg) == LB_EINVAL);
    // the largest squares whose species planes fit 32-bit byte offsets, and the next size up
    const int edge[][3] = {{LB_F64, 7680, 7744}, {LB_F32, 10880, 10944}, {LB_F16DEV, 15424, 15488},
                           {LB_MOM32, 13376, 13440}};
    for (auto& e : edge) {
        p = good(); p.storage = e[0]; p.nx = p.ny = e[1];
        EXPECT(lbh::validate(&p, -1, &msg) == LB_OK);
        p.nx = p.ny = e[2];
        EXPECT(lbh::validate(&p, -1, &msg) == LB_EINVAL);
    }
}

static lbh::TuneCache parse(const std::string& s) { return lbh::parse_cache(s.data(), s.size()); }

static void test_cache()
{
    lbh::TuneCache c = parse(
        "{\n\"gfx950/f32/4096x4096\": {\"bx\": 512, \"ly\": 128, \"grid\": 0, \"fusion\": 2, \"ly2\": 0, \"ms\": 0.35},\n"
        "\"gfx950/f16dev/4096x4096\": {\"bx\": 256, \"ly\": 32, \"grid\": 0, \"ms\": 0.39}\n}\n");
    EXPECT(c.size() == 2);
    if (c.size() == 2) {
        EXPECT(c[0].first == "gfx950/f32/4096x4096" && c[0].second.bx == 512 && c[0].second.ly == 128 &&
               c[0].second.fusion == 2 && c[0].second.ms == 0.35);
        EXPECT(c[1].second.fusion == 1 && c[1].second.ly2 == 0);
    }
    // round trip
    lbh::TuneCache back = parse(lbh::format_cache(c));
    EXPECT(back.size() == c.size());
    for (size_t i = 0; i < back.size() && i < c.size(); ++i)
        EXPECT(back[i].first == c[i].first && back[i].second.bx == c[i].second.bx &&
               back[i].second.ly2 == c[i].second.ly2 && back[i].second.fusion == c[i].second.fusion);
    // malformed lines are skipped, never read out of bounds
    const char* bad[] = {
        "", "\"", "\"\"", "\"k\"", "\"k\": {", "\"k\": {\"bx\":", "\"k\": {\"bx\": }",
        "\"k\": {\"bx\": 99999999999999999999999, \"ly\": 8}", "\"k\": {\"bx\": 100, \"ly\": 8}",
        "\"k\": {\"bx\": 256, \"ly\": -3}", "\"k\": {\"bx\": 256, \"ly\": 8, \"fusion\": 3}",
        "\"k\": {\"bx\": 256, \"ly\": 8, \"ms\": nan}", "\"k\": {\"bx\": 256, \"ly\": 8, \"ms\": 1e999}",
        "\"k\": {\"bx\": 256, \"ly\": 8, \"grid\": -1}", "\"k\": {\"bx\": 256}", "\"k\x01\": {\"bx\": 256, \"ly\": 8}",
        "\"k\": {\"bx\": 256, \"ly\": 8, \"ly2\": 99999999999}", "{\"bx\": 256, \"ly\": 8}", "\"k\" \"bx\": 256",
    };
    for (const char* b : bad) EXPECT(parse(b).empty());
    // long lines, binary noise, truncations of a valid file
    std::string longkey(100000, 'a');
    EXPECT(parse("\"" + longkey + "\": {\"bx\": 64, \"ly\": 8}").size() == 1);
    const std::string valid = lbh::format_cache(c);
    for (size_t k = 0; k <= valid.size(); ++k) (void)parse(valid.substr(0, k));
    std::mt19937 rng(12345);
    for (int t = 0; t < 3000; ++t) {
        std::string s = valid;
        const int edits = 1 + (int)(rng() % 8);
        for (int e = 0; e < edits && !s.empty(); ++e) s[rng() % s.size()] = (char)(rng() & 0xff);
        for (const auto& kv : parse(s)) {
            EXPECT(kv.second.bx == 64 || kv.second.bx == 128 || kv.second.bx == 256 || kv.second.bx == 512);
            EXPECT(kv.second.ly >= 0 && kv.second.grid >= 0 && kv.second.ly2 >= 0);
            EXPECT(kv.second.fusion == 1 || kv.second.fusion == 2);
            EXPECT(std::isfinite(kv.second.ms));
        }
        std::string noise(rng() % 300, '\0');
        for (auto& ch : noise) ch = (char)(rng() & 0xff);
        (void)parse(noise);
    }
    EXPECT(lbh::parse_cache(nullptr, 10).empty());
    EXPECT(lbh::read_cache("/nonexistent/dir/cache.json").empty());
    EXPECT(lbh::read_cache(nullptr).empty());
}

static void test_checkpoint()
{
    const uint64_t fb = 18ull * 64 * 8 * 4, sb = 2ull * 64 * 8, pb = 0;
    const lbh::CkptHeader want = lbh::make_header(LB_F32, 64, 8, 64, 0, 100, 40, fb, sb, pb);
    std::vector<char> buf(sizeof want + fb + sb + pb, 0);
    std::memcpy(buf.data(), &want, sizeof want);
    lbh::CkptHeader got;
    std::string msg;
    EXPECT(lbh::check_checkpoint(buf.data(), buf.size(), want, &got, &msg) == LB_OK && got.t == 100 &&
           got.nsamples == 40);
    // every truncation is refused
    for (size_t k = 0; k < buf.size(); k += 97)
        EXPECT(lbh::check_checkpoint(buf.data(), k, want, &got, &msg) != LB_OK);
    EXPECT(lbh::check_checkpoint(nullptr, buf.size(), want, &got, &msg) == LB_EINVAL);
    // a header of another lattice, or with inconsistent sections, is refused
    auto with = [&](auto edit) {
        lbh::CkptHeader h = want;
        edit(h);
        std::vector<char> b = buf;
        std::memcpy(b.data(), &h, sizeof h);
        return lbh::check_checkpoint(b.data(), b.size(), want, &got, &msg);
    };
    EXPECT(with([](lbh::CkptHeader& h) { h.magic[0] = 'X'; }) == LB_ESTATE);
    EXPECT(with([](lbh::CkptHeader& h) { h.version = 1; }) == LB_ESTATE);
    EXPECT(with([](lbh::CkptHeader& h) { h.storage = LB_F16DEV; }) == LB_ESTATE);
    EXPECT(with([](lbh::CkptHeader& h) { h.nx = 65; }) == LB_ESTATE);
    EXPECT(with([](lbh::CkptHeader& h) { h.pitch = 128; }) == LB_ESTATE);
    EXPECT(with([](lbh::CkptHeader& h) { h.profile = 1; }) == LB_ESTATE);
    EXPECT(with([](lbh::CkptHeader& h) { h.fbytes = ~0ull; }) == LB_ESTATE);
    EXPECT(with([](lbh::CkptHeader& h) { h.sbytes = ~0ull - 7; h.pbytes = 8; }) == LB_ESTATE);
    EXPECT(with([](lbh::CkptHeader& h) { h.t = -1; h.nsamples = -1; }) == LB_ESTATE);
    EXPECT(with([](lbh::CkptHeader& h) { h.nsamples = h.t + 1; }) == LB_ESTATE);
    // random headers
    std::mt19937 rng(7);
    for (int t = 0; t < 20000; ++t) {
        std::vector<char> b = buf;
        const int edits = 1 + (int)(rng() % 6);
        for (int e = 0; e < edits; ++e) b[rng() % sizeof(lbh::CkptHeader)] = (char)(rng() & 0xff);
        const size_t len = (rng() & 1) ? b.size() : rng() % (b.size() + 1);
        if (lbh::check_checkpoint(b.data(), len, want, &got, &msg) == LB_OK) {
            EXPECT(len >= sizeof got + fb + sb + pb && got.fbytes == fb && got.sbytes == sb && got.pbytes == pb);
            EXPECT(got.nx == 64 && got.ny == 8 && got.storage == LB_F32);
        }
    }
}

// Fused segments: every tile at most ly2 rows (ly2 >= 1), at least ceil(ny / ly2)
// segments, never more segments than rows, and no equal split into a multiple
// of 16 rows while a finer split exists.
static void test_fused_segments()
{
    for (int ny = 1; ny <= 1100; ++ny)
        for (int ly2 = 1; ly2 <= ny + 3; ly2 += (ly2 < 40 ? 1 : 7)) {
            const int n = lbh::fused_nseg(ny, ly2);
            EXPECT(n >= 1 && n <= ny);
            EXPECT(n >= (ny + ly2 - 1) / ly2 || ly2 > ny);
            EXPECT((ny + n - 1) / n <= ly2 || ly2 >= ny);
            if (n < ny) EXPECT(!(ny % n == 0 && (ny / n) % 16 == 0));
        }
    EXPECT(lbh::fused_nseg(4096, 92) == 45);
    EXPECT(lbh::fused_nseg(1024, 140) == 9);    // 8 x 128 rows avoided
    EXPECT(lbh::fused_nseg(384, 204) == 5);     // 3 x 128 and 4 x 96 avoided
    EXPECT(lbh::fused_nseg(16, 16) == 2 && lbh::fused_nseg(16, 8) == 2);
}

// Initial-field checks of several lattices over 1..16 threads: the same sums,
// bit for bit, as one sequential pass per lattice, and the first offending
// site of each kind.
static void test_fields()
{
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> U(0.05, 1.5);
    const size_t sizes[] = {1, 2, 3, 64, 1000, 4097, 20000, 7, 512, 999};
    const int n = (int)(sizeof sizes / sizeof sizes[0]);
    std::vector<std::vector<double>> a(n), b(n), u(n), v(n);
    std::vector<const double*> pa(n), pb(n), pu(n), pv(n);
    std::vector<double> ref0(n), ref1(n);
    for (int k = 0; k < n; ++k) {
        for (size_t i = 0; i < sizes[k]; ++i) {
            a[k].push_back(U(rng));
            b[k].push_back(U(rng));
            u[k].push_back(U(rng) - 0.5);
            v[k].push_back(U(rng) - 0.5);
        }
        double s0 = 0, s1 = 0;
        for (size_t i = 0; i < sizes[k]; ++i) {
            s0 += a[k][i];
            s1 += b[k][i];
        }
        ref0[k] = s0;
        ref1[k] = s1;
        pa[k] = a[k].data();
        pb[k] = b[k].data();
        pu[k] = u[k].data();
        pv[k] = (k % 3 == 1) ? nullptr : v[k].data();   // some lattices without u_y
    }
    for (int threads : {1, 2, 3, 16, 0}) {
        std::vector<lbh::FieldCheck> c(n);
        lbh::check_fields(n, sizes, pa.data(), pb.data(), pu.data(), pv.data(), c.data(), threads);
        for (int k = 0; k < n; ++k)
            EXPECT(c[k].what == 0 && c[k].sum[0] == ref0[k] && c[k].sum[1] == ref1[k]);
        lbh::check_fields(n, sizes, pa.data(), pb.data(), nullptr, nullptr, c.data(), threads);
        for (int k = 0; k < n; ++k) EXPECT(c[k].what == 0 && c[k].sum[0] == ref0[k]);
    }
    // planted faults: the first one in site order is reported, densities
    // before u_x before u_y at one site
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    a[4][700] = -0.0;
    u[4][300] = inf;
    b[5][10] = nan;
    u[6][5000] = nan;
    v[6][5000] = nan;
    v[9][998] = -inf;
    a[3][63] = 0.0;
    u[0][0] = nan;
    for (int threads : {1, 4, 0}) {
        std::vector<lbh::FieldCheck> c(n);
        lbh::check_fields(n, sizes, pa.data(), pb.data(), pu.data(), pv.data(), c.data(), threads);
        EXPECT(c[0].what == 2 && c[0].site == 0);
        EXPECT(c[1].what == 0 && c[2].what == 0 && c[7].what == 0 && c[8].what == 0);
        EXPECT(c[3].what == 1 && c[3].site == 63);
        EXPECT(c[4].what == 2 && c[4].site == 300);
        EXPECT(c[5].what == 1 && c[5].site == 10);
        EXPECT(c[6].what == 2 && c[6].site == 5000);
        EXPECT(c[9].what == 3 && c[9].site == 998);
        EXPECT(c[1].sum[0] == ref0[1] && c[8].sum[1] == ref1[8]);
    }
    lbh::check_fields(0, sizes, pa.data(), pb.data(), nullptr, nullptr, nullptr, 4);   // nothing to do
}

int main()
{
    test_fused_segments();
    test_validate();
    test_fields();
    test_cache();
    test_checkpoint();
    if (failures) {
        std::fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    std::printf("host logic: all checks passed under the sanitizers\n");
    return 0;
}
