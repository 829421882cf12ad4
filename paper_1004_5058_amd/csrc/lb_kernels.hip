// HIP kernels (gfx950) of the two-species multirange Shan-Chen lattice
// Boltzmann step: Eq. (1) with the velocity-shift forcing, the forces of
// Eq. (2) on the 24-offset stencil of Fig. 1, and the pseudo-potential
// psi = rho0 (1 - exp(-rho/rho0)) (section "Lattice Boltzmann with multirange
// interactions" of arXiv:1004.5058).
//
// The step kernel is one fused pass per time step over populations stored
// structure-of-arrays, f[s][i][y][x] with x fastest:
//   * a block owns a strip of BX columns (one thread per column) and marches
//     down a segment of ly rows;
//   * for the row two ahead of the one it collides, each thread loads its
//     18 populations (aligned, coalesced), sums the two densities and stores
//     (psi_A, psi_B, rho_A, rho_B) in a six-row LDS ring; four lanes of wave 0
//     do the same for the two halo columns on each side;
//   * after one barrier the thread collides its centre row with the force read
//     from the 5x5 LDS neighbourhood and pushes the 18 post-collision
//     populations to their neighbours (row y-1, y, y+1 of the other buffer),
//     bouncing back at the walls and summing the wall momentum per column in
//     FP64.
// The three population rows in flight live in registers, so every
// population is read once and written once per step; the only re-reads are
// the halo columns and the two halo rows at each end of a segment.
#include "lb_device.hpp"
#include "lb_kernels.hpp"
#include <type_traits>

namespace lbk {

// ---------------------------------------------------------------- storage --

// Every format stores the deviation d_is = f_is - w_i rho_ref_s of a population
// from the rest equilibrium at the lattice's reference densities; arithmetic
// is FP64 for FP64 storage and FP32 otherwise.  fast_psi: the pseudo-potential
// from the hardware 2^x instead of expm1 (see dpsi).
struct StF64 { using S = double;   using C = double; static constexpr bool fast_psi = false; };
struct StF32 { using S = float;    using C = float;  static constexpr bool fast_psi = false; };
struct StF16 { using S = _Float16; using C = float;  static constexpr bool fast_psi = true; };
struct StBF16 { using S = __bf16;  using C = float;  static constexpr bool fast_psi = true; };

template <class C> struct V4;
template <> struct V4<float> { using T = float4; };
template <> struct V4<double> { using T = double4; };

// Raw buffer access.  A block addresses each species' plane stack through a
// buffer resource: the per-lane column byte offset is the VGPR offset and the
// uniform (direction, row) byte offset is the SGPR offset, so the 18 loads and
// 18 stores of a row need no 64-bit address arithmetic.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int RSRC_WORD3 = 0x00020000;

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, RSRC_WORD3);
}

template <class S> __device__ __forceinline__ S bload(rsrc_t r, unsigned voff, unsigned soff);
template <> __device__ __forceinline__ float bload<float>(rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, (int)soff, 0));
}
template <> __device__ __forceinline__ double bload<double>(rsrc_t r, unsigned voff, unsigned soff)
{
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(double, (u2)__builtin_amdgcn_raw_buffer_load_b64(r, voff, (int)soff, 0));
}
template <> __device__ __forceinline__ _Float16 bload<_Float16>(rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, (int)soff, 0));
}
template <> __device__ __forceinline__ __bf16 bload<__bf16>(rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, (int)soff, 0));
}

// Buffer store of one value; CP is the instruction's cache policy (0: default,
// CP_NT: non-temporal).
constexpr int CP_NT = 2;
template <class S, int CP = 0> __device__ __forceinline__ void bstore(S v, rsrc_t r, unsigned voff, unsigned soff)
{
    if constexpr (std::is_same<S, float>::value) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, (int)soff, CP);
    } else if constexpr (std::is_same<S, double>::value) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, (int)soff, CP);
    } else {
        static_assert(sizeof(S) == 2, "2-, 4- and 8-byte values");
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, voff, (int)soff, CP);
    }
}

// Load / store one deviation, converting between the storage and the
// arithmetic type (round to nearest even on the way down).  The SGPR offset is
// uniform by construction; readfirstlane states it, so a store under a
// divergent branch does not become a per-lane loop.
template <class P>
__device__ __forceinline__ typename P::C ld(rsrc_t r, unsigned voff, unsigned soff)
{
    return (typename P::C)bload<typename P::S>(r, voff, __builtin_amdgcn_readfirstlane(soff));
}

template <class P>
__device__ __forceinline__ void st(rsrc_t r, unsigned voff, unsigned soff, typename P::C v)
{
    bstore<typename P::S>((typename P::S)v, r, voff, (unsigned)__builtin_amdgcn_readfirstlane((int)soff));
}
template <class P, int CP = 0>
__device__ __forceinline__ void st_s(rsrc_t r, unsigned voff, unsigned soff, typename P::S v)
{
    bstore<typename P::S, CP>(v, r, voff, (unsigned)__builtin_amdgcn_readfirstlane((int)soff));
}

// A value of the arithmetic type, rounded to the storage format on its own:
// the value is first rounded to the arithmetic type, so the compiler cannot
// fuse the conversion into the multiply-add that produced it (for FP16 that
// fusion, v_fma_mixlo_f16, rounds once and can differ in the last bit; which
// stores it fuses would otherwise depend on the code around them).
template <class S, class C>
__device__ __forceinline__ S to_store(C x)
{
    if constexpr (std::is_same<S, C>::value) {
        return x;
    } else {
        asm("" : "+v"(x));
        return (S)x;
    }
}

// Two values of the arithmetic type rounded to the storage format on their own
// (FP16 as to_store, BF16 as the plain conversion).  16-bit storage from FP32:
// one packed conversion, which rounds each half as the single conversion does.
template <class S, class C>
__device__ __forceinline__ void to_store2(C a, C b, S& sa, S& sb)
{
    if constexpr (sizeof(S) == 2 && std::is_same<C, float>::value) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        typedef S s2 __attribute__((ext_vector_type(2)));
        if constexpr (std::is_same<S, _Float16>::value) {
            asm("" : "+v"(a));
            asm("" : "+v"(b));
        }
        const s2 h = __builtin_convertvector((f2){a, b}, s2);
        sa = h.x;
        sb = h.y;
    } else {
        sa = to_store<S>(a);
        sb = to_store<S>(b);
    }
}

// The 18 populations of one site held in registers between the row load and
// the collision: the arithmetic type for 32/64-bit storage; for 16-bit storage
// the raw values, two per VGPR (d16 loads fill the low and high halves), and
// converted when read.  Besides single values a row gives the sums the
// collision needs, in one fixed order (left to right): the species densities
// (dens), the momentum (mom), the deviation f_q - x of one population from a
// value (dev), and the post-collision value f_q - w t in the storage format,
// rounded from its FP32 value (post).
template <class P, bool PACK = (sizeof(typename P::S) == 2)> struct Row;

// The sums in the arithmetic type, through the row's operator[].
template <class R, class C>
__device__ __forceinline__ void row_dens(const R& f, C& da, C& db)
{
    da = f[0];
    db = f[9];
#pragma unroll
    for (int q = 1; q < 9; ++q) { da += f[q]; db += f[9 + q]; }
}
template <class R, class C>
__device__ __forceinline__ void row_mom(const R& f, C& jx, C& jy)
{
    jx = (f[1] - f[3] + f[5] - f[6] - f[7] + f[8]) + (f[10] - f[12] + f[14] - f[15] - f[16] + f[17]);
    jy = (f[2] - f[4] + f[5] + f[6] - f[7] - f[8]) + (f[11] - f[13] + f[14] + f[15] - f[16] - f[17]);
}

// FP16 halves enter FP32 sums through the mixed-precision multiply-add
// v_fma_mix_f32 (an operand may be the low or high FP16 half of a VGPR): the
// widening is exact and a*1 + c rounds once, so each step equals the FP32 add
// of the converted value bit for bit, without the conversion instruction.
// mix_acc: x + s h, mix_pair: a + s b, mix_dev: h - x (s = +1 or -1; h, a, b
// the halves H, HA, HB of the packed pairs).
template <int H, bool NEG>
__device__ __forceinline__ float mix_acc(unsigned p, float x)
{
    float r;
    if constexpr (NEG && H)
        asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(p), "v"(x));
    else if constexpr (NEG)
        asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[0,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(p), "v"(x));
    else if constexpr (H)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(p), "v"(x));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[0,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(p), "v"(x));
    return r;
}
template <int HA, int HB, bool NEG>
__device__ __forceinline__ float mix_pair(unsigned a, unsigned b)
{
    float r;
    if constexpr (NEG)
        asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[%c3,0,%c4] op_sel_hi:[1,0,1]"
            : "=v"(r) : "v"(b), "v"(a), "n"(HB), "n"(HA));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[%c3,0,%c4] op_sel_hi:[1,0,1]"
            : "=v"(r) : "v"(b), "v"(a), "n"(HB), "n"(HA));
    return r;
}
template <int H>
__device__ __forceinline__ float mix_dev(unsigned p, float x)
{
    float r;
    if constexpr (H)
        asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(p), "v"(x));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel:[0,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(p), "v"(x));
    return r;
}

template <class P> struct Row<P, false> {
    using C = typename P::C;
    C v[18];
    __device__ __forceinline__ C operator[](int q) const { return v[q]; }
    __device__ __forceinline__ void dens(C& da, C& db) const { row_dens(*this, da, db); }
    __device__ __forceinline__ void mom(C& jx, C& jy) const { row_mom(*this, jx, jy); }
    __device__ __forceinline__ C dev(int q, C x) const { return v[q] - x; }
    __device__ __forceinline__ C post(int q, C w, C t) const { return v[q] - w * t; }   // S = C
    // Planes are stored shifted in x by c_ix: population q of the lane's node
    // sits one column left (c_ix = +1: vl), in place (vc) or one column right
    // (c_ix = -1: vr).  so: uniform SGPR byte offset; v*: per-lane byte offsets.
    __device__ __forceinline__ void load(rsrc_t r0, rsrc_t r1, unsigned vl, unsigned vc, unsigned vr, unsigned so,
                                         unsigned pbytes)
    {
#pragma unroll
        for (int q = 0; q < 18; ++q) {
            const int cx = CX[q % 9];
            v[q] = ld<P>(q < 9 ? r0 : r1, cx > 0 ? vl : (cx < 0 ? vr : vc), so + (q % 9) * pbytes);
        }
    }
};

template <class P> struct Row<P, true> {
    using S = typename P::S;
    typedef S S2 __attribute__((ext_vector_type(2)));
    S2 v[9];
    static constexpr bool MIX = std::is_same<S, _Float16>::value;
    __device__ __forceinline__ float operator[](int q) const
    {
        return (float)((q & 1) ? v[q >> 1].y : v[q >> 1].x);
    }
    template <int Q> __device__ __forceinline__ unsigned u() const { return __builtin_bit_cast(unsigned, v[Q >> 1]); }
    template <int Q, bool NEG> __device__ __forceinline__ float acc(float x) const
    {
        return mix_acc<Q & 1, NEG>(u<Q>(), x);
    }
    template <int QA, int QB, bool NEG> __device__ __forceinline__ float pair() const
    {
        return mix_pair<QA & 1, QB & 1, NEG>(u<QA>(), u<QB>());
    }
    __device__ __forceinline__ void dens(float& da, float& db) const
    {
        if constexpr (MIX) {
            da = acc<8, false>(acc<7, false>(acc<6, false>(acc<5, false>(
                acc<4, false>(acc<3, false>(acc<2, false>(pair<0, 1, false>())))))));
            db = acc<17, false>(acc<16, false>(acc<15, false>(acc<14, false>(
                acc<13, false>(acc<12, false>(acc<11, false>(pair<9, 10, false>())))))));
        } else {
            row_dens(*this, da, db);
        }
    }
    __device__ __forceinline__ void mom(float& jx, float& jy) const
    {
        if constexpr (MIX) {
            const float ax = acc<8, false>(acc<7, true>(acc<6, true>(acc<5, false>(pair<1, 3, true>()))));
            const float bx = acc<17, false>(acc<16, true>(acc<15, true>(acc<14, false>(pair<10, 12, true>()))));
            const float ay = acc<8, true>(acc<7, true>(acc<6, false>(acc<5, false>(pair<2, 4, true>()))));
            const float by = acc<17, true>(acc<16, true>(acc<15, false>(acc<14, false>(pair<11, 13, true>()))));
            jx = ax + bx;
            jy = ay + by;
        } else {
            row_mom(*this, jx, jy);
        }
    }
    __device__ __forceinline__ float dev(int q, float x) const
    {
        if constexpr (MIX) {
            const unsigned p = __builtin_bit_cast(unsigned, v[q >> 1]);
            return (q & 1) ? mix_dev<1>(p, x) : mix_dev<0>(p, x);
        } else {
            return (*this)[q] - x;
        }
    }
    // the FP32 value rounded to the storage format (FP16 through to_store:
    // the compiler would otherwise fuse the conversion into the multiply-add
    // at some stores and not at others; BF16 has no such fusion)
    __device__ __forceinline__ S post(int q, float w, float t) const
    {
        if constexpr (MIX) return to_store<S>((*this)[q] - w * t);
        else return (S)((*this)[q] - w * t);
    }
    __device__ __forceinline__ void load(rsrc_t r0, rsrc_t r1, unsigned vl, unsigned vc, unsigned vr, unsigned so,
                                         unsigned pbytes)
    {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int q0 = 2 * k, q1 = 2 * k + 1;
            const int c0 = CX[q0 % 9], c1 = CX[q1 % 9];
            v[k].x = bload<S>(q0 < 9 ? r0 : r1, c0 > 0 ? vl : (c0 < 0 ? vr : vc),
                              (unsigned)__builtin_amdgcn_readfirstlane((int)(so + (q0 % 9) * pbytes)));
            v[k].y = bload<S>(q1 < 9 ? r0 : r1, c1 > 0 ? vl : (c1 < 0 ? vr : vc),
                              (unsigned)__builtin_amdgcn_readfirstlane((int)(so + (q1 % 9) * pbytes)));
        }
    }
};

// Deviation of the pseudo-potential from its value at the reference density:
// psi(rho_ref + d) - psi(rho_ref) = -E expm1(-d/rho0), E = rho0 exp(-rho_ref/rho0).
__device__ __forceinline__ float dpsi_of(float d, float e, float inv_rho0)
{
    return -e * expm1f(-d * inv_rho0);
}
__device__ __forceinline__ double dpsi_of(double d, double e, double inv_rho0)
{
    return -e * expm1(-d * inv_rho0);
}
// The same deviation as E (1 - 2^(-d log2(e) / rho0)) with the hardware
// base-2 exponential (one transcendental and two multiply-adds instead of the
// ~24 instructions of expm1f).  Its absolute error is a few 1e-8 of E: far
// below the storage rounding of the 16-bit forms, about one FP32 rounding of
// the populations per step in the FP32 moment form.  The forms whose step is
// bound by arithmetic use it (fast_psi); FP32 and FP64 population storage
// keep expm1.
template <class P>
__device__ __forceinline__ typename P::C dpsi(typename P::C d, typename P::C e, typename P::C inv_rho0)
{
    if constexpr (P::fast_psi) {
        const float t = __builtin_amdgcn_exp2f(d * (-1.4426950408889634f * inv_rho0));
        return e - e * t;
    } else {
        return dpsi_of(d, e, inv_rho0);
    }
}

// Reciprocal: the hardware approximation (<= 1 ulp) in FP32, exact division in FP64.
__device__ __forceinline__ float rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double rcp(double v) { return 1.0 / v; }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// A 32-bit lane move by DPP control CTRL applied to both halves of an FP64
// value (all 64 lanes active).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = __builtin_amdgcn_update_dpp(0u, (unsigned)b, CTRL, 0xF, 0xF, false);
    const unsigned hi = __builtin_amdgcn_update_dpp(0u, (unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The wave-wide sums of two vectors at once (FP64, all 64 lanes active),
// without the LDS crossbar: the sum of d0 ends in lanes 0..31, of d1 in lanes
// 32..63.  The gfx950 row swap v_permlane32_swap exchanges the upper half of
// d0 with the lower half of d1, so one addition does the lane-distance-32
// step of both; v_permlane16_swap then pairs 16-lane rows; the rest is the
// xor butterfly over lane distances 1 and 2 (DPP quad permutations), then 4
// and 8 (the half-row and row mirrors: after the first steps every lane of a
// quad, then of an 8-lane group, holds the same value, so the mirror's
// partner holds what the xor partner holds).  About half the work of two
// separate wave sums.
__device__ __forceinline__ double wave_sum2_dpp(double d0, double d1)
{
    auto lo = [](double x) { return (unsigned)__builtin_bit_cast(unsigned long long, x); };
    auto hi = [](double x) { return (unsigned)(__builtin_bit_cast(unsigned long long, x) >> 32); };
    auto mk = [](unsigned l, unsigned h) { return __builtin_bit_cast(double, ((unsigned long long)h << 32) | l); };
    // first result: d0's lower half, then d1's lower half moved up; second:
    // d0's upper half moved down, then d1's upper half
    const auto l32 = __builtin_amdgcn_permlane32_swap(lo(d0), lo(d1), false, false);
    const auto h32 = __builtin_amdgcn_permlane32_swap(hi(d0), hi(d1), false, false);
    double v = mk(l32[0], h32[0]) + mk(l32[1], h32[1]);
    // with both operands v: the first result holds, in odd rows, the even row
    // below; the second, in even rows, the odd row above
    const auto l16 = __builtin_amdgcn_permlane16_swap(lo(v), lo(v), false, false);
    const auto h16 = __builtin_amdgcn_permlane16_swap(hi(v), hi(v), false, false);
    const bool odd = (__lane_id() >> 4) & 1;
    v += odd ? mk(l16[0], h16[0]) : mk(l16[1], h16[1]);
    v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]: lane l^1
    v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]: lane l^2
    v += dpp_move<0x141>(v);   // row_half_mirror: the other quad of the 8-lane group
    v += dpp_move<0x140>(v);   // row_mirror: the other 8-lane group of the 16-lane row
    return v;
}

// Force stencil sums of one site.  P(dy, dx) and R(dy, dx) return the staged
// (species A, species B) psi and rho deviations of the neighbour at offset
// (dx, dy).  Out: s[0..3] = x and y sums of the psi terms (A, then B) with
// the belt weights and couplings folded in (ks), s[4..7] = x and y sums of the
// belt-1 cross terms on the other species' density (kx); the force follows by
// multiplying with the centre's psi and rho.
//
// PAIR: the antisymmetric pair form.  Offsets c and -c lie in the same shell
// (same weight) and have opposite c, so each pair contributes
// w(c) c [g(x + c) - g(x - c)]: 20 fewer multiply-adds per species and site
// than the plain sum over the offsets, which reads the neighbourhood row by
// row instead.  Both are the same sum in exact arithmetic; the FP32
// population kernels use the row order (with pairs, whose two rows lie in
// ring slots more than 2 KiB apart, the fused kernel measured 2 % slower),
// the others the pair form.
template <bool PAIR, class C, class FP, class FR>
__device__ __forceinline__ void stencil_sums(FP P, FR R, const C* ks0, const C* ks1, C kx1, C kx2, C (&s)[8])
{
    C sxA = 0, syA = 0, sxB = 0, syB = 0, cxA = 0, cyA = 0, cxB = 0, cyB = 0;
    if constexpr (PAIR) {
#pragma unroll
        for (int dy = 2; dy >= 0; --dy) {
#pragma unroll
            for (int dx = -2; dx <= 2; ++dx) {
                if (dy == 0 && dx <= 0) continue;   // one offset of each pair
                const auto a = P(dy, dx), b = P(-dy, -dx);
                const C gA = a.x - b.x, gB = a.y - b.y;
                const int sh = shell_of(dx, dy);
                if (dx != 0) {
                    sxA += (ks0[sh] * (C)dx) * gA;
                    sxB += (ks1[sh] * (C)dx) * gB;
                }
                if (dy != 0) {
                    syA += (ks0[sh] * (C)dy) * gA;
                    syB += (ks1[sh] * (C)dy) * gB;
                }
                if (sh <= 1) {
                    const auto m = R(dy, dx), n = R(-dy, -dx);
                    const C rA = m.y - n.y, rB = m.x - n.x;   // A feels rho_B, B feels rho_A
                    const C kk = (sh == 0) ? kx1 : kx2;
                    if (dx != 0) { cxA += (kk * (C)dx) * rA; cxB += (kk * (C)dx) * rB; }
                    if (dy != 0) { cyA += (kk * (C)dy) * rA; cyB += (kk * (C)dy) * rB; }
                }
            }
            // keep the LDS reads of the outer pairs of stencil rows (dy = 2, 1)
            // next to their multiply-adds, then the centre row (bounds the
            // registers the neighbourhood occupies; one pair at a time exposed
            // more LDS latency: about 1 % on the 16-bit steps)
            if (dy == 1)
                asm volatile("" : "+v"(sxA), "+v"(syA), "+v"(sxB), "+v"(syB), "+v"(cxA), "+v"(cyA),
                             "+v"(cxB), "+v"(cyB)::"memory");
        }
    } else {
#pragma unroll
        for (int dy = -2; dy <= 2; ++dy) {
#pragma unroll
            for (int dx = -2; dx <= 2; ++dx) {
                if (dx == 0 && dy == 0) continue;
                const auto n = P(dy, dx);
                const int sh = shell_of(dx, dy);
                if (dx != 0) {
                    sxA += (ks0[sh] * (C)dx) * n.x;
                    sxB += (ks1[sh] * (C)dx) * n.y;
                }
                if (dy != 0) {
                    syA += (ks0[sh] * (C)dy) * n.x;
                    syB += (ks1[sh] * (C)dy) * n.y;
                }
                if (sh <= 1) {
                    const auto m = R(dy, dx);
                    const C kk = (sh == 0) ? kx1 : kx2;
                    if (dx != 0) { cxA += (kk * (C)dx) * m.y; cxB += (kk * (C)dx) * m.x; }
                    if (dy != 0) { cyA += (kk * (C)dy) * m.y; cyB += (kk * (C)dy) * m.x; }
                }
            }
            // keep the LDS reads of two stencil rows next to their multiply-adds
            // (bounds the registers the neighbourhood occupies; one row at a
            // time exposed more LDS latency: 0.304 against 0.303 ms per step
            // two steps per pass at 4096^2)
            if (dy == -1 || dy == 1)
                asm volatile("" : "+v"(sxA), "+v"(syA), "+v"(sxB), "+v"(syB), "+v"(cxA), "+v"(cyA),
                             "+v"(cxB), "+v"(cyB)::"memory");
        }
    }
    s[0] = sxA; s[1] = syA; s[2] = sxB; s[3] = syB;
    s[4] = cxA; s[5] = cyA; s[6] = cxB; s[7] = cyB;
}

// Work item l of a lattice with n tiles -> its tile, or -1 for a padding item.
// Each lattice's items start at a multiple of 8 and fill a multiple of 8
// slots, and blocks go to the eight XCDs in turn (block b to XCD b mod 8), so
// XCD x runs items x, x + 8, x + 16, ...: they map to the contiguous tiles
// x c .. x c + c - 1 (c = ceil(n / 8), tiles numbered strip-fastest), so
// neighbouring tiles, which share halo rows and columns, share an XCD's L2.
__device__ __forceinline__ int xcd_tile(int l, int n)
{
    const int c = (n + 7) >> 3;
    if (l >= 8 * c) return -1;
    const int lin = (l & 7) * c + (l >> 3);
    return lin < n ? lin : -1;
}

template <class P>
__device__ __forceinline__ int map_row(int r, int ny, int walls)
{
    if (walls) {
        if (r < 0) r = -1 - r;
        else if (r >= ny) r = 2 * ny - 1 - r;
    } else {
        r %= ny;
        if (r < 0) r += ny;
    }
    return r;
}

// ------------------------------------------------------------------ step ---

template <class C> struct V2;
template <> struct V2<float> { using T = float2; };
template <> struct V2<double> { using T = double2; };

// Workgroup barrier that orders LDS only: this wave's LDS reads and writes
// complete (lgkmcnt 0), then s_barrier.  Global loads issued before it stay in
// flight (the row prefetch), and so do direct-to-LDS halo loads: only the wave
// that issued those reads their data, behind its own vmcnt wait.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);   // gfx9 encoding: lgkmcnt(0), vmcnt/expcnt unchanged
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Largest segment (rows per tile).
constexpr int LY_MAX = 256;

// Dynamic LDS of the step kernel: the four halo columns of a segment
// (rows y0-2 .. y1+1), staged only by the formats without the direct-to-LDS
// halo (4-byte storage always has it), and the per-wave row sums of u_x for
// the profile.
template <class P>
__host__ __device__ constexpr size_t step_halo_lds(int ly)
{
    return sizeof(typename P::S) == 4 ? 0 : sizeof(typename P::C) * 4 * 4 * (size_t)(ly + 4);
}
template <class P>
__host__ __device__ constexpr size_t step_dyn_lds(int bx, int ly)
{
    return step_halo_lds<P>(ly) + sizeof(double) * (size_t)(bx / 64) * ly;
}

template <int BX, class P>
__global__ void __launch_bounds__(BX)
k_step(char* __restrict__ base, const LatDesc* __restrict__ descs, const int* __restrict__ tiles, int ntot,
       int src)
{
    using S = typename P::S;
    using C = typename P::C;
    using C2 = typename V2<C>::T;
    using C4 = typename V4<C>::T;
    // Six-row rings of (dpsi_A, dpsi_B) and (drho_A, drho_B); columns x0-2 .. x0+BX+1.
    __shared__ C2 ringP[6][BX + 4];
    __shared__ C2 ringR[6][BX + 4];
    extern __shared__ __align__(16) char dyn_lds[];
    // The four halo columns of a row arrive by direct buffer-to-LDS dword
    // loads (no registers), one row ahead, in a four-row ring.  4-byte
    // storage: one dword per halo column and plane, taken from the plane's
    // shifted column.  2-byte storage: three column pairs on each side,
    // x0-4 .. x0+1 and x0+BX-2 .. x0+BX+3, which hold the four halo columns
    // under every shift (needs an even nx).  Otherwise the halo of a whole
    // tile is staged once per tile.
    constexpr bool DMA32 = (sizeof(S) == 4), DMA16 = (sizeof(S) == 2);
    using HT = std::conditional_t<DMA16, unsigned short, unsigned>;
    __shared__ HT hst[(DMA32 || DMA16) ? 4 : 1][18][DMA16 ? 12 : 4];

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    // The halo work of row r (its direct-to-LDS loads and the halo densities)
    // falls to wave r mod HW, so that it spreads over the SIMDs instead of
    // gating every row's barrier on wave 0 (2-3 % on 16-bit storage).  Blocks
    // of eight waves keep it on wave 0 (HW = 1), which measured faster there.
    // The wave that issues a row's halo loads is the one that reads them back,
    // and rows r and r + 4, which share a slot of the four-row halo ring, have
    // the same halo wave: the prologue reuses slots without a barrier between.
    constexpr int HW = BX / 64 <= 4 ? BX / 64 : 1;
    auto halo_wave = [&](int r) { return r & (HW - 1); };

    for (int w = blockIdx.x; w < ntot; w += gridDim.x) {
        const int L = tiles[w];          // owning lattice, -1 for alignment padding
        if (L < 0) continue;
        const LatDesc& d = descs[L];
        const int lin = xcd_tile(w - d.item_begin, d.nitems);
        if (lin < 0) continue;
        const int nstrip = d.nstrip;
        const int strip = lin % nstrip, seg = lin / nstrip;
        const int nx = d.nx, ny = d.ny, pitch = d.pitch, walls = d.walls;
        const long long plane = d.plane;
        const int x0 = strip * BX;
        const int y0 = seg * d.ly;
        const int y1 = min(y0 + d.ly, ny);
        const unsigned x = (unsigned)(x0 + tid);
        const bool valid = x < (unsigned)nx;
        const unsigned xc = x % (unsigned)nx;
        const unsigned xp = (xc + 1 == (unsigned)nx) ? 0u : xc + 1;
        const unsigned xm = (xc == 0) ? (unsigned)(nx - 1) : xc - 1;

        const C tau = coef<C>(d.tau, d.ftau), omega = coef<C>(d.omega, d.fomega);
        const C inv_rho0 = coef<C>(d.inv_rho0, d.finv_rho0);
        C ks0[5], ks1[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            ks0[k] = coef<C>(d.ks[0][k], d.fks[0][k]);
            ks1[k] = coef<C>(d.ks[1][k], d.fks[1][k]);
        }
        const C kx1 = coef<C>(d.kx[0], d.fkx[0]), kx2 = coef<C>(d.kx[1], d.fkx[1]);
        const C u_top = coef<C>(d.u_top, d.fu_top), u_bot = coef<C>(d.u_bot, d.fu_bot);
        const C rref0 = coef<C>(d.rref[0], d.frref[0]), rref1 = coef<C>(d.rref[1], d.frref[1]);
        const C pref0 = coef<C>(d.psiref[0], d.fpsiref[0]), pref1 = coef<C>(d.psiref[1], d.fpsiref[1]);
        const C e0 = coef<C>(d.epsi[0], d.fepsi[0]), e1 = coef<C>(d.epsi[1], d.fepsi[1]);

        // One buffer resource per species and buffer; byte offsets stay below 2^32.
        const unsigned sbytes = (unsigned)(9 * plane * (long long)sizeof(S));
        const char* fin = base + d.off_f[src];
        const char* fout = base + d.off_f[src ^ 1];
        const rsrc_t rin0 = make_rsrc(fin, sbytes), rin1 = make_rsrc(fin + sbytes, sbytes);
        const rsrc_t rout0 = make_rsrc(fout, sbytes), rout1 = make_rsrc(fout + sbytes, sbytes);
        const int es = (int)sizeof(S);
        const unsigned vc = xc * es, vp = xp * es, vm = xm * es;   // columns x, x+1, x-1
        const unsigned pbytes = (unsigned)(plane * es), rbytes = (unsigned)(pitch * es);
        const bool dma_halo = DMA32 || (DMA16 && (nx % 2) == 0);
        // DMA lanes (of the row's halo wave).  4-byte storage, lanes 0..3: halo column x0-2, x0-1,
        // x0+BX, x0+BX+1 and its left and right neighbours (byte offsets).
        // 2-byte storage, lanes 0..5: the pair starts x0-4, x0-2, x0,
        // x0+BX-2, x0+BX, x0+BX+2.
        auto wrap = [&](int c) { c %= nx; return c < 0 ? c + nx : c; };
        unsigned vh = 0, vhl = 0, vhr = 0;
        if (lane < 6) {
            const int hc = DMA16 ? ((lane < 3) ? x0 - 4 + 2 * lane : x0 + BX - 8 + 2 * lane)
                                 : ((lane < 2) ? x0 - 2 + lane : x0 + BX + lane - 2);
            vh = (unsigned)wrap(hc) * es;
            vhl = (unsigned)wrap(hc - 1) * es;
            vhr = (unsigned)wrap(hc + 1) * es;
        }
        const int ndma = DMA16 ? 6 : 4;
        double* __restrict__ stress = (double*)(base + d.off_stress);
        double* __restrict__ prof = d.off_prof >= 0 ? (double*)(base + d.off_prof) : nullptr;
        const double* __restrict__ body = d.off_body >= 0 ? (const double*)(base + d.off_body) : nullptr;
        C4* halo = (C4*)dyn_lds;                                     // [(ly + 4) * 4], unused by DMA32
        double* profS = (double*)(dyn_lds + step_halo_lds<P>(d.ly));  // [BX/64][ly]
        C mom_b = 0, mom_t = 0;   // wall momentum of this thread's column, summed over the segment

        // 18 deviations of row r (any row; mapped through the walls or the
        // periodic wrap) at column byte offset voff.
        using R = Row<P>;
        // 18 deviations of row r (uniform across the block; mapped through the
        // walls or the periodic wrap) at column byte offset voff.
        auto load = [&](R& fr, int r) {
            const unsigned ro = (unsigned)(map_row<P>(r, ny, walls) * rbytes);
            fr.load(rin0, rin1, vm + ro, vc + ro, vp + ro, 0, pbytes);
        };
        // The same for a row and column that differ between lanes: both go into
        // the per-lane offsets and the SGPR offset keeps only the uniform plane.
        auto load_lane = [&](R& fr, int r, int col) {
            const unsigned ro = (unsigned)(map_row<P>(r, ny, walls) * rbytes);
            fr.load(rin0, rin1, (unsigned)wrap(col - 1) * es + ro, (unsigned)col * es + ro,
                    (unsigned)wrap(col + 1) * es + ro, 0, pbytes);
        };
        auto dens = [&](const R& fr, C& da, C& db) { fr.dens(da, db); };

        // Halo columns x0-2, x0-1, x0+BX, x0+BX+1 for every row of the segment
        // (formats without the direct-to-LDS halo).
        if (!dma_halo) {
            const int nh = (y1 - y0 + 4) * 4;
            for (int s = tid; s < nh; s += BX) {
                const int c = s & 3, rr = s >> 2;
                const int hc = wrap((c < 2) ? x0 - 2 + c : x0 + BX + c - 2);
                R h;
                load_lane(h, y0 - 2 + rr, hc);
                C da, db;
                dens(h, da, db);
                C4 v;
                v.x = dpsi<P>(da, e0, inv_rho0);
                v.y = dpsi<P>(db, e1, inv_rho0);
                v.z = da;
                v.w = db;
                halo[rr * 4 + c] = v;
            }
        }
        if (!dma_halo) lds_barrier();

        // Issue the direct-to-LDS loads of row r's four halo columns (lanes 0..3 of
        // the row's halo wave).
        auto halo_fetch = [&](int r) {
            if constexpr (DMA32 || DMA16) {
                if (dma_halo && wave == halo_wave(r) && lane < ndma) {
                    const unsigned ro = (unsigned)(map_row<P>(r, ny, walls) * rbytes);
                    // the slot's LDS base, opaque to the compiler (one scalar
                    // add per load instead of hoisted, spilled destinations)
                    __attribute__((address_space(3))) char* hb =
                        (__attribute__((address_space(3))) char*)&hst[r & 3][0][0];
                    asm volatile("" : "+s"(hb));
#pragma unroll
                    for (int q = 0; q < 18; ++q) {
                        const int cx = CX[q % 9];
                        const unsigned vo = ro + ((DMA32 && cx > 0) ? vhl : ((DMA32 && cx < 0) ? vhr : vh));
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(
                            q < 9 ? rin0 : rin1, (__attribute__((address_space(3))) void*)(hb + q * sizeof(hst[0][0])),
                            4, vo, __builtin_amdgcn_readfirstlane((int)((q % 9) * pbytes)), 0, 0);
                    }
                }
            }
        };
        // Plane q of halo column tid (0..3) from the DMA ring.  2-byte storage:
        // the 12-element window row holds columns x0-4 .. x0+1 (elements 0..5)
        // and x0+BX-2 .. x0+BX+3 (6..11); halo column tid under shift c_ix is
        // element hb16 - c_ix (hb16: the unshifted element of the column).
        const int hb16 = (lane < 2) ? 2 + lane : 6 + lane;
        auto hval = [&](int r, int q) -> C {
            if constexpr (DMA32) {
                return (C)__builtin_bit_cast(float, hst[r & 3][q][lane]);
            } else if constexpr (DMA16) {
                return (C)__builtin_bit_cast(S, hst[r & 3][q][hb16 - CX[q % 9]]);
            } else {
                return (C)0;
            }
        };

        // Stage row r (populations already in fr): (dpsi, drho) into the ring,
        // plus the four halo entries (lanes 0..3 of the row's halo wave).
        auto stage = [&](const R& fr, int r) {
            const int slot = __builtin_amdgcn_readfirstlane((r - y0 + 2) % 6);
            C da, db;
            dens(fr, da, db);
            C2 pv, rv;
            pv.x = dpsi<P>(da, e0, inv_rho0);
            pv.y = dpsi<P>(db, e1, inv_rho0);
            rv.x = da;
            rv.y = db;
            ringP[slot][tid + 2] = pv;
            ringR[slot][tid + 2] = rv;
            if (wave == halo_wave(r) && lane < 4) {
                const int hidx = (lane < 2) ? lane : BX + lane;
                C2 a, b;
                if (dma_halo) {
                    // the row's own loads have completed (da, db above); the halo
                    // loads were issued before them, so their data is in LDS
                    asm volatile("" ::"v"(da), "v"(db) : "memory");
                    C ha = hval(r, 0), hb = hval(r, 9);
#pragma unroll
                    for (int q = 1; q < 9; ++q) {
                        ha += hval(r, q);
                        hb += hval(r, 9 + q);
                    }
                    a.x = dpsi<P>(ha, e0, inv_rho0);
                    a.y = dpsi<P>(hb, e1, inv_rho0);
                    b.x = ha;
                    b.y = hb;
                } else {
                    const C4 hv = halo[(r - y0 + 2) * 4 + lane];
                    a.x = hv.x;
                    a.y = hv.y;
                    b.x = hv.z;
                    b.y = hv.w;
                }
                ringP[slot][hidx] = a;
                ringR[slot][hidx] = b;
            }
        };

        // Collide row y (populations in f, neighbourhood in LDS) and push.
        auto collide = [&](const R& f, int y) {
            int sl[5];
            sl[0] = __builtin_amdgcn_readfirstlane((y - y0) % 6);
#pragma unroll
            for (int k = 1; k < 5; ++k) sl[k] = (sl[k - 1] == 5) ? 0 : sl[k - 1] + 1;
            C ss[8];
            stencil_sums<!std::is_same<S, float>::value, C>(
                [&](int dy, int dx) { return ringP[sl[dy + 2]][tid + 2 + dx]; },
                [&](int dy, int dx) { return ringR[sl[dy + 2]][tid + 2 + dx]; }, ks0, ks1, kx1, kx2, ss);
            const C sxA = ss[0], syA = ss[1], sxB = ss[2], syB = ss[3];
            const C cxA = ss[4], cyA = ss[5], cxB = ss[6], cyB = ss[7];
            const C2 p0 = ringP[sl[2]][tid + 2];
            const C2 r0c = ringR[sl[2]][tid + 2];
            // absolute densities and potentials of the centre site
            const C ra = rref0 + r0c.x, rb = rref1 + r0c.y;
            const C pa = pref0 + p0.x, pb = pref1 + p0.y;
            const C FxA = -pa * sxA - ra * cxA, FyA = -pa * syA - ra * cyA;
            const C FxB = -pb * sxB - rb * cxB, FyB = -pb * syB - rb * cyB;

            C jx, jy;
            f.mom(jx, jy);
            const C inv_rho = rcp(ra + rb);
            const C ux = jx * inv_rho, uy = jy * inv_rho;
            // external body force of the row, shared by density: the same
            // acceleration F_x(y) / (rho_A + rho_B) for both species
            const C gx = (body != nullptr) ? (C)body[y] * inv_rho : (C)0;

            if (prof != nullptr && x0 + 64 * wave < nx) {    // wave-uniform condition
                double su = valid ? (double)ux : 0.0;
                su = wave_sum(su);
                if ((tid & 63) == 0) profS[wave * d.ly + (y - y0)] = su;
            }

            const bool bot = walls && (y == 0);
            const bool top = walls && (y == ny - 1);
            // byte offsets of the destination rows y-1, y, y+1 (periodic wrap in y;
            // at a wall the row beyond it is never written).  The push is in y
            // only: every store goes to the lane's own column, the x part of the
            // move happens when the next step loads the shifted planes.
            const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
            const unsigned vrow_m = (unsigned)(ym * rbytes), vrow_0 = (unsigned)(y * rbytes),
                           vrow_p = (unsigned)(yp * rbytes);
            // BGK relaxation of the deviations towards
            // f^eq_i - w_i rho_ref = w_i [drho + rho (3 c.v + 4.5 (c.v)^2 - 1.5 v.v)],
            // then the push of species s to the neighbours (bounce-back at walls).
            auto relax_push = [&](int s, C rs, C drs, C Fx, C Fy) {
                const C inv = rcp(rs);
                const C vx = ux + tau * (Fx * inv + gx);
                const C vy = uy + tau * Fy * inv;
                const C usq = (C)1.5 * (vx * vx + vy * vy);
                const C r0 = rs * (C)(4.0 / 9.0), r1 = rs * (C)(1.0 / 9.0), r2 = rs * (C)(1.0 / 36.0);
                const C d1 = drs * (C)(1.0 / 9.0), d2 = drs * (C)(1.0 / 36.0);
                const int o = 9 * s;
                // t_i = f_i - f^eq_i; the post-collision value f_i - omega t_i
                // is stored rounded once to the storage format (post); the
                // wall rows also use it in the arithmetic type (fs)
                C t[9];
                t[0] = f.dev(o + 0, drs * (C)(4.0 / 9.0) - r0 * usq);
                auto pair = [&](int ip, int im, C rw, C dw, C cu) {
                    const C sym = dw + rw * ((C)4.5 * cu * cu - usq);
                    const C anti = rw * ((C)3 * cu);
                    t[ip] = f.dev(o + ip, sym + anti);
                    t[im] = f.dev(o + im, sym - anti);
                };
                pair(1, 3, r1, d1, vx);
                pair(2, 4, r1, d1, vy);
                pair(5, 7, r2, d2, vx + vy);
                pair(6, 8, r2, d2, vy - vx);
                if (!valid) return;
                // the nine stored values (post), before any wall branch; the
                // wall rows also use them in the arithmetic type (fs)
                S ps[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) ps[i] = f.post(o + i, omega, t[i]);
                auto fs = [&](int i) -> C { return f[o + i] - omega * t[i]; };
                const rsrc_t ro = (s == 0) ? rout0 : rout1;
                // non-temporal stores: the launch never reads what it writes
                // (1.3-2 % faster per step at 4096^2; the two-step kernel's
                // stores ran slower with this policy)
                if (!(bot || top)) {
                    // interior row: push to rows y-1, y, y+1 (periodic wrap)
#pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        const int cy = CY[i];
                        const unsigned vrow = (cy < 0) ? vrow_m : (cy > 0 ? vrow_p : vrow_0);
                        st_s<P, CP_NT>(ro, vrow + vc, i * pbytes, ps[i]);
                    }
                    return;
                }
                // wall row: a population leaving through the wall returns to this
                // node as OPP[i]; in the shifted layout that slot is column x + c_ix
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const int cx = CX[i], cy = CY[i];
                    const unsigned vback = (cx == 0) ? vc : (cx > 0 ? vp : vm);
                    if ((cy < 0 && bot) || (cy > 0 && top)) {
                        const C uw = (cy < 0) ? u_bot : u_top;
                        if (cx != 0) {
                            const C back = fs(i) - (C)(1.0 / 6.0) * rs * (C)cx * uw;
                            st_s<P, CP_NT>(ro, vrow_0 + vback, OPP[i] * pbytes, to_store<S>(back));
                            if (cy < 0) mom_b += (C)cx * (fs(i) + back);
                            else mom_t += (C)cx * (fs(i) + back);
                        } else {
                            st_s<P, CP_NT>(ro, vrow_0 + vback, OPP[i] * pbytes, ps[i]);
                        }
                    } else {
                        const unsigned vrow = (cy < 0) ? vrow_m : (cy > 0 ? vrow_p : vrow_0);
                        st_s<P, CP_NT>(ro, vrow + vc, i * pbytes, ps[i]);
                    }
                }
            };
            relax_push(0, ra, r0c.x, FxA, FyA);
            relax_push(1, rb, r0c.y, FxB, FyB);
        };

        // Pipeline: entering iteration y, rows y and y+1 are staged and held,
        // row y+2 is loaded (in flight); the iteration stages row y+2, issues
        // row y+3's loads, waits on the LDS barrier and collides row y.
        // A row's halo loads are issued just before its own loads.
        R F0, F1, F2, F3;
        halo_fetch(y0 - 2);
        load(F2, y0 - 2);
        halo_fetch(y0 - 1);
        load(F3, y0 - 1);
        stage(F2, y0 - 2);
        stage(F3, y0 - 1);
        halo_fetch(y0);
        load(F0, y0);
        halo_fetch(y0 + 1);
        load(F1, y0 + 1);
        halo_fetch(y0 + 2);
        load(F2, y0 + 2);
        stage(F0, y0);
        stage(F1, y0 + 1);
        auto iter = [&](int y, const R& fc, const R& fs2, R& fl) {
            stage(fs2, y + 2);
            if (y + 3 <= y1 + 1) {
                halo_fetch(y + 3);
                load(fl, y + 3);
            }
            lds_barrier();
            collide(fc, y);
        };
        for (int y = y0; y < y1; y += 4) {
            iter(y, F0, F2, F3);
            if (y + 1 < y1) iter(y + 1, F1, F3, F0);
            if (y + 2 < y1) iter(y + 2, F2, F0, F1);
            if (y + 3 < y1) iter(y + 3, F3, F1, F2);
        }
        // FP64 accumulators, once per tile: wall momentum of the boundary rows
        // and the per-64-column row sums of u_x.
        if (valid && walls && y0 == 0) stress[xc] += (double)mom_b;
        if (valid && walls && y1 == ny) stress[nx + xc] += (double)mom_t;
        __syncthreads();
        if (prof != nullptr) {
            const int nr = y1 - y0;
            for (int e = tid; e < (BX / 64) * nr; e += BX) {
                const int wv = e / nr, r = e % nr;
                if (x0 + 64 * wv < nx) prof[(long long)(x0 / 64 + wv) * ny + y0 + r] += profS[wv * d.ly + r];
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------ two fused steps ---
//
// Steps t and t+1 in one pass over HBM.  A block of 2 BW threads (BW = 64 NW
// lanes per step) owns a tile of TW output columns x ly2 rows; thread j of
// each half holds column X - XO + j (periodic), X the tile's first output
// column.  Waves 0..NW-1 run step t as k_step does with x0 = X - XO on rows
// y0-3 .. y1+2, but push the post-collision populations into an LDS ring
// instead of HBM.  Waves NW..2NW-1 run step t+1 behind them: in the tick in
// which step t collides row a they pull row a-3's populations from that ring
// (the shift in x of the layout becomes a shift of the ring column) and stage
// its psi/rho, then collide row a-5; they cover rows y0-2 .. y1+1 (staged)
// and y0 .. y1-1 (collided, columns X .. X+TW-1, stored to HBM).  Both halves
// meet at one LDS barrier per tick.  The step t+1 pipeline runs, per row,
// exactly the operations of k_step on values rounded to the storage format,
// so the pair of steps is bitwise that of two k_step launches; each
// population crosses HBM once per two updates.
//
// Column offset XO.  FP32 at 128 lanes per step: 3 (TW = BW - 6); step t's
// stencil reads the two columns beyond each side of its lanes as halo columns
// (direct-to-LDS loads by one wave per row, as in k_step).  The 16-bit forms
// and FP32 at 192 or 256 lanes: 5 (TW = BW - 10); the tile overlaps its
// neighbours by two more columns each side instead, so every wave does the
// same work per tick (no halo wave for the others to wait for at the
// barrier).  At 4096^2 the overlap form ran FP16 about 3 % and BF16 4 %
// faster per step than the halo form, and FP32 at 256 lanes 6 % faster (then
// 1 % faster than the 128-lane halo form); at 128 lanes, where the two more
// columns cost 3 % of the tile, FP32 ran 7 % slower with it.  The edge lanes'
// results feed no output.
//
// The population ring is split by the y direction of the population, since
// each class lives for a different number of ticks (rows r written at
// tick w, read by step t+1 at tick r+3, before that tick's barrier):
//   c_y = +1 (2, 5, 6): written at tick r-1 (row 0 at a bottom wall: tick 0), four rows;
//   c_y =  0 (0, 1, 3): written at tick r, three rows;
//   c_y = -1 (4, 7, 8): written at tick r+1, two rows; at a top wall the
//     populations that return into row ny-1 are computed at tick ny-1 and
//     held in registers until tick ny, when the slot's previous row is read.
// Nine rows of six planes instead of four rows of eighteen; with the
// five-row rho ring (the rho stencil is belt 1 only) three blocks of 128
// FP32 lanes per step fit in a CU's 160 KiB of LDS.
template <class P, int NW> struct Fuse2Geom {
    // FP32 at two waves per step: halo columns by direct-to-LDS loads; the
    // other widths and the 16-bit forms: overlapping tiles
    static constexpr bool HALO = sizeof(typename P::S) == 4 && NW == 2;
    static constexpr int XO = HALO ? 3 : 5;
};
constexpr int pr_class(int cy) { return cy > 0 ? 0 : (cy == 0 ? 1 : 2); }
// index of direction i within its class: (2, 5, 6), (0, 1, 3), (4, 7, 8)
constexpr int pr_k(int i) { return (i == 2 || i == 0 || i == 4) ? 0 : ((i == 5 || i == 1 || i == 7) ? 1 : 2); }

template <class P, int NW>
__global__ void __launch_bounds__(128 * NW)
k_step2(char* __restrict__ base, const LatDesc* __restrict__ descs, const int* __restrict__ tiles, int ntot,
        int src)
{
    constexpr int BW = 64 * NW;
    using S = typename P::S;
    using C = typename P::C;
    using C2 = typename V2<C>::T;
    static_assert(sizeof(S) <= 4, "two fused steps: 4- and 2-byte storage");
    constexpr bool DMA16 = sizeof(S) == 2;   // 2-byte storage: rows packed two per VGPR
    constexpr bool HALO = Fuse2Geom<P, NW>::HALO;
    constexpr int XO = Fuse2Geom<P, NW>::XO;
    constexpr int TW = BW - 2 * XO;
    // psi rings [step][slot][column index j + 2] (six rows), rho rings (five
    // rows); indices 0, 1, BW + 2 and BW + 3 are step t's halo columns (FP32)
    // or stay zero (16-bit)
    __shared__ C2 ringP[2][6][BW + 4];
    __shared__ C2 ringR[2][5][BW + 4];
    // step t+1's input, after streaming: class rows 0..3 (c_y = +1, slot r & 3),
    // 4..6 (c_y = 0), 7..8 (c_y = -1, slot r & 1); six planes (species x the
    // class's three directions); index j + 1, one spare entry each side for the
    // values a wall returns to the neighbouring column
    __shared__ S pring[9][6][BW + 2];
    // FP32: step t's four halo columns by direct-to-LDS loads, four rows (a
    // multiple of the number of halo waves, so rows sharing a slot share a wave)
    constexpr int HS = HALO ? ((NW == 3) ? 6 : 4) : 1;
    __shared__ unsigned hst[HS][18][HALO ? 4 : 1];
    __shared__ C momx[2][BW];          // step t's wall momentum, handed to step t+1

    const int tid = threadIdx.x;
    const int role = __builtin_amdgcn_readfirstlane(tid / BW);   // 0: step t, 1: step t+1
    const int j = tid - role * BW;
    const int wave = __builtin_amdgcn_readfirstlane(j >> 6), lane = tid & 63;
    // FP32: step t's per-row halo work rotates over its waves (rows reach down
    // to y0 - 5 >= -5; 24 is a multiple of NW and HS, so the unsigned
    // remainders are those of r)
    auto halo_wave = [&](int r) { return (int)((unsigned)(r + 24) % (unsigned)NW); };
    auto hslot = [&](int r) { return (int)((unsigned)(r + 24) % (unsigned)HS); };
    // 16-bit: step t's tile overlaps its neighbours by two more columns each
    // side instead of loading halo columns, and the edge lanes read ring
    // entries no lane writes (no output depends on them): zero, so that they
    // compute finite values.  The first tick's barrier orders these stores
    // before any read.  Entries: the 22 psi/rho ring rows (ringP 2 x 6, then
    // ringR 2 x 5) with four each (0, 1, BW + 2, BW + 3), 88 in all, then the
    // 54 population ring rows (9 x 6) with two each (0, BW + 1).
    if constexpr (!HALO)
    for (int e = tid; e < 22 * 4 + 54 * 2; e += 128 * NW) {
        if (e < 88) {
            const int r = e >> 2, c = e & 3, idx = c < 2 ? c : BW + c;
            if (r < 12) ringP[r / 6][r % 6][idx] = C2{(C)0, (C)0};
            else ringR[(r - 12) / 5][(r - 12) % 5][idx] = C2{(C)0, (C)0};
        } else {
            const int r = (e - 88) >> 1;
            pring[r / 6][r % 6][(e & 1) ? BW + 1 : 0] = (S)0;
        }
    }

    for (int w = blockIdx.x; w < ntot; w += gridDim.x) {
        const int L = tiles[w];
        if (L < 0) continue;
        const LatDesc& d = descs[L];
        const int lin = xcd_tile(w - d.item_begin2, d.nitems2);
        if (lin < 0) continue;
        const int nstrip = d.nstrip2;
        const int strip = lin % nstrip, seg = lin / nstrip;
        const int nx = d.nx, ny = d.ny, pitch = d.pitch, walls = d.walls;
        const long long plane = d.plane;
        const int X = strip * TW;
        // nseg2 segments of near-equal height: the first ny mod nseg2 of them
        // one row taller (no short last segment)
        const int sb = ny / d.nseg2, sx = ny - sb * d.nseg2;
        const int y0 = seg * sb + min(seg, sx);
        const int y1 = y0 + sb + (seg < sx ? 1 : 0);
        auto wrap = [&](int c) { c %= nx; return c < 0 ? c + nx : c; };
        const int x0 = X - XO;
        const unsigned xc = (unsigned)wrap(x0 + j);
        const unsigned xp = (xc + 1 == (unsigned)nx) ? 0u : xc + 1;
        const unsigned xm = (xc == 0) ? (unsigned)(nx - 1) : xc - 1;
        // the columns this tile stores and whose wall momentum it counts
        const bool own = j >= XO && j < XO + TW && X + (j - XO) < nx;

        const C tau = coef<C>(d.tau, d.ftau), omega = coef<C>(d.omega, d.fomega);
        const C inv_rho0 = coef<C>(d.inv_rho0, d.finv_rho0);
        C ks0[5], ks1[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            ks0[k] = coef<C>(d.ks[0][k], d.fks[0][k]);
            ks1[k] = coef<C>(d.ks[1][k], d.fks[1][k]);
        }
        const C kx1 = coef<C>(d.kx[0], d.fkx[0]), kx2 = coef<C>(d.kx[1], d.fkx[1]);
        const C u_top = coef<C>(d.u_top, d.fu_top), u_bot = coef<C>(d.u_bot, d.fu_bot);
        const C rref0 = coef<C>(d.rref[0], d.frref[0]), rref1 = coef<C>(d.rref[1], d.frref[1]);
        const C pref0 = coef<C>(d.psiref[0], d.fpsiref[0]), pref1 = coef<C>(d.psiref[1], d.fpsiref[1]);
        const C e0 = coef<C>(d.epsi[0], d.fepsi[0]), e1 = coef<C>(d.epsi[1], d.fepsi[1]);

        const unsigned sbytes = (unsigned)(9 * plane * (long long)sizeof(S));
        const char* fin = base + d.off_f[src];
        const char* fout = base + d.off_f[src ^ 1];
        const rsrc_t rin0 = make_rsrc(fin, sbytes), rin1 = make_rsrc(fin + sbytes, sbytes);
        const rsrc_t rout0 = make_rsrc(fout, sbytes), rout1 = make_rsrc(fout + sbytes, sbytes);
        const int es = (int)sizeof(S);
        const unsigned vc = xc * es, vp = xp * es, vm = xm * es;
        const unsigned pbytes = (unsigned)(plane * es), rbytes = (unsigned)(pitch * es);
        // FP32 halo, lanes 0..3 of the row's halo wave: columns x0-2, x0-1,
        // x0+BW, x0+BW+1 and their left and right neighbours (the planes are
        // stored shifted by c_ix)
        unsigned vh = 0, vhl = 0, vhr = 0;
        if (HALO && lane < 4) {
            const int hc = (lane < 2) ? x0 - 2 + lane : x0 + BW + lane - 2;
            vh = (unsigned)wrap(hc) * es;
            vhl = (unsigned)wrap(hc - 1) * es;
            vhr = (unsigned)wrap(hc + 1) * es;
        }
        double* __restrict__ stress = (double*)(base + d.off_stress);
        const double* __restrict__ body = d.off_body >= 0 ? (const double*)(base + d.off_body) : nullptr;
        // line profile: each wave adds the sum of u_x over its own columns of
        // every collided row of this tile to its partial, per step (state
        // memory is ordinary device memory, where FP64 atomics are native)
        double* __restrict__ prof2 =
            d.off_prof >= 0 ? (double*)(base + d.off_prof) + (long long)d.ngroups * ny : nullptr;
        C mom_b = 0, mom_t = 0;
        // populations returned into row ny - 1 at a top wall, held one tick,
        // already in the storage format (the values k_step stores)
        S held[2][3] = {{(S)0, (S)0, (S)0}, {(S)0, (S)0, (S)0}};

        using R = Row<P>;
        auto load = [&](R& fr, int r) {
            const unsigned ro = (unsigned)(map_row<P>(r, ny, walls) * rbytes);
            fr.load(rin0, rin1, vm + ro, vc + ro, vp + ro, 0, pbytes);
        };
        auto dens = [&](const R& fr, C& da, C& db) { fr.dens(da, db); };
        // ring slots: every row index here is >= y0 - 6, so the operands are
        // non-negative and unsigned remainders (cheaper scalar code) are exact
        auto slot6 = [&](int r) { return __builtin_amdgcn_readfirstlane((int)((unsigned)(r - y0 + 8) % 6u)); };
        auto slot5 = [&](int r) { return __builtin_amdgcn_readfirstlane((int)((unsigned)(r - y0 + 10) % 5u)); };
        // ring row of population class c (pr_class) for row r
        auto prow = [&](int c, int r) {
            return __builtin_amdgcn_readfirstlane(
                c == 0 ? (r & 3) : (c == 1 ? 4 + (int)((unsigned)(r - y0 + 9) % 3u) : 7 + (r & 1)));
        };

        auto halo_fetch = [&](int r) {
            if constexpr (HALO) {
                if (wave == halo_wave(r) && lane < 4) {
                    const unsigned ro = (unsigned)(map_row<P>(r, ny, walls) * rbytes);
                    const int hs = hslot(r);
                    // the slot's LDS base, opaque to the compiler: the destination
                    // of each plane is then one scalar add per load instead of a
                    // value hoisted out of the tick loop (and spilled)
                    __attribute__((address_space(3))) char* hb =
                        (__attribute__((address_space(3))) char*)&hst[hs][0][0];
                    asm volatile("" : "+s"(hb));
#pragma unroll
                    for (int q = 0; q < 18; ++q) {
                        const int cx = CX[q % 9];
                        const unsigned vo = ro + (cx > 0 ? vhl : (cx < 0 ? vhr : vh));
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(
                            q < 9 ? rin0 : rin1, (__attribute__((address_space(3))) void*)(hb + q * sizeof(hst[0][0])),
                            4, vo, __builtin_amdgcn_readfirstlane((int)((q % 9) * pbytes)), 0, 0);
                    }
                }
            }
        };
        // Step t: stage row r (HBM populations in fr) into ring 0, plus (FP32)
        // the four halo entries (lanes 0..3 of the row's halo wave).
        auto stage1 = [&](const R& fr, int r) {
            const int sp = slot6(r), sr = slot5(r);
            C da, db;
            dens(fr, da, db);
            ringP[0][sp][j + 2] = C2{dpsi<P>(da, e0, inv_rho0), dpsi<P>(db, e1, inv_rho0)};
            ringR[0][sr][j + 2] = C2{da, db};
            if constexpr (HALO) {
                if (wave == halo_wave(r) && lane < 4) {
                    // the row's own loads have completed (da, db); its halo loads
                    // were issued before them, so their data is in LDS
                    asm volatile("" ::"v"(da), "v"(db) : "memory");
                    const int hs = hslot(r);
                    auto hval = [&](int q) -> C { return (C)__builtin_bit_cast(float, hst[hs][q][lane]); };
                    C ha = hval(0), hb = hval(9);
#pragma unroll
                    for (int q = 1; q < 9; ++q) {
                        ha += hval(q);
                        hb += hval(9 + q);
                    }
                    const int hidx = (lane < 2) ? lane : BW + lane;
                    ringP[0][sp][hidx] = C2{dpsi<P>(ha, e0, inv_rho0), dpsi<P>(hb, e1, inv_rho0)};
                    ringR[0][sr][hidx] = C2{ha, hb};
                }
            }
        };
        // Step t+1: row r's populations from the LDS ring, pulled in x (column
        // j - c_ix), staged into ring 1.  Beyond a wall the ghost rows are the
        // even mirror: the bottom ones are written with their fluid rows 0 and
        // 1 (staged later), the top ones copy their staged fluid rows.
        auto stage2 = [&](R& fr, int r) {
            const int sp = slot6(r), sr = slot5(r);
            if (walls && r >= ny) {
                const int m = 2 * ny - 1 - r;
                ringP[1][sp][j + 2] = ringP[1][slot6(m)][j + 2];
                ringR[1][sr][j + 2] = ringR[1][slot5(m)][j + 2];
                return;
            }
            if (walls && r < 0) return;
            int pr[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) pr[c] = prow(c, r);
#pragma unroll
            for (int q = 0; q < 18; ++q) {
                const int i = q % 9, s = q / 9;
                const S v = pring[pr[pr_class(CY[i])]][3 * s + pr_k(i)][j + 1 - CX[i]];
                if constexpr (DMA16) {
                    if (q & 1) fr.v[q >> 1].y = v;
                    else fr.v[q >> 1].x = v;
                } else {
                    fr.v[q] = (C)v;
                }
            }
            C da, db;
            dens(fr, da, db);
            const C2 pv = C2{dpsi<P>(da, e0, inv_rho0), dpsi<P>(db, e1, inv_rho0)};
            const C2 rv = C2{da, db};
            ringP[1][sp][j + 2] = pv;
            ringR[1][sr][j + 2] = rv;
            if (walls && r <= 1 && -1 - r >= y0 - 2) {
                ringP[1][slot6(-1 - r)][j + 2] = pv;
                ringR[1][slot5(-1 - r)][j + 2] = rv;
            }
        };

        // Collide row y of step `k` (0: t, pushes into the LDS ring; 1: t+1,
        // stores to HBM).  The arithmetic is k_step's.
        auto collide = [&](const R& f, int y, int k, C& pu) {
            int sl[5], sr[5];
            sl[0] = slot6(y - 2);
            sr[0] = slot5(y - 2);
#pragma unroll
            for (int q = 1; q < 5; ++q) {
                sl[q] = (sl[q - 1] == 5) ? 0 : sl[q - 1] + 1;
                sr[q] = (sr[q - 1] == 4) ? 0 : sr[q - 1] + 1;
            }
            C ss[8];
            stencil_sums<!std::is_same<S, float>::value, C>(
                [&](int dy, int dx) { return ringP[k][sl[dy + 2]][j + 2 + dx]; },
                [&](int dy, int dx) { return ringR[k][sr[dy + 2]][j + 2 + dx]; }, ks0, ks1, kx1, kx2, ss);
            const C sxA = ss[0], syA = ss[1], sxB = ss[2], syB = ss[3];
            const C cxA = ss[4], cyA = ss[5], cxB = ss[6], cyB = ss[7];
            const C2 p0 = ringP[k][sl[2]][j + 2];
            const C2 r0c = ringR[k][sr[2]][j + 2];
            const C ra = rref0 + r0c.x, rb = rref1 + r0c.y;
            const C pa = pref0 + p0.x, pb = pref1 + p0.y;
            const C FxA = -pa * sxA - ra * cxA, FyA = -pa * syA - ra * cyA;
            const C FxB = -pb * sxB - rb * cxB, FyB = -pb * syB - rb * cyB;
            C jx, jy;
            f.mom(jx, jy);
            const C inv_rho = rcp(ra + rb);
            const C ux = jx * inv_rho, uy = jy * inv_rho;
            C gx = (C)0;
            if (body != nullptr) {
                const int yw = ((y % ny) + ny) % ny;   // periodic image of a step-t row (any ny)
                gx = (C)body[yw] * inv_rho;
            }
            if (prof2 != nullptr && y >= y0 && y < y1) {
                // line profile: rows y0, y0+1, ... are collided in consecutive
                // ticks; the first row of each pair holds its own-column u_x
                // in pu, the second sums both rows in one FP64 wave sum (a
                // last unpaired row alone) and adds each row's sum to the
                // wave's partial of (step, strip, wave, row).  Each partial
                // gets one add per launch: a no-return atomic gives the
                // read-modify-write without waiting for the read (which would
                // also wait for every load issued before it, the next rows'
                // populations); no other wave touches the address, so the
                // result is deterministic.
                const C cur = own ? ux : (C)0;
                const bool second = ((y - y0) & 1) != 0;
                if (!second && y + 1 < y1) {
                    pu = cur;
                } else {
                    const double sum = second ? wave_sum2_dpp((double)pu, (double)cur)
                                              : wave_sum2_dpp((double)cur, 0.0);
                    const int yr = second ? y - 1 + (lane >> 5) : y;
                    if ((lane & 31) == 0 && (second || lane == 0))
                        unsafeAtomicAdd(&prof2[((long long)(k * nstrip + strip) * NW + wave) * ny + yr], sum);
                }
            }
            const bool bot = walls && (y == 0);
            const bool top = walls && (y == ny - 1);
            const bool count = own && y >= y0 && y < y1;   // wall momentum owned by this tile
            const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
            const unsigned vrow_m = (unsigned)(ym * rbytes), vrow_0 = (unsigned)(y * rbytes),
                           vrow_p = (unsigned)(yp * rbytes);
            int pr[3][3];   // ring rows of rows y-1, y, y+1 per class
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int dr = -1; dr <= 1; ++dr) pr[c][dr + 1] = prow(c, y + dr);
            auto relax_push = [&](int s, C rs, C drs, C Fx, C Fy) {
                const C inv = rcp(rs);
                const C vx = ux + tau * (Fx * inv + gx);
                const C vy = uy + tau * Fy * inv;
                const C usq = (C)1.5 * (vx * vx + vy * vy);
                const C r0 = rs * (C)(4.0 / 9.0), r1 = rs * (C)(1.0 / 9.0), r2 = rs * (C)(1.0 / 36.0);
                const C d1 = drs * (C)(1.0 / 9.0), d2 = drs * (C)(1.0 / 36.0);
                const int o = 9 * s;
                // t_i = f_i - f^eq_i; stored values as k_step's (post: rounded
                // once to the storage format; fs: the arithmetic type, for the
                // wall rows)
                C t[9];
                t[0] = f.dev(o + 0, drs * (C)(4.0 / 9.0) - r0 * usq);
                auto pair = [&](int ip, int im, C rw, C dw, C cu) {
                    const C sym = dw + rw * ((C)4.5 * cu * cu - usq);
                    const C anti = rw * ((C)3 * cu);
                    t[ip] = f.dev(o + ip, sym + anti);
                    t[im] = f.dev(o + im, sym - anti);
                };
                pair(1, 3, r1, d1, vx);
                pair(2, 4, r1, d1, vy);
                pair(5, 7, r2, d2, vx + vy);
                pair(6, 8, r2, d2, vy - vx);
                // the stored values and the wall rows' fs, as k_step's
                auto fs = [&](int i) -> C { return f[o + i] - omega * t[i]; };
                S ps[9];
                if (sizeof(S) == 2 && k == 0) {
                    // step t's values go to LDS, where the high half of a
                    // packed pair has its own store
#pragma unroll
                    for (int i = 0; i < 8; i += 2) to_store2<S>(fs(i), fs(i + 1), ps[i], ps[i + 1]);
                    ps[8] = f.post(o + 8, omega, t[8]);
                } else {
#pragma unroll
                    for (int i = 0; i < 9; ++i) ps[i] = f.post(o + i, omega, t[i]);
                }
                auto post = [&](int i) -> S { return ps[i]; };
                if (k == 0) {
                    // into the ring: row y + c_iy at the lane's own index; a
                    // population leaving through a wall returns as OPP[i] at
                    // index j + c_ix of row y (the layout's shift, as in HBM)
#pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        const int cx = CX[i], cy = CY[i];
                        if ((cy < 0 && bot) || (cy > 0 && top)) {
                            const C uw = (cy < 0) ? u_bot : u_top;
                            S sback = post(i);
                            if (cx != 0) {
                                const C back = fs(i) - (C)(1.0 / 6.0) * rs * (C)cx * uw;
                                sback = to_store<S>(back);
                                if (count) {
                                    if (cy < 0) mom_b += (C)cx * (fs(i) + back);
                                    else mom_t += (C)cx * (fs(i) + back);
                                }
                            }
                            if (cy < 0) {
                                const int oi = OPP[i];
                                pring[pr[pr_class(CY[oi])][1]][3 * s + pr_k(oi)][j + 1 + cx] = sback;
                            } else {
                                held[s][pr_k(OPP[i])] = sback;   // written at tick ny
                            }
                        } else {
                            pring[pr[pr_class(cy)][cy + 1]][3 * s + pr_k(i)][j + 1] = post(i);
                        }
                    }
                    return;
                }
                if (!own) return;
                const rsrc_t ro = (s == 0) ? rout0 : rout1;
                if (!(bot || top)) {
#pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        const int cy = CY[i];
                        const unsigned vrow = (cy < 0) ? vrow_m : (cy > 0 ? vrow_p : vrow_0);
                        st_s<P>(ro, vrow + vc, i * pbytes, post(i));
                    }
                    return;
                }
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const int cx = CX[i], cy = CY[i];
                    const unsigned vback = (cx == 0) ? vc : (cx > 0 ? vp : vm);
                    if ((cy < 0 && bot) || (cy > 0 && top)) {
                        const C uw = (cy < 0) ? u_bot : u_top;
                        if (cx != 0) {
                            const C back = fs(i) - (C)(1.0 / 6.0) * rs * (C)cx * uw;
                            st_s<P>(ro, vrow_0 + vback, OPP[i] * pbytes, to_store<S>(back));
                            if (cy < 0) mom_b += (C)cx * (fs(i) + back);
                            else mom_t += (C)cx * (fs(i) + back);
                        } else {
                            st_s<P>(ro, vrow_0 + vback, OPP[i] * pbytes, post(i));
                        }
                    } else {
                        const unsigned vrow = (cy < 0) ? vrow_m : (cy > 0 ? vrow_p : vrow_0);
                        st_s<P>(ro, vrow + vc, i * pbytes, post(i));
                    }
                }
            };
            relax_push(0, ra, r0c.x, FxA, FyA);
            relax_push(1, rb, r0c.y, FxB, FyB);
        };
        // The populations a top wall returned into row ny - 1 (directions 4,
        // 7, 8 at index j + c_ix of their source direction 2, 5, 6), written
        // in the tick after that row's collision: row ny - 3, which shares
        // their ring slot, has been read before this tick's barrier.
        auto put_held = [&]() {
            const int pr = prow(2, ny - 1);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                pring[pr][3 * s + pr_k(4)][j + 1] = held[s][pr_k(4)];
                pring[pr][3 * s + pr_k(7)][j + 1 + CX[5]] = held[s][pr_k(7)];
                pring[pr][3 * s + pr_k(8)][j + 1 + CX[6]] = held[s][pr_k(8)];
            }
        };

        // Step t collides rows A0 .. A1-1; tick a stages row a+2 and collides
        // row a of step t, and stages row a-3 and collides row a-5 of step
        // t+1, each half around the same barrier.  The two halves run loops
        // of their own over the same ticks A0 .. T1 with exactly one barrier
        // per tick (the counts match by construction), each with its own
        // rotating register rows.  Step t's prologue stages rows A0-2 .. A0+1
        // and has rows A0 .. A0+2 loaded, as k_step's; its loads run up to
        // row A1+1.
        const int A0 = y0 - 3, A1 = y1 + 3, T1 = y1 + 4;
        R F0, F1, F2, F3;
        if (role == 0) {
            halo_fetch(A0 - 2);
            load(F2, A0 - 2);
            halo_fetch(A0 - 1);
            load(F3, A0 - 1);
            stage1(F2, A0 - 2);
            stage1(F3, A0 - 1);
            halo_fetch(A0);
            load(F0, A0);
            halo_fetch(A0 + 1);
            load(F1, A0 + 1);
            halo_fetch(A0 + 2);
            load(F2, A0 + 2);
            stage1(F0, A0);
            stage1(F1, A0 + 1);
            const bool top_here = walls && ny - 1 >= A0 && ny - 1 < A1;
            auto tick = [&](int a, const R& fc, const R& fs2, R& fl, C& pu) {
                if (a < A1) {
                    stage1(fs2, a + 2);
                    if (a + 3 <= A1 + 1) {
                        halo_fetch(a + 3);
                        load(fl, a + 3);
                    }
                }
                lds_barrier();
                if (a < A1 && (!walls || (a >= 0 && a < ny))) collide(fc, a, 0, pu);
                if (top_here && a == ny) put_held();
            };
            C pu = (C)0;
            for (int a = A0; a <= T1; a += 4) {
                tick(a, F0, F2, F3, pu);
                if (a + 1 <= T1) tick(a + 1, F1, F3, F0, pu);
                if (a + 2 <= T1) tick(a + 2, F2, F0, F1, pu);
                if (a + 3 <= T1) tick(a + 3, F3, F1, F2, pu);
            }
        } else {
            // row a-3 is complete since tick a-2 and visible since the
            // previous barrier; staging it before this tick's barrier
            // balances the two halves (each: stage, barrier, collide).  The
            // row staged in tick a is collided in tick a+2.
            auto tick = [&](int a, const R& fc, R& fs2, C& pu) {
                const int r = a - 3;
                if (r >= y0 - 2 && r <= y1 + 1) stage2(fs2, r);
                lds_barrier();
                const int c = a - 5;
                if (c >= y0 && c < y1) collide(fc, c, 1, pu);
            };
            C pu = (C)0;
            for (int a = A0; a <= T1; a += 4) {
                tick(a, F0, F2, pu);
                if (a + 1 <= T1) tick(a + 1, F1, F3, pu);
                if (a + 2 <= T1) tick(a + 2, F2, F0, pu);
                if (a + 3 <= T1) tick(a + 3, F3, F1, pu);
            }
        }
        // wall momentum in FP64, step t's first, then step t+1's (the order
        // of two single steps)
        if (role == 0) {
            momx[0][j] = mom_b;
            momx[1][j] = mom_t;
        }
        __syncthreads();
        if (role == 1 && own && walls) {
            if (y0 == 0) {
                stress[xc] += (double)momx[0][j];
                stress[xc] += (double)mom_b;
            }
            if (y1 == ny) {
                stress[nx + xc] += (double)momx[1][j];
                stress[nx + xc] += (double)mom_t;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- auxiliary ---

template <class P>
__device__ __forceinline__ double decode(const typename P::S* p, const LatDesc& d, int q)
{
    return d.wref[q] + (double)*p;
}

// Column holding population q of the node in column x: each plane is stored
// shifted in x by its direction's c_ix (periodic), the layout the step kernel
// reads (it pulls in x and pushes in y).
__device__ __forceinline__ int col_of(int x, int q, int nx)
{
    const int c = x - CX[q % 9];
    return c < 0 ? c + nx : (c >= nx ? c - nx : c);
}

// One rounding, to nearest-even, of an FP64 value to the storage format.  The
// 16-bit formats pass through FP32 rounded to odd (truncated, last bit set if
// anything was cut off): with at least two more significant bits than the
// target, that leaves a single correct rounding (Boldo and Melquiond, rounding
// to odd, IEEE Trans. Computers 57(4), 2008); a plain FP32 step would round
// twice.
template <class S> __device__ __forceinline__ S to_storage(double x) { return (S)x; }
__device__ __forceinline__ float odd_f32(double x)
{
    float t = __double2float_rz(x);
    if ((double)t != x) t = __builtin_bit_cast(float, __builtin_bit_cast(unsigned, t) | 1u);
    return t;
}
template <> __device__ __forceinline__ _Float16 to_storage<_Float16>(double x) { return (_Float16)odd_f32(x); }
template <> __device__ __forceinline__ __bf16 to_storage<__bf16>(double x) { return (__bf16)odd_f32(x); }

// f_is(r, 0) = f^eq_i(rho_s(r), u(r)), evaluated in FP64 and rounded once to
// the storage format.
template <class P>
__global__ void k_init(char* __restrict__ base, const LatDesc* __restrict__ dd, int buf,
                       const double* __restrict__ ra, const double* __restrict__ rb,
                       const double* __restrict__ ux, const double* __restrict__ uy)
{
    using S = typename P::S;
    const LatDesc& d = *dd;
    const long long n = (long long)d.nx * d.ny;
    const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    S* f = (S*)(base + d.off_f[buf]);
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / d.nx), x = (int)(k % d.nx);
        const double u = ux ? ux[k] : 0.0, v = uy ? uy[k] : 0.0;
        const double uu = u * u + v * v;
        S* out = f + (long long)y * d.pitch;
        for (int s = 0; s < 2; ++s) {
            const double rho = s == 0 ? ra[k] : rb[k];
            for (int i = 0; i < 9; ++i) {
                const double cu = CX[i] * u + CY[i] * v;
                const double feq = W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                out[(9 * s + i) * d.plane + col_of(x, i, d.nx)] = to_storage<S>(feq - d.wref[9 * s + i]);
            }
        }
    }
}

// Densities and barycentric velocity of the stored populations, in FP64.
template <class P>
__global__ void k_fields(char* __restrict__ base, const LatDesc* __restrict__ dd, int buf,
                         double* __restrict__ ra, double* __restrict__ rb,
                         double* __restrict__ ux, double* __restrict__ uy)
{
    using S = typename P::S;
    const LatDesc& d = *dd;
    const long long n = (long long)d.nx * d.ny;
    const S* f = (const S*)(base + d.off_f[buf]);
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / d.nx), x = (int)(k % d.nx);
        const S* in = f + (long long)y * d.pitch;
        double rho[2] = {0, 0}, jx = 0, jy = 0;
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < 9; ++i) {
                const double v = decode<P>(in + (9 * s + i) * d.plane + col_of(x, i, d.nx), d, 9 * s + i);
                rho[s] += v;
                jx += v * CX[i];
                jy += v * CY[i];
            }
        if (ra) ra[k] = rho[0];
        if (rb) rb[k] = rho[1];
        if (ux) ux[k] = jx / (rho[0] + rho[1]);
        if (uy) uy[k] = jy / (rho[0] + rho[1]);
    }
}

template <class P>
__global__ void k_export(char* __restrict__ base, const LatDesc* __restrict__ dd, int buf, int q,
                         double* __restrict__ out)
{
    using S = typename P::S;
    const LatDesc& d = *dd;
    const long long n = (long long)d.nx * d.ny;
    const S* f = (const S*)(base + d.off_f[buf]);
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / d.nx), x = (int)(k % d.nx);
        out[k] = decode<P>(f + (long long)y * d.pitch + col_of(x, q, d.nx) + q * d.plane, d, q);
    }
}

constexpr int RED_THREADS = 256;

// Per-block FP64 partial sums of rho_A, rho_B, j_x, j_y and of the count of
// sites whose density is non-finite or non-positive.
template <class P>
__global__ void __launch_bounds__(RED_THREADS)
k_sums(char* __restrict__ base, const LatDesc* __restrict__ dd, int buf, double* __restrict__ partials)
{
    using S = typename P::S;
    const LatDesc& d = *dd;
    const long long n = (long long)d.nx * d.ny;
    const S* f = (const S*)(base + d.off_f[buf]);
    double acc[5] = {0, 0, 0, 0, 0};
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / d.nx), x = (int)(k % d.nx);
        const S* in = f + (long long)y * d.pitch;
        double rho[2] = {0, 0};
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < 9; ++i) {
                const double v = decode<P>(in + (9 * s + i) * d.plane + col_of(x, i, d.nx), d, 9 * s + i);
                rho[s] += v;
                acc[2] += v * CX[i];
                acc[3] += v * CY[i];
            }
        acc[0] += rho[0];
        acc[1] += rho[1];
        const bool ok = (rho[0] > 0.0) && (rho[1] > 0.0) && (rho[0] < 1e300) && (rho[1] < 1e300);
        if (!ok) acc[4] += 1.0;
    }
    __shared__ double red[RED_THREADS / 64][5];
#pragma unroll
    for (int m = 0; m < 5; ++m) acc[m] = wave_sum(acc[m]);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int m = 0; m < 5; ++m) red[wave][m] = acc[m];
    __syncthreads();
    if (threadIdx.x < 5) {
        double t = 0;
        for (int wv = 0; wv < RED_THREADS / 64; ++wv) t += red[wv][threadIdx.x];
        partials[blockIdx.x * 5 + threadIdx.x] = t;
    }
}

// Sums nparts partial rows of 5 in a fixed order into out[5]; sets *flag if
// the bad-site count is non-zero (the flag is never cleared here).
__global__ void __launch_bounds__(64)
k_sums_final(const double* __restrict__ partials, int nparts, double* __restrict__ out,
             int* __restrict__ flag)
{
    const int t = threadIdx.x;
    if (t < 5) {
        double s = 0;
        for (int b = 0; b < nparts; ++b) s += partials[b * 5 + t];
        out[t] = s;
        if (t == 4 && s > 0.0 && flag) *flag = 1;
    }
}

// out[y] = (1/nx) sum_x u_x(x, y) of the stored populations, FP64; one block per row.
template <class P>
__global__ void __launch_bounds__(256)
k_line_profile(char* __restrict__ base, const LatDesc* __restrict__ dd, int buf, double* __restrict__ out)
{
    using S = typename P::S;
    const LatDesc& d = *dd;
    const int y = blockIdx.x;
    const S* f = (const S*)(base + d.off_f[buf]) + (long long)y * d.pitch;
    double acc = 0;
    for (int x = threadIdx.x; x < d.nx; x += blockDim.x) {
        double rho = 0, jx = 0;
        for (int q = 0; q < 18; ++q) {
            const double v = decode<P>(f + q * d.plane + col_of(x, q, d.nx), d, q);
            rho += v;
            jx += v * CX[q % 9];
        }
        acc += jx / rho;
    }
    __shared__ double red[4];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[y] = (red[0] + red[1] + red[2] + red[3]) / d.nx;
}

// Per lattice k: out[2k] = sum_x bottom accumulator, out[2k+1] = sum_x top.
__global__ void __launch_bounds__(256)
k_stress_reduce(char* __restrict__ base, const LatDesc* __restrict__ descs, double* __restrict__ out)
{
    const LatDesc& d = descs[blockIdx.x];
    const double* st = (const double*)(base + d.off_stress);
    __shared__ double red[4][2];
    double a = 0, b = 0;
    for (int x = threadIdx.x; x < d.nx; x += blockDim.x) {
        a += st[x];
        b += st[d.nx + x];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[wave][0] = a; red[wave][1] = b; }
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0;
        for (int wv = 0; wv < 4; ++wv) s += red[wv][threadIdx.x];
        out[2 * blockIdx.x + threadIdx.x] = s;
    }
}

// out[y] = sum over the 64-column groups of the profile accumulator.
__global__ void k_profile_reduce(char* __restrict__ base, const LatDesc* __restrict__ dd,
                                 double* __restrict__ out)
{
    const LatDesc& d = *dd;
    const double* pr = (const double*)(base + d.off_prof);
    for (int y = blockIdx.x * blockDim.x + threadIdx.x; y < d.ny; y += gridDim.x * blockDim.x) {
        double s = 0;
        for (int g = 0; g < d.ngroups + d.ngroups2; ++g) s += pr[(long long)g * d.ny + y];
        out[y] = s;
    }
}

__global__ void k_fill(double* __restrict__ p, long long n, double v)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        p[k] = v;
}

// Streaming copy (16 bytes per lane per access): the achievable read+write
// HBM bandwidth the step kernel is compared with.
__global__ void __launch_bounds__(256)
k_copy(const float4* __restrict__ src, float4* __restrict__ dst, long long n)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        dst[k] = src[k];
}

// ------------------------------------------------------------ moment form ---
//
// At tau = 1 the BGK collision of Eq. (1) replaces every population by the
// equilibrium at the shifted velocity, f*_is = f^eq_i(rho_s, v_s), so the
// post-collision state of a site is the six numbers (rho_s, v_s) of the two
// species.  The moment form stores them instead of the 18 populations and
// rebuilds each incoming population from its source site,
//   f_is(x, t) = f^eq_i(rho_s, v_s)(x - c_i, t - 1),
// or, across a wall, from the bounced population of the site itself.  It is
// the same recurrence as the population form at tau = 1 and moves 6 loads and
// 6 stores per site instead of 36.
//
// Planes, each [y][pitch]: 0, 1 = rho_A - rho_ref_A, rho_B - rho_ref_B;
// 2, 3 = v_x of A, B; 4, 5 = v_y of A, B.  Before the first step the buffer
// holds the initial state itself, (rho_s - rho_ref_s, u, u), and the first
// step reads it in place: the initial populations are local equilibria, not
// streamed ones.
struct MomF32 { using S = float;  using C = float;  static constexpr bool fast_psi = true; };
struct MomF64 { using S = double; using C = double; static constexpr bool fast_psi = false; };

// Deviation of the equilibrium population i of one species from w_i rho_ref:
// w_i [drho + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)], rho = rho_ref + drho.
template <int I, class C>
__device__ __forceinline__ C eq_dev(C drho, C rho, C vx, C vy)
{
    constexpr double W = (I == 0) ? 4.0 / 9.0 : (I < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    const C cu = (C)CX[I] * vx + (C)CY[I] * vy;
    const C usq = vx * vx + vy * vy;
    return (C)W * (drho + rho * ((C)3 * cu + (C)4.5 * cu * cu - (C)1.5 * usq));
}

template <class C>
__host__ __device__ constexpr size_t mom_dyn_lds(int bx, int ly)
{
    return sizeof(double) * (size_t)(bx / 64) * ly;
}

template <int BX, class P>
__global__ void __launch_bounds__(BX)
k_step_mom(char* __restrict__ base, const LatDesc* __restrict__ descs, const int* __restrict__ tiles, int ntot,
           int src, int first)
{
    using S = typename P::S;
    using C = typename P::C;
    using C2 = typename V2<C>::T;
    // Overlapped tiles: the BX lanes hold columns x0-2 .. x0+BX-3 and every
    // lane rebuilds its own column, so the psi/rho neighbourhood of the BX-4
    // columns x0 .. x0+BX-5 that the tile collides needs no extra halo work.
    // Moment rows in flight: four rows of the pairs (drho, v_x, v_y) of A and B
    // for columns x0-3 .. x0+BX-2 (index column - x0 + 3); psi and rho pairs of
    // the six rows around the collided one for the lanes' columns (index tid).
    __shared__ C2 mring[4][3][BX + 2];
    __shared__ C2 ringP[6][BX];
    __shared__ C2 ringR[6][BX];
    extern __shared__ __align__(16) char dyn_lds[];

    const int tid = threadIdx.x;
    const int wave = tid >> 6;

    for (int w = blockIdx.x; w < ntot; w += gridDim.x) {
        const int L = tiles[w];
        if (L < 0) continue;
        const LatDesc& d = descs[L];
        const int lin = xcd_tile(w - d.item_begin, d.nitems);
        if (lin < 0) continue;
        const int nstrip = d.nstrip;
        const int strip = lin % nstrip, seg = lin / nstrip;
        const int nx = d.nx, ny = d.ny, pitch = d.pitch, walls = d.walls;
        const long long plane = d.plane;
        const int x0 = strip * (BX - 4);
        const int y0 = seg * d.ly;
        const int y1 = min(y0 + d.ly, ny);
        auto wrap = [&](int c) { c %= nx; return c < 0 ? c + nx : c; };
        const int x = x0 - 2 + tid;                       // the lane's column
        const bool valid = tid >= 2 && tid < BX - 2 && x < nx;   // collided by this tile
        const unsigned xc = (unsigned)wrap(x);

        const C inv_rho0 = coef<C>(d.inv_rho0, d.finv_rho0);
        C ks0[5], ks1[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            ks0[k] = coef<C>(d.ks[0][k], d.fks[0][k]);
            ks1[k] = coef<C>(d.ks[1][k], d.fks[1][k]);
        }
        const C kx1 = coef<C>(d.kx[0], d.fkx[0]), kx2 = coef<C>(d.kx[1], d.fkx[1]);
        const C u_top = coef<C>(d.u_top, d.fu_top), u_bot = coef<C>(d.u_bot, d.fu_bot);
        const C rref0 = coef<C>(d.rref[0], d.frref[0]), rref1 = coef<C>(d.rref[1], d.frref[1]);
        const C pref0 = coef<C>(d.psiref[0], d.fpsiref[0]), pref1 = coef<C>(d.psiref[1], d.fpsiref[1]);
        const C e0 = coef<C>(d.epsi[0], d.fepsi[0]), e1 = coef<C>(d.epsi[1], d.fepsi[1]);

        const int es = (int)sizeof(S);
        const unsigned mbytes = (unsigned)(6 * plane * (long long)es);
        const rsrc_t rin = make_rsrc(base + d.off_f[src], mbytes);
        const rsrc_t rout = make_rsrc(base + d.off_f[src ^ 1], mbytes);
        const unsigned pbytes = (unsigned)(plane * es), rbytes = (unsigned)(pitch * es);
        const unsigned vc = xc * es;
        const int cm = tid + 1;                           // the lane's moment-ring index
        // lanes 0 and 1 also load the two outer moment columns x0-3 and
        // x0+BX-2 (ring indices 0 and BX+1)
        const int hm = (tid == 0) ? 0 : BX + 1;
        const unsigned vhm = (unsigned)wrap(x0 - 3 + hm) * es;
        double* __restrict__ stress = (double*)(base + d.off_stress);
        double* __restrict__ prof = d.off_prof >= 0 ? (double*)(base + d.off_prof) : nullptr;
        const double* __restrict__ body = d.off_body >= 0 ? (const double*)(base + d.off_body) : nullptr;
        double* profS = (double*)dyn_lds;                   // [BX/64][ly] per-wave row sums
        C mom_b = 0, mom_t = 0;

        // One moment row in registers: the lane's column and, for lanes 0 and
        // 1, an outer column.  Rows beyond a wall do not exist and are skipped.
        struct MR { C v[6]; C h[6]; };
        auto mrow_ok = [&](int r) { return !walls || (r >= 0 && r < ny); };
        auto mload = [&](MR& m, int r) {
            if (!mrow_ok(r)) return;
            const unsigned so = (unsigned)map_row<P>(r, ny, walls) * rbytes;
#pragma unroll
            for (int p = 0; p < 6; ++p) m.v[p] = ld<P>(rin, vc, so + p * pbytes);
            if (tid < 2) {
#pragma unroll
                for (int p = 0; p < 6; ++p) m.h[p] = ld<P>(rin, vhm, so + p * pbytes);
            }
        };
        auto mput = [&](const MR& m, int r) {
            if (!mrow_ok(r)) return;
            const int sl = r & 3;
            mring[sl][0][cm] = C2{m.v[0], m.v[1]};
            mring[sl][1][cm] = C2{m.v[2], m.v[3]};
            mring[sl][2][cm] = C2{m.v[4], m.v[5]};
            if (tid < 2) {
                mring[sl][0][hm] = C2{m.h[0], m.h[1]};
                mring[sl][1][hm] = C2{m.h[2], m.h[3]};
                mring[sl][2][hm] = C2{m.h[4], m.h[5]};
            }
        };

        // Incoming populations of row r (a fluid row) at the lane's column,
        // summed into the density deviations of A and B and the momentum j.
        auto pull = [&](int r, C& dA, C& dB, C& jx, C& jy) {
            if (first) {
                const int sl = r & 3;
                const C2 m0 = mring[sl][0][cm], m1 = mring[sl][1][cm], m2 = mring[sl][2][cm];
                dA = m0.x;
                dB = m0.y;
                const C ra = rref0 + dA, rb = rref1 + dB;
                jx = ra * m1.x + rb * m1.y;
                jy = ra * m2.x + rb * m2.y;
                return;
            }
            const bool bot = walls && r == 0, top = walls && r == ny - 1;
            dA = dB = jx = jy = 0;
            auto one = [&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int cx = CX[i], cy = CY[i];
                C fa, fb;
                if ((cy > 0 && bot) || (cy < 0 && top)) {
                    // source beyond the wall: the site's own population OPP[i],
                    // returned with the moving-wall term (1/6) rho_s c_ix u_w
                    constexpr int o = OPP[i];
                    const int sl = r & 3;
                    const C2 m0 = mring[sl][0][cm], m1 = mring[sl][1][cm], m2 = mring[sl][2][cm];
                    const C ra = rref0 + m0.x, rb = rref1 + m0.y;
                    const C uw = (cy > 0) ? u_bot : u_top;
                    fa = eq_dev<o>(m0.x, ra, m1.x, m2.x);
                    fb = eq_dev<o>(m0.y, rb, m1.y, m2.y);
                    if (cx != 0) {
                        fa += (C)(1.0 / 6.0) * ra * (C)cx * uw;
                        fb += (C)(1.0 / 6.0) * rb * (C)cx * uw;
                    }
                } else {
                    const int sl = (r - cy) & 3;
                    const int cs = cm - cx;
                    const C2 m0 = mring[sl][0][cs], m1 = mring[sl][1][cs], m2 = mring[sl][2][cs];
                    fa = eq_dev<i>(m0.x, rref0 + m0.x, m1.x, m2.x);
                    fb = eq_dev<i>(m0.y, rref1 + m0.y, m1.y, m2.y);
                }
                dA += fa;
                dB += fb;
                if (cx != 0) jx += (C)cx * (fa + fb);
                if (cy != 0) jy += (C)cy * (fa + fb);
                // keep each direction's LDS reads next to their arithmetic (bounds
                // the registers the pull occupies: three waves per SIMD)
                asm volatile("" : "+v"(dA), "+v"(dB), "+v"(jx), "+v"(jy)::"memory");
            };
            one(std::integral_constant<int, 0>{});
            one(std::integral_constant<int, 1>{});
            one(std::integral_constant<int, 2>{});
            one(std::integral_constant<int, 3>{});
            one(std::integral_constant<int, 4>{});
            one(std::integral_constant<int, 5>{});
            one(std::integral_constant<int, 6>{});
            one(std::integral_constant<int, 7>{});
            one(std::integral_constant<int, 8>{});
        };

        auto slot6 = [&](int r) { return __builtin_amdgcn_readfirstlane((r - y0 + 2) % 6); };
        // Stage row r: (psi, rho) deviations of the lane's column into the
        // rings and its momentum into J.  A row beyond a wall is the even
        // mirror of the fluid rows.
        auto stage = [&](int r, C2& J) {
            const int sl = slot6(r);
            if (walls && (r < 0 || r >= ny)) {
                const int sm = slot6((r < 0) ? -1 - r : 2 * ny - 1 - r);
                ringP[sl][tid] = ringP[sm][tid];
                ringR[sl][tid] = ringR[sm][tid];
                return;
            }
            C dA, dB, jx, jy;
            pull(r, dA, dB, jx, jy);
            ringP[sl][tid] = C2{dpsi<P>(dA, e0, inv_rho0), dpsi<P>(dB, e1, inv_rho0)};
            ringR[sl][tid] = C2{dA, dB};
            J = C2{jx, jy};
        };

        // Collide row y: the force from the 5x5 neighbourhood, the shifted
        // velocities (tau = 1) and the six new moments of the site.
        auto collide = [&](int y, const C2& J) {
            int sl[5];
            sl[0] = __builtin_amdgcn_readfirstlane((y - y0) % 6);
#pragma unroll
            for (int k = 1; k < 5; ++k) sl[k] = (sl[k - 1] == 5) ? 0 : sl[k - 1] + 1;
            // neighbour columns clamped to the tile: the edge lanes read in
            // range and are not collided
            auto cn = [&](int dx) { return min(max(tid + dx, 0), BX - 1); };
            C ss[8];
            stencil_sums<true, C>([&](int dy, int dx) { return ringP[sl[dy + 2]][cn(dx)]; },
                            [&](int dy, int dx) { return ringR[sl[dy + 2]][cn(dx)]; }, ks0, ks1, kx1, kx2, ss);
            const C sxA = ss[0], syA = ss[1], sxB = ss[2], syB = ss[3];
            const C cxA = ss[4], cyA = ss[5], cxB = ss[6], cyB = ss[7];
            const C2 p0 = ringP[sl[2]][tid];
            const C2 r0c = ringR[sl[2]][tid];
            const C ra = rref0 + r0c.x, rb = rref1 + r0c.y;
            const C pa = pref0 + p0.x, pb = pref1 + p0.y;
            const C FxA = -pa * sxA - ra * cxA, FyA = -pa * syA - ra * cyA;
            const C FxB = -pb * sxB - rb * cxB, FyB = -pb * syB - rb * cyB;
            const C inv_rho = rcp(ra + rb);
            const C ux = J.x * inv_rho, uy = J.y * inv_rho;
            const C gx = (body != nullptr) ? (C)body[y] * inv_rho : (C)0;
            if (prof != nullptr) {
                double su = valid ? (double)ux : 0.0;
                su = wave_sum(su);
                if ((tid & 63) == 0) profS[wave * d.ly + (y - y0)] = su;
            }
            const C iA = rcp(ra), iB = rcp(rb);
            const C vAx = ux + (FxA * iA + gx), vAy = uy + FyA * iA;
            const C vBx = ux + (FxB * iB + gx), vBy = uy + FyB * iB;
            if (!valid) return;
            const unsigned so = (unsigned)y * rbytes;
            st<P>(rout, vc, so, r0c.x);
            st<P>(rout, vc, so + pbytes, r0c.y);
            st<P>(rout, vc, so + 2 * pbytes, vAx);
            st<P>(rout, vc, so + 3 * pbytes, vBx);
            st<P>(rout, vc, so + 4 * pbytes, vAy);
            st<P>(rout, vc, so + 5 * pbytes, vBy);
            // wall momentum of the links that leave through a wall this step:
            // c_ix (f*_i + back), back = f*_i - (1/6) rho_s c_ix u_w
            if (walls && (y == 0 || y == ny - 1)) {
                auto link = [&](auto I, C uw, C& acc) {
                    constexpr int i = decltype(I)::value;
                    constexpr int cx = CX[i];
                    const C fa = (C)(i < 5 ? 1.0 / 9.0 : 1.0 / 36.0) * ra + eq_dev<i>((C)0, ra, vAx, vAy);
                    const C fb = (C)(i < 5 ? 1.0 / 9.0 : 1.0 / 36.0) * rb + eq_dev<i>((C)0, rb, vBx, vBy);
                    const C ba = fa - (C)(1.0 / 6.0) * ra * (C)cx * uw;
                    const C bb = fb - (C)(1.0 / 6.0) * rb * (C)cx * uw;
                    acc += (C)cx * (fa + ba) + (C)cx * (fb + bb);
                };
                if (y == 0) {
                    link(std::integral_constant<int, 7>{}, u_bot, mom_b);
                    link(std::integral_constant<int, 8>{}, u_bot, mom_b);
                }
                if (y == ny - 1) {
                    link(std::integral_constant<int, 5>{}, u_top, mom_t);
                    link(std::integral_constant<int, 6>{}, u_top, mom_t);
                }
            }
        };

        // Prologue: moment rows y0-3 .. y0+3 through the ring, psi/rho rows
        // y0-2 .. y0+1 staged (fluid rows first, then the mirrored ghost rows),
        // row y0+4 prefetched.  Loop: entering iteration y, moment rows
        // y+1 .. y+3 are in LDS, row y+4 in registers, and psi/rho rows
        // y-2 .. y+1 staged.
        C2 J0 = C2{0, 0}, J1 = C2{0, 0}, J2 = C2{0, 0}, J3 = C2{0, 0}, Jx = C2{0, 0};
        {
            MR a, b, c, e;
            mload(a, y0 - 3);
            mload(b, y0 - 2);
            mload(c, y0 - 1);
            mload(e, y0);
            mput(a, y0 - 3);
            mput(b, y0 - 2);
            mput(c, y0 - 1);
            mput(e, y0);
            lds_barrier();
            if (mrow_ok(y0 - 2)) stage(y0 - 2, Jx);
            if (mrow_ok(y0 - 1)) stage(y0 - 1, Jx);
            lds_barrier();
            mload(a, y0 + 1);
            mload(b, y0 + 2);
            mput(a, y0 + 1);
            mput(b, y0 + 2);
            lds_barrier();
            if (mrow_ok(y0)) stage(y0, J0);
            if (mrow_ok(y0 + 1)) stage(y0 + 1, J1);
            for (int r = y0 - 2; r <= y0 + 1; ++r)
                if (!mrow_ok(r)) stage(r, Jx);
            lds_barrier();
            mload(a, y0 + 3);
            mput(a, y0 + 3);
        }
        MR pf;
        if (y0 + 4 <= y1 + 2) mload(pf, y0 + 4);
        lds_barrier();
        auto iter = [&](int y, const C2& Jc, C2& Js) {
            if (y + 4 <= y1 + 2) mput(pf, y + 4);
            if (y + 5 <= y1 + 2) mload(pf, y + 5);
            stage(y + 2, Js);
            lds_barrier();
            collide(y, Jc);
        };
        for (int y = y0; y < y1; y += 4) {
            iter(y, J0, J2);
            if (y + 1 < y1) iter(y + 1, J1, J3);
            if (y + 2 < y1) iter(y + 2, J2, J0);
            if (y + 3 < y1) iter(y + 3, J3, J1);
        }
        if (valid && walls && y0 == 0) stress[xc] += (double)mom_b;
        if (valid && walls && y1 == ny) stress[nx + xc] += (double)mom_t;
        __syncthreads();
        if (prof != nullptr) {
            // one accumulator row per tile: the per-wave sums in wave order
            for (int r = tid; r < y1 - y0; r += BX) {
                double t = 0;
                for (int wv = 0; wv < BX / 64; ++wv) t += profS[wv * d.ly + r];
                prof[(long long)strip * ny + y0 + r] += t;
            }
        }
        __syncthreads();
    }
}

// Population i of species s at site (x, y) in the moment form, FP64: the
// equilibrium of its source site, across a wall the bounced population of the
// site itself, or, before the first step, the local equilibrium.
template <class P>
__device__ double mom_pop(const LatDesc& d, const typename P::S* m, int first, int x, int y, int s, int i)
{
    int xs = x, ys = y, q = i;
    double extra = 0;
    if (!first) {
        const int cx = CX[i], cy = CY[i];
        if (d.walls && ((cy > 0 && y == 0) || (cy < 0 && y == d.ny - 1))) {
            q = OPP[i];
            const double uw = (cy > 0) ? d.u_bot : d.u_top;
            extra = (1.0 / 6.0) * (d.rref[s] + (double)m[s * d.plane + (long long)y * d.pitch + x]) * cx * uw;
        } else {
            xs = x - cx;
            xs = xs < 0 ? xs + d.nx : (xs >= d.nx ? xs - d.nx : xs);
            ys = y - cy;
            ys = ys < 0 ? ys + d.ny : (ys >= d.ny ? ys - d.ny : ys);
        }
    }
    const long long o = (long long)ys * d.pitch + xs;
    const double rho = d.rref[s] + (double)m[s * d.plane + o];
    const double vx = (double)m[(2 + s) * d.plane + o], vy = (double)m[(4 + s) * d.plane + o];
    const double w = (q == 0) ? 4.0 / 9.0 : (q < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    const double cu = CX[q] * vx + CY[q] * vy;
    return w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (vx * vx + vy * vy)) + extra;
}

// Initial state of the moment form: (rho_s - rho_ref_s, u, u).
template <class P>
__global__ void k_init_mom(char* __restrict__ base, const LatDesc* __restrict__ dd, int buf,
                           const double* __restrict__ ra, const double* __restrict__ rb,
                           const double* __restrict__ ux, const double* __restrict__ uy)
{
    using S = typename P::S;
    const LatDesc& d = *dd;
    const long long n = (long long)d.nx * d.ny;
    S* m = (S*)(base + d.off_f[buf]);
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / d.nx), x = (int)(k % d.nx);
        const long long o = (long long)y * d.pitch + x;
        const double u = ux ? ux[k] : 0.0, v = uy ? uy[k] : 0.0;
        m[o] = (S)(ra[k] - d.rref[0]);
        m[d.plane + o] = (S)(rb[k] - d.rref[1]);
        m[2 * d.plane + o] = (S)u;
        m[3 * d.plane + o] = (S)u;
        m[4 * d.plane + o] = (S)v;
        m[5 * d.plane + o] = (S)v;
    }
}

template <class P>
__global__ void k_fields_mom(char* __restrict__ base, const LatDesc* __restrict__ dd, int buf, int first,
                             double* __restrict__ ra, double* __restrict__ rb,
                             double* __restrict__ ux, double* __restrict__ uy)
{
    using S = typename P::S;
    const LatDesc& d = *dd;
    const long long n = (long long)d.nx * d.ny;
    const S* m = (const S*)(base + d.off_f[buf]);
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / d.nx), x = (int)(k % d.nx);
        double rho[2] = {0, 0}, jx = 0, jy = 0;
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < 9; ++i) {
                const double v = mom_pop<P>(d, m, first, x, y, s, i);
                rho[s] += v;
                jx += v * CX[i];
                jy += v * CY[i];
            }
        if (ra) ra[k] = rho[0];
        if (rb) rb[k] = rho[1];
        if (ux) ux[k] = jx / (rho[0] + rho[1]);
        if (uy) uy[k] = jy / (rho[0] + rho[1]);
    }
}

template <class P>
__global__ void k_export_mom(char* __restrict__ base, const LatDesc* __restrict__ dd, int buf, int first, int q,
                             double* __restrict__ out)
{
    using S = typename P::S;
    const LatDesc& d = *dd;
    const long long n = (long long)d.nx * d.ny;
    const S* m = (const S*)(base + d.off_f[buf]);
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / d.nx), x = (int)(k % d.nx);
        out[k] = mom_pop<P>(d, m, first, x, y, q / 9, q % 9);
    }
}

template <class P>
__global__ void __launch_bounds__(RED_THREADS)
k_sums_mom(char* __restrict__ base, const LatDesc* __restrict__ dd, int buf, int first,
           double* __restrict__ partials)
{
    using S = typename P::S;
    const LatDesc& d = *dd;
    const long long n = (long long)d.nx * d.ny;
    const S* m = (const S*)(base + d.off_f[buf]);
    double acc[5] = {0, 0, 0, 0, 0};
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / d.nx), x = (int)(k % d.nx);
        double rho[2] = {0, 0};
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < 9; ++i) {
                const double v = mom_pop<P>(d, m, first, x, y, s, i);
                rho[s] += v;
                acc[2] += v * CX[i];
                acc[3] += v * CY[i];
            }
        acc[0] += rho[0];
        acc[1] += rho[1];
        const bool ok = (rho[0] > 0.0) && (rho[1] > 0.0) && (rho[0] < 1e300) && (rho[1] < 1e300);
        if (!ok) acc[4] += 1.0;
    }
    __shared__ double red[RED_THREADS / 64][5];
#pragma unroll
    for (int q = 0; q < 5; ++q) acc[q] = wave_sum(acc[q]);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 5; ++q) red[wave][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < 5) {
        double t = 0;
        for (int wv = 0; wv < RED_THREADS / 64; ++wv) t += red[wv][threadIdx.x];
        partials[blockIdx.x * 5 + threadIdx.x] = t;
    }
}

template <class P>
__global__ void __launch_bounds__(256)
k_line_profile_mom(char* __restrict__ base, const LatDesc* __restrict__ dd, int buf, int first,
                   double* __restrict__ out)
{
    using S = typename P::S;
    const LatDesc& d = *dd;
    const int y = blockIdx.x;
    const S* m = (const S*)(base + d.off_f[buf]);
    double acc = 0;
    for (int x = threadIdx.x; x < d.nx; x += blockDim.x) {
        double rho = 0, jx = 0;
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < 9; ++i) {
                const double v = mom_pop<P>(d, m, first, x, y, s, i);
                rho += v;
                jx += v * CX[i];
            }
        acc += jx / rho;
    }
    __shared__ double red[4];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[y] = (red[0] + red[1] + red[2] + red[3]) / d.nx;
}

// ---------------------------------------------------------- host launchers --

template <int BX, class P>
static hipError_t step_bx(char* base, const LatDesc* descs, const int* tiles, int ntot, int src, int grid,
                          int ly, hipStream_t s)
{
    const size_t dyn = step_dyn_lds<P>(BX, ly);
    hipLaunchKernelGGL((k_step<BX, P>), dim3(grid), dim3(BX), dyn, s, base, descs, tiles, ntot, src);
    return hipGetLastError();
}

template <class P>
static hipError_t step_p(int bx, char* base, const LatDesc* descs, const int* tiles, int ntot, int src,
                         int grid, int ly, hipStream_t s)
{
    switch (bx) {
    case 64: return step_bx<64, P>(base, descs, tiles, ntot, src, grid, ly, s);
    case 128: return step_bx<128, P>(base, descs, tiles, ntot, src, grid, ly, s);
    case 256: return step_bx<256, P>(base, descs, tiles, ntot, src, grid, ly, s);
    case 512:   // 4- and 2-byte storage only: halves the share of halo columns
        if constexpr (sizeof(typename P::S) <= 4) return step_bx<512, P>(base, descs, tiles, ntot, src, grid, ly, s);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

#define LBK_DISPATCH(storage, CALL)                                  \
    switch (storage) {                                               \
    case 0: { using P = StF64; return CALL; }                        \
    case 1: { using P = StF32; return CALL; }                        \
    case 2: { using P = StF16; return CALL; }                        \
    case 3: { using P = StBF16; return CALL; }                       \
    default: return hipErrorInvalidValue;                            \
    }

template <int BX, class P>
static hipError_t step_mom_bx(char* base, const LatDesc* descs, const int* tiles, int ntot, int src, int first,
                              int grid, int ly, hipStream_t s)
{
    const size_t dyn = mom_dyn_lds<typename P::C>(BX, ly);
    hipLaunchKernelGGL((k_step_mom<BX, P>), dim3(grid), dim3(BX), dyn, s, base, descs, tiles, ntot, src, first);
    return hipGetLastError();
}

template <class P>
static hipError_t step_mom_p(int bx, char* base, const LatDesc* descs, const int* tiles, int ntot, int src,
                             int first, int grid, int ly, hipStream_t s)
{
    switch (bx) {
    case 64: return step_mom_bx<64, P>(base, descs, tiles, ntot, src, first, grid, ly, s);
    case 128: return step_mom_bx<128, P>(base, descs, tiles, ntot, src, first, grid, ly, s);
    case 256: return step_mom_bx<256, P>(base, descs, tiles, ntot, src, first, grid, ly, s);
    default: return hipErrorInvalidValue;
    }
}

// Moment-form storage (tau = 1): codes 4 (FP32) and 5 (FP64).
#define LBK_DISPATCH_MOM(storage, CALL)                              \
    switch (storage) {                                               \
    case 4: { using P = MomF32; return CALL; }                       \
    case 5: { using P = MomF64; return CALL; }                       \
    default: break;                                                  \
    }

// LDS of one block: the kernel's static shared memory plus the dynamic part.
template <class K>
static size_t lds_of(K kernel, size_t dyn)
{
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel)) != hipSuccess) return 0;
    return fa.sharedSizeBytes + dyn;
}

size_t step_lds_bytes(int storage, int bx, int ly)
{
    switch (storage * 1000 + bx) {
    case 0 * 1000 + 64: return lds_of(k_step<64, StF64>, step_dyn_lds<StF64>(64, ly));
    case 0 * 1000 + 128: return lds_of(k_step<128, StF64>, step_dyn_lds<StF64>(128, ly));
    case 0 * 1000 + 256: return lds_of(k_step<256, StF64>, step_dyn_lds<StF64>(256, ly));
    case 1 * 1000 + 64: return lds_of(k_step<64, StF32>, step_dyn_lds<StF32>(64, ly));
    case 1 * 1000 + 128: return lds_of(k_step<128, StF32>, step_dyn_lds<StF32>(128, ly));
    case 1 * 1000 + 256: return lds_of(k_step<256, StF32>, step_dyn_lds<StF32>(256, ly));
    case 1 * 1000 + 512: return lds_of(k_step<512, StF32>, step_dyn_lds<StF32>(512, ly));
    case 2 * 1000 + 64: return lds_of(k_step<64, StF16>, step_dyn_lds<StF16>(64, ly));
    case 2 * 1000 + 128: return lds_of(k_step<128, StF16>, step_dyn_lds<StF16>(128, ly));
    case 2 * 1000 + 256: return lds_of(k_step<256, StF16>, step_dyn_lds<StF16>(256, ly));
    case 2 * 1000 + 512: return lds_of(k_step<512, StF16>, step_dyn_lds<StF16>(512, ly));
    case 3 * 1000 + 64: return lds_of(k_step<64, StBF16>, step_dyn_lds<StBF16>(64, ly));
    case 3 * 1000 + 128: return lds_of(k_step<128, StBF16>, step_dyn_lds<StBF16>(128, ly));
    case 3 * 1000 + 256: return lds_of(k_step<256, StBF16>, step_dyn_lds<StBF16>(256, ly));
    case 3 * 1000 + 512: return lds_of(k_step<512, StBF16>, step_dyn_lds<StBF16>(512, ly));
    case 4 * 1000 + 64: return lds_of(k_step_mom<64, MomF32>, mom_dyn_lds<MomF32::C>(64, ly));
    case 4 * 1000 + 128: return lds_of(k_step_mom<128, MomF32>, mom_dyn_lds<MomF32::C>(128, ly));
    case 4 * 1000 + 256: return lds_of(k_step_mom<256, MomF32>, mom_dyn_lds<MomF32::C>(256, ly));
    case 5 * 1000 + 64: return lds_of(k_step_mom<64, MomF64>, mom_dyn_lds<MomF64::C>(64, ly));
    case 5 * 1000 + 128: return lds_of(k_step_mom<128, MomF64>, mom_dyn_lds<MomF64::C>(128, ly));
    case 5 * 1000 + 256: return lds_of(k_step_mom<256, MomF64>, mom_dyn_lds<MomF64::C>(256, ly));
    default: return 0;
    }
}

template <class P, int NW>
static hipError_t step2_nw(char* base, const LatDesc* descs, const int* tiles, int ntot, int src, int grid,
                           hipStream_t s)
{
    hipLaunchKernelGGL((k_step2<P, NW>), dim3(grid), dim3(128 * NW), 0, s, base, descs, tiles, ntot, src);
    return hipGetLastError();
}

template <class P>
static hipError_t step2_p(int nw, char* base, const LatDesc* descs, const int* tiles, int ntot, int src, int grid,
                          hipStream_t s)
{
    switch (nw) {
    case 2: return step2_nw<P, 2>(base, descs, tiles, ntot, src, grid, s);
    case 3: return step2_nw<P, 3>(base, descs, tiles, ntot, src, grid, s);
    case 4: return step2_nw<P, 4>(base, descs, tiles, ntot, src, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step2(int storage, int nw, char* base, const LatDesc* descs, const int* tiles, int ntot, int src,
                        int grid, hipStream_t s)
{
    switch (storage) {
    case 1: return step2_p<StF32>(nw, base, descs, tiles, ntot, src, grid, s);
    case 2: return step2_p<StF16>(nw, base, descs, tiles, ntot, src, grid, s);
    case 3: return step2_p<StBF16>(nw, base, descs, tiles, ntot, src, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <class K>
static int blocks_per_cu_of(K kernel, int threads)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(kernel), threads, 0) !=
        hipSuccess)
        return 0;
    return n;
}

#define LBK_STEP2_CASES(F)                                                                          \
    switch (storage * 10 + nw) {                                                                     \
    case 12: return F((k_step2<StF32, 2>), 256);                                                     \
    case 13: return F((k_step2<StF32, 3>), 384);                                                     \
    case 14: return F((k_step2<StF32, 4>), 512);                                                     \
    case 22: return F((k_step2<StF16, 2>), 256);                                                     \
    case 23: return F((k_step2<StF16, 3>), 384);                                                     \
    case 24: return F((k_step2<StF16, 4>), 512);                                                     \
    case 32: return F((k_step2<StBF16, 2>), 256);                                                    \
    case 33: return F((k_step2<StBF16, 3>), 384);                                                    \
    case 34: return F((k_step2<StBF16, 4>), 512);                                                    \
    default: return 0;                                                                               \
    }

size_t step2_lds_bytes(int storage, int nw)
{
#define LDS_F(K, T) lds_of(K, 0)
    LBK_STEP2_CASES(LDS_F)
#undef LDS_F
}

int step2_blocks_per_cu(int storage, int nw)
{
#define OCC_F(K, T) blocks_per_cu_of(K, T)
    LBK_STEP2_CASES(OCC_F)
#undef OCC_F
}

hipError_t launch_step(int storage, int bx, char* base, const LatDesc* descs, const int* tiles, int ntot,
                       int src, int first, int grid, int ly, hipStream_t s)
{
    LBK_DISPATCH_MOM(storage, (step_mom_p<P>(bx, base, descs, tiles, ntot, src, first, grid, ly, s)));
    LBK_DISPATCH(storage, (step_p<P>(bx, base, descs, tiles, ntot, src, grid, ly, s)));
}

static int grid_for(long long n, int threads)
{
    long long g = (n + threads - 1) / threads;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

template <class P>
static hipError_t init_p(char* base, const LatDesc* d, long long n, int buf, const double* ra,
                         const double* rb, const double* ux, const double* uy, hipStream_t s)
{
    hipLaunchKernelGGL((k_init<P>), dim3(grid_for(n, 256)), dim3(256), 0, s, base, d, buf, ra, rb, ux, uy);
    return hipGetLastError();
}

template <class P>
static hipError_t init_mom_p(char* base, const LatDesc* d, long long n, int buf, const double* ra,
                             const double* rb, const double* ux, const double* uy, hipStream_t s)
{
    hipLaunchKernelGGL((k_init_mom<P>), dim3(grid_for(n, 256)), dim3(256), 0, s, base, d, buf, ra, rb, ux, uy);
    return hipGetLastError();
}

hipError_t launch_init(int storage, char* base, const LatDesc* d, long long nsites, int buf,
                       const double* ra, const double* rb, const double* ux, const double* uy,
                       hipStream_t s)
{
    LBK_DISPATCH_MOM(storage, (init_mom_p<P>(base, d, nsites, buf, ra, rb, ux, uy, s)));
    LBK_DISPATCH(storage, (init_p<P>(base, d, nsites, buf, ra, rb, ux, uy, s)));
}

template <class P>
static hipError_t fields_p(char* base, const LatDesc* d, long long n, int buf, double* ra,
                           double* rb, double* ux, double* uy, hipStream_t s)
{
    hipLaunchKernelGGL((k_fields<P>), dim3(grid_for(n, 256)), dim3(256), 0, s, base, d, buf, ra, rb, ux, uy);
    return hipGetLastError();
}

template <class P>
static hipError_t fields_mom_p(char* base, const LatDesc* d, long long n, int buf, int first, double* ra,
                               double* rb, double* ux, double* uy, hipStream_t s)
{
    hipLaunchKernelGGL((k_fields_mom<P>), dim3(grid_for(n, 256)), dim3(256), 0, s, base, d, buf, first, ra, rb, ux,
                       uy);
    return hipGetLastError();
}

hipError_t launch_fields(int storage, char* base, const LatDesc* d, long long nsites, int buf, int first,
                         double* ra, double* rb, double* ux, double* uy, hipStream_t s)
{
    LBK_DISPATCH_MOM(storage, (fields_mom_p<P>(base, d, nsites, buf, first, ra, rb, ux, uy, s)));
    LBK_DISPATCH(storage, (fields_p<P>(base, d, nsites, buf, ra, rb, ux, uy, s)));
}

template <class P>
static hipError_t export_p(char* base, const LatDesc* d, long long n, int buf, int q, double* out,
                           hipStream_t s)
{
    hipLaunchKernelGGL((k_export<P>), dim3(grid_for(n, 256)), dim3(256), 0, s, base, d, buf, q, out);
    return hipGetLastError();
}

template <class P>
static hipError_t export_mom_p(char* base, const LatDesc* d, long long n, int buf, int first, int q, double* out,
                               hipStream_t s)
{
    hipLaunchKernelGGL((k_export_mom<P>), dim3(grid_for(n, 256)), dim3(256), 0, s, base, d, buf, first, q, out);
    return hipGetLastError();
}

hipError_t launch_export(int storage, char* base, const LatDesc* d, long long nsites, int buf, int first,
                         int q, double* out, hipStream_t s)
{
    LBK_DISPATCH_MOM(storage, (export_mom_p<P>(base, d, nsites, buf, first, q, out, s)));
    LBK_DISPATCH(storage, (export_p<P>(base, d, nsites, buf, q, out, s)));
}

template <class P>
static hipError_t sums_p(char* base, const LatDesc* d, int buf, int nblocks, double* partials,
                         double* out, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL((k_sums<P>), dim3(nblocks), dim3(RED_THREADS), 0, s, base, d, buf, partials);
    hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(64), 0, s, partials, nblocks, out, flag);
    return hipGetLastError();
}

template <class P>
static hipError_t sums_mom_p(char* base, const LatDesc* d, int buf, int first, int nblocks, double* partials,
                             double* out, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL((k_sums_mom<P>), dim3(nblocks), dim3(RED_THREADS), 0, s, base, d, buf, first, partials);
    hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(64), 0, s, partials, nblocks, out, flag);
    return hipGetLastError();
}

hipError_t launch_sums(int storage, char* base, const LatDesc* d, int buf, int first, int nblocks,
                       double* partials, double* out, int* flag, hipStream_t s)
{
    LBK_DISPATCH_MOM(storage, (sums_mom_p<P>(base, d, buf, first, nblocks, partials, out, flag, s)));
    LBK_DISPATCH(storage, (sums_p<P>(base, d, buf, nblocks, partials, out, flag, s)));
}

template <class P>
static hipError_t line_profile_p(char* base, const LatDesc* desc, int ny, int buf, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_line_profile<P>, dim3(ny), dim3(256), 0, s, base, desc, buf, out);
    return hipGetLastError();
}

template <class P>
static hipError_t line_profile_mom_p(char* base, const LatDesc* desc, int ny, int buf, int first, double* out,
                                     hipStream_t s)
{
    hipLaunchKernelGGL(k_line_profile_mom<P>, dim3(ny), dim3(256), 0, s, base, desc, buf, first, out);
    return hipGetLastError();
}

hipError_t launch_line_profile(int storage, char* base, const LatDesc* desc, int ny, int buf, int first,
                               double* out, hipStream_t s)
{
    LBK_DISPATCH_MOM(storage, (line_profile_mom_p<P>(base, desc, ny, buf, first, out, s)));
    LBK_DISPATCH(storage, (line_profile_p<P>(base, desc, ny, buf, out, s)));
}

hipError_t launch_stress_reduce(char* base, const LatDesc* descs, int nlat, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_stress_reduce, dim3(nlat), dim3(256), 0, s, base, descs, out);
    return hipGetLastError();
}

hipError_t launch_profile_reduce(char* base, const LatDesc* d, int ny, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_profile_reduce, dim3(grid_for(ny, 256)), dim3(256), 0, s, base, d, out);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, long long n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, long long n16, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, (const float4*)src, (float4*)dst, n16);
    return hipGetLastError();
}

int sums_blocks() { return 1024; }

}  // namespace lbk
