// Device-side types shared by the library's kernels and its host runtime.
// Part of the HIP library only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbk {

// Per-lattice descriptor read by every kernel (device copy in the state).
// All coefficients are precomputed on the host in FP64.
struct LatDesc {
    long long off_f[2];    // byte offsets (from the state base) of the two population buffers,
                           // layout [s][i][y][pitch]
    long long off_stress;  // [2][nx] FP64: x momentum received by bottom / top wall, summed over steps
    long long off_prof;    // [ngroups + ngroups2][ny] FP64: sums over steps of partial row sums of u_x
                           // (per 64 columns, then the fused kernel's per step, strip and wave); < 0: off
    long long off_body;    // [ny] FP64: external body force F_x(y) of each row; < 0: none
    long long plane;       // elements per (species, direction) plane = ny * pitch
    int nx, ny, pitch, walls;
    int item_begin;        // first global work item of this lattice (multiple of 8)
    int nitems;            // nstrip * nseg
    int nstrip, nseg, ly;  // tiles: strips of bx columns, segments of ly rows
    int ngroups;           // ceil(nx / 64) (moment form: ceil(nx / 60))
    int ngroups2;          // partial sums of the fused two-step kernel, 2 steps x nstrip2 x waves per step
                           // (rows reserved for its widest layout; 0: no fused kernel for the storage)
    // Tiles of the fused two-step kernel: strips of fuse2_tw columns, nseg2
    // segments of near-equal height (ny / nseg2 rows, the first ny mod nseg2
    // one row more; ly2 the tallest), items item_begin2 .. item_begin2 +
    // nitems2 - 1 of its own table.
    int item_begin2, nitems2, nstrip2, nseg2, ly2;
    double tau, omega, rho0, inv_rho0;
    double ks[2][5];       // psi-stencil coefficient of species s on the shells |c|^2 = 1,2,4,5,8
    double kx[2];          // cross coefficient (G_AB/rho0) w on |c|^2 = 1, 2
    double u_top, u_bot;
    double wref[18];       // storage base w_i rho_ref_s, index s*9 + i (populations are stored
                           // as deviations from it)
    double rref[2];        // reference densities rho_ref_s
    double psiref[2];      // psi(rho_ref_s)
    double epsi[2];        // rho0 exp(-rho_ref_s / rho0)
    // The same coefficients rounded to FP32, for the FP32-arithmetic kernels.
    float ftau, fomega, frho0, finv_rho0;
    float fks[2][5];
    float fkx[2];
    float fu_top, fu_bot;
    float frref[2], fpsiref[2], fepsi[2];
};

template <class C> __device__ __forceinline__ C coef(const double& d, const float& f);
template <> __device__ __forceinline__ double coef<double>(const double& d, const float&) { return d; }
template <> __device__ __forceinline__ float coef<float>(const double&, const float& f) { return f; }

// D2Q9 in the ABI's order.
constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// Shell index of an offset of the 5x5 stencil: |c|^2 = 1,2,4,5,8 -> 0..4.
constexpr int shell_of(int dx, int dy)
{
    return (dx * dx + dy * dy == 1) ? 0 : (dx * dx + dy * dy == 2) ? 1
         : (dx * dx + dy * dy == 4) ? 2 : (dx * dx + dy * dy == 5) ? 3 : 4;
}

}  // namespace lbk
