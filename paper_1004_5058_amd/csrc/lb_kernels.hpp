// Host-side launchers of the library's kernels (internal to the HIP library).
// `base` is the start of the caller's device state; descriptors hold byte
// offsets from it.
#pragma once
#include <hip/hip_runtime.h>
#include "lb_device.hpp"

namespace lbk {

// ly: the largest rows-per-tile of the lattices (sizes the dynamic LDS).
// first: the step starts from the initial state (moment storage only: it then
// reads the local equilibria in place instead of pulling from neighbours).
hipError_t launch_step(int storage, int bx, char* base, const LatDesc* descs, const int* tiles, int ntot,
                       int src, int first, int grid, int ly, hipStream_t s);
// Steps t and t+1 in one launch (k_step2): reads buffer src, writes buffer
// src ^ 1.  FP32 and 16-bit storage (codes 1, 2, 3); nw = 2, 3 or 4 waves per
// step, blocks of 128 nw threads, tiles of fuse2_tw(storage, nw) output
// columns (the step t+1 columns of a 64 nw lane strip less the overlap).
// Column offset: FP32 at two waves per step loads halo columns (3); the
// other forms overlap their tiles by two more columns instead (5).
constexpr int fuse2_xo(int storage, int nw) { return (storage == 1 && nw == 2) ? 3 : 5; }
constexpr int fuse2_tw(int storage, int nw) { return 64 * nw - 2 * fuse2_xo(storage, nw); }
constexpr int FUSE2_NW_MIN = 2, FUSE2_NW_MAX = 4;
hipError_t launch_step2(int storage, int nw, char* base, const LatDesc* descs, const int* tiles, int ntot, int src,
                        int grid, hipStream_t s);
// LDS bytes of one fused block, and how many blocks the device keeps on one
// compute unit (0: no such kernel).
size_t step2_lds_bytes(int storage, int nw);
int step2_blocks_per_cu(int storage, int nw);
// Shared memory (bytes) one step block needs for tile width bx and ly rows;
// 0 if the storage has no step kernel of that width.
size_t step_lds_bytes(int storage, int bx, int ly);
hipError_t launch_init(int storage, char* base, const LatDesc* d, long long nsites, int buf,
                       const double* ra, const double* rb, const double* ux, const double* uy,
                       hipStream_t s);
hipError_t launch_fields(int storage, char* base, const LatDesc* d, long long nsites, int buf, int first,
                         double* ra, double* rb, double* ux, double* uy, hipStream_t s);
hipError_t launch_export(int storage, char* base, const LatDesc* d, long long nsites, int buf, int first,
                         int q, double* out, hipStream_t s);
hipError_t launch_sums(int storage, char* base, const LatDesc* d, int buf, int first, int nblocks,
                       double* partials, double* out, int* flag, hipStream_t s);
hipError_t launch_line_profile(int storage, char* base, const LatDesc* desc, int ny, int buf, int first,
                               double* out, hipStream_t s);
hipError_t launch_stress_reduce(char* base, const LatDesc* descs, int nlat, double* out, hipStream_t s);
hipError_t launch_profile_reduce(char* base, const LatDesc* d, int ny, double* out, hipStream_t s);
hipError_t launch_fill(double* p, long long n, double v, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, long long n16, int blocks, hipStream_t s);
int sums_blocks();

}  // namespace lbk
