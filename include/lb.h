/*
 * lb.h - C ABI of the MI355X (gfx950) two-species multirange lattice
 * Boltzmann library.
 *
 * The method (Benzi, Bernaschi, Sbragaglia & Succi, arXiv:1004.5058, section
 * "Lattice Boltzmann with multirange interactions"):
 *   f_is(r + c_i, t + 1) - f_is(r, t) =
 *       -(1/tau) [ f_is(r, t) - f^eq_is(rho_s, u + tau F_s / rho_s) ]     Eq. (1)
 *   rho_s = sum_i f_is,  u = sum_s sum_i f_is c_i / sum_s rho_s
 *   f^eq_i(rho, v) = w_i rho [1 + v.c_i/c_S^2 + (v.c_i)^2/(2 c_S^4) - v.v/(2 c_S^2)]
 *   F_s = F^a_s + F^r_s + F^X_s                                           Eq. (2)
 *   F^a_s = -G^a_s psi_s(r) sum_{belt 1}     w_i c_i psi_s(r + c_i)
 *   F^r_s = -G^r_s psi_s(r) sum_{belts 1-2}  p_i c_i psi_s(r + c_i)
 *   F^X_s = -(G_AB / rho0) rho_s(r) sum_{belt 1} w_i c_i rho_s'(r + c_i)
 *   psi(rho) = rho0 (1 - exp(-rho / rho0))
 * on the D2Q9 lattice (c_S^2 = 1/3) with the 24-offset interaction stencil of
 * Fig. 1.  Belt 1 uses the D2Q9 weights; belts 1-2 use the isotropic two-belt
 * weights p = 4/63, 4/135, 1/180, 2/945, 1/15120 for |c|^2 = 1, 2, 4, 5, 8.
 * G < 0 attracts, G > 0 repels.
 *
 * Geometry: x (index fastest) is periodic.  y is either periodic or bounded by
 * half-way bounce-back walls at y = -1/2 and y = ny - 1/2 moving along x at
 * u_bot and u_top.  A population leaving through a wall returns to its node
 * reversed, plus 2 w_i rho_s (c_i . u_wall)/c_S^2 with rho_s the node's
 * pre-collision density.  psi and rho beyond a wall are the even mirror of the
 * first two fluid rows.
 *
 * D2Q9 direction order used wherever populations cross this ABI:
 *   0 (0,0)  1 (1,0)  2 (0,1)  3 (-1,0)  4 (0,-1)
 *   5 (1,1)  6 (-1,1) 7 (-1,-1) 8 (1,-1)
 *
 * Conventions
 *   - Every function returns an lb_status; a negative value is an error and
 *     lb_last_error() (thread-local) describes it.  No C++ exception crosses
 *     this boundary.
 *   - Device memory: the caller allocates the device state (any allocator; a
 *     torch uint8 tensor works) of the size lb_state_bytes / lbb_state_bytes
 *     report, keeps it alive until *_destroy, and frees it afterwards.  The
 *     handle owns only host metadata and HIP graphs; *_destroy never frees the
 *     caller's memory.  The state must be 256-byte aligned.
 *   - Streams: all device work is enqueued on the hipStream_t given at init
 *     (NULL = the legacy default stream).  lb_step / lbb_step only enqueue;
 *     functions that return host data synchronise that stream.
 *   - Host arrays of fields are float64, row-major (ny, nx), x fastest.
 *   - Calls on one handle must not overlap (not thread-safe per handle).
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LB_OK = 0,
    LB_EINVAL = -1,      /* invalid argument (bad size, tau <= 1/2, non-finite or rho <= 0 input, ...) */
    LB_ENOMEM = -2,      /* caller's device state too small, or a host allocation failed */
    LB_EDEVICE = -3,     /* a HIP runtime call failed (message has the HIP error string) */
    LB_ENONFINITE = -4,  /* the watchdog found a non-finite or non-positive density */
    LB_ESTATE = -5       /* call out of order (e.g. load of a checkpoint of another shape) */
} lb_status;

/* Storage of the state.  The population formats (LB_F64 .. LB_BF16DEV) store
 * the deviation d_is = f_is - w_i rho_ref_s from the rest equilibrium at the
 * reference densities, rounded to nearest-even, and the step computes on
 * deviations (density deviations, deviations of psi from psi(rho_ref)), so the
 * rounding error scales with the departure from the reference state rather
 * than with f itself.  Arithmetic is FP64 for LB_F64 and FP32 otherwise; a
 * step stores each post-collision deviation computed in the arithmetic type
 * and then rounded to the storage format (one rule for every kernel and launch
 * shape).
 *
 * LB_MOM32 / LB_MOM64 (FP32 / FP64): the moment form, valid only at tau = 1
 * (lb_params.tau must be exactly 1; anything else is LB_EINVAL).  With tau = 1
 * the BGK collision of Eq. (1) replaces every population by the equilibrium at
 * the shifted velocity, so the post-collision state is the six moments
 * (rho_s - rho_ref_s, v_s) per site; each step rebuilds the incoming
 * populations from their source sites.  Same recurrence, 6 loads and 6 stores
 * per site instead of 36.  lb_populations, lb_fields and lb_sums return the
 * same quantities as for the population formats. */
typedef enum { LB_F64 = 0, LB_F32 = 1, LB_F16DEV = 2, LB_BF16DEV = 3, LB_MOM32 = 4, LB_MOM64 = 5 } lb_storage;

typedef struct {
    int32_t nx, ny;       /* lattice sites along x (periodic) and y; 1 <= nx, 2 <= ny */
    int32_t walls_y;      /* 0: periodic in y; 1: moving bounce-back walls */
    int32_t storage;      /* lb_storage */
    double tau;           /* BGK relaxation time, > 1/2 (Eq. (1)) */
    double rho0;          /* psi reference density and F^X normaliser, > 0 */
    double g_aa1, g_aa2;  /* G^a_AA (belt 1), G^r_AA (belts 1-2) */
    double g_bb1, g_bb2;  /* G^a_BB, G^r_BB */
    double g_ab;          /* G^X_AB = G^X_BA (belt 1) */
    double u_top, u_bot;  /* wall velocities along x (walls_y = 1) */
    double rho_ref_a, rho_ref_b; /* storage base; <= 0 selects the domain mean of
                                    the initial density of that species */
    int32_t profile;      /* 1: accumulate the line-averaged u_x(y) every step */
    int32_t reserved;
    double fx_amp;        /* external body force along x per site, F_x(y) = fx_amp sin(fx_k y) with
                             y the row index (the driving of section "Numerical Results"); it is
                             shared between the species in proportion to their density, so both
                             receive the acceleration F_x / (rho_A + rho_B); 0 = none */
    double fx_k;          /* wavenumber of the body force (2 pi / L in the paper's protocol) */
} lb_params;

typedef struct lb_handle lb_handle;
typedef struct lbb_handle lbb_handle;

/* Device bytes a single lattice with these parameters needs. */
lb_status lb_state_bytes(const lb_params* p, size_t* bytes);

/* Validates p, lays the lattice out in dev_state and sets
 * f_is(r, 0) = f^eq_i(rho_s(r), u(r)).  rho_a, rho_b: host (ny, nx) float64,
 * finite and > 0.  ux, uy: host (ny, nx) float64 or NULL for zero.  Blocks
 * until the initial state is on the device. */
lb_status lb_init(const lb_params* p, void* dev_state, size_t bytes, void* hip_stream,
                  const double* rho_a, const double* rho_b, const double* ux, const double* uy,
                  lb_handle** out);

/* Enqueues n >= 0 time steps of Eq. (1) (collision, forcing, streaming, walls)
 * and the wall-stress accumulation.  Asynchronous. */
lb_status lb_step(lb_handle* h, int32_t n);

/* Moments of the current populations, computed in FP64 on the device and
 * copied to host arrays (any may be NULL): rho_a, rho_b, and u = j / rho.
 * Synchronises the stream. */
lb_status lb_fields(lb_handle* h, double* rho_a, double* rho_b, double* ux, double* uy);

/* Same, into caller-provided device arrays (ny*nx float64 each, any may be
 * NULL).  Asynchronous. */
lb_status lb_fields_device(lb_handle* h, double* rho_a, double* rho_b, double* ux, double* uy);

/* The current populations decoded to float64, host array of shape
 * (2, 9, ny, nx) in the direction order above.  Synchronises. */
lb_status lb_populations(lb_handle* h, double* f);

/* Time-averaged wall shear stress over the steps since init or the last
 * lb_stress_reset: sigma_bot = <F_bot,x>/nx and sigma_top = -<F_top,x>/nx
 * with F the x momentum a wall receives per step (both positive when the top
 * wall moves faster than the bottom one).  nsamples = steps averaged.  The
 * per-step sums are accumulated in FP64 on the device.  Synchronises. */
lb_status lb_stress(lb_handle* h, double* sig_bot, double* sig_top, int64_t* nsamples);
lb_status lb_stress_reset(lb_handle* h);

/* Instantaneous line-averaged speed U_x(y, t) = (1/nx) sum_x u_x(x, y, t) of the
 * current populations, u the barycentric velocity (section "Numerical
 * Results": the profile whose sine transform is the response R(t)).  FP64 on
 * the device; prof: host array of ny doubles.  Leaves the time-averaging
 * accumulators alone.  Synchronises. */
lb_status lb_line_profile(lb_handle* h, double* prof);

/* Time average of U_x(y) = (1/nx) sum_x u_x(x, y) over the same window as
 * lb_stress (requires p->profile = 1).  prof: host array of ny doubles.  The
 * u_x averaged is the pre-collision barycentric velocity of each step. */
lb_status lb_profile(lb_handle* h, double* prof, int64_t* nsamples);

/* FP64 domain sums: out[0] = mass A, out[1] = mass B, out[2] = sum j_x,
 * out[3] = sum j_y, out[4] = number of sites with a non-finite or
 * non-positive density.  Synchronises; returns LB_ENONFINITE if out[4] > 0. */
lb_status lb_sums(lb_handle* h, double out[5]);

/* Run the sums every `every` steps inside lb_step (0 = off, the default) and
 * latch a device flag; lb_fields/lb_stress/lb_sums then report
 * LB_ENONFINITE. */
lb_status lb_set_watchdog(lb_handle* h, int32_t every);

/* Launch shape of the step kernel: bx threads per block (64, 128 or 256, and
 * 512 for FP32 and 16-bit population storage) = lattice columns per tile, ly
 * rows per tile (>= 1).  0 keeps the current choice.  LB_EINVAL for another
 * bx or for a shape whose shared memory per block (it grows with bx and ly)
 * exceeds the device's limit.  Results are bitwise independent of the shape. */
lb_status lb_set_launch(lb_handle* h, int32_t bx, int32_t ly);

/* HIP graph use in lb_step: steps per captured graph (0 = launch each step
 * directly).  Default 32. */
lb_status lb_set_graph(lb_handle* h, int32_t steps_per_graph);

/* Time steps per pass of the step kernel over the populations: 1 (default)
 * or 2.  With 2, lb_step advances pairs of steps (Eq. (1) applied twice) with
 * one kernel that keeps the intermediate populations in on-chip memory, so
 * each population crosses HBM once per two updates; an odd remaining step
 * runs alone.  Populations and wall stress are bitwise those of single
 * steps; the line profile (lb_profile), when on, is accumulated too, from
 * partial sums grouped by the fused kernel's tiles, so it agrees with single
 * steps to FP64 rounding.  Tiles of W columns (W from lb_set_fusion_tile)
 * and at most ly2 rows: each lattice's rows are cut into ceil(ny / ly2)
 * segments of near-equal height, one more while they would all be the same
 * multiple of 16 rows; a batch hands out its lattices' tiles tallest segments
 * first.  ly2 = 0: the height whose tiles, handed out greedily to the blocks
 * the device runs at once at h + 8 ticks per tile of h rows, finish first.
 * Results are bitwise independent of the tiles.  LB_EINVAL unless the storage
 * is LB_F32, LB_F16DEV or LB_BF16DEV and the device grants the kernel's
 * shared memory. */
lb_status lb_set_fusion(lb_handle* h, int32_t steps_per_pass, int32_t ly2);

/* Block width of the two-steps-per-pass kernel: lanes = 128, 192 or 256
 * threads per time step (the block has twice as many), or 0 for the width
 * with the most waves resident per compute unit.  A tile stores lanes - 6
 * columns (FP32 at 128 lanes) or lanes - 10 (the other widths and the 16-bit
 * forms): the step-t columns beyond them are the overlap step t+1 needs (for
 * lanes - 10 also the two columns each side whose densities step t's stencil
 * needs, which FP32 at 128 lanes loads as halo columns).
 * Results are bitwise independent of the width.
 * LB_EINVAL for another value. */
lb_status lb_set_fusion_tile(lb_handle* h, int32_t lanes);
/* The width in effect (automatic choice resolved) and its stored columns per
 * tile; either pointer may be NULL. */
lb_status lb_get_fusion_tile(lb_handle* h, int32_t* lanes, int32_t* columns);

/* The launch configuration in effect (as lb_set_launch / lb_set_fusion /
 * lb_autotune left it): tile width bx and height ly of the single-step
 * kernel, time steps per pass, and the fused tiles' height with the automatic
 * choice resolved (reported whatever the steps per pass).  Any pointer may be
 * NULL.  Host only, never fails on a valid handle. */
lb_status lb_get_launch(lb_handle* h, int32_t* bx, int32_t* ly, int32_t* steps_per_pass, int32_t* ly2);

/* Checkpoint: the populations in their storage format, the step count and
 * the FP64 stress/profile accumulators.  lb_save with buf = NULL reports the
 * size in *bytes.  Both synchronise.  lb_load requires a handle of the same
 * shape and storage (else LB_ESTATE). */
lb_status lb_save(lb_handle* h, void* buf, size_t* bytes);
lb_status lb_load(lb_handle* h, const void* buf, size_t bytes);

/* Autotuner: after about 0.3 s of steps to bring the GPU's clocks up, times
 * `steps` steps of every candidate launch shape (bx in {64, 128, 256, 512} as
 * lb_set_launch admits them, ly in {8..256}, shapes within the device's shared
 * memory per block; for batches also persistent grids of 1, 2 and 4 blocks
 * per compute unit) on this lattice; where lb_set_fusion admits two steps per
 * pass (FP32, 16-bit), also that mode behind the best shape, for each block
 * width of lb_set_fusion_tile the device grants, at the automatic tile height
 * and at heights of 20 to 300 rows (odd multiples of 4); then times the four
 * fastest candidates twice more over 4 x steps steps.  Applies the fastest of
 * those (shape, steps per pass and fused width; *ms is its time per step) and
 * restores the simulation state exactly (populations, accumulators, step
 * count).  cache_path (may be NULL): JSON file of {key: {bx, ly, grid,
 * fusion, ly2, fw, ms}}, key "<gfx arch>/<storage>/<nx>x<ny>" (batches:
 * "batch<n>_<sites>"); a cached entry is applied without timing (its fusion
 * only where admitted; entries without it mean one step per pass, without fw
 * the automatic width), a new result is added.  Synchronises.  Allocates a
 * temporary device copy of the state while timing. */
lb_status lb_autotune(lb_handle* h, const char* cache_path, int32_t steps, int32_t* bx, int32_t* ly,
                      double* ms);
lb_status lbb_autotune(lbb_handle* h, const char* cache_path, int32_t steps, int32_t* bx, int32_t* ly,
                       int32_t* grid, double* ms);

/* Achievable read+write HBM bandwidth: copies `bytes` (multiple of 16,
 * 16-byte aligned device buffers) src -> dst `reps` times with a streaming
 * 16-byte-per-lane kernel on hip_stream and returns (read + write bytes) /
 * time in GB/s.  Synchronises.  A measurement reference, not part of a step. */
lb_status lb_copy_peak(void* dst, const void* src, size_t bytes, void* hip_stream, int32_t reps, double* gbs);

/* Steps taken since init (or restored by lb_load). */
lb_status lb_time(lb_handle* h, int64_t* t);

/* Releases the handle (not the caller's device memory). */
lb_status lb_destroy(lb_handle* h);

/* Message of the last error on this thread ("" if none). */
const char* lb_last_error(void);

/* ------------------------------------------------------------------------
 * Batched form: n independent lattices of their own sizes and parameters,
 * advanced together by one persistent step kernel per time step (HIP graph
 * of many steps).  All lattices share the storage precision of params[0].
 * Arrays of per-lattice host pointers follow the single-lattice rules.
 * lbb_init checks the lattices' initial fields on up to 16 host threads, one
 * lattice at a time each (the threads end before it returns); a bad field
 * fails with LB_EINVAL naming the lowest-numbered lattice at fault and its
 * first offending site, before any device work.
 */
lb_status lbb_state_bytes(const lb_params* params, int32_t n, size_t* bytes);
lb_status lbb_init(const lb_params* params, int32_t n, void* dev_state, size_t bytes,
                   void* hip_stream, const double* const* rho_a, const double* const* rho_b,
                   const double* const* ux, const double* const* uy, lbb_handle** out);
lb_status lbb_step(lbb_handle* h, int32_t nsteps);
/* Per-lattice time-averaged wall stresses (arrays of n) and sample count. */
lb_status lbb_stress(lbb_handle* h, double* sig_bot, double* sig_top, int64_t* nsamples);
/* lbb_stress for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * results, bitwise, with the per-lattice reduction staged in a device array
 * the library holds (16 bytes per lattice, 64 KiB on each GPU it runs on, until
 * the process ends) instead of the caller's state, and no host or device
 * allocation by the library.  Batches of at most 4096 lattices (LB_EINVAL
 * beyond).  sig_bot / sig_top: host arrays of n doubles (either may be NULL).
 * The handle's device must be current.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (other threads or processes' streams)
 * race.  Synchronises the handle's stream. */
lb_status lbb_stress_noalloc(lbb_handle* h, double* sig_bot, double* sig_top, int64_t* nsamples);
lb_status lbb_stress_reset(lbb_handle* h);
/* Lattice k's fields / profile, as lb_fields / lb_profile. */
lb_status lbb_fields(lbb_handle* h, int32_t k, double* rho_a, double* rho_b, double* ux, double* uy);
lb_status lbb_profile(lbb_handle* h, int32_t k, double* prof, int64_t* nsamples);
lb_status lbb_line_profile(lbb_handle* h, int32_t k, double* prof);
/* Launch shape (as lb_set_launch) and grid size (0 = one block per tile,
 * > 0 = persistent grid of that many blocks). */
lb_status lbb_set_launch(lbb_handle* h, int32_t bx, int32_t ly, int32_t grid);
lb_status lbb_set_graph(lbb_handle* h, int32_t steps_per_graph);
lb_status lbb_destroy(lbb_handle* h);

/* Device time of the last `nsteps` steps of one lattice or batch, measured
 * with HIP events around the step kernels on the handle's stream: average
 * milliseconds per time step (a two-steps-per-pass launch counts as two
 * steps).  Enqueues nsteps steps and synchronises.  Used by the benchmark for
 * the roofline figure. */
lb_status lb_time_steps(lb_handle* h, int32_t nsteps, double* ms_per_step);
lb_status lbb_time_steps(lbb_handle* h, int32_t nsteps, double* ms_per_step);
/* lb_set_fusion, lb_set_fusion_tile and lb_get_fusion_tile for a batch. */
lb_status lbb_set_fusion(lbb_handle* h, int32_t steps_per_pass, int32_t ly2);
lb_status lbb_set_fusion_tile(lbb_handle* h, int32_t lanes);
lb_status lbb_get_fusion_tile(lbb_handle* h, int32_t* lanes, int32_t* columns);
/* lb_get_launch for a batch, with its persistent grid (0: one block per tile). */
lb_status lbb_get_launch(lbb_handle* h, int32_t* bx, int32_t* ly, int32_t* grid, int32_t* steps_per_pass,
                         int32_t* ly2);

#ifdef __cplusplus
}
#endif
#endif /* LB_H */
