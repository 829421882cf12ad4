/*
 * Plain FP64 CPU oracle for the two-species multirange Shan-Chen lattice
 * Boltzmann step of Benzi, Bernaschi, Sbragaglia & Succi, "Herschel-Bulkley
 * rheology from lattice kinetic theory of soft-glassy materials"
 * (arXiv:1004.5058).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition the HIP path is checked against.  Only the test-suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or helper with the HIP library.
 *
 * Everything is double precision, written as plain loops in the order the
 * paper states the method:
 *   1. moments       rho_s = sum_i f_is,  u = sum_s sum_i f_is c_i / sum_s rho_s
 *                    (Section "Lattice Boltzmann with multirange interactions",
 *                    definitions under Eq. (1))
 *   2. pseudo-potential  psi(rho) = rho0 (1 - exp(-rho/rho0))   (same section)
 *   3. forces        F_s = F^a_s + F^r_s + F^X_s                  (Eq. (2) and
 *                    the two force definitions after it)
 *   4. collision     f*_is = f_is - (f_is - f^eq_is(rho_s, u + tau F_s/rho_s))/tau
 *                    (Eq. (1), right-hand side, with the quadratic equilibrium)
 *                    where F_s also carries the species' share of the external
 *                    body force of the paper's driving, F_x(y) = F0 sin(k_f y)
 *                    (section "Numerical Results")
 *   5. streaming     f_is(r + c_i, t+1) = f*_is(r, t)             (Eq. (1), left)
 *
 * Readings of points the paper leaves open:
 *   - populations live on D2Q9; the 25-point two-belt set of Fig. 1 is the
 *     interaction stencil only (the paper ties c_S^2 and w_i to the D2Q9 set);
 *   - F^a and F^X use the D2Q9 weights on belt 1; F^r uses the two-belt weights
 *     p(|c|^2) = {4/63, 4/135, 1/180, 2/945, 1/15120} for |c|^2 = {1,2,4,5,8}
 *     (the unique isotropic set with the D2Q9 second moment whose fourth
 *     moment is 12/7 of the D2Q9 one, as the surface-tension combination
 *     G^a + (12/7) G^r requires);
 *   - G < 0 attracts, G > 0 repels (the force formulas govern the footnote);
 *   - walls (optional): half-way bounce-back at y = -1/2 and y = NY - 1/2 moving
 *     at u_bot, u_top along x, with the node's own pre-collision density in
 *     the moving-wall term; psi and rho beyond a wall are the even mirror of
 *     the fluid rows (row -1 <- row 0, row -2 <- row 1);
 *   - the external body force acts on the fluid as a whole and is shared
 *     between the species in proportion to their density,
 *     F_ext,s = (rho_s / (rho_A + rho_B)) F0 sin(k_f y), so that both
 *     species receive the same acceleration; y is the node's row index.
 *
 * Layout of a population array: f[((s*9 + i)*ny + y)*nx + x], s = 0 (A), 1 (B).
 * D2Q9 order: 0 (0,0); 1 (1,0); 2 (0,1); 3 (-1,0); 4 (0,-1);
 *             5 (1,1); 6 (-1,1); 7 (-1,-1); 8 (1,-1).
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nx, ny;
    int walls;          /* 0: periodic in y; 1: moving bounce-back walls in y */
    double tau;         /* BGK relaxation time, Eq. (1) */
    double rho0;        /* reference density of psi and of the F^X normaliser */
    double g_att[2];    /* G^a_AA, G^a_BB: belt 1, D2Q9 weights */
    double g_rep[2];    /* G^r_AA, G^r_BB: belts 1-2, two-belt weights */
    double g_ab;        /* G^X_AB = G^X_BA: belt 1, D2Q9 weights, acts on rho */
    double u_top, u_bot;/* wall velocities along x */
    double fx_amp, fx_k;/* body force F_x(y) = fx_amp sin(fx_k y); 0 = none */
} orc_params;

/* ---- lattice tables ---------------------------------------------------- */

static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0;

/* D2Q9 weight of an offset of belt 1 (|c|^2 = 1 or 2), zero elsewhere. */
static double w_belt1(int cx, int cy)
{
    int r2 = cx * cx + cy * cy;
    if (r2 == 1) return 1.0 / 9.0;
    if (r2 == 2) return 1.0 / 36.0;
    return 0.0;
}

/* Two-belt weight of an offset with max(|cx|,|cy|) <= 2, zero at the origin. */
static double w_belt12(int cx, int cy)
{
    switch (cx * cx + cy * cy) {
    case 1: return 4.0 / 63.0;
    case 2: return 4.0 / 135.0;
    case 4: return 1.0 / 180.0;
    case 5: return 2.0 / 945.0;
    case 8: return 1.0 / 15120.0;
    default: return 0.0;
    }
}

void orc_tables(int* cx, int* cy, double* w, int* opp)
{
    for (int i = 0; i < 9; ++i) { cx[i] = CX[i]; cy[i] = CY[i]; w[i] = W9[i]; opp[i] = OPP[i]; }
}

/* Weights the force uses for offset (cx, cy): belt-1 D2Q9 and two-belt. */
void orc_stencil_weight(int cx, int cy, double* wb1, double* wb12)
{
    *wb1 = w_belt1(cx, cy);
    *wb12 = (cx == 0 && cy == 0) ? 0.0 : w_belt12(cx, cy);
}

/* ---- pointwise pieces ---------------------------------------------------- */

/* Quadratic equilibrium of the D2Q9 lattice (definition under Eq. (1)):
 * f^eq_i = w_i rho [1 + u.c_i / cs2 + (u.c_i)^2/(2 cs2^2) - u.u/(2 cs2)]. */
void orc_equilibrium(double rho, double ux, double uy, double* feq)
{
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        feq[i] = W9[i] * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Shan-Chen pseudo-potential psi(rho) = rho0 (1 - exp(-rho/rho0)).  expm1 is
 * the same function evaluated without cancellation at small rho/rho0. */
double orc_psi(double rho, double rho0)
{
    return -rho0 * expm1(-rho / rho0);
}

/* ---- field helpers ------------------------------------------------------- */

static int wrap(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* Value of a scalar field at (x, y): periodic in x; in y periodic, or the even
 * mirror about the wall planes y = -1/2 and y = ny - 1/2. */
static double field_at(const orc_params* p, const double* g, int x, int y)
{
    int xx = wrap(x, p->nx);
    int yy;
    if (!p->walls) {
        yy = wrap(y, p->ny);
    } else {
        yy = y;
        if (yy < 0) yy = -1 - yy;
        if (yy >= p->ny) yy = 2 * p->ny - 1 - yy;
    }
    return g[(size_t)yy * p->nx + xx];
}

/* Moments of the populations (definitions under Eq. (1)). */
void orc_fields(const orc_params* p, const double* f, double* rho_a, double* rho_b,
                double* ux, double* uy)
{
    size_t n = (size_t)p->nx * p->ny;
    for (size_t k = 0; k < n; ++k) {
        double rho[2] = {0.0, 0.0}, jx = 0.0, jy = 0.0;
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < 9; ++i) {
                double v = f[(size_t)(s * 9 + i) * n + k];
                rho[s] += v;
                jx += v * CX[i];
                jy += v * CY[i];
            }
        if (rho_a) rho_a[k] = rho[0];
        if (rho_b) rho_b[k] = rho[1];
        if (ux) ux[k] = jx / (rho[0] + rho[1]);
        if (uy) uy[k] = jy / (rho[0] + rho[1]);
    }
}

/* Forces of Eq. (2) from the density fields.
 *   F^{a}_s = -G^a_s psi_s(r) sum_{belt 1}    w_i c_i psi_s(r + c_i)
 *   F^{r}_s = -G^r_s psi_s(r) sum_{belts 1-2} p_i c_i psi_s(r + c_i)
 *   F^{X}_s = -(G_AB/rho0) rho_s(r) sum_{belt 1} w_i c_i rho_s'(r + c_i), s != s'
 * Outputs are nx*ny arrays; any output pointer may be NULL. */
void orc_force(const orc_params* p, const double* rho_a, const double* rho_b,
               double* fax, double* fay, double* fbx, double* fby)
{
    int nx = p->nx, ny = p->ny;
    size_t n = (size_t)nx * ny;
    double* psi[2];
    psi[0] = (double*)malloc(n * sizeof(double));
    psi[1] = (double*)malloc(n * sizeof(double));
    for (size_t k = 0; k < n; ++k) {
        psi[0][k] = orc_psi(rho_a[k], p->rho0);
        psi[1][k] = orc_psi(rho_b[k], p->rho0);
    }
    const double* rho[2] = {rho_a, rho_b};

#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t k = (size_t)y * nx + x;
            for (int s = 0; s < 2; ++s) {
                int o = 1 - s;
                double sa_x = 0, sa_y = 0, sr_x = 0, sr_y = 0, sx_x = 0, sx_y = 0;
                for (int cy = -2; cy <= 2; ++cy)
                    for (int cx = -2; cx <= 2; ++cx) {
                        if (cx == 0 && cy == 0) continue;
                        double wb1 = w_belt1(cx, cy);
                        double wb12 = w_belt12(cx, cy);
                        double ps = field_at(p, psi[s], x + cx, y + cy);
                        if (wb1 != 0.0) {
                            double ro = field_at(p, rho[o], x + cx, y + cy);
                            sa_x += wb1 * cx * ps;
                            sa_y += wb1 * cy * ps;
                            sx_x += wb1 * cx * ro;
                            sx_y += wb1 * cy * ro;
                        }
                        sr_x += wb12 * cx * ps;
                        sr_y += wb12 * cy * ps;
                    }
                double ps0 = psi[s][k];
                double r0 = rho[s][k];
                double Fx = -p->g_att[s] * ps0 * sa_x - p->g_rep[s] * ps0 * sr_x
                            - (p->g_ab / p->rho0) * r0 * sx_x;
                double Fy = -p->g_att[s] * ps0 * sa_y - p->g_rep[s] * ps0 * sr_y
                            - (p->g_ab / p->rho0) * r0 * sx_y;
                if (s == 0) {
                    if (fax) fax[k] = Fx;
                    if (fay) fay[k] = Fy;
                } else {
                    if (fbx) fbx[k] = Fx;
                    if (fby) fby[k] = Fy;
                }
            }
        }
    }
    free(psi[0]);
    free(psi[1]);
}

/* Initial populations: the equilibrium of the given densities and velocity. */
void orc_init(const orc_params* p, const double* rho_a, const double* rho_b,
              const double* ux, const double* uy, double* f)
{
    size_t n = (size_t)p->nx * p->ny;
    for (size_t k = 0; k < n; ++k) {
        double u = ux ? ux[k] : 0.0, v = uy ? uy[k] : 0.0;
        double feq[9];
        for (int s = 0; s < 2; ++s) {
            orc_equilibrium(s == 0 ? rho_a[k] : rho_b[k], u, v, feq);
            for (int i = 0; i < 9; ++i) f[(size_t)(s * 9 + i) * n + k] = feq[i];
        }
    }
}

/* Post-collision populations f* (right-hand side of Eq. (1)), written into
 * fstar.  Also returns the pre-collision densities (needed by the walls). */
void orc_collide(const orc_params* p, const double* f, double* fstar,
                 double* rho_a, double* rho_b)
{
    int nx = p->nx, ny = p->ny;
    size_t n = (size_t)nx * ny;
    double* ux = (double*)malloc(n * sizeof(double));
    double* uy = (double*)malloc(n * sizeof(double));
    double* F[4];
    for (int q = 0; q < 4; ++q) F[q] = (double*)malloc(n * sizeof(double));

    orc_fields(p, f, rho_a, rho_b, ux, uy);
    orc_force(p, rho_a, rho_b, F[0], F[1], F[2], F[3]);

#pragma omp parallel for schedule(static)
    for (long long kk = 0; kk < (long long)n; ++kk) {
        size_t k = (size_t)kk;
        double fext = p->fx_amp * sin(p->fx_k * (double)(k / (size_t)nx));
        for (int s = 0; s < 2; ++s) {
            double rs = (s == 0) ? rho_a[k] : rho_b[k];
            double fsx = F[2 * s][k] + fext * rs / (rho_a[k] + rho_b[k]);
            double vx = ux[k] + p->tau * fsx / rs;
            double vy = uy[k] + p->tau * F[2 * s + 1][k] / rs;
            double feq[9];
            orc_equilibrium(rs, vx, vy, feq);
            for (int i = 0; i < 9; ++i) {
                size_t a = (size_t)(s * 9 + i) * n + k;
                fstar[a] = f[a] - (f[a] - feq[i]) / p->tau;
            }
        }
    }
    free(ux);
    free(uy);
    for (int q = 0; q < 4; ++q) free(F[q]);
}

/* Streaming with the boundary conditions.  Every post-collision population
 * moves to r + c_i.  With walls, a population whose target row lies beyond a
 * wall returns to its own node with the opposite velocity, shifted by the
 * moving-wall term 2 w_i rho_s (c_ibar . u_w) / cs2.  The momentum each such
 * link hands to the wall, c_i (f*_i + f_new_ibar), is summed into
 * wall_fx[0] (bottom wall) and wall_fx[1] (top wall), x component. */
void orc_stream(const orc_params* p, const double* fstar, const double* rho_a,
                const double* rho_b, double* fnew, double* wall_fx)
{
    int nx = p->nx, ny = p->ny;
    size_t n = (size_t)nx * ny;
    double fb = 0.0, ft = 0.0;
    for (int s = 0; s < 2; ++s) {
        const double* rho = (s == 0) ? rho_a : rho_b;
        for (int i = 0; i < 9; ++i) {
            for (int y = 0; y < ny; ++y) {
                for (int x = 0; x < nx; ++x) {
                    size_t src = (size_t)(s * 9 + i) * n + (size_t)y * nx + x;
                    int yt = y + CY[i];
                    int xt = wrap(x + CX[i], nx);
                    if (!p->walls) {
                        yt = wrap(yt, ny);
                        fnew[(size_t)(s * 9 + i) * n + (size_t)yt * nx + xt] = fstar[src];
                    } else if (yt >= 0 && yt < ny) {
                        fnew[(size_t)(s * 9 + i) * n + (size_t)yt * nx + xt] = fstar[src];
                    } else {
                        int ib = OPP[i];
                        double uw = (yt < 0) ? p->u_bot : p->u_top;
                        double rw = rho[(size_t)y * nx + x];
                        double back = fstar[src] + 2.0 * W9[ib] * rw * (CX[ib] * uw) / CS2;
                        fnew[(size_t)(s * 9 + ib) * n + (size_t)y * nx + x] = back;
                        double dpx = CX[i] * (fstar[src] + back);
                        if (yt < 0) fb += dpx; else ft += dpx;
                    }
                }
            }
        }
    }
    if (wall_fx) { wall_fx[0] = fb; wall_fx[1] = ft; }
}

/* One full time step f(t) -> f(t+1).  wall_fx as in orc_stream. */
void orc_step(const orc_params* p, const double* f, double* fnew, double* wall_fx)
{
    size_t n = (size_t)p->nx * p->ny;
    double* fstar = (double*)malloc(18 * n * sizeof(double));
    double* ra = (double*)malloc(n * sizeof(double));
    double* rb = (double*)malloc(n * sizeof(double));
    orc_collide(p, f, fstar, ra, rb);
    orc_stream(p, fstar, ra, rb, fnew, wall_fx);
    free(fstar);
    free(ra);
    free(rb);
}

/* nsteps steps in place on f.  stress[0..1] receive the sums over the steps of
 * the instantaneous wall shear stresses sigma_bot = F_bot,x / nx and
 * sigma_top = -F_top,x / nx (both positive for a top wall faster than the
 * bottom one). */
void orc_run(const orc_params* p, double* f, int nsteps, double* stress)
{
    size_t n = (size_t)p->nx * p->ny;
    double* g = (double*)malloc(18 * n * sizeof(double));
    double sb = 0.0, st = 0.0;
    for (int t = 0; t < nsteps; ++t) {
        double wf[2];
        orc_step(p, f, g, wf);
        sb += wf[0] / p->nx;
        st += -wf[1] / p->nx;
        memcpy(f, g, 18 * n * sizeof(double));
    }
    free(g);
    if (stress) { stress[0] = sb; stress[1] = st; }
}

/* Domain sums of the two species masses and of the total momentum. */
void orc_sums(const orc_params* p, const double* f, double* out4)
{
    size_t n = (size_t)p->nx * p->ny;
    double m[2] = {0, 0}, jx = 0, jy = 0;
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < 9; ++i)
            for (size_t k = 0; k < n; ++k) {
                double v = f[(size_t)(s * 9 + i) * n + k];
                m[s] += v;
                jx += v * CX[i];
                jy += v * CY[i];
            }
    out4[0] = m[0];
    out4[1] = m[1];
    out4[2] = jx;
    out4[3] = jy;
}

/* Threads the parallel loops above run on (reported beside the oracle's timing). */
int orc_threads(void)
{
    return omp_get_max_threads();
}
