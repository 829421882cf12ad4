/*
 * A plain C client of the library: no torch, no Python.  It allocates the
 * device state with the HIP runtime's C API, initialises a lattice from raw
 * float64 fields, advances it and writes the fields and the averaged wall
 * stress back out.  Used by the tests to show that include/lb.h is a C header
 * and that the library is driven through it alone.
 *
 *   lb_client NX NY STEPS STORAGE STEPS_PER_PASS U_WALL IN_PATH OUT_PATH
 *
 * IN_PATH holds rho_a, rho_b, ux, uy (each NY*NX float64, row-major); OUT_PATH
 * receives rho_a, rho_b, ux, uy after STEPS steps, then sigma_bot, sigma_top
 * (float64) and nsamples (int64).  Exit status 0 on success, 1 on any error
 * (the library's message goes to stderr).
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "lb.h"

static int fail(const char* what)
{
    fprintf(stderr, "lb_client: %s: %s\n", what, lb_last_error());
    return 1;
}

int main(int argc, char** argv)
{
    if (argc != 9) {
        fprintf(stderr, "usage: lb_client NX NY STEPS STORAGE STEPS_PER_PASS U_WALL IN OUT\n");
        return 1;
    }
    const int nx = atoi(argv[1]), ny = atoi(argv[2]), steps = atoi(argv[3]);
    const int storage = atoi(argv[4]), per_pass = atoi(argv[5]);
    const double u = atof(argv[6]);
    const size_t n = (size_t)nx * (size_t)ny;
    if (nx < 1 || ny < 2 || steps < 0) return 1;
    double* fields = malloc(4 * n * sizeof(double));
    if (!fields) return 1;
    FILE* in = fopen(argv[7], "rb");
    if (!in || fread(fields, sizeof(double), 4 * n, in) != 4 * n) {
        fprintf(stderr, "lb_client: cannot read %s\n", argv[7]);
        return 1;
    }
    fclose(in);

    lb_params p = {0};
    p.nx = nx;
    p.ny = ny;
    p.walls_y = 1;
    p.storage = storage;
    p.tau = 1.0;
    p.rho0 = 0.83;
    p.g_aa1 = -9.0;
    p.g_aa2 = 8.1;
    p.g_bb1 = -9.0;
    p.g_bb2 = 8.1;
    p.g_ab = 0.405;
    p.u_top = u;
    p.u_bot = -u;

    size_t bytes = 0;
    if (lb_state_bytes(&p, &bytes) != LB_OK) return fail("lb_state_bytes");
    void* state = NULL;
    if (hipMalloc(&state, bytes) != hipSuccess) {
        fprintf(stderr, "lb_client: hipMalloc of %zu bytes failed\n", bytes);
        return 1;
    }
    lb_handle* h = NULL;
    if (lb_init(&p, state, bytes, NULL, fields, fields + n, fields + 2 * n, fields + 3 * n, &h) != LB_OK)
        return fail("lb_init");
    if (lb_set_fusion(h, per_pass, 0) != LB_OK) return fail("lb_set_fusion");
    if (lb_step(h, steps) != LB_OK) return fail("lb_step");
    if (lb_fields(h, fields, fields + n, fields + 2 * n, fields + 3 * n) != LB_OK) return fail("lb_fields");
    double sig[2];
    int64_t ns = 0;
    if (lb_stress(h, &sig[0], &sig[1], &ns) != LB_OK) return fail("lb_stress");
    if (lb_destroy(h) != LB_OK) return fail("lb_destroy");
    if (hipFree(state) != hipSuccess) return 1;

    FILE* out = fopen(argv[8], "wb");
    if (!out || fwrite(fields, sizeof(double), 4 * n, out) != 4 * n || fwrite(sig, sizeof(double), 2, out) != 2 ||
        fwrite(&ns, sizeof(int64_t), 1, out) != 1) {
        fprintf(stderr, "lb_client: cannot write %s\n", argv[8]);
        return 1;
    }
    fclose(out);
    free(fields);
    return 0;
}
