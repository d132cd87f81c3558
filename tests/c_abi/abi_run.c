/*
 * abi_run.c -- drives the library through its C ABI alone (no Python, no
 * torch): device buffers from the HIP runtime, one D2Q9 FP64 run of the
 * coupled step, the FP64 sums, and the particle budget checked.
 *
 * Usage: abi_run [steps]  (prints one JSON line; exit status 0 when the
 * budget sum C + deposit closes to 1e-12).  The initial concentration uses
 * exact arithmetic only, so any other caller can rebuild it bit for bit:
 *   C(x, y) = (y >= ny/2 ? 1 : 0) + 1e-3 * ((7x + 13y) mod 17) / 17.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "lbw.h"

#define CHECK_HIP(call)                                                          \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));          \
            return 2;                                                            \
        }                                                                        \
    } while (0)

#define CHECK_LBW(call)                                                          \
    do {                                                                         \
        int rc_ = (call);                                                        \
        if (rc_ != LBW_OK) {                                                     \
            fprintf(stderr, "%s: %d %s\n", #call, rc_, lbw_last_error());       \
            return 3;                                                            \
        }                                                                        \
    } while (0)

int main(int argc, char **argv)
{
    const int nx = 64, ny = 128, steps = argc > 1 ? atoi(argv[1]) : 100;
    const size_t n = (size_t)nx * ny;
    lbw_config cfg = {0};
    lbw_buffers buf = {0};
    lbw_handle *h = NULL;
    double *c = NULL, mass0 = 0.0, mass = 0.0, dep = 0.0, fluid0 = 0.0, fluid = 0.0;
    size_t scratch = 0;
    int x, y, ok;

    if (lbw_version() != LBW_ABI_VERSION) {
        fprintf(stderr, "library ABI %d, header %d\n", lbw_version(), LBW_ABI_VERSION);
        return 4;
    }
    cfg.lattice = LBW_D2Q9;
    cfg.precision = LBW_FP64;
    cfg.nx = nx;
    cfg.ny = ny;
    cfg.nz = 1;
    cfg.fluid_mode = LBW_FLUID_LBM;
    cfg.scheme_c = LBW_WENO5;
    cfg.tau = 0.6;
    cfg.vs = 1e-3;
    cfg.kappa_c = 1e-3;
    cfg.gp_c = 1e-5;
    cfg.weno_eps = 1e-6;

    CHECK_HIP(hipMalloc(&buf.f, 9 * n * sizeof(double)));
    CHECK_HIP(hipMalloc(&buf.c, n * sizeof(double)));
    CHECK_HIP(hipMalloc(&buf.c_s1, n * sizeof(double)));
    CHECK_HIP(hipMalloc(&buf.c_s2, n * sizeof(double)));
    CHECK_HIP(hipMalloc(&buf.u, 2 * n * sizeof(double)));
    CHECK_HIP(hipMalloc((void **)&buf.deposit, (size_t)nx * sizeof(double)));
    CHECK_HIP(hipMemset(buf.deposit, 0, (size_t)nx * sizeof(double)));
    CHECK_LBW(lbw_scratch_bytes(&cfg, 1, &scratch));
    CHECK_HIP(hipMalloc(&buf.scratch, scratch));
    buf.scratch_bytes = scratch;

    c = (double *)malloc(n * sizeof(double));
    if (!c) return 5;
    for (y = 0; y < ny; y++)
        for (x = 0; x < nx; x++)
            c[x + (size_t)nx * y] = (y >= ny / 2 ? 1.0 : 0.0) + 1e-3 * (double)((7 * x + 13 * y) % 17) / 17.0;
    CHECK_HIP(hipMemcpy(buf.c, c, n * sizeof(double), hipMemcpyHostToDevice));

    CHECK_LBW(lbw_create(&cfg, &buf, 1, NULL, &h));
    CHECK_LBW(lbw_init_equilibrium(h, 0, NULL, NULL));
    CHECK_LBW(lbw_reduce(h, LBW_MASS_C, &mass0));
    CHECK_LBW(lbw_reduce(h, LBW_MASS_FLUID, &fluid0));
    CHECK_LBW(lbw_step(h, steps));
    CHECK_LBW(lbw_reduce(h, LBW_MASS_C, &mass));
    CHECK_LBW(lbw_reduce(h, LBW_DEPOSIT, &dep));
    CHECK_LBW(lbw_reduce(h, LBW_MASS_FLUID, &fluid));
    lbw_destroy(h);

    ok = fabs(mass + dep - mass0) <= 1e-12 * mass0 && fabs(fluid - fluid0) <= 1e-12 * fluid0;
    printf("{\"steps\": %d, \"mass0\": %.17g, \"mass\": %.17g, \"deposit\": %.17g, "
           "\"fluid0\": %.17g, \"fluid\": %.17g, \"budget_closed\": %s}\n",
           steps, mass0, mass, dep, fluid0, fluid, ok ? "true" : "false");
    free(c);
    hipFree(buf.f);
    hipFree(buf.c);
    hipFree(buf.c_s1);
    hipFree(buf.c_s2);
    hipFree(buf.u);
    hipFree(buf.deposit);
    hipFree(buf.scratch);
    return ok ? 0 : 1;
}
