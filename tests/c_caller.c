/* A plain C99 caller of liblbm (include/lbm.h), as a C user would write one:
 * a 48^3 lid-driven cavity (D3Q19 TRT, FP32 arithmetic over FP16S storage,
 * lid velocity 0.05 along y at the top z face) on the null stream, 300 steps,
 * then the FP64 diagnostics and the host moments.  Prints one line of
 * key=value figures and exits 0, or prints the library's error and exits 1.
 * Also checks that a few invalid calls are refused with LBM_EINVAL. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"

#define CHECK(call)                                                          \
    do {                                                                     \
        lbm_status st_ = (call);                                             \
        if (st_ != LBM_OK) {                                                 \
            fprintf(stderr, "%s -> %d: %s\n", #call, (int)st_, lbm_last_error()); \
            return 1;                                                        \
        }                                                                    \
    } while (0)

int main(void) {
    const int n = 48, steps = 300;
    const size_t N = (size_t)n * n * n;
    lbm_params p;
    memset(&p, 0, sizeof p);
    p.nx = p.ny = p.nz = n;
    p.q = LBM_D3Q19;
    p.collision = LBM_TRT;
    p.storage = LBM_FP16S;
    p.arith = LBM_ARITH_FP32;
    p.tau = 0.6;
    p.trt_magic = 0.25;
    p.wall_u[1] = 0.05;
    p.eq_rho = 1.0;

    if (lbm_step(NULL, 1) != LBM_EINVAL) return 2;
    p.tau = 0.5;
    lbm_handle* bad = NULL;
    if (lbm_create(&p, 1, NULL, NULL, NULL, NULL, &bad) != LBM_EINVAL || bad != NULL) return 2;
    p.tau = 0.6;

    uint8_t* flags = calloc(N, 1);
    double* rho = malloc(N * sizeof(double));
    double* u = malloc(3 * N * sizeof(double));
    if (!flags || !rho || !u) return 1;
    size_t fluid = 0;
    for (int z = 0; z < n; z++)
        for (int y = 0; y < n; y++)
            for (int x = 0; x < n; x++) {
                const size_t c = (size_t)x + (size_t)n * ((size_t)y + (size_t)n * z);
                const int wall = x == 0 || y == 0 || z == 0 || x == n - 1 || y == n - 1 || z == n - 1;
                flags[c] = wall ? (uint8_t)(LBM_FLAG_SOLID | (z == n - 1 ? LBM_FLAG_MOVING : 0u)) : 0u;
                fluid += !wall;
            }

    lbm_handle* h = NULL;
    CHECK(lbm_create(&p, 1, NULL, NULL, NULL, NULL, &h));
    CHECK(lbm_set_boundaries(h, 0, flags));
    CHECK(lbm_step(h, steps));
    lbm_diag d;
    CHECK(lbm_diagnostics(h, 0, NULL, &d));
    CHECK(lbm_get_rho_u(h, 0, rho, u));
    /* one more step that also reduces the state it reads: the same sums */
    lbm_diag d2;
    CHECK(lbm_step_diagnostics(h, NULL, &d2));
    const int fused_same = d2.mass == d.mass && d2.kinetic_energy == d.kinetic_energy && d2.u_max == d.u_max &&
                           d2.momentum[0] == d.momentum[0] && d2.momentum[1] == d.momentum[1] &&
                           d2.momentum[2] == d.momentum[2] && d2.force_on_solid[1] == d.force_on_solid[1] &&
                           d2.step == d.step;
    lbm_info info;
    CHECK(lbm_info_get(h, &info));
    if (lbm_set_boundaries(h, 1, flags) != LBM_EINVAL) return 2;      /* one lattice only */
    lbm_destroy(h);

    /* host sums over the fluid cells, to compare with the device's FP64 sums */
    double mass = 0.0, py = 0.0;
    for (size_t c = 0; c < N; c++)
        if (!flags[c]) {
            mass += rho[c];
            py += rho[c] * u[N + c];
        }
    printf("c_caller fluid=%zu steps=%lld mass=%.12e host_mass=%.12e momentum_y=%.12e host_momentum_y=%.12e "
           "u_max=%.6e nonfinite=%lld device_bytes=%lld fused_same=%d steps_after=%lld\n",
           fluid, (long long)d.step, d.mass, mass, d.momentum[1], py, d.u_max, (long long)d.nonfinite_cells,
           (long long)info.device_bytes, fused_same, (long long)info.step);
    free(flags);
    free(rho);
    free(u);
    return 0;
}
