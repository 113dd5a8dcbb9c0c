/* A plain C99 user of the library's C ABI (test infrastructure): a D2Q37
 * lattice with both populations, the decay initial state of the
 * small-grid workload, 20 steps, then moments and FP64 totals.  Prints one
 * line per result with full precision; exits non-zero on any error.
 *
 *   c_abi_example <nx> <ny> <storage code>
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "esbgk.h"

#define CHECK(call)                                                                  \
    do {                                                                             \
        int rc_ = (call);                                                            \
        if (rc_ != ESBGK_OK) {                                                       \
            fprintf(stderr, "%s failed (%d): %s\n", #call, rc_, esbgk_last_error()); \
            return 1;                                                                \
        }                                                                            \
    } while (0)

int main(int argc, char **argv) {
    if (argc != 4) {
        fprintf(stderr, "usage: %s nx ny storage\n", argv[0]);
        return 2;
    }
    const int64_t nx = atoll(argv[1]), ny = atoll(argv[2]);
    const int storage = atoi(argv[3]);
    const int64_t dims[2] = {nx, ny};
    const size_t n = (size_t)(nx * ny);
    const double pi = 3.14159265358979323846;
    double *rho = malloc(n * sizeof *rho), *u = malloc(2 * n * sizeof *u), *T = malloc(n * sizeof *T);
    double *orho = malloc(n * sizeof *orho), *ou = malloc(2 * n * sizeof *ou), *oT = malloc(n * sizeof *oT);
    if (!rho || !u || !T || !orho || !ou || !oT) return 1;
    for (int64_t y = 0; y < ny; y++)
        for (int64_t x = 0; x < nx; x++) {
            const size_t k = (size_t)(y * nx + x);
            rho[k] = 1.0;
            u[k] = 1e-3 * sin(2 * pi * (double)y / (double)ny);
            u[n + k] = 0.0;
            T[k] = 1.0 + 1e-3 * cos(2 * pi * (double)x / (double)nx);
        }
    esbgk_t *h = NULL;
    CHECK(esbgk_create(2, 37, 3, 0.71, 0.8, dims, storage, &h));
    CHECK(esbgk_init_fields(h, rho, u, T));
    CHECK(esbgk_step(h, 20));
    int64_t steps = 0;
    CHECK(esbgk_step_count(h, &steps));
    CHECK(esbgk_read_moments(h, orho, ou, oT, NULL));
    double tot[4];
    CHECK(esbgk_totals(h, tot));
    double s_rho = 0, s_ux = 0, s_T = 0;
    for (size_t k = 0; k < n; k++) {
        s_rho += orho[k];
        s_ux += ou[k] * sin(2 * pi * (double)(k / (size_t)nx) / (double)ny);
        s_T += (oT[k] - 1.0) * cos(2 * pi * (double)(k % (size_t)nx) / (double)nx);
    }
    printf("steps %lld\n", (long long)steps);
    printf("moments %.17g %.17g %.17g\n", s_rho, s_ux, s_T);
    printf("cell0 %.17g %.17g %.17g %.17g\n", orho[0], ou[0], ou[n], oT[0]);
    printf("totals %.17g %.17g %.17g %.17g\n", tot[0], tot[1], tot[2], tot[3]);
    esbgk_destroy(h);
    free(rho); free(u); free(T); free(orho); free(ou); free(oT);
    return 0;
}
