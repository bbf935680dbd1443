/* Test infrastructure: exercises the C oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built and run by tests/test_sanitizers.py on
 * the CPU).  Small grids of every dimension, the generic-order and colour-
 * pass steps, the float32-storage option, the energy and the rejected
 * arguments; it prints "ok" and returns 0 when every check holds, and the
 * sanitizers abort the run at the first invalid access or undefined
 * operation. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t dim;
    int32_t n;
    double h;
    double kappa1, kappa2, mu, gamma;
} kgso_grid;

int kgso_step(const kgso_grid *g, double tau, double *P, double *Q, double *U, double *V,
              int64_t nsteps);
int kgso_step_order(const kgso_grid *g, double tau, double *P, double *Q, double *U, double *V,
                    const int64_t *order, int64_t nsteps);
int kgso_step_passes(const kgso_grid *g, double tau, double *P, double *Q, double *U, double *V,
                     int64_t nsteps, int32_t storage_bits, int32_t nthreads);
int64_t kgso_checkerboard_order(int32_t dim, int32_t n, int64_t *order);
double kgso_energy(const kgso_grid *g, const double *P, const double *Q, const double *U,
                   const double *V);

static int failures;

static void check(int ok, const char *what, int dim, int n)
{
    if (!ok) {
        printf("FAIL %s dim=%d n=%d\n", what, dim, n);
        ++failures;
    }
}

static double *fields(int64_t m, unsigned seed)
{
    double *a = (double *)malloc((size_t)(4 * m) * sizeof(double));
    srand(seed);
    for (int64_t i = 0; i < 4 * m; ++i) a[i] = (double)rand() / RAND_MAX - 0.5;
    return a;
}

int main(void)
{
    const int ns[] = {2, 4, 6, 8};
    for (int dim = 1; dim <= 3; ++dim) {
        for (size_t k = 0; k < sizeof(ns) / sizeof(ns[0]); ++k) {
            const int n = ns[k];
            int64_t m = 1;
            for (int a = 0; a < dim; ++a) m *= n;
            kgso_grid g = {dim, n, 8.0 / n, 0.9, 1.1, 0.8, 1.3};
            double *x = fields(m, 17u + (unsigned)(dim * 100 + n));
            double *y = (double *)malloc((size_t)(4 * m) * sizeof(double));
            double *z = (double *)malloc((size_t)(4 * m) * sizeof(double));
            memcpy(y, x, (size_t)(4 * m) * sizeof(double));
            memcpy(z, x, (size_t)(4 * m) * sizeof(double));
            const double e0 = kgso_energy(&g, x, x + m, x + 2 * m, x + 3 * m);
            check(kgso_step(&g, 0.01, y, y + m, y + 2 * m, y + 3 * m, 3) == 0, "step", dim, n);
            const double e1 = kgso_energy(&g, y, y + m, y + 2 * m, y + 3 * m);
            check(fabs(e1 - e0) <= 1e-12 * fabs(e0) + 1e-300, "energy conserved", dim, n);
            /* colour passes on 1 and 3 threads: bitwise the generic-order step */
            for (int t = 1; t <= 3; t += 2) {
                memcpy(z, x, (size_t)(4 * m) * sizeof(double));
                check(kgso_step_passes(&g, 0.01, z, z + m, z + 2 * m, z + 3 * m, 3, 64, t) == 0,
                      "step_passes", dim, n);
                check(memcmp(y, z, (size_t)(4 * m) * sizeof(double)) == 0, "passes == step", dim, n);
            }
            /* float32 storage runs and stays finite */
            memcpy(z, x, (size_t)(4 * m) * sizeof(double));
            check(kgso_step_passes(&g, 0.01, z, z + m, z + 2 * m, z + 3 * m, 2, 32, 2) == 0,
                  "step_passes fp32", dim, n);
            for (int64_t i = 0; i < 4 * m; ++i) check(isfinite(z[i]), "finite", dim, n);
            /* reversibility: -tau undoes +tau */
            check(kgso_step(&g, -0.01, y, y + m, y + 2 * m, y + 3 * m, 3) == 0, "step back", dim, n);
            double worst = 0.0;
            for (int64_t i = 0; i < 4 * m; ++i) worst = fmax(worst, fabs(y[i] - x[i]));
            check(worst <= 1e-13, "reversible", dim, n);
            /* a reversed lexicographic order through the generic-order step */
            int64_t *order = (int64_t *)malloc((size_t)m * sizeof(int64_t));
            for (int64_t i = 0; i < m; ++i) order[i] = m - 1 - i;
            check(kgso_step_order(&g, 0.02, y, y + m, y + 2 * m, y + 3 * m, order, 2) == 0,
                  "step_order", dim, n);
            check(kgso_checkerboard_order(dim, n, order) == m, "checkerboard order", dim, n);
            free(order);
            free(x);
            free(y);
            free(z);
        }
    }
    /* rejected arguments */
    kgso_grid odd = {2, 5, 1.0, 1.0, 1.0, 1.0, 1.0};
    double buf[4 * 25];
    memset(buf, 0, sizeof(buf));
    check(kgso_step_passes(&odd, 0.01, buf, buf + 25, buf + 50, buf + 75, 1, 64, 1) != 0,
          "odd n refused", 2, 5);
    kgso_grid ok = {2, 4, 1.0, 1.0, 1.0, 1.0, 1.0};
    check(kgso_step_passes(&ok, 0.01, buf, buf + 16, buf + 32, buf + 48, 1, 16, 1) != 0,
          "storage bits refused", 2, 4);
    check(kgso_step_passes(&ok, 0.01, buf, buf + 16, buf + 32, buf + 48, -1, 64, 1) != 0,
          "negative steps refused", 2, 4);
    check(kgso_step(NULL, 0.01, buf, buf, buf, buf, 1) != 0, "null grid refused", 0, 0);
    if (failures) return 1;
    printf("ok\n");
    return 0;
}
