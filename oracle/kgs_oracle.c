/*
 * kgs_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, double-precision CPU reference of the DP-AVF2 scheme for
 * the periodic Klein-Gordon-Schroedinger (KGS) equations, written from the paper
 * "dual-partition AVF methods for the KGS equations" (arXiv 2502.09537).  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg load
 * this file.  The GPU library never does, and the two share no code, header,
 * table or helper.
 *
 * What it computes
 * ----------------
 * The real state is P = Re psi, Q = Im psi, U = u and V = u_t on a periodic
 * grid of n^dim points with one spacing h on every axis (sec. 2, real
 * first-order form of the KGS system and the grid Omega_h).  Arrays are in
 * natural C order: point (i0, ..., i_{dim-1}) has linear index
 * ((i0*n)+i1)*n+i2, axis 0 slowest.
 *
 * One DP-AVF2 step of size tau is the symmetric composition of the DP-AVF
 * method with its adjoint, each with tau/2 (sec. 3.1, eq. dp-comp).  Given a
 * grid-point update order, the DP-AVF half step visits the points in that
 * order and at each point solves the first equation of the explicit pointwise
 * scheme for Psi, then the last two equations for (U, V) (sec. 4.1, eq.
 * scheme1, and Algorithm 1).  The adjoint half step visits the points in the
 * reverse order and solves (U, V) first, then Psi (eq. scheme1-adj).  The
 * state is overwritten in place, so a neighbour that comes earlier in the
 * order already holds its new value (the S, W, E, N rule of sec. 3.2).
 *
 * The GPU order is the checkerboard order (sec. 4.2): a point is red when the
 * sum of its 1-based indices is odd (Algorithm 3), red points come first in
 * the DP-AVF half step, and blue points first in the adjoint half step.
 *
 * Readings where the paper is ambiguous (each is pinned by a test):
 *  - scheme1-adj prints U^n on the right-hand side of the Psi equation; the
 *    pointwise adjoint scheme (eq. dp-avf-kj-adj) has U^{n+1} on both sides.
 *    This oracle uses the value U currently holds at the point on both sides.
 *  - the adjoint half step solves (U, V) before Psi at every point (sec. 4.1,
 *    Algorithm 1), also for the blue pass that Algorithm 3 labels otherwise.
 *  - in d dimensions the Laplacian has 2d neighbours, so the "4" of the 2-D
 *    scheme becomes 2d: the Psi coefficient is d*tau*kappa1/(2h^2) and the
 *    (U, V) coefficient is d*tau*kappa2/h^2 + tau*mu^2/2.
 *  - the energy is h^dim times the discrete energy E_h of sec. 2, written
 *    with forward differences (summation by parts turns -p^T D p into the sum
 *    of squared forward differences).
 *
 * Built with -ffp-contract=off: every product and sum is rounded as written;
 * the two explicit fma() calls in the (U, V) solve are the only fused
 * operations.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int32_t dim;     /* 1, 2 or 3 */
    int32_t n;       /* points per axis */
    double h;        /* grid spacing, the same on every axis */
    double kappa1, kappa2, mu, gamma;
} kgso_grid;

enum { KGSO_OK = 0, KGSO_EINVAL = -1, KGSO_ENOMEM = -2 };

static int grid_ok(const kgso_grid *g)
{
    return g && g->dim >= 1 && g->dim <= 3 && g->n >= 2 && isfinite(g->h) && g->h > 0.0;
}

static int64_t npoints(const kgso_grid *g)
{
    int64_t m = 1;
    for (int a = 0; a < g->dim; ++a) m *= g->n;
    return m;
}

/* Linear index of the neighbour of point idx one cell away along axis
 * (dir = -1 or +1), with periodic wrap. */
static int64_t neighbour(const kgso_grid *g, int64_t idx, int axis, int dir)
{
    int64_t stride = 1;
    for (int a = g->dim - 1; a > axis; --a) stride *= g->n;
    int64_t c = (idx / stride) % g->n;
    int64_t c2 = (c + dir + g->n) % g->n;
    return idx + (c2 - c) * stride;
}

/* Sum of the 2*dim nearest neighbours of idx in the fixed order
 * axis 0 minus, axis 0 plus, axis 1 minus, axis 1 plus, ... */
static double neighbour_sum(const kgso_grid *g, const double *f, int64_t idx)
{
    double s = 0.0;
    for (int a = 0; a < g->dim; ++a) {
        s = s + f[neighbour(g, idx, a, -1)];
        s = s + f[neighbour(g, idx, a, +1)];
    }
    return s;
}

/* Red/blue colour of the checkerboard (sec. 4.2, Algorithm 3): red when the
 * sum of the 1-based indices is odd. */
int32_t kgso_is_red(int32_t dim, int32_t n, int64_t idx)
{
    int64_t s = 0;
    for (int a = 0; a < dim; ++a) {
        s += idx % n + 1;
        idx /= n;
    }
    return (int32_t)(s % 2);
}

/* First equation of the explicit pointwise scheme, solved for the new Psi at
 * point idx with time step tau (sec. 4.1, eq. scheme1; the adjoint eq.
 * scheme1-adj has the same form, see the reading on U above):
 *
 *   (i - d tau k1/(2h^2) + tau g/2 U_i) Psi_i^new
 *       = (i + d tau k1/(2h^2) - tau g/2 U_i) Psi_i - tau k1/(2h^2) sum_nb Psi_nb
 *
 * U_i and the neighbours take the values currently stored. */
void kgso_psi_update(const kgso_grid *g, double tau, double *P, double *Q, const double *U,
                     int64_t idx)
{
    const double r = tau * g->kappa1 / (2.0 * g->h * g->h);
    const double lap = (double)g->dim * r;
    const double w = tau * g->gamma / 2.0 * U[idx];
    const double complex S = neighbour_sum(g, P, idx) + I * neighbour_sum(g, Q, idx);
    const double complex psi = P[idx] + I * Q[idx];
    const double complex lhs = I - lap + w;
    const double complex rhs = (I + lap - w) * psi - r * S;
    const double complex psi_new = rhs / lhs;
    P[idx] = creal(psi_new);
    Q[idx] = cimag(psi_new);
}

/* Inverse of the constant 2x2 matrix of the (U, V) equations, which
 * Algorithm 1 computes once before the time loop:
 *   [[1, -tau/2], [beta, 1]]^{-1} = (1/det) [[1, tau/2], [-beta, 1]],
 * beta = d tau k2/h^2 + tau mu^2/2, det = 1 + beta tau/2.
 *
 * 1/det is kept as an unevaluated sum of two doubles (computed in binary128).
 * Every (U, V) solve reuses this one constant, so a single rounding of it
 * scales every solve by the same factor (1 + delta); the energy then changes
 * by about 2 delta w^2 per solve (w the midpoint velocity), always with the
 * same sign, and drifts linearly in time (about 2e-12 over 1e4 steps of the
 * 1-D soliton problem).  With 1/det exact to ~1e-32 the remaining roundings
 * depend on the data and only random-walk. */
typedef struct {
    double beta, half_tau, recip_hi, recip_lo;
} uv_inverse;

static uv_inverse uv_matrix_inverse(const kgso_grid *g, double tau)
{
    uv_inverse m;
    m.beta = (double)g->dim * tau * g->kappa2 / (g->h * g->h) + tau * g->mu * g->mu / 2.0;
    m.half_tau = tau / 2.0;
    const __float128 det = (__float128)1.0 + (__float128)m.beta * (__float128)m.half_tau;
    const __float128 inv = (__float128)1.0 / det;
    m.recip_hi = (double)inv;
    m.recip_lo = (double)(inv - (__float128)m.recip_hi);
    return m;
}

/* Last two equations of the explicit pointwise scheme, solved for the new
 * (U_i, V_i) with time step tau (sec. 4.1, eq. scheme1 and scheme1-adj):
 *
 *   U_i^new - tau/2 V_i^new = U_i + tau/2 V_i                                  (= r1)
 *   beta U_i^new + V_i^new  = V_i - beta U_i + tau k2/h^2 sum_nb U_nb + tau g |Psi_i|^2   (= r2)
 *
 * |Psi_i|^2 is the value currently stored: Psi^{n+1} in the base scheme,
 * Psi^n in the adjoint one. */
static void uv_update(const kgso_grid *g, double tau, const uv_inverse *m, const double *P,
                      const double *Q, double *U, double *V, int64_t idx)
{
    const double su = neighbour_sum(g, U, idx);
    const double r1 = U[idx] + m->half_tau * V[idx];
    const double r2 = V[idx] - m->beta * U[idx] + tau * g->kappa2 / (g->h * g->h) * su +
                      tau * g->gamma * (P[idx] * P[idx] + Q[idx] * Q[idx]);
    const double xu = r1 + m->half_tau * r2; /* det * U_new */
    const double xv = r2 - m->beta * r1;     /* det * V_new */
    /* one rounding of xu*(recip_hi + recip_lo): a separately rounded
     * xu*recip_hi would swallow the low word and bring the bias back */
    U[idx] = fma(xu, m->recip_hi, xu * m->recip_lo);
    V[idx] = fma(xv, m->recip_hi, xv * m->recip_lo);
}

void kgso_uv_update(const kgso_grid *g, double tau, const double *P, const double *Q, double *U,
                    double *V, int64_t idx)
{
    const uv_inverse m = uv_matrix_inverse(g, tau);
    uv_update(g, tau, &m, P, Q, U, V, idx);
}

/* DP-AVF half step (eq. dp-avf-kj): points in the given order, Psi then (U, V). */
void kgso_base_half(const kgso_grid *g, double tau, double *P, double *Q, double *U, double *V,
                    const int64_t *order, int64_t m)
{
    const uv_inverse inv = uv_matrix_inverse(g, tau);
    for (int64_t t = 0; t < m; ++t) {
        const int64_t idx = order[t];
        kgso_psi_update(g, tau, P, Q, U, idx);
        uv_update(g, tau, &inv, P, Q, U, V, idx);
    }
}

/* Adjoint half step (eq. dp-avf-kj-adj): points in the reverse order,
 * (U, V) then Psi. */
void kgso_adjoint_half(const kgso_grid *g, double tau, double *P, double *Q, double *U, double *V,
                       const int64_t *order, int64_t m)
{
    const uv_inverse inv = uv_matrix_inverse(g, tau);
    for (int64_t t = m - 1; t >= 0; --t) {
        const int64_t idx = order[t];
        uv_update(g, tau, &inv, P, Q, U, V, idx);
        kgso_psi_update(g, tau, P, Q, U, idx);
    }
}

/* nsteps DP-AVF2 steps of size tau for an arbitrary update order (a
 * permutation of all n^dim points): the DP-AVF half step with tau/2, then its
 * adjoint with tau/2 (eq. dp-comp). */
int kgso_step_order(const kgso_grid *g, double tau, double *P, double *Q, double *U, double *V,
                    const int64_t *order, int64_t nsteps)
{
    if (!grid_ok(g) || !order || nsteps < 0) return KGSO_EINVAL;
    const int64_t m = npoints(g);
    for (int64_t s = 0; s < nsteps; ++s) {
        kgso_base_half(g, tau / 2.0, P, Q, U, V, order, m);
        kgso_adjoint_half(g, tau / 2.0, P, Q, U, V, order, m);
    }
    return KGSO_OK;
}

/* The checkerboard update order: all red points in lexicographic order,
 * then all blue points in lexicographic order. */
int64_t kgso_checkerboard_order(int32_t dim, int32_t n, int64_t *order)
{
    int64_t m = 1;
    for (int a = 0; a < dim; ++a) m *= n;
    int64_t t = 0;
    for (int colour = 1; colour >= 0; --colour)
        for (int64_t idx = 0; idx < m; ++idx)
            if (kgso_is_red(dim, n, idx) == colour) order[t++] = idx;
    return t;
}

/* nsteps DP-AVF2 steps in the checkerboard order. */
int kgso_step(const kgso_grid *g, double tau, double *P, double *Q, double *U, double *V,
              int64_t nsteps)
{
    if (!grid_ok(g) || nsteps < 0) return KGSO_EINVAL;
    const int64_t m = npoints(g);
    int64_t *order = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    if (!order) return KGSO_ENOMEM;
    kgso_checkerboard_order(g->dim, g->n, order);
    const int rc = kgso_step_order(g, tau, P, Q, U, V, order, nsteps);
    free(order);
    return rc;
}

/* h^dim times the discrete energy of sec. 2:
 *   sum_i [ 1/2 ( k1 sum_axes ((P_{i+e}-P_i)^2 + (Q_{i+e}-Q_i)^2)/h^2
 *               + k2 sum_axes (U_{i+e}-U_i)^2/h^2 + V_i^2 + mu^2 U_i^2 )
 *           - g (P_i^2 + Q_i^2) U_i ]
 * summed over the points in natural order with Neumaier's compensated sum. */
double kgso_energy(const kgso_grid *g, const double *P, const double *Q, const double *U,
                   const double *V)
{
    if (!grid_ok(g)) return NAN;
    const int64_t m = npoints(g);
    const double h2 = g->h * g->h;
    double sum = 0.0, comp = 0.0;
    for (int64_t idx = 0; idx < m; ++idx) {
        double gp = 0.0, gq = 0.0, gu = 0.0;
        for (int a = 0; a < g->dim; ++a) {
            const int64_t j = neighbour(g, idx, a, +1);
            const double dp = P[j] - P[idx], dq = Q[j] - Q[idx], du = U[j] - U[idx];
            gp = gp + dp * dp;
            gq = gq + dq * dq;
            gu = gu + du * du;
        }
        const double term =
            0.5 * (g->kappa1 * (gp + gq) / h2 + g->kappa2 * gu / h2 + V[idx] * V[idx] +
                   g->mu * g->mu * (U[idx] * U[idx])) -
            g->gamma * (P[idx] * P[idx] + Q[idx] * Q[idx]) * U[idx];
        const double t = sum + term;
        if (fabs(sum) >= fabs(term))
            comp += (sum - t) + term;
        else
            comp += (term - t) + sum;
        sum = t;
    }
    double hd = 1.0;
    for (int a = 0; a < g->dim; ++a) hd *= g->h;
    return hd * (sum + comp);
}

/* ------------------------------------------------------------------------
 * The checkerboard step written colour pass by colour pass (sec. 4.2,
 * Algorithm 3, with the adjoint passes read as (U, V) then Psi):
 *   red   points: Psi, then (U, V)      DP-AVF half step with tau/2
 *   blue  points: Psi, then (U, V)
 *   blue  points: (U, V), then Psi      adjoint half step with tau/2
 *   red   points: (U, V), then Psi
 * Points of one colour have no neighbour of that colour, so the points of a
 * pass may be visited in any order and the result is bitwise that of
 * kgso_step.  Two options, neither of which changes an operation:
 *
 *  - nthreads > 1 splits every pass over that many OpenMP threads (the
 *    all-cores timing of the oracle); the result is bitwise that of one
 *    thread.
 *  - storage_bits = 32 describes a state stored in float32 between passes:
 *    the values are rounded to float32 (round to nearest even) on entry,
 *    at the end of every red pass for the red points, and at the end of the
 *    blue adjoint pass for the blue points, which are exactly the places
 *    where a float32 state is written back to memory when each colour pass
 *    is one sweep over the grid and the two blue passes are one.  All
 *    arithmetic stays in float64.  storage_bits = 64 rounds nothing.
 * ---------------------------------------------------------------------- */
static void round_points_f32(double *P, double *Q, double *U, double *V, const int64_t *pts,
                             int64_t m, int nthreads)
{
#pragma omp parallel for schedule(static) num_threads(nthreads) if (nthreads > 1)
    for (int64_t t = 0; t < m; ++t) {
        const int64_t idx = pts[t];
        P[idx] = (double)(float)P[idx];
        Q[idx] = (double)(float)Q[idx];
        U[idx] = (double)(float)U[idx];
        V[idx] = (double)(float)V[idx];
    }
}

static void colour_pass(const kgso_grid *g, double tau_half, const uv_inverse *inv, double *P,
                        double *Q, double *U, double *V, const int64_t *pts, int64_t m,
                        int adjoint, int nthreads)
{
#pragma omp parallel for schedule(static) num_threads(nthreads) if (nthreads > 1)
    for (int64_t t = 0; t < m; ++t) {
        const int64_t idx = pts[t];
        if (adjoint) {
            uv_update(g, tau_half, inv, P, Q, U, V, idx);
            kgso_psi_update(g, tau_half, P, Q, U, idx);
        } else {
            kgso_psi_update(g, tau_half, P, Q, U, idx);
            uv_update(g, tau_half, inv, P, Q, U, V, idx);
        }
    }
}

int kgso_step_passes(const kgso_grid *g, double tau, double *P, double *Q, double *U, double *V,
                     int64_t nsteps, int32_t storage_bits, int32_t nthreads)
{
    /* odd n: two neighbours share a colour, the passes are not independent */
    if (!grid_ok(g) || (g->n & 1) || nsteps < 0 || (storage_bits != 32 && storage_bits != 64) ||
        nthreads < 1)
        return KGSO_EINVAL;
    const int64_t m = npoints(g);
    int64_t *order = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    if (!order) return KGSO_ENOMEM;
    kgso_checkerboard_order(g->dim, g->n, order);
    const int64_t nred = m / 2; /* n even: half of the points are red */
    const int64_t *red = order, *blue = order + nred;
    const int f32 = storage_bits == 32;
    const uv_inverse inv = uv_matrix_inverse(g, tau / 2.0);
    if (f32) round_points_f32(P, Q, U, V, order, m, nthreads);
    for (int64_t s = 0; s < nsteps; ++s) {
        colour_pass(g, tau / 2.0, &inv, P, Q, U, V, red, nred, 0, nthreads);
        if (f32) round_points_f32(P, Q, U, V, red, nred, nthreads);
        colour_pass(g, tau / 2.0, &inv, P, Q, U, V, blue, m - nred, 0, nthreads);
        colour_pass(g, tau / 2.0, &inv, P, Q, U, V, blue, m - nred, 1, nthreads);
        if (f32) round_points_f32(P, Q, U, V, blue, m - nred, nthreads);
        colour_pass(g, tau / 2.0, &inv, P, Q, U, V, red, nred, 1, nthreads);
        if (f32) round_points_f32(P, Q, U, V, red, nred, nthreads);
    }
    free(order);
    return KGSO_OK;
}
