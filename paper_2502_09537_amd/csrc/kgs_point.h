// Device-side point updates of the explicit DP-AVF scheme (sec. 4.1 of the
// paper, eq. scheme1 and scheme1-adj), shared by every sweep kernel.  The
// library is compiled with -ffp-contract=off and every fused multiply-add is
// written out, so all kernels round identically and agree bitwise.
#pragma once

#include <hip/hip_runtime.h>

#include "kgs_internal.h"

namespace kgs {

// Psi at one point, given the neighbour sum S = sr + i si of the 2*dim
// neighbours and the value u currently held at the point (u^n in the base
// scheme, u^{n+1} in the adjoint scheme, where (u,v) is solved first):
//   (i - c) psi' = (i + c) psi - b S,   c = a - e u,
// i.e. psi' = num (-c - i) / (1 + c^2) with num = (i + c) psi - b S.
// 1/x for x >= 1: the hardware reciprocal estimate refined by two
// Newton-Raphson steps r <- r + r (1 - x r) (each squares the relative
// error), which leaves the error of the last rounding, within one unit in
// the last place of the correctly rounded quotient.  x = 1 + c^2 >= 1 rules
// out the zeros, denormals and overflow that a general division must
// handle, so the five instructions replace a full IEEE division.
__device__ __forceinline__ double recip_ge1(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ void psi_update(const Coef &k, double &pr, double &pi, double u,
                                           double sr, double si)
{
    const double c = fma(-k.e, u, k.a);                // a - e u
    const double nr = fma(-k.b, sr, fma(c, pr, -pi));  // c pr - pi - b sr
    const double ni = fma(-k.b, si, fma(c, pi, pr));   // pr + c pi - b si
    const double inv = recip_ge1(fma(c, c, 1.0));
    pr = fma(-c, nr, ni) * inv;                        // (ni - c nr) / (1 + c^2)
    pi = -fma(c, ni, nr) * inv;                        // -(nr + c ni) / (1 + c^2)
}

// (u, v) at one point, given the neighbour sum su of u and the value |psi|^2
// currently held at the point: the 2x2 system
//   u' - t2 v' = u + t2 v = r1,   beta u' + v' = v - beta u + s su + g |psi|^2 = r2
// solved with its constant inverse (1/det) [[1, t2], [-beta, 1]].  1/det is
// the double-double rd_hi + rd_lo applied with one fused rounding, so the
// reused constant does not scale every solve by the same rounding error
// (which would make the energy drift in one direction).
__device__ __forceinline__ void uv_update(const Coef &k, double pr, double pi, double &u,
                                          double &v, double su)
{
    const double A = fma(pr, pr, pi * pi);
    const double r1 = fma(k.t2, v, u);
    const double r2 = fma(k.g, A, fma(k.s, su, fma(-k.beta, u, v)));
    const double xu = fma(k.t2, r2, r1);
    const double xv = fma(-k.beta, r1, r2);
    u = fma(xu, k.rd_hi, xu * k.rd_lo);
    v = fma(xv, k.rd_hi, xv * k.rd_lo);
}

// The point updates of one colour sweep (see PassKind), with the neighbour
// sums computed once: the other colour does not change within a sweep.  T is
// the storage type: the fused red sweep of two consecutive steps rounds the
// state to T between the steps exactly as storing it at a step boundary
// would, so a run gives bitwise the same state however its steps are split
// into calls (float32 state; a no-op for float64).
template <int KIND, typename T>
__device__ __forceinline__ void sweep_point(const Coef &k, double &pr, double &pi, double &u,
                                            double &v, double sr, double si, double su)
{
    if (KIND == PASS_R_BASE) {
        psi_update(k, pr, pi, u, sr, si);
        uv_update(k, pr, pi, u, v, su);
    } else if (KIND == PASS_B_FULL) {
        psi_update(k, pr, pi, u, sr, si);
        uv_update(k, pr, pi, u, v, su);
        uv_update(k, pr, pi, u, v, su);
        psi_update(k, pr, pi, u, sr, si);
    } else if (KIND == PASS_R_ADJ) {
        uv_update(k, pr, pi, u, v, su);
        psi_update(k, pr, pi, u, sr, si);
    } else {  // PASS_R_ADJ_BASE
        uv_update(k, pr, pi, u, v, su);
        psi_update(k, pr, pi, u, sr, si);
        pr = static_cast<double>(static_cast<T>(pr));
        pi = static_cast<double>(static_cast<T>(pi));
        u = static_cast<double>(static_cast<T>(u));
        v = static_cast<double>(static_cast<T>(v));
        psi_update(k, pr, pi, u, sr, si);
        uv_update(k, pr, pi, u, v, su);
    }
}

}  // namespace kgs
