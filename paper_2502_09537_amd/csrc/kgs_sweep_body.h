// Device body of one point of one colour sweep, shared by the one-instance
// sweep kernel and the batched sweep kernel (layout of kgs_internal.h).
#pragma once

#include <hip/hip_runtime.h>

#include "kgs_internal.h"
#include "kgs_point.h"

namespace kgs {
namespace sweep_detail {

template <typename T>
__device__ __forceinline__ double ld(const T *p)
{
    return static_cast<double>(*p);
}

// Index sum of the non-x coordinates of a row, and the rows one step away
// along each non-x axis (periodic), in axis order.
template <int DIM>
struct RowInfo {
    int s;
    int64_t nb[2 * (DIM - 1) > 0 ? 2 * (DIM - 1) : 1];
};

template <int DIM>
__device__ __forceinline__ RowInfo<DIM> row_info(int64_t row, int n)
{
    RowInfo<DIM> r;
    if (DIM == 1) {
        r.s = 0;
        r.nb[0] = 0;
    } else if (DIM == 2) {
        const int i0 = static_cast<int>(row);
        r.s = i0;
        r.nb[0] = i0 == 0 ? n - 1 : i0 - 1;
        r.nb[1] = i0 == n - 1 ? 0 : i0 + 1;
    } else {
        const int i0 = static_cast<int>(row / n);
        const int i1 = static_cast<int>(row - static_cast<int64_t>(i0) * n);
        r.s = i0 + i1;
        const int64_t i0m = i0 == 0 ? n - 1 : i0 - 1, i0p = i0 == n - 1 ? 0 : i0 + 1;
        const int64_t i1m = i1 == 0 ? n - 1 : i1 - 1, i1p = i1 == n - 1 ? 0 : i1 + 1;
        r.nb[0] = i0m * n + i1;
        r.nb[1] = i0p * n + i1;
        r.nb[2] = static_cast<int64_t>(i0) * n + i1m;
        r.nb[3] = static_cast<int64_t>(i0) * n + i1p;
    }
    return r;
}

// Neighbour sum of one other-colour plane f at point (row, xh) whose own
// x-offset is o, in the fixed axis order (axis 0 -, axis 0 +, ..., x -, x +).
template <int DIM, typename T>
__device__ __forceinline__ double nb_sum(const T *__restrict__ f, const RowInfo<DIM> &r,
                                         int64_t row, int xh, int xm, int xp, int H)
{
    double acc;
    if (DIM == 1) {
        acc = ld(f + xm);
        acc = acc + ld(f + xp);
    } else {
        acc = ld(f + r.nb[0] * H + xh);
        acc = acc + ld(f + r.nb[1] * H + xh);
        if (DIM == 3) {
            acc = acc + ld(f + r.nb[2] * H + xh);
            acc = acc + ld(f + r.nb[3] * H + xh);
        }
        acc = acc + ld(f + row * H + xm);
        acc = acc + ld(f + row * H + xp);
    }
    return acc;
}

// One point of one colour sweep: point t of colour `colour` in the plane set
// at `base` (layout of kgs_internal.h).
template <int DIM, typename T, int KIND>
__device__ __forceinline__ void sweep_one(T *__restrict__ base, int64_t stride, int n, int colour,
                                          const Coef &k, int64_t t)
{
    const int H = n >> 1;
    const int64_t row = t / H;
    const int xh = static_cast<int>(t - row * H);
    const RowInfo<DIM> r = row_info<DIM>(row, n);
    const int o = (r.s + DIM + 1 + colour) & 1;
    int xm = xh - 1 + o;
    if (xm < 0) xm += H;
    int xp = xh + o;
    if (xp >= H) xp -= H;

    T *own = base + static_cast<int64_t>(4 * colour) * stride;
    const T *oth = base + static_cast<int64_t>(4 * (colour ^ 1)) * stride;
    const double sr = nb_sum<DIM>(oth + F_P * stride, r, row, xh, xm, xp, H);
    const double si = nb_sum<DIM>(oth + F_Q * stride, r, row, xh, xm, xp, H);
    const double su = nb_sum<DIM>(oth + F_U * stride, r, row, xh, xm, xp, H);
    double pr = ld(own + F_P * stride + t);
    double pi = ld(own + F_Q * stride + t);
    double u = ld(own + F_U * stride + t);
    double v = ld(own + F_V * stride + t);
    sweep_point<KIND, T>(k, pr, pi, u, v, sr, si, su);
    own[F_P * stride + t] = static_cast<T>(pr);
    own[F_Q * stride + t] = static_cast<T>(pi);
    own[F_U * stride + t] = static_cast<T>(u);
    own[F_V * stride + t] = static_cast<T>(v);
}


}  // namespace sweep_detail
}  // namespace kgs
