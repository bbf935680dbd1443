// Device body of one point of one colour sweep, shared by the one-instance
// sweep kernel and the batched sweep kernel (layout of kgs_internal.h).
#pragma once

#include <hip/hip_runtime.h>

#include "kgs_internal.h"
#include "kgs_layout.h"
#include "kgs_point.h"

namespace kgs {
namespace sweep_detail {

template <typename T>
__device__ __forceinline__ double ld(const T *p)
{
    return static_cast<double>(ld_global(p));
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

// Other-colour point indices of the 2*DIM neighbours of (row, xh) in the
// fixed axis order (axis 0 -, axis 0 +, ..., x -, x +), given the x
// neighbours xm, xp.
template <int DIM>
__device__ __forceinline__ void nb_index(const RowInfo<DIM> &r, int64_t row, int xh, int xm,
                                         int xp, int H, int64_t *j)
{
    if (DIM == 1) {
        j[0] = xm;
        j[1] = xp;
    } else {
        j[0] = r.nb[0] * H + xh;
        j[1] = r.nb[1] * H + xh;
        if (DIM == 3) {
            j[2] = r.nb[2] * H + xh;
            j[3] = r.nb[3] * H + xh;
        }
        j[2 * DIM - 2] = row * H + xm;
        j[2 * DIM - 1] = row * H + xp;
    }
}

// Neighbour sums of P, Q (one pair load per neighbour) and U (U alone) of
// the other colour, each added in the fixed axis order.
template <int DIM, typename T>
__device__ __forceinline__ void nb_sums(const T *__restrict__ pq, const T *__restrict__ uv,
                                        const int64_t *j, double &sr, double &si, double &su)
{
    Pair<T> a = ld_pair(pq, j[0]);
    sr = static_cast<double>(a.x);
    si = static_cast<double>(a.y);
    su = ld(uv + 2 * j[0]);
#pragma unroll
    for (int m = 1; m < 2 * DIM; ++m) {
        a = ld_pair(pq, j[m]);
        sr = sr + static_cast<double>(a.x);
        si = si + static_cast<double>(a.y);
        su = su + ld(uv + 2 * j[m]);
    }
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

    int64_t j[2 * DIM];
    nb_index<DIM>(r, row, xh, xm, xp, H, j);
    double sr, si, su;
    nb_sums<DIM>(pair_plane(base, stride, colour ^ 1, PAIR_PQ),
                 pair_plane(base, stride, colour ^ 1, PAIR_UV), j, sr, si, su);
    T *own_pq = pair_plane(base, stride, colour, PAIR_PQ);
    T *own_uv = pair_plane(base, stride, colour, PAIR_UV);
    const Pair<T> pq = ld_pair(own_pq, t), uv = ld_pair(own_uv, t);
    double pr = pq.x, pi = pq.y, u = uv.x, v = uv.y;
    sweep_point<KIND, T>(k, pr, pi, u, v, sr, si, su);
    st_pair(own_pq, t, static_cast<T>(pr), static_cast<T>(pi));
    st_pair(own_uv, t, static_cast<T>(u), static_cast<T>(v));
}


}  // namespace sweep_detail
}  // namespace kgs
