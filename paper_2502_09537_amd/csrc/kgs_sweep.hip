// Colour-sweep kernels (one thread per point of the swept colour) and the
// layout kernels between the natural C-order arrays and the colour-split
// planes.  The layout is described in kgs_internal.h.
#include <hip/hip_runtime.h>

#include "kgs_internal.h"
#include "kgs_point.h"

namespace kgs {
namespace {

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

template <int DIM, typename T, int KIND>
__global__ void __launch_bounds__(1024)
sweep_kernel(T *__restrict__ base, int64_t stride, int n, int colour, Coef k, int64_t count)
{
    // (Giving each XCD a contiguous eighth of the rows measured 3% slower
    // than the hardware's round-robin order on 256^3, so blocks stay in order.)
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= count) return;
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
    sweep_point<KIND>(k, pr, pi, u, v, sr, si, su);
    own[F_P * stride + t] = static_cast<T>(pr);
    own[F_Q * stride + t] = static_cast<T>(pi);
    own[F_U * stride + t] = static_cast<T>(u);
    own[F_V * stride + t] = static_cast<T>(v);
}

// natural C-order point idx -> (colour, compressed index)
template <int DIM>
__device__ __forceinline__ void split_index(int64_t idx, int n, int &colour, int64_t &ci)
{
    const int64_t row = idx / n;
    const int x = static_cast<int>(idx - row * n);
    int s = 0;
    if (DIM == 2) s = static_cast<int>(row);
    if (DIM == 3) s = static_cast<int>(row / n) + static_cast<int>(row % n);
    colour = ((s + x + DIM) & 1) ? RED : BLUE;
    ci = row * (n >> 1) + (x >> 1);
}

template <int DIM, typename T>
__global__ void __launch_bounds__(256)
scatter_kernel(T *__restrict__ base, int64_t stride, int n, int64_t total,
               const double *__restrict__ P, const double *__restrict__ Q,
               const double *__restrict__ U, const double *__restrict__ V)
{
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    int c;
    int64_t ci;
    split_index<DIM>(idx, n, c, ci);
    T *p = base + static_cast<int64_t>(4 * c) * stride + ci;
    p[F_P * stride] = static_cast<T>(P[idx]);
    p[F_Q * stride] = static_cast<T>(Q[idx]);
    p[F_U * stride] = static_cast<T>(U[idx]);
    p[F_V * stride] = static_cast<T>(V[idx]);
}

template <int DIM, typename T>
__global__ void __launch_bounds__(256)
gather_kernel(const T *__restrict__ base, int64_t stride, int n, int64_t total,
              double *__restrict__ P, double *__restrict__ Q, double *__restrict__ U,
              double *__restrict__ V)
{
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    int c;
    int64_t ci;
    split_index<DIM>(idx, n, c, ci);
    const T *p = base + static_cast<int64_t>(4 * c) * stride + ci;
    P[idx] = static_cast<double>(p[F_P * stride]);
    Q[idx] = static_cast<double>(p[F_Q * stride]);
    U[idx] = static_cast<double>(p[F_U * stride]);
    V[idx] = static_cast<double>(p[F_V * stride]);
}

bool geometry_ok(const Geometry &g)
{
    if (g.dim < 1 || g.dim > 3 || g.n < 2 || (g.n & 1) || g.half != g.n / 2) return false;
    int64_t rows = 1;
    for (int a = 1; a < g.dim; ++a) rows *= g.n;
    return rows == g.rows && g.count == rows * g.half && g.stride >= g.count;
}

template <typename T, int KIND>
hipError_t sweep_dim(const Geometry &g, T *base, int colour, const Coef &k, int block,
                     hipStream_t s)
{
    const int64_t blocks = (g.count + block - 1) / block;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(blocks)), threads(block);
    switch (g.dim) {
    case 1:
        hipLaunchKernelGGL((sweep_kernel<1, T, KIND>), grid, threads, 0, s, base, g.stride, g.n,
                           colour, k, g.count);
        break;
    case 2:
        hipLaunchKernelGGL((sweep_kernel<2, T, KIND>), grid, threads, 0, s, base, g.stride, g.n,
                           colour, k, g.count);
        break;
    default:
        hipLaunchKernelGGL((sweep_kernel<3, T, KIND>), grid, threads, 0, s, base, g.stride, g.n,
                           colour, k, g.count);
        break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t sweep_typed(const Geometry &g, T *base, int kind, const Coef &k, int block,
                       hipStream_t s)
{
    switch (kind) {
    case PASS_R_BASE: return sweep_dim<T, PASS_R_BASE>(g, base, RED, k, block, s);
    case PASS_B_FULL: return sweep_dim<T, PASS_B_FULL>(g, base, BLUE, k, block, s);
    case PASS_R_ADJ: return sweep_dim<T, PASS_R_ADJ>(g, base, RED, k, block, s);
    case PASS_R_ADJ_BASE: return sweep_dim<T, PASS_R_ADJ_BASE>(g, base, RED, k, block, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t layout_typed(const Geometry &g, T *base, bool scatter, const double *P, const double *Q,
                        const double *U, const double *V, double *oP, double *oQ, double *oU,
                        double *oV, hipStream_t s)
{
    const int64_t total = 2 * g.count;
    const int64_t blocks = (total + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(blocks)), threads(256);
#define KGS_LAYOUT(D)                                                                           \
    if (scatter)                                                                                \
        hipLaunchKernelGGL((scatter_kernel<D, T>), grid, threads, 0, s, base, g.stride, g.n,    \
                           total, P, Q, U, V);                                                  \
    else                                                                                        \
        hipLaunchKernelGGL((gather_kernel<D, T>), grid, threads, 0, s, base, g.stride, g.n,     \
                           total, oP, oQ, oU, oV);
    switch (g.dim) {
    case 1: KGS_LAYOUT(1) break;
    case 2: KGS_LAYOUT(2) break;
    default: KGS_LAYOUT(3) break;
    }
#undef KGS_LAYOUT
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep(const Geometry &g, int precision, void *state, int kind, const Coef &k,
                        int block, hipStream_t s)
{
    if (!geometry_ok(g) || !state || block < 64 || block > 1024 || (block % 64)) {
        return hipErrorInvalidValue;
    }
    if (precision == 0) return sweep_typed(g, static_cast<double *>(state), kind, k, block, s);
    return sweep_typed(g, static_cast<float *>(state), kind, k, block, s);
}

hipError_t launch_scatter(const Geometry &g, int precision, void *state, const double *P,
                          const double *Q, const double *U, const double *V, hipStream_t s)
{
    if (!geometry_ok(g) || !state || !P || !Q || !U || !V) return hipErrorInvalidValue;
    if (precision == 0)
        return layout_typed(g, static_cast<double *>(state), true, P, Q, U, V, nullptr, nullptr,
                            nullptr, nullptr, s);
    return layout_typed(g, static_cast<float *>(state), true, P, Q, U, V, nullptr, nullptr,
                        nullptr, nullptr, s);
}

hipError_t launch_gather(const Geometry &g, int precision, const void *state, double *P,
                         double *Q, double *U, double *V, hipStream_t s)
{
    if (!geometry_ok(g) || !state || !P || !Q || !U || !V) return hipErrorInvalidValue;
    if (precision == 0)
        return layout_typed(g, const_cast<double *>(static_cast<const double *>(state)), false,
                            nullptr, nullptr, nullptr, nullptr, P, Q, U, V, s);
    return layout_typed(g, const_cast<float *>(static_cast<const float *>(state)), false, nullptr,
                        nullptr, nullptr, nullptr, P, Q, U, V, s);
}

}  // namespace kgs
