// Discrete energy E_h of sec. 2 (without the h^dim factor, which the host
// applies): a deterministic, compensated float64 reduction.
//
// Each thread sums the energy density of its points into a double-double
// (TwoSum), a wavefront of 64 lanes combines its lanes with shuffles in a
// fixed tree, the waves of a workgroup combine through LDS in a fixed order,
// and one final workgroup combines the per-workgroup partials in a fixed
// order.  The grid size depends only on the problem size, so the result is
// bitwise reproducible run to run.
//
// 2-D and 3-D grids stream along axis 0: a thread owns one column (a row
// position along the other axes and a compressed x position, both colours)
// and walks it through a chunk of consecutive planes of axis 0.  The forward
// neighbour along axis 0 of a point is the other colour at the same column
// in the next plane, which the thread loads anyway as its next plane's own
// values, so the state is read from memory about once; the forward
// neighbours along the other axes are other columns of the same plane
// (cache hits).  1-D grids keep one thread per position.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kgs_internal.h"
#include "kgs_layout.h"

namespace kgs {
namespace {

constexpr int kBlock = 256;
constexpr int kSlots = 2048;  // maximum number of per-workgroup partials

struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD two_sum(double a, double b)
{
    const double s = a + b;
    const double bb = s - a;
    const double err = (a - (s - bb)) + (b - bb);
    return {s, err};
}

__device__ __forceinline__ DD dd_add(DD a, DD b)
{
    const DD s = two_sum(a.hi, b.hi);
    const double lo = s.lo + (a.lo + b.lo);
    const double hi = s.hi + lo;
    return {hi, lo - (hi - s.hi)};
}

__device__ __forceinline__ DD dd_add(DD a, double b)
{
    const DD s = two_sum(a.hi, b);
    const double lo = s.lo + a.lo;
    const double hi = s.hi + lo;
    return {hi, lo - (hi - s.hi)};
}

// Fixed-order tree over the 64 lanes; the result is valid in lane 0.
__device__ __forceinline__ DD wave_reduce(DD v)
{
    for (int off = 32; off > 0; off >>= 1) {
        DD o;
        o.hi = __shfl_down(v.hi, off, 64);
        o.lo = __shfl_down(v.lo, off, 64);
        v = dd_add(v, o);
    }
    return v;
}

// Reduce a workgroup of kBlock threads; the result is valid in thread 0.
__device__ __forceinline__ DD block_reduce(DD v)
{
    __shared__ double s_hi[kBlock / 64], s_lo[kBlock / 64];
    v = wave_reduce(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        s_hi[wave] = v.hi;
        s_lo[wave] = v.lo;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        DD acc = {s_hi[0], s_lo[0]};
        for (int w = 1; w < kBlock / 64; ++w) acc = dd_add(acc, DD{s_hi[w], s_lo[w]});
        v = acc;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ double ld(const T *p)
{
    return static_cast<double>(*p);
}

// Energy density of the point of colour c at (row, xh), with forward
// differences to the other colour:
//   1/2 (k1/h^2 sum_axes (dP^2 + dQ^2) + k2/h^2 sum_axes dU^2 + V^2 + mu^2 U^2)
//   - gamma (P^2 + Q^2) U.
template <int DIM, typename T>
__device__ __forceinline__ double density(const T *__restrict__ base, int64_t stride, int n,
                                          int c, int64_t row, int xh, const EnergyCoef &k)
{
    const int H = n >> 1;
    int s = 0;
    int64_t fwd0 = 0, fwd1 = 0;  // rows one step forward along axis 0 and axis 1
    if (DIM == 2) {
        const int i0 = static_cast<int>(row);
        s = i0;
        fwd0 = i0 == n - 1 ? 0 : i0 + 1;
    } else if (DIM == 3) {
        const int i0 = static_cast<int>(row / n);
        const int i1 = static_cast<int>(row - static_cast<int64_t>(i0) * n);
        s = i0 + i1;
        fwd0 = static_cast<int64_t>(i0 == n - 1 ? 0 : i0 + 1) * n + i1;
        fwd1 = static_cast<int64_t>(i0) * n + (i1 == n - 1 ? 0 : i1 + 1);
    }
    const int o = (s + DIM + 1 + c) & 1;
    int xp = xh + o;
    if (xp >= H) xp -= H;
    const T *oth_pq = pair_plane(base, stride, c ^ 1, PAIR_PQ);
    const T *oth_uv = pair_plane(base, stride, c ^ 1, PAIR_UV);
    const int64_t i = row * H + xh;
    const Pair<T> own_pq = ld_pair(pair_plane(base, stride, c, PAIR_PQ), i);
    const Pair<T> own_uv = ld_pair(pair_plane(base, stride, c, PAIR_UV), i);
    const double p = own_pq.x, q = own_pq.y;
    const double u = own_uv.x, v = own_uv.y;
    double gp = 0.0, gq = 0.0, gu = 0.0;
    auto add = [&](int64_t j) {
        const Pair<T> o_pq = ld_pair(oth_pq, j);
        const double dp = static_cast<double>(o_pq.x) - p;
        const double dq = static_cast<double>(o_pq.y) - q;
        const double du = ld(oth_uv + 2 * j) - u;
        gp = gp + dp * dp;
        gq = gq + dq * dq;
        gu = gu + du * du;
    };
    if (DIM >= 2) add(fwd0 * H + xh);
    if (DIM == 3) add(fwd1 * H + xh);
    add(row * H + xp);
    return 0.5 * (k.k1_h2 * (gp + gq) + k.k2_h2 * gu + v * v + k.mu2 * (u * u)) -
           k.gamma * (p * p + q * q) * u;
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock)
energy_partial_kernel(const T *__restrict__ base, int64_t stride, int n, int64_t count,
                      EnergyCoef k, double *__restrict__ partials)
{
    const int H = n >> 1;
    DD acc = {0.0, 0.0};
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; t < count;
         t += static_cast<int64_t>(gridDim.x) * kBlock) {
        const int64_t row = t / H;
        const int xh = static_cast<int>(t - row * H);
        acc = dd_add(acc, density<DIM>(base, stride, n, RED, row, xh, k));
        acc = dd_add(acc, density<DIM>(base, stride, n, BLUE, row, xh, k));
    }
    acc = block_reduce(acc);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = acc.hi;
        partials[2 * blockIdx.x + 1] = acc.lo;
    }
}

// Energy density of one point from its own values (p, q, u, v) and the
// other colour's forward neighbours: (P, Q) and U along axis 0, axis 1 (3-D
// only) and x, in that order (the order of density()).
template <int DIM>
__device__ __forceinline__ double density_from(double p, double q, double u, double v,
                                               const double (&nb)[3][3], const EnergyCoef &k)
{
    double gp = 0.0, gq = 0.0, gu = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double dp = nb[a][0] - p;
        const double dq = nb[a][1] - q;
        const double du = nb[a][2] - u;
        gp = gp + dp * dp;
        gq = gq + dq * dq;
        gu = gu + du * du;
    }
    return 0.5 * (k.k1_h2 * (gp + gq) + k.k2_h2 * gu + v * v + k.mu2 * (u * u)) -
           k.gamma * (p * p + q * q) * u;
}

template <typename T>
struct Col {
    double p[2], q[2], u[2], v[2];  // per colour
};

template <typename T>
__device__ __forceinline__ Col<T> load_column(const T *__restrict__ base, int64_t stride,
                                              int64_t i)
{
    Col<T> x;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const Pair<T> pq = ld_pair(pair_plane(base, stride, c, PAIR_PQ), i);
        const Pair<T> uv = ld_pair(pair_plane(base, stride, c, PAIR_UV), i);
        x.p[c] = pq.x;
        x.q[c] = pq.y;
        x.u[c] = uv.x;
        x.v[c] = uv.y;
    }
    return x;
}

// The other colour's forward neighbours in one plane that the own column
// does not hold: along axis 1 for both colours (3-D), and along x for the
// colour whose x neighbour is the next compressed position.
template <typename T>
struct PlaneNb {
    double a1[2][3];  // axis 1, per colour: P, Q, U of the other colour
    double x[3];      // x, for the colour with offset 1
};

template <int DIM, typename T>
__device__ __forceinline__ PlaneNb<T> load_plane_nb(const T *__restrict__ base, int64_t stride,
                                                    int64_t plane, int64_t fwd1, int64_t xrow,
                                                    int z, int i1)
{
    PlaneNb<T> nb;
    if (DIM == 3) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int oc = c ^ 1;
            const int64_t j = plane + fwd1;
            const Pair<T> pq = ld_pair(pair_plane(base, stride, oc, PAIR_PQ), j);
            nb.a1[c][0] = pq.x;
            nb.a1[c][1] = pq.y;
            nb.a1[c][2] = static_cast<double>(ld_global(pair_plane(base, stride, oc, PAIR_UV) + 2 * j));
        }
    }
    // colour c has x offset (s + DIM + 1 + c) & 1; offset 1 for c = (s + DIM) & 1
    const int s = DIM == 3 ? z + i1 : z;
    const int oc = ((s + DIM) & 1) ^ 1;
    const int64_t j = plane + xrow;
    const Pair<T> pq = ld_pair(pair_plane(base, stride, oc, PAIR_PQ), j);
    nb.x[0] = pq.x;
    nb.x[1] = pq.y;
    nb.x[2] = static_cast<double>(ld_global(pair_plane(base, stride, oc, PAIR_UV) + 2 * j));
    return nb;
}

// Workgroup (blockIdx.x, blockIdx.y): columns [256 blockIdx.x, +256) of a
// plane (cols per plane: n/2 in 2-D, n * n/2 in 3-D) and planes
// [chunk * blockIdx.y, +chunk) of axis 0.  Loads run ahead of their use:
// the own column two planes ahead, the in-plane neighbours one plane ahead.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock)
energy_stream_kernel(const T *__restrict__ base, int64_t stride, int n, int chunk, EnergyCoef k,
                     double *__restrict__ partials)
{
    const int H = n >> 1;
    const int64_t cols = DIM == 3 ? static_cast<int64_t>(n) * H : H;
    const int64_t col = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int z0 = blockIdx.y * chunk;
    const int z1 = min(n, z0 + chunk);
    DD acc = {0.0, 0.0};
    if (col < cols) {
        const int i1 = DIM == 3 ? static_cast<int>(col / H) : 0;
        const int xh = static_cast<int>(col - static_cast<int64_t>(i1) * H);
        const int xn = xh + 1 == H ? 0 : xh + 1;
        // columns of the forward neighbours inside a plane: the next row
        // along axis 1 (3-D) and the next compressed x position
        const int64_t fwd1 = DIM == 3 ? static_cast<int64_t>(i1 == n - 1 ? 0 : i1 + 1) * H + xh : 0;
        const int64_t xrow = static_cast<int64_t>(i1) * H + xn;
        auto wrapz = [&](int z) { return z >= n ? z - n : z; };
        Col<T> cur = load_column(base, stride, static_cast<int64_t>(z0) * cols + col);
        Col<T> nxt = load_column(base, stride, static_cast<int64_t>(wrapz(z0 + 1)) * cols + col);
        PlaneNb<T> nbc = load_plane_nb<DIM>(base, stride, static_cast<int64_t>(z0) * cols, fwd1,
                                            xrow, z0, i1);
        for (int z = z0; z < z1; ++z) {
            Col<T> nn = nxt;
            PlaneNb<T> nbn = nbc;
            if (z + 1 < z1) {
                nn = load_column(base, stride, static_cast<int64_t>(wrapz(z + 2)) * cols + col);
                nbn = load_plane_nb<DIM>(base, stride, static_cast<int64_t>(z + 1) * cols, fwd1,
                                         xrow, z + 1, i1);
            }
            const int s = DIM == 3 ? z + i1 : z;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int o = (s + DIM + 1 + c) & 1;  // x = 2 xh + o for colour c
                const int oc = c ^ 1;
                double nb[3][3];
                // axis 0: the other colour at this column of the next plane
                nb[0][0] = nxt.p[oc];
                nb[0][1] = nxt.q[oc];
                nb[0][2] = nxt.u[oc];
                int a = 1;
                if (DIM == 3) {
                    nb[1][0] = nbc.a1[c][0];
                    nb[1][1] = nbc.a1[c][1];
                    nb[1][2] = nbc.a1[c][2];
                    a = 2;
                }
                // x: the other colour at compressed position xh + o
                nb[a][0] = o ? nbc.x[0] : cur.p[oc];
                nb[a][1] = o ? nbc.x[1] : cur.q[oc];
                nb[a][2] = o ? nbc.x[2] : cur.u[oc];
                acc = dd_add(acc, density_from<DIM>(cur.p[c], cur.q[c], cur.u[c], cur.v[c], nb, k));
            }
            cur = nxt;
            nxt = nn;
            nbc = nbn;
        }
    }
    acc = block_reduce(acc);
    if (threadIdx.x == 0) {
        const int b = blockIdx.y * gridDim.x + blockIdx.x;
        partials[2 * b] = acc.hi;
        partials[2 * b + 1] = acc.lo;
    }
}

__global__ void __launch_bounds__(kBlock)
energy_final_kernel(const double *__restrict__ partials, int nparts, double *__restrict__ out)
{
    DD acc = {0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += kBlock)
        acc = dd_add(acc, DD{partials[2 * i], partials[2 * i + 1]});
    acc = block_reduce(acc);
    if (threadIdx.x == 0) {
        out[0] = acc.hi;
        out[1] = acc.lo;
    }
}

}  // namespace

int energy_partial_slots() { return kSlots; }

hipError_t launch_energy(const Geometry &g, int precision, const void *state,
                         const EnergyCoef &k, double *partials, double *out, hipStream_t s)
{
    if (!state || !partials || !out || g.dim < 1 || g.dim > 3 || g.n < 2 || (g.n & 1) ||
        g.count <= 0 || g.stride < g.count)
        return hipErrorInvalidValue;
    int64_t blocks = (g.count + kBlock - 1) / kBlock;
    if (blocks > kSlots) blocks = kSlots;
    // 2-D and 3-D: columns of a plane of axis 0 in workgroups of kBlock,
    // and chunks of planes long enough for about 2^18 threads in all but no
    // shorter than needed to keep the workgroups within kSlots (grids with
    // more than kSlots workgroups of columns per plane use one thread per
    // position instead)
    const int64_t cols = g.dim == 3 ? static_cast<int64_t>(g.n) * (g.n / 2) : g.n / 2;
    const int64_t bx = (cols + kBlock - 1) / kBlock;
    if (g.dim >= 2 && bx <= kSlots) {
        int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(32, cols * g.n / (1 << 18)));
        while (bx * ((g.n + chunk - 1) / chunk) > kSlots) ++chunk;
        const int64_t by = (g.n + chunk - 1) / chunk;
        blocks = bx * by;
        const dim3 grid2(static_cast<unsigned>(bx), static_cast<unsigned>(by));
#define KGS_ENERGY_S(D, T)                                                                      \
    hipLaunchKernelGGL((energy_stream_kernel<D, T>), grid2, dim3(kBlock), 0, s,                 \
                       static_cast<const T *>(state), g.stride, g.n, static_cast<int>(chunk), k, \
                       partials)
        if (precision == 0) {
            if (g.dim == 2) KGS_ENERGY_S(2, double);
            else KGS_ENERGY_S(3, double);
        } else {
            if (g.dim == 2) KGS_ENERGY_S(2, float);
            else KGS_ENERGY_S(3, float);
        }
#undef KGS_ENERGY_S
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(kBlock), 0, s, partials,
                           static_cast<int>(blocks), out);
        return hipGetLastError();
    }
    const dim3 grid(static_cast<unsigned>(blocks)), threads(kBlock);
#define KGS_ENERGY(D, T)                                                                        \
    hipLaunchKernelGGL((energy_partial_kernel<D, T>), grid, threads, 0, s,                      \
                       static_cast<const T *>(state), g.stride, g.n, g.count, k, partials)
    if (precision == 0) {
        if (g.dim == 1) KGS_ENERGY(1, double);
        else if (g.dim == 2) KGS_ENERGY(2, double);
        else KGS_ENERGY(3, double);
    } else {
        if (g.dim == 1) KGS_ENERGY(1, float);
        else if (g.dim == 2) KGS_ENERGY(2, float);
        else KGS_ENERGY(3, float);
    }
#undef KGS_ENERGY
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(kBlock), 0, s, partials,
                       static_cast<int>(blocks), out);
    return hipGetLastError();
}

}  // namespace kgs
