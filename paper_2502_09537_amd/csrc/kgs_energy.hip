// Discrete energy E_h of sec. 2 (without the h^dim factor, which the host
// applies): a deterministic, compensated float64 reduction.
//
// Each thread sums the energy of its points into a double-double
// (TwoSum), a wavefront of 64 lanes combines its lanes with shuffles in a
// fixed tree, the waves of a workgroup combine through LDS in a fixed order,
// and one final workgroup combines the per-workgroup partials in a fixed
// order.  The grid size depends only on the problem size, so the result is
// bitwise reproducible run to run.
//
// 2-D and 3-D grids stream along axis 0: a thread owns one column (a row
// position along the other axes and a compressed x position, both colours)
// and walks it through a chunk of consecutive planes of axis 0.  The energy
// is summed edge by edge: on the checkerboard every edge of the grid joins a
// red and a blue point, so the red point of a column takes the squared
// differences to all of its 2*dim blue neighbours and both points add their
// own terms.  These are the blue neighbours that the adjoint red sweep
// reads, so the same pass can first apply the sweep that closes a step
// (energy_closing_kernel): it rewrites only red points, each from its own
// old values, which no other thread reads, so it runs in place.  The blue
// neighbours along axis 0 are the thread's own column one plane back and
// ahead (registers), the other ones are other columns of the same plane
// (cache hits).  1-D grids keep one thread per position and forward
// differences.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kgs_energy.h"
#include "kgs_internal.h"
#include "kgs_layout.h"
#include "kgs_plan.h"
#include "kgs_point.h"

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

// (P, Q, U, V) of one point, and (P, Q, U) of a neighbour, as float64.
struct Pt {
    double p, q, u, v;
};

struct Nb {
    double p, q, u;
};

template <typename T>
__device__ __forceinline__ Pt load_pt(const T *__restrict__ pq, const T *__restrict__ uv, int64_t i)
{
    const Pair<T> a = ld_pair(pq, i), b = ld_pair(uv, i);
    return Pt{static_cast<double>(a.x), static_cast<double>(a.y), static_cast<double>(b.x),
              static_cast<double>(b.y)};
}

template <typename T>
__device__ __forceinline__ Nb load_nb(const T *__restrict__ pq, const T *__restrict__ uv, int64_t j)
{
    const Pair<T> a = ld_pair(pq, j);
    return Nb{static_cast<double>(a.x), static_cast<double>(a.y),
              static_cast<double>(ld_global(uv + 2 * j))};
}

// The in-plane blue neighbours of a red point: axis 1 -, + (3-D) and x -, +.
struct PlaneNb {
    Nb y_m, y_p, x_m, x_p;
};

// Workgroup (blockIdx.x, blockIdx.y): columns [256 blockIdx.x, +256) of a
// plane (columns per plane: n/2 in 2-D, n * n/2 in 3-D) and planes
// [chunk * blockIdx.y, +chunk) of axis 0.  Per plane a thread adds, in this
// order: the red point's squared differences to its blue neighbours (axis 0
// -, +, axis 1 -, + in 3-D, x -, +) with its own terms, then the blue
// point's own terms.  With CLOSE the red point first takes the adjoint red
// sweep (the neighbour sums in the order of the sweep kernels, so the state
// is bitwise that of the sweep) and is stored; its energy uses the stored
// values.  Loads run one plane ahead of their use.
template <int DIM, typename T, bool CLOSE>
__global__ void __launch_bounds__(kBlock)
energy_stream_kernel(T *__restrict__ base, int64_t stride, int n, int chunk, EnergyCoef k, Coef kc,
                     double *__restrict__ partials)
{
    const int H = n >> 1;
    const int64_t cols = DIM == 3 ? static_cast<int64_t>(n) * H : H;
    const int64_t col = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int z0 = blockIdx.y * chunk;
    const int z1 = min(n, z0 + chunk);
    DD acc = {0.0, 0.0};
    if (col < cols) {
        T *rpq = pair_plane(base, stride, RED, PAIR_PQ), *ruv = pair_plane(base, stride, RED, PAIR_UV);
        const T *bpq = pair_plane(base, stride, BLUE, PAIR_PQ);
        const T *buv = pair_plane(base, stride, BLUE, PAIR_UV);
        const int i1 = DIM == 3 ? static_cast<int>(col / H) : 0;
        const int xh = static_cast<int>(col - static_cast<int64_t>(i1) * H);
        const int xhm = xh == 0 ? H - 1 : xh - 1, xhp = xh + 1 == H ? 0 : xh + 1;
        const int64_t row = static_cast<int64_t>(i1) * H;  // first column of this row in a plane
        const int64_t ym = DIM == 3 ? static_cast<int64_t>(i1 == 0 ? n - 1 : i1 - 1) * H + xh : 0;
        const int64_t yp = DIM == 3 ? static_cast<int64_t>(i1 == n - 1 ? 0 : i1 + 1) * H + xh : 0;
        auto wrapz = [&](int z) { return z < 0 ? z + n : z >= n ? z - n : z; };
        auto plane_nb = [&](int z) {
            const int64_t pl = static_cast<int64_t>(z) * cols;
            const int s = DIM == 3 ? z + i1 : z;
            const int o = (s + DIM + 1 + RED) & 1;  // red point at x = 2 xh + o
            PlaneNb nb;
            if (DIM == 3) {
                nb.y_m = load_nb(bpq, buv, pl + ym);
                nb.y_p = load_nb(bpq, buv, pl + yp);
            }
            nb.x_m = load_nb(bpq, buv, pl + row + (o ? xh : xhm));
            nb.x_p = load_nb(bpq, buv, pl + row + (o ? xhp : xh));
            return nb;
        };
        auto blue_at = [&](int z) { return load_pt(bpq, buv, static_cast<int64_t>(wrapz(z)) * cols + col); };
        Pt b_m = blue_at(z0 - 1), b_0 = blue_at(z0), b_p = blue_at(z0 + 1);
        Pt r_0 = load_pt(rpq, ruv, static_cast<int64_t>(z0) * cols + col);
        PlaneNb nb_0 = plane_nb(z0);
        for (int z = z0; z < z1; ++z) {
            Pt b_pp = b_p, r_1 = r_0;
            PlaneNb nb_1 = nb_0;
            if (z + 1 < z1) {
                b_pp = blue_at(z + 2);
                r_1 = load_pt(rpq, ruv, static_cast<int64_t>(z + 1) * cols + col);
                nb_1 = plane_nb(z + 1);
            }
            double pr = r_0.p, pi = r_0.q, u = r_0.u, v = r_0.v;
            if (CLOSE) {
                double sr = b_m.p, si = b_m.q, su = b_m.u;
                sr = sr + b_p.p;
                si = si + b_p.q;
                su = su + b_p.u;
                if (DIM == 3) {
                    sr = sr + nb_0.y_m.p;
                    si = si + nb_0.y_m.q;
                    su = su + nb_0.y_m.u;
                    sr = sr + nb_0.y_p.p;
                    si = si + nb_0.y_p.q;
                    su = su + nb_0.y_p.u;
                }
                sr = sr + nb_0.x_m.p;
                si = si + nb_0.x_m.q;
                su = su + nb_0.x_m.u;
                sr = sr + nb_0.x_p.p;
                si = si + nb_0.x_p.q;
                su = su + nb_0.x_p.u;
                sweep_point<PASS_R_ADJ, T>(kc, pr, pi, u, v, sr, si, su);
                const T tp = static_cast<T>(pr), tq = static_cast<T>(pi);
                const T tu = static_cast<T>(u), tv = static_cast<T>(v);
                const int64_t i = static_cast<int64_t>(z) * cols + col;
                st_pair(rpq, i, tp, tq);
                st_pair(ruv, i, tu, tv);
                pr = tp;
                pi = tq;
                u = tu;
                v = tv;
            }
            double gp = 0.0, gq = 0.0, gu = 0.0;
            auto edge = [&](double bp, double bq, double bu) {
                const double dp = bp - pr, dq = bq - pi, du = bu - u;
                gp = gp + dp * dp;
                gq = gq + dq * dq;
                gu = gu + du * du;
            };
            edge(b_m.p, b_m.q, b_m.u);
            edge(b_p.p, b_p.q, b_p.u);
            if (DIM == 3) {
                edge(nb_0.y_m.p, nb_0.y_m.q, nb_0.y_m.u);
                edge(nb_0.y_p.p, nb_0.y_p.q, nb_0.y_p.u);
            }
            edge(nb_0.x_m.p, nb_0.x_m.q, nb_0.x_m.u);
            edge(nb_0.x_p.p, nb_0.x_p.q, nb_0.x_p.u);
            acc = dd_add(acc, 0.5 * (k.k1_h2 * (gp + gq) + k.k2_h2 * gu + v * v + k.mu2 * (u * u)) -
                                  k.gamma * (pr * pr + pi * pi) * u);
            acc = dd_add(acc, 0.5 * (b_0.v * b_0.v + k.mu2 * (b_0.u * b_0.u)) -
                                  k.gamma * (b_0.p * b_0.p + b_0.q * b_0.q) * b_0.u);
            b_m = b_0;
            b_0 = b_p;
            b_p = b_pp;
            r_0 = r_1;
            nb_0 = nb_1;
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

namespace {

// The streaming launch shape of a 2-D or 3-D grid (energy_grid): the same
// for the plain and the closing form, so both sum in the same order.  False
// when the grid does not stream.  Measured on MI355X at 256^3 float64, the
// closing form: 167 us with 768 workgroups (one round of three per CU)
// against 179 us with 1024 (32 planes each).
bool stream_shape(const Geometry &g, int64_t &bx, int64_t &by, int64_t &chunk)
{
    return energy_grid(g.dim, g.n, device_cus(), &bx, &by, &chunk);
}

bool geometry_ok(const Geometry &g)
{
    return g.dim >= 1 && g.dim <= 3 && g.n >= 2 && !(g.n & 1) && g.count > 0 && g.stride >= g.count;
}

template <bool CLOSE>
hipError_t launch_stream(const Geometry &g, int precision, void *state, const EnergyCoef &k,
                         const Coef &kc, double *partials, double *out, hipStream_t s)
{
    int64_t bx = 0, by = 0, chunk = 0;
    if (!stream_shape(g, bx, by, chunk)) return hipErrorNotSupported;
    const dim3 grid2(static_cast<unsigned>(bx), static_cast<unsigned>(by));
#define KGS_ENERGY_S(D, T)                                                                      \
    hipLaunchKernelGGL((energy_stream_kernel<D, T, CLOSE>), grid2, dim3(kBlock), 0, s,          \
                       static_cast<T *>(state), g.stride, g.n, static_cast<int>(chunk), k, kc,  \
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
                       static_cast<int>(bx * by), out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_energy(const Geometry &g, int precision, const void *state,
                         const EnergyCoef &k, double *partials, double *out, hipStream_t s)
{
    if (!state || !partials || !out || !geometry_ok(g)) return hipErrorInvalidValue;
    // the streaming kernel only reads the state without CLOSE
    hipError_t e = launch_stream<false>(g, precision, const_cast<void *>(state), k, Coef{},
                                        partials, out, s);
    if (e != hipErrorNotSupported) return e;
    int64_t blocks = (g.count + kBlock - 1) / kBlock;
    if (blocks > kSlots) blocks = kSlots;
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
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(kBlock), 0, s, partials,
                       static_cast<int>(blocks), out);
    return hipGetLastError();
}

hipError_t launch_energy_closing(const Geometry &g, int precision, void *state,
                                 const EnergyCoef &k, const Coef &kc, double *partials,
                                 double *out, hipStream_t s)
{
    if (!state || !partials || !out || !geometry_ok(g)) return hipErrorInvalidValue;
    return launch_stream<true>(g, precision, state, k, kc, partials, out, s);
}

}  // namespace kgs
