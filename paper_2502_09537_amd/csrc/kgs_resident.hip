// Resident kernel: a whole simulation lives in one workgroup for a whole run
// of K DP-AVF2 steps (all 2K+1 colour sweeps of the run in one launch).
//
// Small grids (the 1-D problems of sec. 5, small 2-D/3-D grids) have too few
// points to fill even one launch of the sweep kernel, so a run of sweeps is
// bound by launch latency (two launches per step).  Here each thread keeps
// the four fields of its points of both colours in registers, and the
// fields that neighbours read (P, Q, U; u_t is never read by a neighbour)
// are published in LDS.  A colour sweep reads the other colour from LDS and
// rewrites its own colour, and one barrier separates consecutive sweeps, so
// HBM is touched only to load the state at the start of the run and to
// store it at the end.
//
// The same kernel advances a batch: workgroup b runs member b (its own
// grid, constants and number of steps), so many small simulations share one
// persistent launch.
//
// Each point goes through the same sweep kinds in the same order with the
// same neighbour summation order as the sweep kernel, and values are rounded
// to the storage type T at the same places, so the result is bitwise that of
// kgs_step with any other kernel.
#include <mutex>
#include <set>

#include <hip/hip_runtime.h>

#include "kgs_internal.h"
#include "kgs_layout.h"
#include "kgs_point.h"
#include "kgs_sweep_body.h"

namespace kgs {
namespace {

constexpr int kMaxThreads = 1024;
constexpr int kMaxPpt = 4;  // points of each colour per thread

// Per-thread data of its points t = threadIdx.x + j blockDim.x, j < PPT.
// P, Q and U of both colours live in LDS (plane (colour, field) at
// lds + (3 colour + field) C); u_t is never read by a neighbour and stays in
// registers.  Neighbour positions: the rows one step away along the non-x
// axes are the same for both colours; the x-neighbours depend on the colour.
template <int DIM, typename T, int PPT>
struct Points {
    T v[2][PPT];                  // u_t, [colour][point]
    int nrow[PPT][2 * DIM - 2 > 0 ? 2 * DIM - 2 : 1];  // (row +- e_a) H + xh
    int nx[PPT][2][2];            // [point][colour]: row H + (x -, x +) of the other colour
};

template <int DIM>
__device__ __forceinline__ void neighbours(int t, int n, int *nrow, int (&nx)[2][2])
{
    const int H = n >> 1;
    const int row = t / H;
    const int xh = t - row * H;
    const sweep_detail::RowInfo<DIM> r = sweep_detail::row_info<DIM>(row, n);
    if (DIM > 1)
        for (int a = 0; a < 2 * (DIM - 1); ++a) nrow[a] = static_cast<int>(r.nb[a]) * H + xh;
    for (int c = 0; c < 2; ++c) {
        const int o = (r.s + DIM + 1 + c) & 1;
        int xm = xh - 1 + o;
        if (xm < 0) xm += H;
        int xp = xh + o;
        if (xp >= H) xp -= H;
        nx[c][0] = row * H + xm;
        nx[c][1] = row * H + xp;
    }
}

// Sum of plane f over the other-colour neighbours of a point, in the
// summation order of the sweep kernel: axis 0 -, axis 0 +, [axis 1 -,
// axis 1 +,] x -, x +.
template <int DIM, typename T>
__device__ __forceinline__ double nsum(const T *f, const int *nrow, const int *nx)
{
    double acc;
    if (DIM == 1) {
        acc = static_cast<double>(f[nx[0]]);
    } else {
        acc = static_cast<double>(f[nrow[0]]);
        for (int a = 1; a < 2 * (DIM - 1); ++a) acc = acc + static_cast<double>(f[nrow[a]]);
        acc = acc + static_cast<double>(f[nx[0]]);
    }
    return acc + static_cast<double>(f[nx[1]]);
}

template <int DIM, typename T, int PPT, int KIND, int colour>
__device__ __forceinline__ void sweep(T *lds, int C, const Coef &k, Points<DIM, T, PPT> &p)
{
    const T *oth = lds + 3 * (colour ^ 1) * C;
    T *mine = lds + 3 * colour * C;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int t = threadIdx.x + j * blockDim.x;
        if (t >= C) continue;
        const double sr = nsum<DIM>(oth, p.nrow[j], p.nx[j][colour]);
        const double si = nsum<DIM>(oth + C, p.nrow[j], p.nx[j][colour]);
        const double su = nsum<DIM>(oth + 2 * C, p.nrow[j], p.nx[j][colour]);
        double pr = static_cast<double>(mine[t]);
        double pi = static_cast<double>(mine[C + t]);
        double u = static_cast<double>(mine[2 * C + t]);
        double v = static_cast<double>(p.v[colour][j]);
        sweep_point<KIND, T>(k, pr, pi, u, v, sr, si, su);
        mine[t] = static_cast<T>(pr);
        mine[C + t] = static_cast<T>(pi);
        mine[2 * C + t] = static_cast<T>(u);
        p.v[colour][j] = static_cast<T>(v);
    }
}

template <int DIM, typename T, int PPT>
__global__ void __launch_bounds__(kMaxThreads)
resident_kernel(ResidentMember one, const ResidentMember *__restrict__ list,
                const int64_t *__restrict__ steps_each, int64_t steps_all)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const ResidentMember m = list ? list[blockIdx.x] : one;
    const int64_t steps = !list ? m.steps : steps_each ? steps_each[blockIdx.x] : steps_all;
    if (steps <= 0) return;  // the whole workgroup leaves together
    T *lds = reinterpret_cast<T *>(lds_raw);
    T *g = static_cast<T *>(m.state);
    const int64_t S = m.stride;
    const int C = m.count;
    Points<DIM, T, PPT> p;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int t = threadIdx.x + j * blockDim.x;
        if (t >= C) continue;
        neighbours<DIM>(t, m.n, p.nrow[j], p.nx[j]);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const Pair<T> pq = ld_pair(pair_plane(g, S, c, PAIR_PQ), t);
            const Pair<T> uv = ld_pair(pair_plane(g, S, c, PAIR_UV), t);
            lds[(3 * c + F_P) * C + t] = pq.x;
            lds[(3 * c + F_Q) * C + t] = pq.y;
            lds[(3 * c + F_U) * C + t] = uv.x;
            p.v[c][j] = uv.y;
        }
    }
    __syncthreads();
    const Coef k = m.k;
    sweep<DIM, T, PPT, PASS_R_BASE, RED>(lds, C, k, p);
    __syncthreads();
    for (int64_t i = 1; i < steps; ++i) {
        sweep<DIM, T, PPT, PASS_B_FULL, BLUE>(lds, C, k, p);
        __syncthreads();
        sweep<DIM, T, PPT, PASS_R_ADJ_BASE, RED>(lds, C, k, p);
        __syncthreads();
    }
    sweep<DIM, T, PPT, PASS_B_FULL, BLUE>(lds, C, k, p);
    __syncthreads();
    sweep<DIM, T, PPT, PASS_R_ADJ, RED>(lds, C, k, p);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int t = threadIdx.x + j * blockDim.x;
        if (t >= C) continue;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            st_pair(pair_plane(g, S, c, PAIR_PQ), t, lds[(3 * c + F_P) * C + t],
                    lds[(3 * c + F_Q) * C + t]);
            st_pair(pair_plane(g, S, c, PAIR_UV), t, lds[(3 * c + F_U) * C + t], p.v[c][j]);
        }
    }
}

// LDS one workgroup may use on the current device (kResidentMaxLds when no
// device can be queried, so host-only callers see the gfx950 figure).
int lds_limit()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return kResidentMaxLds;
    return v < kResidentMaxLds ? v : kResidentMaxLds;
}

template <int DIM, typename T, int PPT>
hipError_t allow_lds(int bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(resident_kernel<DIM, T, PPT>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <int DIM>
hipError_t allow_lds_dim(int bytes)
{
    hipError_t e = hipSuccess;
    for (hipError_t r : {allow_lds<DIM, double, 1>(bytes), allow_lds<DIM, double, 2>(bytes),
                         allow_lds<DIM, double, 4>(bytes), allow_lds<DIM, float, 1>(bytes),
                         allow_lds<DIM, float, 2>(bytes), allow_lds<DIM, float, 4>(bytes)})
        if (r != hipSuccess) e = r;
    return e;
}

template <int DIM, typename T, int PPT>
hipError_t launch_typed(const ResidentMember &one, const ResidentMember *list,
                        const int64_t *steps_each, int64_t steps_all, int nm, int threads,
                        size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((resident_kernel<DIM, T, PPT>), dim3(nm), dim3(threads), lds, s, one, list,
                       steps_each, steps_all);
    return hipGetLastError();
}

template <int DIM, typename T>
hipError_t launch_ppt(int ppt, const ResidentMember &one, const ResidentMember *list,
                      const int64_t *steps_each, int64_t steps_all, int nm, int threads,
                      size_t lds, hipStream_t s)
{
    if (ppt == 1) return launch_typed<DIM, T, 1>(one, list, steps_each, steps_all, nm, threads, lds, s);
    if (ppt == 2) return launch_typed<DIM, T, 2>(one, list, steps_each, steps_all, nm, threads, lds, s);
    return launch_typed<DIM, T, 4>(one, list, steps_each, steps_all, nm, threads, lds, s);
}

}  // namespace

bool resident_fits(int64_t count, int elem_bytes)
{
    return count >= 1 && count <= static_cast<int64_t>(kMaxThreads) * kMaxPpt &&
           6 * count * elem_bytes <= lds_limit();
}

hipError_t resident_prepare()
{
    static std::mutex mu;
    static std::set<int> ready;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if (ready.count(dev)) return hipSuccess;
    const int bytes = lds_limit();
    for (hipError_t r : {allow_lds_dim<1>(bytes), allow_lds_dim<2>(bytes), allow_lds_dim<3>(bytes)})
        if (r != hipSuccess) e = r;
    if (e == hipSuccess) ready.insert(dev);
    return e;
}

hipError_t launch_resident(int dim, int precision, const ResidentMember &one,
                           const ResidentMember *list, const int64_t *steps_each,
                           int64_t steps_all, int nm, int64_t max_count, hipStream_t s)
{
    const int eb = precision == 0 ? 8 : 4;
    if (dim < 1 || dim > 3 || nm < 1 || (!list && nm != 1) || !resident_fits(max_count, eb))
        return hipErrorInvalidValue;
    if (!list && (one.count != max_count || one.n < 2 || one.state == nullptr))
        return hipErrorInvalidValue;
    int threads = static_cast<int>((max_count + 63) / 64 * 64);
    if (threads > kMaxThreads) threads = kMaxThreads;
    const int64_t need = (max_count + threads - 1) / threads;
    const int ppt = need <= 1 ? 1 : need <= 2 ? 2 : 4;
    const size_t lds = static_cast<size_t>(6 * max_count * eb);
    if (lds > static_cast<size_t>(lds_limit())) return hipErrorInvalidValue;
    hipError_t e = resident_prepare();
    if (e != hipSuccess) return e;
#define KGS_RES(D, T) \
    return launch_ppt<D, T>(ppt, one, list, steps_each, steps_all, nm, threads, lds, s)
    if (precision == 0) {
        if (dim == 1) KGS_RES(1, double);
        if (dim == 2) KGS_RES(2, double);
        KGS_RES(3, double);
    }
    if (dim == 1) KGS_RES(1, float);
    if (dim == 2) KGS_RES(2, float);
    KGS_RES(3, float);
#undef KGS_RES
}

}  // namespace kgs
