// 2-D streaming kernel: S consecutive colour sweeps (S/2 DP-AVF2 steps) of
// many 2-D simulations in one launch, each read from one buffer and written
// to another.
//
// Work decomposition.  A task is one wave: 64 lanes across a tile of
// compressed x positions, streaming along y through a chunk of rows.  Each
// sweep widens the dependency cone by one point along each axis, so the tile
// carries a halo of kHalo = 2 compressed positions on each side (enough for
// S <= 4 sweeps; recomputed by the neighbouring tile) and the chunk is
// extended by S rows before and after.  The tile geometry does not depend on
// S, so launches of 2 and 4 sweeps share their task lists.  A row of n/2 <= 64
// compressed positions fits one wave whole: the tile is the periodic row
// itself and needs no halo.
//
// Pipeline (as in the 3-D kernel, with rows in place of planes): at step p
// the wave loads row y0 - S + p (both colours, level 0), and sweep stage j
// (colour j&1, level j+1) updates row (y0 - S + p) - 1 - j.  The y
// neighbours are rows of the previous level held in per-level register
// FIFOs; of the two x neighbours one is at the lane's own position and the
// other one lane to the left or right, read with a lane shuffle.  Tasks
// never communicate, so the kernel needs neither LDS nor barriers.  The
// neighbour sums use the order of the one-sweep kernel (axis 0 -, +, x -,
// +), so results are bitwise those of every other kernel.
#include <hip/hip_runtime.h>

#include "kgs_internal.h"
#include "kgs_layout.h"
#include "kgs_point.h"

namespace kgs {
namespace {

constexpr int kWaves = 4;           // waves (tasks) per workgroup
constexpr int kHalo = 2;            // compressed positions of halo per side
constexpr int kTile = 64 - 2 * kHalo;  // compressed positions a tile writes

template <typename T>
struct Vals {
    T f[4];  // P, Q, U, V
};

// Plane FIFOs as rings indexed by the pipeline step modulo 3 (see the 3-D
// kernel): R/B level 0 of the red/blue rows, Bn the next blue row, F[j]
// the output rows of stage j.
template <typename T, int S>
struct Pipe {
    Vals<T> R[3], B[3], Bn, F[S - 1][3];
};

// The four values of point pt of colour c: two pair loads.
template <typename T>
__device__ __forceinline__ Vals<T> load_vals(const T *base, int64_t stride, int c, int64_t pt)
{
    const Pair<T> pq = ld_pair(pair_plane(base, stride, c, PAIR_PQ), pt);
    const Pair<T> uv = ld_pair(pair_plane(base, stride, c, PAIR_UV), pt);
    return Vals<T>{{pq.x, pq.y, uv.x, uv.y}};
}

template <typename T>
__device__ __forceinline__ void store_vals(T *base, int64_t stride, int c, int64_t pt,
                                           const Vals<T> &x)
{
    st_pair(pair_plane(base, stride, c, PAIR_PQ), pt, x.f[0], x.f[1]);
    st_pair(pair_plane(base, stride, c, PAIR_UV), pt, x.f[2], x.f[3]);
}

__device__ __forceinline__ int wrap(int v, int m)
{
    v %= m;
    return v < 0 ? v + m : v;
}

template <typename T>
__device__ __forceinline__ T lane_read(T v, int src)
{
    return __shfl(v, src, 64);
}

struct Task {
    const Stream2dMember *m;
    int n, H, lane, xh, src_m, src_p;
    bool in_tile;
    int y0, L;
};

template <typename T, int S, int PH>
__device__ __forceinline__ void step2d(Pipe<T, S> &st, const Task &t, const T *__restrict__ in,
                                       T *__restrict__ out, int64_t stride, int p, int steps,
                                       int &y_load, bool first, const Coef &k)
{
    constexpr int s0 = PH % 3, s1 = (PH + 2) % 3, s2 = (PH + 1) % 3;  // steps p, p-1, p-2
    const int n = t.n, H = t.H;
    st.B[s0] = st.Bn;
    if (p + 1 < steps) {
        const int yn = y_load + 1 == n ? 0 : y_load + 1;
        const int64_t pt = static_cast<int64_t>(yn) * H + t.xh;
        st.R[s2] = load_vals(in, stride, RED, pt);
        st.Bn = load_vals(in, stride, BLUE, pt);
    }
    // x-offset of the updated colour in the updated rows: the same for every
    // stage of the step
    const int o = y_load & 1;
    const int src = o ? t.src_p : t.src_m;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        if (p < 2 * j + 2) continue;  // pipeline not yet filled for stage j
        const int c = j & 1;
        const Vals<T> &up = (j == 0) ? st.B[s0] : st.F[j > 0 ? j - 1 : 0][s0];
        const Vals<T> &mid = (j == 0) ? st.B[s1] : st.F[j > 0 ? j - 1 : 0][s1];
        const Vals<T> &dn = (j == 0) ? st.B[s2] : st.F[j > 0 ? j - 1 : 0][s2];
        double sum[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const T other = lane_read(mid.f[q], src);
            const double xm = static_cast<double>(o ? mid.f[q] : other);
            const double xp = static_cast<double>(o ? other : mid.f[q]);
            double a = static_cast<double>(dn.f[q]);
            a = a + static_cast<double>(up.f[q]);
            a = a + xm;
            a = a + xp;
            sum[q] = a;
        }
        const Vals<T> &own = (j == 0) ? st.R[s1] : (j == 1) ? st.B[s2] : st.F[j > 1 ? j - 2 : 0][s2];
        double pr = own.f[0], pi = own.f[1], u = own.f[2], v = own.f[3];
        if (c == RED) {
            if (j == 0 && first)
                sweep_point<PASS_R_BASE, T>(k, pr, pi, u, v, sum[0], sum[1], sum[2]);
            else
                sweep_point<PASS_R_ADJ_BASE, T>(k, pr, pi, u, v, sum[0], sum[1], sum[2]);
        } else {
            sweep_point<PASS_B_FULL, T>(k, pr, pi, u, v, sum[0], sum[1], sum[2]);
        }
        Vals<T> res;
        res.f[0] = static_cast<T>(pr);
        res.f[1] = static_cast<T>(pi);
        res.f[2] = static_cast<T>(u);
        res.f[3] = static_cast<T>(v);
        if (j < S - 1) {
            st.F[j < S - 1 ? j : 0][s0] = res;
        } else if (t.in_tile) {
            // final level S at row z: colour c from this stage, the other
            // colour from stage S-2 one step ago
            const int z = wrap(y_load - S, n);
            const int64_t pt = static_cast<int64_t>(z) * H + t.xh;
            store_vals(out, stride, c, pt, res);
            store_vals(out, stride, c ^ 1, pt, st.F[S - 2][s1]);
        }
    }
    y_load = y_load + 1 == n ? 0 : y_load + 1;
}

template <typename T, int S>
__global__ void __launch_bounds__(64 * kWaves)
stream2d_kernel(Stream2dMember one, const Stream2dMember *__restrict__ list, int nm,
                int64_t total_tasks)
{
    static_assert((S + 1) / 2 <= kHalo, "halo too narrow for S sweeps");
    // the task is uniform across its wave: the member lookup and the
    // descriptor stay in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int64_t task = static_cast<int64_t>(blockIdx.x) * kWaves + wave;
    if (task >= total_tasks) return;  // whole waves leave; nothing waits for them
    Stream2dMember mb = one;
    if (list) {
        int lo = 0, hi = nm - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (list[mid].task_begin <= task) lo = mid;
            else hi = mid - 1;
        }
        mb = list[lo];
    }
    Task t;
    t.n = mb.n;
    t.H = t.n >> 1;
    t.lane = threadIdx.x & 63;
    const int64_t local = task - mb.task_begin;
    const int tile = static_cast<int>(local % mb.tiles_x);
    const int chunk_i = static_cast<int>(local / mb.tiles_x);
    if (t.H <= 64) {
        // the whole periodic row in one wave, lanes >= H duplicate lanes - H
        t.xh = t.lane % t.H;
        t.src_m = t.xh == 0 ? t.H - 1 : t.xh - 1;
        t.src_p = t.xh + 1 == t.H ? 0 : t.xh + 1;
        t.in_tile = t.lane < t.H;
    } else {
        const int xu = tile * kTile - kHalo + t.lane;  // unwrapped compressed x
        t.xh = wrap(xu, t.H);
        t.src_m = t.lane > 0 ? t.lane - 1 : 0;  // edge lanes read themselves:
        t.src_p = t.lane < 63 ? t.lane + 1 : 63;  // their results are not used
        t.in_tile = t.lane >= kHalo && t.lane < 64 - kHalo && xu < t.H;
    }
    t.y0 = chunk_i * mb.chunk;
    t.L = min(mb.chunk, t.n - t.y0);
    const T *in = static_cast<const T *>(mb.in);
    T *out = static_cast<T *>(mb.out);
    const int64_t stride = mb.stride;
    const Coef k = mb.k;
    const bool first = mb.first != 0;

    Pipe<T, S> st;
    {
        const Vals<T> zero = {{T(0), T(0), T(0), T(0)}};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            st.R[i] = st.B[i] = zero;
#pragma unroll
            for (int j = 0; j < S - 1; ++j) st.F[j][i] = zero;
        }
        st.Bn = zero;
    }
    const int steps = t.L + 2 * S;
    int y_load = wrap(t.y0 - S, t.n);
    {
        const int64_t pt = static_cast<int64_t>(y_load) * t.H + t.xh;
        st.R[0] = load_vals(in, stride, RED, pt);
        st.Bn = load_vals(in, stride, BLUE, pt);
    }
    for (int p = 0; p < steps; p += 3) {
        step2d<T, S, 0>(st, t, in, out, stride, p, steps, y_load, first, k);
        if (p + 1 < steps) step2d<T, S, 1>(st, t, in, out, stride, p + 1, steps, y_load, first, k);
        if (p + 2 < steps) step2d<T, S, 2>(st, t, in, out, stride, p + 2, steps, y_load, first, k);
    }
}

template <typename T, int S>
hipError_t launch_typed(const Stream2dMember &one, const Stream2dMember *list, int nm,
                        int64_t total_tasks, hipStream_t s)
{
    const int64_t blocks = (total_tasks + kWaves - 1) / kWaves;
    hipLaunchKernelGGL((stream2d_kernel<T, S>), dim3(static_cast<unsigned>(blocks)),
                       dim3(64 * kWaves), 0, s, one, list, nm, total_tasks);
    return hipGetLastError();
}

}  // namespace

int stream2d_tiles_x(int n)
{
    const int H = n / 2;
    return H <= 64 ? 1 : (H + kTile - 1) / kTile;
}

int64_t stream2d_tasks(int n, int chunk)
{
    if (n < 2 || (n & 1) || chunk < 1) return 0;
    return static_cast<int64_t>(stream2d_tiles_x(n)) * ((n + chunk - 1) / chunk);
}

hipError_t launch_stream2d(int precision, int stages, const Stream2dMember &one,
                           const Stream2dMember *list, int nm, int64_t total_tasks, hipStream_t s)
{
    if ((stages != 2 && stages != 4) || nm < 1 || (!list && nm != 1) || total_tasks < 1 ||
        (total_tasks + kWaves - 1) / kWaves > 0x7fffffff)
        return hipErrorInvalidValue;
    if (!list && (one.in == nullptr || one.out == nullptr || one.in == one.out || one.n < 2 ||
                  (one.n & 1) || one.chunk < 1 || one.task_begin != 0 ||
                  one.tiles_x != stream2d_tiles_x(one.n) ||
                  total_tasks != stream2d_tasks(one.n, one.chunk)))
        return hipErrorInvalidValue;
    if (precision == 0)
        return stages == 2 ? launch_typed<double, 2>(one, list, nm, total_tasks, s)
                           : launch_typed<double, 4>(one, list, nm, total_tasks, s);
    return stages == 2 ? launch_typed<float, 2>(one, list, nm, total_tasks, s)
                       : launch_typed<float, 4>(one, list, nm, total_tasks, s);
}

}  // namespace kgs
