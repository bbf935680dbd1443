// 3-D z-streaming kernel: S consecutive colour sweeps (S/2 DP-AVF2 steps) in
// one launch, reading the state from one buffer and writing it to another.
//
// Why: one colour sweep per launch moves 88 bytes per point and step in
// float64 (own 4 fields read+written, the other colour's psi and u read
// again); one launch per S sweeps moves 64*2/S bytes.
//
// Work decomposition.  A workgroup owns an output tile of tile_y rows (axis
// 1) x tile_x compressed positions (axis 2, one red and one blue point per
// position) and a chunk of planes along axis 0 ("z"), and streams through the
// chunk plane by plane.  Each sweep widens the dependency cone by one point
// in every direction, so the workgroup loads and updates a halo of S rows and
// ceil(S/2) compressed positions around the tile (recomputing what the
// neighbouring tiles also compute) and S planes before and after the chunk.
// Only the tile is written.
//
// Pipeline.  At pipeline step p the workgroup loads plane l_p = z0 - S + p
// (level 0, both colours) and sweep stage j (colour j&1; level j+1) updates
// plane l_p - 1 - j.  Stage j therefore finds its z-neighbours (planes l_p - j
// and l_p - 2 - j of level j) in the registers of the same thread: a
// three-plane FIFO per level.  In-plane neighbours come from the other
// threads through LDS, published at the end of the previous step
// (double-buffered, one barrier per step).  The neighbour sums use the same
// order as the one-sweep kernel (axis 0 -, +, axis 1 -, +, axis 2 -, +), so
// both kernels give bitwise the same state.
#include <hip/hip_runtime.h>

#include "kgs_internal.h"
#include "kgs_point.h"

namespace kgs {
namespace {

template <typename T>
struct Vals {
    T f[4];  // P, Q, U, V
};

__device__ __forceinline__ int wrap(int v, int m)
{
    v %= m;
    return v < 0 ? v + m : v;
}

template <typename T>
__device__ __forceinline__ T rnd(double x)
{
    return static_cast<T>(x);  // rounding of a stored state value
}

// Largest workgroup per instantiation: the float64 four-sweep pipeline keeps
// about 60 doubles of FIFO per thread and needs more than 128 VGPRs.
template <typename T, int S>
constexpr int max_threads()
{
    return (S == 4 && sizeof(T) == 8) ? 512 : 1024;
}

template <typename T, int S, bool FIRST>
__global__ void __launch_bounds__((max_threads<T, S>()))
stream3d_kernel(const T *__restrict__ in, T *__restrict__ out, int64_t stride, int n,
                int tiles_x, int tiles_y, int tile_x, int tile_y, int chunk_len, Coef k)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);

    constexpr int HX = (S + 1) / 2;
    constexpr int HY = S;
    const int H = n >> 1;
    const int BX = tile_x + 2 * HX;
    const int BY = tile_y + 2 * HY;
    const int NT = BX * BY;
    const int tid = threadIdx.x;
    const bool live = tid < NT;
    const int ltx = live ? tid % BX : 0;
    const int lty = live ? tid / BX : 0;

    // work item: XCD-aware (consecutive items run on the same XCD)
    const int G = gridDim.x;
    int item = blockIdx.x;
    if ((G & 7) == 0) item = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
    const int ntiles = tiles_x * tiles_y;
    const int tile = item % ntiles;
    const int chunk = item / ntiles;
    const int x0 = (tile % tiles_x) * tile_x;
    const int y0 = (tile / tiles_x) * tile_y;
    const int z0 = chunk * chunk_len;
    const int L = min(chunk_len, n - z0);

    const int xu = x0 - HX + ltx;  // unwrapped compressed x of this thread
    const int yu = y0 - HY + lty;  // unwrapped row
    const int xh = wrap(xu, H);
    const int y = wrap(yu, n);
    const bool in_tile = live && ltx >= HX && ltx < HX + tile_x && lty >= HY &&
                         lty < HY + tile_y && xu < H && yu < n;
    // in-plane neighbour slots in the block (clamped: edge threads compute
    // values nobody valid depends on)
    const int i_self = lty * BX + ltx;
    const int i_ym = max(lty - 1, 0) * BX + ltx;
    const int i_yp = min(lty + 1, BY - 1) * BX + ltx;

    const int64_t plane_elems = static_cast<int64_t>(n) * H;
    const int64_t col = static_cast<int64_t>(y) * H + xh;  // offset inside a plane
    T *const out_c[2] = {out, out + 4 * stride};

    // FIFOs (slot 0 = produced at this step): level 0 red (2 slots), level 0
    // blue (3 slots), levels 1..S-1 (3 slots, colour of the producing stage)
    Vals<T> r0[2], b0[3], f[S - 1][3];
    Vals<T> pre_r[2], pre_b[2];  // input planes prefetched two steps ahead
    {
        const Vals<T> zero = {{T(0), T(0), T(0), T(0)}};
        r0[0] = r0[1] = b0[0] = b0[1] = b0[2] = zero;
        pre_r[0] = pre_r[1] = pre_b[0] = pre_b[1] = zero;
#pragma unroll
        for (int j = 0; j < S - 1; ++j) f[j][0] = f[j][1] = f[j][2] = zero;
    }

    auto load_plane = [&](int z, Vals<T> &rv, Vals<T> &bv) {
        const T *pr_ = in + static_cast<int64_t>(z) * plane_elems + col;
        const T *pb_ = pr_ + 4 * stride;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            rv.f[q] = pr_[q * stride];
            bv.f[q] = pb_[q * stride];
        }
    };

    const int steps = L + 2 * S;
    // planes are tracked wrapped and advanced by one per step
    int z_load = wrap(z0 - S, n);  // plane loaded (consumed) at step p
    int z_pf = z_load;             // next plane to prefetch
    if (live) load_plane(z_pf, pre_r[0], pre_b[0]);
    z_pf = z_pf + 1 == n ? 0 : z_pf + 1;
    if (live && steps > 1) load_plane(z_pf, pre_r[1], pre_b[1]);
    z_pf = z_pf + 1 == n ? 0 : z_pf + 1;

    for (int p = 0; p < steps; ++p) {
        const int rb = (p - 1) & 1, wb = p & 1;
        // shift the level-0 FIFO and take the plane prefetched two steps ago
        r0[1] = r0[0];
        b0[2] = b0[1];
        b0[1] = b0[0];
        r0[0] = pre_r[0];
        b0[0] = pre_b[0];
        pre_r[0] = pre_r[1];
        pre_b[0] = pre_b[1];
        if (live && p + 2 < steps) load_plane(z_pf, pre_r[1], pre_b[1]);
        z_pf = z_pf + 1 == n ? 0 : z_pf + 1;

#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (p < 2 * j + 2) continue;  // pipeline not yet filled for stage j
            const int c = j & 1;
            int z = z_load - 1 - j;  // plane updated by stage j (wrapped)
            while (z < 0) z += n;
            const int o = (z + y + c) & 1;  // x-offset of colour c in this row
            const int i_xm = lty * BX + max(ltx - 1 + o, 0);
            const int i_xp = lty * BX + min(ltx + o, BX - 1);
            // level-j neighbours: z +/- 1 from registers, in-plane from LDS
            const Vals<T> *upp = (j == 0) ? &b0[0] : &f[max(j - 1, 0)][0];
            const Vals<T> *dnp = (j == 0) ? &b0[2] : &f[max(j - 1, 0)][2];
            const T *pub = lds + (static_cast<size_t>(rb) * S + j) * 3 * NT;
            double sum[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const T *pl = pub + q * NT;
                double a = static_cast<double>(dnp->f[q]);
                a = a + static_cast<double>(upp->f[q]);
                a = a + static_cast<double>(pl[i_ym]);
                a = a + static_cast<double>(pl[i_yp]);
                a = a + static_cast<double>(pl[i_xm]);
                a = a + static_cast<double>(pl[i_xp]);
                sum[q] = a;
            }
            // own values at level j
            const Vals<T> &own = (j == 0) ? r0[1] : (j == 1) ? b0[2] : f[max(j - 2, 0)][2];
            double pr = own.f[0], pi = own.f[1], u = own.f[2], v = own.f[3];
            if (c == RED) {
                if (FIRST && j == 0)
                    sweep_point<PASS_R_BASE, T>(k, pr, pi, u, v, sum[0], sum[1], sum[2]);
                else
                    sweep_point<PASS_R_ADJ_BASE, T>(k, pr, pi, u, v, sum[0], sum[1], sum[2]);
            } else {
                sweep_point<PASS_B_FULL, T>(k, pr, pi, u, v, sum[0], sum[1], sum[2]);
            }
            Vals<T> res;
            res.f[0] = rnd<T>(pr);
            res.f[1] = rnd<T>(pi);
            res.f[2] = rnd<T>(u);
            res.f[3] = rnd<T>(v);
            if (j < S - 1) {
                f[j][2] = f[j][1];
                f[j][1] = f[j][0];
                f[j][0] = res;
            } else if (in_tile) {
                // final level S at plane z: colour c from this stage, the
                // other colour from stage S-2 one step ago
                const Vals<T> &oth = f[S - 2][1];
                T *oc = out_c[c] + static_cast<int64_t>(z) * plane_elems + col;
                T *oo = out_c[c ^ 1] + static_cast<int64_t>(z) * plane_elems + col;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    oc[q * stride] = res.f[q];
                    oo[q * stride] = oth.f[q];
                }
            }
        }
        z_load = z_load + 1 == n ? 0 : z_load + 1;
        // publish the newest plane of every level that a stage reads next step
        if (live) {
            T *pw = lds + static_cast<size_t>(wb) * S * 3 * NT;
#pragma unroll
            for (int q = 0; q < 3; ++q) pw[q * NT + i_self] = b0[0].f[q];
#pragma unroll
            for (int j = 1; j < S; ++j) {
#pragma unroll
                for (int q = 0; q < 3; ++q) pw[(j * 3 + q) * NT + i_self] = f[j - 1][0].f[q];
            }
        }
        __syncthreads();
    }
}

template <typename T, int S>
hipError_t launch_typed(const Geometry &g, const StreamShape &sh, const T *in, T *out, bool first,
                        const Coef &k, hipStream_t s)
{
    const int HX = (S + 1) / 2, HY = S;
    const int H = g.n / 2;
    const int BX = sh.tile_x + 2 * HX, BY = sh.tile_y + 2 * HY;
    const int NT = BX * BY;
    const int threads = (NT + 63) / 64 * 64;
    const int tiles_x = (H + sh.tile_x - 1) / sh.tile_x;
    const int tiles_y = (g.n + sh.tile_y - 1) / sh.tile_y;
    const int chunks = (g.n + sh.chunk - 1) / sh.chunk;
    const int64_t items = static_cast<int64_t>(tiles_x) * tiles_y * chunks;
    const size_t lds = static_cast<size_t>(2) * S * 3 * NT * sizeof(T);
    if (threads > max_threads<T, S>() || items > 0x7fffffff || lds > 160 * 1024)
        return hipErrorInvalidValue;
    auto kern = first ? stream3d_kernel<T, S, true> : stream3d_kernel<T, S, false>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(items)), dim3(threads), lds, s, in, out,
                       g.stride, g.n, tiles_x, tiles_y, sh.tile_x, sh.tile_y, sh.chunk, k);
    return hipGetLastError();
}

}  // namespace

bool stream3d_shape_ok(const Geometry &g, const StreamShape &sh, int elem_bytes)
{
    if (g.dim != 3 || g.n < 2 || (g.n & 1) || g.count != static_cast<int64_t>(g.n) * g.n * (g.n / 2))
        return false;
    if (sh.steps != 1 && sh.steps != 2) return false;
    if (sh.tile_x < 1 || sh.tile_y < 1 || sh.chunk < 1) return false;
    const int S = 2 * sh.steps;
    const int BX = sh.tile_x + 2 * ((S + 1) / 2), BY = sh.tile_y + 2 * S;
    const int NT = BX * BY;
    const int limit = (S == 4 && elem_bytes == 8) ? 512 : 1024;
    if ((NT + 63) / 64 * 64 > limit) return false;
    return static_cast<size_t>(2) * S * 3 * NT * elem_bytes <= 160 * 1024;
}

hipError_t launch_stream3d(const Geometry &g, int precision, const StreamShape &sh, int stages,
                           const void *in, void *out, bool first, const Coef &k, hipStream_t s)
{
    const int eb = precision == 0 ? 8 : 4;
    StreamShape sh2 = sh;
    sh2.steps = stages / 2;
    if (!in || !out || in == out || (stages != 2 && stages != 4) || !stream3d_shape_ok(g, sh2, eb))
        return hipErrorInvalidValue;
    if (precision == 0) {
        if (stages == 2)
            return launch_typed<double, 2>(g, sh, static_cast<const double *>(in),
                                           static_cast<double *>(out), first, k, s);
        return launch_typed<double, 4>(g, sh, static_cast<const double *>(in),
                                       static_cast<double *>(out), first, k, s);
    }
    if (stages == 2)
        return launch_typed<float, 2>(g, sh, static_cast<const float *>(in),
                                      static_cast<float *>(out), first, k, s);
    return launch_typed<float, 4>(g, sh, static_cast<const float *>(in), static_cast<float *>(out),
                                  first, k, s);
}

}  // namespace kgs
