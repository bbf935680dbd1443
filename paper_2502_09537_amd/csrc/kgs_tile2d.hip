// 2-D tiled kernel: S = 2, 4 or 8 consecutive colour sweeps (S/2 DP-AVF2
// steps) of a 2-D grid in one launch, each workgroup holding one tile of the
// grid plus a halo in LDS, reading the state from one buffer and writing it
// to another.
//
// Why: a 2-D grid of moderate size (1024^2 is 0.5 M points per colour) has
// too few rows for the y-streaming kernel to give every SIMD more than about
// one wave, and a streaming task spends 2S pipeline steps filling and
// draining.  Here a workgroup loads a block of TY + 2S rows by TXC + 2*HX
// compressed positions of both colours (HX = ceil(S/2): each sweep reaches
// one point further along every axis, half a compressed position along x),
// runs the S sweeps in LDS with one barrier after each, and writes the TY x
// TXC interior.  Neighbours outside the block are replaced by the nearest
// block position; the values this spoils stay in the halo, which is never
// written.  Sweep j runs only on the positions that a later sweep still
// needs: the interior grown by S-1-j rows and ceil((S-1-j)/2) compressed
// positions.
//
// P, Q and U of both colours live in LDS (the neighbours read them); u_t of
// the points a thread owns stays in its registers.  The neighbour sums use
// the order of the one-sweep kernel (axis 0 -, +, x -, +) and values are
// rounded to the storage type at the same places, so the state is bitwise
// that of every other kernel.
#include <hip/hip_runtime.h>

#include "kgs_internal.h"
#include "kgs_layout.h"
#include "kgs_point.h"

namespace kgs {
namespace {

// Threads per workgroup (NT): 256 for blocks (tile plus halo) of up to
// 1024 points, 512 with 4 points each for larger blocks up to kMaxBlock.
// The 16 x 32 float64 tile with the halo of 8 sweeps is a 1280-point
// block: 512 threads run it 1.16 times as fast as 256 threads with 8 points
// each (2-D 1024^2 on MI355X).
constexpr int kMaxBlock = 2048;

__device__ __forceinline__ int wrap(int v, int m)
{
    v %= m;
    return v < 0 ? v + m : v;
}

// The positions p = threadIdx.x + j NT (j < PPT) a thread owns.
template <typename T, int PPT>
struct Owned {
    T v[2][PPT];        // u_t [colour][point]
    int ly[PPT], lx[PPT];
    int ym[PPT], yp[PPT];      // block positions one row down / up
    int xm[PPT][2], xp[PPT][2];  // other-colour x neighbours [point][colour]
};

template <typename T, int NT, int PPT, int KIND, int COLOUR>
__device__ __forceinline__ void tile_sweep(T *lds, int NB, const Coef &k, Owned<T, PPT> &w,
                                           int y_lo, int y_hi, int x_lo, int x_hi)
{
    const T *op = lds + 3 * (COLOUR ^ 1) * NB, *oq = op + NB, *ou = oq + NB;
    T *mp = lds + 3 * COLOUR * NB, *mq = mp + NB, *mu = mq + NB;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int p = threadIdx.x + j * NT;
        if (p >= NB || w.ly[j] < y_lo || w.ly[j] >= y_hi || w.lx[j] < x_lo || w.lx[j] >= x_hi)
            continue;
        const int a0 = w.ym[j], a1 = w.yp[j], a2 = w.xm[j][COLOUR], a3 = w.xp[j][COLOUR];
        double sr = static_cast<double>(op[a0]);
        sr = sr + static_cast<double>(op[a1]);
        sr = sr + static_cast<double>(op[a2]);
        sr = sr + static_cast<double>(op[a3]);
        double si = static_cast<double>(oq[a0]);
        si = si + static_cast<double>(oq[a1]);
        si = si + static_cast<double>(oq[a2]);
        si = si + static_cast<double>(oq[a3]);
        double su = static_cast<double>(ou[a0]);
        su = su + static_cast<double>(ou[a1]);
        su = su + static_cast<double>(ou[a2]);
        su = su + static_cast<double>(ou[a3]);
        double pr = static_cast<double>(mp[p]);
        double pi = static_cast<double>(mq[p]);
        double u = static_cast<double>(mu[p]);
        double v = static_cast<double>(w.v[COLOUR][j]);
        sweep_point<KIND, T>(k, pr, pi, u, v, sr, si, su);
        mp[p] = static_cast<T>(pr);
        mq[p] = static_cast<T>(pi);
        mu[p] = static_cast<T>(u);
        w.v[COLOUR][j] = static_cast<T>(v);
    }
}

// Workgroup b runs tile b - task_begin of the member whose task_begin is the
// largest one <= b (the member `one` when list is null); the member
// descriptor gives its buffers, constants, n and tiles per row.  FIRST: this
// launch starts every member's run (the first red sweep is the base pass).
template <typename T, int S, int NT, int PPT, bool FIRST>
__global__ void __launch_bounds__(NT)
tile2d_kernel(Stream2dMember one, const Stream2dMember *__restrict__ list, int nm, int ty,
              int txc)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);
    constexpr int HY = S, HX = (S + 1) / 2;
    const int64_t task = blockIdx.x;
    Stream2dMember mb = one;  // a copy: uniform values stay in scalar registers
    if (list) {
        int lo = 0, hi = nm - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (list[mid].task_begin <= task) lo = mid;
            else hi = mid - 1;
        }
        mb = list[lo];
    }
    const T *__restrict__ in = static_cast<const T *>(mb.in);
    T *__restrict__ out = static_cast<T *>(mb.out);
    const int64_t stride = mb.stride;
    const int n = mb.n, tiles_x = mb.tiles_x;
    const Coef k = mb.k;
    const int H = n >> 1;
    const int BY = ty + 2 * HY, BX = txc + 2 * HX, NB = BY * BX;
    const int tile = static_cast<int>(task - mb.task_begin);
    const int x0 = (tile % tiles_x) * txc, y0 = (tile / tiles_x) * ty;

    Owned<T, PPT> w;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int p = threadIdx.x + j * NT;
        const int q = p < NB ? p : 0;
        const int ly = q / BX, lx = q - (q / BX) * BX;
        w.ly[j] = ly;
        w.lx[j] = lx;
        w.ym[j] = (ly > 0 ? ly - 1 : 0) * BX + lx;
        w.yp[j] = (ly < BY - 1 ? ly + 1 : BY - 1) * BX + lx;
        // the block starts at an even point x, so a block-local position
        // has the parity of its global one; a row's colour offset follows
        // the parity of its global row index
        const int yu = y0 - HY + ly;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int o = (yu + 3 + c) & 1;
            const int xm = lx - 1 + o, xp = lx + o;
            w.xm[j][c] = ly * BX + (xm > 0 ? xm : 0);
            w.xp[j][c] = ly * BX + (xp < BX - 1 ? xp : BX - 1);
        }
        w.v[0][j] = w.v[1][j] = T(0);
        if (p < NB) {
            const int64_t pt = static_cast<int64_t>(wrap(yu, n)) * H + wrap(x0 - HX + lx, H);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const Pair<T> pq = ld_pair(pair_plane(in, stride, c, PAIR_PQ), pt);
                const Pair<T> uv = ld_pair(pair_plane(in, stride, c, PAIR_UV), pt);
                lds[(3 * c) * NB + p] = pq.x;
                lds[(3 * c + 1) * NB + p] = pq.y;
                lds[(3 * c + 2) * NB + p] = uv.x;
                w.v[c][j] = uv.y;
            }
        }
    }
    __syncthreads();
    // sweep j updates the interior grown by m = S-1-j rows and ceil(m/2)
    // compressed positions
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int m = S - 1 - j, mx = (m + 1) / 2;
        const int y_lo = HY - m, y_hi = HY + ty + m, x_lo = HX - mx, x_hi = HX + txc + mx;
        if (j & 1) {
            tile_sweep<T, NT, PPT, PASS_B_FULL, BLUE>(lds, NB, k, w, y_lo, y_hi, x_lo, x_hi);
        } else if (FIRST && j == 0) {
            tile_sweep<T, NT, PPT, PASS_R_BASE, RED>(lds, NB, k, w, y_lo, y_hi, x_lo, x_hi);
        } else {
            tile_sweep<T, NT, PPT, PASS_R_ADJ_BASE, RED>(lds, NB, k, w, y_lo, y_hi, x_lo, x_hi);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int p = threadIdx.x + j * NT;
        const int ly = w.ly[j], lx = w.lx[j];
        const int yu = y0 - HY + ly, xu = x0 - HX + lx;
        if (p >= NB || ly < HY || ly >= HY + ty || lx < HX || lx >= HX + txc || yu >= n || xu >= H)
            continue;
        const int64_t pt = static_cast<int64_t>(yu) * H + xu;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            st_pair(pair_plane(out, stride, c, PAIR_PQ), pt, lds[(3 * c) * NB + p],
                    lds[(3 * c + 1) * NB + p]);
            st_pair(pair_plane(out, stride, c, PAIR_UV), pt, lds[(3 * c + 2) * NB + p], w.v[c][j]);
        }
    }
}

template <typename T, int S, int NT, int PPT>
hipError_t launch_ppt(int ty, int txc, bool first, const Stream2dMember &one,
                      const Stream2dMember *list, int nm, int64_t tiles, hipStream_t s)
{
    constexpr int HY = S, HX = (S + 1) / 2;
    const int NB = (ty + 2 * HY) * (txc + 2 * HX);
    const size_t lds = static_cast<size_t>(6) * NB * sizeof(T);
    auto kern = first ? tile2d_kernel<T, S, NT, PPT, true> : tile2d_kernel<T, S, NT, PPT, false>;
    hipError_t e = allow_dynamic_lds(reinterpret_cast<const void *>(kern), static_cast<int>(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(tiles)), dim3(NT), lds, s, one, list,
                       nm, ty, txc);
    return hipGetLastError();
}

template <typename T, int S>
hipError_t launch_typed(int ty, int txc, bool first, const Stream2dMember &one,
                        const Stream2dMember *list, int nm, int64_t tiles, hipStream_t s)
{
    const int NB = (ty + 2 * S) * (txc + 2 * ((S + 1) / 2));
    if (NB <= 2 * 256) return launch_ppt<T, S, 256, 2>(ty, txc, first, one, list, nm, tiles, s);
    if (NB <= 4 * 256) return launch_ppt<T, S, 256, 4>(ty, txc, first, one, list, nm, tiles, s);
    return launch_ppt<T, S, 512, 4>(ty, txc, first, one, list, nm, tiles, s);  // NB <= kMaxBlock
}

bool block_fits(int ty, int txc, int stages, int elem_bytes)
{
    if ((stages != 2 && stages != 4 && stages != 8) || ty < 1 || txc < 1 || ty > 4096 || txc > 4096)
        return false;
    const int NB = (ty + 2 * stages) * (txc + 2 * ((stages + 1) / 2));
    return NB <= kMaxBlock && static_cast<size_t>(6) * NB * elem_bytes <= 160 * 1024;
}

}  // namespace

int tile2d_tiles_x(int n, int txc) { return txc < 1 ? 0 : (n / 2 + txc - 1) / txc; }

int64_t tile2d_member_tiles(int n, int ty, int txc)
{
    if (n < 2 || (n & 1) || ty < 1 || txc < 1) return 0;
    return static_cast<int64_t>(tile2d_tiles_x(n, txc)) * ((n + ty - 1) / ty);
}

int64_t tile2d_tiles(const Geometry &g, int ty, int txc) { return tile2d_member_tiles(g.n, ty, txc); }

void tile2d_group_shape(const int *n, int count, int &ty, int &txc)
{
    // the largest tile that still gives about four workgroups per CU of
    // MI355X (larger tiles recompute less halo)
    static const int shapes[][2] = {{16, 32}, {16, 16}, {8, 16}, {8, 8}};
    for (const auto &sh : shapes) {
        int64_t tiles = 0;
        for (int i = 0; i < count; ++i) tiles += tile2d_member_tiles(n[i], sh[0], sh[1]);
        ty = sh[0];
        txc = sh[1];
        if (tiles >= 1024) return;
    }
}

bool tile2d_shape_ok(const Geometry &g, int ty, int txc, int stages, int elem_bytes)
{
    if (g.dim != 2 || g.n < 2 || (g.n & 1) || g.count != static_cast<int64_t>(g.n) * (g.n / 2))
        return false;
    return block_fits(ty, txc, stages, elem_bytes) && tile2d_tiles(g, ty, txc) <= 0x7fffffff;
}

hipError_t launch_tile2d(const Geometry &g, int precision, int stages, int ty, int txc,
                         const void *in, void *out, bool first, const Coef &k, hipStream_t s)
{
    const int eb = precision == 0 ? 8 : 4;
    if (!in || !out || in == out || !tile2d_shape_ok(g, ty, txc, stages, eb))
        return hipErrorInvalidValue;
    Stream2dMember m;
    m.in = in;
    m.out = out;
    m.stride = g.stride;
    m.task_begin = 0;
    m.k = k;
    m.n = g.n;
    m.chunk = ty;
    m.tiles_x = tile2d_tiles_x(g.n, txc);
    m.first = first ? 1 : 0;
    return launch_tile2d_list(precision, stages, ty, txc, m, nullptr, 1, tile2d_tiles(g, ty, txc),
                              s);
}

hipError_t launch_tile2d_list(int precision, int stages, int ty, int txc, const Stream2dMember &one,
                              const Stream2dMember *list, int nm, int64_t total_tiles,
                              hipStream_t s, int first_launch)
{
    // every member of a launch is at the same point of its run: the first
    // launch of a run (the descriptors' `first`) is a template choice
    const bool first = list ? first_launch != 0 : one.first != 0;
    const int eb = precision == 0 ? 8 : 4;
    if (!block_fits(ty, txc, stages, eb) || nm < 1 || (!list && nm != 1) || total_tiles < 1 ||
        total_tiles > 0x7fffffff)
        return hipErrorInvalidValue;
    if (!list && (one.in == nullptr || one.out == nullptr || one.in == one.out || one.n < 2 ||
                  (one.n & 1) || one.task_begin != 0 || one.tiles_x != tile2d_tiles_x(one.n, txc) ||
                  total_tiles != tile2d_member_tiles(one.n, ty, txc)))
        return hipErrorInvalidValue;
    if (precision == 0)
        return stages == 2   ? launch_typed<double, 2>(ty, txc, first, one, list, nm, total_tiles, s)
               : stages == 4 ? launch_typed<double, 4>(ty, txc, first, one, list, nm, total_tiles, s)
                             : launch_typed<double, 8>(ty, txc, first, one, list, nm, total_tiles, s);
    return stages == 2   ? launch_typed<float, 2>(ty, txc, first, one, list, nm, total_tiles, s)
           : stages == 4 ? launch_typed<float, 4>(ty, txc, first, one, list, nm, total_tiles, s)
                         : launch_typed<float, 8>(ty, txc, first, one, list, nm, total_tiles, s);
}

}  // namespace kgs
