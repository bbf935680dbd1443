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
// (double-buffered, one barrier per step) as (P, Q) pairs and U, so that a
// neighbour costs two LDS reads.  The neighbour sums use the same
// order as the one-sweep kernel (axis 0 -, +, axis 1 -, +, axis 2 -, +), so
// both kernels give bitwise the same state.
#include <hip/hip_runtime.h>

#include "kgs_internal.h"
#include "kgs_layout.h"
#include "kgs_point.h"

namespace kgs {
namespace {

template <typename T>
struct Vals {
    T f[4];  // P, Q, U, V
};

// Element at a uniform plane pointer plus a per-thread 32-bit byte offset
// (the scalar-base + vector-offset addressing of global memory).
template <typename T>
__device__ __forceinline__ T *at(T *base, uint32_t byte_offset)
{
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_offset);
}

template <typename T>
__device__ __forceinline__ const T *at(const T *base, uint32_t byte_offset)
{
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_offset);
}

// The four values of a column of colour c in the z-plane whose pair planes
// start at zb2 (uniform), at byte offset colb2 inside each pair plane: two
// pair loads.
template <typename T>
__device__ __forceinline__ Vals<T> load_col(const T *zb2, int64_t stride, int c, uint32_t colb2)
{
    const Pair<T> pq = *(const Global<Pair<T>> *)(at(pair_plane(zb2, stride, c, PAIR_PQ), colb2));
    const Pair<T> uv = *(const Global<Pair<T>> *)(at(pair_plane(zb2, stride, c, PAIR_UV), colb2));
    return Vals<T>{{pq.x, pq.y, uv.x, uv.y}};
}

// Streaming stores: the next launch reads them back, this one never does,
// so they need not occupy L2.  Both helpers address global memory
// explicitly: state pointers read from member descriptors carry no address
// space of their own.
template <typename T>
__device__ __forceinline__ void store_col(T *zb2, int64_t stride, int c, uint32_t colb2,
                                          const Vals<T> &x)
{
    Pair<T> pq, uv;
    pq.x = x.f[0];
    pq.y = x.f[1];
    uv.x = x.f[2];
    uv.y = x.f[3];
    __builtin_nontemporal_store(pq, (Global<Pair<T>> *)(at(pair_plane(zb2, stride, c, PAIR_PQ), colb2)));
    __builtin_nontemporal_store(uv, (Global<Pair<T>> *)(at(pair_plane(zb2, stride, c, PAIR_UV), colb2)));
}

__device__ __forceinline__ int wrap(int v, int m)
{
    v %= m;
    return v < 0 ? v + m : v;
}

// Row pitch of a published plane in LDS: the block width made odd, so that
// a column of the block (rows one pitch apart), which the ring threads
// read, falls in distinct banks.
__host__ __device__ constexpr int lds_pitch(int bx) { return bx | 1; }

// Slots of one published plane, even so that every (P, Q) pair array starts
// on a pair boundary.  A level's publication is NL (P, Q) pairs followed by
// NL values of U.
__host__ __device__ constexpr int lds_plane(int bx, int by) { return (lds_pitch(bx) * by + 1) & ~1; }

// Largest workgroup per instantiation: the four-sweep float64 pipeline
// keeps 16 planes of FIFO per thread (128 VGPRs) and needs more, so at most
// 3 waves per SIMD (12 per workgroup); in float32 the same FIFO takes 64
// VGPRs and the kernel fits 128, so 16 waves.  A compiled-in tile has
// exactly its block of threads.
template <typename T, int S, int TX = 0, int TY = 0>
constexpr int max_threads()
{
    return TX ? ((TX + 2 * ((S + 1) / 2)) * (TY + 2 * S) + 63) / 64 * 64
              : S == 4 && sizeof(T) == 8 ? 768 : 1024;
}

// Per-thread pipeline registers.  Plane FIFOs are rings indexed by the
// pipeline step modulo 3, so that with the step loop unrolled three times
// every slot is a fixed register and no value is moved between slots:
//   R[q % 3]     red level 0, plane loaded at step q (own values of stage 0)
//   B[q % 3]     blue level 0, plane loaded at step q
//   F[j][q % 3]  output of stage j (level j + 1) produced at step q
// Bn holds the blue plane of the next step while B still needs all three
// slots.
template <typename T, int S>
struct Pipe {
    Vals<T> R[3], B[3], Bn, F[S - 1][3];
};

// Thread geometry shared by all steps of a workgroup.
struct Geo {
    int NT;              // threads with a column of the block
    int NL;              // LDS slots per published plane (odd row pitch, even total)
    int wave;            // first thread of this thread's wave
    int need[5];         // stage j runs on threads below need[S - 1 - j]
    bool live, in_tile;  // has a column / writes its column
    int y;               // wrapped row of the column
    uint32_t colb2;      // byte offset of the column inside a z-plane of a pair plane (< 2^31)
    int i_self, i_ym, i_yp;
    int i_xm0, i_xm1, i_xp0, i_xp1;  // x-neighbour slots for x-offset o = 0, 1
};

// Threads are ordered by concentric rings around the output tile, so that
// the columns each sweep stage needs are the first threads of the
// workgroup and whole waves can skip a stage.  R(m) is the tile grown by m
// rows and ceil(m/2) compressed positions on every side: the columns a
// stage with m sweeps still to follow must update (each sweep reaches one
// point further along every axis, i.e. half a compressed position in x).
// R(S) is the whole block.  Ring m = R(m) minus R(m-1) is enumerated as its
// top row, bottom row, left column, right column.
__device__ __forceinline__ int ring_x(int m) { return (m + 1) >> 1; }

template <int S>
__device__ __forceinline__ int ring_area(int m, int tile_x, int tile_y)
{
    return (tile_x + 2 * ring_x(m)) * (tile_y + 2 * m);
}

template <int S>
__device__ __forceinline__ void ring_position(int tid, int tile_x, int tile_y, int &ltx, int &lty)
{
    constexpr int HX = (S + 1) / 2, HY = S;
    if (tid < tile_x * tile_y) {
        ltx = HX + tid % tile_x;
        lty = HY + tid / tile_x;
        return;
    }
    int m = 1;
    while (m < S && tid >= ring_area<S>(m, tile_x, tile_y)) ++m;
    int k = tid - ring_area<S>(m - 1, tile_x, tile_y);
    const int wm = tile_x + 2 * ring_x(m), x0m = HX - ring_x(m), y0m = HY - m;
    const int hm = tile_y + 2 * m;
    const int wp = tile_x + 2 * ring_x(m - 1), x0p = HX - ring_x(m - 1), y0p = HY - (m - 1);
    const int hp = tile_y + 2 * (m - 1);
    const int lw = x0p - x0m;  // 0 or 1
    if (k < wm) {
        ltx = x0m + k;
        lty = y0m;
    } else if ((k -= wm) < wm) {
        ltx = x0m + k;
        lty = y0m + hm - 1;
    } else if ((k -= wm) < hp * lw) {
        ltx = x0m;
        lty = y0p + k;
    } else {
        k -= hp * lw;
        ltx = x0p + wp;
        lty = y0p + k;
    }
}

template <typename T, int S, bool FIRST, int TX, int TY, int PH>
__device__ __forceinline__ void pipeline_step(Pipe<T, S> &st, const Geo &g, T *lds,
                                              const T *__restrict__ in, T *__restrict__ out,
                                              int64_t stride, int64_t plane_elems, int n, int p,
                                              int steps, int &z_load, const Coef &k)
{
    constexpr int HX = (S + 1) / 2, HY = S;
    const int NL = TX ? lds_plane(TX + 2 * HX, TY + 2 * HY) : g.NL;
    constexpr int s0 = PH % 3, s1 = (PH + 2) % 3, s2 = (PH + 1) % 3;  // steps p, p-1, p-2
    // the blue plane of step p arrived in Bn; fetch step p + 1 (red plane
    // into the slot of step p - 2, which no stage reads any more)
    st.B[s0] = st.Bn;
    if (g.live && p + 1 < steps) {
        const int zn = z_load + 1 == n ? 0 : z_load + 1;
        const T *zb2 = in + 2 * static_cast<int64_t>(zn) * plane_elems;  // uniform
        st.R[s2] = load_col(zb2, stride, RED, g.colb2);
        st.Bn = load_col(zb2, stride, BLUE, g.colb2);
    }
    // x-offset of the updated colour in this row: the same for every stage
    // of the step (the plane moves back by one when the colour flips)
    const int o = (z_load + g.y + 1) & 1;
    const int i_xm = o ? g.i_xm1 : g.i_xm0, i_xp = o ? g.i_xp1 : g.i_xp0;
    const T *pub = lds + static_cast<size_t>((p - 1) & 1) * S * 3 * NL;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        if (p < 2 * j + 2) continue;  // pipeline not yet filled for stage j
        if (g.wave >= g.need[S - 1 - j]) continue;  // no column of this wave is needed
        const int c = j & 1;
        // level-j neighbours: z -/+ 1 from registers, in-plane from LDS
        const Vals<T> &up = (j == 0) ? st.B[s0] : st.F[j > 0 ? j - 1 : 0][s0];
        const Vals<T> &dn = (j == 0) ? st.B[s2] : st.F[j > 0 ? j - 1 : 0][s2];
        // level-j publication: (P, Q) pairs, then U
        const Pair<T> *ppq = reinterpret_cast<const Pair<T> *>(pub + j * 3 * NL);
        const T *pu = pub + j * 3 * NL + 2 * NL;
        double sum[3];
        {
            const Pair<T> n0 = ppq[g.i_ym], n1 = ppq[g.i_yp], n2 = ppq[i_xm], n3 = ppq[i_xp];
            double a = static_cast<double>(dn.f[0]);
            a = a + static_cast<double>(up.f[0]);
            a = a + static_cast<double>(n0.x);
            a = a + static_cast<double>(n1.x);
            a = a + static_cast<double>(n2.x);
            a = a + static_cast<double>(n3.x);
            sum[0] = a;
            double b = static_cast<double>(dn.f[1]);
            b = b + static_cast<double>(up.f[1]);
            b = b + static_cast<double>(n0.y);
            b = b + static_cast<double>(n1.y);
            b = b + static_cast<double>(n2.y);
            b = b + static_cast<double>(n3.y);
            sum[1] = b;
            double c = static_cast<double>(dn.f[2]);
            c = c + static_cast<double>(up.f[2]);
            c = c + static_cast<double>(pu[g.i_ym]);
            c = c + static_cast<double>(pu[g.i_yp]);
            c = c + static_cast<double>(pu[i_xm]);
            c = c + static_cast<double>(pu[i_xp]);
            sum[2] = c;
        }
        // own values at level j: the last output of this colour
        const Vals<T> &own = (j == 0) ? st.R[s1] : (j == 1) ? st.B[s2] : st.F[j > 1 ? j - 2 : 0][s2];
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
        res.f[0] = static_cast<T>(pr);
        res.f[1] = static_cast<T>(pi);
        res.f[2] = static_cast<T>(u);
        res.f[3] = static_cast<T>(v);
        if (j < S - 1) {
            st.F[j < S - 1 ? j : 0][s0] = res;
        } else if (g.in_tile) {
            // final level S at plane z: colour c from this stage, the other
            // colour from stage S-2 one step ago
            const int z = wrap(z_load - S, n);  // n may be smaller than S
            T *zo2 = out + 2 * static_cast<int64_t>(z) * plane_elems;  // uniform
            store_col(zo2, stride, c, g.colb2, res);
            store_col(zo2, stride, c ^ 1, g.colb2, st.F[S - 2][s1]);
        }
    }
    z_load = z_load + 1 == n ? 0 : z_load + 1;
    // publish the newest plane of every level that a stage reads next step
    if (g.live) {
        T *pw = lds + static_cast<size_t>(p & 1) * S * 3 * NL;
        auto publish = [&](int j, const Vals<T> &x) {
            Pair<T> pq;
            pq.x = x.f[0];
            pq.y = x.f[1];
            reinterpret_cast<Pair<T> *>(pw + j * 3 * NL)[g.i_self] = pq;
            pw[j * 3 * NL + 2 * NL + g.i_self] = x.f[2];
        };
        publish(0, st.B[s0]);
#pragma unroll
        for (int j = 1; j < S; ++j) publish(j, st.F[j - 1][s0]);
    }
    __syncthreads();
}

// TX, TY > 0: tile shape fixed at compile time (LDS offsets become
// immediates); 0: taken from the arguments.
// One work item (a tile of the grid and a chunk of its z-planes) of a
// launch; `item` counts the tiles first, then the chunks.
template <typename T, int S, bool FIRST, int TX, int TY>
__device__ __forceinline__ void stream3d_item(const T *__restrict__ in, T *__restrict__ out,
                                              int64_t stride, int n, int tiles_x, int tiles_y,
                                              int tile_x_arg, int tile_y_arg, int chunk_len,
                                              int item, const Coef &k)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);

    constexpr int HX = (S + 1) / 2;
    constexpr int HY = S;
    const int tile_x = TX ? TX : tile_x_arg;
    const int tile_y = TY ? TY : tile_y_arg;
    const int H = n >> 1;
    const int BX = tile_x + 2 * HX;
    const int BY = tile_y + 2 * HY;
    const int PX = lds_pitch(BX);
    Geo g;
    g.NT = BX * BY;
    g.NL = lds_plane(BX, BY);
    const int tid = threadIdx.x;
    g.live = tid < g.NT;
    g.wave = tid & ~63;
#pragma unroll
    for (int m = 0; m < S; ++m) g.need[m] = ring_area<S>(m, tile_x, tile_y);
    int ltx = 0, lty = 0;
    if (g.live) ring_position<S>(tid, tile_x, tile_y, ltx, lty);

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
    g.y = wrap(yu, n);
    g.in_tile = g.live && ltx >= HX && ltx < HX + tile_x && lty >= HY && lty < HY + tile_y &&
                xu < H && yu < n;
    // in-plane neighbour slots in the block (clamped: edge threads compute
    // values nobody valid depends on)
    g.i_self = lty * PX + ltx;
    g.i_ym = max(lty - 1, 0) * PX + ltx;
    g.i_yp = min(lty + 1, BY - 1) * PX + ltx;
    g.i_xm0 = lty * PX + max(ltx - 1, 0);
    g.i_xm1 = g.i_self;
    g.i_xp0 = g.i_self;
    g.i_xp1 = lty * PX + min(ltx + 1, BX - 1);

    const int64_t plane_elems = static_cast<int64_t>(n) * H;
    g.colb2 = static_cast<uint32_t>(g.y * H + xh) * static_cast<uint32_t>(2 * sizeof(T));

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
    const int steps = L + 2 * S;
    int z_load = wrap(z0 - S, n);  // plane loaded (consumed) at step p
    // the first plane: red into the slot of step 0, blue into Bn
    if (g.live) {
        const T *zb2 = in + 2 * static_cast<int64_t>(z_load) * plane_elems;
        st.R[0] = load_col(zb2, stride, RED, g.colb2);
        st.Bn = load_col(zb2, stride, BLUE, g.colb2);
    }
    const int64_t pe = plane_elems;
    for (int p = 0; p < steps; p += 3) {
        pipeline_step<T, S, FIRST, TX, TY, 0>(st, g, lds, in, out, stride, pe, n, p, steps, z_load, k);
        if (p + 1 < steps)
            pipeline_step<T, S, FIRST, TX, TY, 1>(st, g, lds, in, out, stride, pe, n, p + 1, steps,
                                                  z_load, k);
        if (p + 2 < steps)
            pipeline_step<T, S, FIRST, TX, TY, 2>(st, g, lds, in, out, stride, pe, n, p + 2, steps,
                                                  z_load, k);
    }
}

// Work item of workgroup blockIdx.x, XCD-aware: the workgroups of a launch
// are dealt to the 8 XCDs in turn, and XCD x takes the x-th of 8 contiguous
// slices of the `items` items, so that consecutive items (neighbouring
// tiles, which share halo loads) run on one XCD and share its L2.  The grid
// is 8 ceil(items / 8) workgroups; those past the last item return at once
// (measured on MI355X: a member-list launch of 2270 items dealt in turn
// took 2.48 us per plane-step, one of 1784 items in slices 1.79).
__device__ __forceinline__ int xcd_item(int items)
{
    const int q = (items + 7) >> 3;  // items per XCD
    return (blockIdx.x & 7) * q + (blockIdx.x >> 3);
}

// Workgroups of a launch of `items` work items (see xcd_item); kMaxItems
// keeps both within int.
__host__ __device__ constexpr int64_t xcd_grid(int64_t items) { return (items + 7) / 8 * 8; }
constexpr int64_t kMaxItems = 0x7ffffff0;

template <typename T, int S, bool FIRST, int TX, int TY>
__global__ void __launch_bounds__((max_threads<T, S, TX, TY>()))
stream3d_kernel(const T *__restrict__ in, T *__restrict__ out, int64_t stride, int n,
                int tiles_x, int tiles_y, int tile_x_arg, int tile_y_arg, int chunk_len, Coef k)
{
    const int items = tiles_x * tiles_y * ((n + chunk_len - 1) / chunk_len);
    const int item = xcd_item(items);
    if (item >= items) return;  // the whole workgroup: no barrier is reached
    stream3d_item<T, S, FIRST, TX, TY>(in, out, stride, n, tiles_x, tiles_y, tile_x_arg,
                                       tile_y_arg, chunk_len, item, k);
}

// Several grids in one launch: member m owns the items [list[m].task_begin,
// list[m + 1].task_begin) of the launch, each grid with its own state
// buffers, constants, size and chunk, all with one tile: TX x TY compiled
// in, or tile_x x tile_y when TX = TY = 0.
template <typename T, int S, bool FIRST, int TX, int TY>
__global__ void __launch_bounds__((max_threads<T, S, TX, TY>()))
stream3d_list_kernel(const Stream2dMember *__restrict__ list, int nm, int items, int tile_x_arg,
                     int tile_y_arg)
{
    const int item = xcd_item(items);
    if (item >= items) return;  // the whole workgroup: no barrier is reached
    int lo = 0, hi = nm - 1;  // last member whose first item is <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (list[mid].task_begin <= item) lo = mid;
        else hi = mid - 1;
    }
    const Stream2dMember &m = list[lo];
    const int n = m.n;
    const Coef k = m.k;
    const int tile_x = TX ? TX : tile_x_arg, tile_y = TY ? TY : tile_y_arg;
    const int tiles_x = ((n >> 1) + tile_x - 1) / tile_x, tiles_y = (n + tile_y - 1) / tile_y;
    stream3d_item<T, S, FIRST, TX, TY>(static_cast<const T *>(m.in), static_cast<T *>(m.out),
                                       m.stride, n, tiles_x, tiles_y, tile_x, tile_y, m.chunk,
                                       item - static_cast<int>(m.task_begin), k);
}

template <typename T, int S>
hipError_t launch_typed(const Geometry &g, const StreamShape &sh, const T *in, T *out, bool first,
                        const Coef &k, hipStream_t s)
{
    const int HX = (S + 1) / 2, HY = S;
    const int H = g.n / 2;
    const int BX = sh.tile_x + 2 * HX, BY = sh.tile_y + 2 * HY;
    const int NT = BX * BY;
    const int NL = lds_plane(BX, BY);
    const int threads = (NT + 63) / 64 * 64;
    const int tiles_x = (H + sh.tile_x - 1) / sh.tile_x;
    const int tiles_y = (g.n + sh.tile_y - 1) / sh.tile_y;
    const int chunks = (g.n + sh.chunk - 1) / sh.chunk;
    const int64_t items = static_cast<int64_t>(tiles_x) * tiles_y * chunks;
    const size_t lds = static_cast<size_t>(2) * S * 3 * NL * sizeof(T);
    if (threads > max_threads<T, S>() || items > kMaxItems || lds > 160 * 1024)
        return hipErrorInvalidValue;
    // four-sweep launches of the 16x16 tile are compiled with the tile fixed
    // (measured on MI355X at 256^3 float64: 16x16 beats tiles of up to 768
    // threads, e.g. 16x28 and 32x13).  Other shapes take it at run time: the
    // float32 default 16x32 (compiled in, it spills registers at the 128
    // VGPRs its 13 waves allow and lost 15%) and the float64 32x13 of large
    // grids (compiled in, no faster).
    auto kern = first ? stream3d_kernel<T, S, true, 0, 0> : stream3d_kernel<T, S, false, 0, 0>;
    if constexpr (S == 4) {
        if (sh.tile_x == 16 && sh.tile_y == 16)
            kern = first ? stream3d_kernel<T, S, true, 16, 16> : stream3d_kernel<T, S, false, 16, 16>;
    }
    hipError_t e = allow_dynamic_lds(reinterpret_cast<const void *>(kern), static_cast<int>(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(xcd_grid(items))), dim3(threads), lds, s, in, out,
                       g.stride, g.n, tiles_x, tiles_y, sh.tile_x, sh.tile_y, sh.chunk, k);
    return hipGetLastError();
}

// Default tile of the launches over member lists (compressed positions x
// rows) per precision.  float64: 16x16, compiled in (8 waves, the LDS and
// registers of a workgroup per CU).  float32: 16x32 at run time (13 waves
// at 128 VGPRs, half the LDS bytes): the halo rings add 0.64 of the tile's
// columns instead of 0.88, and each SIMD holds 3-4 waves (measured on
// MI355X at 256^3: 213 against 249 us per 2-step launch).  A launch may
// take another tile (float64 groups of large grids: 32x13, 12 waves); the
// tile of a member's launches stays the same through a sequence, so that
// the member owns the same items in every launch.
struct ListTile {
    int x, y;
};

ListTile list_tile(int elem_bytes) { return elem_bytes == 8 ? ListTile{16, 16} : ListTile{16, 32}; }

template <typename T, int S>
hipError_t launch_list_typed(int tile_x, int tile_y, const Stream2dMember *list, int nm,
                             int64_t items, bool first, hipStream_t s)
{
    const int BX = tile_x + 2 * ((S + 1) / 2), BY = tile_y + 2 * S;
    const int threads = (BX * BY + 63) / 64 * 64;
    const size_t lds = static_cast<size_t>(2) * S * 3 * lds_plane(BX, BY) * sizeof(T);
    // the float64 16x16 tile is compiled in, every other tile taken at run time
    const bool fixed = sizeof(T) == 8 && tile_x == 16 && tile_y == 16;
    auto kern = first ? stream3d_list_kernel<T, S, true, 0, 0>
                      : stream3d_list_kernel<T, S, false, 0, 0>;
    int limit = max_threads<T, S>();
    if constexpr (sizeof(T) == 8) {
        if (fixed) {
            kern = first ? stream3d_list_kernel<T, S, true, 16, 16>
                         : stream3d_list_kernel<T, S, false, 16, 16>;
            limit = max_threads<T, S, 16, 16>();
        }
    }
    if (tile_x < 1 || tile_y < 1 || threads > limit || lds > 160 * 1024)
        return hipErrorInvalidValue;
    hipError_t e = allow_dynamic_lds(reinterpret_cast<const void *>(kern), static_cast<int>(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(xcd_grid(items))), dim3(threads), lds, s, list, nm,
                       static_cast<int>(items), tile_x, tile_y);
    return hipGetLastError();
}

}  // namespace

void stream3d_list_tile(int elem_bytes, int *tile_x, int *tile_y)
{
    const ListTile tl = list_tile(elem_bytes);
    *tile_x = tl.x;
    *tile_y = tl.y;
}

int64_t stream3d_member_items(int n, int chunk, int tile_x, int tile_y)
{
    const int64_t tx = (n / 2 + tile_x - 1) / tile_x, ty = (n + tile_y - 1) / tile_y;
    return tx * ty * ((n + chunk - 1) / chunk);
}

bool stream3d_list_ok(const Geometry &g, int chunk, int elem_bytes, int tile_x, int tile_y)
{
    const StreamShape sh = {tile_x, tile_y, chunk, 2};
    return stream3d_shape_ok(g, sh, elem_bytes);
}

hipError_t launch_stream3d_list(int precision, int stages, int tile_x, int tile_y,
                                const Stream2dMember *list, int nm, int64_t total_items,
                                bool first, hipStream_t s)
{
    if (!list || nm < 1 || total_items < 1 || total_items > kMaxItems ||
        (stages != 2 && stages != 4))
        return hipErrorInvalidValue;
    if (precision == 0)
        return stages == 2
                   ? launch_list_typed<double, 2>(tile_x, tile_y, list, nm, total_items, first, s)
                   : launch_list_typed<double, 4>(tile_x, tile_y, list, nm, total_items, first, s);
    return stages == 2
               ? launch_list_typed<float, 2>(tile_x, tile_y, list, nm, total_items, first, s)
               : launch_list_typed<float, 4>(tile_x, tile_y, list, nm, total_items, first, s);
}

bool stream3d_shape_ok(const Geometry &g, const StreamShape &sh, int elem_bytes)
{
    if (g.dim != 3 || g.n < 2 || (g.n & 1) || g.count != static_cast<int64_t>(g.n) * g.n * (g.n / 2))
        return false;
    if (sh.steps != 1 && sh.steps != 2) return false;
    if (sh.tile_x < 1 || sh.tile_y < 1 || sh.chunk < 1) return false;
    // per-thread offsets inside a z-plane of a pair plane are 32-bit byte
    // offsets
    if (2 * static_cast<int64_t>(g.n) * (g.n / 2) * elem_bytes >= (int64_t(1) << 31)) return false;
    const int S = 2 * sh.steps;
    const int BX = sh.tile_x + 2 * ((S + 1) / 2), BY = sh.tile_y + 2 * S;
    const int NT = BX * BY;
    const int limit = elem_bytes == 8 ? (S == 4 ? max_threads<double, 4>() : max_threads<double, 2>())
                                      : (S == 4 ? max_threads<float, 4>() : max_threads<float, 2>());
    if ((NT + 63) / 64 * 64 > limit) return false;
    return static_cast<size_t>(2) * S * 3 * lds_plane(BX, BY) * elem_bytes <= 160 * 1024;
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
