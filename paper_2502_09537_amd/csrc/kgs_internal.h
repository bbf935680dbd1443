// Internal interface between the host side of the library (kgs_api.cpp,
// compiled by the host compiler) and the HIP kernels (*.hip, gfx950).
//
// Device layout of a simulation ("colour-split pair planes"):
//   2 colours (0 = red, 1 = blue) x 2 pair planes of 2*stride elements:
//   (P, Q) = (Re psi, Im psi) at base + 4*colour*stride and (U, V) = (u, u_t)
//   at base + (4*colour + 2)*stride, the two values of point t at elements
//   2t and 2t + 1 of its pair plane.  Field f (F_P, F_Q, F_U, F_V) of point
//   t of colour c is therefore element (4c + (f & 2))*stride + 2t + (f & 1),
//   and the whole state is 8*stride elements.  A pair is one vector access;
//   the neighbours of a point, which need P, Q and U of the other colour,
//   read a (P, Q) pair and U alone.
//   Point t = row * H + xh, where H = n/2,
//   row = i0 (2-D) or i0*n + i1 (3-D) or 0 (1-D) enumerates the grid lines
//   along the last (fastest) axis x, and xh = x/2 is x compressed to the
//   points of one colour.  In row r with index sum s (i0 + i1 in 3-D, i0 in
//   2-D, 0 in 1-D) the points of colour c sit at x = 2 xh + o_c with
//   o_c = (s + dim + 1 + c) & 1: red points have an odd sum of 1-based
//   indices (Algorithm 3 of the paper).
//   Consequences used by every kernel: the two x-neighbours of (r, xh, o) in
//   the other colour are xh - 1 + o and xh + o (mod H); the neighbours along
//   every other axis sit at the same xh in the neighbouring rows.
#pragma once

#include <cstdint>

#include <hip/hip_runtime_api.h>

namespace kgs {

enum Colour { RED = 0, BLUE = 1 };
enum Field { F_P = 0, F_Q = 1, F_U = 2, F_V = 3 };

// Colour-sweep kinds.  A run of K steps is
//   R_BASE, (B_FULL, R_ADJ_BASE)^(K-1), B_FULL, R_ADJ
// because blue points do not change between the base and the adjoint blue
// sweeps, and red points do not change between the adjoint red sweep of a
// step and the base red sweep of the next (the paper's four masked passes per
// step, Algorithm 3, fused into two sweeps).
enum PassKind {
    PASS_R_BASE = 0,     // red:  psi, then (u,v)                   (base)
    PASS_B_FULL = 1,     // blue: psi, (u,v) (base); (u,v), psi (adjoint)
    PASS_R_ADJ = 2,      // red:  (u,v), then psi                   (adjoint)
    PASS_R_ADJ_BASE = 3, // red:  (u,v), psi (adjoint); psi, (u,v) (next base)
};

// Per-half-step constants of the explicit point updates, tau' = tau/2.
// psi:   (i - c) psi' = (i + c) psi - b S,   c = a - e u,
// (u,v): u' - t2 v' = u + t2 v,  beta u' + v' = v - beta u + s S_u + g |psi|^2.
struct Coef {
    double b;      // tau' kappa1 / (2 h^2)
    double a;      // dim * b
    double e;      // (tau' gamma) / 2
    double s;      // tau' kappa2 / h^2
    double beta;   // dim tau' kappa2 / h^2 + tau' mu^2 / 2
    double t2;     // tau' / 2
    double g;      // tau' gamma
    double rd_hi;  // 1 / (1 + t2 beta) as the unevaluated sum rd_hi + rd_lo
    double rd_lo;
};

// Constants of the energy density (multiplied by h^dim on the host).
struct EnergyCoef {
    double k1_h2;  // kappa1 / h^2
    double k2_h2;  // kappa2 / h^2
    double mu2;    // mu^2
    double gamma;
};

struct Geometry {
    int dim;
    int n;
    int half;        // n / 2
    int64_t rows;    // n^(dim-1)
    int64_t count;   // points per colour = rows * half
    int64_t stride;  // count rounded up to 64; a pair plane spans 2*stride elements
};

// Shape of the 3-D z-streaming kernel: output tile of tile_y rows x tile_x
// compressed positions, chunk planes per workgroup, 1 or 2 DP-AVF2 steps
// (2 or 4 colour sweeps) per launch.
struct StreamShape {
    int tile_x;
    int tile_y;
    int chunk;
    int steps;
};

// One member of a batched sweep (kgs_batch.hip): a simulation's current
// state buffer and constants, and the first workgroup it owns in the grid.
struct BatchMember {
    void *state;
    int64_t stride;
    int64_t count;        // points per colour
    int64_t block_begin;  // first workgroup of this member
    Coef k;
    int n;
    int pad;
};

// One simulation advanced by the resident kernel (kgs_resident.hip): its
// state buffer, constants, and the number of DP-AVF2 steps to take (<= 0:
// the member is skipped).
struct ResidentMember {
    void *state;
    int64_t stride;
    int64_t steps;
    Coef k;
    int n;
    int count;  // points per colour
};

// One member of a 2-D streaming launch (kgs_stream2d.hip): S sweeps from
// `in` to `out` (distinct buffers), tasks (one wave each) [task_begin,
// task_begin + tiles_x * ceil(n / chunk)) of the launch; `first` makes the
// first sweep R_BASE instead of R_ADJ_BASE.
struct Stream2dMember {
    const void *in;
    void *out;
    int64_t stride;
    int64_t task_begin;
    Coef k;
    int n;
    int chunk;
    int tiles_x;
    int first;
};

// Upper bound on the LDS one resident workgroup may use (the device limit
// can lower it).
constexpr int kResidentMaxLds = 160 * 1024;

// Lets `kernel` take `bytes` of dynamic LDS on the current device: one
// runtime call the first time a kernel needs more than it was allowed, none
// afterwards (kgs_launch.cpp).
hipError_t allow_dynamic_lds(const void *kernel, int bytes);

// Kernel launchers (kgs_sweep.hip, kgs_energy.hip, kgs_stream3d.hip).  They check the launch
// shape against the geometry on the host and return hipErrorInvalidValue
// rather than launch a kernel whose indexing would not fit.
hipError_t launch_scatter(const Geometry &g, int precision, void *state, const double *P,
                          const double *Q, const double *U, const double *V, hipStream_t s);
hipError_t launch_gather(const Geometry &g, int precision, const void *state, double *P,
                         double *Q, double *U, double *V, hipStream_t s);
hipError_t launch_sweep(const Geometry &g, int precision, void *state, int kind, const Coef &k,
                        int block, hipStream_t s);
// `stages` (2 or 4) colour sweeps from `in` to `out` (distinct buffers);
// the first stage is R_BASE when `first`, else R_ADJ_BASE.
bool stream3d_shape_ok(const Geometry &g, const StreamShape &sh, int elem_bytes);
hipError_t launch_stream3d(const Geometry &g, int precision, const StreamShape &sh, int stages,
                           const void *in, void *out, bool first, const Coef &k, hipStream_t s);
// 3-D streaming over several grids of one precision in one launch, all
// with the tile tile_x x tile_y (compressed positions x rows;
// stream3d_list_tile() gives the precision's default, element bytes 8 or
// 4): member m (sorted by task_begin, the first workgroup it owns) takes
// stream3d_member_items(n, chunk, tile_x, tile_y) workgroups and advances
// `stages` (2 or 4) sweeps from in to out (the Stream2dMember fields
// tiles_x and first are not read: the launch's first sweep is R_BASE when
// `first`).  stream3d_list_ok: whether a grid fits a list launch with that
// chunk and tile (checked by the caller for every member).
void stream3d_list_tile(int elem_bytes, int *tile_x, int *tile_y);
int64_t stream3d_member_items(int n, int chunk, int tile_x, int tile_y);
bool stream3d_list_ok(const Geometry &g, int chunk, int elem_bytes, int tile_x, int tile_y);
hipError_t launch_stream3d_list(int precision, int stages, int tile_x, int tile_y,
                                const Stream2dMember *list, int nm, int64_t total_items,
                                bool first, hipStream_t s);
// Batched sweep over `nm` members (sorted by block_begin, blocks of
// batch_block() threads).  Kinds: kinds[launch * nm + i] (-1 = idle) if
// kinds != NULL, else uniform_kind for every member.
int batch_block();
hipError_t launch_batch_sweep(int dim, int precision, const BatchMember *members, int nm,
                              int64_t total_blocks, const int *kinds, int launch,
                              int uniform_kind, hipStream_t s);
// Resident kernel: whether a grid of `count` points per colour fits one
// workgroup; a one-time per-device set-up (LDS limits of the kernel
// variants; launch_resident calls it, callers that capture launches into a
// graph call it first); and a launch over one member (list == NULL, nm == 1,
// one.steps steps) or over the nm members of `list` (device memory, one
// workgroup each, all of one dimension and precision and each with count <=
// max_count), member i taking steps_each[i] steps (device memory) or, with
// steps_each == NULL, steps_all steps.
bool resident_fits(int64_t count, int elem_bytes);
hipError_t resident_prepare();
hipError_t launch_resident(int dim, int precision, const ResidentMember &one,
                           const ResidentMember *list, const int64_t *steps_each,
                           int64_t steps_all, int nm, int64_t max_count, hipStream_t s);
// 2-D streaming kernel: tiles along x and tasks of one member (the same for
// 2 and 4 sweeps per launch); a launch of `stages` (2 or 4) sweeps over one
// member (list == NULL, nm == 1) or over the nm members of `list` (device
// memory, sorted by task_begin, all of one precision).
int stream2d_tiles_x(int n);
int64_t stream2d_tasks(int n, int chunk);
hipError_t launch_stream2d(int precision, int stages, const Stream2dMember &one,
                           const Stream2dMember *list, int nm, int64_t total_tasks, hipStream_t s);

// 2-D tiled kernel (kgs_tile2d.hip): `stages` (2 or 4) sweeps per launch
// from `in` to `out`, tiles of ty rows x txc compressed positions, each with
// its halo in LDS.  One grid (launch_tile2d), or many: a member list with
// the Stream2dMember meaning of task_begin (first tile of the member, in
// ascending order) and tiles_x = tile2d_tiles_x(n, txc), one workgroup per
// tile; whether the launch starts the members' runs is `first_launch` for a
// list and `one.first` otherwise.
int tile2d_tiles_x(int n, int txc);
int64_t tile2d_member_tiles(int n, int ty, int txc);
int64_t tile2d_tiles(const Geometry &g, int ty, int txc);
// Tile shape for one launch over grids of sizes n[0..count).
void tile2d_group_shape(const int *n, int count, int &ty, int &txc);
bool tile2d_shape_ok(const Geometry &g, int ty, int txc, int stages, int elem_bytes);
hipError_t launch_tile2d(const Geometry &g, int precision, int stages, int ty, int txc,
                         const void *in, void *out, bool first, const Coef &k, hipStream_t s);
hipError_t launch_tile2d_list(int precision, int stages, int ty, int txc, const Stream2dMember &one,
                              const Stream2dMember *list, int nm, int64_t total_tiles,
                              hipStream_t s, int first_launch = 0);
// Writes the double-double sum of the energy density (without h^dim) to
// out[0] + out[1] (device memory); `partials` holds 2*energy_partial_slots()
// doubles.
int energy_partial_slots();
hipError_t launch_energy(const Geometry &g, int precision, const void *state,
                         const EnergyCoef &k, double *partials, double *out, hipStream_t s);

}  // namespace kgs
