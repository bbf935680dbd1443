/*
 * kgs.h -- C ABI of the MI355X (gfx950) DP-AVF2 solver for the periodic
 * Klein-Gordon-Schroedinger (KGS) equations.
 *
 * The equations (sec. 1, eq. kgs) are
 *     i psi_t + (kappa1/2) Lap psi + gamma u psi = 0,
 *     u_tt - kappa2 Lap u + mu^2 u - gamma |psi|^2 = 0,
 * on the periodic box [lo, hi)^dim, dim = 1, 2 or 3, with psi complex and u
 * real.  They are discretised by central differences on n points per axis,
 * h = (hi - lo)/n (sec. 2), and advanced in time by DP-AVF2: the symmetric
 * composition of the dual-partition AVF method and its adjoint, each with
 * tau/2 (sec. 3.1, eq. dp-comp), with every grid point updated by the
 * explicit closed form of sec. 4.1 (eq. scheme1 / scheme1-adj) and the
 * points visited in checkerboard order (sec. 4.2): red points, then blue
 * points for the base half step; blue, then red for the adjoint half step.
 * A point is red when the sum of its 1-based indices is odd (Algorithm 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Arrays.  psi_re, psi_im, u and v_t (= u_t) are float64 arrays of n^dim
 * elements in C order (axis 0 slowest); element (i0, .., i_{dim-1}) is the
 * value at x = lo + (i0, .., i_{dim-1}) h, the paper's x_j = a + (j-1)h
 * re-based to 0 (sec. 2).  The boundary is always float64, whatever the
 * precision of the stored state.
 *
 * Memory kinds.  `mem` is KGS_HOST (ordinary host pointers) or KGS_DEVICE
 * (device pointers on the handle's GPU, e.g. a PyTorch tensor's data_ptr()).
 * The caller owns every array it passes; the library copies on entry and
 * keeps no alias.  The library owns the device state of a handle from
 * kgs_init until kgs_free.
 *
 * Streams.  Every GPU operation of a handle is enqueued on the stream given
 * at kgs_init (a hipStream_t; NULL is the default stream).  kgs_step only
 * enqueues and returns; kgs_energy, kgs_read_state (and kgs_sync) wait for
 * the stream.  A handle is not thread-safe; several handles may share a
 * stream.
 *
 * Errors.  Every function returns a KGS_* status and never aborts.  The
 * message of the last failure is available from kgs_last_error(handle), or
 * kgs_last_error(NULL) for failures that happen before a handle exists.
 */
#ifndef KGS_H
#define KGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    KGS_OK = 0,
    KGS_EINVAL = 1,     /* NULL pointer, dim not 1..3, n < 2, hi <= lo, tau 0 or
                           non-finite, non-finite parameter, bad enum value   */
    KGS_EODDN = 2,      /* odd n: with periodic wrap the points 0 and n-1 of an
                           axis would share a colour and be neighbours, so the
                           colour classes would not be independent (sec. 4.2) */
    KGS_ESINGULAR = 3,  /* the constant 2x2 (u, v) matrix is singular or its
                           inverse, which Algorithm 1 precomputes, is not
                           finite                                             */
    KGS_ENOMEM = 4,     /* device allocation failed or exceeds the limit      */
    KGS_EDEVICE = 5,    /* a HIP call failed; see kgs_last_error              */
    KGS_ENONFINITE = 6, /* the energy is NaN or infinite                      */
};

enum { KGS_FP64 = 0, KGS_FP32 = 1 };   /* precision of the stored state */
enum { KGS_HOST = 0, KGS_DEVICE = 1 }; /* memory kind of boundary arrays */

typedef struct kgs_sim kgs_sim; /* opaque handle; owns the device state */

typedef struct {
    int32_t dim;       /* 1, 2 or 3                                           */
    int32_t n;         /* points per axis, even, >= 2                         */
    double lo, hi;     /* periodic box [lo, hi)^dim; h = (hi - lo)/n          */
    double tau;        /* full time step; non-zero and finite (a negative tau
                          runs the scheme backwards: step(-tau) inverts
                          step(tau))                                          */
    double kappa1, kappa2, mu, gamma; /* finite; kappa1 may be negative     */
    int32_t precision; /* KGS_FP64 or KGS_FP32.  With KGS_FP32 the state is
                          stored in float32; every point update and the
                          energy are still computed in float64.              */
    int32_t reserved;  /* must be 0                                           */
} kgs_config;

/* Create a simulation from the initial state (psi_re + i psi_im, u, v_t at
 * time 0, laid out as described above) and return it in *out.  The state is
 * copied to the GPU in the colour-split layout (kgs_read_state reverses it).
 * `stream` is a hipStream_t (or NULL) on which all work of the handle runs.
 * Validates cfg (KGS_EINVAL, KGS_EODDN, KGS_ESINGULAR) before it allocates.
 * On failure *out is NULL and no memory is held. */
int kgs_init(const kgs_config *cfg, const double *psi_re, const double *psi_im, const double *u,
             const double *v_t, int32_t mem, void *stream, kgs_sim **out);

/* Enqueue nsteps DP-AVF2 steps (nsteps >= 0; 0 does nothing).  Asynchronous:
 * returns once the kernels are launched (KGS_EINVAL for nsteps < 0).  The
 * adjoint red sweep that closes the last step (Algorithm 3: a step ends with
 * the red points of the adjoint half) may be left pending: the next
 * kgs_step fuses it with its first red sweep, as consecutive steps within
 * one call are fused, and every call that reads or replaces the state
 * (kgs_energy, kgs_read_state, kgs_write_state, kgs_sync, batches,
 * kgs_autotune)
 * applies it first.  What any call observes is bitwise the state after
 * nsteps full steps. */
int kgs_step(kgs_sim *sim, int64_t nsteps);

/* Discrete energy of the current state: h^dim times E_h of sec. 2,
 *   sum_i [ 1/2 ( kappa1 |grad_h psi|_i^2 + kappa2 |grad_h u|_i^2 + v_i^2
 *                 + mu^2 u_i^2 ) - gamma |psi_i|^2 u_i ],
 * with forward differences grad_h, reduced on the GPU in float64 with
 * compensated (double-double) partial sums in a fixed, deterministic order.
 * Waits for the stream.  Writes *energy and returns KGS_ENONFINITE if it is
 * not finite. */
int kgs_energy(kgs_sim *sim, double *energy);

/* Copy the current state out (float64, layout as above) to host or device
 * arrays of n^dim elements.  Waits for the stream. */
int kgs_read_state(kgs_sim *sim, double *psi_re, double *psi_im, double *u, double *v_t,
                   int32_t mem);

/* Replace the current state (float64 arrays as above).  The copy runs on
 * the handle's stream after the work already enqueued, and the call returns
 * when it has finished.  Reading the state, writing it back and stepping
 * gives bitwise the same result as stepping without the round trip (float64
 * state). */
int kgs_write_state(kgs_sim *sim, const double *psi_re, const double *psi_im, const double *u,
                    const double *v_t, int32_t mem);

/* Complete the handle's steps (a pending closing sweep of the last step is
 * applied) and wait until all work enqueued for it has finished. */
int kgs_sync(kgs_sim *sim);

/* Release the device state.  NULL is accepted.  Waits for the stream.  The
 * handle is gone afterwards whatever the status: every release is
 * attempted, and KGS_EDEVICE (message from kgs_last_error(NULL)) reports a
 * failed wait or release. */
int kgs_free(kgs_sim *sim);

/* Message of the last failure on this handle (or, for NULL, of the last
 * failure in this thread before a handle existed); never NULL. */
const char *kgs_last_error(const kgs_sim *sim);

/* Name of a status code; never NULL. */
const char *kgs_status_string(int status);

/* ------------------------------------------------------------------------
 * Stepping without device allocation.  For callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc.  Not a step of the paper's method: the same
 * DP-AVF2 steps as kgs_step, on fields the caller owns.
 *
 * kgs_step_fields advances psi_re + i psi_im, u, v_t (device arrays of n^dim
 * float64 in the layout above, distinct and owned by the caller) by nsteps
 * steps of the grid and scheme of cfg, in place.  It enqueues a scatter into
 * the colour-split layout, the kernels kgs_step would run, and a gather back
 * into the four arrays, all on `stream` (a hipStream_t, NULL = the null
 * stream), and returns without waiting.  The result is bitwise that of
 * kgs_init + kgs_step + kgs_read_state on a handle with the same cfg (with
 * KGS_FP32 the fields come back rounded to float32, also for nsteps = 0).
 *
 * It calls no hipMalloc, hipFree or other allocating routine.  The working
 * state lives in a fixed scratch area of KGS_STEP_FIELDS_SCRATCH_BYTES per
 * device, which each device the library runs on holds until the process
 * ends.  A grid whose state (32 bytes per point with KGS_FP64, 16 with
 * KGS_FP32) does not fit is rejected with KGS_ENOMEM before anything is
 * enqueued; where the state fits but not twice the state, the in-place
 * kernels run instead of the ping-pong ones (same result).  Calls on one
 * device share that area: calls that overlap in time on one device (other
 * streams or threads) race and must not be issued.  Consecutive calls on
 * one stream are ordered and safe; nothing of an earlier call's contents is
 * read.  Errors: as kgs_init for cfg, KGS_EINVAL for a NULL array or
 * nsteps < 0, KGS_ENOMEM as above, KGS_EDEVICE for a runtime failure; the
 * message is kgs_last_error(NULL).
 */
#define KGS_STEP_FIELDS_SCRATCH_BYTES (64LL << 20)

int kgs_step_fields(const kgs_config *cfg, double *psi_re, double *psi_im, double *u,
                    double *v_t, int64_t nsteps, void *stream);

/* ------------------------------------------------------------------------
 * Launch configuration.  Every configuration computes bitwise the same
 * state (same-colour points are independent, sec. 4.2), so these knobs only
 * change speed.
 * ---------------------------------------------------------------------- */
enum {
    KGS_KERNEL_AUTO = 0,   /* library's choice for the grid                    */
    KGS_KERNEL_SWEEP = 1,  /* one launch per colour sweep, one thread per point */
    KGS_KERNEL_STREAM = 2, /* 2-D and 3-D: streaming kernels, 2 or 4 colour
                              sweeps (1 or 2 full steps) per launch between
                              two state buffers (the handle then holds twice
                              the state); 3-D streams along axis 0 with
                              tile_x x tile_y tiles, 2-D along axis 0 with
                              one wave per 64-lane tile of axis 1          */
    KGS_KERNEL_RESIDENT = 3, /* small grids (at most 4096 points per colour and
                                6 x points-per-colour x element bytes <= 160 KiB,
                                e.g. 1-D n <= 6826 float64 / 8192 float32):
                                the whole grid in one workgroup's LDS and
                                registers, all steps of a call in one launch */
    KGS_KERNEL_TILE = 4,   /* 2-D: 2, 4 or 8 colour sweeps per launch between two
                              state buffers, each workgroup running them on a
                              tile_y x tile_x tile (rows x points of one
                              colour) plus a halo held in LDS              */
};

typedef struct {
    int32_t kernel;        /* KGS_KERNEL_*                                    */
    int32_t block;         /* KGS_KERNEL_SWEEP: threads per workgroup (64..1024,
                              multiple of 64); 0 = default                      */
    int32_t tile_x;        /* KGS_KERNEL_STREAM, 3-D, and KGS_KERNEL_TILE: output
                              tile width in points of one colour along the
                              last axis                                    */
    int32_t tile_y;        /* KGS_KERNEL_STREAM, 3-D: output tile height (axis
                              1); KGS_KERNEL_TILE: rows (axis 0)           */
    int32_t chunk;         /* KGS_KERNEL_STREAM: planes (3-D) or rows (2-D) of
                              axis 0 per workgroup (3-D) or wave (2-D)        */
    int32_t steps_per_launch; /* KGS_KERNEL_STREAM: 1 or 2 DP-AVF2 steps (2 or
                              4 colour sweeps) per launch; KGS_KERNEL_TILE:
                              1, 2 or 4 (the last launches of a call take
                              the remaining steps, 2 or 1 at a time)        */
    int32_t reserved[2];   /* must be 0                                       */
} kgs_tuning;

/* Read / replace the launch configuration of a handle (KGS_EINVAL for a
 * configuration that does not apply to the grid). */
int kgs_get_tuning(const kgs_sim *sim, kgs_tuning *out);
int kgs_set_tuning(kgs_sim *sim, const kgs_tuning *t);

/* Autotuner: time each candidate launch configuration that fits the grid
 * (sweep block sizes; for 3-D grids also streaming tile/chunk shapes, for
 * 2-D grids streaming chunks and tiles, with 1 or 2 steps per launch) over
 * `steps` DP-AVF2 steps (the faster of two timings) on the handle's current
 * state, restore the state after every candidate, and keep the fastest.  The
 * state is unchanged on return.  With use_cache != 0 a winner found earlier
 * for the same (dim, n, precision, GPU architecture) is reused without
 * timing: found in this process, or read (once per process and file name)
 * from the file that the environment variable KGS_TUNE_CACHE names, to
 * which every winner is appended as one
 * text line ("kgs-tune-v1 arch dim n precision kernel block tile_x tile_y
 * chunk steps_per_launch"; the last line for a key wins; lines that do not
 * parse, or whose configuration no longer fits the grid, are ignored).
 * Writes the chosen configuration to *best (may be NULL).  Needs one extra
 * copy of the state in device memory while it runs. */
int kgs_autotune(kgs_sim *sim, int32_t steps, int32_t use_cache, kgs_tuning *best);

/* Sizes of a handle: bytes of device memory it holds and the name of the
 * kernel family that kgs_step launches. */
typedef struct {
    int64_t points;        /* n^dim                                           */
    int64_t device_bytes;  /* device memory held by the handle                */
    int32_t kernel;        /* KGS_KERNEL_* in use                             */
    int32_t precision;
} kgs_info;

int kgs_get_info(const kgs_sim *sim, kgs_info *out);

/* Device memory in bytes that kgs_init would allocate for cfg (0 for an
 * invalid cfg); lets a caller admit simulations against a memory budget. */
int64_t kgs_required_bytes(const kgs_config *cfg);

/* ------------------------------------------------------------------------
 * Batches: many independent simulations (any dimensions, sizes, parameters
 * and precisions) advanced together, one launch per (dimension, precision)
 * class over all members instead of one launch per simulation: members that
 * fit one workgroup run a whole call in one persistent launch; 2-D members
 * run 2 steps per launch (y-streaming or tiled kernel) and 3-D members of
 * n >= 32 run 2 steps per launch of the z-streaming kernel (float32: 16x32
 * tiles; float64: 16x16, or 32x13 where the launch planner expects the
 * class to end sooner with it), in uniform runs of 2 or more steps; every
 * other run is one launch per colour sweep.  A uniform run can be captured
 * once in a hipGraph and replayed.
 * Every member ends bitwise where kgs_step would have left it (points of one
 * colour are independent, sec. 4.2, so the launch layout does not matter).
 * ---------------------------------------------------------------------- */
typedef struct kgs_batch kgs_batch;

/* Group `count` distinct simulations (same GPU) into a batch whose work is
 * ordered on `stream` (hipStream_t or NULL): it starts after earlier work on
 * `stream` and later work on `stream` waits for it.  The batch keeps
 * pointers to the handles (not their data); free the batch before them.
 * Members keep working on their own: the batch uses their current state. */
int kgs_batch_create(kgs_sim *const *sims, int32_t count, void *stream, kgs_batch **out);

/* Advance every member by nsteps DP-AVF2 steps (asynchronous). */
int kgs_batch_step(kgs_batch *b, int64_t nsteps);

/* Advance member i by nsteps[i] steps (uneven counts, 0 allowed) in one
 * batched run: members that finish early drop out of the later launches. */
int kgs_batch_step_each(kgs_batch *b, const int64_t *nsteps);

/* With enable != 0, kgs_batch_step captures the launch sequence of a K-step
 * run in a hipGraph the first time K is used and replays it afterwards. */
int kgs_batch_set_graph(kgs_batch *b, int32_t enable);

/* Wait for the batch's work and release it (not the member simulations).
 * The batch is gone afterwards whatever the status; KGS_EDEVICE reports a
 * failed wait or release (every release is attempted). */
int kgs_batch_free(kgs_batch *b);

/* Time the launch configurations of each streaming group of the batch (the
 * 2-D members: y-streaming chunks of 8..64 rows and tiles of 8x8 .. 32x32
 * points of one colour; the 3-D members: plane chunks of 8..128, in
 * float64 with 16x16 and 32x13 tiles) over
 * uniform runs of `steps` steps (>= 2; a warm-up, then the faster of two
 * timed runs, each from the members' states, which are restored), and keep
 * the fastest for each group.  Every configuration gives bitwise the same
 * states.  With use_cache != 0 a winner found earlier for a group of the
 * same GPU architecture, dimension, precision and member sizes is reused
 * without timing: found in this process, or read from the file that
 * KGS_TUNE_CACHE names (see kgs_autotune; group lines carry the tag
 * "kgs-group-v1").  Graphs captured before are discarded.  Needs one copy of
 * a group's states in device memory while it runs; synchronises the batch's
 * stream. */
int kgs_batch_autotune(kgs_batch *b, int32_t steps, int32_t use_cache);

/* Message of the last failure of b (or of kgs_batch_create for NULL). */
const char *kgs_batch_last_error(const kgs_batch *b);

/* ------------------------------------------------------------------------
 * Serving loop with continuous batching.  Requests (any dimension, size,
 * parameters, precision and step count) are submitted at any time and are
 * admitted in arrival order while their device memory fits the budget.  Two
 * lanes share the GPU on streams of their own: grids that fit one workgroup
 * start together in one persistent resident launch per round and run all
 * their steps; all other grids advance in rounds of up to steps_per_round
 * steps, the requests with the least remaining work first, up to round_work
 * point-steps per round (3-D grids of n >= 96 together in launches of the
 * z-streaming kernel over a member list, 2-D grids advanced together 2 steps
 * per launch, the rest in one
 * batched launch sequence).  A request that arrives while
 * others run joins at the next round.  Finished requests are retired to host
 * memory and their device memory returns to the server's pool.  Host copies
 * of inputs and results are pinned (one transfer each at the full link
 * rate); the server keeps its pinned blocks for reuse and returns them to
 * the system in kgs_server_free (pinning is capped at a quarter of the
 * host's memory, at most 64 GiB; beyond it, plain host memory).  A freed
 * server's streams are kept and given to the next server created on the
 * same device (a server made with new streams after other device work can
 * run markedly slower).  Host code
 * does not wait for the GPU between rounds, except to keep at most two
 * rounds queued ahead.  A request's result is bitwise the state that
 * kgs_step gives when the same simulation runs alone.
 * Not thread-safe: one thread drives a server.
 * ---------------------------------------------------------------------- */
typedef struct kgs_server kgs_server;

enum { KGS_REQ_QUEUED = 0, KGS_REQ_RUNNING = 1, KGS_REQ_DONE = 2, KGS_REQ_FAILED = 3,
       KGS_REQ_CANCELLED = 4 };

typedef struct {
    int64_t budget_bytes;    /* device memory running requests may hold: each
                                holds kgs_required_bytes plus 32 bytes per point
                                for its gathered result                        */
    int32_t max_active;      /* cap on running requests, 0 = none              */
    int32_t steps_per_round; /* steps per running request per round, 0 = all  */
    int64_t round_work;      /* point-steps per round of the big-grid lane,
                                0 = 2^31 (about 25 ms of float64 3-D work)     */
    int32_t reserved[2];     /* must be 0                                      */
} kgs_server_config;

typedef struct {
    int32_t state;           /* KGS_REQ_*                                      */
    int32_t status;          /* KGS_* status of a failed request               */
    int64_t steps_done, nsteps;
    int64_t device_bytes;    /* device memory while running                    */
    double t_submit, t_admit, t_done; /* seconds since kgs_server_create       */
    double energy_start, energy_end;  /* kgs_energy at admission and at the end */
} kgs_request_info;

typedef struct {
    int64_t device_bytes_used;  /* running requests (bounded by the budget)    */
    int64_t queued_input_bytes; /* device copies of queued device inputs       */
    int32_t running, queued;
    int64_t rounds;
    double now;              /* seconds since kgs_server_create                */
} kgs_server_stats_t;

/* Create a server whose GPU work is ordered on `stream` (hipStream_t/NULL). */
int kgs_server_create(const kgs_server_config *cfg, void *stream, kgs_server **out);

/* Queue a request: the initial state (float64 arrays as for kgs_init) is
 * copied, host inputs into host memory before this call returns, device
 * inputs into a device buffer held until admission (kgs_server_stats reports
 * it; it is not part of the running budget) by a copy enqueued on the
 * server's stream: work the caller orders after it on that stream may
 * overwrite the inputs.  *id receives the request's handle.  Invalid
 * configurations are rejected here with kgs_init's status. */
int kgs_server_submit(kgs_server *s, const kgs_config *cfg, const double *psi_re,
                      const double *psi_im, const double *u, const double *v_t, int32_t mem,
                      int64_t nsteps, int64_t *id);

/* Run up to `rounds` rounds (admit, advance, retire); returns early when
 * nothing is left.  Reports how many requests are on the device (running or
 * retiring) and how many wait afterwards.  When nothing is left to enqueue
 * it waits for the retirements, so a loop that runs until both counts are 0
 * ends with every request finished. */
int kgs_server_run(kgs_server *s, int32_t rounds, int32_t *n_running, int32_t *n_queued);

/* State, progress, timestamps and energies of a request. */
int kgs_server_poll(const kgs_server *s, int64_t id, kgs_request_info *info);

/* Copy the result of a finished request (float64 arrays, host or device). */
int kgs_server_result(kgs_server *s, int64_t id, double *psi_re, double *psi_im, double *u,
                      double *v_t, int32_t mem);

/* Forget a request that is queued or finished (its result is dropped). */
int kgs_server_release(kgs_server *s, int64_t id);

/* Cancel a queued or running request: it reports KGS_REQ_CANCELLED at once;
 * its device memory returns to the pool after the work already queued. */
int kgs_server_cancel(kgs_server *s, int64_t id);

int kgs_server_stats(const kgs_server *s, kgs_server_stats_t *st);

/* Wait for the server's work and release everything it holds.  The server
 * is gone afterwards whatever the status; KGS_EDEVICE reports a failed wait
 * or a failed release, including one of a request's buffers earlier in the
 * server's life (every release is attempted). */
int kgs_server_free(kgs_server *s);

const char *kgs_server_last_error(const kgs_server *s);

#ifdef __cplusplus
}
#endif

#endif /* KGS_H */
