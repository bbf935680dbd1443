// Serving loop with continuous batching: requests (simulations of any
// dimension, size, parameters, precision and step count) arrive at any time,
// wait in a queue, are admitted in arrival order while their device memory
// fits the budget, run, and are retired to host memory.
//
// Two lanes run side by side on the GPU, each on its own stream:
//   * small lane: grids that fit one workgroup (the resident kernel).  Each
//     round, the requests admitted since the last round start together in
//     one persistent launch per (dimension, precision), each taking all of
//     its steps, so small requests never wait behind big ones;
//   * big lane: every other grid, in rounds.  A round advances the running
//     requests with the least remaining work (points x steps left) first, up
//     to round_work point-steps per round and steps_per_round steps per
//     request: 3-D grids of the z-streaming kernel together in member-list
//     launches of that kernel, 2-D grids together in 2-D streaming launches
//     (one task list over all of them), the rest in one batched launch
//     sequence per (dimension, precision) with per-request step counts.  Shortest-remaining-work-
//     first keeps the mean and median latency low when the device is
//     oversubscribed.
// The host does not wait for the GPU in steady state: device memory comes
// from a private pool in stream order, energies land in pinned slots, a
// finished request's state is gathered on the device and, once its event has
// passed, copied to host memory by a worker thread on a stream of its own
// (so the round loop keeps feeding the GPU while large results copy), and at
// most kMaxAhead rounds are queued ahead of the device on each lane.
//
// Each request ends bitwise where running it alone ends: points of one
// colour are independent and step boundaries store the state exactly as a
// continuous run's fused sweeps round it.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include <unistd.h>

#include <hip/hip_runtime_api.h>

#include "kgs.h"
#include "kgs_trace.h"
#include "kgs_internal.h"
#include "kgs_plan.h"
#include "kgs_sim.h"

namespace {

constexpr int64_t kDefaultRoundWork = int64_t(1) << 31;  // point-steps per big-lane round
constexpr size_t kMaxAhead = 2;                          // rounds queued ahead, per lane
constexpr int kRingSlots = 16;                           // staging slots per lane
constexpr int kSlotChunk = 1024;                         // energy slots per allocation

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum Lane { LANE_BIG = 0, LANE_SMALL = 1 };

// Host arrays of a request (its input, then its result) are pinned: the
// runtime then moves them to and from the device in one copy at the full
// link rate, where pageable memory goes through staging in 1 MiB pieces,
// each a copy kernel on the CUs the solver uses (measured on MI355X, 256
// MiB: 4.7 against 15.2 ms to the host, 4.7 against 8.9 ms to the device;
// pinning 256 MiB took 1 ms).
//
// hipHostFree waits for all work queued on the device (measured: a free
// issued behind 290 ms of queued kernels returned after them), so a
// server keeps its pinned blocks for reuse and frees them only when it is
// freed itself.  Pinned memory per server is capped at a quarter of the
// host's physical memory, at most 64 GiB; beyond the cap, or if pinning
// fails, arrays are plain host memory.
class PinnedCache {
public:
    PinnedCache() = default;
    PinnedCache(const PinnedCache &) = delete;
    PinnedCache &operator=(const PinnedCache &) = delete;
    ~PinnedCache()
    {
        for (auto &kv : size_) (void)hipHostFree(kv.first);  // kgs_server_free released them
    }

    // A free block of at least `bytes` and at most twice that, else a new
    // one; at the cap (or when pinning fails) the smallest free block that
    // is large enough, else NULL.
    void *take(size_t bytes)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = free_.lower_bound(bytes);
        auto reuse = [&] {
            void *q = it->second;
            free_.erase(it);
            return q;
        };
        if (it != free_.end() && it->first <= 2 * bytes) return reuse();
        void *p = nullptr;
        if (total_ + bytes > cap() ||
            hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess || !p)
            return it != free_.end() ? reuse() : nullptr;
        size_[p] = bytes;
        total_ += bytes;
        return p;
    }

    void give(void *p)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = size_.find(p);
        if (it != size_.end()) free_.emplace(it->second, p);
    }

    // Frees every block (all of them returned); the first failure goes to err.
    void release(kgs::FirstError &err)
    {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto &kv : size_) err(hipHostFree(kv.first));
        size_.clear();
        free_.clear();
        total_ = 0;
    }

private:
    static size_t cap()
    {
        const long pages = sysconf(_SC_PHYS_PAGES), page = sysconf(_SC_PAGE_SIZE);
        const size_t quarter = pages > 0 && page > 0 ? static_cast<size_t>(pages) * page / 4 : 0;
        return std::min(quarter, size_t(64) << 30);
    }

    std::mutex mu_;
    std::multimap<size_t, void *> free_;  // bytes -> free block
    std::map<void *, size_t> size_;       // every block -> bytes
    size_t total_ = 0;
};

struct HostDeleter {
    PinnedCache *cache = nullptr;  // pinned: back to its cache
    void operator()(double *p) const
    {
        if (!p) return;
        if (cache)
            cache->give(p);
        else
            delete[] p;
    }
};
using HostArray = std::unique_ptr<double[], HostDeleter>;

HostArray host_array(PinnedCache &c, size_t n)
{
    if (void *p = c.take(n * sizeof(double)))
        return HostArray(static_cast<double *>(p), HostDeleter{&c});
    return HostArray(new (std::nothrow) double[n], HostDeleter{nullptr});
}

struct Request {
    int64_t id = 0;
    kgs_config cfg;
    int64_t nsteps = 0;
    int64_t done_steps = 0;  // steps enqueued on the device
    int32_t state = KGS_REQ_QUEUED;
    int32_t status = KGS_OK;
    int64_t bytes = 0;   // device bytes while running: state(s) + gathered result
    int64_t points = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    double e0 = 0, e1 = 0;
    HostArray host;                  // 4 arrays of `points` doubles: input, then the result
    double *dev_in = nullptr;        // pooled device copy of the input until admission
    kgs_sim *sim = nullptr;
    int lane = LANE_BIG;
    int slot = -1;                   // energy slot
    double *staging = nullptr;       // pooled gathered result during retirement
    hipEvent_t ev = nullptr;         // retirement complete on the device
    bool retiring = false;
    bool copying = false;            // result handed to the copy worker
    bool dropped = false;            // cancelled while retiring
    std::string err;
};

// Copies of gathered results to host memory, done by a worker thread.
struct CopyJob {
    int64_t id;
    double *src;  // pooled device buffer, released by the worker
    size_t n;     // doubles
};

struct CopyDone {
    int64_t id;
    HostArray host;
    hipError_t status;
    double t;  // completion, seconds on the server clock
};

// Pinned host staging with a device twin, reused round-robin; a slot is
// rewritten only after the event recorded behind its last reader has passed.
struct Ring {
    struct Slot {
        char *h = nullptr, *d = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool used = false;
    };
    Slot slots[kRingSlots];
    int next = 0;
};

struct EnergyChunk {
    double *d = nullptr;  // device, 4 doubles per slot: start (hi, lo), end (hi, lo)
    double *h = nullptr;  // pinned mirror
};

}  // namespace

struct kgs_server {
    // first member: destroyed after every host array that returns to it
    PinnedCache pinned;
    kgs_server_config cfg;
    hipStream_t user = nullptr;  // caller's stream: device input copies
    hipStream_t lane[2] = {nullptr, nullptr};
    hipStream_t copy = nullptr;  // host <-> device copies of inputs and results
    hipMemPool_t pool = nullptr;
    hipEvent_t ev_submit = nullptr;
    bool submitted = false;  // device input copies on the caller's stream since the last round
    int device = 0;
    double t0 = 0;
    int64_t next_id = 1;
    int64_t used = 0;        // device bytes held by running and retiring requests
    int64_t queued_dev = 0;  // device bytes held by queued device-submitted inputs
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::deque<int64_t> queue;
    std::vector<int64_t> running[2];  // per lane: requests with steps left to enqueue
    std::vector<int64_t> retiring;    // in order of retirement
    Ring ring[2];
    std::vector<EnergyChunk> energy;
    std::vector<int> free_slots;
    std::deque<hipEvent_t> ahead;  // one event per queued round and lane
    std::vector<hipEvent_t> spare_events;
    int64_t rounds = 0;
    std::string err;
    // the first failed release of a resource (reported by kgs_server_free);
    // the copy worker updates it under `mu`
    kgs::FirstError release_err;
    // result-copy worker
    std::thread copier;
    hipStream_t copy_out = nullptr;
    std::mutex mu;
    std::condition_variable cv_jobs, cv_done;
    std::deque<CopyJob> jobs;
    std::deque<CopyDone> done;
    int in_flight = 0;  // jobs queued or being copied
    bool stop = false;
};

namespace {

thread_local std::string g_srv_err;

// Streams of servers that have been freed, per device, for the next server
// of the device to take: lane 0, lane 1, copy, copy_out.  (Measured on
// MI355X: a server made after other device work, with new streams, ran the
// serving mix 1.55x slower than the first server of the process; driving
// the mix again through the first server's streams ran at full speed.)
std::mutex g_stream_mu;
std::map<int, std::vector<std::array<hipStream_t, 4>>> g_free_streams;

hipError_t take_streams(kgs_server *s)
{
    {
        std::lock_guard<std::mutex> lock(g_stream_mu);
        auto &v = g_free_streams[s->device];
        if (!v.empty()) {
            const auto st = v.back();
            v.pop_back();
            s->lane[0] = st[0];
            s->lane[1] = st[1];
            s->copy = st[2];
            s->copy_out = st[3];
            return hipSuccess;
        }
    }
    hipError_t e = hipSuccess;
    for (int l = 0; l < 2 && e == hipSuccess; ++l)
        e = hipStreamCreateWithFlags(&s->lane[l], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_out, hipStreamNonBlocking);
    return e;
}

// Hands a freed server's streams to the next server of its device when all
// four exist and have finished their work, and destroys them otherwise.
void give_streams(kgs_server *s)
{
    hipStream_t st[4] = {s->lane[0], s->lane[1], s->copy, s->copy_out};
    bool whole = true;
    for (hipStream_t x : st) whole = whole && x && hipStreamSynchronize(x) == hipSuccess;
    if (whole) {
        std::lock_guard<std::mutex> lock(g_stream_mu);
        g_free_streams[s->device].push_back({st[0], st[1], st[2], st[3]});
        return;
    }
    for (hipStream_t x : st)
        if (x) s->release_err(hipStreamDestroy(x));
}

int sfail(kgs_server *s, int code, const std::string &msg)
{
    if (s) s->err = msg;
    else g_srv_err = msg;
    return code;
}

int shipfail(kgs_server *s, hipError_t e, const char *what)
{
    return sfail(s, e == hipErrorOutOfMemory ? KGS_ENOMEM : KGS_EDEVICE,
                 std::string(what) + ": " + hipGetErrorName(e));
}

int status_of(hipError_t e) { return e == hipErrorOutOfMemory ? KGS_ENOMEM : KGS_EDEVICE; }

int64_t total_running(const kgs_server *s)
{
    return static_cast<int64_t>(s->running[0].size() + s->running[1].size() + s->retiring.size());
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---- events -------------------------------------------------------------

hipEvent_t take_event(kgs_server *s)
{
    if (!s->spare_events.empty()) {
        hipEvent_t e = s->spare_events.back();
        s->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void give_event(kgs_server *s, hipEvent_t e)
{
    if (e) s->spare_events.push_back(e);
}

// ---- energy slots -------------------------------------------------------

int take_slot(kgs_server *s)
{
    if (s->free_slots.empty()) {
        EnergyChunk c;
        const size_t bytes = 4 * kSlotChunk * sizeof(double);
        if (hipMalloc(reinterpret_cast<void **>(&c.d), bytes) != hipSuccess) return -1;
        if (hipHostMalloc(reinterpret_cast<void **>(&c.h), bytes, hipHostMallocDefault) !=
            hipSuccess) {
            s->release_err(hipFree(c.d));
            return -1;
        }
        const int base = static_cast<int>(s->energy.size()) * kSlotChunk;
        s->energy.push_back(c);
        for (int i = kSlotChunk - 1; i >= 0; --i) s->free_slots.push_back(base + i);
    }
    const int slot = s->free_slots.back();
    s->free_slots.pop_back();
    return slot;
}

double *slot_dev(kgs_server *s, int slot, int which)
{
    return s->energy[slot / kSlotChunk].d + 4 * (slot % kSlotChunk) + 2 * which;
}

double *slot_host(kgs_server *s, int slot, int which)
{
    return s->energy[slot / kSlotChunk].h + 4 * (slot % kSlotChunk) + 2 * which;
}

// Energy of the request's current state into part `which` of its slot
// (0 = start, 1 = end), device -> pinned, in the order of its lane stream.
hipError_t enqueue_energy(kgs_server *s, Request *r, int which)
{
    kgs_sim *m = r->sim;
    double *d = slot_dev(s, r->slot, which);
    hipError_t e = kgs::launch_energy(m->geo, m->cfg.precision, m->state, m->ecoef, m->partials, d,
                                      m->stream);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(slot_host(s, r->slot, which), d, 2 * sizeof(double),
                          hipMemcpyDeviceToHost, m->stream);
}

// ---- staging ring -------------------------------------------------------

// The next slot of a lane's ring with room for `bytes`, its earlier use done.
Ring::Slot *ring_take(kgs_server *s, int lane, size_t bytes, int &rc)
{
    Ring &g = s->ring[lane];
    Ring::Slot &sl = g.slots[g.next];
    g.next = (g.next + 1) % kRingSlots;
    rc = KGS_OK;
    hipError_t e;
    if (sl.used && (e = hipEventSynchronize(sl.ev)) != hipSuccess) {
        rc = shipfail(s, e, "hipEventSynchronize (staging)");
        return nullptr;
    }
    if (sl.cap < bytes) {
        if (sl.h) s->release_err(hipHostFree(sl.h));
        if (sl.d) s->release_err(hipFree(sl.d));
        sl.h = sl.d = nullptr;
        sl.cap = 0;
        size_t cap = 4096;
        while (cap < bytes) cap *= 2;
        if ((e = hipHostMalloc(reinterpret_cast<void **>(&sl.h), cap, hipHostMallocDefault)) !=
                hipSuccess ||
            (e = hipMalloc(reinterpret_cast<void **>(&sl.d), cap)) != hipSuccess) {
            rc = shipfail(s, e, "staging allocation");
            return nullptr;
        }
        sl.cap = cap;
    }
    if (!sl.ev && hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
        rc = sfail(s, KGS_EDEVICE, "hipEventCreate");
        return nullptr;
    }
    return &sl;
}

// Marks the slot busy until the lane stream has passed its readers.
hipError_t ring_done(kgs_server *s, int lane, Ring::Slot *sl)
{
    sl->used = true;
    return hipEventRecord(sl->ev, s->lane[lane]);
}

// ---- request life cycle -------------------------------------------------

// Returns a request's device memory in stream order (after the work queued
// on the stream each buffer was last used on).
void free_request_memory(kgs_server *s, Request *r)
{
    if (r->sim) {
        kgs::sim_destroy_pooled(r->sim);
        r->sim = nullptr;
    }
    if (r->dev_in) {
        s->release_err(hipFreeAsync(r->dev_in, s->user));
        r->dev_in = nullptr;
    }
    if (r->staging) {
        s->release_err(hipFreeAsync(r->staging, s->copy));
        r->staging = nullptr;
    }
}

void finish(kgs_server *s, Request *r, int32_t state, int32_t status)
{
    r->state = state;
    r->status = status;
    r->t_done = now_s() - s->t0;
}

// Admit queued requests in arrival order while they fit the budget.
void admit(kgs_server *s)
{
    while (!s->queue.empty()) {
        if (s->cfg.max_active > 0 && total_running(s) >= s->cfg.max_active) break;
        Request *r = s->reqs[s->queue.front()].get();
        const int64_t P = r->points;
        const size_t in_bytes = 4 * static_cast<size_t>(P) * sizeof(double);
        if (r->bytes > s->cfg.budget_bytes) {
            s->queue.pop_front();
            if (r->dev_in) s->queued_dev -= static_cast<int64_t>(in_bytes);
            free_request_memory(s, r);
            r->host.reset();
            r->err = "request needs more device memory than the whole budget";
            finish(s, r, KGS_REQ_FAILED, KGS_ENOMEM);
            continue;
        }
        if (s->used + r->bytes > s->cfg.budget_bytes) break;  // wait for retirements
        s->queue.pop_front();
        const int lane = kgs::default_kernel(r->cfg) == KGS_KERNEL_RESIDENT ? LANE_SMALL : LANE_BIG;
        hipStream_t st = s->lane[lane];
        hipError_t e = hipSuccess;
        if (!r->dev_in) {
            // host input: a pooled device copy made on the copy stream (no
            // kernels there, so waiting for it waits for the copy only)
            e = hipMallocFromPoolAsync(reinterpret_cast<void **>(&r->dev_in), in_bytes, s->pool,
                                       s->copy);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->dev_in, r->host.get(), in_bytes, hipMemcpyHostToDevice,
                                   s->copy);
            if (e == hipSuccess) e = hipStreamSynchronize(s->copy);
            r->host.reset();
        } else {
            s->queued_dev -= static_cast<int64_t>(in_bytes);
        }
        std::string msg;
        int rc = e == hipSuccess ? KGS_OK : status_of(e);
        if (rc == KGS_OK)
            rc = kgs::sim_create_pooled(&r->cfg, r->dev_in, r->dev_in + P, r->dev_in + 2 * P,
                                        r->dev_in + 3 * P, st, s->pool, &r->sim, msg);
        else
            msg = std::string("input copy: ") + hipGetErrorName(e);
        if (r->dev_in) {
            s->release_err(hipFreeAsync(r->dev_in, st));
            r->dev_in = nullptr;
        }
        if (rc == KGS_OK && (r->slot = take_slot(s)) < 0) {
            rc = KGS_ENOMEM;
            msg = "energy slot allocation failed";
        }
        if (rc == KGS_OK && (e = enqueue_energy(s, r, 0)) != hipSuccess) {
            rc = status_of(e);
            msg = std::string("energy kernel: ") + hipGetErrorName(e);
        }
        if (rc != KGS_OK) {
            free_request_memory(s, r);
            r->slot = -1;  // a copy into it may be in flight: not reused
            r->err = msg;
            finish(s, r, KGS_REQ_FAILED, rc);
            continue;
        }
        r->lane = lane;
        r->state = KGS_REQ_RUNNING;
        r->t_admit = now_s() - s->t0;
        s->used += r->bytes;
        s->running[lane].push_back(r->id);
    }
}

// Enqueue the end of a request that took all its steps: the final energy,
// the state gathered into a pooled float64 buffer, the handle's memory back
// to the pool, and an event behind them.
void start_retire(kgs_server *s, Request *r)
{
    kgs_sim *m = r->sim;
    const int64_t P = r->points;
    const size_t bytes = 4 * static_cast<size_t>(P) * sizeof(double);
    hipError_t e = enqueue_energy(s, r, 1);
    if (e == hipSuccess)
        e = hipMallocFromPoolAsync(reinterpret_cast<void **>(&r->staging), bytes, s->pool,
                                   m->stream);
    if (e == hipSuccess)
        e = kgs::launch_gather(m->geo, m->cfg.precision, m->state, r->staging, r->staging + P,
                               r->staging + 2 * P, r->staging + 3 * P, m->stream);
    if (e == hipSuccess && !(r->ev = take_event(s))) e = hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipEventRecord(r->ev, m->stream);
    if (e != hipSuccess && r->ev) {
        give_event(s, r->ev);
        r->ev = nullptr;
    }
    if (e != hipSuccess && r->status == KGS_OK) {
        r->status = status_of(e);
        r->err = std::string("retirement: ") + hipGetErrorName(e);
    }
    kgs::sim_destroy_pooled(m);  // in stream order: after the gather
    r->sim = nullptr;
    r->retiring = true;
    s->retiring.push_back(r->id);
}

// The copy worker: takes gathered results, copies them to new (pinned) host
// arrays on its own stream, returns the device buffers to the pool.
void copy_worker(kgs_server *s)
{
    // without the server's device current no copy may run: every job then
    // fails with this error
    const hipError_t dev = hipSetDevice(s->device);
    for (;;) {
        CopyJob job;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_jobs.wait(lk, [&] { return s->stop || !s->jobs.empty(); });
            if (s->jobs.empty()) return;  // stop requested and nothing left
            job = s->jobs.front();
            s->jobs.pop_front();
        }
        HostArray h = dev == hipSuccess ? host_array(s->pinned, job.n) : HostArray();
        hipError_t e = dev != hipSuccess ? dev
                       : h ? hipMemcpyAsync(h.get(), job.src, job.n * sizeof(double),
                                            hipMemcpyDeviceToHost, s->copy_out)
                           : hipErrorOutOfMemory;
        if (e == hipSuccess) e = hipStreamSynchronize(s->copy_out);
        const hipError_t freed = dev == hipSuccess ? hipFreeAsync(job.src, s->copy_out) : dev;
        if (e != hipSuccess) h.reset();
        std::lock_guard<std::mutex> lk(s->mu);
        s->release_err(freed);
        s->done.push_back(CopyDone{job.id, std::move(h), e, now_s() - s->t0});
        --s->in_flight;
        s->cv_done.notify_all();
    }
}

// The final accounting of a retired request.
void end_retire(kgs_server *s, Request *r, int32_t status, double t_done)
{
    r->retiring = false;
    r->copying = false;
    s->used -= r->bytes;
    if (r->dropped) {
        r->host.reset();  // already reported as cancelled
        return;
    }
    r->state = status == KGS_OK ? KGS_REQ_DONE : KGS_REQ_FAILED;
    r->status = status;
    r->t_done = t_done;
}

// A retirement whose event has passed: energies from the pinned slot, the
// gathered result handed to the copy worker (or dropped).
void start_copy(kgs_server *s, Request *r)
{
    if (r->slot >= 0) {
        // h^dim as kgs_energy forms it
        const double h = (r->cfg.hi - r->cfg.lo) / r->cfg.n;
        double hd = 1.0;
        for (int a = 0; a < r->cfg.dim; ++a) hd *= h;
        const double *h0 = slot_host(s, r->slot, 0), *h1 = slot_host(s, r->slot, 1);
        r->e0 = hd * (h0[0] + h0[1]);
        r->e1 = hd * (h1[0] + h1[1]);
        s->free_slots.push_back(r->slot);
        r->slot = -1;
    }
    give_event(s, r->ev);
    r->ev = nullptr;
    if (r->status == KGS_OK && !(std::isfinite(r->e0) && std::isfinite(r->e1))) {
        r->status = KGS_ENONFINITE;
        r->err = "energy is not finite";
    }
    if (r->status != KGS_OK || r->dropped || !r->staging) {
        free_request_memory(s, r);
        end_retire(s, r, r->status, now_s() - s->t0);
        return;
    }
    CopyJob job{r->id, r->staging, 4 * static_cast<size_t>(r->points)};
    r->staging = nullptr;  // the worker returns it to the pool
    r->copying = true;
    std::lock_guard<std::mutex> lk(s->mu);
    s->jobs.push_back(job);
    ++s->in_flight;
    s->cv_jobs.notify_one();
}

// Retirements: start the copies of those whose events have passed and
// complete those whose copies are done; with `wait`, all of them.
void collect(kgs_server *s, bool wait)
{
    for (int64_t id : s->retiring) {
        Request *r = s->reqs[id].get();
        if (r->copying) continue;
        hipError_t q = hipSuccess;
        if (r->ev) q = wait ? hipEventSynchronize(r->ev) : hipEventQuery(r->ev);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess && r->status == KGS_OK) {
            r->status = KGS_EDEVICE;
            r->err = std::string("retirement event: ") + hipGetErrorName(q);
        }
        start_copy(s, r);
    }
    std::deque<CopyDone> done;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        if (wait) s->cv_done.wait(lk, [&] { return s->in_flight == 0; });
        done.swap(s->done);
    }
    for (CopyDone &d : done) {
        Request *r = s->reqs[d.id].get();
        int32_t status = r->status;
        if (d.status != hipSuccess) {
            status = status_of(d.status);
            r->err = std::string("result copy: ") + hipGetErrorName(d.status);
        }
        r->host = std::move(d.host);
        end_retire(s, r, status, d.t);
    }
    std::vector<int64_t> still;
    for (int64_t id : s->retiring)
        if (s->reqs[id]->retiring) still.push_back(id);
    s->retiring.swap(still);
}

// ---- small lane ---------------------------------------------------------

// One resident launch per (dimension, precision) over the newly admitted
// small requests, each taking all of its steps; then their retirement.
int run_small(kgs_server *s)
{
    std::vector<int64_t> &ids = s->running[LANE_SMALL];
    if (ids.empty()) return KGS_OK;
    std::map<int, std::vector<Request *>> cls;
    for (int64_t id : ids) {
        Request *r = s->reqs[id].get();
        cls[r->cfg.dim * 2 + r->cfg.precision].push_back(r);
    }
    size_t bytes = 0;
    for (auto &kv : cls)
        bytes += align_up(kv.second.size() * sizeof(kgs::ResidentMember), 256) +
                 align_up(kv.second.size() * sizeof(int64_t), 256);
    int rc = KGS_OK;
    Ring::Slot *sl = ring_take(s, LANE_SMALL, bytes, rc);
    if (!sl) return rc;
    struct Launch {
        int dim, prec, nm;
        size_t mem_off, steps_off;
        int64_t max_count;
    };
    std::vector<Launch> launches;
    size_t off = 0;
    for (auto &kv : cls) {
        Launch L;
        L.dim = kv.first / 2;
        L.prec = kv.first % 2;
        L.nm = static_cast<int>(kv.second.size());
        L.mem_off = off;
        L.max_count = 0;
        auto *m = reinterpret_cast<kgs::ResidentMember *>(sl->h + off);
        for (int i = 0; i < L.nm; ++i) {
            const kgs_sim *x = kv.second[i]->sim;
            std::memset(&m[i], 0, sizeof(m[i]));
            m[i].state = x->state;
            m[i].stride = x->geo.stride;
            m[i].steps = kv.second[i]->nsteps;
            m[i].k = x->coef;
            m[i].n = x->geo.n;
            m[i].count = static_cast<int>(x->geo.count);
            L.max_count = std::max<int64_t>(L.max_count, x->geo.count);
        }
        off = align_up(off + L.nm * sizeof(kgs::ResidentMember), 256);
        L.steps_off = off;
        auto *k = reinterpret_cast<int64_t *>(sl->h + off);
        for (int i = 0; i < L.nm; ++i) k[i] = kv.second[i]->nsteps;
        off = align_up(off + L.nm * sizeof(int64_t), 256);
        launches.push_back(L);
    }
    hipError_t e = hipMemcpyAsync(sl->d, sl->h, off, hipMemcpyHostToDevice, s->lane[LANE_SMALL]);
    for (const Launch &L : launches) {
        if (e != hipSuccess) break;
        kgs::ResidentMember none;
        std::memset(&none, 0, sizeof(none));
        e = kgs::launch_resident(L.dim, L.prec, none,
                                 reinterpret_cast<const kgs::ResidentMember *>(sl->d + L.mem_off),
                                 reinterpret_cast<const int64_t *>(sl->d + L.steps_off), 0, L.nm,
                                 L.max_count, s->lane[LANE_SMALL]);
    }
    const hipError_t e2 = ring_done(s, LANE_SMALL, sl);
    if (e == hipSuccess) e = e2;
    for (int64_t id : ids) {
        Request *r = s->reqs[id].get();
        r->done_steps = r->nsteps;
        if (e != hipSuccess) {
            r->status = status_of(e);
            r->err = std::string("resident kernel launch: ") + hipGetErrorName(e);
        }
        start_retire(s, r);
    }
    ids.clear();
    return KGS_OK;
}

// ---- big lane -----------------------------------------------------------

// 2-D requests of one precision taking k >= 2 steps this round: launches of
// 2 steps (and of 1 step where needed to keep their number even, so that
// every request ends in its own buffer) over all of them, of the
// y-streaming kernel, or of the tiled kernel when the group is too small for
// long streaming chunks and every grid is below n = 2048, then the closing
// red sweep as one batched sweep.
int run_stream2d(kgs_server *s, int prec, int64_t k, const std::vector<Request *> &rs)
{
    const int nm = static_cast<int>(rs.size());
    int chunk = 64;
    auto tasks = [&](int ch) {
        int64_t t = 0;
        for (const Request *r : rs) t += kgs::stream2d_tasks(r->sim->geo.n, ch);
        return t;
    };
    while (chunk > 8 && tasks(chunk) < 2048) chunk /= 2;
    // tiles when the group is too small for long streaming chunks
    bool tile = chunk < 32;
    std::vector<int> ns(static_cast<size_t>(nm));
    for (int i = 0; i < nm; ++i) {
        ns[i] = rs[i]->sim->geo.n;
        if (ns[i] >= 2048) tile = false;
    }
    int ty = 0, tx = 0;
    kgs::tile2d_group_shape(ns.data(), nm, ty, tx);
    const size_t s2_bytes = align_up(3 * nm * sizeof(kgs::Stream2dMember), 256);
    const size_t bm_bytes = align_up(nm * sizeof(kgs::BatchMember), 256);
    int rc = KGS_OK;
    Ring::Slot *sl = ring_take(s, LANE_BIG, s2_bytes + bm_bytes, rc);
    if (!sl) return rc;
    auto *d = reinterpret_cast<kgs::Stream2dMember *>(sl->h);
    auto *bm = reinterpret_cast<kgs::BatchMember *>(sl->h + s2_bytes);
    const int bb = kgs::batch_block();
    int64_t tb = 0, blocks = 0;
    for (int i = 0; i < nm; ++i) {
        const kgs_sim *x = rs[i]->sim;
        for (int v = 0; v < 3; ++v) {  // [first launch | even | odd]
            kgs::Stream2dMember &m = d[v * nm + i];
            std::memset(&m, 0, sizeof(m));
            m.in = v == 2 ? x->state2 : x->state;
            m.out = v == 2 ? x->state : x->state2;
            m.stride = x->geo.stride;
            m.task_begin = tb;
            m.k = x->coef;
            m.n = x->geo.n;
            m.chunk = tile ? ty : chunk;
            m.tiles_x = tile ? kgs::tile2d_tiles_x(x->geo.n, tx) : kgs::stream2d_tiles_x(x->geo.n);
            m.first = v == 0 ? 1 : 0;
        }
        tb += tile ? kgs::tile2d_member_tiles(x->geo.n, ty, tx) : kgs::stream2d_tasks(x->geo.n, chunk);
        std::memset(&bm[i], 0, sizeof(bm[i]));
        bm[i].state = x->state;
        bm[i].stride = x->geo.stride;
        bm[i].count = x->geo.count;
        bm[i].block_begin = blocks;
        bm[i].k = x->coef;
        bm[i].n = x->geo.n;
        blocks += (x->geo.count + bb - 1) / bb;
    }
    hipStream_t st = s->lane[LANE_BIG];
    hipError_t e = hipMemcpyAsync(sl->d, sl->h, s2_bytes + bm_bytes, hipMemcpyHostToDevice, st);
    const int64_t a = k / 2, r = k % 2, split = (a + r) % 2;
    std::vector<int> stages(static_cast<size_t>(a - split), 4);
    for (int64_t i = 0; i < 2 * split + r; ++i) stages.push_back(2);
    const auto *dd = reinterpret_cast<const kgs::Stream2dMember *>(sl->d);
    kgs::Stream2dMember none;
    std::memset(&none, 0, sizeof(none));
    for (size_t i = 0; i < stages.size() && e == hipSuccess; ++i) {
        const kgs::Stream2dMember *list = dd + (i == 0 ? 0 : (i % 2 ? 2 * nm : nm));
        e = tile ? kgs::launch_tile2d_list(prec, stages[i], ty, tx, none, list, nm, tb, st,
                                           i == 0 ? 1 : 0)
                 : kgs::launch_stream2d(prec, stages[i], none, list, nm, tb, st);
    }
    if (e == hipSuccess && blocks > 0x7fffffff) e = hipErrorInvalidValue;
    if (e == hipSuccess)
        e = kgs::launch_batch_sweep(2, prec, reinterpret_cast<const kgs::BatchMember *>(sl->d + s2_bytes),
                                    nm, blocks, nullptr, 0, kgs::PASS_R_ADJ, st);
    const hipError_t e2 = ring_done(s, LANE_BIG, sl);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess)
        for (Request *q : rs) {
            q->status = status_of(e);
            q->err = std::string("2-D tiled/streaming launch: ") + hipGetErrorName(e);
        }
    return KGS_OK;
}

// Whether a 3-D grid fits a member-list launch with the default tile of
// its precision (chunk 8, the shortest the planner takes).
bool list_fits(const kgs::Geometry &g, int elem_bytes)
{
    int tx = 0, ty = 0;
    kgs::stream3d_list_tile(elem_bytes, &tx, &ty);
    return kgs::stream3d_list_ok(g, 8, elem_bytes, tx, ty);
}

// 3-D requests of one precision taking k >= 2 steps this round: the same
// launch sequence as run_stream2d with the z-streaming kernel's member-list
// launch over all of them (the tile and plane chunk estimated to end the
// launch first), then the closing red sweep as one batched sweep.
int run_stream3d(kgs_server *s, int prec, int64_t k, const std::vector<Request *> &rs)
{
    const int nm = static_cast<int>(rs.size());
    const int eb = prec == KGS_FP64 ? 8 : 4;
    std::vector<int> sizes;
    for (const Request *r : rs) sizes.push_back(r->sim->geo.n);
    int tx = 0, ty = 0, chunk = 0;
    kgs::stream3d_list_plan(sizes.data(), nm, eb, &tx, &ty, &chunk);
    for (const Request *r : rs)
        if (!kgs::stream3d_list_ok(r->sim->geo, chunk, eb, tx, ty)) {
            // every request was admitted for the default tile
            kgs::stream3d_list_tile(eb, &tx, &ty);
            chunk = kgs::stream3d_chunk(sizes.data(), nm, tx, ty, kgs::device_cus());
            break;
        }
    const size_t s3_bytes = align_up(3 * nm * sizeof(kgs::Stream2dMember), 256);
    const size_t bm_bytes = align_up(nm * sizeof(kgs::BatchMember), 256);
    int rc = KGS_OK;
    Ring::Slot *sl = ring_take(s, LANE_BIG, s3_bytes + bm_bytes, rc);
    if (!sl) return rc;
    auto *d = reinterpret_cast<kgs::Stream2dMember *>(sl->h);
    auto *bm = reinterpret_cast<kgs::BatchMember *>(sl->h + s3_bytes);
    const int bb = kgs::batch_block();
    int64_t tb = 0, blocks = 0;
    for (int i = 0; i < nm; ++i) {
        const kgs_sim *x = rs[i]->sim;
        for (int v = 0; v < 3; ++v) {  // [first launch | even | odd]
            kgs::Stream2dMember &m = d[v * nm + i];
            std::memset(&m, 0, sizeof(m));
            m.in = v == 2 ? x->state2 : x->state;
            m.out = v == 2 ? x->state : x->state2;
            m.stride = x->geo.stride;
            m.task_begin = tb;
            m.k = x->coef;
            m.n = x->geo.n;
            m.chunk = kgs::member_chunk(x->geo.n, chunk);
            m.first = v == 0 ? 1 : 0;
        }
        tb += kgs::stream3d_member_items(x->geo.n, kgs::member_chunk(x->geo.n, chunk), tx, ty);
        std::memset(&bm[i], 0, sizeof(bm[i]));
        bm[i].state = x->state;
        bm[i].stride = x->geo.stride;
        bm[i].count = x->geo.count;
        bm[i].block_begin = blocks;
        bm[i].k = x->coef;
        bm[i].n = x->geo.n;
        blocks += (x->geo.count + bb - 1) / bb;
    }
    hipStream_t st = s->lane[LANE_BIG];
    hipError_t e = hipMemcpyAsync(sl->d, sl->h, s3_bytes + bm_bytes, hipMemcpyHostToDevice, st);
    const int64_t a = k / 2, r = k % 2, split = (a + r) % 2;
    std::vector<int> stages(static_cast<size_t>(a - split), 4);
    for (int64_t i = 0; i < 2 * split + r; ++i) stages.push_back(2);
    const auto *dd = reinterpret_cast<const kgs::Stream2dMember *>(sl->d);
    for (size_t i = 0; i < stages.size() && e == hipSuccess; ++i) {
        const kgs::Stream2dMember *list = dd + (i == 0 ? 0 : (i % 2 ? 2 * nm : nm));
        e = kgs::launch_stream3d_list(prec, stages[i], tx, ty, list, nm, tb, i == 0, st);
    }
    if (e == hipSuccess && blocks > 0x7fffffff) e = hipErrorInvalidValue;
    if (e == hipSuccess)
        e = kgs::launch_batch_sweep(3, prec, reinterpret_cast<const kgs::BatchMember *>(sl->d + s3_bytes),
                                    nm, blocks, nullptr, 0, kgs::PASS_R_ADJ, st);
    const hipError_t e2 = ring_done(s, LANE_BIG, sl);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess)
        for (Request *q : rs) {
            q->status = status_of(e);
            q->err = std::string("3-D streaming launch: ") + hipGetErrorName(e);
        }
    return KGS_OK;
}

// One round: the requests with the least remaining work first, up to the
// round's work quantum (at least one request).
int run_big(kgs_server *s)
{
    std::vector<int64_t> &ids = s->running[LANE_BIG];
    if (ids.empty()) return KGS_OK;
    const int64_t spr = s->cfg.steps_per_round > 0 ? s->cfg.steps_per_round : INT64_MAX;
    const int64_t quantum = s->cfg.round_work > 0 ? s->cfg.round_work : kDefaultRoundWork;
    std::vector<Request *> order;
    for (int64_t id : ids) order.push_back(s->reqs[id].get());
    std::stable_sort(order.begin(), order.end(), [](const Request *a, const Request *b) {
        return a->points * (a->nsteps - a->done_steps) < b->points * (b->nsteps - b->done_steps);
    });
    std::vector<std::pair<Request *, int64_t>> pick;
    int64_t work = 0;
    for (Request *r : order) {
        const int64_t k = std::min(spr, r->nsteps - r->done_steps);
        if (!pick.empty() && work + r->points * k > quantum) break;
        pick.emplace_back(r, k);
        work += r->points * k;
    }
    hipStream_t st = s->lane[LANE_BIG];
    // 2-D and 3-D streaming grids taking >= 2 steps streamed together by
    // (precision, steps); 3-D streaming grids taking 1 step with their own
    // kernel; the rest batched by (dim, precision)
    std::map<int, std::vector<std::pair<Request *, int64_t>>> cls;
    std::map<std::pair<int, int64_t>, std::vector<Request *>> s2, s3;
    for (auto &pk : pick) {
        Request *r = pk.first;
        if (pk.second == 0) continue;
        if (r->cfg.dim == 2 && pk.second >= 2) {
            if (kgs::sim_ensure_state2(r->sim) == KGS_OK) {
                s2[{r->cfg.precision, pk.second}].push_back(r);
                continue;
            }
            r->sim->err.clear();  // no second buffer: sweeps instead
        }
        if (r->cfg.dim == 3 && r->sim->tuning.kernel == KGS_KERNEL_STREAM && pk.second >= 2 &&
            list_fits(r->sim->geo, r->cfg.precision == KGS_FP64 ? 8 : 4) &&
            r->sim->state2) {
            s3[{r->cfg.precision, pk.second}].push_back(r);
            continue;
        }
        if (r->cfg.dim == 3 && r->sim->tuning.kernel == KGS_KERNEL_STREAM) {
            if (kgs_step(r->sim, pk.second) != KGS_OK ||
                kgs::sim_close(r->sim, r->sim->stream) != KGS_OK) {
                r->status = KGS_EDEVICE;
                r->err = kgs_last_error(r->sim);
            }
        } else {
            cls[r->cfg.dim * 2 + r->cfg.precision].push_back(pk);
        }
    }
    for (auto &kv : s2) {
        const int rc = run_stream2d(s, kv.first.first, kv.first.second, kv.second);
        if (rc != KGS_OK) return rc;
    }
    for (auto &kv : s3) {
        const int rc = run_stream3d(s, kv.first.first, kv.first.second, kv.second);
        if (rc != KGS_OK) return rc;
    }
    if (!cls.empty()) {
        const int bb = kgs::batch_block();
        size_t bytes = 0;
        for (auto &kv : cls) {
            int64_t kmax = 0;
            for (auto &pk : kv.second) kmax = std::max(kmax, pk.second);
            bytes += align_up(kv.second.size() * sizeof(kgs::BatchMember), 256) +
                     align_up((2 * kmax + 1) * kv.second.size() * sizeof(int), 256);
        }
        int rc = KGS_OK;
        Ring::Slot *sl = ring_take(s, LANE_BIG, bytes, rc);
        if (!sl) return rc;
        struct Launch {
            int dim, prec, nm;
            size_t mem_off, kinds_off;
            int64_t blocks, launches;
        };
        std::vector<Launch> launches;
        size_t off = 0;
        for (auto &kv : cls) {
            Launch L;
            L.dim = kv.first / 2;
            L.prec = kv.first % 2;
            L.nm = static_cast<int>(kv.second.size());
            L.mem_off = off;
            auto *m = reinterpret_cast<kgs::BatchMember *>(sl->h + off);
            int64_t blocks = 0, kmax = 0;
            for (int i = 0; i < L.nm; ++i) {
                const kgs_sim *x = kv.second[i].first->sim;
                std::memset(&m[i], 0, sizeof(m[i]));
                m[i].state = x->state;
                m[i].stride = x->geo.stride;
                m[i].count = x->geo.count;
                m[i].block_begin = blocks;
                m[i].k = x->coef;
                m[i].n = x->geo.n;
                blocks += (x->geo.count + bb - 1) / bb;
                kmax = std::max(kmax, kv.second[i].second);
            }
            L.blocks = blocks;
            off = align_up(off + L.nm * sizeof(kgs::BatchMember), 256);
            // kinds[launch][member]: red 0, blue 0, red 1, ..., blue k-1, red k
            L.launches = 2 * kmax + 1;
            L.kinds_off = off;
            auto *kinds = reinterpret_cast<int *>(sl->h + off);
            for (int64_t l = 0; l < L.launches; ++l) {
                const int64_t i = l / 2;
                const bool red = (l % 2) == 0;
                for (int j = 0; j < L.nm; ++j) {
                    const int64_t k = kv.second[j].second;
                    int kind = -1;
                    if (red) {
                        if (i == 0) kind = kgs::PASS_R_BASE;
                        else if (i < k) kind = kgs::PASS_R_ADJ_BASE;
                        else if (i == k) kind = kgs::PASS_R_ADJ;
                    } else if (i < k) {
                        kind = kgs::PASS_B_FULL;
                    }
                    kinds[l * L.nm + j] = kind;
                }
            }
            off = align_up(off + L.launches * L.nm * sizeof(int), 256);
            launches.push_back(L);
        }
        hipError_t e = hipMemcpyAsync(sl->d, sl->h, off, hipMemcpyHostToDevice, st);
        for (const Launch &L : launches) {
            if (e == hipSuccess && L.blocks > 0x7fffffff) e = hipErrorInvalidValue;
            for (int64_t l = 0; l < L.launches && e == hipSuccess; ++l)
                e = kgs::launch_batch_sweep(
                    L.dim, L.prec, reinterpret_cast<const kgs::BatchMember *>(sl->d + L.mem_off),
                    L.nm, L.blocks, reinterpret_cast<const int *>(sl->d + L.kinds_off),
                    static_cast<int>(l), -1, st);
        }
        const hipError_t e2 = ring_done(s, LANE_BIG, sl);
        if (e == hipSuccess) e = e2;
        if (e != hipSuccess)
            for (auto &kv : cls)
                for (auto &pk : kv.second) {
                    pk.first->status = status_of(e);
                    pk.first->err = std::string("batched sweep launch: ") + hipGetErrorName(e);
                }
    }
    for (auto &pk : pick) pk.first->done_steps += pk.second;
    std::vector<int64_t> still;
    for (int64_t id : ids) {
        Request *r = s->reqs[id].get();
        if (r->done_steps >= r->nsteps || r->status != KGS_OK) start_retire(s, r);
        else still.push_back(id);
    }
    ids.swap(still);
    return KGS_OK;
}

// At most kMaxAhead rounds queued on each lane.
int throttle(kgs_server *s, const bool used[2])
{
    for (int l = 0; l < 2; ++l) {
        if (!used[l]) continue;
        hipEvent_t e = take_event(s);
        if (!e) return sfail(s, KGS_EDEVICE, "hipEventCreate");
        const hipError_t r = hipEventRecord(e, s->lane[l]);
        if (r != hipSuccess) {
            give_event(s, e);
            return shipfail(s, r, "hipEventRecord (round)");
        }
        s->ahead.push_back(e);
    }
    while (s->ahead.size() > 2 * kMaxAhead) {
        hipEvent_t e = s->ahead.front();
        s->ahead.pop_front();
        const hipError_t q = hipEventSynchronize(e);
        give_event(s, e);
        if (q != hipSuccess) return shipfail(s, q, "hipEventSynchronize (round)");
    }
    return KGS_OK;
}

int round_once(kgs_server *s)
{
    collect(s, false);
    if (s->submitted) {
        // the lanes read device inputs copied on the caller's stream
        hipError_t e = hipEventRecord(s->ev_submit, s->user);
        for (int l = 0; l < 2 && e == hipSuccess; ++l)
            e = hipStreamWaitEvent(s->lane[l], s->ev_submit, 0);
        if (e != hipSuccess) return shipfail(s, e, "input ordering");
        s->submitted = false;
    }
    admit(s);
    const bool used[2] = {!s->running[LANE_BIG].empty(), !s->running[LANE_SMALL].empty()};
    int rc = run_small(s);
    if (rc == KGS_OK) rc = run_big(s);
    if (rc != KGS_OK) return rc;
    if (used[0] || used[1]) {
        s->rounds++;
        rc = throttle(s, used);
        if (rc != KGS_OK) return rc;
        collect(s, false);
    } else {
        collect(s, true);  // nothing left to enqueue: wait for the retirements
    }
    return KGS_OK;
}

}  // namespace

extern "C" {

const char *kgs_server_last_error(const kgs_server *s) { return s ? s->err.c_str() : g_srv_err.c_str(); }

int kgs_server_create(const kgs_server_config *cfg, void *stream, kgs_server **out)
{
    KGS_TRACE("kgs_server_create");
    if (!out) return sfail(nullptr, KGS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg || cfg->budget_bytes <= 0 || cfg->max_active < 0 || cfg->steps_per_round < 0 ||
        cfg->round_work < 0 || cfg->reserved[0] || cfg->reserved[1])
        return sfail(nullptr, KGS_EINVAL, "invalid server configuration");
    kgs_server *s = new (std::nothrow) kgs_server();
    if (!s) return sfail(nullptr, KGS_ENOMEM, "host allocation failed");
    s->cfg = *cfg;
    s->user = static_cast<hipStream_t>(stream);
    hipError_t e = hipGetDevice(&s->device);
    int pools = 0;
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, s->device);
    if (e == hipSuccess && !pools) e = hipErrorNotSupported;
    if (e == hipSuccess) e = take_streams(s);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_submit, hipEventDisableTiming);
    if (e == hipSuccess) {
        hipMemPoolProps props;
        std::memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = s->device;
        e = hipMemPoolCreate(&s->pool, &props);
    }
    if (e == hipSuccess) {
        // keep freed blocks for reuse rather than releasing them at every sync
        uint64_t keep = UINT64_MAX;
        e = hipMemPoolSetAttribute(s->pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    if (e != hipSuccess) {
        const std::string msg = std::string("server set-up: ") + hipGetErrorName(e);
        kgs_server_free(s);
        return sfail(nullptr, KGS_EDEVICE, msg);
    }
    s->t0 = now_s();
    try {
        s->copier = std::thread(copy_worker, s);
    } catch (...) {
        kgs_server_free(s);
        return sfail(nullptr, KGS_ENOMEM, "could not start the copy thread");
    }
    *out = s;
    return KGS_OK;
}

int kgs_server_submit(kgs_server *s, const kgs_config *cfg, const double *psi_re,
                      const double *psi_im, const double *u, const double *v_t, int32_t mem,
                      int64_t nsteps, int64_t *id)
{
    KGS_TRACE("kgs_server_submit");
    if (!s || !id) return sfail(s, KGS_EINVAL, "server or id is NULL");
    *id = 0;
    if (!cfg || !psi_re || !psi_im || !u || !v_t) return sfail(s, KGS_EINVAL, "NULL argument");
    if (mem != KGS_HOST && mem != KGS_DEVICE) return sfail(s, KGS_EINVAL, "bad memory kind");
    if (nsteps < 0) return sfail(s, KGS_EINVAL, "nsteps must be >= 0");
    const int64_t bytes = kgs_required_bytes(cfg);
    if (bytes <= 0) {
        // reuse kgs_init's validation for the message and status
        kgs_sim *tmp = nullptr;
        int rc = kgs_init(cfg, psi_re, psi_im, u, v_t, mem, s->user, &tmp);
        if (tmp) kgs_free(tmp);
        return sfail(s, rc != KGS_OK ? rc : KGS_EINVAL, kgs_last_error(nullptr));
    }
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return sfail(s, KGS_ENOMEM, "host allocation failed");
    r->id = s->next_id++;
    r->cfg = *cfg;
    r->nsteps = nsteps;
    r->points = 1;
    for (int a = 0; a < cfg->dim; ++a) r->points *= cfg->n;
    const size_t nb = static_cast<size_t>(r->points) * sizeof(double);
    r->bytes = bytes + static_cast<int64_t>(4 * nb);  // state + gathered result
    // 2-D grids beyond one workgroup stream in the big lane: a second buffer
    const int dk = kgs::default_kernel(*cfg);
    if (cfg->dim == 2 && dk != KGS_KERNEL_RESIDENT && dk != KGS_KERNEL_STREAM &&
        dk != KGS_KERNEL_TILE)
        r->bytes += kgs::state_bytes(*cfg);
    const double *src[4] = {psi_re, psi_im, u, v_t};
    if (mem == KGS_HOST) {
        r->host = host_array(s->pinned, 4 * static_cast<size_t>(r->points));
        if (!r->host) return sfail(s, KGS_ENOMEM, "host allocation failed");
        for (int f = 0; f < 4; ++f) std::memcpy(r->host.get() + f * r->points, src[f], nb);
    } else {
        // device inputs: a pooled copy ordered on the caller's stream, held
        // until admission (reported by kgs_server_stats, outside the budget)
        hipError_t e = hipMallocFromPoolAsync(reinterpret_cast<void **>(&r->dev_in), 4 * nb,
                                              s->pool, s->user);
        for (int f = 0; f < 4 && e == hipSuccess; ++f)
            e = hipMemcpyAsync(r->dev_in + f * r->points, src[f], nb, hipMemcpyDeviceToDevice,
                               s->user);
        if (e != hipSuccess) {
            free_request_memory(s, r.get());
            return shipfail(s, e, "device copy of the initial state");
        }
        s->queued_dev += static_cast<int64_t>(4 * nb);
        s->submitted = true;
    }
    r->t_submit = now_s() - s->t0;
    *id = r->id;
    s->queue.push_back(r->id);
    s->reqs[r->id] = std::move(r);
    return KGS_OK;
}

int kgs_server_run(kgs_server *s, int32_t rounds, int32_t *n_running, int32_t *n_queued)
{
    KGS_TRACE("kgs_server_run");
    if (!s || rounds < 0) return sfail(s, KGS_EINVAL, "bad arguments");
    if (hipSetDevice(s->device) != hipSuccess) return sfail(s, KGS_EDEVICE, "hipSetDevice failed");
    for (int32_t i = 0; i < rounds; ++i) {
        int rc = round_once(s);
        if (rc != KGS_OK) return rc;
        if (total_running(s) == 0 && s->queue.empty()) break;
    }
    if (n_running) *n_running = static_cast<int32_t>(total_running(s));
    if (n_queued) *n_queued = static_cast<int32_t>(s->queue.size());
    return KGS_OK;
}

int kgs_server_poll(const kgs_server *s, int64_t id, kgs_request_info *info)
{
    if (!s || !info) return KGS_EINVAL;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return KGS_EINVAL;
    const Request *r = it->second.get();
    std::memset(info, 0, sizeof(*info));
    info->state = r->state;
    info->status = r->status;
    info->steps_done = r->done_steps;
    info->nsteps = r->nsteps;
    info->device_bytes = r->bytes;
    info->t_submit = r->t_submit;
    info->t_admit = r->t_admit;
    info->t_done = r->t_done;
    info->energy_start = r->e0;
    info->energy_end = r->e1;
    return KGS_OK;
}

int kgs_server_result(kgs_server *s, int64_t id, double *psi_re, double *psi_im, double *u,
                      double *v_t, int32_t mem)
{
    KGS_TRACE("kgs_server_result");
    if (!s) return sfail(nullptr, KGS_EINVAL, "server is NULL");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return sfail(s, KGS_EINVAL, "unknown request");
    Request *r = it->second.get();
    if (r->state != KGS_REQ_DONE || !r->host) return sfail(s, KGS_EINVAL, "request has no result");
    if (!psi_re || !psi_im || !u || !v_t || (mem != KGS_HOST && mem != KGS_DEVICE))
        return sfail(s, KGS_EINVAL, "bad output arguments");
    const size_t nb = static_cast<size_t>(r->points) * sizeof(double);
    double *dst[4] = {psi_re, psi_im, u, v_t};
    for (int f = 0; f < 4; ++f) {
        const double *src = r->host.get() + f * r->points;
        if (mem == KGS_HOST) std::memcpy(dst[f], src, nb);
        else if (hipMemcpy(dst[f], src, nb, hipMemcpyHostToDevice) != hipSuccess)
            return sfail(s, KGS_EDEVICE, "copy of the result failed");
    }
    return KGS_OK;
}

int kgs_server_release(kgs_server *s, int64_t id)
{
    if (!s) return KGS_EINVAL;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return sfail(s, KGS_EINVAL, "unknown request");
    Request *r = it->second.get();
    if (r->state == KGS_REQ_RUNNING || r->retiring)
        return sfail(s, KGS_EINVAL, "request is still on the device");
    if (r->state == KGS_REQ_QUEUED) {
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), id));
        if (r->dev_in) s->queued_dev -= 4 * r->points * static_cast<int64_t>(sizeof(double));
    }
    free_request_memory(s, r);
    s->reqs.erase(it);
    return KGS_OK;
}

int kgs_server_cancel(kgs_server *s, int64_t id)
{
    KGS_TRACE("kgs_server_cancel");
    if (!s) return KGS_EINVAL;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return sfail(s, KGS_EINVAL, "unknown request");
    Request *r = it->second.get();
    if (r->state == KGS_REQ_QUEUED) {
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), id));
        if (r->dev_in) s->queued_dev -= 4 * r->points * static_cast<int64_t>(sizeof(double));
        free_request_memory(s, r);
        r->host.reset();
        finish(s, r, KGS_REQ_CANCELLED, KGS_OK);
        return KGS_OK;
    }
    if (r->state != KGS_REQ_RUNNING) return sfail(s, KGS_EINVAL, "request already finished");
    if (r->retiring) {
        // its device work ends at the next collection; the result is dropped
        r->dropped = true;
        finish(s, r, KGS_REQ_CANCELLED, KGS_OK);
        return KGS_OK;
    }
    // work already queued for the request stays ordered before its memory's return
    std::vector<int64_t> &lane = s->running[r->lane];
    lane.erase(std::find(lane.begin(), lane.end(), id));
    free_request_memory(s, r);
    r->slot = -1;  // its start energy may still be in flight into the slot: not reused
    s->used -= r->bytes;
    finish(s, r, KGS_REQ_CANCELLED, KGS_OK);
    return KGS_OK;
}

int kgs_server_stats(const kgs_server *s, kgs_server_stats_t *st)
{
    if (!s || !st) return KGS_EINVAL;
    std::memset(st, 0, sizeof(*st));
    st->device_bytes_used = s->used;
    st->queued_input_bytes = s->queued_dev;
    st->running = static_cast<int32_t>(total_running(s));
    st->queued = static_cast<int32_t>(s->queue.size());
    st->rounds = s->rounds;
    st->now = now_s() - s->t0;
    return KGS_OK;
}

int kgs_server_free(kgs_server *s)
{
    KGS_TRACE("kgs_server_free");
    if (!s) return KGS_OK;
    int rc = KGS_OK;
    if (hipSetDevice(s->device) != hipSuccess) rc = KGS_EDEVICE;
    collect(s, true);
    if (s->copier.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_jobs.notify_all();
        s->copier.join();
    }
    for (auto &kv : s->reqs) free_request_memory(s, kv.second.get());
    for (hipStream_t st : {s->lane[0], s->lane[1], s->copy, s->copy_out})
        if (st && hipStreamSynchronize(st) != hipSuccess) rc = KGS_EDEVICE;
    s->done.clear();
    s->reqs.clear();  // their host arrays return to the pinned cache
    s->pinned.release(s->release_err);
    if (hipStreamSynchronize(s->user) != hipSuccess) rc = KGS_EDEVICE;
    for (hipEvent_t e : s->ahead) give_event(s, e);
    for (hipEvent_t e : s->spare_events)
        s->release_err(hipEventDestroy(e));
    for (auto &g : s->ring)
        for (auto &sl : g.slots) {
            if (sl.h) s->release_err(hipHostFree(sl.h));
            if (sl.d) s->release_err(hipFree(sl.d));
            if (sl.ev) s->release_err(hipEventDestroy(sl.ev));
        }
    for (auto &c : s->energy) {
        if (c.d) s->release_err(hipFree(c.d));
        if (c.h) s->release_err(hipHostFree(c.h));
    }
    if (s->ev_submit) s->release_err(hipEventDestroy(s->ev_submit));
    give_streams(s);
    if (s->pool && hipMemPoolDestroy(s->pool) != hipSuccess) rc = KGS_EDEVICE;
    if (!s->release_err.ok()) rc = KGS_EDEVICE;
    delete s;
    return rc;
}

}  // extern "C"
