// Batches of simulations: many independent DP-AVF2 runs of uneven sizes
// advanced together, one batched launch per colour sweep and per
// (dimension, storage precision) class instead of one launch per simulation,
// optionally with the whole step loop captured in a hipGraph and replayed.
// Members small enough for one workgroup form classes of their own that the
// resident kernel advances through a whole run in a single launch (one
// workgroup per member).  Uniform runs of 2-D classes use the 2-D streaming
// kernel, and of 3-D classes the z-streaming kernel's member-list launch:
// two steps per launch over all members, between each member's two state
// buffers, with an even number of launches so that every member ends in
// its own buffer.
#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "kgs.h"
#include "kgs_trace.h"
#include "kgs_internal.h"
#include "kgs_plan.h"
#include "kgs_sim.h"

namespace {

struct BatchClass {
    int dim = 0, precision = 0;
    bool resident = false;     // advanced by the resident kernel
    std::vector<int> members;  // indices into kgs_batch::sims
    kgs::BatchMember *d_members = nullptr;    // sweep classes
    kgs::BatchMember *h_members = nullptr;    // pinned staging
    kgs::ResidentMember *d_res = nullptr;     // resident classes
    kgs::ResidentMember *h_res = nullptr;     // pinned staging
    int64_t blocks = 0;     // sweep classes: workgroups per launch
    int64_t max_count = 0;  // resident classes: largest member
    int64_t step_off = 0;   // resident classes: first slot in kgs_batch::d_steps
    // 2-D streaming (uniform runs of 2-D sweep classes): descriptors for the
    // first launch, the even and the odd launches, 3 x members each
    bool s2 = false;
    kgs::Stream2dMember *d_s2 = nullptr, *h_s2 = nullptr;
    int64_t s2_tasks = 0;
    int s2_chunk = 0;
    // members all below n = 2048: the tiled kernel (tiles of s2_ty rows x
    // s2_tx points of one colour) instead of the y-streaming kernel
    bool s2_tile = false;
    // 3-D streaming (uniform runs of 3-D sweep classes whose members are all
    // n >= kStream3dMinN): the same descriptor triple, s2_tasks workgroups
    // of the z-streaming kernel's member-list launch, nominal chunk s2_chunk
    // (a member of n planes takes member_chunk(n, s2_chunk)), tile s2_tx
    // compressed positions x s2_ty rows
    bool s3 = false;
    int s2_ty = 0, s2_tx = 0;
};


}  // namespace

struct kgs_batch {
    std::vector<kgs_sim *> sims;
    std::vector<BatchClass> classes;
    hipStream_t user = nullptr;  // caller's stream
    hipStream_t own = nullptr;   // the batch's stream (capturable)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int device = 0;
    bool use_graph = false;
    bool uploaded = false;  // descriptors copied to the device at least once
    std::map<int64_t, hipGraphExec_t> graphs;  // uniform K-step runs
    int *d_kinds = nullptr, *h_kinds = nullptr;  // per-launch member kinds
    int64_t kinds_cap = 0;
    int64_t *d_steps = nullptr, *h_steps = nullptr;  // per-member steps, resident classes
    std::string err;
};

namespace {

int bfail(kgs_batch *b, int code, const std::string &msg)
{
    if (b) b->err = msg;
    return code;
}

int bhip(kgs_batch *b, hipError_t e, const char *what)
{
    return bfail(b, e == hipErrorOutOfMemory ? KGS_ENOMEM : KGS_EDEVICE,
                 std::string(what) + ": " + hipGetErrorName(e));
}

thread_local std::string g_batch_err;

// 3-D members stream together when every member has n >= kStream3dMinN
// (at least one full tile along x); the tile and plane chunk of such a
// launch are those stream3d_list_plan estimates to end it first.
constexpr int kStream3dMinN = 32;

// Releases everything the batch holds; the first runtime error, if any.
hipError_t destroy(kgs_batch *b)
{
    kgs::FirstError err;
    for (auto &kv : b->graphs) err(hipGraphExecDestroy(kv.second));
    b->graphs.clear();
    for (auto &c : b->classes) {
        if (c.d_members) err(hipFree(c.d_members));
        if (c.h_members) err(hipHostFree(c.h_members));
        if (c.d_res) err(hipFree(c.d_res));
        if (c.h_res) err(hipHostFree(c.h_res));
        if (c.d_s2) err(hipFree(c.d_s2));
        if (c.h_s2) err(hipHostFree(c.h_s2));
    }
    if (b->d_steps) err(hipFree(b->d_steps));
    if (b->h_steps) err(hipHostFree(b->h_steps));
    if (b->d_kinds) err(hipFree(b->d_kinds));
    if (b->h_kinds) err(hipHostFree(b->h_kinds));
    if (b->ev_in) err(hipEventDestroy(b->ev_in));
    if (b->ev_out) err(hipEventDestroy(b->ev_out));
    if (b->own) err(hipStreamDestroy(b->own));
    return err.e;
}

// The launch configuration of a streaming class.
kgs::GroupTuning group_of(const BatchClass &c)
{
    kgs::GroupTuning t;
    t.mode = c.s3 ? kgs::GROUP_STREAM3D : c.s2_tile ? kgs::GROUP_TILE2D : kgs::GROUP_STREAM2D;
    t.chunk = c.s2_chunk;
    t.ty = c.s2_ty;
    t.tx = c.s2_tx;
    return t;
}

// Gives a streaming class the configuration t if it fits every member
// (else leaves the class as it is and returns false): the class fields and
// the host copy of its member descriptors, apart from the state buffers and
// the first-launch flags that refresh_descriptors writes.
bool apply_group(kgs_batch *b, BatchClass &c, const kgs::GroupTuning &t)
{
    const size_t nm = c.members.size();
    const int eb = c.precision == KGS_FP64 ? 8 : 4;
    if ((t.mode == kgs::GROUP_STREAM3D) != (c.dim == 3) || t.chunk < 1) return false;
    // 3-D: a tile of 0 x 0 is the precision's default list tile
    int tx3 = t.tx, ty3 = t.ty;
    if (t.mode == kgs::GROUP_STREAM3D && (tx3 < 1 || ty3 < 1))
        kgs::stream3d_list_tile(eb, &tx3, &ty3);
    int64_t tb = 0;
    for (size_t i = 0; i < nm; ++i) {
        const kgs_sim *x = b->sims[c.members[i]];
        const int n = x->geo.n;
        if (t.mode == kgs::GROUP_STREAM3D) {
            if (n < kStream3dMinN || !kgs::stream3d_list_ok(x->geo, t.chunk, eb, tx3, ty3))
                return false;
            tb += kgs::stream3d_member_items(n, kgs::member_chunk(n, t.chunk), tx3, ty3);
        } else if (t.mode == kgs::GROUP_TILE2D) {
            if (!kgs::tile2d_shape_ok(x->geo, t.ty, t.tx, 4, eb)) return false;
            tb += kgs::tile2d_member_tiles(n, t.ty, t.tx);
        } else {
            if (kgs::stream2d_tasks(n, t.chunk) < 1) return false;
            tb += kgs::stream2d_tasks(n, t.chunk);
        }
    }
    if (tb > 0x7ffffff0) return false;  // the launch's item limit
    c.s3 = t.mode == kgs::GROUP_STREAM3D;
    c.s2 = !c.s3;
    c.s2_tile = t.mode == kgs::GROUP_TILE2D;
    c.s2_chunk = t.chunk;
    c.s2_ty = c.s3 ? ty3 : t.ty;
    c.s2_tx = c.s3 ? tx3 : t.tx;
    tb = 0;
    for (size_t i = 0; i < nm; ++i) {
        const kgs_sim *x = b->sims[c.members[i]];
        const int n = x->geo.n;
        for (int v = 0; v < 3; ++v) {
            kgs::Stream2dMember &m = c.h_s2[v * nm + i];
            std::memset(&m, 0, sizeof(m));
            m.stride = x->geo.stride;
            m.task_begin = tb;
            m.k = x->coef;
            m.n = n;
            m.chunk = c.s3 ? kgs::member_chunk(n, c.s2_chunk) : c.s2_tile ? c.s2_ty : c.s2_chunk;
            m.tiles_x = c.s3 ? 0 : c.s2_tile ? kgs::tile2d_tiles_x(n, c.s2_tx)
                                             : kgs::stream2d_tiles_x(n);
            // in/out/first are set by refresh_descriptors
        }
        tb += c.s3 ? kgs::stream3d_member_items(n, kgs::member_chunk(n, c.s2_chunk), c.s2_tx,
                                                c.s2_ty)
                   : c.s2_tile ? kgs::tile2d_member_tiles(n, c.s2_ty, c.s2_tx)
                               : kgs::stream2d_tasks(n, c.s2_chunk);
    }
    c.s2_tasks = tb;
    return true;
}

// Copy every member's current state buffer (the 3-D streaming kernel swaps
// buffers) into the device descriptors when one has changed.  The pinned
// staging may still be read by an earlier queued copy, so wait for the batch
// stream before rewriting it.
int refresh_descriptors(kgs_batch *b)
{
    auto held = [&](const BatchClass &c, size_t i) {
        return c.resident ? c.h_res[i].state : c.h_members[i].state;
    };
    bool changed = false;
    for (auto &c : b->classes)
        for (size_t i = 0; i < c.members.size(); ++i) {
            const kgs_sim *m = b->sims[c.members[i]];
            changed |= held(c, i) != m->state;
            if (c.s2 || c.s3) changed |= c.h_s2[i].out != m->state2;
        }
    if (!changed && b->uploaded) return KGS_OK;
    hipError_t e = hipStreamSynchronize(b->own);
    if (e != hipSuccess) return bhip(b, e, "hipStreamSynchronize");
    for (auto &c : b->classes) {
        const size_t nm = c.members.size();
        if (c.resident) {
            for (size_t i = 0; i < nm; ++i) c.h_res[i].state = b->sims[c.members[i]]->state;
            e = hipMemcpyAsync(c.d_res, c.h_res, nm * sizeof(kgs::ResidentMember),
                               hipMemcpyHostToDevice, b->own);
        } else {
            for (size_t i = 0; i < nm; ++i) c.h_members[i].state = b->sims[c.members[i]]->state;
            e = hipMemcpyAsync(c.d_members, c.h_members, nm * sizeof(kgs::BatchMember),
                               hipMemcpyHostToDevice, b->own);
            if (e == hipSuccess && (c.s2 || c.s3)) {
                // [first launch | even launches | odd launches]
                for (size_t i = 0; i < nm; ++i) {
                    const kgs_sim *m = b->sims[c.members[i]];
                    kgs::Stream2dMember &f = c.h_s2[i], &ev = c.h_s2[nm + i], &od = c.h_s2[2 * nm + i];
                    f.in = ev.in = m->state;
                    od.out = m->state;
                    f.out = ev.out = m->state2;
                    od.in = m->state2;
                    f.first = 1;
                    ev.first = od.first = 0;
                }
                e = hipMemcpyAsync(c.d_s2, c.h_s2, 3 * nm * sizeof(kgs::Stream2dMember),
                                   hipMemcpyHostToDevice, b->own);
            }
        }
        if (e != hipSuccess) return bhip(b, e, "hipMemcpyAsync (batch descriptors)");
    }
    b->uploaded = true;
    return KGS_OK;
}

// A uniform run of nsteps >= 2 steps of a streaming class: launches of 2
// steps, and of 1 step where needed to keep the number of launches even (so
// that every member ends in its own buffer), then the closing red sweep.
hipError_t enqueue_stream_class(kgs_batch *b, const BatchClass &c, int64_t nsteps)
{
    // K = 2a + r steps: a launches of 4 sweeps and r of 2, one 4 split into
    // two 2s when that count is odd
    const int64_t a = nsteps / 2, r = nsteps % 2;
    const int64_t split = (a + r) % 2;
    std::vector<int> stages(static_cast<size_t>(a - split), 4);
    for (int64_t i = 0; i < 2 * split + r; ++i) stages.push_back(2);
    const int nm = static_cast<int>(c.members.size());
    kgs::Stream2dMember none;
    std::memset(&none, 0, sizeof(none));
    for (size_t i = 0; i < stages.size(); ++i) {
        const kgs::Stream2dMember *list = c.d_s2 + (i == 0 ? 0 : (i % 2 ? 2 * nm : nm));
        hipError_t e;
        if (c.s3)
            e = kgs::launch_stream3d_list(c.precision, stages[i], c.s2_tx, c.s2_ty, list, nm,
                                          c.s2_tasks, i == 0, b->own);
        else if (c.s2_tile)
            e = kgs::launch_tile2d_list(c.precision, stages[i], c.s2_ty, c.s2_tx, none, list, nm,
                                        c.s2_tasks, b->own, i == 0 ? 1 : 0);
        else
            e = kgs::launch_stream2d(c.precision, stages[i], none, list, nm, c.s2_tasks, b->own);
        if (e != hipSuccess) return e;
    }
    return kgs::launch_batch_sweep(c.dim, c.precision, c.d_members, nm, c.blocks, nullptr, 0,
                                   kgs::PASS_R_ADJ, b->own);
}

// Launch sequence of a uniform K-step run: one resident launch per resident
// class, then R_BASE, (B_FULL, R_ADJ_BASE)^(K-1), B_FULL, R_ADJ, each as one
// batched launch per sweep class.
hipError_t enqueue_uniform(kgs_batch *b, int64_t nsteps)
{
    for (auto &c : b->classes) {
        if (!c.resident) continue;
        kgs::ResidentMember none;
        std::memset(&none, 0, sizeof(none));
        hipError_t e = kgs::launch_resident(c.dim, c.precision, none, c.d_res, nullptr, nsteps,
                                            static_cast<int>(c.members.size()), c.max_count,
                                            b->own);
        if (e != hipSuccess) return e;
    }
    // 2-D and 3-D streaming classes
    const bool streamed = nsteps >= 2;
    for (auto &c : b->classes) {
        if (!(c.s2 || c.s3) || !streamed) continue;
        hipError_t e = enqueue_stream_class(b, c, nsteps);
        if (e != hipSuccess) return e;
    }
    auto sweep = [&](int kind) {
        for (auto &c : b->classes) {
            if (c.resident || ((c.s2 || c.s3) && streamed)) continue;
            hipError_t e = kgs::launch_batch_sweep(c.dim, c.precision, c.d_members,
                                                   static_cast<int>(c.members.size()), c.blocks,
                                                   nullptr, 0, kind, b->own);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipError_t e = sweep(kgs::PASS_R_BASE);
    for (int64_t i = 1; i < nsteps && e == hipSuccess; ++i) {
        e = sweep(kgs::PASS_B_FULL);
        if (e == hipSuccess) e = sweep(kgs::PASS_R_ADJ_BASE);
    }
    if (e == hipSuccess) e = sweep(kgs::PASS_B_FULL);
    if (e == hipSuccess) e = sweep(kgs::PASS_R_ADJ);
    return e;
}

int begin(kgs_batch *b)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return bhip(b, e, "hipGetDevice");
    if (dev != b->device && (e = hipSetDevice(b->device)) != hipSuccess)
        return bhip(b, e, "hipSetDevice");
    // members left open by kgs_step get their closing sweep first, ordered
    // like the batch's own work
    for (kgs_sim *x : b->sims)
        if (kgs::sim_close(x, b->user) != KGS_OK) return bfail(b, KGS_EDEVICE, x->err.c_str());
    if ((e = hipEventRecord(b->ev_in, b->user)) != hipSuccess) return bhip(b, e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(b->own, b->ev_in, 0)) != hipSuccess)
        return bhip(b, e, "hipStreamWaitEvent");
    return refresh_descriptors(b);
}

int end(kgs_batch *b)
{
    hipError_t e = hipEventRecord(b->ev_out, b->own);
    if (e != hipSuccess) return bhip(b, e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(b->user, b->ev_out, 0)) != hipSuccess)
        return bhip(b, e, "hipStreamWaitEvent");
    return KGS_OK;
}

}  // namespace

extern "C" {

const char *kgs_batch_last_error(const kgs_batch *b) { return b ? b->err.c_str() : g_batch_err.c_str(); }

int kgs_batch_create(kgs_sim *const *sims, int32_t count, void *stream, kgs_batch **out)
{
    KGS_TRACE("kgs_batch_create");
    if (!out) {
        g_batch_err = "out is NULL";
        return KGS_EINVAL;
    }
    *out = nullptr;
    if (!sims || count < 1) {
        g_batch_err = "need at least one simulation";
        return KGS_EINVAL;
    }
    kgs_batch *b = new (std::nothrow) kgs_batch();
    if (!b) {
        g_batch_err = "host allocation failed";
        return KGS_ENOMEM;
    }
    b->user = static_cast<hipStream_t>(stream);
    int code = KGS_OK;
    for (int32_t i = 0; i < count && code == KGS_OK; ++i) {
        if (!sims[i]) code = bfail(b, KGS_EINVAL, "simulation pointer is NULL");
        else if (i > 0 && sims[i]->device != sims[0]->device)
            code = bfail(b, KGS_EINVAL, "all simulations must live on one GPU");
        else if (std::find(b->sims.begin(), b->sims.end(), sims[i]) != b->sims.end())
            code = bfail(b, KGS_EINVAL, "a simulation appears twice");
        else b->sims.push_back(sims[i]);
    }
    hipError_t e = hipSuccess;
    if (code == KGS_OK) {
        b->device = sims[0]->device;
        if ((e = hipSetDevice(b->device)) != hipSuccess) code = bhip(b, e, "hipSetDevice");
    }
    if (code == KGS_OK && (e = hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking)) != hipSuccess)
        code = bhip(b, e, "hipStreamCreate");
    if (code == KGS_OK && (e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming)) != hipSuccess)
        code = bhip(b, e, "hipEventCreate");
    if (code == KGS_OK && (e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming)) != hipSuccess)
        code = bhip(b, e, "hipEventCreate");
    // group by (dim, precision, resident), larger simulations first
    if (code == KGS_OK) {
        auto fits = [](const kgs_sim *s) {
            return kgs::resident_fits(s->geo.count, s->cfg.precision == KGS_FP64 ? 8 : 4);
        };
        std::vector<int> order(b->sims.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            return b->sims[x]->geo.count > b->sims[y]->geo.count;
        });
        for (int i : order) {
            const kgs_sim *s = b->sims[i];
            const bool res = fits(s);
            auto it = std::find_if(b->classes.begin(), b->classes.end(), [&](const BatchClass &c) {
                return c.dim == s->cfg.dim && c.precision == s->cfg.precision && c.resident == res;
            });
            if (it == b->classes.end()) {
                b->classes.emplace_back();
                it = b->classes.end() - 1;
                it->dim = s->cfg.dim;
                it->precision = s->cfg.precision;
                it->resident = res;
            }
            it->members.push_back(i);
        }
        const int bb = kgs::batch_block();
        int64_t step_slots = 0;
        for (auto &c : b->classes) {
            if (c.resident) {
                const size_t bytes = c.members.size() * sizeof(kgs::ResidentMember);
                if ((e = hipMalloc(reinterpret_cast<void **>(&c.d_res), bytes)) != hipSuccess) {
                    code = bhip(b, e, "hipMalloc (batch descriptors)");
                    break;
                }
                if ((e = hipHostMalloc(reinterpret_cast<void **>(&c.h_res), bytes,
                                       hipHostMallocDefault)) != hipSuccess) {
                    code = bhip(b, e, "hipHostMalloc (batch descriptors)");
                    break;
                }
                for (size_t i = 0; i < c.members.size(); ++i) {
                    const kgs_sim *s = b->sims[c.members[i]];
                    kgs::ResidentMember &m = c.h_res[i];
                    std::memset(&m, 0, sizeof(m));
                    m.state = s->state;
                    m.stride = s->geo.stride;
                    m.k = s->coef;
                    m.n = s->geo.n;
                    m.count = static_cast<int>(s->geo.count);
                    c.max_count = std::max<int64_t>(c.max_count, s->geo.count);
                }
                c.step_off = step_slots;
                step_slots += static_cast<int64_t>(c.members.size());
                continue;
            }
            const size_t bytes = c.members.size() * sizeof(kgs::BatchMember);
            if ((e = hipMalloc(reinterpret_cast<void **>(&c.d_members), bytes)) != hipSuccess) {
                code = bhip(b, e, "hipMalloc (batch descriptors)");
                break;
            }
            if ((e = hipHostMalloc(reinterpret_cast<void **>(&c.h_members), bytes,
                                   hipHostMallocDefault)) != hipSuccess) {
                code = bhip(b, e, "hipHostMalloc (batch descriptors)");
                break;
            }
            int64_t blocks = 0;
            for (size_t i = 0; i < c.members.size(); ++i) {
                const kgs_sim *s = b->sims[c.members[i]];
                kgs::BatchMember &m = c.h_members[i];
                std::memset(&m, 0, sizeof(m));
                m.state = s->state;
                m.stride = s->geo.stride;
                m.count = s->geo.count;
                m.block_begin = blocks;
                m.k = s->coef;
                m.n = s->geo.n;
                blocks += (s->geo.count + bb - 1) / bb;
            }
            if (blocks > 0x7fffffff) {
                code = bfail(b, KGS_EINVAL, "batch too large for one launch");
                break;
            }
            c.blocks = blocks;
            if (c.dim == 2) {
                // 2-D runs of several steps between two buffers (every
                // member needs its second buffer): the y-streaming kernel
                // with a row chunk that gives >= 2048 tasks (waves) where
                // the members allow it, or the tiled kernel when that chunk
                // is short and all members are below n = 2048
                c.s2 = true;
                const size_t nm = c.members.size();
                for (size_t i = 0; i < nm && code == KGS_OK; ++i)
                    code = kgs::sim_ensure_state2(b->sims[c.members[i]]);
                if (code != KGS_OK) {
                    b->err = "second state buffer for the 2-D streaming kernel";
                    break;
                }
                int chunk = 64;
                auto tasks = [&](int ch) {
                    int64_t t = 0;
                    for (size_t i = 0; i < nm; ++i) t += kgs::stream2d_tasks(b->sims[c.members[i]]->geo.n, ch);
                    return t;
                };
                while (chunk > 8 && tasks(chunk) < 2048) chunk /= 2;
                c.s2_chunk = chunk;
                // tiles when the members are too few for long streaming
                // chunks (measured: 64 uneven grids of n <= 1024 stream at
                // chunk 64 1.2x faster than they run tiles)
                c.s2_tile = chunk < 32;
                std::vector<int> ns(nm);
                for (size_t i = 0; i < nm; ++i) {
                    ns[i] = b->sims[c.members[i]]->geo.n;
                    if (ns[i] >= 2048) c.s2_tile = false;
                }
                kgs::tile2d_group_shape(ns.data(), static_cast<int>(nm), c.s2_ty, c.s2_tx);
                const size_t s2bytes = 3 * nm * sizeof(kgs::Stream2dMember);
                if ((e = hipMalloc(reinterpret_cast<void **>(&c.d_s2), s2bytes)) != hipSuccess ||
                    (e = hipHostMalloc(reinterpret_cast<void **>(&c.h_s2), s2bytes,
                                       hipHostMallocDefault)) != hipSuccess) {
                    code = bhip(b, e, "descriptor allocation (2-D streaming)");
                    break;
                }
                if (!apply_group(b, c, group_of(c))) {
                    code = bfail(b, KGS_EINVAL, "2-D group does not fit its launch");
                    break;
                }
            } else if (c.dim == 3) {
                // 3-D runs of several steps: the z-streaming kernel over all
                // members in one launch when every member is large enough
                // for its tile (else batched sweeps), with the tile and plane
                // chunk (8..128) estimated to end the launch first
                const size_t nm = c.members.size();
                const int eb = c.precision == KGS_FP64 ? 8 : 4;
                std::vector<int> sizes(nm);
                for (size_t i = 0; i < nm; ++i) sizes[i] = b->sims[c.members[i]]->geo.n;
                int tx = 0, ty = 0, chunk = 0;
                kgs::stream3d_list_plan(sizes.data(), static_cast<int>(nm), eb, &tx, &ty, &chunk);
                int64_t items = 0;
                for (size_t i = 0; i < nm; ++i)
                    items += kgs::stream3d_member_items(sizes[i], kgs::member_chunk(sizes[i], chunk),
                                                        tx, ty);
                bool ok = items <= 0x7ffffff0;  // the launch's item limit
                for (size_t i = 0; i < nm && ok; ++i) {
                    const kgs_sim *x = b->sims[c.members[i]];
                    ok = x->geo.n >= kStream3dMinN &&
                         kgs::stream3d_list_ok(x->geo, chunk, eb, tx, ty);
                }
                if (!ok) continue;
                for (size_t i = 0; i < nm && code == KGS_OK; ++i)
                    code = kgs::sim_ensure_state2(b->sims[c.members[i]]);
                if (code != KGS_OK) {
                    b->err = "second state buffer for the 3-D streaming kernel";
                    break;
                }
                c.s3 = true;
                c.s2_chunk = chunk;
                c.s2_tx = tx;
                c.s2_ty = ty;
                const size_t s3bytes = 3 * nm * sizeof(kgs::Stream2dMember);
                if ((e = hipMalloc(reinterpret_cast<void **>(&c.d_s2), s3bytes)) != hipSuccess ||
                    (e = hipHostMalloc(reinterpret_cast<void **>(&c.h_s2), s3bytes,
                                       hipHostMallocDefault)) != hipSuccess) {
                    code = bhip(b, e, "descriptor allocation (3-D streaming)");
                    break;
                }
                if (!apply_group(b, c, group_of(c))) {
                    code = bfail(b, KGS_EINVAL, "3-D group does not fit its launch");
                    break;
                }
            }
        }
        if (code == KGS_OK && step_slots > 0) {
            const size_t bytes = static_cast<size_t>(step_slots) * sizeof(int64_t);
            if ((e = hipMalloc(reinterpret_cast<void **>(&b->d_steps), bytes)) != hipSuccess)
                code = bhip(b, e, "hipMalloc (batch steps)");
            else if ((e = hipHostMalloc(reinterpret_cast<void **>(&b->h_steps), bytes,
                                        hipHostMallocDefault)) != hipSuccess)
                code = bhip(b, e, "hipHostMalloc (batch steps)");
            // kernel attributes are set before any launch can be captured
            else if ((e = kgs::resident_prepare()) != hipSuccess)
                code = bhip(b, e, "resident kernel set-up");
        }
    }
    if (code != KGS_OK) {
        g_batch_err = b->err;
        (void)destroy(b);  // the first error is the one reported
        delete b;
        return code;
    }
    *out = b;
    return KGS_OK;
}

int kgs_batch_set_graph(kgs_batch *b, int32_t enable)
{
    if (!b) return KGS_EINVAL;
    b->use_graph = enable != 0;
    return KGS_OK;
}

int kgs_batch_step(kgs_batch *b, int64_t nsteps)
{
    KGS_TRACE("kgs_batch_step");
    if (!b) return KGS_EINVAL;
    if (nsteps < 0) return bfail(b, KGS_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return KGS_OK;
    int rc = begin(b);
    if (rc != KGS_OK) return rc;
    hipError_t e;
    if (b->use_graph) {
        auto it = b->graphs.find(nsteps);
        if (it == b->graphs.end()) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            if ((e = hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return bhip(b, e, "hipStreamBeginCapture");
            hipError_t le = enqueue_uniform(b, nsteps);
            e = hipStreamEndCapture(b->own, &g);
            if (le != hipSuccess) {
                // the launch error is the one reported; the graph is discarded
                if (g) (void)hipGraphDestroy(g);
                return bhip(b, le, "batched sweep launch (capture)");
            }
            if (e != hipSuccess) return bhip(b, e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            const hipError_t gd = hipGraphDestroy(g);
            if (e != hipSuccess) return bhip(b, e, "hipGraphInstantiate");
            if (gd != hipSuccess) {
                (void)hipGraphExecDestroy(ge);  // the first error is the one reported
                return bhip(b, gd, "hipGraphDestroy");
            }
            it = b->graphs.emplace(nsteps, ge).first;
        }
        if ((e = hipGraphLaunch(it->second, b->own)) != hipSuccess) return bhip(b, e, "hipGraphLaunch");
    } else {
        if ((e = enqueue_uniform(b, nsteps)) != hipSuccess)
            return bhip(b, e, "batched sweep launch");
    }
    return end(b);
}

int kgs_batch_step_each(kgs_batch *b, const int64_t *nsteps)
{
    KGS_TRACE("kgs_batch_step_each");
    if (!b || !nsteps) return bfail(b, KGS_EINVAL, "batch or nsteps is NULL");
    int64_t kmax = 0;
    for (size_t i = 0; i < b->sims.size(); ++i) {
        if (nsteps[i] < 0) return bfail(b, KGS_EINVAL, "nsteps must be >= 0");
        kmax = std::max(kmax, nsteps[i]);
    }
    if (kmax == 0) return KGS_OK;
    // launch sequence per class: red 0, blue 0, red 1, ..., blue kmax-1, red kmax
    const int64_t launches = 2 * kmax + 1;
    size_t nmax = 0, nsweep = 0;
    for (auto &c : b->classes)
        if (!c.resident) {
            nmax = std::max(nmax, c.members.size());
            ++nsweep;
        }
    const int64_t need = std::max<int64_t>(
        1, launches * static_cast<int64_t>(nmax) * static_cast<int64_t>(nsweep));
    if (need > (int64_t(1) << 31)) return bfail(b, KGS_EINVAL, "schedule too large");
    int rc = begin(b);
    if (rc != KGS_OK) return rc;
    hipError_t e;
    if (need > b->kinds_cap) {
        // the previous table may still be read by queued work
        if ((e = hipStreamSynchronize(b->own)) != hipSuccess) return bhip(b, e, "hipStreamSynchronize");
        kgs::FirstError err;
        if (b->d_kinds) err(hipFree(b->d_kinds));
        if (b->h_kinds) err(hipHostFree(b->h_kinds));
        if (!err.ok()) return bhip(b, err.e, "releasing the schedule");
        b->d_kinds = nullptr;
        b->h_kinds = nullptr;
        b->kinds_cap = 0;
        if ((e = hipMalloc(reinterpret_cast<void **>(&b->d_kinds), need * sizeof(int))) != hipSuccess)
            return bhip(b, e, "hipMalloc (schedule)");
        if ((e = hipHostMalloc(reinterpret_cast<void **>(&b->h_kinds), need * sizeof(int),
                               hipHostMallocDefault)) != hipSuccess)
            return bhip(b, e, "hipHostMalloc (schedule)");
        b->kinds_cap = need;
    } else if ((e = hipStreamSynchronize(b->own)) != hipSuccess) {
        // pinned staging is reused: wait until the previous schedule was consumed
        return bhip(b, e, "hipStreamSynchronize");
    }
    // steps of the members of resident classes
    for (auto &c : b->classes)
        if (c.resident)
            for (size_t m = 0; m < c.members.size(); ++m)
                b->h_steps[c.step_off + m] = nsteps[c.members[m]];
    if (b->d_steps) {
        int64_t slots = 0;
        for (auto &c : b->classes)
            if (c.resident) slots += static_cast<int64_t>(c.members.size());
        if ((e = hipMemcpyAsync(b->d_steps, b->h_steps, slots * sizeof(int64_t),
                                hipMemcpyHostToDevice, b->own)) != hipSuccess)
            return bhip(b, e, "hipMemcpyAsync (steps)");
        for (auto &c : b->classes) {
            if (!c.resident) continue;
            kgs::ResidentMember none;
            std::memset(&none, 0, sizeof(none));
            e = kgs::launch_resident(c.dim, c.precision, none, c.d_res, b->d_steps + c.step_off, 0,
                                     static_cast<int>(c.members.size()), c.max_count, b->own);
            if (e != hipSuccess) return bhip(b, e, "resident kernel launch");
        }
    }
    // kinds table of the sweep classes: [class][launch][member]
    int64_t off = 0;
    std::vector<int64_t> class_off;
    for (auto &c : b->classes) {
        class_off.push_back(off);
        if (c.resident) continue;
        const int nm = static_cast<int>(c.members.size());
        for (int64_t L = 0; L < launches; ++L) {
            const int64_t i = L / 2;  // step index
            const bool red = (L % 2) == 0;
            for (int m = 0; m < nm; ++m) {
                const int64_t k = nsteps[c.members[m]];
                int kind = -1;
                if (red) {
                    if (k > 0 && i == 0) kind = kgs::PASS_R_BASE;
                    else if (i > 0 && i < k) kind = kgs::PASS_R_ADJ_BASE;
                    else if (k > 0 && i == k) kind = kgs::PASS_R_ADJ;
                } else if (i < k) {
                    kind = kgs::PASS_B_FULL;
                }
                b->h_kinds[off + L * nm + m] = kind;
            }
        }
        off += launches * nm;
    }
    if (nsweep == 0) return end(b);
    if ((e = hipMemcpyAsync(b->d_kinds, b->h_kinds, off * sizeof(int), hipMemcpyHostToDevice,
                            b->own)) != hipSuccess)
        return bhip(b, e, "hipMemcpyAsync (schedule)");
    for (int64_t L = 0; L < launches; ++L) {
        for (size_t ci = 0; ci < b->classes.size(); ++ci) {
            auto &c = b->classes[ci];
            if (c.resident) continue;
            e = kgs::launch_batch_sweep(c.dim, c.precision, c.d_members,
                                        static_cast<int>(c.members.size()), c.blocks,
                                        b->d_kinds + class_off[ci], static_cast<int>(L), -1, b->own);
            if (e != hipSuccess) return bhip(b, e, "batched sweep launch");
        }
    }
    return end(b);
}

int kgs_batch_autotune(kgs_batch *b, int32_t steps, int32_t use_cache)
{
    KGS_TRACE("kgs_batch_autotune");
    if (!b) return KGS_EINVAL;
    if (steps < 2) return bfail(b, KGS_EINVAL, "steps must be >= 2 (streaming runs)");
    int rc = begin(b);
    if (rc != KGS_OK) return rc;
    hipError_t e = hipSuccess;
    hipEvent_t ea = nullptr, eb = nullptr;
    void *backup = nullptr;
    bool retuned = false;
    if ((e = hipEventCreate(&ea)) != hipSuccess || (e = hipEventCreate(&eb)) != hipSuccess)
        rc = bhip(b, e, "hipEventCreate");
    for (auto &c : b->classes) {
        if (rc != KGS_OK) break;
        if (!(c.s2 || c.s3)) continue;
        std::vector<int> sizes;
        for (int m : c.members) sizes.push_back(b->sims[m]->geo.n);
        const std::string sig = kgs::group_signature(b->device, c.dim, c.precision, sizes);
        kgs::GroupTuning cached;
        if (use_cache && kgs::group_cache_get(sig, cached) && apply_group(b, c, cached)) {
            retuned = true;
            continue;
        }
        // the members' states, restored after every timed run
        size_t total = 0;
        for (int m : c.members) total += 8 * b->sims[m]->plane_bytes;
        if ((e = hipMalloc(&backup, total)) != hipSuccess) {
            rc = bhip(b, e, "hipMalloc (autotune state copy)");
            break;
        }
        auto copy_states = [&](bool save) {
            size_t off = 0;
            for (int m : c.members) {
                kgs_sim *x = b->sims[m];
                const size_t bytes = 8 * x->plane_bytes;
                char *bk = static_cast<char *>(backup) + off;
                hipError_t r = hipMemcpyAsync(save ? bk : x->state, save ? x->state : bk, bytes,
                                              hipMemcpyDeviceToDevice, b->own);
                if (r != hipSuccess) return r;
                off += bytes;
            }
            return hipSuccess;
        };
        e = copy_states(true);
        std::vector<kgs::GroupTuning> cands{group_of(c)};  // the default first
        if (c.dim == 3) {
            // float64 also tries the 12-wave 32x13 tile (GroupTuning: ty, tx)
            for (int ch : {8, 16, 32, 64, 128}) {
                cands.push_back({kgs::GROUP_STREAM3D, ch, 0, 0});
                if (c.precision == KGS_FP64) cands.push_back({kgs::GROUP_STREAM3D, ch, 13, 32});
            }
        } else {
            for (int ch : {8, 16, 32, 64}) cands.push_back({kgs::GROUP_STREAM2D, ch, 0, 0});
            const int tiles[][2] = {{8, 8}, {8, 16}, {16, 16}, {16, 32}, {32, 32}};
            for (const auto &t : tiles) cands.push_back({kgs::GROUP_TILE2D, t[0], t[0], t[1]});
        }
        const kgs::GroupTuning original = group_of(c);
        kgs::GroupTuning best = original;
        float best_ms = -1.0f;
        for (const kgs::GroupTuning &t : cands) {
            if (e != hipSuccess) break;
            if (!apply_group(b, c, t)) continue;
            b->uploaded = false;
            if ((rc = refresh_descriptors(b)) != KGS_OK) break;
            // one warm-up run, then the faster of two timed runs, each from
            // the saved states
            float ms = -1.0f;
            for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
                float m = 0.0f;
                if ((e = hipEventRecord(ea, b->own)) != hipSuccess ||
                    (e = enqueue_stream_class(b, c, steps)) != hipSuccess ||
                    (e = hipEventRecord(eb, b->own)) != hipSuccess ||
                    (e = hipEventSynchronize(eb)) != hipSuccess ||
                    (e = hipEventElapsedTime(&m, ea, eb)) != hipSuccess ||
                    (e = copy_states(false)) != hipSuccess)
                    break;
                if (rep > 0 && (ms < 0.0f || m < ms)) ms = m;
            }
            if (e == hipSuccess && (best_ms < 0.0f || ms < best_ms)) {
                best_ms = ms;
                best = t;
            }
        }
        const hipError_t s2 = hipStreamSynchronize(b->own);
        if (e == hipSuccess) e = s2;
        const hipError_t fr = hipFree(backup);
        backup = nullptr;
        if (e == hipSuccess) e = fr;
        if (e != hipSuccess && rc == KGS_OK) rc = bhip(b, e, "autotune run");
        apply_group(b, c, rc == KGS_OK ? best : original);
        if (rc == KGS_OK) kgs::group_cache_put(sig, best);
        retuned = true;
    }
    kgs::FirstError err;
    if (ea) err(hipEventDestroy(ea));
    if (eb) err(hipEventDestroy(eb));
    if (backup) err(hipFree(backup));
    if (retuned) {
        // captured runs embed the old launches
        for (auto &kv : b->graphs) err(hipGraphExecDestroy(kv.second));
        b->graphs.clear();
        b->uploaded = false;
        const int r2 = refresh_descriptors(b);
        if (rc == KGS_OK) rc = r2;
    }
    if (!err.ok() && rc == KGS_OK) rc = bhip(b, err.e, "autotune release");
    const int r3 = end(b);
    return rc == KGS_OK ? r3 : rc;
}

int kgs_batch_free(kgs_batch *b)
{
    KGS_TRACE("kgs_batch_free");
    if (!b) return KGS_OK;
    int rc = KGS_OK;
    if (hipSetDevice(b->device) != hipSuccess || hipStreamSynchronize(b->own) != hipSuccess)
        rc = KGS_EDEVICE;
    if (destroy(b) != hipSuccess) rc = KGS_EDEVICE;
    delete b;
    return rc;
}

}  // extern "C"
