// Serving loop with continuous batching: requests (simulations of any
// dimension, size, parameters, precision and step count) arrive at any time,
// wait in a queue, are admitted when their device memory fits the budget,
// and then advance together in rounds: every running request moves by up to
// steps_per_round steps per round, 3-D float64 ones with their own
// z-streaming kernel and all others in one batched run with per-request step
// counts.  Finished requests are retired (energy and state copied to the
// host, device memory freed) and queued ones join at the next round.
//
// Each request ends bitwise where running it alone ends: points of one
// colour are independent and step boundaries store the state exactly as a
// continuous run's fused sweeps round it.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "kgs.h"
#include "kgs_internal.h"
#include "kgs_sim.h"

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    int64_t id = 0;
    kgs_config cfg;
    int64_t nsteps = 0;
    int64_t done_steps = 0;
    int32_t state = KGS_REQ_QUEUED;
    int32_t status = KGS_OK;
    int64_t bytes = 0;        // device bytes while running
    int64_t points = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    double e0 = 0, e1 = 0;
    std::vector<double> host;  // 4 arrays of `points` doubles: host input, then the result
    double *dev_in = nullptr;  // device copy of a device-submitted input (until admitted)
    kgs_sim *sim = nullptr;
    std::string err;
};

}  // namespace

struct kgs_server {
    kgs_server_config cfg;
    hipStream_t stream = nullptr;
    int device = 0;
    double t0 = 0;
    int64_t next_id = 1;
    int64_t used = 0;        // device bytes held by running requests
    int64_t queued_dev = 0;  // device bytes held by queued device-submitted inputs
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::deque<int64_t> queue;
    std::vector<int64_t> running;
    // batch over the running requests that use batched sweeps
    kgs_batch *batch = nullptr;
    std::vector<int64_t> batch_ids;
    int64_t rounds = 0;
    bool pending_copy = false;  // device inputs copied on the stream, not yet waited for
    std::string err;
};

namespace {

thread_local std::string g_srv_err;

int sfail(kgs_server *s, int code, const std::string &msg)
{
    if (s) s->err = msg;
    else g_srv_err = msg;
    return code;
}

void release_request(Request *r)
{
    if (r->sim) {
        if (kgs_free(r->sim) != KGS_OK) {
        }
        r->sim = nullptr;
    }
    if (r->dev_in) {
        if (hipFree(r->dev_in) != hipSuccess) {
        }
        r->dev_in = nullptr;
    }
    std::vector<double>().swap(r->host);
}

bool uses_own_kernel(const kgs_sim *sim) { return sim->tuning.kernel == KGS_KERNEL_STREAM; }

void drop_batch(kgs_server *s)
{
    if (s->batch) {
        if (kgs_batch_free(s->batch) != KGS_OK) {
        }
        s->batch = nullptr;
    }
    s->batch_ids.clear();
}

// Admit queued requests in arrival order while they fit the budget.
int admit(kgs_server *s)
{
    while (!s->queue.empty()) {
        if (s->cfg.max_active > 0 && static_cast<int>(s->running.size()) >= s->cfg.max_active) break;
        Request *r = s->reqs[s->queue.front()].get();
        // the state plus kgs_init's transient staging copy (host inputs) must fit
        const int64_t peak =
            r->bytes + (r->dev_in ? 0 : 4 * r->points * static_cast<int64_t>(sizeof(double)));
        if (peak > s->cfg.budget_bytes) {
            s->queue.pop_front();
            r->state = KGS_REQ_FAILED;
            r->status = KGS_ENOMEM;
            r->err = "request needs more device memory than the whole budget";
            r->t_done = now_s() - s->t0;
            continue;
        }
        if (s->used + peak > s->cfg.budget_bytes) break;  // wait for running ones to retire
        s->queue.pop_front();
        const int64_t P = r->points;
        const bool dev = r->dev_in != nullptr;
        const double *in = dev ? r->dev_in : r->host.data();
        int rc = kgs_init(&r->cfg, in, in + P, in + 2 * P, in + 3 * P, dev ? KGS_DEVICE : KGS_HOST,
                          s->stream, &r->sim);
        if (rc == KGS_OK) {
            // the input copy is no longer needed
            if (r->dev_in) {
                if (hipFree(r->dev_in) != hipSuccess) {
                }
                r->dev_in = nullptr;
                s->queued_dev -= 4 * P * static_cast<int64_t>(sizeof(double));
            }
            std::vector<double>().swap(r->host);
        }
        if (rc == KGS_OK) rc = kgs_energy(r->sim, &r->e0);
        if (rc != KGS_OK && rc != KGS_ENONFINITE) {
            r->err = kgs_last_error(r->sim);
            if (r->err.empty()) r->err = kgs_last_error(nullptr);
            if (r->sim) {
                if (kgs_free(r->sim) != KGS_OK) {
                }
                r->sim = nullptr;
            }
            if (rc == KGS_ENOMEM) {  // the device is fuller than the budget says: retry later
                s->queue.push_front(r->id);
                break;
            }
            if (r->dev_in) s->queued_dev -= 4 * r->points * static_cast<int64_t>(sizeof(double));
            release_request(r);
            r->state = KGS_REQ_FAILED;
            r->status = rc;
            r->t_done = now_s() - s->t0;
            continue;
        }
        r->state = KGS_REQ_RUNNING;
        r->t_admit = now_s() - s->t0;
        s->used += r->bytes;
        s->running.push_back(r->id);
        drop_batch(s);  // membership changed
    }
    return KGS_OK;
}

int retire(kgs_server *s, Request *r)
{
    const int64_t P = r->points;
    int rc = kgs_energy(r->sim, &r->e1);
    if (rc == KGS_OK || rc == KGS_ENONFINITE) {
        r->host.assign(static_cast<size_t>(4 * P), 0.0);
        double *h = r->host.data();
        rc = kgs_read_state(r->sim, h, h + P, h + 2 * P, h + 3 * P, KGS_HOST);
    }
    if (rc != KGS_OK) r->err = kgs_last_error(r->sim);
    if (kgs_free(r->sim) != KGS_OK) {
    }
    r->sim = nullptr;
    s->used -= r->bytes;
    r->state = rc == KGS_OK ? KGS_REQ_DONE : KGS_REQ_FAILED;
    r->status = rc;
    r->t_done = now_s() - s->t0;
    return KGS_OK;
}

int round_once(kgs_server *s)
{
    admit(s);
    if (s->running.empty()) return KGS_OK;
    const int64_t spr = s->cfg.steps_per_round > 0 ? s->cfg.steps_per_round : INT64_MAX;
    // requests on their own kernel
    std::vector<int64_t> batched;
    for (int64_t id : s->running) {
        Request *r = s->reqs[id].get();
        if (uses_own_kernel(r->sim)) {
            const int64_t k = std::min(spr, r->nsteps - r->done_steps);
            int rc = kgs_step(r->sim, k);
            if (rc != KGS_OK) return sfail(s, rc, kgs_last_error(r->sim));
            r->done_steps += k;
        } else {
            batched.push_back(id);
        }
    }
    if (!batched.empty()) {
        if (!s->batch || s->batch_ids != batched) {
            drop_batch(s);
            std::vector<kgs_sim *> sims;
            for (int64_t id : batched) sims.push_back(s->reqs[id]->sim);
            int rc = kgs_batch_create(sims.data(), static_cast<int32_t>(sims.size()), s->stream,
                                      &s->batch);
            if (rc != KGS_OK) return sfail(s, rc, kgs_batch_last_error(nullptr));
            s->batch_ids = batched;
        }
        std::vector<int64_t> k(batched.size());
        for (size_t i = 0; i < batched.size(); ++i) {
            Request *r = s->reqs[batched[i]].get();
            k[i] = std::min(spr, r->nsteps - r->done_steps);
            r->done_steps += k[i];
        }
        int rc = kgs_batch_step_each(s->batch, k.data());
        if (rc != KGS_OK) return sfail(s, rc, kgs_batch_last_error(s->batch));
    }
    s->rounds++;
    // retire finished requests (their reads wait for the stream)
    std::vector<int64_t> still;
    bool changed = false;
    for (int64_t id : s->running) {
        Request *r = s->reqs[id].get();
        if (r->done_steps >= r->nsteps) {
            if (!changed) drop_batch(s);  // the batch must not outlive its members
            changed = true;
            retire(s, r);
        } else {
            still.push_back(id);
        }
    }
    s->running.swap(still);
    return KGS_OK;
}

}  // namespace

extern "C" {

const char *kgs_server_last_error(const kgs_server *s) { return s ? s->err.c_str() : g_srv_err.c_str(); }

int kgs_server_create(const kgs_server_config *cfg, void *stream, kgs_server **out)
{
    if (!out) return sfail(nullptr, KGS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg || cfg->budget_bytes <= 0 || cfg->max_active < 0 || cfg->steps_per_round < 0 ||
        cfg->reserved[0] || cfg->reserved[1] || cfg->reserved[2] || cfg->reserved[3])
        return sfail(nullptr, KGS_EINVAL, "invalid server configuration");
    kgs_server *s = new (std::nothrow) kgs_server();
    if (!s) return sfail(nullptr, KGS_ENOMEM, "host allocation failed");
    s->cfg = *cfg;
    s->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return sfail(nullptr, KGS_EDEVICE, "hipGetDevice failed");
    }
    s->t0 = now_s();
    *out = s;
    return KGS_OK;
}

int kgs_server_submit(kgs_server *s, const kgs_config *cfg, const double *psi_re,
                      const double *psi_im, const double *u, const double *v_t, int32_t mem,
                      int64_t nsteps, int64_t *id)
{
    if (!s || !id) return sfail(s, KGS_EINVAL, "server or id is NULL");
    *id = 0;
    if (!cfg || !psi_re || !psi_im || !u || !v_t) return sfail(s, KGS_EINVAL, "NULL argument");
    if (mem != KGS_HOST && mem != KGS_DEVICE) return sfail(s, KGS_EINVAL, "bad memory kind");
    if (nsteps < 0) return sfail(s, KGS_EINVAL, "nsteps must be >= 0");
    const int64_t bytes = kgs_required_bytes(cfg);
    if (bytes <= 0) {
        // reuse kgs_init's validation for the message and status
        kgs_sim *tmp = nullptr;
        int rc = kgs_init(cfg, psi_re, psi_im, u, v_t, mem, s->stream, &tmp);
        if (tmp) kgs_free(tmp);
        return sfail(s, rc != KGS_OK ? rc : KGS_EINVAL, kgs_last_error(nullptr));
    }
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return sfail(s, KGS_ENOMEM, "host allocation failed");
    r->id = s->next_id++;
    r->cfg = *cfg;
    r->nsteps = nsteps;
    r->bytes = bytes;
    r->points = 1;
    for (int a = 0; a < cfg->dim; ++a) r->points *= cfg->n;
    const size_t nb = static_cast<size_t>(r->points) * sizeof(double);
    const double *src[4] = {psi_re, psi_im, u, v_t};
    if (mem == KGS_HOST) {
        try {
            r->host.resize(static_cast<size_t>(4 * r->points));
        } catch (...) {
            return sfail(s, KGS_ENOMEM, "host allocation failed");
        }
        for (int f = 0; f < 4; ++f) std::memcpy(r->host.data() + f * r->points, src[f], nb);
    } else {
        // device inputs stay on the device until admission (not counted in
        // the running budget; see kgs_server_stats)
        if (hipMalloc(reinterpret_cast<void **>(&r->dev_in), 4 * nb) != hipSuccess) {
            r->dev_in = nullptr;
            return sfail(s, KGS_ENOMEM, "device allocation for the queued input failed");
        }
        for (int f = 0; f < 4; ++f) {
            if (hipMemcpyAsync(r->dev_in + f * r->points, src[f], nb, hipMemcpyDeviceToDevice,
                               s->stream) != hipSuccess) {
                release_request(r.get());
                return sfail(s, KGS_EDEVICE, "copy of the initial state failed");
            }
        }
        s->queued_dev += static_cast<int64_t>(4 * nb);
        s->pending_copy = true;
    }
    r->t_submit = now_s() - s->t0;
    *id = r->id;
    s->queue.push_back(r->id);
    s->reqs[r->id] = std::move(r);
    return KGS_OK;
}

int kgs_server_run(kgs_server *s, int32_t rounds, int32_t *n_running, int32_t *n_queued)
{
    if (!s || rounds < 0) return sfail(s, KGS_EINVAL, "bad arguments");
    if (hipSetDevice(s->device) != hipSuccess) return sfail(s, KGS_EDEVICE, "hipSetDevice failed");
    if (s->pending_copy) {
        // callers may reuse device inputs once this call returns
        if (hipStreamSynchronize(s->stream) != hipSuccess)
            return sfail(s, KGS_EDEVICE, "hipStreamSynchronize failed");
        s->pending_copy = false;
    }
    for (int32_t i = 0; i < rounds; ++i) {
        int rc = round_once(s);
        if (rc != KGS_OK) return rc;
        if (s->running.empty() && s->queue.empty()) break;
    }
    if (n_running) *n_running = static_cast<int32_t>(s->running.size());
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
    if (!s) return sfail(nullptr, KGS_EINVAL, "server is NULL");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return sfail(s, KGS_EINVAL, "unknown request");
    Request *r = it->second.get();
    if (r->state != KGS_REQ_DONE) return sfail(s, KGS_EINVAL, "request has no result");
    if (!psi_re || !psi_im || !u || !v_t || (mem != KGS_HOST && mem != KGS_DEVICE))
        return sfail(s, KGS_EINVAL, "bad output arguments");
    const size_t nb = static_cast<size_t>(r->points) * sizeof(double);
    double *dst[4] = {psi_re, psi_im, u, v_t};
    for (int f = 0; f < 4; ++f) {
        const double *src = r->host.data() + f * r->points;
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
    if (r->state == KGS_REQ_RUNNING) return sfail(s, KGS_EINVAL, "request is running");
    if (r->state == KGS_REQ_QUEUED) {
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), id));
        if (r->dev_in) s->queued_dev -= 4 * r->points * static_cast<int64_t>(sizeof(double));
    }
    release_request(r);
    s->reqs.erase(it);
    return KGS_OK;
}

int kgs_server_cancel(kgs_server *s, int64_t id)
{
    if (!s) return KGS_EINVAL;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return sfail(s, KGS_EINVAL, "unknown request");
    Request *r = it->second.get();
    if (r->state == KGS_REQ_QUEUED) {
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), id));
        if (r->dev_in) s->queued_dev -= 4 * r->points * static_cast<int64_t>(sizeof(double));
    } else if (r->state == KGS_REQ_RUNNING) {
        drop_batch(s);
        if (hipStreamSynchronize(s->stream) != hipSuccess) return sfail(s, KGS_EDEVICE, "sync failed");
        s->running.erase(std::find(s->running.begin(), s->running.end(), id));
        s->used -= r->bytes;
    } else {
        return sfail(s, KGS_EINVAL, "request already finished");
    }
    release_request(r);
    r->state = KGS_REQ_CANCELLED;
    r->t_done = now_s() - s->t0;
    return KGS_OK;
}

int kgs_server_stats(const kgs_server *s, kgs_server_stats_t *st)
{
    if (!s || !st) return KGS_EINVAL;
    std::memset(st, 0, sizeof(*st));
    st->device_bytes_used = s->used;
    st->queued_input_bytes = s->queued_dev;
    st->running = static_cast<int32_t>(s->running.size());
    st->queued = static_cast<int32_t>(s->queue.size());
    st->rounds = s->rounds;
    st->now = now_s() - s->t0;
    return KGS_OK;
}

int kgs_server_free(kgs_server *s)
{
    if (!s) return KGS_OK;
    drop_batch(s);
    int rc = hipStreamSynchronize(s->stream) == hipSuccess ? KGS_OK : KGS_EDEVICE;
    for (auto &kv : s->reqs) release_request(kv.second.get());
    delete s;
    return rc;
}

}  // extern "C"
