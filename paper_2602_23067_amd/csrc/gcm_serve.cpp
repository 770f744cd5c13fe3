// gcm_serve.cpp -- continuous-batching serving loop.
//
// Callers submit encrypt / decrypt-verify requests whose buffers already live
// in HBM; keys come from the resident key table.  One scheduler thread
//   1. retires finished batches (a HIP event per stream slot), returning
//      their bytes to the HBM budget and recording each request's latency
//      (submit -> result known on the host),
//   2. admits waiting requests in arrival order while the budget allows,
//   3. packs admitted requests into a batch and launches it on a free stream
//      slot -- the same persistent tile kernel, combine and zero-fill as
//      gcm_batch -- while earlier batches are still running.
// Requests that arrive while others are on the GPU are admitted as soon as
// budget and a stream slot free up; results do not depend on how requests
// are grouped.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/gcm_mi355.h"
#include "gcm_host.h"
#include "serve_policy.h"

using namespace gcm;

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct ReqState {
    gcm_request r;
    uint64_t need = 0;
    int64_t t_submit = 0, t_done = 0;
    int state = 0;  // 0 queued, 1 running, 2 done
    int accept = 1;
    int status = GCM_OK;  // a failure of the batch that carried the request
};

// Device and pinned staging of one stream slot; grown on demand while idle.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> ids;
    uint8_t *d_mem = nullptr;  // descs | items | flags | workspace
    uint64_t d_bytes = 0;
    uint64_t in_use = 0;       // bytes of d_mem the running batch uses
    uint8_t *h_mem = nullptr;  // pinned: descs | items | flags
    uint64_t h_bytes = 0;
    uint64_t flag_off = 0;  // offset of the accept flags in both blocks
};

uint64_t align256(uint64_t x) { return (x + 255) / 256 * 256; }

}  // namespace

struct gcm_serve {
    gcm_ctx *ctx = nullptr;
    gcm_serve_config cfg{};
    ServePolicy policy;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::unordered_map<uint64_t, ReqState> reqs;
    uint64_t next_id = 1;
    std::vector<Slot> slots;
    std::thread worker;
    bool stopping = false;
    int worker_error = GCM_OK;
    char error_msg[256] = {0};
    // statistics
    std::vector<double> lat_ms;
    uint64_t submitted = 0, completed = 0, rejected = 0, failed = 0, batches = 0, bytes_done = 0;
    uint64_t overlapped_admissions = 0, max_inflight = 0;
    int64_t t_first = 0, t_last = 0;
};

// Stream-slot memory not used by a running batch counts against the HBM
// budget (caller holds s->mu).
static void update_slack(gcm_serve *s)
{
    uint64_t slack = 0;
    for (const Slot &sl : s->slots)
        slack += sl.busy ? sl.d_bytes - sl.in_use : sl.d_bytes;
    s->policy.set_slack(slack);
}

// Give slot `sl` at least dbytes of device memory and hbytes of pinned
// staging.  A slot that must grow takes twice its old size when that still
// fits the budget (fewer regrowths), else exactly dbytes: its requests'
// admitted bytes already cover dbytes, so the budget holds either way.
static int slot_reserve(gcm_serve *s, Slot &sl, uint64_t dbytes, uint64_t hbytes)
{
    if (sl.d_bytes < dbytes) {
        const uint64_t others = s->policy.slack() - sl.d_bytes;  // the slot is idle: all of it is slack
        uint64_t want = dbytes;
        const uint64_t grown = std::max<uint64_t>(dbytes, 2 * sl.d_bytes);
        if (grown > dbytes && s->policy.admitted_bytes() + others + (grown - dbytes) <= s->cfg.hbm_budget)
            want = grown;
        std::lock_guard<std::mutex> g(s->ctx->mu);  // the context's allocation bookkeeping
        ctx_free(s->ctx, sl.d_mem, sl.d_bytes);
        sl.d_mem = nullptr;
        sl.d_bytes = 0;
        int rc = ctx_alloc(s->ctx, reinterpret_cast<void **>(&sl.d_mem), want);
        if (rc)
            return rc;
        sl.d_bytes = want;
    }
    if (sl.h_bytes < hbytes) {
        if (sl.h_mem)
            (void)hipHostFree(sl.h_mem);
        sl.h_mem = nullptr;
        sl.h_bytes = 0;
        const uint64_t want = std::max<uint64_t>(hbytes, 1ull << 16);
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&sl.h_mem), want, hipHostMallocDefault);
        if (e != hipSuccess)
            return fail(GCM_E_NOMEM, "serving staging: hipHostMalloc: %s", hipGetErrorString(e));
        sl.h_bytes = want;
    }
    return GCM_OK;
}

// Free the device memory of idle slots (when the head of the queue does not
// fit beside it and nothing is running).
static void release_idle_slots(gcm_serve *s)
{
    std::lock_guard<std::mutex> g(s->ctx->mu);
    for (Slot &sl : s->slots)
        if (!sl.busy && sl.d_mem) {
            ctx_free(s->ctx, sl.d_mem, sl.d_bytes);
            sl.d_mem = nullptr;
            sl.d_bytes = 0;
        }
}

// Launch one batch on a free slot (caller holds s->mu).
static int launch_batch(gcm_serve *s, Slot &sl, const std::vector<PolicyReq> &batch)
{
    gcm_ctx *ctx = s->ctx;
    const uint32_t n = (uint32_t)batch.size();
    std::vector<PlanMsg> msgs(n);
    uint64_t total_m = 0, payload = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const gcm_request &r = s->reqs[batch[i].id].r;
        PlanMsg &pm = msgs[i];
        pm.op = r.op;
        pm.key_slot = r.key_slot;
        std::memcpy(pm.iv, r.iv, 12);
        pm.aad = (uint64_t)r.aad_d;
        pm.aad_len = r.aad_len;
        pm.in = (uint64_t)r.in_d;
        pm.out = (uint64_t)r.out_d;
        pm.len = r.len;
        pm.tag = (uint64_t)r.tag_d;
        total_m += ghash_blocks(r.aad_len, r.len);
        payload += r.len;
    }
    BatchPlan plan;
    Shape sh;
    {
        std::lock_guard<std::mutex> g(ctx->mu);  // key table and autotune caches
        sh = batch_shape(ctx, n, payload, total_m);
        plan_batch(msgs.data(), n, slot_view(ctx), sh.waves, sh.log2B, &plan);
    }
    const uint64_t n_items = plan.items.size();
    const uint64_t desc_b = align256(n * sizeof(MsgDesc)), item_b = align256(n_items * sizeof(WorkItem));
    const uint64_t flag_b = align256(4ull * n), ws_b = plan.workspace_bytes();
    const uint64_t dbytes = desc_b + item_b + flag_b + ws_b;
    int rc = slot_reserve(s, sl, dbytes, desc_b + item_b + flag_b);
    if (rc)
        return rc;
    MsgDesc *h_desc = reinterpret_cast<MsgDesc *>(sl.h_mem);
    WorkItem *h_item = reinterpret_cast<WorkItem *>(sl.h_mem + desc_b);
    MsgDesc *d_desc = reinterpret_cast<MsgDesc *>(sl.d_mem);
    WorkItem *d_item = reinterpret_cast<WorkItem *>(sl.d_mem + desc_b);
    int32_t *d_flags = reinterpret_cast<int32_t *>(sl.d_mem + desc_b + item_b);
    int32_t *h_flags = reinterpret_cast<int32_t *>(sl.h_mem + desc_b + item_b);
    uint8_t *d_ws = sl.d_mem + desc_b + item_b + flag_b;
    sl.flag_off = desc_b + item_b;
    for (uint32_t i = 0; i < n; ++i) {
        plan.descs[i].ok = (uint64_t)(d_flags + i);
        h_desc[i] = plan.descs[i];
        // a decrypt is accepted only once the device has written 1 here
        h_flags[i] = 0;
    }
    if (n_items)
        std::memcpy(h_item, plan.items.data(), n_items * sizeof(WorkItem));
    const uint32_t grid =
        (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(n_items, (uint64_t)ctx->cu_count * sh.gpc));
    hipError_t e = hipMemcpyAsync(sl.d_mem, sl.h_mem, desc_b + item_b, hipMemcpyHostToDevice, sl.stream);
    uint32_t *counters = reinterpret_cast<uint32_t *>(d_ws);
    uint8_t *partials = d_ws + workspace_counter_bytes(n);
    if (e == hipSuccess)
        e = launch_tiles((int)sh.waves, d_desc, d_item, (uint32_t)n_items, nullptr, ctx->d_tables, partials, counters,
                         grid, sl.stream);
    if (e == hipSuccess)
        e = launch_combine(d_desc, n, nullptr, partials, counters, sh.fanin, sl.stream);
    if (e == hipSuccess && plan.any_decrypt)
        e = launch_zerofill(d_desc, nullptr, counters, (uint32_t)std::max(1, ctx->cu_count * 2), sl.stream);
    if (e == hipSuccess && plan.any_decrypt)
        e = hipMemcpyAsync(h_flags, d_flags, 4ull * n, hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess)
        e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess)
        return fail_hip(e, "serving batch launch");
    sl.busy = true;
    sl.in_use = dbytes;
    sl.ids.clear();
    for (const PolicyReq &p : batch) {
        sl.ids.push_back(p.id);
        s->reqs[p.id].state = 1;
    }
    s->batches++;
    update_slack(s);
    return GCM_OK;
}

// Complete a request (caller holds s->mu): err != GCM_OK marks a request
// whose batch failed; it is reported with that status and never accepted.
static void finish(gcm_serve *s, uint64_t id, int64_t t, int accept, int err)
{
    ReqState &st = s->reqs[id];
    st.state = 2;
    st.t_done = t;
    st.status = err;
    st.accept = err ? 0 : accept;
    s->policy.complete(st.need);
    s->lat_ms.push_back((double)(t - st.t_submit) * 1e-6);
    s->completed++;
    if (err)
        s->failed++;
    else {
        s->bytes_done += st.r.len;
        if (!st.accept)
            s->rejected++;
    }
}

static void record_error(gcm_serve *s, int code)
{
    s->worker_error = code;
    std::snprintf(s->error_msg, sizeof s->error_msg, "%s", gcm_last_error());
}

// A batch's event completed (err == GCM_OK) or reported a failure.
static void retire(gcm_serve *s, Slot &sl, int err)
{
    const int64_t t = now_ns();
    const int32_t *h_flags = reinterpret_cast<const int32_t *>(sl.h_mem + sl.flag_off);
    for (size_t i = 0; i < sl.ids.size(); ++i) {
        const ReqState &st = s->reqs[sl.ids[i]];
        const int accept = st.r.op == 1 ? (h_flags[i] == 1 ? 1 : 0) : 1;
        finish(s, sl.ids[i], t, accept, err);
    }
    s->t_last = t;
    sl.busy = false;
    sl.in_use = 0;
    sl.ids.clear();
    update_slack(s);
}

static void worker_loop(gcm_serve *s, std::unique_lock<std::mutex> &lk)
{
    std::vector<PolicyReq> batch;
    std::vector<uint64_t> admitted;
    for (;;) {
        bool any_busy = false, progressed = false;
        for (Slot &sl : s->slots) {
            if (!sl.busy)
                continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                retire(s, sl, GCM_OK);
                progressed = true;
            } else if (q == hipErrorNotReady) {
                any_busy = true;
            } else {
                record_error(s, fail_hip(q, "serving batch"));
                retire(s, sl, s->worker_error);
                progressed = true;
            }
        }
        if (progressed)
            s->cv_done.notify_all();
        admitted.clear();
        s->policy.admit(&admitted);
        if (admitted.empty() && s->policy.pending() > 0 && s->policy.ready() == 0) {
            bool idle = true;
            for (const Slot &sl : s->slots)
                idle &= !sl.busy;
            if (idle && s->policy.slack() > 0) {
                // the head request does not fit beside the retained slot memory
                release_idle_slots(s);
                update_slack(s);
                s->policy.admit(&admitted);
            }
        }
        if (any_busy)
            s->overlapped_admissions += admitted.size();
        uint64_t inflight = 0;
        for (Slot &sl : s->slots) {
            if (!sl.busy && s->policy.ready() > 0 && s->policy.next_batch(&batch)) {
                int rc = launch_batch(s, sl, batch);
                if (rc) {
                    // the batch could not be launched: its requests fail with that status
                    record_error(s, rc);
                    const int64_t t = now_ns();
                    for (const PolicyReq &p : batch)
                        finish(s, p.id, t, 0, rc);
                    s->t_last = t;
                    s->cv_done.notify_all();
                }
            }
            inflight += sl.busy ? 1 : 0;
        }
        s->max_inflight = std::max<uint64_t>(s->max_inflight, inflight);
        if (s->stopping && inflight == 0 && s->policy.pending() == 0 && s->policy.ready() == 0)
            break;
        if (inflight) {
            // poll without sleeping while batches are on the GPU: a timed
            // sleep rounds up to the kernel's timer slack (~50 us), which
            // would add that much to every request's latency
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
}

// The scheduler thread.  If its host bookkeeping throws (a failed
// allocation), it waits for the batches already on the GPU, completes every
// request not yet done as rejected, records the error (new submissions then
// fail with it) and ends, so that waiters return and stop can join.
static void worker_main(gcm_serve *s)
{
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    try {
        worker_loop(s, lk);
    } catch (...) {
        if (!lk.owns_lock())
            lk.lock();
        record_error(s, abi_exception());
        for (Slot &sl : s->slots)
            if (sl.busy) {
                (void)hipEventSynchronize(sl.done);
                sl.busy = false;
            }
        const int64_t t = now_ns();
        for (auto &kv : s->reqs)
            if (kv.second.state != 2) {
                kv.second.state = 2;
                kv.second.accept = 0;
                kv.second.status = s->worker_error;
                kv.second.t_done = t;
                s->failed++;
            }
        s->cv_done.notify_all();
    }
}

extern "C" int gcm_serve_start(gcm_ctx *ctx, const gcm_serve_config *cfg, gcm_serve **out)
{
    GCM_ABI_TRY
        if (!ctx || !out)
            return fail(GCM_E_ARG, "gcm_serve_start: NULL argument");
        *out = nullptr;
        gcm_serve_config c{};
        c.n_streams = 4;
        c.hbm_budget = 64ull << 30;
        c.max_batch_reqs = 256;
        c.max_batch_bytes = 256ull << 20;
        c.max_queue = 1u << 16;
        if (cfg) {
            if (cfg->n_streams)
                c.n_streams = cfg->n_streams;
            if (cfg->hbm_budget)
                c.hbm_budget = cfg->hbm_budget;
            if (cfg->max_batch_reqs)
                c.max_batch_reqs = cfg->max_batch_reqs;
            if (cfg->max_batch_bytes)
                c.max_batch_bytes = cfg->max_batch_bytes;
            if (cfg->max_queue)
                c.max_queue = cfg->max_queue;
        }
        if (c.n_streams > 16)
            return fail(GCM_E_ARG, "gcm_serve_start: at most 16 streams");
        gcm_serve *s = new (std::nothrow) gcm_serve();
        if (!s)
            return fail(GCM_E_NOMEM, "gcm_serve_start: host allocation failed");
        s->ctx = ctx;
        s->cfg = c;
        PolicyConfig pc;
        pc.budget = c.hbm_budget;
        pc.max_batch_reqs = c.max_batch_reqs;
        pc.max_batch_bytes = c.max_batch_bytes;
        pc.max_queue = c.max_queue;
        s->policy = ServePolicy(pc);
        s->slots.resize(c.n_streams);
        hipError_t e = hipSetDevice(ctx->device);
        for (Slot &sl : s->slots) {
            if (e == hipSuccess)
                e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        }
        if (e != hipSuccess) {
            for (Slot &sl : s->slots) {
                if (sl.done)
                    (void)hipEventDestroy(sl.done);
                if (sl.stream)
                    (void)hipStreamDestroy(sl.stream);
            }
            delete s;
            return fail_hip(e, "serving stream creation");
        }
        s->worker = std::thread(worker_main, s);
        *out = s;
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_serve_submit(gcm_serve *s, const gcm_request *req, uint64_t *id_out)
{
    GCM_ABI_TRY
        if (!s || !req || !id_out)
            return fail(GCM_E_ARG, "gcm_serve_submit: NULL argument");
        const gcm_request &r = *req;
        if (r.op > 1 || r.reserved)
            return fail(GCM_E_ARG, "gcm_serve_submit: bad op or reserved field");
        if (!r.tag_d)
            return fail(GCM_E_ARG, "gcm_serve_submit: tag_d is required");
        int rc = check_message(r.aad_len, r.len, r.aad_d, r.in_d, r.out_d, r.tag_d, 16);
        if (rc)
            return rc;
        {
            std::lock_guard<std::mutex> g(s->ctx->mu);
            if (r.key_slot >= s->ctx->n_slots || !s->ctx->slot_used[r.key_slot])
                return fail(GCM_E_SLOT, "key slot %u is not registered", r.key_slot);
        }
        const uint64_t need = r.len + (r.out_d != r.in_d ? r.len : 0) + r.aad_len + batch_overhead_bound(r.aad_len, r.len);
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stopping)
            return fail(GCM_E_ARG, "gcm_serve_submit: server is stopping");
        if (s->worker_error)
            return fail(s->worker_error, "gcm_serve_submit: the serving loop hit an earlier error");
        const uint64_t id = s->next_id;
        const int o = s->policy.offer(PolicyReq{id, need, r.len});
        if (o == ServePolicy::kTooLarge)
            return fail(GCM_E_NOMEM, "request needs %llu bytes, more than the %llu-byte HBM budget",
                        (unsigned long long)need, (unsigned long long)s->cfg.hbm_budget);
        if (o == ServePolicy::kQueueFull)
            return fail(GCM_E_BUSY, "serving queue is full");
        s->next_id++;
        ReqState st;
        st.r = r;
        st.need = need;
        st.t_submit = now_ns();
        if (!s->t_first)
            s->t_first = st.t_submit;
        s->reqs.emplace(id, st);
        s->submitted++;
        *id_out = id;
        s->cv_work.notify_one();
        return GCM_OK;
    GCM_ABI_CATCH
}

static int report(gcm_serve *s, uint64_t id, int *done, int *accept, uint64_t *latency_ns, bool consume)
{
    auto it = s->reqs.find(id);
    if (it == s->reqs.end())
        return fail(GCM_E_ARG, "unknown or already collected request id %llu", (unsigned long long)id);
    const ReqState &st = it->second;
    if (done)
        *done = st.state == 2;
    if (st.state == 2) {
        const int status = st.status;
        if (accept)
            *accept = st.accept;
        if (latency_ns)
            *latency_ns = (uint64_t)(st.t_done - st.t_submit);
        if (consume)
            s->reqs.erase(it);
        if (status != GCM_OK)
            return fail(status, "request %llu: its batch failed: %s", (unsigned long long)id, s->error_msg);
    }
    return GCM_OK;
}

extern "C" int gcm_serve_poll(gcm_serve *s, uint64_t id, int *done, int *accept, uint64_t *latency_ns)
{
    GCM_ABI_TRY
        if (!s)
            return fail(GCM_E_ARG, "gcm_serve_poll: NULL server");
        std::lock_guard<std::mutex> g(s->mu);
        return report(s, id, done, accept, latency_ns, true);
    GCM_ABI_CATCH
}

extern "C" int gcm_serve_wait(gcm_serve *s, uint64_t id, int *accept, uint64_t *latency_ns)
{
    GCM_ABI_TRY
        if (!s)
            return fail(GCM_E_ARG, "gcm_serve_wait: NULL server");
        std::unique_lock<std::mutex> lk(s->mu);
        for (;;) {
            auto it = s->reqs.find(id);
            if (it == s->reqs.end())
                return fail(GCM_E_ARG, "unknown or already collected request id %llu", (unsigned long long)id);
            if (it->second.state == 2)
                return report(s, id, nullptr, accept, latency_ns, true);
            s->cv_done.wait(lk);
        }
    GCM_ABI_CATCH
}

extern "C" int gcm_serve_drain(gcm_serve *s)
{
    GCM_ABI_TRY
        if (!s)
            return fail(GCM_E_ARG, "gcm_serve_drain: NULL server");
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] {
            for (auto &kv : s->reqs)
                if (kv.second.state != 2)
                    return false;
            return true;
        });
        return s->worker_error;
    GCM_ABI_CATCH
}

static double pct(std::vector<double> v, double q)
{
    if (v.empty())
        return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t lo = (size_t)pos;
    const size_t hi = std::min(lo + 1, v.size() - 1);
    return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
}

extern "C" int gcm_serve_get_stats(gcm_serve *s, gcm_serve_stats *out)
{
    GCM_ABI_TRY
        if (!s || !out)
            return fail(GCM_E_ARG, "gcm_serve_get_stats: NULL argument");
        std::lock_guard<std::mutex> g(s->mu);
        std::memset(out, 0, sizeof *out);
        out->submitted = s->submitted;
        out->completed = s->completed;
        out->rejected = s->rejected;
        out->failed = s->failed;
        out->batches = s->batches;
        out->bytes_completed = s->bytes_done;
        out->budget_high_water = s->policy.high_water();
        out->overlapped_admissions = s->overlapped_admissions;
        out->max_inflight_batches = s->max_inflight;
        out->p50_ms = pct(s->lat_ms, 0.50);
        out->p99_ms = pct(s->lat_ms, 0.99);
        out->max_ms = s->lat_ms.empty() ? 0.0 : *std::max_element(s->lat_ms.begin(), s->lat_ms.end());
        double sum = 0;
        for (double x : s->lat_ms)
            sum += x;
        out->mean_ms = s->lat_ms.empty() ? 0.0 : sum / (double)s->lat_ms.size();
        out->wall_s = s->t_last > s->t_first ? (double)(s->t_last - s->t_first) * 1e-9 : 0.0;
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_serve_stop(gcm_serve *s)
{
    GCM_ABI_TRY
        if (!s)
            return fail(GCM_E_ARG, "gcm_serve_stop: NULL server");
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->stopping = true;
        }
        s->cv_work.notify_all();
        if (s->worker.joinable())
            s->worker.join();
        const int err = s->worker_error;
        (void)hipSetDevice(s->ctx->device);
        for (Slot &sl : s->slots) {
            if (sl.stream)
                (void)hipStreamSynchronize(sl.stream);
            {
                std::lock_guard<std::mutex> g(s->ctx->mu);
                ctx_free(s->ctx, sl.d_mem, sl.d_bytes);
            }
            if (sl.h_mem)
                (void)hipHostFree(sl.h_mem);
            if (sl.done)
                (void)hipEventDestroy(sl.done);
            if (sl.stream)
                (void)hipStreamDestroy(sl.stream);
        }
        delete s;
        return err;
    GCM_ABI_CATCH
}
