// gcm_batch.cpp -- many uneven messages in one persistent launch.
//
// A plan is built once on the host: one descriptor per message (its own
// tile size, so a 4 KiB message and a 64 MiB one both map onto whole wave
// tiles), the prefix sum of tiles over messages (each message's first
// partial-hash slot), and a work list of workgroup items -- `waves`
// consecutive wave tiles of one message -- ordered by key slot so that a
// persistent workgroup reloads its GHASH table only when the key changes.
// Launching a plan enqueues three kernels (tiles, per-message combine,
// zero-fill of rejected messages) and allocates nothing, so it can be
// captured into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/gcm_mi355.h"
#include "gcm_host.h"

using namespace gcm;

struct gcm_batch {
    gcm_ctx *ctx = nullptr;
    uint32_t n = 0;
    uint32_t n_items = 0;
    Shape shape;
    uint32_t grid = 1;
    bool any_decrypt = false;
    uint64_t total_tiles = 0;
    uint64_t payload_bytes = 0;
    MsgDesc *d_descs = nullptr;
    WorkItem *d_items = nullptr;
    uint8_t *d_ws = nullptr;  // counters + reject list, then partials
    uint64_t dev_bytes = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
};

// Validate the jobs against the base allocation and the key table and plan
// them, with `forced` as the shape if given (caller holds ctx->mu).
int gcm::plan_jobs(const gcm_ctx *ctx, const gcm_job *jobs, uint32_t n, uint8_t *base_d, uint64_t base_bytes,
                   const Shape *forced, Shape *sh_out, BatchPlan *plan)
{
    const SlotView sv = slot_view(ctx);
    PlanError err;
    for (uint32_t i = 0; i < n; ++i)
        if (check_job(jobs[i], i, base_bytes, sv, &err))
            return plan_error(err);
    std::vector<PlanMsg> msgs(n);
    uint64_t total_m = 0, payload = 0;
    for (uint32_t i = 0; i < n; ++i) {
        msgs[i] = plan_msg_from_job(jobs[i], (uint64_t)base_d);
        total_m += ghash_blocks(jobs[i].aad_len, jobs[i].len);
        payload += jobs[i].len;
    }
    const Shape sh = forced ? *forced : batch_shape(ctx, n, payload, total_m);
    plan_batch(msgs.data(), n, sv, sh.waves, sh.log2B, plan);
    *sh_out = sh;
    return GCM_OK;
}

int gcm::batch_create_locked(gcm_ctx *ctx, const gcm_job *jobs, uint32_t n, uint8_t *base_d, uint64_t base_bytes,
                             const Shape *forced, gcm_batch **out)
{
    BatchPlan plan;
    Shape sh;
    int rc = plan_jobs(ctx, jobs, n, base_d, base_bytes, forced, &sh, &plan);
    if (rc)
        return rc;
    gcm_batch *b = new gcm_batch();
    b->ctx = ctx;
    b->n = n;
    b->shape = sh;
    b->total_tiles = plan.total_tiles;
    b->any_decrypt = plan.any_decrypt;
    b->payload_bytes = plan.payload;
    b->n_items = (uint32_t)plan.items.size();
    b->grid = std::max<uint32_t>(1, std::min<uint32_t>(b->n_items, (uint32_t)ctx->cu_count * sh.gpc));

    const uint64_t desc_bytes = (uint64_t)n * sizeof(MsgDesc);
    const uint64_t item_bytes = (uint64_t)plan.items.size() * sizeof(WorkItem);
    const uint64_t ws_bytes = plan.workspace_bytes();
    b->dev_bytes = ((desc_bytes + 255) / 256 + (item_bytes + 255) / 256) * 256 + ws_bytes;
    uint8_t *mem = nullptr;
    rc = ctx_alloc(ctx, reinterpret_cast<void **>(&mem), b->dev_bytes);
    if (rc) {
        delete b;
        return rc;
    }
    b->d_descs = reinterpret_cast<MsgDesc *>(mem);
    b->d_items = reinterpret_cast<WorkItem *>(mem + (desc_bytes + 255) / 256 * 256);
    b->d_ws = mem + ((desc_bytes + 255) / 256 + (item_bytes + 255) / 256) * 256;
    hipError_t e = hipSuccess;
    if (n)
        e = hipMemcpy(b->d_descs, plan.descs.data(), desc_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && !plan.items.empty())
        e = hipMemcpy(b->d_items, plan.items.data(), item_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        ctx_free(ctx, mem, b->dev_bytes);
        delete b;
        return fail_hip(e, "batch table upload");
    }
    *out = b;
    return GCM_OK;
}

extern "C" int gcm_batch_create(gcm_ctx *ctx, const gcm_job *jobs, uint32_t n, uint8_t *base_d, uint64_t base_bytes,
                                gcm_batch **out)
{
    GCM_ABI_TRY
        if (!ctx || !out || (n && (!jobs || !base_d)))
            return fail(GCM_E_ARG, "gcm_batch_create: NULL argument");
        *out = nullptr;
        if ((uintptr_t)base_d & 255)
            return fail(GCM_E_ARG, "gcm_batch_create: base_d must be 256-byte aligned");
        std::lock_guard<std::mutex> g(ctx->mu);
        return batch_create_locked(ctx, jobs, n, base_d, base_bytes, nullptr, out);
    GCM_ABI_CATCH
}

void gcm::batch_free_locked(gcm_batch *b)
{
    gcm_ctx *ctx = b->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (b->graph_exec)
        (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    if (b->cap_stream)
        (void)hipStreamDestroy(b->cap_stream);
    ctx_free(ctx, b->d_descs, b->dev_bytes);
    delete b;
}

hipError_t gcm::batch_enqueue(gcm_batch *b, hipStream_t s)
{
    gcm_ctx *ctx = b->ctx;
    if (b->n == 0)
        return hipSuccess;
    uint32_t *counters = reinterpret_cast<uint32_t *>(b->d_ws);
    uint8_t *partials = b->d_ws + workspace_counter_bytes(b->n);
    hipError_t e = prof_begin(ctx, s);
    if (e == hipSuccess)
        e = launch_tiles((int)b->shape.waves, b->d_descs, b->d_items, b->n_items, nullptr, ctx->d_tables, partials,
                         counters, b->grid, s);
    if (e == hipSuccess)
        e = prof_end(ctx, s);
    if (e == hipSuccess)
        e = launch_combine(b->d_descs, b->n, nullptr, partials, counters, b->shape.fanin, s);
    if (e == hipSuccess && b->any_decrypt)
        e = launch_zerofill(b->d_descs, nullptr, counters, (uint32_t)std::max(1, ctx->cu_count * 4), s);
    return e;
}

extern "C" int gcm_batch_launch(gcm_batch *b, void *stream)
{
    GCM_ABI_TRY
        if (!b)
            return fail(GCM_E_ARG, "gcm_batch_launch: NULL batch");
        std::lock_guard<std::mutex> g(b->ctx->mu);
        hipError_t e = hipSetDevice(b->ctx->device);
        if (e == hipSuccess)
            e = batch_enqueue(b, reinterpret_cast<hipStream_t>(stream));
        if (e != hipSuccess)
            return fail_hip(e, "batch launch");
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_batch_graph_launch(gcm_batch *b, void *stream)
{
    GCM_ABI_TRY
        if (!b)
            return fail(GCM_E_ARG, "gcm_batch_graph_launch: NULL batch");
        std::lock_guard<std::mutex> g(b->ctx->mu);
        hipError_t e = hipSetDevice(b->ctx->device);
        if (e != hipSuccess)
            return fail_hip(e, "hipSetDevice");
        if (!b->graph_exec) {
            // capture on a private stream (the null stream cannot be captured)
            e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
            if (e == hipSuccess)
                e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const bool prof = b->ctx->prof;
                b->ctx->prof = false;  // no event records inside the graph
                hipError_t le = batch_enqueue(b, b->cap_stream);
                b->ctx->prof = prof;
                e = hipStreamEndCapture(b->cap_stream, &b->graph);
                if (le != hipSuccess)
                    e = le;
            }
            if (e == hipSuccess)
                e = hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0);
            if (e != hipSuccess)
                return fail_hip(e, "batch graph capture");
        }
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        e = prof_begin(b->ctx, s);
        if (e == hipSuccess)
            e = hipGraphLaunch(b->graph_exec, s);
        if (e == hipSuccess)
            e = prof_end(b->ctx, s);
        if (e != hipSuccess)
            return fail_hip(e, "batch graph launch");
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_batch_destroy(gcm_batch *b)
{
    GCM_ABI_TRY
        if (!b)
            return fail(GCM_E_ARG, "gcm_batch_destroy: NULL batch");
        std::lock_guard<std::mutex> g(b->ctx->mu);
        batch_free_locked(b);
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_batch_info(const gcm_batch *b, uint64_t *payload_bytes, uint64_t *total_tiles, uint32_t *work_items)
{
    GCM_ABI_TRY
        if (!b)
            return fail(GCM_E_ARG, "gcm_batch_info: NULL batch");
        if (payload_bytes)
            *payload_bytes = b->payload_bytes;
        if (total_tiles)
            *total_tiles = b->total_tiles;
        if (work_items)
            *work_items = b->n_items;
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_batch_run(gcm_ctx *ctx, const gcm_job *jobs, uint32_t n, uint8_t *base_d, uint64_t base_bytes,
                             void *stream)
{
    GCM_ABI_TRY
        gcm_batch *b = nullptr;
        int rc = gcm_batch_create(ctx, jobs, n, base_d, base_bytes, &b);
        if (rc)
            return rc;
        rc = gcm_batch_launch(b, stream);
        if (rc == GCM_OK) {
            hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
            if (e != hipSuccess)
                rc = fail_hip(e, "batch synchronize");
        }
        gcm_batch_destroy(b);
        return rc;
    GCM_ABI_CATCH
}
