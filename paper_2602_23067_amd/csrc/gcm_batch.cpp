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
    uint32_t waves = 16;
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

static uint32_t ceil_log2_u64(uint64_t x)
{
    uint32_t l = 0;
    while ((1ull << l) < x)
        ++l;
    return l;
}

static int check_job(const gcm_ctx *ctx, const gcm_job &j, uint32_t idx, uint64_t base_bytes)
{
    if (j.op > 1)
        return fail(GCM_E_ARG, "job %u: op %u is neither 0 (encrypt) nor 1 (decrypt-verify)", idx, j.op);
    if (j.reserved != 0)
        return fail(GCM_E_ARG, "job %u: reserved field must be 0", idx);
    if (j.key_slot >= ctx->n_slots || !ctx->slot_used[j.key_slot])
        return fail(GCM_E_SLOT, "job %u: key slot %u is not registered", idx, j.key_slot);
    if (j.len > kMaxLen || j.aad_len > kMaxAad)
        return fail(GCM_E_TOOLONG, "job %u: len %llu / aad_len %llu beyond the SP 800-38D limits", idx,
                    (unsigned long long)j.len, (unsigned long long)j.aad_len);
    auto inside = [&](uint64_t off, uint64_t len) { return off <= base_bytes && len <= base_bytes - off; };
    if (!inside(j.in_off, j.len) || !inside(j.out_off, j.len) || !inside(j.aad_off, j.aad_len) ||
        !inside(j.tag_off, 16) || (j.op == 1 && !inside(j.ok_off, 4)))
        return fail(GCM_E_ARG, "job %u: a buffer lies outside the %llu-byte base allocation", idx,
                    (unsigned long long)base_bytes);
    if ((j.len && ((j.in_off | j.out_off) & 15)) || (j.aad_len && (j.aad_off & 15)) || (j.op == 1 && (j.ok_off & 3)))
        return fail(GCM_E_ARG, "job %u: payload offsets must be 16-byte aligned and ok_off 4-byte aligned", idx);
    if (j.len && j.in_off != j.out_off && j.in_off < j.out_off + j.len && j.out_off < j.in_off + j.len)
        return fail(GCM_E_ALIAS, "job %u: input and output overlap without being identical", idx);
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
        for (uint32_t i = 0; i < n; ++i) {
            int rc = check_job(ctx, jobs[i], i, base_bytes);
            if (rc)
                return rc;
        }
        gcm_batch *b = new (std::nothrow) gcm_batch();
        if (!b)
            return fail(GCM_E_NOMEM, "gcm_batch_create: host allocation failed");
        b->ctx = ctx;
        b->n = n;

        // launch shape: per-message tiles of about one workgroup item when small,
        // capped so the whole batch still gives every resident wave ~2 tiles
        uint32_t log2B_cfg, waves, gpc;
        uint64_t total_m = 0;
        for (uint32_t i = 0; i < n; ++i)
            total_m += (jobs[i].aad_len + 15) / 16 + (jobs[i].len + 15) / 16 + 1;
        launch_shape(ctx, std::max<uint64_t>(1, total_m), &log2B_cfg, &waves, &gpc);
        b->waves = waves;

        std::vector<MsgDesc> descs(n);
        uint64_t tile_base = 0;
        for (uint32_t i = 0; i < n; ++i) {
            const gcm_job &j = jobs[i];
            const uint64_t m = (j.aad_len + 15) / 16 + (j.len + 15) / 16 + 1;
            // about one workgroup item for small messages; items of at most
            // waves * 2^12 blocks (1 MiB at 16 waves) for large ones, so the
            // persistent workgroups see items of similar cost
            uint32_t log2B = std::max<uint32_t>(6, ceil_log2_u64((m + waves - 1) / waves));
            log2B = std::min(log2B, ctx->cfg_log2B ? ctx->cfg_log2B : std::min<uint32_t>(12, std::max<uint32_t>(8, log2B_cfg)));
            fill_desc(&descs[i], j.op, j.iv, (uint64_t)(base_d + j.aad_off), j.aad_len, (uint64_t)(base_d + j.in_off),
                      (uint64_t)(base_d + j.out_off), j.len, (uint64_t)(base_d + j.tag_off),
                      (uint64_t)(base_d + j.ok_off), (uint64_t)(ctx->d_slots + kSlotBytes * j.key_slot),
                      ctx->slot_nr[j.key_slot], log2B, waves, tile_base);
            // per-lane fix-up tables only pay off when many work items share the key
            tile_base += descs[i].n_tiles + 2;  // partials, then the E_K(J0) and J0 slots
            b->total_tiles += descs[i].n_tiles;
            b->any_decrypt |= j.op == 1;
            b->payload_bytes += j.len;
        }

        // work items, messages grouped by key slot
        std::vector<uint32_t> order(n);
        std::iota(order.begin(), order.end(), 0u);
        std::stable_sort(order.begin(), order.end(),
                         [&](uint32_t a, uint32_t c) { return jobs[a].key_slot < jobs[c].key_slot; });
        std::vector<WorkItem> items;
        for (uint32_t i : order)
            for (uint64_t t = 0; t < descs[i].n_tiles; t += waves)
                items.push_back(WorkItem{i, (uint32_t)t});
        b->n_items = (uint32_t)items.size();
        b->grid = std::max<uint32_t>(1, std::min<uint32_t>(b->n_items, (uint32_t)ctx->cu_count * gpc));

        const uint64_t desc_bytes = (uint64_t)n * sizeof(MsgDesc);
        const uint64_t item_bytes = (uint64_t)items.size() * sizeof(WorkItem);
        const uint64_t ws_bytes = workspace_bytes_for(b->total_tiles, n);
        b->dev_bytes = ((desc_bytes + 255) / 256 + (item_bytes + 255) / 256) * 256 + ws_bytes;
        uint8_t *mem = nullptr;
        int rc = ctx_alloc(ctx, reinterpret_cast<void **>(&mem), b->dev_bytes);
        if (rc) {
            delete b;
            return rc;
        }
        b->d_descs = reinterpret_cast<MsgDesc *>(mem);
        b->d_items = reinterpret_cast<WorkItem *>(mem + (desc_bytes + 255) / 256 * 256);
        b->d_ws = mem + ((desc_bytes + 255) / 256 + (item_bytes + 255) / 256) * 256;
        hipError_t e = hipSuccess;
        if (n)
            e = hipMemcpy(b->d_descs, descs.data(), desc_bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess && !items.empty())
            e = hipMemcpy(b->d_items, items.data(), item_bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            ctx_free(ctx, mem, b->dev_bytes);
            delete b;
            return fail_hip(e, "batch table upload");
        }
        *out = b;
        return GCM_OK;
    GCM_ABI_CATCH
}

static hipError_t batch_enqueue(gcm_batch *b, hipStream_t s)
{
    gcm_ctx *ctx = b->ctx;
    if (b->n == 0)
        return hipSuccess;
    uint32_t *counters = reinterpret_cast<uint32_t *>(b->d_ws);
    uint8_t *partials = b->d_ws + workspace_counter_bytes(b->n);
    hipError_t e = prof_begin(ctx, s);
    if (e == hipSuccess)
        e = launch_tiles((int)b->waves, b->d_descs, b->d_items, b->n_items, nullptr, ctx->d_tables, partials, counters,
                         b->grid, s);
    if (e == hipSuccess)
        e = prof_end(ctx, s);
    if (e == hipSuccess)
        e = launch_combine(b->d_descs, b->n, nullptr, partials, counters, s);
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
        gcm_ctx *ctx = b->ctx;
        std::lock_guard<std::mutex> g(ctx->mu);
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
