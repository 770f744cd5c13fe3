// gcm_pipeline.cpp -- host-to-host AES-GCM: the message stays in host memory
// and moves through a ring of device chunk buffers, with the host-to-device
// copy of one chunk, the tile kernel of the previous one and the
// device-to-host copy of the one before that in flight at the same time on
// three streams (the paper's dual-stream pipeline over pinned memory, here
// for one message).
//
// Chunks are whole runs of wave tiles, so one message is still one GCM
// computation: every chunk's tile launch writes its tiles' partial hashes
// into the same workspace, and a single combine after the last chunk forms
// the tag exactly as for a device-resident message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "../../include/gcm_mi355.h"
#include "gcm_host.h"

using namespace gcm;

static constexpr uint64_t kDefaultChunk = 64ull << 20;

void gcm::pipeline_release(gcm_ctx *ctx)
{
    for (int b = 0; b < gcm_ctx::kPipeBufs; ++b) {
        ctx_free(ctx, ctx->pipe_buf[b], ctx->pipe_buf_bytes);
        ctx->pipe_buf[b] = nullptr;
        if (ctx->pipe_in[b])
            (void)hipEventDestroy(ctx->pipe_in[b]);
        if (ctx->pipe_done[b])
            (void)hipEventDestroy(ctx->pipe_done[b]);
        if (ctx->pipe_free[b])
            (void)hipEventDestroy(ctx->pipe_free[b]);
        ctx->pipe_in[b] = ctx->pipe_done[b] = ctx->pipe_free[b] = nullptr;
        ctx->pipe_used[b] = false;
    }
    ctx->pipe_buf_bytes = 0;
    ctx_free(ctx, ctx->pipe_aad, ctx->pipe_aad_bytes);
    ctx->pipe_aad = nullptr;
    ctx->pipe_aad_bytes = 0;
    for (hipStream_t *s : {&ctx->pipe_h2d, &ctx->pipe_comp, &ctx->pipe_d2h}) {
        if (*s)
            (void)hipStreamDestroy(*s);
        *s = nullptr;
    }
    ctx->pipe_ready = false;
}

// streams and events (once per context); default priority, non-blocking
static int pipeline_streams(gcm_ctx *ctx)
{
    if (ctx->pipe_ready)
        return GCM_OK;
    hipError_t e = hipSuccess;
    for (hipStream_t *s : {&ctx->pipe_h2d, &ctx->pipe_comp, &ctx->pipe_d2h})
        if (e == hipSuccess && !*s)
            e = hipStreamCreateWithFlags(s, hipStreamNonBlocking);
    for (int b = 0; b < gcm_ctx::kPipeBufs && e == hipSuccess; ++b) {
        for (hipEvent_t *ev : {&ctx->pipe_in[b], &ctx->pipe_done[b], &ctx->pipe_free[b]})
            if (e == hipSuccess && !*ev)
                e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        pipeline_release(ctx);
        return fail_hip(e, "pipeline stream/event creation");
    }
    ctx->pipe_ready = true;
    return GCM_OK;
}

static int pipeline_buffers(gcm_ctx *ctx, uint64_t chunk_bytes, uint64_t aad_bytes)
{
    if (ctx->pipe_buf_bytes < chunk_bytes) {
        for (int b = 0; b < gcm_ctx::kPipeBufs; ++b) {
            ctx_free(ctx, ctx->pipe_buf[b], ctx->pipe_buf_bytes);
            ctx->pipe_buf[b] = nullptr;
            ctx->pipe_used[b] = false;
        }
        ctx->pipe_buf_bytes = 0;
        for (int b = 0; b < gcm_ctx::kPipeBufs; ++b) {
            int rc = ctx_alloc(ctx, reinterpret_cast<void **>(&ctx->pipe_buf[b]), chunk_bytes);
            if (rc) {
                for (int q = 0; q < b; ++q) {
                    ctx_free(ctx, ctx->pipe_buf[q], chunk_bytes);
                    ctx->pipe_buf[q] = nullptr;
                }
                return rc;
            }
        }
        ctx->pipe_buf_bytes = chunk_bytes;
    }
    if (aad_bytes && ctx->pipe_aad_bytes < aad_bytes) {
        ctx_free(ctx, ctx->pipe_aad, ctx->pipe_aad_bytes);
        ctx->pipe_aad = nullptr;
        ctx->pipe_aad_bytes = 0;
        int rc = ctx_alloc(ctx, reinterpret_cast<void **>(&ctx->pipe_aad), aad_bytes);
        if (rc)
            return rc;
        ctx->pipe_aad_bytes = aad_bytes;
    }
    return GCM_OK;
}

// wait for everything the pipeline enqueued (error paths included)
static hipError_t pipeline_drain(gcm_ctx *ctx)
{
    hipError_t e = hipSuccess;
    for (hipStream_t s : {ctx->pipe_h2d, ctx->pipe_comp, ctx->pipe_d2h}) {
        const hipError_t q = hipStreamSynchronize(s);
        if (e == hipSuccess)
            e = q;
    }
    return e;
}

static int run_pipeline(gcm_ctx *ctx, uint32_t op, const uint8_t *key, size_t key_len, const uint8_t *iv,
                        size_t iv_len, const uint8_t *aad_h, uint64_t aad_len, const uint8_t *in_h, uint64_t len,
                        uint8_t *out_h, const uint8_t *tag_in, uint8_t *tag_out, int *accept)
{
    if (!ctx || !key || !iv || (op == 0 && !tag_out) || (op == 1 && (!tag_in || !accept)))
        return fail(GCM_E_ARG, "NULL argument");
    if (key_len != 16 && key_len != 24 && key_len != 32)
        return fail(GCM_E_KEYLEN, "key length %zu is not 16, 24 or 32", key_len);
    if (!valid_iv_len(iv_len))
        return fail(GCM_E_IVLEN, "IV length %zu is not in 1..%d", iv_len, kMaxIvBytes);
    if (len > kMaxLen || aad_len > kMaxAad)
        return fail(GCM_E_TOOLONG, "len %llu / aad_len %llu beyond the SP 800-38D limits", (unsigned long long)len,
                    (unsigned long long)aad_len);
    if ((len && (!in_h || !out_h)) || (aad_len && !aad_h))
        return fail(GCM_E_ARG, "NULL host buffer with non-zero length");
    const uintptr_t i = (uintptr_t)in_h, o = (uintptr_t)out_h;
    if (len && i != o && i < o + len && o < i + len)
        return fail(GCM_E_ALIAS, "input and output overlap without being identical");

    std::lock_guard<std::mutex> g(ctx->mu);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess)
        return fail_hip(e, "hipSetDevice");
    int rc = pipeline_streams(ctx);
    if (rc)
        return rc;
    const uint32_t nr = (uint32_t)(key_len / 4 + 6);
    const Shape shape = message_shape(ctx, (nr - 6) * 4, len, aad_len);
    const uint32_t log2B = shape.log2B, waves = shape.waves;
    const uint64_t B = 1ull << log2B;
    MsgDesc d;
    static const uint8_t zero_iv[12] = {0};
    fill_desc(&d, op, zero_iv, 0, aad_len, 0, 0, len, (uint64_t)ctx->d_io, (uint64_t)(ctx->d_io + 16), 0, nr,
              log2B, waves, 0);
    const uint64_t want = ctx->pipe_chunk ? ctx->pipe_chunk : kDefaultChunk;
    const uint64_t tiles_per_chunk = std::max<uint64_t>(1, want / (B * 16));
    rc = ensure_ws_locked(ctx, workspace_bytes_for(d.n_tiles, 1));
    if (rc == GCM_OK)
        rc = pipeline_buffers(ctx, tiles_per_chunk * B * 16, (aad_len + 255) / 256 * 256);
    if (rc)
        return rc;

    hipStream_t sh = ctx->pipe_h2d, sc = ctx->pipe_comp, sd = ctx->pipe_d2h;
    uint32_t slot;
    rc = cached_slot_locked(ctx, key, key_len, &slot, sc);
    if (rc)
        return rc;
    d.slot = (uint64_t)(ctx->d_slots + kSlotBytes * slot);
    d.aad = aad_len ? (uint64_t)ctx->pipe_aad : 0;
    rc = set_iv(&d, iv, iv_len, ctx->d_ws, sc);
    if (rc) {
        (void)pipeline_drain(ctx);
        return rc;
    }
    if (aad_len)
        e = hipMemcpyAsync(ctx->pipe_aad, aad_h, aad_len, hipMemcpyHostToDevice, sc);
    if (e == hipSuccess && op == 1)
        e = hipMemcpyAsync(ctx->d_io, tag_in, 16, hipMemcpyHostToDevice, sc);
    if (e != hipSuccess) {
        (void)pipeline_drain(ctx);
        return fail_hip(e, "pipeline upload");
    }

    // chunk c covers tiles [c*K, (c+1)*K) and data blocks [jlo, jhi) of them
    const int64_t shift = (int64_t)d.z + (int64_t)d.na;  // virtual index of data block j is j + shift
    const uint64_t n_chunks = (d.n_tiles + tiles_per_chunk - 1) / tiles_per_chunk;
    for (uint64_t c = 0; c < n_chunks && rc == GCM_OK; ++c) {
        const uint64_t t0 = c * tiles_per_chunk, t1 = std::min(d.n_tiles, t0 + tiles_per_chunk);
        const int64_t vlo = (int64_t)(t0 * B) - shift, vhi = (int64_t)(t1 * B) - shift;
        const uint64_t jlo = (uint64_t)std::min<int64_t>(std::max<int64_t>(vlo, 0), (int64_t)d.n);
        const uint64_t jhi = (uint64_t)std::min<int64_t>(std::max<int64_t>(vhi, 0), (int64_t)d.n);
        const uint64_t blo = jlo * 16, bhi = std::min(jhi * 16, len);
        const int b = (int)(c % gcm_ctx::kPipeBufs);
        uint8_t *buf = ctx->pipe_buf[b];
        const bool data = bhi > blo;
        if (data) {
            if (ctx->pipe_used[b])
                e = hipStreamWaitEvent(sh, ctx->pipe_free[b], 0);  // the chunk before in this buffer is out
            if (e == hipSuccess)
                e = hipMemcpyAsync(buf, in_h + blo, bhi - blo, hipMemcpyHostToDevice, sh);
            if (e == hipSuccess)
                e = hipEventRecord(ctx->pipe_in[b], sh);
            if (e == hipSuccess)
                e = hipStreamWaitEvent(sc, ctx->pipe_in[b], 0);
        }
        if (e != hipSuccess)
            break;
        // the kernel addresses the message by block index: the buffer stands
        // for message bytes [blo, bhi), and this launch touches no others
        MsgDesc dc = d;
        dc.tile_lo = t0;
        dc.tile_hi = t1;
        dc.in = dc.out = (uint64_t)buf - blo;
        rc = launch_tile_range(ctx, dc, shape, ctx->d_ws, sc);
        if (rc)
            break;
        if (data) {
            e = hipEventRecord(ctx->pipe_done[b], sc);
            if (e == hipSuccess)
                e = hipStreamWaitEvent(sd, ctx->pipe_done[b], 0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(out_h + blo, buf, bhi - blo, hipMemcpyDeviceToHost, sd);
            if (e == hipSuccess)
                e = hipEventRecord(ctx->pipe_free[b], sd);
            if (e != hipSuccess)
                break;
            ctx->pipe_used[b] = true;
        }
    }
    if (rc == GCM_OK && e == hipSuccess) {
        uint32_t *counters = reinterpret_cast<uint32_t *>(ctx->d_ws);
        const uint8_t *partials = ctx->d_ws + workspace_counter_bytes(1);
        e = launch_combine(nullptr, 1, &d, partials, counters, shape.fanin, sc);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->h_io, ctx->d_io, 32, hipMemcpyDeviceToHost, sc);
    }
    const hipError_t ed = pipeline_drain(ctx);
    if (rc)
        return rc;
    if (e == hipSuccess)
        e = ed;
    if (e != hipSuccess)
        return fail_hip(e, "pipeline");
    if (op == 0) {
        std::memcpy(tag_out, ctx->h_io, 16);
    } else {
        int32_t ok;
        std::memcpy(&ok, ctx->h_io + 16, 4);
        *accept = ok == 1 ? 1 : 0;
        if (!*accept && len)
            std::memset(out_h, 0, len);  // no plaintext leaves a rejected message
    }
    return GCM_OK;
}

extern "C" int gcm_set_pipeline(gcm_ctx *ctx, uint64_t chunk_bytes)
{
    GCM_ABI_TRY
        if (!ctx)
            return fail(GCM_E_ARG, "gcm_set_pipeline: NULL context");
        if (chunk_bytes && (chunk_bytes < 4096 || chunk_bytes > (1ull << 34)))
            return fail(GCM_E_ARG, "gcm_set_pipeline: chunk_bytes must be 0 or 4 KiB..16 GiB");
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->pipe_chunk = chunk_bytes;
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_encrypt_host(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                                const uint8_t *aad_h, uint64_t aad_len, const uint8_t *pt_h, uint64_t len,
                                uint8_t *ct_h, uint8_t tag_out[16])
{
    GCM_ABI_TRY
        return run_pipeline(ctx, 0, key, key_len, iv, iv_len, aad_h, aad_len, pt_h, len, ct_h, nullptr, tag_out,
                            nullptr);
    GCM_ABI_CATCH
}

extern "C" int gcm_decrypt_verify_host(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv,
                                       size_t iv_len, const uint8_t *aad_h, uint64_t aad_len, const uint8_t *ct_h,
                                       uint64_t len, const uint8_t tag[16], uint8_t *pt_h, int *accept)
{
    GCM_ABI_TRY
        return run_pipeline(ctx, 1, key, key_len, iv, iv_len, aad_h, aad_len, ct_h, len, pt_h, tag, nullptr, accept);
    GCM_ABI_CATCH
}
