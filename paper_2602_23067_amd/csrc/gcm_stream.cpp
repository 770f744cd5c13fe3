// gcm_stream.cpp -- streamed AES-GCM: one message fed as a sequence of
// device-resident segments (the paper's map-reduce across pieces of a
// message too large to hold at once).
//
// GHASH is linear in its input, so the GHASH of X = X_1 || X_2 || ... || X_K
// is the XOR over segments of GHASH(X_k) * H^(blocks after X_k).  Each update
// therefore runs only the tile kernel over its segment (its counters start
// after the blocks fed so far) and leaves the segment's tile partials in the
// stream's partials buffer; nothing depends on the previous segment.  The
// final call reduces every segment's partials in one batched combine launch
// (each segment's value lifted by H^(blocks after it), the length block
// included), and one small kernel XORs the lifted values, the length block's
// term L * H and E_K(J0) into the tag or the accept flag.  (A message with
// neither AAD nor payload runs its length block as a segment of its own.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/gcm_mi355.h"
#include "gcm_host.h"

using namespace gcm;

struct gcm_stream {
    gcm_ctx *ctx = nullptr;
    uint32_t op = 0;
    uint32_t slot = 0;
    uint32_t nr = 0;
    uint64_t aad_len = 0;
    uint64_t len = 0;      // payload bytes fed so far
    bool tail = false;     // a segment that was not a whole number of blocks has been fed
    bool closed = false;   // final was called
    uint8_t iv[12] = {0};  // a 96-bit IV (!j0dev)
    bool j0dev = false;    // J0 (other IV lengths) is in the header at kJ0Off
    // header (256 B: the tile kernel's counter word, J0 at kJ0Off), then per
    // segment its tile partials and the slot where its tile-0 wave leaves
    // E_K(J0)
    uint8_t *d_part = nullptr;
    uint64_t part_bytes = 0;  // allocated
    uint64_t part_slots = 0;  // 16-byte slots in use after the header
    std::vector<MsgDesc> segs;
    // pinned staging of the final call's segment descriptors
    MsgDesc *h_desc = nullptr;
    uint64_t h_desc_bytes = 0;
    // recorded after the final call's kernels; it travels with the buffers
    // (a pooled one may still mark an earlier stream's last work, which the
    // host waits for before it rewrites the staging: ev_host_wait)
    hipEvent_t ev = nullptr;
    bool ev_host_wait = false;
    bool ev_recorded = false;  // by this stream's final call
    uint32_t fanin = 2;
};

static constexpr uint64_t kHeader = 256;  // workspace_counter_bytes(1)
static constexpr uint64_t kJ0Off = 128;   // 16 bytes of the header the kernels leave alone
static constexpr size_t kPoolMax = 4;     // buffer sets kept for later streams

// room for `slots` more 16-byte slots (and `extra` bytes after them); a
// larger buffer takes over the slots written so far (stream-ordered copy)
static int part_reserve(gcm_stream *st, uint64_t slots, uint64_t extra, hipStream_t s)
{
    const uint64_t need = kHeader + 16 * (st->part_slots + slots) + extra;
    if (need <= st->part_bytes)
        return GCM_OK;
    const uint64_t want = std::max<uint64_t>(need, std::max<uint64_t>(2 * st->part_bytes, 4ull << 20));
    uint8_t *p = nullptr;
    int rc = ctx_alloc(st->ctx, reinterpret_cast<void **>(&p), want);
    if (rc)
        return rc;
    if (st->d_part && (st->part_slots || st->j0dev)) {
        hipError_t e = hipMemcpyAsync(p, st->d_part, kHeader + 16 * st->part_slots, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);  // the old buffer is freed below
        if (e != hipSuccess) {
            ctx_free(st->ctx, p, want);
            return fail_hip(e, "stream partials copy");
        }
    }
    ctx_free(st->ctx, st->d_part, st->part_bytes);
    st->d_part = p;
    st->part_bytes = want;
    return GCM_OK;
}

// A segment of d.m GHASH blocks (AAD blocks, data blocks, or the length block
// alone): tile launch with the single-message shape for that size; its
// partials and E_K(J0) slot go to the next free slots of the buffer (J0 is
// read from the buffer's header, wherever the buffer is now).
static int run_segment(gcm_stream *st, MsgDesc d, hipStream_t s)
{
    gcm_ctx *ctx = st->ctx;
    const Shape sh = message_shape(ctx, (st->nr - 6) * 4, d.m * 16, 0);
    const uint64_t B = 1ull << sh.log2B;
    d.log2B = sh.log2B;
    d.n_tiles = (d.m + B - 1) / B;
    d.z = d.n_tiles * B - d.m;
    d.tile_lo = 0;
    d.tile_hi = d.n_tiles;
    d.groups = (uint32_t)((d.n_tiles + sh.waves - 1) / sh.waves);
    int rc = part_reserve(st, d.n_tiles + 1, 0, s);
    if (rc)
        return rc;
    d.tile_base = st->part_slots;
    d.j0 = st->j0dev ? (uint64_t)(st->d_part + kJ0Off) : 0;
    rc = launch_tile_range(ctx, d, sh, st->d_part, s);
    if (rc)
        return rc;
    st->part_slots += d.n_tiles + 1;
    st->fanin = sh.fanin;
    st->segs.push_back(d);
    return GCM_OK;
}

static void segment_desc(const gcm_stream *st, MsgDesc *d)
{
    fill_desc(d, st->op, st->iv, 0, 0, 0, 0, 0, 0, 0, (uint64_t)(st->ctx->d_slots + kSlotBytes * st->slot), st->nr, 6,
              16, 0);
}

static void bufs_free(gcm_ctx *ctx, gcm_ctx::StreamBufs &b)
{
    if (b.ev) {
        (void)hipEventSynchronize(b.ev);
        (void)hipEventDestroy(b.ev);
    }
    ctx_free(ctx, b.d_part, b.part_bytes);
    if (b.h_desc)
        (void)hipHostFree(b.h_desc);
}

// The stream's buffers go back to the context's pool (or are freed when it
// is full); queued work that still uses them finishes before st->ev
// completes.  Caller holds ctx->mu.
static void stream_free(gcm_stream *st)
{
    gcm_ctx *ctx = st->ctx;
    gcm_ctx::StreamBufs b = {st->d_part, st->part_bytes, st->h_desc, st->h_desc_bytes, st->ev};
    if (st->d_part && ctx->stream_pool.size() < kPoolMax)
        ctx->stream_pool.push_back(b);
    else
        bufs_free(ctx, b);
    delete st;
}

void gcm::stream_pool_release(gcm_ctx *ctx)
{
    for (auto &b : ctx->stream_pool)
        bufs_free(ctx, b);
    ctx->stream_pool.clear();
}

extern "C" int gcm_stream_begin(gcm_ctx *ctx, uint32_t op, uint32_t slot, const uint8_t *iv, size_t iv_len,
                                const uint8_t *aad_d, uint64_t aad_len, gcm_stream **out, void *stream)
{
    GCM_ABI_TRY
        if (!ctx || !iv || !out)
            return fail(GCM_E_ARG, "NULL argument");
        *out = nullptr;
        if (op > 1)
            return fail(GCM_E_ARG, "op must be 0 (encrypt) or 1 (decrypt-verify)");
        if (!valid_iv_len(iv_len))
            return fail(GCM_E_IVLEN, "IV length %zu is not in 1..%d", iv_len, kMaxIvBytes);
        int rc = check_message(aad_len, 0, aad_d, nullptr, nullptr);
        if (rc)
            return rc;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        std::lock_guard<std::mutex> g(ctx->mu);
        if (slot >= ctx->n_slots || !ctx->slot_used[slot])
            return fail(GCM_E_SLOT, "key slot %u is not registered", slot);
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess)
            return fail_hip(e, "hipSetDevice");
        gcm_stream *st = new (std::nothrow) gcm_stream();
        if (!st)
            return fail(GCM_E_NOMEM, "host allocation failed");
        st->ctx = ctx;
        st->op = op;
        st->slot = slot;
        st->nr = ctx->slot_nr[slot];
        st->aad_len = aad_len;
        if (!ctx->stream_pool.empty()) {
            // this stream's work waits for the last work on the buffers
            const gcm_ctx::StreamBufs b = ctx->stream_pool.back();
            ctx->stream_pool.pop_back();
            st->d_part = b.d_part;
            st->part_bytes = b.part_bytes;
            st->h_desc = b.h_desc;
            st->h_desc_bytes = b.h_desc_bytes;
            st->ev = b.ev;
            if (st->ev) {
                st->ev_host_wait = true;
                e = hipStreamWaitEvent(s, st->ev, 0);
                if (e != hipSuccess)
                    rc = fail_hip(e, "hipStreamWaitEvent");
            }
        }
        if (rc == GCM_OK && iv_len == 12) {
            std::memcpy(st->iv, iv, 12);
        } else if (rc == GCM_OK) {
            // J0 = GHASH_H(IV || 0-pad || [len(IV)]_64) on the device, into
            // the partials buffer's header
            st->j0dev = true;
            rc = part_reserve(st, 0, 0, s);
            if (rc == GCM_OK) {
                IvArg a;
                std::memset(&a, 0, sizeof a);
                a.len = (uint32_t)iv_len;
                std::memcpy(a.b, iv, iv_len);
                e = launch_j0(a, (uint64_t)(ctx->d_slots + kSlotBytes * slot), st->d_part + kJ0Off, nullptr, s);
                if (e != hipSuccess)
                    rc = fail_hip(e, "J0 kernel launch");
            }
        }
        if (rc == GCM_OK && aad_len) {
            // segment 0: the AAD blocks
            MsgDesc d;
            segment_desc(st, &d);
            d.aad = (uint64_t)aad_d;
            d.aad_len = aad_len;
            d.na = (aad_len + 15) / 16;
            d.n = 0;
            d.m = d.na;
            rc = run_segment(st, d, s);
        }
        if (rc) {
            (void)hipStreamSynchronize(s);
            stream_free(st);
            return rc;
        }
        *out = st;
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_stream_update(gcm_stream *st, const uint8_t *in_d, uint64_t len, uint8_t *out_d, void *stream)
{
    GCM_ABI_TRY
        if (!st)
            return fail(GCM_E_ARG, "NULL stream");
        if (st->closed)
            return fail(GCM_E_ARG, "gcm_stream_update after gcm_stream_final");
        if (len == 0)
            return GCM_OK;
        if (st->tail)
            return fail(GCM_E_ARG, "only the last segment may end inside a 16-byte block");
        if (st->len + len > kMaxLen || st->len + len < st->len)
            return fail(GCM_E_TOOLONG, "streamed length beyond the SP 800-38D limit");
        int rc = check_message(0, len, nullptr, in_d, out_d);
        if (rc)
            return rc;
        gcm_ctx *ctx = st->ctx;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        std::lock_guard<std::mutex> g(ctx->mu);
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess)
            return fail_hip(e, "hipSetDevice");
        MsgDesc d;
        segment_desc(st, &d);
        d.in = (uint64_t)in_d;
        d.out = (uint64_t)out_d;
        d.len = len;
        d.na = 0;
        d.n = (len + 15) / 16;
        d.m = d.n;
        d.ctr_off = (uint32_t)(st->len / 16);  // counters continue mod 2^32
        rc = run_segment(st, d, s);
        if (rc)
            return rc;
        st->len += len;
        st->tail = (len & 15) != 0;
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_stream_final(gcm_stream *st, uint8_t *tag_d, int32_t *accept_d, void *stream)
{
    GCM_ABI_TRY
        if (!st || !tag_d || (st->op == 1 && !accept_d))
            return fail(GCM_E_ARG, "NULL argument");
        if (st->closed)
            return fail(GCM_E_ARG, "gcm_stream_final called twice");
        gcm_ctx *ctx = st->ctx;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        std::lock_guard<std::mutex> g(ctx->mu);
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess)
            return fail_hip(e, "hipSetDevice");
        // GHASH's last block, the length block [8|A|]_64 || [8|C|]_64: with
        // nothing before it (no AAD, no payload) it runs as a segment of its
        // own, whose tile-0 wave also leaves E_K(J0); otherwise the fold
        // kernel adds its term L * H, and E_K(J0) is the one the first
        // segment's tile-0 wave left
        const uint64_t abits = st->aad_len * 8, cbits = st->len * 8;
        const uint32_t lenblk[4] = {__builtin_bswap32((uint32_t)(abits >> 32)), __builtin_bswap32((uint32_t)abits),
                                    __builtin_bswap32((uint32_t)(cbits >> 32)), __builtin_bswap32((uint32_t)cbits)};
        const bool len_seg = st->segs.empty();
        int rc = GCM_OK;
        if (len_seg) {
            MsgDesc d;
            segment_desc(st, &d);
            d.aad_len = st->aad_len;
            d.len = st->len;
            d.na = 0;
            d.n = 0;
            d.m = 1;
            rc = run_segment(st, d, s);
            if (rc)
                return rc;
        }
        const uint32_t k = (uint32_t)st->segs.size();
        const uint64_t desc_bytes = (uint64_t)k * sizeof(MsgDesc);
        rc = part_reserve(st, k, desc_bytes + 16, s);
        if (rc)
            return rc;
        uint8_t *vals = st->d_part + kHeader + 16 * st->part_slots;
        MsgDesc *d_descs = reinterpret_cast<MsgDesc *>(vals + 16 * (uint64_t)k);
        // segment j's value is lifted by H^(GHASH blocks after it)
        uint64_t after = len_seg ? 0 : 1;
        for (uint32_t j = k; j-- > 0;) {
            st->segs[j].yout = (uint64_t)(vals + 16 * (uint64_t)j);
            st->segs[j].lift = after;
            after += st->segs[j].m;
        }
        if (after >= (1ull << kTab4Levels))
            return fail(GCM_E_TOOLONG, "streamed message of %llu GHASH blocks is beyond the lift tables",
                        (unsigned long long)after);
        if (st->ev_host_wait) {
            // an earlier stream's copy from the staging must have been read
            e = hipEventSynchronize(st->ev);
            if (e != hipSuccess)
                return fail_hip(e, "hipEventSynchronize");
            st->ev_host_wait = false;
        }
        if (st->h_desc_bytes < desc_bytes) {
            // this stream's own staging (a pooled one comes back only after
            // the device has finished with it)
            if (st->h_desc)
                (void)hipHostFree(st->h_desc);
            st->h_desc = nullptr;
            st->h_desc_bytes = 0;
            const uint64_t want = std::max<uint64_t>(desc_bytes, 64 * sizeof(MsgDesc));
            e = hipHostMalloc(reinterpret_cast<void **>(&st->h_desc), want, hipHostMallocDefault);
            if (e != hipSuccess) {
                st->h_desc = nullptr;
                return fail_hip(e, "pinned descriptor staging");
            }
            st->h_desc_bytes = want;
        }
        std::memcpy(st->h_desc, st->segs.data(), desc_bytes);
        e = hipMemcpyAsync(d_descs, st->h_desc, desc_bytes, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = launch_combine(d_descs, k, nullptr, st->d_part + kHeader, reinterpret_cast<uint32_t *>(st->d_part),
                               st->fanin, s);
        const MsgDesc &first = st->segs.front();
        if (e == hipSuccess)
            e = launch_fold(vals, k, st->d_part + kHeader + 16 * (first.tile_base + first.n_tiles), tag_d, accept_d,
                            st->op, 16, first.slot, len_seg ? nullptr : lenblk, s);
        if (e == hipSuccess && !st->ev)
            e = hipEventCreateWithFlags(&st->ev, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventRecord(st->ev, s);
        if (e != hipSuccess)
            return fail_hip(e, "stream final kernels");
        st->ev_recorded = true;
        st->closed = true;
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_stream_destroy(gcm_stream *st)
{
    GCM_ABI_TRY
        if (!st)
            return fail(GCM_E_ARG, "NULL stream");
        gcm_ctx *ctx = st->ctx;
        std::lock_guard<std::mutex> g(ctx->mu);
        (void)hipSetDevice(ctx->device);
        // after a final call the buffers' event marks their last use; a
        // stream abandoned before it may still have work queued anywhere
        if (!st->ev_recorded)
            (void)hipDeviceSynchronize();
        stream_free(st);
        return GCM_OK;
    GCM_ABI_CATCH
}
