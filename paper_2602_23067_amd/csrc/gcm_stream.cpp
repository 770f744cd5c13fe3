// gcm_stream.cpp -- streamed AES-GCM: one message fed as a sequence of
// device-resident segments, with (GHASH value, block count) carried across
// calls on the device (the monoid combine(L, R) = L*H^|R| ^ R, applied here
// as a Horner continuation).
//
// Each segment is an ordinary tile launch of the device-J0 kernel variant:
// its counters start at J0 + 1 + (blocks before it), the running GHASH value
// Y is XORed into its first block (Horner from Y over X_1..X_m equals Horner
// from zero over X_1 ^ Y, X_2, ..., X_m), and the combine writes the result
// back as the new Y.  The AAD is the first segment; the final call is a
// segment made of the length block alone, whose combine adds E_K(J0) and
// writes (or checks) the tag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>

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
    uint8_t *d_state = nullptr;  // 16 B running GHASH value, then 16 B J0
    void *ws = nullptr;
    uint64_t ws_bytes = 0;
};

static constexpr uint64_t kStateBytes = 256;

static int stream_ws(gcm_stream *st, uint64_t bytes)
{
    if (st->ws_bytes >= bytes)
        return GCM_OK;
    ctx_free(st->ctx, st->ws, st->ws_bytes);
    st->ws = nullptr;
    st->ws_bytes = 0;
    const uint64_t want = std::max<uint64_t>(bytes, 1ull << 16);
    int rc = ctx_alloc(st->ctx, &st->ws, want);
    if (rc)
        return rc;
    st->ws_bytes = want;
    return GCM_OK;
}

// one segment: n_aad AAD blocks or data blocks (never both), or the length
// block alone (final); geometry over exactly its own blocks
static int run_segment(gcm_stream *st, const MsgDesc &base, hipStream_t s)
{
    gcm_ctx *ctx = st->ctx;
    MsgDesc d = base;
    // the single-message shape for a message of this segment's blocks
    const Shape sh = message_shape(ctx, (st->nr - 6) * 4, d.m * 16, 0);
    const uint32_t log2B = sh.log2B, waves = sh.waves;
    const uint64_t B = 1ull << log2B;
    d.log2B = log2B;
    d.n_tiles = (d.m + B - 1) / B;
    d.z = d.n_tiles * B - d.m;
    d.tile_lo = 0;
    d.tile_hi = d.n_tiles;
    d.groups = (uint32_t)((d.n_tiles + waves - 1) / waves);
    int rc = stream_ws(st, workspace_bytes_for(d.n_tiles, 1));
    if (rc)
        return rc;
    rc = launch_tile_range(ctx, d, sh, st->ws, s);
    if (rc)
        return rc;
    uint32_t *counters = reinterpret_cast<uint32_t *>(st->ws);
    const uint8_t *partials = reinterpret_cast<const uint8_t *>(st->ws) + workspace_counter_bytes(1);
    hipError_t e = launch_combine(nullptr, 1, &d, partials, counters, sh.fanin, s);
    if (e != hipSuccess)
        return fail_hip(e, "combine launch");
    return GCM_OK;
}

static void segment_desc(const gcm_stream *st, MsgDesc *d)
{
    static const uint8_t zero_iv[12] = {0};
    fill_desc(d, st->op, zero_iv, 0, 0, 0, 0, 0, 0, 0, (uint64_t)(st->ctx->d_slots + kSlotBytes * st->slot), st->nr,
              6, 16, 0);
    d->j0 = (uint64_t)(st->d_state + 16);
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
        rc = ctx_alloc(ctx, reinterpret_cast<void **>(&st->d_state), kStateBytes);
        if (rc) {
            delete st;
            return rc;
        }
        // J0 (any IV length) and Y = 0
        IvArg a;
        std::memset(&a, 0, sizeof a);
        a.len = (uint32_t)iv_len;
        std::memcpy(a.b, iv, iv_len);
        e = launch_j0(a, (uint64_t)(ctx->d_slots + kSlotBytes * slot), st->d_state + 16, st->d_state, s);
        if (e != hipSuccess)
            rc = fail_hip(e, "J0 kernel launch");
        if (rc == GCM_OK && aad_len) {
            // segment 0: the AAD blocks, from Y = 0
            MsgDesc d;
            segment_desc(st, &d);
            d.aad = (uint64_t)aad_d;
            d.aad_len = aad_len;
            d.na = (aad_len + 15) / 16;
            d.n = 0;
            d.m = d.na;
            d.yout = (uint64_t)st->d_state;
            rc = run_segment(st, d, s);
        }
        if (rc) {
            (void)hipStreamSynchronize(s);
            ctx_free(ctx, st->ws, st->ws_bytes);
            ctx_free(ctx, st->d_state, kStateBytes);
            delete st;
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
        d.ystate = (uint64_t)st->d_state;
        d.yout = (uint64_t)st->d_state;
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
        // the length block alone: S = (Y ^ [8|A|]_64 || [8|C|]_64) * H, tag = S ^ E_K(J0)
        MsgDesc d;
        segment_desc(st, &d);
        d.aad_len = st->aad_len;
        d.len = st->len;
        d.na = 0;
        d.n = 0;
        d.m = 1;
        d.ystate = (uint64_t)st->d_state;
        d.tag = (uint64_t)tag_d;
        d.ok = (uint64_t)accept_d;
        int rc = run_segment(st, d, s);
        if (rc)
            return rc;
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
        (void)hipDeviceSynchronize();  // the stream's queued segments may still read its state
        ctx_free(ctx, st->ws, st->ws_bytes);
        ctx_free(ctx, st->d_state, kStateBytes);
        delete st;
        return GCM_OK;
    GCM_ABI_CATCH
}
