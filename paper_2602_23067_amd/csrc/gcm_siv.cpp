// gcm_siv.cpp -- AES-GCM-SIV (RFC 8452) on the device, for callers that need
// nonce-misuse resistance (the alternative AEAD the paper names under future
// directions).
//
// Per message, all on the caller's stream:
//   k_siv_derive + k_key_tables   message keys from the key-generating key
//                                 and the nonce, expanded into a key slot in
//                                 the workspace (encryption round keys, H'
//                                 and every GHASH table for H').
//   k_siv_tiles (hash)            encrypt: POLYVAL of AAD and plaintext as
//                                 GHASH_H' over byte-reversed blocks, in
//                                 tiles; the combine writes the value.
//   k_siv_tag                     tag = AES(POLYVAL ^ nonce, msb cleared).
//   k_siv_tiles (ctr)             encrypt: counter mode from the tag.
// Decrypt-verify fuses counter mode with the POLYVAL of its output (one
// pass), then k_siv_tag compares tags and the zero-fill clears a rejected
// plaintext.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "../../include/gcm_mi355.h"
#include "gcm_host.h"

using namespace gcm;

namespace {

constexpr uint64_t kSivMax = 1ull << 36;  // P_MAX = A_MAX = 2^36 bytes
constexpr uint64_t kSivStateOff = kSlotBytes;         // 16 B POLYVAL-as-GHASH value, then 16 B counter block
constexpr uint64_t kSivTilesOff = kSlotBytes + 256;   // counters and partials

// GCM-SIV's tile kernels take the untuned single-message shape (the
// autotuner times GCM's kernels, not these): the wave count that spreads a
// message over the most compute units, then the tile size; explicit
// gcm_set_launch settings apply.
Shape siv_shape(const gcm_ctx *ctx, uint64_t m)
{
    Shape sh;
    sh.waves = ctx->cfg_waves                       ? ctx->cfg_waves
               : (ctx->cfg_log2B || ctx->cfg_gpc) ? 16u
                                                  : heuristic_waves(m, (uint64_t)ctx->cu_count, groups_per_cu);
    sh.gpc = ctx->cfg_gpc ? ctx->cfg_gpc : groups_per_cu(sh.waves);
    sh.log2B = ctx->cfg_log2B ? ctx->cfg_log2B : heuristic_log2B(m, (uint64_t)ctx->cu_count * sh.gpc * sh.waves);
    sh.fanin = ctx->cfg_fanin ? ctx->cfg_fanin : 2;
    return sh;
}

uint64_t siv_tiles(const gcm_ctx *ctx, uint64_t len, uint64_t aad_len, Shape *sh)
{
    const uint64_t m = ghash_blocks(aad_len, len);
    *sh = siv_shape(ctx, m);
    return (m + (1ull << sh->log2B) - 1) >> sh->log2B;
}

int launch_siv_pass(gcm_ctx *ctx, int pass, const MsgDesc &d, uint32_t waves, uint32_t gpc, void *partials,
                    hipStream_t s)
{
    const uint32_t items = (uint32_t)((d.n_tiles + waves - 1) / waves);
    if (items == 0)
        return GCM_OK;
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(items, (uint32_t)ctx->cu_count * gpc));
    hipError_t e = launch_siv_tiles((int)waves, pass, d, items, ctx->d_tables, partials, grid, s);
    if (e != hipSuccess)
        return fail_hip(e, "GCM-SIV tile kernel launch");
    return GCM_OK;
}

int siv_common(gcm_ctx *ctx, uint32_t op, uint32_t slot, const uint8_t *nonce, size_t nonce_len,
               const uint8_t *aad_d, uint64_t aad_len, const uint8_t *in_d, uint64_t len, uint8_t *out_d,
               uint8_t *tag_d, int32_t *ok_d, void *ws, uint64_t ws_bytes, void *stream)
{
    if (!ctx || !nonce || !tag_d || (op == 1 && !ok_d) || !ws)
        return fail(GCM_E_ARG, "NULL argument");
    if (nonce_len != 12)
        return fail(GCM_E_IVLEN, "GCM-SIV nonces are 12 bytes, not %zu", nonce_len);
    if (len > kSivMax || aad_len > kSivMax)
        return fail(GCM_E_TOOLONG, "len %llu / aad_len %llu beyond the 2^36-byte limits",
                    (unsigned long long)len, (unsigned long long)aad_len);
    PlanError err;
    if (check_buffers((uint64_t)aad_d, aad_len, (uint64_t)in_d, (uint64_t)out_d, len, (uint64_t)tag_d, 16,
                      (uint64_t)ok_d, &err))
        return plan_error(err);
    int rc = GCM_OK;
    if ((uintptr_t)ws & 255)
        return fail(GCM_E_ARG, "workspace must be 256-byte aligned");
    std::lock_guard<std::mutex> g(ctx->mu);
    if (slot >= ctx->n_slots || !ctx->slot_used[slot])
        return fail(GCM_E_SLOT, "key slot %u is not registered", slot);
    const uint32_t nr = ctx->slot_nr[slot];
    if (nr != 10 && nr != 14)
        return fail(GCM_E_KEYLEN, "GCM-SIV key-generating keys are 16 or 32 bytes");
    Shape sh;
    const uint64_t T = siv_tiles(ctx, len, aad_len, &sh);
    const uint32_t log2B = sh.log2B, waves = sh.waves, gpc = sh.gpc;
    const uint64_t need = kSivTilesOff + workspace_bytes_for(T, 1);
    if (ws_bytes < need)
        return fail(GCM_E_ARG, "workspace of %llu bytes is smaller than the %llu needed",
                    (unsigned long long)ws_bytes, (unsigned long long)need);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess)
        return fail_hip(e, "hipSetDevice");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint8_t *base = reinterpret_cast<uint8_t *>(ws);
    const uint64_t mslot = (uint64_t)base;
    uint8_t *gval = base + kSivStateOff, *ctr = base + kSivStateOff + 16;
    uint32_t *counters = reinterpret_cast<uint32_t *>(base + kSivTilesOff);
    uint8_t *partials = base + kSivTilesOff + workspace_counter_bytes(1);
    static const uint8_t zero_iv[12] = {0};

    e = launch_siv_derive((uint64_t)(ctx->d_slots + kSlotBytes * slot), nonce, mslot, op == 1 ? tag_d : nullptr,
                          ctr, ctx->d_tables, ctx->d_tables + 256, ctx->d_frob, s);
    if (e != hipSuccess)
        return fail_hip(e, "GCM-SIV key derivation launch");
    // hash (encrypt) or fused decrypt pass over AAD || data || length block
    MsgDesc d;
    fill_desc(&d, op, zero_iv, (uint64_t)aad_d, aad_len, (uint64_t)in_d, (uint64_t)out_d, len, 0,
              (uint64_t)ok_d, mslot, nr, log2B, waves, 0);
    d.j0 = (uint64_t)ctr;
    d.yout = (uint64_t)gval;
    rc = launch_siv_pass(ctx, op == 0 ? 0 : 2, d, waves, gpc, partials, s);
    if (rc)
        return rc;
    e = launch_combine(nullptr, 1, &d, partials, counters, sh.fanin, s);
    if (e == hipSuccess)
        e = launch_siv_tag(mslot, gval, nonce, op == 0 ? tag_d : nullptr, ctr, op == 1 ? tag_d : nullptr, ok_d,
                           counters, ctx->d_tables, ctx->d_tables + 256, s);
    if (e != hipSuccess)
        return fail_hip(e, "GCM-SIV kernel launch");
    if (op == 1) {
        const uint64_t chunks = (len / 16 + 255) / 256;
        const uint32_t zgrid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(chunks, 4096));
        e = launch_zerofill(nullptr, &d, counters, zgrid, s);
        if (e != hipSuccess)
            return fail_hip(e, "zero-fill launch");
        return GCM_OK;
    }
    if (len == 0)
        return GCM_OK;
    // encrypt: counter mode from the tag, over the data blocks alone
    const Shape cs = siv_shape(ctx, (len + 15) / 16 + 1);
    const uint32_t cl = cs.log2B, cw = cs.waves, cg = cs.gpc;
    MsgDesc dc;
    fill_desc(&dc, 2, zero_iv, 0, 0, (uint64_t)in_d, (uint64_t)out_d, len, 0, 0, mslot, nr, cl, cw, 0);
    dc.j0 = (uint64_t)ctr;
    return launch_siv_pass(ctx, 1, dc, cw, cg, nullptr, s);
}

}  // namespace

extern "C" uint64_t gcm_siv_workspace_size(gcm_ctx *ctx, uint64_t len, uint64_t aad_len)
{
    GCM_ABI_TRY
        if (!ctx)
            return 0;
        std::lock_guard<std::mutex> g(ctx->mu);
        Shape sh;
        const uint64_t T = siv_tiles(ctx, len, aad_len, &sh);
        if (ctx->cfg_log2B)
            return kSivTilesOff + workspace_bytes_for(T, 1);
        return kSivTilesOff +
               workspace_bytes_for(tiles_bound_upto(ghash_blocks(aad_len, len), T, resident_bound(ctx)), 1);
    GCM_ABI_CATCH_VALUE(0)
}

extern "C" int gcm_siv_encrypt_async(gcm_ctx *ctx, uint32_t slot, const uint8_t *nonce, size_t nonce_len,
                                     const uint8_t *aad_d, uint64_t aad_len, const uint8_t *pt_d, uint64_t len,
                                     uint8_t *ct_d, uint8_t *tag_d, void *workspace_d, uint64_t workspace_bytes,
                                     void *stream)
{
    GCM_ABI_TRY
        return siv_common(ctx, 0, slot, nonce, nonce_len, aad_d, aad_len, pt_d, len, ct_d, tag_d, nullptr, workspace_d,
                          workspace_bytes, stream);
    GCM_ABI_CATCH
}

extern "C" int gcm_siv_decrypt_verify_async(gcm_ctx *ctx, uint32_t slot, const uint8_t *nonce, size_t nonce_len,
                                            const uint8_t *aad_d, uint64_t aad_len, const uint8_t *ct_d,
                                            uint64_t len, const uint8_t *tag_d, uint8_t *pt_d, int32_t *accept_d,
                                            void *workspace_d, uint64_t workspace_bytes, void *stream)
{
    GCM_ABI_TRY
        return siv_common(ctx, 1, slot, nonce, nonce_len, aad_d, aad_len, ct_d, len, pt_d, const_cast<uint8_t *>(tag_d),
                          accept_d, workspace_d, workspace_bytes, stream);
    GCM_ABI_CATCH
}
