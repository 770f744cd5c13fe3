// gcm_autotune.cpp -- exhaustive launch-shape search (the paper tunes its
// kernel parameters per GPU the same way: an exhaustive sweep, keeping the
// fastest), with a bit-equality check across every candidate.
//
// For one (key size, message size) point the search times every shape in
// {log2 tile blocks} x {waves per workgroup} on a scratch message with HIP
// events, requires all of them to produce the same tag (the counter map and
// GHASH exponents derive from block indices only), and records the fastest in
// the context's cache, keyed by (key bytes, floor(log2(len))).  The launch
// planner consults the cache whenever no explicit shape is set.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gcm_mi355.h"
#include "gcm_host.h"

using namespace gcm;

static uint32_t size_bucket(uint64_t len)
{
    uint32_t b = 0;
    while (b < 63 && (2ull << b) <= len)
        ++b;
    return b;
}

bool gcm::tuned_shape(const gcm_ctx *ctx, uint32_t key_len, uint64_t len, uint32_t *log2B, uint32_t *waves)
{
    auto it = ctx->tuned.find((uint64_t)key_len << 32 | size_bucket(len));
    if (it == ctx->tuned.end())
        return false;
    *log2B = it->second.first;
    *waves = it->second.second;
    return true;
}

extern "C" int gcm_autotune(gcm_ctx *ctx, uint32_t key_len, uint64_t len, uint32_t reps, gcm_tune_result *out,
                            void *stream)
{
    GCM_ABI_TRY
        if (!ctx)
            return fail(GCM_E_ARG, "gcm_autotune: NULL context");
        if (key_len != 16 && key_len != 24 && key_len != 32)
            return fail(GCM_E_KEYLEN, "gcm_autotune: key length %u", key_len);
        if (len == 0 || len > kMaxLen)
            return fail(GCM_E_ARG, "gcm_autotune: len must be in 1..2^36-32");
        if (reps == 0)
            reps = 3;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        std::lock_guard<std::mutex> g(ctx->mu);
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess)
            return fail_hip(e, "hipSetDevice");

        // scratch: payload in/out + workspace sized for the smallest tile
        const uint64_t m = (len + 15) / 16 + 1;
        const uint64_t ws_bytes = workspace_bytes_for((m + 63) / 64, 1);
        uint8_t *buf = nullptr;
        int rc = ctx_alloc(ctx, reinterpret_cast<void **>(&buf), 2 * ((len + 255) / 256 * 256) + ws_bytes + 256);
        if (rc)
            return rc;
        const uint64_t bytes = 2 * ((len + 255) / 256 * 256) + ws_bytes + 256;
        uint8_t *in = buf, *outp = buf + (len + 255) / 256 * 256, *ws = outp + (len + 255) / 256 * 256;
        uint8_t *tag = ws + ws_bytes;
        e = hipMemsetAsync(in, 0x5c, len, s);
        uint8_t key[32];
        for (uint32_t i = 0; i < 32; ++i)
            key[i] = (uint8_t)(0x3d * i + 7);
        const uint8_t iv[12] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12};
        uint32_t slot = 0;
        if (e == hipSuccess) {
            rc = register_key_locked(ctx, key, key_len, &slot, s);
            if (rc) {
                ctx_free(ctx, buf, bytes);
                return rc;
            }
        }
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        if (e == hipSuccess)
            e = hipEventCreate(&ev0);
        if (e == hipSuccess)
            e = hipEventCreate(&ev1);

        const uint32_t wave_opts[3] = {8, 12, 16};
        float best_ms = 1e30f;
        uint32_t best_l = 0, best_w = 0, tried = 0;
        bool all_equal = true;
        uint8_t ref_tag[16], cur_tag[16];
        bool have_ref = false;
        const bool save_prof = ctx->prof;
        ctx->prof = false;
        for (uint32_t l = 8; l <= 16 && e == hipSuccess && rc == GCM_OK; ++l) {
            if ((1ull << l) > 4 * m && l > 8)
                break;  // tiles larger than the whole message add nothing
            for (uint32_t w : wave_opts) {
                const uint32_t gpc = (uint32_t)max_groups_per_cu((int)w);
                MsgDesc d;
                fill_desc(&d, 0, iv, 0, 0, (uint64_t)in, (uint64_t)outp, len, (uint64_t)tag, 0,
                          (uint64_t)(ctx->d_slots + kSlotBytes * slot), key_len / 4 + 6, l, w, 0);
                rc = launch_single(ctx, d, w, gpc, ws, s);  // warm-up
                float total = 0.f;
                for (uint32_t r = 0; r < reps && rc == GCM_OK && e == hipSuccess; ++r) {
                    e = hipEventRecord(ev0, s);
                    if (e == hipSuccess)
                        rc = launch_single(ctx, d, w, gpc, ws, s);
                    if (e == hipSuccess && rc == GCM_OK)
                        e = hipEventRecord(ev1, s);
                    if (e == hipSuccess)
                        e = hipEventSynchronize(ev1);
                    float ms = 0.f;
                    if (e == hipSuccess)
                        e = hipEventElapsedTime(&ms, ev0, ev1);
                    total += ms;
                }
                if (e == hipSuccess && rc == GCM_OK)
                    e = hipMemcpy(cur_tag, tag, 16, hipMemcpyDeviceToHost);
                if (e != hipSuccess || rc != GCM_OK)
                    break;
                if (!have_ref) {
                    std::memcpy(ref_tag, cur_tag, 16);
                    have_ref = true;
                } else if (std::memcmp(ref_tag, cur_tag, 16) != 0) {
                    all_equal = false;
                }
                ++tried;
                const float ms = total / (float)reps;
                if (ms < best_ms) {
                    best_ms = ms;
                    best_l = l;
                    best_w = w;
                }
            }
        }
        ctx->prof = save_prof;
        if (ev0)
            (void)hipEventDestroy(ev0);
        if (ev1)
            (void)hipEventDestroy(ev1);
        (void)hipStreamSynchronize(s);
        ctx->slot_used[slot] = 0;
        ctx_free(ctx, buf, bytes);
        if (rc)
            return rc;
        if (e != hipSuccess)
            return fail_hip(e, "autotune");
        if (!all_equal)
            return fail(GCM_E_HIP, "autotune: launch shapes disagree on the tag (geometry dependence)");
        ctx->tuned[(uint64_t)key_len << 32 | size_bucket(len)] = {best_l, best_w};
        if (out) {
            out->log2_tile_blocks = best_l;
            out->waves_per_group = best_w;
            out->candidates = tried;
            out->best_ms = best_ms;
            out->gbs = (double)len / (best_ms * 1e-3) / 1e9;
        }
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_autotune_save(gcm_ctx *ctx, const char *path)
{
    GCM_ABI_TRY
        if (!ctx || !path)
            return fail(GCM_E_ARG, "gcm_autotune_save: NULL argument");
        std::lock_guard<std::mutex> g(ctx->mu);
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, ctx->device) != hipSuccess)
            std::strcpy(p.gcnArchName, "unknown");
        FILE *f = std::fopen(path, "w");
        if (!f)
            return fail(GCM_E_ARG, "gcm_autotune_save: cannot open %s", path);
        std::fprintf(f, "{\"arch\": \"%s\", \"entries\": [", p.gcnArchName);
        bool first = true;
        for (auto &kv : ctx->tuned) {
            std::fprintf(f, "%s{\"key_bytes\": %u, \"len_log2\": %u, \"log2_tile_blocks\": %u, \"waves\": %u}",
                         first ? "" : ", ", (uint32_t)(kv.first >> 32), (uint32_t)(kv.first & 0xffffffffu),
                         kv.second.first, kv.second.second);
            first = false;
        }
        std::fprintf(f, "]}\n");
        std::fclose(f);
        return GCM_OK;
    GCM_ABI_CATCH
}

// Minimal reader for the format gcm_autotune_save writes (entries with the
// four integer fields in that order); entries for another architecture are
// ignored as a whole.
extern "C" int gcm_autotune_load(gcm_ctx *ctx, const char *path)
{
    GCM_ABI_TRY
        if (!ctx || !path)
            return fail(GCM_E_ARG, "gcm_autotune_load: NULL argument");
        FILE *f = std::fopen(path, "r");
        if (!f)
            return fail(GCM_E_ARG, "gcm_autotune_load: cannot open %s", path);
        std::string text;
        char buf[4096];
        size_t n;
        while ((n = std::fread(buf, 1, sizeof buf, f)) > 0)
            text.append(buf, n);
        std::fclose(f);
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, ctx->device) != hipSuccess)
            return fail(GCM_E_HIP, "gcm_autotune_load: device query failed");
        if (text.find(std::string("\"arch\": \"") + p.gcnArchName + "\"") == std::string::npos)
            return fail(GCM_E_ARG, "gcm_autotune_load: cache is for another architecture");
        std::lock_guard<std::mutex> g(ctx->mu);
        size_t pos = 0;
        uint32_t loaded = 0;
        while ((pos = text.find("{\"key_bytes\":", pos)) != std::string::npos) {
            unsigned kb, ll, lt, wv;
            if (std::sscanf(text.c_str() + pos,
                            "{\"key_bytes\": %u, \"len_log2\": %u, \"log2_tile_blocks\": %u, \"waves\": %u}", &kb, &ll,
                            &lt, &wv) == 4 &&
                (kb == 16 || kb == 24 || kb == 32) && ll < 64 && lt >= 6 && lt <= 20 && (wv == 8 || wv == 12 || wv == 16)) {
                ctx->tuned[(uint64_t)kb << 32 | ll] = {lt, wv};
                ++loaded;
            }
            ++pos;
        }
        return loaded ? GCM_OK : fail(GCM_E_ARG, "gcm_autotune_load: no entries in %s", path);
    GCM_ABI_CATCH
}
