// gcm_autotune.cpp -- exhaustive launch-shape search (the paper tunes its
// kernel parameters per GPU the same way: an exhaustive sweep, keeping the
// fastest), with a bit-equality check across every candidate.
//
// Single messages: for one (key size, message size) point the search times
// every shape in {log2 tile blocks} x {waves per workgroup} x {groups per
// CU} x {reduction-tree fan-in} on a scratch message with HIP events,
// requires all of them to produce the same tag (the counter map and GHASH
// exponents derive from block indices only), and records the fastest in the
// context's cache, keyed by (key bytes, floor(log2 len)).
//
// Batches: the same search over {waves} x {groups per CU} x {cap on the
// messages' tile sizes} x {fan-in} on the caller's own batch, every point's
// tags and accept flags compared with the first point's, recorded under
// (floor(log2 messages), floor(log2 payload bytes)).
//
// Every planner (one-shot, asynchronous, batches, the serving loop, host
// pipeline, streamed segments) consults these caches when no explicit shape
// is set with gcm_set_launch.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gcm_mi355.h"
#include "gcm_host.h"

using namespace gcm;

namespace {

const uint32_t kWaveOpts[3] = {8, 12, 16};
const uint32_t kFaninOpts[4] = {2, 4, 8, 16};

// Candidate groups per CU for a workgroup size: 1 .. what the occupancy
// calculator allows (the tile kernel's 144 KiB of LDS holds it to one on
// gfx950, so this dimension has a single point there).
std::vector<uint32_t> gpc_options(uint32_t waves)
{
    std::vector<uint32_t> v;
    const uint32_t mx = (uint32_t)max_groups_per_cu((int)waves);
    for (uint32_t g = 1; g <= mx && g <= 4; ++g)
        v.push_back(g);
    return v;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t init()
    {
        hipError_t e = hipEventCreate(&a);
        return e == hipSuccess ? hipEventCreate(&b) : e;
    }
    ~Timer()
    {
        if (a)
            (void)hipEventDestroy(a);
        if (b)
            (void)hipEventDestroy(b);
    }
};

}  // namespace

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
        const uint64_t m = ghash_blocks(0, len);
        const uint64_t ws_bytes = workspace_bytes_for((m + 63) / 64, 1);
        const uint64_t pay = (len + 255) / 256 * 256;
        const uint64_t bytes = 2 * pay + ws_bytes + 256;
        uint8_t *buf = nullptr;
        int rc = ctx_alloc(ctx, reinterpret_cast<void **>(&buf), bytes);
        if (rc)
            return rc;
        uint8_t *in = buf, *outp = buf + pay, *ws = outp + pay;
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
        Timer tm;
        if (e == hipSuccess)
            e = tm.init();

        float best_ms = 1e30f;
        Shape best;
        uint32_t tried = 0;
        bool all_equal = true;
        uint8_t ref_tag[16], cur_tag[16];
        bool have_ref = false;
        const bool save_prof = ctx->prof;
        ctx->prof = false;
        for (uint32_t l = 8; l <= 16 && e == hipSuccess && rc == GCM_OK; ++l) {
            if ((1ull << l) > 4 * m && l > 8)
                break;  // tiles larger than the whole message add nothing
            for (uint32_t w : kWaveOpts)
                for (uint32_t gpc : gpc_options(w))
                    for (uint32_t f : kFaninOpts) {
                        if (e != hipSuccess || rc != GCM_OK)
                            break;
                        Shape sh;
                        sh.log2B = l;
                        sh.waves = w;
                        sh.gpc = gpc;
                        sh.fanin = f;
                        MsgDesc d;
                        fill_desc(&d, 0, iv, 0, 0, (uint64_t)in, (uint64_t)outp, len, (uint64_t)tag, 0,
                                  (uint64_t)(ctx->d_slots + kSlotBytes * slot), key_len / 4 + 6, l, w, 0);
                        rc = launch_single(ctx, d, sh, ws, s);  // warm-up
                        float total = 0.f;
                        for (uint32_t r = 0; r < reps && rc == GCM_OK && e == hipSuccess; ++r) {
                            e = hipEventRecord(tm.a, s);
                            if (e == hipSuccess)
                                rc = launch_single(ctx, d, sh, ws, s);
                            if (e == hipSuccess && rc == GCM_OK)
                                e = hipEventRecord(tm.b, s);
                            if (e == hipSuccess)
                                e = hipEventSynchronize(tm.b);
                            float ms = 0.f;
                            if (e == hipSuccess)
                                e = hipEventElapsedTime(&ms, tm.a, tm.b);
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
                            best = sh;
                        }
                    }
        }
        ctx->prof = save_prof;
        (void)hipStreamSynchronize(s);
        ctx->slot_used[slot] = 0;
        ctx_free(ctx, buf, bytes);
        if (rc)
            return rc;
        if (e != hipSuccess)
            return fail_hip(e, "autotune");
        if (!all_equal)
            return fail(GCM_E_INTERNAL, "autotune: launch shapes disagree on the tag (geometry dependence)");
        ctx->tuned[(uint64_t)key_len << 32 | size_bucket(len)] = best;
        if (out) {
            std::memset(out, 0, sizeof *out);
            out->log2_tile_blocks = best.log2B;
            out->waves_per_group = best.waves;
            out->candidates = tried;
            out->best_ms = best_ms;
            out->gbs = (double)len / (best_ms * 1e-3) / 1e9;
            out->groups_per_cu = best.gpc;
            out->combine_fanin = best.fanin;
        }
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_batch_autotune(gcm_ctx *ctx, const gcm_job *jobs, uint32_t n, uint8_t *base_d, uint64_t base_bytes,
                                  uint32_t reps, gcm_tune_result *out, void *stream)
{
    GCM_ABI_TRY
        if (!ctx || (n && (!jobs || !base_d)))
            return fail(GCM_E_ARG, "gcm_batch_autotune: NULL argument");
        if (n == 0)
            return fail(GCM_E_ARG, "gcm_batch_autotune: empty batch");
        if ((uintptr_t)base_d & 255)
            return fail(GCM_E_ARG, "gcm_batch_autotune: base_d must be 256-byte aligned");
        // every point reruns the batch, so it must leave its inputs intact
        for (uint32_t i = 0; i < n; ++i)
            if (jobs[i].len && jobs[i].in_off == jobs[i].out_off)
                return fail(GCM_E_ARG, "gcm_batch_autotune: job %u runs in place (a rerun would read its output)",
                            i);
        if (reps == 0)
            reps = 3;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        std::lock_guard<std::mutex> g(ctx->mu);
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess)
            return fail_hip(e, "hipSetDevice");
        uint64_t payload = 0;
        for (uint32_t i = 0; i < n; ++i)
            payload += jobs[i].len;

        // results of every point: tags (16 B) and, for decrypts, flags (4 B)
        std::vector<uint8_t> ref(20ull * n), cur(20ull * n);
        auto fetch = [&](std::vector<uint8_t> &dst) -> hipError_t {
            hipError_t r = hipStreamSynchronize(s);
            for (uint32_t i = 0; i < n && r == hipSuccess; ++i) {
                r = hipMemcpy(dst.data() + 20ull * i, base_d + jobs[i].tag_off, 16, hipMemcpyDeviceToHost);
                if (r == hipSuccess && jobs[i].op == 1)
                    r = hipMemcpy(dst.data() + 20ull * i + 16, base_d + jobs[i].ok_off, 4, hipMemcpyDeviceToHost);
            }
            return r;
        };
        Timer tm;
        e = tm.init();
        if (e != hipSuccess)
            return fail_hip(e, "hipEventCreate");
        float best_ms = 1e30f;
        Shape best;
        uint32_t tried = 0;
        bool have_ref = false, all_equal = true;
        int rc = GCM_OK;
        const bool save_prof = ctx->prof;
        ctx->prof = false;
        for (uint32_t w : kWaveOpts)
            for (uint32_t gpc : gpc_options(w))
                for (uint32_t cap = 8; cap <= 12; ++cap)
                    for (uint32_t f : kFaninOpts) {
                        if (rc || e != hipSuccess)
                            break;
                        Shape sh;
                        sh.log2B = cap;
                        sh.waves = w;
                        sh.gpc = gpc;
                        sh.fanin = f;
                        gcm_batch *b = nullptr;
                        rc = batch_create_locked(ctx, jobs, n, base_d, base_bytes, &sh, &b);
                        if (rc)
                            break;
                        e = batch_enqueue(b, s);  // warm-up
                        float total = 0.f;
                        for (uint32_t r = 0; r < reps && e == hipSuccess; ++r) {
                            e = hipEventRecord(tm.a, s);
                            if (e == hipSuccess)
                                e = batch_enqueue(b, s);
                            if (e == hipSuccess)
                                e = hipEventRecord(tm.b, s);
                            if (e == hipSuccess)
                                e = hipEventSynchronize(tm.b);
                            float ms = 0.f;
                            if (e == hipSuccess)
                                e = hipEventElapsedTime(&ms, tm.a, tm.b);
                            total += ms;
                        }
                        if (e == hipSuccess)
                            e = fetch(have_ref ? cur : ref);
                        batch_free_locked(b);
                        if (e != hipSuccess)
                            break;
                        if (!have_ref)
                            have_ref = true;
                        else if (cur != ref)
                            all_equal = false;
                        ++tried;
                        const float ms = total / (float)reps;
                        if (ms < best_ms) {
                            best_ms = ms;
                            best = sh;
                        }
                    }
        ctx->prof = save_prof;
        if (rc)
            return rc;
        if (e != hipSuccess)
            return fail_hip(e, "batch autotune");
        if (!all_equal)
            return fail(GCM_E_INTERNAL, "batch autotune: launch shapes disagree on a tag or flag (geometry dependence)");
        ctx->tuned_batch[(uint64_t)size_bucket(n) << 32 | size_bucket(payload)] = best;
        if (out) {
            std::memset(out, 0, sizeof *out);
            out->log2_tile_blocks = best.log2B;
            out->waves_per_group = best.waves;
            out->candidates = tried;
            out->best_ms = best_ms;
            out->gbs = (double)payload / (best_ms * 1e-3) / 1e9;
            out->groups_per_cu = best.gpc;
            out->combine_fanin = best.fanin;
        }
        return GCM_OK;
    GCM_ABI_CATCH
}

// Cache file: {"arch": ..., "entries": [...], "batch_entries": [...]}, each
// entry four size/shape integers and the groups per CU and fan-in.
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
            std::fprintf(f,
                         "%s{\"key_bytes\": %u, \"len_log2\": %u, \"log2_tile_blocks\": %u, \"waves\": %u, "
                         "\"groups_per_cu\": %u, \"fanin\": %u}",
                         first ? "" : ", ", (uint32_t)(kv.first >> 32), (uint32_t)(kv.first & 0xffffffffu),
                         kv.second.log2B, kv.second.waves, kv.second.gpc, kv.second.fanin);
            first = false;
        }
        std::fprintf(f, "], \"batch_entries\": [");
        first = true;
        for (auto &kv : ctx->tuned_batch) {
            std::fprintf(f,
                         "%s{\"msgs_log2\": %u, \"payload_log2\": %u, \"tile_cap_log2\": %u, \"waves\": %u, "
                         "\"groups_per_cu\": %u, \"fanin\": %u}",
                         first ? "" : ", ", (uint32_t)(kv.first >> 32), (uint32_t)(kv.first & 0xffffffffu),
                         kv.second.log2B, kv.second.waves, kv.second.gpc, kv.second.fanin);
            first = false;
        }
        std::fprintf(f, "]}\n");
        std::fclose(f);
        return GCM_OK;
    GCM_ABI_CATCH
}

static bool valid_entry(unsigned lt, unsigned wv, unsigned gp, unsigned fi)
{
    return lt >= 6 && lt <= 20 && (wv == 8 || wv == 12 || wv == 16) && gp >= 1 && gp <= 64 && valid_fanin(fi);
}

// Minimal reader for the format gcm_autotune_save writes; a cache for another
// architecture is rejected as a whole.
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
            unsigned kb, ll, lt, wv, gp, fi;
            if (std::sscanf(text.c_str() + pos,
                            "{\"key_bytes\": %u, \"len_log2\": %u, \"log2_tile_blocks\": %u, \"waves\": %u, "
                            "\"groups_per_cu\": %u, \"fanin\": %u}",
                            &kb, &ll, &lt, &wv, &gp, &fi) == 6 &&
                (kb == 16 || kb == 24 || kb == 32) && ll < 64 && valid_entry(lt, wv, gp, fi)) {
                ctx->tuned[(uint64_t)kb << 32 | ll] = Shape{lt, wv, gp, fi};
                ++loaded;
            }
            ++pos;
        }
        pos = 0;
        while ((pos = text.find("{\"msgs_log2\":", pos)) != std::string::npos) {
            unsigned nl, pl, lt, wv, gp, fi;
            if (std::sscanf(text.c_str() + pos,
                            "{\"msgs_log2\": %u, \"payload_log2\": %u, \"tile_cap_log2\": %u, \"waves\": %u, "
                            "\"groups_per_cu\": %u, \"fanin\": %u}",
                            &nl, &pl, &lt, &wv, &gp, &fi) == 6 &&
                nl < 64 && pl < 64 && valid_entry(lt, wv, gp, fi)) {
                ctx->tuned_batch[(uint64_t)nl << 32 | pl] = Shape{lt, wv, gp, fi};
                ++loaded;
            }
            ++pos;
        }
        return loaded ? GCM_OK : fail(GCM_E_ARG, "gcm_autotune_load: no entries in %s", path);
    GCM_ABI_CATCH
}
