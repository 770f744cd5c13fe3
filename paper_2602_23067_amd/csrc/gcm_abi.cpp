// gcm_abi.cpp -- host runtime behind the C ABI in include/gcm_mi355.h:
// device context, resident key table (with a small cache for the one-shot
// calls), launch planning and the single-message entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <list>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/gcm_mi355.h"
#include "gcm_host.h"

using namespace gcm;

static_assert(kNoAllocScratchBytes == GCM_NOALLOC_SCRATCH_BYTES, "scratch size and its public constant differ");

// ---------------------------------------------------------------- errors

// a fixed buffer: recording an error never allocates (and so never throws)
static thread_local char g_last_error[512];

int gcm::fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return code;
}

int gcm::fail_hip(hipError_t e, const char *what)
{
    return fail(GCM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int gcm::abi_exception() noexcept
{
    try {
        throw;
    } catch (const std::bad_alloc &) {
        return fail(GCM_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(GCM_E_INTERNAL, "host runtime failure: %s", e.what());
    } catch (...) {
        return fail(GCM_E_INTERNAL, "host runtime failure");
    }
}

int gcm::plan_error(const PlanError &e) { return fail(e.code, "%s", e.msg); }

extern "C" const char *gcm_last_error(void) { return g_last_error; }

// placeholder IV for fill_desc when set_iv fills the descriptor's IV afterwards
static const uint8_t kZeroIv[12] = {0};

// ---------------------------------------------------------------- context

int gcm::ctx_alloc(gcm_ctx *ctx, void **p, uint64_t bytes)
{
    if (ctx->budget && ctx->used + bytes > ctx->budget && !ctx->stream_pool.empty())
        stream_pool_release(ctx);
    if (ctx->budget && ctx->used + bytes > ctx->budget)
        return fail(GCM_E_NOMEM, "allocation of %llu bytes exceeds the context budget (%llu of %llu used)",
                    (unsigned long long)bytes, (unsigned long long)ctx->used, (unsigned long long)ctx->budget);
    hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(GCM_E_NOMEM, "hipMalloc(%llu): %s", (unsigned long long)bytes, hipGetErrorString(e));
    }
    ctx->used += bytes;
    return GCM_OK;
}

void gcm::ctx_free(gcm_ctx *ctx, void *p, uint64_t bytes)
{
    if (p) {
        (void)hipFree(p);
        ctx->used -= bytes;
    }
}

extern "C" int gcm_ctx_create(gcm_ctx **out, int device, uint64_t hbm_budget_bytes, uint32_t key_slots)
{
    GCM_ABI_TRY
        if (!out)
            return fail(GCM_E_ARG, "gcm_ctx_create: out is NULL");
        *out = nullptr;
        if (key_slots == 0 || key_slots > (1u << 20))
            return fail(GCM_E_ARG, "gcm_ctx_create: key_slots must be in 1..2^20");
        int ndev = 0;
        hipError_t e = hipGetDeviceCount(&ndev);
        if (e != hipSuccess)
            return fail_hip(e, "hipGetDeviceCount");
        if (device < 0 || device >= ndev)
            return fail(GCM_E_ARG, "gcm_ctx_create: device %d out of range (%d devices)", device, ndev);
        e = hipSetDevice(device);
        if (e != hipSuccess)
            return fail_hip(e, "hipSetDevice");

        gcm_ctx *ctx = new (std::nothrow) gcm_ctx();
        if (!ctx)
            return fail(GCM_E_NOMEM, "gcm_ctx_create: host allocation failed");
        ctx->device = device;
        ctx->budget = hbm_budget_bytes;
        ctx->n_slots = key_slots;
        int cus = 0;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
        ctx->cu_count = cus > 0 ? cus : 1;

        int rc = ctx_alloc(ctx, reinterpret_cast<void **>(&ctx->d_tables), kAesTableWords * sizeof(uint32_t));
        if (rc == GCM_OK)
            rc = ctx_alloc(ctx, &ctx->d_frob, frob_table_bytes());
        if (rc == GCM_OK)
            rc = ctx_alloc(ctx, reinterpret_cast<void **>(&ctx->d_slots), kSlotBytes * key_slots);
        if (rc == GCM_OK)
            rc = ctx_alloc(ctx, reinterpret_cast<void **>(&ctx->d_io), 256);
        if (rc == GCM_OK) {
            e = hipHostMalloc(reinterpret_cast<void **>(&ctx->h_io), 256, hipHostMallocDefault);
            if (e != hipSuccess)
                rc = fail(GCM_E_NOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
        }
        if (rc == GCM_OK) {
            // optional: without a mapped result block the one-shot calls copy
            if (hipHostMalloc(reinterpret_cast<void **>(&ctx->h_map), 256,
                              hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess) {
                if (hipHostGetDevicePointer(reinterpret_cast<void **>(&ctx->d_map), ctx->h_map, 0) != hipSuccess) {
                    (void)hipHostFree(ctx->h_map);
                    ctx->h_map = nullptr;
                    ctx->d_map = nullptr;
                }
            } else {
                ctx->h_map = nullptr;
            }
            (void)hipGetLastError();
        }
        if (rc == GCM_OK) {
            e = scratch_address(device, &ctx->d_scratch);
            if (e != hipSuccess)
                rc = fail_hip(e, "hipGetSymbolAddress(scratch)");
        }
        if (rc == GCM_OK) {
            e = launch_init_tables(ctx->d_tables, ctx->d_tables + 256, ctx->d_frob, nullptr);
            if (e == hipSuccess)
                e = hipDeviceSynchronize();
            if (e != hipSuccess)
                rc = fail_hip(e, "AES table initialisation");
        }
        if (rc != GCM_OK) {
            gcm_ctx_destroy(ctx);
            return rc;
        }
        ctx->slot_used.assign(key_slots, 0);
        ctx->slot_nr.assign(key_slots, 0);
        ctx->cache_cap = std::max<uint32_t>(1, std::min<uint32_t>(16, key_slots / 2 ? key_slots / 2 : 1));
        *out = ctx;
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_ctx_destroy(gcm_ctx *ctx)
{
    GCM_ABI_TRY
        if (!ctx)
            return fail(GCM_E_ARG, "gcm_ctx_destroy: NULL context");
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        ctx_free(ctx, ctx->d_tables, kAesTableWords * sizeof(uint32_t));
        ctx_free(ctx, ctx->d_frob, frob_table_bytes());
        ctx_free(ctx, ctx->d_slots, kSlotBytes * ctx->n_slots);
        ctx_free(ctx, ctx->d_io, 256);
        ctx_free(ctx, ctx->d_ws, ctx->ws_bytes);
        stream_pool_release(ctx);
        pipeline_release(ctx);
        for (auto &pr : ctx->prof_pending) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        for (auto &pr : ctx->prof_free) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        if (ctx->h_io)
            (void)hipHostFree(ctx->h_io);
        if (ctx->h_map)
            (void)hipHostFree(ctx->h_map);
        delete ctx;
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_set_launch(gcm_ctx *ctx, uint32_t log2_tile_blocks, uint32_t waves_per_group,
                              uint32_t groups_per_cu)
{
    GCM_ABI_TRY
        if (!ctx)
            return fail(GCM_E_ARG, "gcm_set_launch: NULL context");
        if (log2_tile_blocks && (log2_tile_blocks < 6 || log2_tile_blocks > 20))
            return fail(GCM_E_ARG, "gcm_set_launch: log2_tile_blocks must be 0 or 6..20");
        if (waves_per_group && waves_per_group != 8 && waves_per_group != 12 && waves_per_group != 16)
            return fail(GCM_E_ARG, "gcm_set_launch: waves_per_group must be 0, 8, 12 or 16");
        if (groups_per_cu > 64)
            return fail(GCM_E_ARG, "gcm_set_launch: groups_per_cu must be <= 64");
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->cfg_log2B = log2_tile_blocks;
        ctx->cfg_waves = waves_per_group;
        ctx->cfg_gpc = groups_per_cu;
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_set_combine(gcm_ctx *ctx, uint32_t fanin)
{
    GCM_ABI_TRY
        if (!ctx)
            return fail(GCM_E_ARG, "gcm_set_combine: NULL context");
        if (fanin && !valid_fanin(fanin))
            return fail(GCM_E_ARG, "gcm_set_combine: fan-in must be 0, 2, 4, 8 or 16");
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->cfg_fanin = fanin;
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_launch_plan(gcm_ctx *ctx, uint32_t key_len, uint64_t len, uint64_t aad_len, gcm_tune_result *out)
{
    GCM_ABI_TRY
        if (!ctx || !out)
            return fail(GCM_E_ARG, "gcm_launch_plan: NULL argument");
        if (key_len != 16 && key_len != 24 && key_len != 32)
            return fail(GCM_E_KEYLEN, "key length %u is not 16, 24 or 32", key_len);
        std::lock_guard<std::mutex> g(ctx->mu);
        const Shape sh = message_shape(ctx, key_len, len, aad_len);
        const uint64_t m = ghash_blocks(aad_len, len);
        std::memset(out, 0, sizeof *out);
        out->log2_tile_blocks = sh.log2B;
        out->waves_per_group = sh.waves;
        out->groups_per_cu = sh.gpc;
        out->combine_fanin = sh.fanin;
        out->candidates = (uint32_t)((m + (1ull << sh.log2B) - 1) >> sh.log2B);
        return GCM_OK;
    GCM_ABI_CATCH
}

// ---------------------------------------------------------------- keys

int gcm::register_keys_locked(gcm_ctx *ctx, const uint8_t *const *keys, const uint32_t *key_lens, uint32_t n,
                              uint32_t *slots_out, hipStream_t s)
{
    std::vector<uint32_t> picked;
    picked.reserve(n);
    for (uint32_t i = 0; i < ctx->n_slots && picked.size() < n; ++i)
        if (!ctx->slot_used[i])
            picked.push_back(i);
    if (picked.size() < n)
        return fail(GCM_E_BUSY, "%u key slots requested, %zu free (%u slots)", n, picked.size(), ctx->n_slots);
    std::vector<uint64_t> addrs(n);
    for (uint32_t i = 0; i < n; ++i)
        addrs[i] = (uint64_t)(ctx->d_slots + kSlotBytes * picked[i]);
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = launch_key_setup(keys, key_lens, addrs.data(), n, ctx->d_tables, ctx->d_tables + 256, ctx->d_frob, s);
    if (e != hipSuccess)
        return fail_hip(e, "key setup launch");
    for (uint32_t i = 0; i < n; ++i) {
        ctx->slot_used[picked[i]] = 1;
        ctx->slot_nr[picked[i]] = key_lens[i] / 4 + 6;
        slots_out[i] = picked[i];
    }
    return GCM_OK;
}

int gcm::register_key_locked(gcm_ctx *ctx, const uint8_t *key, size_t key_len, uint32_t *slot_out, hipStream_t s)
{
    const uint32_t len = (uint32_t)key_len;
    return register_keys_locked(ctx, &key, &len, 1, slot_out, s);
}

static bool valid_key_len(size_t n) { return n == 16 || n == 24 || n == 32; }

extern "C" int gcm_key_register(gcm_ctx *ctx, const uint8_t *key, size_t key_len, uint32_t *slot_out, void *stream)
{
    GCM_ABI_TRY
        if (!ctx || !key || !slot_out)
            return fail(GCM_E_ARG, "gcm_key_register: NULL argument");
        if (!valid_key_len(key_len))
            return fail(GCM_E_KEYLEN, "key length %zu is not 16, 24 or 32", key_len);
        std::lock_guard<std::mutex> g(ctx->mu);
        return register_key_locked(ctx, key, key_len, slot_out, reinterpret_cast<hipStream_t>(stream));
    GCM_ABI_CATCH
}

extern "C" int gcm_key_register_many(gcm_ctx *ctx, const uint8_t *keys, const uint32_t *key_lens, uint32_t n,
                                     uint32_t *slots_out, void *stream)
{
    GCM_ABI_TRY
        if (!ctx || (n && (!keys || !key_lens || !slots_out)))
            return fail(GCM_E_ARG, "gcm_key_register_many: NULL argument");
        std::vector<const uint8_t *> ptrs(n);
        uint64_t off = 0;
        for (uint32_t i = 0; i < n; ++i) {
            if (!valid_key_len(key_lens[i]))
                return fail(GCM_E_KEYLEN, "key %u: length %u is not 16, 24 or 32", i, key_lens[i]);
            ptrs[i] = keys + off;
            off += key_lens[i];
        }
        std::lock_guard<std::mutex> g(ctx->mu);
        return register_keys_locked(ctx, ptrs.data(), key_lens, n, slots_out, reinterpret_cast<hipStream_t>(stream));
    GCM_ABI_CATCH
}

extern "C" int gcm_key_release(gcm_ctx *ctx, uint32_t slot)
{
    GCM_ABI_TRY
        if (!ctx)
            return fail(GCM_E_ARG, "gcm_key_release: NULL context");
        std::lock_guard<std::mutex> g(ctx->mu);
        if (slot >= ctx->n_slots || !ctx->slot_used[slot])
            return fail(GCM_E_SLOT, "key slot %u is not registered", slot);
        for (auto &kv : ctx->cache)
            if (kv.second == slot)
                return fail(GCM_E_ARG, "key slot %u belongs to the one-shot key cache", slot);
        ctx->slot_used[slot] = 0;
        return GCM_OK;
    GCM_ABI_CATCH
}

// one-shot path: look the key up in the cache, expand it on a miss (LRU eviction
// among cache-owned slots only; the one-shot calls synchronise before
// returning, so an evicted slot has no work in flight)
int gcm::cached_slot_locked(gcm_ctx *ctx, const uint8_t *key, size_t key_len, uint32_t *slot, hipStream_t s)
{
    std::string k(reinterpret_cast<const char *>(key), key_len);
    auto it = ctx->cache.find(k);
    if (it != ctx->cache.end()) {
        ctx->lru.remove(k);
        ctx->lru.push_front(k);
        *slot = it->second;
        return GCM_OK;
    }
    if (ctx->cache.size() >= ctx->cache_cap && !ctx->lru.empty()) {
        const std::string victim = ctx->lru.back();
        ctx->lru.pop_back();
        ctx->slot_used[ctx->cache[victim]] = 0;
        ctx->cache.erase(victim);
    }
    int rc = register_key_locked(ctx, key, key_len, slot, s);
    if (rc)
        return rc;
    ctx->cache[k] = *slot;
    ctx->lru.push_front(k);
    return GCM_OK;
}

// ---------------------------------------------------------------- planning

SlotView gcm::slot_view(const gcm_ctx *ctx)
{
    SlotView v;
    v.base = (uint64_t)ctx->d_slots;
    v.n_slots = ctx->n_slots;
    v.used = ctx->slot_used.data();
    v.nr = ctx->slot_nr.data();
    return v;
}

// groups of the tile kernel a compute unit holds (occupancy query, once per
// process: every device is the same part)
uint32_t gcm::groups_per_cu(uint32_t waves)
{
    static const uint32_t g8 = (uint32_t)max_groups_per_cu(8), g12 = (uint32_t)max_groups_per_cu(12),
                          g16 = (uint32_t)max_groups_per_cu(16);
    return waves == 8 ? g8 : waves == 12 ? g12 : waves == 16 ? g16 : (uint32_t)max_groups_per_cu((int)waves);
}

uint64_t gcm::resident_bound(const gcm_ctx *ctx)
{
    uint64_t r = 0;
    for (uint32_t w : {8u, 12u, 16u})
        r = std::max<uint64_t>(r, (uint64_t)ctx->cu_count * (ctx->cfg_gpc ? ctx->cfg_gpc : groups_per_cu(w)) * w);
    return r;
}

Shape gcm::message_shape(const gcm_ctx *ctx, uint32_t key_bytes, uint64_t len, uint64_t aad_len)
{
    Shape sh;
    TuneEntry t;
    bool tuned = false;
    if (!ctx->cfg_log2B && !ctx->cfg_waves) {
        auto it = ctx->tuned.find((uint64_t)key_bytes << 32 | size_bucket(len));
        if (it != ctx->tuned.end()) {
            t = it->second;
            tuned = true;
        }
    }
    const uint64_t m = ghash_blocks(aad_len, len);
    if (ctx->cfg_waves)
        sh.waves = ctx->cfg_waves;
    else if (tuned)
        sh.waves = t.waves;
    else if (ctx->cfg_log2B || ctx->cfg_gpc)
        sh.waves = 16;
    else
        sh.waves = heuristic_waves(m, (uint64_t)ctx->cu_count, groups_per_cu);
    sh.gpc = ctx->cfg_gpc ? ctx->cfg_gpc : (tuned && t.gpc) ? t.gpc : groups_per_cu(sh.waves);
    sh.log2B = ctx->cfg_log2B ? ctx->cfg_log2B
               : tuned        ? t.log2B
                              : heuristic_log2B(m, (uint64_t)ctx->cu_count * sh.gpc * sh.waves);
    sh.fanin = ctx->cfg_fanin ? ctx->cfg_fanin : (tuned && t.fanin) ? t.fanin : 2;
    return sh;
}

Shape gcm::batch_shape(const gcm_ctx *ctx, uint64_t n, uint64_t payload, uint64_t m)
{
    Shape sh;
    TuneEntry t;
    bool tuned = false;
    if (!ctx->cfg_log2B && !ctx->cfg_waves) {
        auto it = ctx->tuned_batch.find((uint64_t)size_bucket(n) << 32 | size_bucket(payload));
        if (it != ctx->tuned_batch.end()) {
            t = it->second;
            tuned = true;
        }
    }
    sh.waves = ctx->cfg_waves ? ctx->cfg_waves : tuned ? t.waves : 16;
    sh.gpc = ctx->cfg_gpc ? ctx->cfg_gpc : (tuned && t.gpc) ? t.gpc : (uint32_t)max_groups_per_cu((int)sh.waves);
    if (ctx->cfg_log2B)
        sh.log2B = ctx->cfg_log2B;
    else if (tuned)
        sh.log2B = t.log2B;
    else  // the single-launch tile size of the whole batch's blocks, within 2^8..2^12
        sh.log2B = std::min<uint32_t>(
            12, std::max<uint32_t>(8, heuristic_log2B(std::max<uint64_t>(1, m),
                                                      (uint64_t)ctx->cu_count * sh.gpc * sh.waves)));
    sh.fanin = ctx->cfg_fanin ? ctx->cfg_fanin : (tuned && t.fanin) ? t.fanin : 2;
    return sh;
}

bool gcm::valid_iv_len(size_t n) { return n >= 1 && n <= (size_t)kMaxIvBytes; }

int gcm::set_iv(MsgDesc *d, const uint8_t *iv, size_t iv_len, void *ws, hipStream_t s)
{
    if (iv_len == 12) {
        for (int i = 0; i < 3; ++i)
            d->iv[i] = (uint32_t)iv[4 * i] | ((uint32_t)iv[4 * i + 1] << 8) | ((uint32_t)iv[4 * i + 2] << 16) |
                       ((uint32_t)iv[4 * i + 3] << 24);
        d->j0 = 0;
        return GCM_OK;
    }
    if (!valid_iv_len(iv_len))
        return fail(GCM_E_IVLEN, "IV length %zu is not in 1..%d", iv_len, kMaxIvBytes);
    IvArg a;
    std::memset(&a, 0, sizeof a);
    a.len = (uint32_t)iv_len;
    std::memcpy(a.b, iv, iv_len);
    // per message: its T tile partials, E_K(J0), then J0
    uint8_t *j0 = reinterpret_cast<uint8_t *>(ws) + workspace_counter_bytes(1) + 16 * (d->tile_base + d->n_tiles + 1);
    hipError_t e = launch_j0(a, d->slot, j0, nullptr, s);
    if (e != hipSuccess)
        return fail_hip(e, "J0 kernel launch");
    d->iv[0] = d->iv[1] = d->iv[2] = 0;
    d->j0 = (uint64_t)j0;
    return GCM_OK;
}

int gcm::check_message(uint64_t aad_len, uint64_t len, const void *aad_d, const void *in_d, const void *out_d,
                       const void *tag_d, uint64_t tag_len, const void *ok_d)
{
    PlanError err;
    if (check_lengths(aad_len, len, &err) ||
        check_buffers((uint64_t)aad_d, aad_len, (uint64_t)in_d, (uint64_t)out_d, len, (uint64_t)tag_d, tag_len,
                      (uint64_t)ok_d, &err))
        return plan_error(err);
    return GCM_OK;
}

// Enqueue the tile kernel for tiles [d.tile_lo, d.tile_hi) of one message on `s`.
int gcm::launch_tile_range(gcm_ctx *ctx, const MsgDesc &d, const Shape &sh, void *ws, hipStream_t s)
{
    const uint32_t waves = sh.waves, gpc = sh.gpc;
    uint32_t *counters = ws ? reinterpret_cast<uint32_t *>(ws) : nullptr;
    uint8_t *partials = ws ? reinterpret_cast<uint8_t *>(ws) + workspace_counter_bytes(1) : nullptr;
    const uint64_t tiles = d.tile_hi - d.tile_lo;
    const uint32_t items = (uint32_t)((tiles + waves - 1) / waves);
    if (items == 0)
        return GCM_OK;
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(items, (uint32_t)ctx->cu_count * gpc));
    hipError_t e = prof_begin(ctx, s);
    if (e == hipSuccess)
        e = launch_tiles((int)waves, nullptr, nullptr, items, &d, ctx->d_tables, partials, counters, grid, s);
    if (e == hipSuccess)
        e = prof_end(ctx, s);
    if (e != hipSuccess)
        return fail_hip(e, "tile kernel launch");
    return GCM_OK;
}

// Enqueue the kernels for one message on `s`: tiles, then (GCM only) the
// combine and, for decrypt-verify, the zero-fill of a rejected output.
int gcm::launch_single(gcm_ctx *ctx, const MsgDesc &d, const Shape &sh, void *ws, hipStream_t s)
{
    int rc = launch_tile_range(ctx, d, sh, ws, s);
    if (rc || d.op == 2)
        return rc;
    uint32_t *counters = reinterpret_cast<uint32_t *>(ws);
    uint8_t *partials = reinterpret_cast<uint8_t *>(ws) + workspace_counter_bytes(1);
    hipError_t e = launch_combine(nullptr, 1, &d, partials, counters, sh.fanin, s);
    if (e == hipSuccess && d.op == 1) {
        const uint64_t chunks = (d.len / 16 + 255) / 256;
        const uint32_t zgrid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(chunks, 4096));
        e = launch_zerofill(nullptr, &d, counters, zgrid, s);
    }
    if (e != hipSuccess)
        return fail_hip(e, "kernel launch");
    return GCM_OK;
}

static uint32_t slot_nr(size_t key_len) { return (uint32_t)(key_len / 4 + 6); }

extern "C" uint64_t gcm_workspace_size(gcm_ctx *ctx, uint64_t len, uint64_t aad_len)
{
    GCM_ABI_TRY
        if (!ctx)
            return 0;
        std::lock_guard<std::mutex> g(ctx->mu);
        const uint64_t m = ghash_blocks(aad_len, len);
        uint32_t best = 64;
        for (uint32_t kb : {16u, 24u, 32u})  // any key size the call may use: the smallest tiles
            best = std::min(best, message_shape(ctx, kb, len, aad_len).log2B);
        const uint64_t T = (m + (1ull << best) - 1) >> best;
        // with explicit launch settings the tile size is fixed, so the count
        // grows with the length; otherwise cover every shorter message too
        if (ctx->cfg_log2B)
            return workspace_bytes_for(T, 1);
        return workspace_bytes_for(tiles_bound_upto(m, T, resident_bound(ctx)), 1);
    GCM_ABI_CATCH_VALUE(0)
}

int gcm::ensure_ws_locked(gcm_ctx *ctx, uint64_t bytes)
{
    if (ctx->ws_bytes >= bytes)
        return GCM_OK;
    ctx_free(ctx, ctx->d_ws, ctx->ws_bytes);
    ctx->d_ws = nullptr;
    ctx->ws_bytes = 0;
    const uint64_t want = std::max<uint64_t>(bytes, 1ull << 20);
    int rc = ctx_alloc(ctx, reinterpret_cast<void **>(&ctx->d_ws), want);
    if (rc)
        return rc;
    ctx->ws_bytes = want;
    return GCM_OK;
}

// ---------------------------------------------------------------- async entry points

int gcm::async_launch(gcm_ctx *ctx, uint32_t op, uint32_t slot, const uint8_t *iv, size_t iv_len,
                      const uint8_t *aad_d, uint64_t aad_len, const uint8_t *in_d, uint64_t len, uint8_t *out_d,
                      const uint8_t *tag_d, int32_t *ok_d, void *ws, uint64_t ws_bytes, bool fit_ws, void *stream)
{
    if (!ctx || !iv || !tag_d || (op == 1 && !ok_d) || !ws)
        return fail(GCM_E_ARG, "NULL argument");
    if (!valid_iv_len(iv_len))
        return fail(GCM_E_IVLEN, "IV length %zu is not in 1..%d", iv_len, kMaxIvBytes);
    int rc = check_message(aad_len, len, aad_d, in_d, out_d, tag_d, 16, ok_d);
    if (rc)
        return rc;
    if ((uintptr_t)ws & 15)
        return fail(GCM_E_ARG, "workspace must be 16-byte aligned");
    std::lock_guard<std::mutex> g(ctx->mu);
    if (slot >= ctx->n_slots || !ctx->slot_used[slot])
        return fail(GCM_E_SLOT, "key slot %u is not registered", slot);
    Shape sh = message_shape(ctx, (ctx->slot_nr[slot] - 6) * 4, len, aad_len);
    const uint64_t m = ghash_blocks(aad_len, len);
    if (fit_ws)  // larger tiles (fewer partials) until the workspace holds them; results do not change
        while (sh.log2B < kFitMaxLog2B && workspace_bytes_for((m + (1ull << sh.log2B) - 1) >> sh.log2B, 1) > ws_bytes)
            ++sh.log2B;
    MsgDesc d;
    fill_desc(&d, op, kZeroIv, (uint64_t)aad_d, aad_len, (uint64_t)in_d, (uint64_t)out_d, len, (uint64_t)tag_d,
              (uint64_t)ok_d, (uint64_t)(ctx->d_slots + kSlotBytes * slot), ctx->slot_nr[slot], sh.log2B, sh.waves, 0);
    if (ws_bytes < workspace_bytes_for(d.n_tiles, 1)) {
        if (fit_ws)
            return fail(GCM_E_NOMEM,
                        "message of %llu data and %llu AAD bytes needs %llu bytes of scratch even with tiles of "
                        "2^%u blocks; the allocation-free path has a fixed %llu",
                        (unsigned long long)len, (unsigned long long)aad_len,
                        (unsigned long long)workspace_bytes_for(d.n_tiles, 1), sh.log2B, (unsigned long long)ws_bytes);
        return fail(GCM_E_ARG, "workspace of %llu bytes is smaller than the %llu needed", (unsigned long long)ws_bytes,
                    (unsigned long long)workspace_bytes_for(d.n_tiles, 1));
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess)
        return fail_hip(e, "hipSetDevice");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    rc = set_iv(&d, iv, iv_len, ws, s);
    if (rc)
        return rc;
    // a fitted workspace is the no-allocation path: no profiling events there
    const bool prof = ctx->prof;
    if (fit_ws)
        ctx->prof = false;
    rc = launch_single(ctx, d, sh, ws, s);
    ctx->prof = prof;
    return rc;
}

extern "C" int gcm_encrypt_async(gcm_ctx *ctx, uint32_t slot, const uint8_t *iv, size_t iv_len, const uint8_t *aad_d,
                                 uint64_t aad_len, const uint8_t *pt_d, uint64_t len, uint8_t *ct_d, uint8_t *tag_d,
                                 void *workspace_d, uint64_t workspace_bytes, void *stream)
{
    GCM_ABI_TRY
        return async_launch(ctx, 0, slot, iv, iv_len, aad_d, aad_len, pt_d, len, ct_d, tag_d, nullptr, workspace_d,
                            workspace_bytes, false, stream);
    GCM_ABI_CATCH
}

extern "C" int gcm_decrypt_verify_async(gcm_ctx *ctx, uint32_t slot, const uint8_t *iv, size_t iv_len,
                                        const uint8_t *aad_d, uint64_t aad_len, const uint8_t *ct_d, uint64_t len,
                                        const uint8_t *tag_d, uint8_t *pt_d, int32_t *accept_d, void *workspace_d,
                                        uint64_t workspace_bytes, void *stream)
{
    GCM_ABI_TRY
        return async_launch(ctx, 1, slot, iv, iv_len, aad_d, aad_len, ct_d, len, pt_d, tag_d, accept_d, workspace_d,
                            workspace_bytes, false, stream);
    GCM_ABI_CATCH
}

extern "C" int gcm_encrypt_async_noalloc(gcm_ctx *ctx, uint32_t slot, const uint8_t *iv, size_t iv_len,
                                         const uint8_t *aad_d, uint64_t aad_len, const uint8_t *pt_d, uint64_t len,
                                         uint8_t *ct_d, uint8_t *tag_d, void *stream)
{
    GCM_ABI_TRY
        if (!ctx)
            return fail(GCM_E_ARG, "NULL context");
        if (!ctx->d_scratch)
            return fail(GCM_E_INTERNAL, "the device scratch address was not looked up");
        return async_launch(ctx, 0, slot, iv, iv_len, aad_d, aad_len, pt_d, len, ct_d, tag_d, nullptr,
                            ctx->d_scratch, kNoAllocScratchBytes, true, stream);
    GCM_ABI_CATCH
}

// ---------------------------------------------------------------- one-shot entry points

static bool valid_tag_len(size_t t) { return t == 16 || t == 15 || t == 14 || t == 13 || t == 12 || t == 8 || t == 4; }

static int oneshot(gcm_ctx *ctx, uint32_t op, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                   const uint8_t *aad_d, uint64_t aad_len, const uint8_t *in_d, uint64_t len, uint8_t *out_d,
                   const uint8_t *tag_in, uint8_t *tag_out, int *accept, void *stream, size_t tag_len = 16)
{
    if (!ctx || !key || !iv || (op == 0 && !tag_out) || (op == 1 && (!tag_in || !accept)))
        return fail(GCM_E_ARG, "NULL argument");
    if (!valid_key_len(key_len))
        return fail(GCM_E_KEYLEN, "key length %zu is not 16, 24 or 32", key_len);
    if (!valid_iv_len(iv_len))
        return fail(GCM_E_IVLEN, "IV length %zu is not in 1..%d", iv_len, kMaxIvBytes);
    if (!valid_tag_len(tag_len))
        return fail(GCM_E_ARG, "tag length %zu is not 16, 15, 14, 13, 12, 8 or 4", tag_len);
    int rc = check_message(aad_len, len, aad_d, in_d, out_d);
    if (rc)
        return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> g(ctx->mu);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess)
        return fail_hip(e, "hipSetDevice");
    const Shape sh = message_shape(ctx, (uint32_t)key_len, len, aad_len);
    const uint64_t m = ghash_blocks(aad_len, len);
    const uint64_t T = (m + (1ull << sh.log2B) - 1) >> sh.log2B;
    rc = ensure_ws_locked(ctx, workspace_bytes_for(T, 1));
    if (rc)
        return rc;
    uint32_t slot;
    rc = cached_slot_locked(ctx, key, key_len, &slot, s);
    if (rc)
        return rc;
    // the tag (16 bytes) and the accept flag (4 bytes): in the mapped result
    // block, which the combine reads and writes directly, else on the device
    // with copies
    const bool mapped = ctx->d_map != nullptr;
    uint8_t *d_tag = mapped ? ctx->d_map : ctx->d_io;
    int32_t *d_ok = reinterpret_cast<int32_t *>(d_tag + 16);
    if (op == 1) {
        if (mapped) {
            std::memcpy(ctx->h_map, tag_in, tag_len);
        } else {
            e = hipMemcpyAsync(d_tag, tag_in, tag_len, hipMemcpyHostToDevice, s);
            if (e != hipSuccess)
                return fail_hip(e, "tag upload");
        }
    }
    MsgDesc d;
    fill_desc(&d, op, kZeroIv, (uint64_t)aad_d, aad_len, (uint64_t)in_d, (uint64_t)out_d, len, (uint64_t)d_tag,
              (uint64_t)d_ok, (uint64_t)(ctx->d_slots + kSlotBytes * slot), slot_nr(key_len), sh.log2B, sh.waves, 0);
    d.tag_len = (uint32_t)tag_len;
    rc = set_iv(&d, iv, iv_len, ctx->d_ws, s);
    if (rc)
        return rc;
    rc = launch_single(ctx, d, sh, ctx->d_ws, s);
    if (rc)
        return rc;
    e = mapped ? hipSuccess : hipMemcpyAsync(ctx->h_io, ctx->d_io, 32, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail_hip(e, "result download");
    const uint8_t *res = mapped ? ctx->h_map : ctx->h_io;
    if (op == 0) {
        std::memcpy(tag_out, res, tag_len);
    } else {
        int32_t ok;
        std::memcpy(&ok, res + 16, 4);
        *accept = ok == 1 ? 1 : 0;
    }
    return GCM_OK;
}

extern "C" int gcm_encrypt_ex(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                              const uint8_t *aad_d, uint64_t aad_len, const uint8_t *pt_d, uint64_t len, uint8_t *ct_d,
                              uint8_t *tag_out, size_t tag_len, void *stream)
{
    GCM_ABI_TRY
        return oneshot(ctx, 0, key, key_len, iv, iv_len, aad_d, aad_len, pt_d, len, ct_d, nullptr, tag_out, nullptr,
                       stream, tag_len);
    GCM_ABI_CATCH
}

extern "C" int gcm_decrypt_verify_ex(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv,
                                     size_t iv_len, const uint8_t *aad_d, uint64_t aad_len, const uint8_t *ct_d,
                                     uint64_t len, const uint8_t *tag, size_t tag_len, uint8_t *pt_d, int *accept,
                                     void *stream)
{
    GCM_ABI_TRY
        return oneshot(ctx, 1, key, key_len, iv, iv_len, aad_d, aad_len, ct_d, len, pt_d, tag, nullptr, accept, stream,
                       tag_len);
    GCM_ABI_CATCH
}

extern "C" int gcm_encrypt(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                           const uint8_t *aad_d, uint64_t aad_len, const uint8_t *pt_d, uint64_t len, uint8_t *ct_d,
                           uint8_t tag_out[16], void *stream)
{
    GCM_ABI_TRY
        return oneshot(ctx, 0, key, key_len, iv, iv_len, aad_d, aad_len, pt_d, len, ct_d, nullptr, tag_out, nullptr,
                       stream);
    GCM_ABI_CATCH
}

extern "C" int gcm_decrypt_verify(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                                  const uint8_t *aad_d, uint64_t aad_len, const uint8_t *ct_d, uint64_t len,
                                  const uint8_t tag[16], uint8_t *pt_d, int *accept, void *stream)
{
    GCM_ABI_TRY
        return oneshot(ctx, 1, key, key_len, iv, iv_len, aad_d, aad_len, ct_d, len, pt_d, tag, nullptr, accept, stream);
    GCM_ABI_CATCH
}

// ---------------------------------------------------------------- counter mode only, GMAC

static int ctr_common(gcm_ctx *ctx, uint32_t slot, uint32_t nr, const uint8_t *iv, const uint8_t *in_d, uint64_t len,
                      uint8_t *out_d, hipStream_t s)
{
    const Shape sh = message_shape(ctx, (nr - 6) * 4, len, 0);
    MsgDesc d;
    fill_desc(&d, 2, iv, 0, 0, (uint64_t)in_d, (uint64_t)out_d, len, 0, 0,
              (uint64_t)(ctx->d_slots + kSlotBytes * slot), nr, sh.log2B, sh.waves, 0);
    return launch_single(ctx, d, sh, nullptr, s);
}

static int check_ctr_args(const void *iv, size_t iv_len, const uint8_t *in_d, uint64_t len, const uint8_t *out_d)
{
    if (!iv)
        return fail(GCM_E_ARG, "NULL argument");
    if (iv_len != 12)
        return fail(GCM_E_IVLEN, "IV length %zu is not 12", iv_len);
    return check_message(0, len, nullptr, in_d, out_d);
}

extern "C" int gcm_ctr_async(gcm_ctx *ctx, uint32_t slot, const uint8_t *iv, size_t iv_len, const uint8_t *in_d,
                             uint64_t len, uint8_t *out_d, void *stream)
{
    GCM_ABI_TRY
        if (!ctx)
            return fail(GCM_E_ARG, "NULL argument");
        int rc = check_ctr_args(iv, iv_len, in_d, len, out_d);
        if (rc)
            return rc;
        std::lock_guard<std::mutex> g(ctx->mu);
        if (slot >= ctx->n_slots || !ctx->slot_used[slot])
            return fail(GCM_E_SLOT, "key slot %u is not registered", slot);
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess)
            return fail_hip(e, "hipSetDevice");
        return ctr_common(ctx, slot, ctx->slot_nr[slot], iv, in_d, len, out_d, reinterpret_cast<hipStream_t>(stream));
    GCM_ABI_CATCH
}

extern "C" int gcm_ctr_xcrypt(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                              const uint8_t *in_d, uint64_t len, uint8_t *out_d, void *stream)
{
    GCM_ABI_TRY
        if (!ctx || !key)
            return fail(GCM_E_ARG, "NULL argument");
        if (!valid_key_len(key_len))
            return fail(GCM_E_KEYLEN, "key length %zu is not 16, 24 or 32", key_len);
        int rc = check_ctr_args(iv, iv_len, in_d, len, out_d);
        if (rc)
            return rc;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        std::lock_guard<std::mutex> g(ctx->mu);
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess)
            return fail_hip(e, "hipSetDevice");
        uint32_t slot;
        rc = cached_slot_locked(ctx, key, key_len, &slot, s);
        if (rc)
            return rc;
        rc = ctr_common(ctx, slot, slot_nr(key_len), iv, in_d, len, out_d, s);
        if (rc)
            return rc;
        // like the other one-shot calls, return with the work done, so that the
        // cached key slot may be reused by the next call on any stream
        e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return fail_hip(e, "hipStreamSynchronize");
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_gmac(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                        const uint8_t *aad_d, uint64_t aad_len, uint8_t tag_out[16], void *stream)
{
    GCM_ABI_TRY
        return oneshot(ctx, 0, key, key_len, iv, iv_len, aad_d, aad_len, nullptr, 0, nullptr, nullptr, tag_out, nullptr,
                       stream);
    GCM_ABI_CATCH
}

// ---------------------------------------------------------------- measurement

hipError_t gcm::prof_begin(gcm_ctx *ctx, hipStream_t s)
{
    if (!ctx->prof)
        return hipSuccess;
    std::pair<hipEvent_t, hipEvent_t> pr;
    if (!ctx->prof_free.empty()) {
        pr = ctx->prof_free.back();
        ctx->prof_free.pop_back();
    } else {
        hipError_t e = hipEventCreate(&pr.first);
        if (e != hipSuccess)
            return e;
        e = hipEventCreate(&pr.second);
        if (e != hipSuccess) {
            (void)hipEventDestroy(pr.first);
            return e;
        }
    }
    ctx->prof_pending.push_back(pr);
    return hipEventRecord(pr.first, s);
}

hipError_t gcm::prof_end(gcm_ctx *ctx, hipStream_t s)
{
    if (!ctx->prof || ctx->prof_pending.empty())
        return hipSuccess;
    return hipEventRecord(ctx->prof_pending.back().second, s);
}

extern "C" int gcm_profile_enable(gcm_ctx *ctx, int enable)
{
    GCM_ABI_TRY
        if (!ctx)
            return fail(GCM_E_ARG, "gcm_profile_enable: NULL context");
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->prof = enable != 0;
        return GCM_OK;
    GCM_ABI_CATCH
}

extern "C" int gcm_profile_read(gcm_ctx *ctx, uint64_t *launches, double *tile_ms_total)
{
    GCM_ABI_TRY
        if (!ctx || !launches || !tile_ms_total)
            return fail(GCM_E_ARG, "gcm_profile_read: NULL argument");
        std::lock_guard<std::mutex> g(ctx->mu);
        double total = 0.0;
        uint64_t n = 0;
        for (auto &pr : ctx->prof_pending) {
            hipError_t e = hipEventSynchronize(pr.second);
            float ms = 0.f;
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms, pr.first, pr.second);
            if (e != hipSuccess)
                return fail_hip(e, "profile event");
            total += ms;
            ++n;
            ctx->prof_free.push_back(pr);
        }
        ctx->prof_pending.clear();
        *launches = n;
        *tile_ms_total = total;
        return GCM_OK;
    GCM_ABI_CATCH
}
