// gcm_host.h -- host-side internals shared by the runtime sources.
#pragma once
#include <hip/hip_runtime.h>

#include <list>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "gcm_internal.h"
#include "gcm_plan.h"

struct gcm_ctx {
    int device = 0;
    int cu_count = 1;
    uint64_t budget = 0;  // 0 = unbounded
    uint64_t used = 0;
    uint32_t *d_tables = nullptr;  // kAesTableWords: TE0, the S-box (as words), TE1..TE3
    void *d_frob = nullptr;        // Frobenius tables x -> x^(2^k), k = 1..47
    uint8_t *d_slots = nullptr;    // n_slots * kSlotBytes
    uint32_t n_slots = 0;
    std::vector<uint8_t> slot_used;
    std::vector<uint32_t> slot_nr;  // AES rounds of each registered slot
    // one-shot key cache
    std::unordered_map<std::string, uint32_t> cache;
    std::list<std::string> lru;
    uint32_t cache_cap = 1;
    // one-shot scratch
    uint8_t *d_ws = nullptr;
    uint64_t ws_bytes = 0;
    uint8_t *d_io = nullptr;  // device tag (16 B) + flag (4 B)
    // the device's fixed scratch (kNoAllocScratchBytes, shared by every
    // context on the device; its address, looked up at context creation)
    void *d_scratch = nullptr;
    uint8_t *h_io = nullptr;  // pinned mirror
    // one-shot results: pinned, host-coherent memory the kernels read the
    // expected tag from and write the tag / flag to directly (d_map is its
    // device address); NULL where the runtime cannot map it (then d_io and
    // copies are used)
    uint8_t *h_map = nullptr;
    uint8_t *d_map = nullptr;
    // launch shape overrides (0 = automatic)
    uint32_t cfg_log2B = 0, cfg_waves = 0, cfg_gpc = 0, cfg_fanin = 0;
    // autotune caches: single messages keyed by (key bytes << 32 | floor(log2
    // len)); batches keyed by (floor(log2 messages) << 32 | floor(log2 payload))
    std::unordered_map<uint64_t, gcm::TuneEntry> tuned;
    std::unordered_map<uint64_t, gcm::TuneEntry> tuned_batch;
    // tile-kernel timing (events recorded on the launch stream)
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_free;
    // host-to-host pipeline (created on first use): streams for H2D, the
    // kernels and D2H, a ring of device chunk buffers and their events
    uint64_t pipe_chunk = 0;  // requested chunk bytes (0 = default)
    bool pipe_ready = false;
    hipStream_t pipe_h2d = nullptr, pipe_comp = nullptr, pipe_d2h = nullptr;
    static constexpr int kPipeBufs = 3;
    hipEvent_t pipe_in[kPipeBufs] = {}, pipe_done[kPipeBufs] = {}, pipe_free[kPipeBufs] = {};
    bool pipe_used[kPipeBufs] = {};
    uint8_t *pipe_buf[kPipeBufs] = {};
    uint64_t pipe_buf_bytes = 0;
    uint8_t *pipe_aad = nullptr;
    uint64_t pipe_aad_bytes = 0;
    // buffers of destroyed streamed messages, kept for the next
    // gcm_stream_begin so that a stream allocates nothing in the common
    // case: the device partials buffer (counted in `used`), the pinned
    // staging of the final call's segment descriptors, and an event recorded
    // after the last work that used them (a later stream's work waits for
    // it; the host waits for it before rewriting the staging or freeing).
    // Released when an allocation would exceed the budget, and at context
    // destruction.
    struct StreamBufs {
        uint8_t *d_part;
        uint64_t part_bytes;
        gcm::MsgDesc *h_desc;
        uint64_t h_desc_bytes;
        hipEvent_t ev;
    };
    std::vector<StreamBufs> stream_pool;
    std::mutex mu;
};

// Every extern "C" entry point runs its body between GCM_ABI_TRY and one of
// the GCM_ABI_CATCH forms, so that no C++ exception (a failed host
// allocation, a thread that cannot be started) crosses the C boundary.
#define GCM_ABI_TRY try {
#define GCM_ABI_CATCH                     \
    }                                     \
    catch (...)                           \
    {                                     \
        return gcm::abi_exception();      \
    }
#define GCM_ABI_CATCH_VALUE(v)            \
    }                                     \
    catch (...)                           \
    {                                     \
        (void)gcm::abi_exception();       \
        return (v);                       \
    }
#define GCM_ABI_CATCH_VOID                \
    }                                     \
    catch (...)                           \
    {                                     \
        (void)gcm::abi_exception();       \
    }

namespace gcm {

int fail(int code, const char *fmt, ...);
// record a planning error as the thread's last error and return its code
int plan_error(const PlanError &e);
int fail_hip(hipError_t e, const char *what);
// The status for the exception in flight (called from a catch block):
// std::bad_alloc -> GCM_E_NOMEM, anything else -> GCM_E_INTERNAL, with the
// message recorded for gcm_last_error.
int abi_exception() noexcept;

int ctx_alloc(gcm_ctx *ctx, void **p, uint64_t bytes);
void ctx_free(gcm_ctx *ctx, void *p, uint64_t bytes);
int register_key_locked(gcm_ctx *ctx, const uint8_t *key, size_t key_len, uint32_t *slot_out, hipStream_t s);
int register_keys_locked(gcm_ctx *ctx, const uint8_t *const *keys, const uint32_t *key_lens, uint32_t n,
                         uint32_t *slots_out, hipStream_t s);

// Launch shape of one message: explicit settings (gcm_set_launch), else the
// autotune cache entry for (key size, message size), else the heuristic.
// Every single-message path (one-shot, asynchronous, counter mode, host
// pipeline, streamed segments, GCM-SIV) and gcm_workspace_size use it.
Shape message_shape(const gcm_ctx *ctx, uint32_t key_bytes, uint64_t len, uint64_t aad_len);
// groups of the tile kernel (`waves` waves each) a compute unit holds
uint32_t groups_per_cu(uint32_t waves);
// the most waves the planners may count as resident (any wave count)
uint64_t resident_bound(const gcm_ctx *ctx);
// frees the buffers kept for streamed messages (caller holds ctx->mu; no
// queued work uses them)
void stream_pool_release(gcm_ctx *ctx);
// Launch shape of a batch of n messages and `payload` bytes holding m GHASH
// blocks in all: explicit settings, else the batch autotune cache, else the
// heuristic (tile cap from the single-launch heuristic, 16 waves).
Shape batch_shape(const gcm_ctx *ctx, uint64_t n, uint64_t payload, uint64_t m);
// the key table as the planner sees it
SlotView slot_view(const gcm_ctx *ctx);
// lengths and device buffers of one message (see check_buffers)
int check_message(uint64_t aad_len, uint64_t len, const void *aad_d, const void *in_d, const void *out_d,
                  const void *tag_d = nullptr, uint64_t tag_len = 16, const void *ok_d = nullptr);
// IV lengths the device path takes (1..kMaxIvBytes bytes)
bool valid_iv_len(size_t n);
// Set the descriptor's IV: 12 bytes go in d.iv; any other length enqueues the
// J0 kernel on `s` (d.slot must be set), writing J0 to the message's J0 slot
// of workspace `ws` (after its partials and E_K(J0)), and points d.j0 there.
int set_iv(MsgDesc *d, const uint8_t *iv, size_t iv_len, void *ws, hipStream_t s);
int launch_single(gcm_ctx *ctx, const MsgDesc &d, const Shape &sh, void *ws, hipStream_t s);
// The asynchronous single-message path (gcm_encrypt_async /
// gcm_decrypt_verify_async): validate, plan with message_shape and enqueue
// on `stream` with the caller's workspace.  With fit_ws (the no-allocation
// path) the tile size is raised (up to 2^kFitMaxLog2B blocks) until the
// partials fit in ws_bytes, a message that still does not fit is
// GCM_E_NOMEM, and no profiling events are recorded.
constexpr uint32_t kFitMaxLog2B = 16;
int async_launch(gcm_ctx *ctx, uint32_t op, uint32_t slot, const uint8_t *iv, size_t iv_len, const uint8_t *aad_d,
                 uint64_t aad_len, const uint8_t *in_d, uint64_t len, uint8_t *out_d, const uint8_t *tag_d,
                 int32_t *ok_d, void *ws, uint64_t ws_bytes, bool fit_ws, void *stream);
// batches (gcm_batch.cpp; caller holds ctx->mu): validate and plan jobs
// (with `forced` as the shape if non-NULL), create a batch, enqueue its
// kernels, free it
int plan_jobs(const gcm_ctx *ctx, const gcm_job *jobs, uint32_t n, uint8_t *base_d, uint64_t base_bytes,
              const Shape *forced, Shape *sh_out, BatchPlan *plan);
int batch_create_locked(gcm_ctx *ctx, const gcm_job *jobs, uint32_t n, uint8_t *base_d, uint64_t base_bytes,
                        const Shape *forced, gcm_batch **out);
hipError_t batch_enqueue(gcm_batch *b, hipStream_t s);
void batch_free_locked(gcm_batch *b);
// release the host pipeline's streams, events and buffers (gcm_ctx_destroy)
void pipeline_release(gcm_ctx *ctx);
// ensure the context's one-shot workspace holds `bytes` (caller holds ctx->mu)
int ensure_ws_locked(gcm_ctx *ctx, uint64_t bytes);
// one-shot key cache lookup / expansion (caller holds ctx->mu)
int cached_slot_locked(gcm_ctx *ctx, const uint8_t *key, size_t key_len, uint32_t *slot, hipStream_t s);
// tile kernel only, for tiles [d.tile_lo, d.tile_hi); ws may be NULL for op 2
int launch_tile_range(gcm_ctx *ctx, const MsgDesc &d, const Shape &sh, void *ws, hipStream_t s);
// bracket the next tile launch with events when profiling is on (caller holds ctx->mu)
hipError_t prof_begin(gcm_ctx *ctx, hipStream_t s);
hipError_t prof_end(gcm_ctx *ctx, hipStream_t s);

// kernels (gcm_kernels.hip)
hipError_t launch_init_tables(uint32_t *te0, uint32_t *sbox, void *frob, hipStream_t s);
size_t frob_table_bytes();
hipError_t launch_key_setup(const uint8_t *const *keys, const uint32_t *key_lens, const uint64_t *slot_addrs,
                            uint32_t n, const uint32_t *te0, const uint32_t *sbox, const void *frob, hipStream_t s);
hipError_t launch_tiles(int waves, const MsgDesc *descs, const WorkItem *items, uint32_t n_items,
                        const MsgDesc *single, const uint32_t *te0, void *partials, uint32_t *counters, uint32_t grid,
                        hipStream_t s);
int max_groups_per_cu(int waves);
// fanin: children per node of the reduction tree over tile partials (2, 4, 8, 16)
hipError_t launch_combine(const MsgDesc *descs, uint32_t n_msgs, const MsgDesc *single, const void *partials,
                          uint32_t *counters, uint32_t fanin, hipStream_t s);
hipError_t launch_j0(const IvArg &iv, uint64_t slot, void *j0_out, void *y_zero, hipStream_t s);
// streamed message: XOR of k lifted segment values, the length block's term
// lenblk * H (lenblk: memory-order words, or NULL when it is one of the
// values; H from the key slot at device address `slot`) and E_K(J0) -> tag
// (op 0) or accept flag (op 1)
hipError_t launch_fold(const void *vals, uint32_t k, const void *ekj0, uint8_t *tag, int32_t *ok, uint32_t op,
                       uint32_t tag_len, uint64_t slot, const uint32_t lenblk[4], hipStream_t s);
// device address of the fixed scratch array on `device` (looked up once per device)
hipError_t scratch_address(int device, void **out);
hipError_t launch_zerofill(const MsgDesc *descs, const MsgDesc *single, const uint32_t *counters, uint32_t grid,
                           hipStream_t s);
// AES-GCM-SIV: message keys into the slot at out_slot (and, with tag_in, the
// counter block from the received tag at ctr_out); the tile passes (0 POLYVAL
// only, 1 counter mode only, 2 counter mode + POLYVAL of the output); the tag
// from the POLYVAL value at g (encrypt: tag_out and the counter block;
// decrypt: compare with tag_in, accept flag and reject count)
hipError_t launch_siv_derive(uint64_t kgk_slot, const uint8_t nonce[12], uint64_t out_slot, const uint8_t *tag_in,
                             void *ctr_out, const uint32_t *te0, const uint32_t *sbox, const void *frob, hipStream_t s);
hipError_t launch_siv_tiles(int waves, int pass, const MsgDesc &d, uint32_t n_items, const uint32_t *te0,
                            void *partials, uint32_t grid, hipStream_t s);
hipError_t launch_siv_tag(uint64_t slot, const void *g, const uint8_t nonce[12], uint8_t *tag_out, void *ctr_out,
                          const uint8_t *tag_in, int32_t *ok, uint32_t *counters, const uint32_t *te0,
                          const uint32_t *sbox, hipStream_t s);

}  // namespace gcm
