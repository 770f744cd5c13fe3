// gcm_plan.h -- launch planning shared by every entry point: argument and
// aliasing checks, tile geometry, per-message descriptors, batch work lists
// and workspace sizes.  It holds no HIP state (plain C++ over the layouts of
// gcm_internal.h), so the same code runs inside the library and in a
// CPU-only harness built with the address and undefined-behaviour
// sanitizers.
//
// Geometry (the paper's map phase over wave tiles): a message's GHASH input
// X = A || 0-pad || C || 0-pad || L has m = n_A + n + 1 blocks (SP 800-38D
// GCM-AE step 5), left-padded with z zero blocks so that m + z = T * 2^log2B
// (GHASH(0^z || X) = GHASH(X)); wave tile t covers padded positions
// [t * 2^log2B, (t + 1) * 2^log2B) and leaves one 16-byte partial.
#pragma once
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "../../include/gcm_mi355.h"
#include "gcm_internal.h"

namespace gcm {

constexpr uint64_t kMaxLen = (1ull << 36) - 32;  // 2^39 - 256 bits (SP 800-38D sec. 5.2.1.1)
constexpr uint64_t kMaxAad = (1ull << 61) - 1;   // < 2^64 bits

// A launch shape: wave tile size (log2 blocks; for a batch, the cap on its
// messages' tile sizes), waves per workgroup, resident workgroups per compute
// unit, and the fan-in of the reduction tree over tile partials.  Results
// never depend on it, only speed does.
struct Shape {
    uint32_t log2B = 16, waves = 16, gpc = 1, fanin = 2;
};
using TuneEntry = Shape;

// size bucket of the autotune caches: floor(log2 x) (0 for x <= 1)
inline uint32_t size_bucket(uint64_t x)
{
    uint32_t b = 0;
    while (b < 63 && (2ull << b) <= x)
        ++b;
    return b;
}

inline bool valid_fanin(uint32_t f) { return f == 2 || f == 4 || f == 8 || f == 16; }

// An error found while planning: a GCM_E_* code and its message.
struct PlanError {
    int code = GCM_OK;
    char msg[256] = {0};
};

inline int plan_fail(PlanError *e, int code, const char *fmt, ...)
{
    if (e) {
        e->code = code;
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(e->msg, sizeof e->msg, fmt, ap);
        va_end(ap);
    }
    return code;
}

// GHASH blocks of a message: AAD blocks, data blocks and the length block.
inline uint64_t ghash_blocks(uint64_t aad_len, uint64_t len) { return (aad_len + 15) / 16 + (len + 15) / 16 + 1; }

inline uint32_t ceil_log2_u64(uint64_t x)
{
    uint32_t l = 0;
    while (l < 63 && (1ull << l) < x)
        ++l;
    return l;
}

// [a, a + alen) and [b, b + blen) share a byte (empty ranges share none);
// written without forming a + alen, so no address can overflow it.
inline bool ranges_overlap(uint64_t a, uint64_t alen, uint64_t b, uint64_t blen)
{
    if (!alen || !blen)
        return false;
    return a >= b ? a - b < blen : b - a < alen;
}

// Tile size of one message launched alone, by makespan: `resident` waves
// run tiles k, k + R, ...; tile 0 holds the zero prefix, whose whole rows are
// skipped; each tile adds a fixed cost (fix-up, partial) of about kTileCost
// blocks.  Tiles of one or two rows only while every tile gets a wave of its
// own.  Ties go to the larger tile (fewer partials).
inline uint32_t heuristic_log2B(uint64_t m, uint64_t resident)
{
    constexpr uint64_t kTileCost = 64;
    if (resident == 0)
        resident = 1;
    uint64_t best_cost = ~0ull;
    uint32_t best_l = 16;
    for (uint32_t l = 16; l >= 6; --l) {
        const uint64_t B = 1ull << l;
        const uint64_t T = (m + B - 1) / B;
        if (l < 8 && T > resident)
            continue;
        const uint64_t z = T * B - m;
        const uint64_t n0 = (T + resident - 1) / resident, n1 = T > 1 ? (T - 1 + resident - 1) / resident : 0;
        const uint64_t c0 = (n0 - 1) * B + (B - z / 64 * 64) + kTileCost * n0;
        const uint64_t c1 = n1 * (B + kTileCost);
        const uint64_t cost = std::max(c0, c1);
        if (cost < best_cost) {
            best_cost = cost;
            best_l = l;
        }
    }
    return best_l;
}

// Rows of 64 blocks that the busiest compute unit runs for one message
// launched with tiles of 2^l blocks in workgroups of `waves` waves: item k
// (tiles [k*waves, (k+1)*waves)) goes to workgroup k mod grid, grid =
// min(items, cus * gpc), and each tile costs its rows plus about one row of
// fix-up.  Used to compare shapes, not to predict times.
inline uint64_t busiest_cu_rows(uint64_t m, uint32_t l, uint32_t waves, uint64_t cus, uint32_t gpc)
{
    const uint64_t B = 1ull << l, T = (m + B - 1) / B;
    const uint64_t items = (T + waves - 1) / waves;
    const uint64_t slots = cus * (gpc ? gpc : 1);
    const uint64_t grid = items < slots ? items : slots;
    uint64_t tiles = 0;  // workgroup 0's, its items k*grid
    for (uint64_t k = 0; k * grid < items; ++k) {
        const uint64_t first = k * grid * waves;
        tiles += T - first < waves ? T - first : waves;
    }
    return tiles * (B / 64 + 1) * (gpc ? gpc : 1);
}

// Waves per workgroup for one message (tile size from heuristic_log2B for
// that many waves).  Sixteen unless the message has fewer tiles than the
// chip has wave slots: then 16-wave workgroups would crowd its tiles onto a
// fraction of the compute units, and 12 or 8 waves a workgroup spread them
// over more.  Among 16, 12 and 8 the one whose busiest compute unit has the
// fewest rows (busiest_cu_rows) wins, ties to more waves.  gpc(w): groups a
// compute unit holds with w waves.
template <typename Gpc>
inline uint32_t heuristic_waves(uint64_t m, uint64_t cus, Gpc gpc)
{
    const uint32_t g16 = gpc(16);
    const uint32_t l16 = heuristic_log2B(m, cus * g16 * 16);
    const uint64_t t16 = (m + (1ull << l16) - 1) >> l16;
    if ((t16 + 15) / 16 >= cus * g16)
        return 16;
    uint32_t best_w = 16;
    uint64_t best = busiest_cu_rows(m, l16, 16, cus, g16);
    for (uint32_t w : {12u, 8u}) {
        const uint32_t g = gpc(w);
        const uint32_t l = heuristic_log2B(m, cus * g * w);
        const uint64_t load = busiest_cu_rows(m, l, w, cus, g);
        if (load < best) {
            best = load;
            best_w = w;
        }
    }
    return best_w;
}

// Tiles that suffice for every message of at most m GHASH blocks planned by
// the heuristics above (t_own: the m-block message's own tile count): a
// tile size below 2^8 blocks is only chosen while the tiles fit the
// resident waves (at most `resident_max` over the wave counts), larger ones
// give at most ceil(m / 256) tiles.  The tile count is not monotonic in the
// length (a longer message may take larger tiles), so a workspace sized for
// the longest message of a set needs this bound, not its own count.
inline uint64_t tiles_bound_upto(uint64_t m, uint64_t t_own, uint64_t resident_max)
{
    const uint64_t small = std::min<uint64_t>((m + 63) / 64, resident_max);
    return std::max<uint64_t>(t_own, std::max<uint64_t>(small, (m + 255) / 256));
}

// Tile size of one message inside a batch: about one workgroup item (waves
// tiles) for small messages, at most 2^cap blocks per tile for large ones,
// so the persistent workgroups see items of similar cost.  cap: 6..20.
inline uint32_t batch_msg_log2B(uint64_t m, uint32_t waves, uint32_t cap)
{
    const uint32_t l = std::max<uint32_t>(6, ceil_log2_u64((m + waves - 1) / waves));
    return std::min(l, std::max<uint32_t>(6, cap));
}

// Workspace: a counter and reject list (4 + 4 * n_msgs bytes, rounded up to
// 256), then per message its T tile partials followed by two 16-byte slots:
// E_K(J0) (left by the tile-0 wave for the combine) and J0 (IVs other than
// 96 bits).
inline uint64_t workspace_counter_bytes(uint64_t n_msgs) { return ((4 + 4 * n_msgs) + 255) / 256 * 256; }
inline uint64_t workspace_bytes_for(uint64_t total_tiles, uint64_t n_msgs)
{
    return workspace_counter_bytes(n_msgs) + 16 * (total_tiles + 2 * n_msgs);
}

inline void fill_desc(MsgDesc *d, uint32_t op, const uint8_t *iv, uint64_t aad, uint64_t aad_len, uint64_t in,
                      uint64_t out, uint64_t len, uint64_t tag, uint64_t ok, uint64_t slot_addr, uint32_t nr,
                      uint32_t log2B, uint32_t waves, uint64_t tile_base)
{
    memset(d, 0, sizeof *d);
    d->in = in;
    d->out = out;
    d->aad = aad;
    d->tag = tag;
    d->ok = ok;
    d->len = len;
    d->aad_len = aad_len;
    d->slot = slot_addr;
    d->n = (len + 15) / 16;
    d->na = (aad_len + 15) / 16;
    d->m = d->na + d->n + 1;
    const uint64_t B = 1ull << log2B;
    d->n_tiles = (d->m + B - 1) / B;
    d->z = d->n_tiles * B - d->m;
    d->tile_lo = 0;
    d->tile_hi = d->n_tiles;
    d->tile_base = tile_base;
    for (int i = 0; i < 3; ++i)
        d->iv[i] = (uint32_t)iv[4 * i] | ((uint32_t)iv[4 * i + 1] << 8) | ((uint32_t)iv[4 * i + 2] << 16) |
                   ((uint32_t)iv[4 * i + 3] << 24);
    d->op = op;
    d->log2B = log2B;
    d->nr = nr;
    d->groups = (uint32_t)((d->n_tiles + waves - 1) / waves);
    d->tag_len = 16;
}

// Device buffers of one message: NULL with a non-zero length, 16-byte
// alignment of AAD and payload, and aliasing.  The output may equal the
// input exactly (in place) but may not overlap it otherwise, nor overlap the
// AAD (still being hashed while other waves write output), the tag (written
// or compared after the output is written) or the accept flag.  tag / ok of
// 0 are not checked.
inline int check_buffers(uint64_t aad, uint64_t aad_len, uint64_t in, uint64_t out, uint64_t len, uint64_t tag,
                         uint64_t tag_len, uint64_t ok, PlanError *err)
{
    if ((len && (!in || !out)) || (aad_len && !aad))
        return plan_fail(err, GCM_E_ARG, "NULL device buffer with non-zero length");
    if ((aad_len && (aad & 15)) || (len && ((in & 15) || (out & 15))))
        return plan_fail(err, GCM_E_ARG, "device buffers must be 16-byte aligned");
    if (len && in != out && ranges_overlap(in, len, out, len))
        return plan_fail(err, GCM_E_ALIAS, "input and output overlap without being identical");
    if (ranges_overlap(out, len, aad, aad_len))
        return plan_fail(err, GCM_E_ALIAS, "output overlaps the AAD");
    if (tag && ranges_overlap(out, len, tag, tag_len))
        return plan_fail(err, GCM_E_ALIAS, "output overlaps the tag");
    if (ok && ranges_overlap(out, len, ok, 4))
        return plan_fail(err, GCM_E_ALIAS, "output overlaps the accept flag");
    return GCM_OK;
}

inline int check_lengths(uint64_t aad_len, uint64_t len, PlanError *err)
{
    if (len > kMaxLen || aad_len > kMaxAad)
        return plan_fail(err, GCM_E_TOOLONG, "len %llu / aad_len %llu beyond the SP 800-38D limits",
                         (unsigned long long)len, (unsigned long long)aad_len);
    return GCM_OK;
}

// The key table as the planner sees it.
struct SlotView {
    uint64_t base = 0;              // device address of slot 0
    uint32_t n_slots = 0;
    const uint8_t *used = nullptr;  // [n_slots] 1 = registered
    const uint32_t *nr = nullptr;   // [n_slots] AES rounds
    uint64_t addr(uint32_t s) const { return base + kSlotBytes * (uint64_t)s; }
    bool valid(uint32_t s) const { return s < n_slots && used[s]; }
};

// One job of a batch against a base allocation of base_bytes bytes.
inline int check_job(const gcm_job &j, uint32_t idx, uint64_t base_bytes, const SlotView &slots, PlanError *err)
{
    if (j.op > 1)
        return plan_fail(err, GCM_E_ARG, "job %u: op %u is neither 0 (encrypt) nor 1 (decrypt-verify)", idx, j.op);
    if (j.reserved != 0)
        return plan_fail(err, GCM_E_ARG, "job %u: reserved field must be 0", idx);
    if (!slots.valid(j.key_slot))
        return plan_fail(err, GCM_E_SLOT, "job %u: key slot %u is not registered", idx, j.key_slot);
    if (j.len > kMaxLen || j.aad_len > kMaxAad)
        return plan_fail(err, GCM_E_TOOLONG, "job %u: len %llu / aad_len %llu beyond the SP 800-38D limits", idx,
                         (unsigned long long)j.len, (unsigned long long)j.aad_len);
    auto inside = [&](uint64_t off, uint64_t len) { return off <= base_bytes && len <= base_bytes - off; };
    if (!inside(j.in_off, j.len) || !inside(j.out_off, j.len) || !inside(j.aad_off, j.aad_len) ||
        !inside(j.tag_off, 16) || (j.op == 1 && !inside(j.ok_off, 4)))
        return plan_fail(err, GCM_E_ARG, "job %u: a buffer lies outside the %llu-byte base allocation", idx,
                         (unsigned long long)base_bytes);
    if ((j.len && ((j.in_off | j.out_off) & 15)) || (j.aad_len && (j.aad_off & 15)) || (j.op == 1 && (j.ok_off & 3)))
        return plan_fail(err, GCM_E_ARG, "job %u: payload offsets must be 16-byte aligned and ok_off 4-byte aligned",
                         idx);
    if (j.len && j.in_off != j.out_off && ranges_overlap(j.in_off, j.len, j.out_off, j.len))
        return plan_fail(err, GCM_E_ALIAS, "job %u: input and output overlap without being identical", idx);
    if (ranges_overlap(j.out_off, j.len, j.aad_off, j.aad_len) || ranges_overlap(j.out_off, j.len, j.tag_off, 16) ||
        (j.op == 1 && ranges_overlap(j.out_off, j.len, j.ok_off, 4)))
        return plan_fail(err, GCM_E_ALIAS, "job %u: output overlaps its AAD, tag or accept flag", idx);
    return GCM_OK;
}

// One message of a batch, with absolute device addresses.
struct PlanMsg {
    uint32_t op = 0;
    uint32_t key_slot = 0;
    uint8_t iv[12] = {0};
    uint64_t aad = 0, aad_len = 0, in = 0, out = 0, len = 0, tag = 0, ok = 0;
};

inline PlanMsg plan_msg_from_job(const gcm_job &j, uint64_t base)
{
    PlanMsg p;
    p.op = j.op;
    p.key_slot = j.key_slot;
    memcpy(p.iv, j.iv, 12);
    p.aad = base + j.aad_off;
    p.aad_len = j.aad_len;
    p.in = base + j.in_off;
    p.out = base + j.out_off;
    p.len = j.len;
    p.tag = base + j.tag_off;
    p.ok = base + j.ok_off;
    return p;
}

// The persistent launch of a batch: descriptors (message i's partials start
// at tile_base, after the n_tiles + 2 slots of the messages before it), and
// the work list -- items of `waves` consecutive wave tiles of one message --
// ordered by key slot so that a persistent workgroup restages its GHASH table
// only when the key changes.
struct BatchPlan {
    std::vector<MsgDesc> descs;
    std::vector<WorkItem> items;
    uint64_t total_tiles = 0;   // sum of n_tiles
    uint64_t partial_slots = 0; // sum of n_tiles + 2 (the workspace's per-message part)
    uint64_t payload = 0;
    bool any_decrypt = false;
    uint64_t workspace_bytes() const { return workspace_counter_bytes(descs.size()) + 16 * partial_slots; }
};

inline void plan_batch(const PlanMsg *msgs, uint32_t n, const SlotView &slots, uint32_t waves, uint32_t cap_log2B,
                       BatchPlan *p)
{
    p->descs.assign(n, MsgDesc{});
    p->items.clear();
    p->total_tiles = p->partial_slots = p->payload = 0;
    p->any_decrypt = false;
    uint64_t tile_base = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const PlanMsg &j = msgs[i];
        const uint32_t log2B = batch_msg_log2B(ghash_blocks(j.aad_len, j.len), waves, cap_log2B);
        fill_desc(&p->descs[i], j.op, j.iv, j.aad, j.aad_len, j.in, j.out, j.len, j.tag, j.ok, slots.addr(j.key_slot),
                  slots.nr[j.key_slot], log2B, waves, tile_base);
        tile_base += p->descs[i].n_tiles + 2;  // partials, then the E_K(J0) and J0 slots
        p->total_tiles += p->descs[i].n_tiles;
        p->any_decrypt |= j.op == 1;
        p->payload += j.len;
    }
    p->partial_slots = tile_base;
    std::vector<uint32_t> order(n);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t c) { return msgs[a].key_slot < msgs[c].key_slot; });
    for (uint32_t i : order)
        for (uint64_t t = 0; t < p->descs[i].n_tiles; t += waves)
            p->items.push_back(WorkItem{i, (uint32_t)t});
}

// Device bytes a message adds to the batch that carries it, for any launch
// shape the library may pick (tiles of at least 64 blocks, items of at least
// 8 waves): its descriptor, work items, accept flag, reject-list entry, tile
// partials with their two extra slots, and room for the four 256-byte
// roundings of a batch's sections.
inline uint64_t batch_overhead_bound(uint64_t aad_len, uint64_t len)
{
    const uint64_t T = (ghash_blocks(aad_len, len) + 63) / 64;
    return sizeof(MsgDesc) + sizeof(WorkItem) * ((T + 7) / 8) + 4 + 4 + 16 * (T + 2) + 4 * 256;
}

}  // namespace gcm
