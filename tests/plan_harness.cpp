// CPU harness for the launch planner (paper_2602_23067_amd/csrc/gcm_plan.h),
// built with the address and undefined-behaviour sanitizers: randomized jobs
// against a plain reference of the validation rules, then the invariants
// the kernels rely on for every batch plan that passes validation.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <set>
#include <vector>

#include "gcm_plan.h"

using namespace gcm;

#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c);    \
            std::exit(1);                                                        \
        }                                                                        \
    } while (0)

typedef unsigned __int128 u128;

// overlap of two byte ranges, in 128-bit arithmetic (the reference)
static bool ref_overlap(uint64_t a, uint64_t al, uint64_t b, uint64_t bl)
{
    if (!al || !bl)
        return false;
    return (u128)a < (u128)b + bl && (u128)b < (u128)a + al;
}

// the validation rules of a batch job, written out independently
static int ref_check_job(const gcm_job &j, uint64_t base_bytes, const SlotView &sv)
{
    if (j.op > 1 || j.reserved)
        return GCM_E_ARG;
    if (j.key_slot >= sv.n_slots || !sv.used[j.key_slot])
        return GCM_E_SLOT;
    if (j.len > (1ull << 36) - 32 || j.aad_len > (1ull << 61) - 1)
        return GCM_E_TOOLONG;
    auto in = [&](uint64_t o, uint64_t l) { return (u128)o + l <= base_bytes; };
    if (!in(j.in_off, j.len) || !in(j.out_off, j.len) || !in(j.aad_off, j.aad_len) || !in(j.tag_off, 16) ||
        (j.op == 1 && !in(j.ok_off, 4)))
        return GCM_E_ARG;
    if ((j.len && (j.in_off % 16 || j.out_off % 16)) || (j.aad_len && j.aad_off % 16) || (j.op == 1 && j.ok_off % 4))
        return GCM_E_ARG;
    if (j.len && j.in_off != j.out_off && ref_overlap(j.in_off, j.len, j.out_off, j.len))
        return GCM_E_ALIAS;
    if (ref_overlap(j.out_off, j.len, j.aad_off, j.aad_len) || ref_overlap(j.out_off, j.len, j.tag_off, 16) ||
        (j.op == 1 && ref_overlap(j.out_off, j.len, j.ok_off, 4)))
        return GCM_E_ALIAS;
    return GCM_OK;
}

static uint64_t pick_len(std::mt19937_64 &r)
{
    switch (r() % 8) {
    case 0:
        return 0;
    case 1:
        return r() % 17;
    case 2:
        return r() % 5000;
    case 3:
        return (1ull << 36) - 32 - r() % 3;  // at and just below the limit
    case 4:
        return (1ull << 36) - 31;            // just above
    default:
        return r() % (1u << 20);
    }
}

static uint64_t pick_off(std::mt19937_64 &r, uint64_t base_bytes, uint64_t len)
{
    const int k = (int)(r() % 6);
    uint64_t o;
    if (k == 0)
        o = base_bytes - std::min(base_bytes, len);  // flush with the end
    else if (k == 1)
        o = base_bytes - std::min(base_bytes, len) + 16;  // one block past it
    else if (k == 2)
        o = ~0ull - (r() % 64);  // near 2^64
    else
        o = base_bytes == ~0ull ? r() : r() % (base_bytes + 1);
    return r() % 4 ? o & ~15ull : o;
}

// every invariant of a plan the kernels rely on
static void check_plan(const std::vector<PlanMsg> &msgs, const BatchPlan &p, uint32_t waves, uint32_t cap,
                       const SlotView &sv)
{
    const uint32_t n = (uint32_t)msgs.size();
    CHECK(p.descs.size() == n);
    uint64_t tb = 0, tiles = 0, payload = 0;
    std::vector<std::vector<uint8_t>> covered(n);
    for (uint32_t i = 0; i < n; ++i) {
        const MsgDesc &d = p.descs[i];
        const PlanMsg &m = msgs[i];
        CHECK(d.len == m.len && d.aad_len == m.aad_len && d.in == m.in && d.out == m.out && d.aad == m.aad);
        CHECK(d.n == (m.len + 15) / 16 && d.na == (m.aad_len + 15) / 16 && d.m == d.na + d.n + 1);
        CHECK(d.log2B >= 6 && d.log2B <= std::max<uint32_t>(6, cap));
        const uint64_t B = 1ull << d.log2B;
        CHECK(d.n_tiles >= 1 && (u128)d.n_tiles * B == (u128)d.m + d.z && d.z < B);
        CHECK(d.tile_lo == 0 && d.tile_hi == d.n_tiles);
        CHECK(d.tile_base == tb);
        CHECK(d.slot == sv.addr(m.key_slot) && d.nr == sv.nr[m.key_slot]);
        CHECK(d.op == m.op && d.tag_len == 16);
        CHECK(d.groups == (d.n_tiles + waves - 1) / waves);
        tb += d.n_tiles + 2;
        tiles += d.n_tiles;
        payload += m.len;
        covered[i].assign(d.n_tiles, 0);
    }
    CHECK(p.total_tiles == tiles && p.partial_slots == tb && p.payload == payload);
    // every partial the kernels write (tile partials, E_K(J0), J0) lies inside the workspace
    CHECK(p.workspace_bytes() >= workspace_counter_bytes(n) + 16 * tb);
    CHECK(workspace_counter_bytes(n) >= 4 + 4ull * n && workspace_counter_bytes(n) % 256 == 0);
    // the work list covers each message's tiles exactly once, grouped by key slot
    uint32_t prev_slot = 0;
    for (size_t k = 0; k < p.items.size(); ++k) {
        const WorkItem &w = p.items[k];
        CHECK(w.msg < n);
        const MsgDesc &d = p.descs[w.msg];
        CHECK(w.first_tile % waves == 0 && w.first_tile < d.n_tiles);
        for (uint64_t t = w.first_tile; t < d.n_tiles && t < (uint64_t)w.first_tile + waves; ++t) {
            CHECK(!covered[w.msg][t]);
            covered[w.msg][t] = 1;
        }
        CHECK(k == 0 || msgs[w.msg].key_slot >= prev_slot);
        prev_slot = msgs[w.msg].key_slot;
    }
    for (uint32_t i = 0; i < n; ++i)
        for (uint8_t c : covered[i])
            CHECK(c == 1);
    // the serving loop's per-request bound covers the batch's device bytes
    uint64_t bound = 0;
    for (const PlanMsg &m : msgs)
        bound += batch_overhead_bound(m.aad_len, m.len);
    auto a256 = [](uint64_t x) { return (x + 255) / 256 * 256; };
    const uint64_t actual = a256(n * sizeof(MsgDesc)) + a256(p.items.size() * sizeof(WorkItem)) + a256(4ull * n) +
                            p.workspace_bytes();
    CHECK(actual <= bound);
}

int main()
{
    std::mt19937_64 r(2602);
    // key table: 64 slots, some unregistered, mixed key sizes
    std::vector<uint8_t> used(64);
    std::vector<uint32_t> nr(64);
    for (int i = 0; i < 64; ++i) {
        used[i] = (uint8_t)(i % 7 != 3);
        nr[i] = 10 + 2 * (uint32_t)(i % 3);
    }
    SlotView sv;
    sv.base = 0x7f0000000000ull;
    sv.n_slots = 64;
    sv.used = used.data();
    sv.nr = nr.data();

    // 1. validation against the reference, on random jobs
    uint64_t accepted = 0, rejected[16] = {0};
    for (int it = 0; it < 200000; ++it) {
        const uint64_t base_bytes = (it % 5 == 0) ? ~0ull - (r() % 4096) : (r() % (1ull << 40)) + 1;
        gcm_job j;
        std::memset(&j, 0, sizeof j);
        j.op = r() % 16 ? (uint32_t)(r() % 2) : 2;
        j.key_slot = r() % 16 ? (uint32_t)(r() % 64) : 64 + (uint32_t)(r() % 4);
        j.reserved = r() % 50 ? 0 : 1;
        j.len = pick_len(r);
        j.aad_len = r() % 4 ? r() % 5000 : (r() % 2 ? (1ull << 61) - 1 : 1ull << 61);
        j.in_off = pick_off(r, base_bytes, j.len);
        j.out_off = r() % 3 ? j.in_off : pick_off(r, base_bytes, j.len);
        if (r() % 5 == 0)
            j.out_off = j.in_off + 16 * (r() % 4);  // overlaps
        j.aad_off = pick_off(r, base_bytes, j.aad_len);
        j.tag_off = r() % 6 ? pick_off(r, base_bytes, 16) : j.out_off + (r() % 64);
        j.ok_off = r() % 6 ? pick_off(r, base_bytes, 4) : j.out_off + (r() % 64);
        PlanError err;
        const int got = check_job(j, (uint32_t)it, base_bytes, sv, &err);
        const int want = ref_check_job(j, base_bytes, sv);
        if (got != want) {
            std::fprintf(stderr, "job %d: planner %d, reference %d (%s)\n", it, got, want, err.msg);
            return 1;
        }
        CHECK(got == GCM_OK || err.msg[0] != 0);
        if (got == GCM_OK)
            ++accepted;
        else
            ++rejected[-got & 15];
    }
    CHECK(accepted > 1000 && rejected[-GCM_E_ALIAS] > 100 && rejected[-GCM_E_ARG] > 100 && rejected[-GCM_E_SLOT] > 100 &&
          rejected[-GCM_E_TOOLONG] > 100);

    // 2. buffer checks of single messages against brute force on small ranges
    for (int it = 0; it < 200000; ++it) {
        const uint64_t aad = 16 * (r() % 24) + (r() % 8 ? 0 : 1), in = 16 * (r() % 24), out = 16 * (r() % 24);
        const uint64_t tag = r() % 3 ? 16 * (r() % 24) + r() % 16 : 0, ok = r() % 3 ? 4 * (r() % 96) : 0;
        const uint64_t aad_len = r() % 80, len = r() % 80, tag_len = 16;
        PlanError err;
        const int got = check_buffers(aad, aad_len, in, out, len, tag, tag_len, ok, &err);
        int want = GCM_OK;
        auto bytes = [](uint64_t a, uint64_t l) {
            std::set<uint64_t> s;
            for (uint64_t k = 0; k < l; ++k)
                s.insert(a + k);
            return s;
        };
        auto meet = [&](uint64_t a, uint64_t al, uint64_t b, uint64_t bl) {
            std::set<uint64_t> x = bytes(a, al);
            for (uint64_t k = 0; k < bl; ++k)
                if (x.count(b + k))
                    return true;
            return false;
        };
        if ((len && (!in || !out)) || (aad_len && !aad))
            want = GCM_E_ARG;
        else if ((aad_len && aad % 16) || (len && (in % 16 || out % 16)))
            want = GCM_E_ARG;
        else if ((len && in != out && meet(in, len, out, len)) || meet(out, len, aad, aad_len) ||
                 (tag && meet(out, len, tag, tag_len)) || (ok && meet(out, len, ok, 4)))
            want = GCM_E_ALIAS;
        CHECK(got == want);
    }
    // ranges next to 2^64 do not wrap
    CHECK(!ranges_overlap(~0ull - 15, 16, 0, 16) && ranges_overlap(~0ull - 15, 16, ~0ull, 1));
    CHECK(!ranges_overlap(0, 16, ~0ull - 15, 16) && !ranges_overlap(5, 0, 0, 100));

    // 3. plans of valid batches: small, ragged, empty, near the length limit,
    // thousands of messages, every launch shape
    const uint32_t wave_opts[3] = {8, 12, 16};
    for (int it = 0; it < 300; ++it) {
        const uint32_t n = it % 10 == 0 ? 4096 + (uint32_t)(r() % 200) : (uint32_t)(r() % 300);
        std::vector<PlanMsg> msgs(n);
        for (uint32_t i = 0; i < n; ++i) {
            PlanMsg &m = msgs[i];
            m.op = (uint32_t)(r() % 2);
            do
                m.key_slot = (uint32_t)(r() % 64);
            while (!used[m.key_slot]);
            m.len = it == 7 && i == 0 ? (1ull << 36) - 32 : (r() % 6 ? r() % 300000 : r() % 64);
            m.aad_len = r() % 4 ? r() % 4097 : 0;
            m.in = 0x10000000ull + 4096ull * i;
            m.out = m.in + (r() % 2 ? 0 : 0x1000000000ull);
            m.aad = m.in + 0x2000000000ull;
            m.tag = 0x3000000000ull + 16ull * i;
            m.ok = 0x4000000000ull + 4ull * i;
            for (int k = 0; k < 12; ++k)
                m.iv[k] = (uint8_t)r();
        }
        const uint32_t waves = wave_opts[r() % 3];
        const uint32_t cap = 6 + (uint32_t)(r() % 15);
        BatchPlan p;
        plan_batch(msgs.data(), n, sv, waves, cap, &p);
        check_plan(msgs, p, waves, cap, sv);
    }

    // 4. the single-launch tile size
    for (int it = 0; it < 20000; ++it) {
        const uint64_t m = it < 100 ? (uint64_t)it + 1 : 1 + r() % ((1ull << 33) + 1);
        const uint64_t resident = 1 + r() % 8192;
        const uint32_t l = heuristic_log2B(m, resident);
        CHECK(l >= 6 && l <= 16);
        const uint64_t T = (m + (1ull << l) - 1) >> l;
        CHECK(l >= 8 || T <= resident);
    }
    // 5. waves per workgroup for one message: 16 once the message fills the
    // chip's wave slots, otherwise the shape whose busiest compute unit has
    // the fewest rows; never more rows there than the 16-wave shape
    {
        const auto gpc1 = [](uint32_t) { return 1u; };
        for (int it = 0; it < 20000; ++it) {
            const uint64_t m = it < 200 ? (uint64_t)it * 97 + 1 : 1 + r() % ((1ull << 27) + 1);
            const uint64_t cus = 1 + r() % 304;
            const uint32_t w = heuristic_waves(m, cus, gpc1);
            CHECK(w == 8 || w == 12 || w == 16);
            const uint32_t l16 = heuristic_log2B(m, cus * 16);
            const uint64_t t16 = (m + (1ull << l16) - 1) >> l16;
            if ((t16 + 15) / 16 >= cus)
                CHECK(w == 16);
            const uint32_t l = heuristic_log2B(m, cus * w);
            CHECK(busiest_cu_rows(m, l, w, cus, 1) <= busiest_cu_rows(m, l16, 16, cus, 1));
        }
        // the workspace bound covers every shorter message, whatever wave
        // count and tile size the planner picks for it
        for (int it = 0; it < 4000; ++it) {
            const uint64_t m = 1 + r() % ((1ull << 26) + 1);
            const uint64_t cus = 1 + r() % 304;
            const uint32_t lm = heuristic_log2B(m, cus * heuristic_waves(m, cus, gpc1));
            const uint64_t bound = tiles_bound_upto(m, (m + (1ull << lm) - 1) >> lm, cus * 16);
            for (int k = 0; k < 8; ++k) {
                const uint64_t m2 = k == 0 ? m : 1 + r() % m;
                const uint32_t w = heuristic_waves(m2, cus, gpc1);
                const uint32_t l = heuristic_log2B(m2, cus * w);
                CHECK(((m2 + (1ull << l) - 1) >> l) <= bound);
                for (uint32_t ww : {8u, 12u, 16u}) {  // any explicit wave count
                    const uint32_t l2 = heuristic_log2B(m2, cus * ww);
                    CHECK(((m2 + (1ull << l2) - 1) >> l2) <= bound);
                }
            }
        }
        // the measured cases on 256 compute units (AES-256, 2880-byte AAD: 180 blocks)
        CHECK(heuristic_waves((1ull << 16) + 181, 256, gpc1) == 8);   // 1 MiB
        CHECK(heuristic_waves((2ull << 16) + 181, 256, gpc1) == 12);  // 2 MiB
        CHECK(heuristic_waves((4ull << 16) + 181, 256, gpc1) == 12);  // 4 MiB
        CHECK(heuristic_waves((16ull << 16) + 1, 256, gpc1) == 16);   // 16 MiB
        CHECK(heuristic_waves((64ull << 16) + 1, 256, gpc1) == 16);   // 64 MiB
        CHECK(heuristic_waves(67109040ull + 181, 256, gpc1) == 16);   // 1 GiB
    }
    std::printf("plan harness: OK\n");
    return 0;
}
