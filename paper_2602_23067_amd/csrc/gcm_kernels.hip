// gcm_kernels.hip -- AES-GCM kernels for CDNA4 (gfx950, wave64).
//
// Pipeline for one message (the paper's GPU pipeline: H-power generation,
// AES-CTR, GHASH map phase, combine_partial_ghash reduce phase, validation
// gate; here CTR and the GHASH map phase are fused into one pass):
//
//   k_key_setup / k_key_tables   once per key: round keys, H, H^(2^k), and
//                                the fixed-multiplier GHASH tables.
//   k_gcm_tiles                  per wave tile: AES-CTR + XOR + store, and a
//                                per-lane Horner over the ciphertext with the
//                                fixed multiplier H^64, then a per-lane
//                                fix-up product and an XOR across the wave
//                                -> one 16-byte partial.
//   k_gcm_combine                per message: tree over the tile partials,
//                                final *H, xor E_K(J0) -> tag / accept flag.
//   k_gcm_zerofill               zero the output of every rejected message.
//
// AES-GCM-SIV (RFC 8452) reuses the same machinery: k_siv_derive builds a
// per-message key slot from the key-generating key and the nonce,
// k_siv_tiles runs POLYVAL (as GHASH over byte-reversed blocks), counter
// mode with the little-endian counter, or both fused, and k_siv_tag forms or
// checks the tag.
//
// No MFMA: the work is byte lookups and XORs, not a real-valued contraction.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "gcm_internal.h"

namespace gcm {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- small helpers

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ u32x4 xor3v(u32x4 a, u32x4 b, u32x4 c)
{
    return u32x4{xor3(a.x, b.x, c.x), xor3(a.y, b.y, c.y), xor3(a.z, b.z, c.z), xor3(a.w, b.w, c.w)};
}

__device__ __forceinline__ uint32_t rotl32(uint32_t x, int n) { return n ? (x << n) | (x >> (32 - n)) : x; }

__device__ __forceinline__ uint32_t byte_of(u32x4 a, int k)
{
    const uint32_t w = (k < 4) ? a.x : (k < 8) ? a.y : (k < 12) ? a.z : a.w;
    return (w >> (8 * (k & 3))) & 0xffu;
}

__device__ __forceinline__ uint32_t bswap32(uint32_t x) { return __builtin_bswap32(x); }

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// XOR of x over the 64 lanes of the wave, returned in every lane, without
// going through the LDS (where a shuffle would queue behind table lookups):
// DPP steps within each row of 16 lanes, then row swaps across the wave.
__device__ __forceinline__ uint32_t wave_xor_u32(uint32_t x)
{
    x ^= __builtin_amdgcn_update_dpp(0u, x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    x ^= __builtin_amdgcn_update_dpp(0u, x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    x ^= __builtin_amdgcn_update_dpp(0u, x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    x ^= __builtin_amdgcn_update_dpp(0u, x, 0x140, 0xF, 0xF, false);  // row_mirror
    const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);  // rows 0<->1, 2<->3
    x = p[0] ^ p[1];
    const auto q = __builtin_amdgcn_permlane32_swap(x, x, false, false);  // rows 0,1 <-> 2,3
    return q[0] ^ q[1];
}

// Workgroup barrier ordering LDS accesses only: a wave's outstanding global
// or spill stores do not hold the other waves at the barrier.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Read-only device data (key slots, descriptors, work lists) is read through
// the constant address space so uniform reads become scalar loads into SGPRs.
#define CONST_AS __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const CONST_AS T *cptr(const void *p)
{
    return (const CONST_AS T *)(p);
}

// whole-struct read through the constant address space (word by word)
template <typename T>
__device__ __forceinline__ T load_const(const void *p)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized struct expected");
    T v;
    uint32_t *dst = reinterpret_cast<uint32_t *>(&v);
    const CONST_AS uint32_t *src = cptr<uint32_t>(p);
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i)
        dst[i] = src[i];
    return v;
}

// Payload buffers are addressed in the global address space so that their
// loads and stores use the vector-memory counter only and never make an LDS
// wait also wait for HBM.
#define GLOBAL_AS __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL_AS T *gptr(uint64_t addr)
{
    return (GLOBAL_AS T *)(addr);
}

// ---------------------------------------------------------------- AES tables
//
// S-box from GF(2^8) antilog/log tables with generator 0x03 (FIPS-197 sec.
// 5.1.1: multiplicative inverse followed by the affine map, written here in
// its rotate form b ^ rotl(b,1) ^ rotl(b,2) ^ rotl(b,3) ^ rotl(b,4) ^ 0x63).
// TE0[x] is the MixColumns column (2s, s, s, 3s) as a memory-order word;
// TE1..TE3 are its byte rotations.

__device__ __forceinline__ uint32_t gf8_xtime(uint32_t a) { return ((a << 1) ^ ((a & 0x80u) ? 0x1bu : 0u)) & 0xffu; }

__device__ __forceinline__ uint32_t rotl8(uint32_t x, int n) { return ((x << n) | (x >> (8 - n))) & 0xffu; }

__global__ void k_init_tables(uint32_t *te0, uint32_t *sbox)
{
    __shared__ uint8_t ex[256], lg[256];
    if (threadIdx.x == 0) {
        uint32_t x = 1;
        for (int i = 0; i < 255; ++i) {
            ex[i] = (uint8_t)x;
            lg[x] = (uint8_t)i;
            x = x ^ gf8_xtime(x);  // x * 0x03
        }
        lg[0] = 0;
    }
    __syncthreads();
    const uint32_t a = threadIdx.x;
    if (a < 256) {
        const uint32_t inv = a ? ex[(255 - lg[a]) % 255] : 0u;
        const uint32_t s = inv ^ rotl8(inv, 1) ^ rotl8(inv, 2) ^ rotl8(inv, 3) ^ rotl8(inv, 4) ^ 0x63u;
        const uint32_t s2 = gf8_xtime(s), s3 = s2 ^ s;
        const uint32_t t0 = s2 | (s << 8) | (s << 16) | (s3 << 24);
        te0[a] = t0;
        sbox[a] = s;
        // TE1..TE3 after the S-box (read by the scalar unit, which has no rotate)
        te0[kTe1Off + a] = rotl32(t0, 8);
        te0[kTe1Off + 256 + a] = rotl32(t0, 16);
        te0[kTe1Off + 512 + a] = rotl32(t0, 24);
    }
}

// One AES block with a fully unrolled round count (key setup only); te0/sb point at LDS copies, rk at registers or LDS.
template <int NR>
__device__ __forceinline__ void aes_block(const uint32_t *rk, const uint32_t *te0, const uint32_t *sb,
                                          const uint32_t in[4], uint32_t out[4])
{
    uint32_t s0 = in[0] ^ rk[0], s1 = in[1] ^ rk[1], s2 = in[2] ^ rk[2], s3 = in[3] ^ rk[3];
#pragma unroll
    for (int r = 1; r < NR; ++r) {
        const uint32_t t0 = te0[s0 & 0xff] ^ rotl32(te0[(s1 >> 8) & 0xff], 8) ^ rotl32(te0[(s2 >> 16) & 0xff], 16) ^
                            rotl32(te0[s3 >> 24], 24) ^ rk[4 * r + 0];
        const uint32_t t1 = te0[s1 & 0xff] ^ rotl32(te0[(s2 >> 8) & 0xff], 8) ^ rotl32(te0[(s3 >> 16) & 0xff], 16) ^
                            rotl32(te0[s0 >> 24], 24) ^ rk[4 * r + 1];
        const uint32_t t2 = te0[s2 & 0xff] ^ rotl32(te0[(s3 >> 8) & 0xff], 8) ^ rotl32(te0[(s0 >> 16) & 0xff], 16) ^
                            rotl32(te0[s1 >> 24], 24) ^ rk[4 * r + 2];
        const uint32_t t3 = te0[s3 & 0xff] ^ rotl32(te0[(s0 >> 8) & 0xff], 8) ^ rotl32(te0[(s1 >> 16) & 0xff], 16) ^
                            rotl32(te0[s2 >> 24], 24) ^ rk[4 * r + 3];
        s0 = t0;
        s1 = t1;
        s2 = t2;
        s3 = t3;
    }
    out[0] = (sb[s0 & 0xff] | (sb[(s1 >> 8) & 0xff] << 8) | (sb[(s2 >> 16) & 0xff] << 16) | (sb[s3 >> 24] << 24)) ^
             rk[4 * NR + 0];
    out[1] = (sb[s1 & 0xff] | (sb[(s2 >> 8) & 0xff] << 8) | (sb[(s3 >> 16) & 0xff] << 16) | (sb[s0 >> 24] << 24)) ^
             rk[4 * NR + 1];
    out[2] = (sb[s2 & 0xff] | (sb[(s3 >> 8) & 0xff] << 8) | (sb[(s0 >> 16) & 0xff] << 16) | (sb[s1 >> 24] << 24)) ^
             rk[4 * NR + 2];
    out[3] = (sb[s3 & 0xff] | (sb[(s0 >> 8) & 0xff] << 8) | (sb[(s1 >> 16) & 0xff] << 16) | (sb[s2 >> 24] << 24)) ^
             rk[4 * NR + 3];
}

// ---------------------------------------------------------------- key setup
//
// FIPS-197 sec. 5.2 key expansion on memory-order words: RotWord is a right
// rotation by 8 of the little-endian word, Rcon enters byte 0.

struct KeyArg {
    uint32_t w[8];
    uint32_t len;
};

// Keys travel to the device as by-value kernel arguments, in chunks that fit
// the 4 KiB argument segment: no staging buffer, stream-ordered, capturable.
struct KeyChunk {
    KeyArg keys[kKeyChunk];
    uint64_t slots[kKeyChunk];
};
struct SlotChunk {
    uint64_t slots[kKeyChunk];
};

__device__ __forceinline__ uint32_t sub_word(uint32_t t, const uint32_t *sb)
{
    return sb[t & 0xff] | (sb[(t >> 8) & 0xff] << 8) | (sb[(t >> 16) & 0xff] << 16) | (sb[t >> 24] << 24);
}

// GF(2^128) in "polynomial order": bit i of (lo, hi) is the coefficient of
// x^i.  Memory order is the same bytes with the bits of each byte reversed.
struct P128 {
    uint64_t lo, hi;
};

__device__ __forceinline__ uint32_t brev_bytes(uint32_t x) { return __builtin_bswap32(__builtin_bitreverse32(x)); }

__device__ __forceinline__ P128 mem_to_poly(const uint32_t m[4])
{
    P128 p;
    p.lo = (uint64_t)brev_bytes(m[0]) | ((uint64_t)brev_bytes(m[1]) << 32);
    p.hi = (uint64_t)brev_bytes(m[2]) | ((uint64_t)brev_bytes(m[3]) << 32);
    return p;
}

__device__ __forceinline__ u32x4 poly_to_mem(P128 p)
{
    return u32x4{brev_bytes((uint32_t)p.lo), brev_bytes((uint32_t)(p.lo >> 32)), brev_bytes((uint32_t)p.hi),
                 brev_bytes((uint32_t)(p.hi >> 32))};
}

// spread the 32 bits of x to the even bit positions of a 64-bit word
__device__ __forceinline__ uint64_t spread32(uint32_t x)
{
    uint64_t v = x;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

// squaring is GF(2)-linear: coefficient i moves to 2i, then the upper 128
// bits fold back through x^128 = x^7 + x^2 + x + 1 (twice at most).
__device__ P128 poly_square(P128 a)
{
    const uint64_t l0 = spread32((uint32_t)a.lo), l1 = spread32((uint32_t)(a.lo >> 32));
    const uint64_t h0 = spread32((uint32_t)a.hi), h1 = spread32((uint32_t)(a.hi >> 32));
    // value = (l0, l1) + (h0, h1) * x^128
    uint64_t tlo = h0 ^ (h0 << 1) ^ (h0 << 2) ^ (h0 << 7);
    uint64_t thi = h1 ^ ((h1 << 1) | (h0 >> 63)) ^ ((h1 << 2) | (h0 >> 62)) ^ ((h1 << 7) | (h0 >> 57));
    const uint64_t ov = (h1 >> 63) ^ (h1 >> 62) ^ (h1 >> 57);
    tlo ^= ov ^ (ov << 1) ^ (ov << 2) ^ (ov << 7);
    P128 r;
    r.lo = l0 ^ tlo;
    r.hi = l1 ^ thi;
    return r;
}

// fold (l0, l1) + (h0, h1) * x^128 back below x^128 (x^128 = x^7 + x^2 + x + 1)
__device__ __forceinline__ P128 poly_reduce(uint64_t l0, uint64_t l1, uint64_t h0, uint64_t h1)
{
    uint64_t tlo = h0 ^ (h0 << 1) ^ (h0 << 2) ^ (h0 << 7);
    uint64_t thi = h1 ^ ((h1 << 1) | (h0 >> 63)) ^ ((h1 << 2) | (h0 >> 62)) ^ ((h1 << 7) | (h0 >> 57));
    const uint64_t ov = (h1 >> 63) ^ (h1 >> 62) ^ (h1 >> 57);
    tlo ^= ov ^ (ov << 1) ^ (ov << 2) ^ (ov << 7);
    P128 r;
    r.lo = l0 ^ tlo;
    r.hi = l1 ^ thi;
    return r;
}

// v * x^i for 0 <= i < 128: a 256-bit shift, then one fold
__device__ __forceinline__ P128 poly_mul_xi(P128 v, int i)
{
    uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
    if (i == 0) {
        w0 = v.lo;
        w1 = v.hi;
    } else if (i < 64) {
        w0 = v.lo << i;
        w1 = (v.hi << i) | (v.lo >> (64 - i));
        w2 = v.hi >> (64 - i);
    } else if (i == 64) {
        w1 = v.lo;
        w2 = v.hi;
    } else {
        const int j = i - 64;
        w1 = v.lo << j;
        w2 = (v.hi << j) | (v.lo >> (64 - j));
        w3 = v.hi >> (64 - j);
    }
    return poly_reduce(w0, w1, w2, w3);
}

// Frobenius tables: squaring is GF(2)-linear and does not depend on the key,
// so x -> x^(2^k) has a fixed byte-position table F_k (16 x 256 entries).
// Built once per context; key setup then forms all H^(2^k) in parallel, one
// lane per k, instead of a chain of 47 squarings.
__global__ __launch_bounds__(256) void k_frob_tables(u32x4 *frob)
{
    __shared__ u32x4 basis[128];  // (x^i)^(2^k), memory order
    const int k = blockIdx.x + 1;
    const int tid = threadIdx.x;
    if (tid < 128) {
        P128 v;
        v.lo = tid < 64 ? (1ull << tid) : 0ull;
        v.hi = tid < 64 ? 0ull : (1ull << (tid - 64));
        for (int q = 0; q < k; ++q)
            v = poly_square(v);
        basis[tid] = poly_to_mem(v);
    }
    __syncthreads();
    u32x4 *tab = frob + (uint64_t)blockIdx.x * 4096;
    for (int e = tid; e < 4096; e += 256) {
        const int j = e >> 8, b = e & 255;
        u32x4 acc = {0, 0, 0, 0};
        for (int t = 0; t < 8; ++t)
            if ((b >> t) & 1)
                acc ^= basis[8 * j + 7 - t];
        tab[e] = acc;
    }
}

// FIPS-197 key expansion with the key length fixed at compile time (fully
// unrolled, so the schedule stays in registers) into w and the slot header.
template <int NK>
__device__ __forceinline__ void expand_key(const uint32_t *kw, KeySlotHdr *hd, const uint32_t *sb, uint32_t *w)
{
    constexpr int NR = NK + 6, NW = 4 * (NR + 1);
#pragma unroll
    for (int i = 0; i < NK; ++i)
        w[i] = kw[i];
    uint32_t rcon = 1;
#pragma unroll
    for (int i = NK; i < NW; ++i) {
        uint32_t t = w[i - 1];
        if (i % NK == 0) {
            t = sub_word((t >> 8) | (t << 24), sb) ^ rcon;
            rcon = gf8_xtime(rcon);
        } else if (NK > 6 && i % NK == 4) {
            t = sub_word(t, sb);
        }
        w[i] = w[i - NK] ^ t;
    }
#pragma unroll
    for (int i = 0; i < 4 * (kMaxNr + 1); ++i)
        hd->rk[i] = i < NW ? w[i] : 0u;
    hd->nr = (uint32_t)NR;
    hd->key_len = (uint32_t)(4 * NK);
}

// key expansion, then H = E_K(0^128)
template <int NK>
__device__ __forceinline__ void expand_and_hash(const KeyArg &key, KeySlotHdr *hd, const uint32_t *te0,
                                                const uint32_t *sb, uint32_t h[4])
{
    constexpr int NR = NK + 6;
    uint32_t w[4 * (NR + 1)];
    expand_key<NK>(key.w, hd, sb, w);
    const uint32_t zero[4] = {0, 0, 0, 0};
    aes_block<NR>(w, te0, sb, zero, h);
}

// Lane k < kPowLevels of the calling wave writes H^(2^k) = F_k(H) to the
// slot header (F_0 is the identity).
__device__ __forceinline__ void write_hpow(KeySlotHdr *hd, const uint32_t *h, const u32x4 *__restrict__ frob)
{
    const int k = threadIdx.x;
    if (k < kPowLevels) {
        const u32x4 H = u32x4{h[0], h[1], h[2], h[3]};
        u32x4 r = H;
        if (k > 0) {
            const u32x4 *F = frob + (uint64_t)(k - 1) * 4096;
            r = u32x4{0, 0, 0, 0};
            for (int j = 0; j < 16; ++j)
                r ^= F[j * 256 + byte_of(H, j)];
        }
        hd->hpow[k][0] = r.x;
        hd->hpow[k][1] = r.y;
        hd->hpow[k][2] = r.z;
        hd->hpow[k][3] = r.w;
    }
}

// AES tables (TE0 and the S-box as words) from global memory into LDS,
// by one 64-thread workgroup; the caller adds the barrier.
__device__ __forceinline__ void stage_aes_tables64(uint32_t *te0, uint32_t *sb, const uint32_t *te0g,
                                                   const uint32_t *sbg)
{
    uint32_t a[4], b[4];  // all eight loads in flight before the stores
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        a[r] = te0g[threadIdx.x + 64 * r];
        b[r] = sbg[threadIdx.x + 64 * r];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        te0[threadIdx.x + 64 * r] = a[r];
        sb[threadIdx.x + 64 * r] = b[r];
    }
}

// One workgroup per key (blockIdx.x indexes `keys`/`slots`): the AES tables
// are staged in LDS, then one thread derives the round keys, H = E_K(0^128)
// and H^(2^k) by repeated squaring.
__global__ __launch_bounds__(64) void k_key_setup(KeyChunk chunk, const uint32_t *te0g, const uint32_t *sbg,
                                                  const u32x4 *__restrict__ frob)
{
    __shared__ uint32_t te0[256], sb[256];
    __shared__ uint32_t h_sh[4];
    stage_aes_tables64(te0, sb, te0g, sbg);
    lds_barrier();
    const KeyArg key = chunk.keys[blockIdx.x];
    KeySlotHdr *hd = reinterpret_cast<KeySlotHdr *>(chunk.slots[blockIdx.x]);
    if (threadIdx.x == 0) {
        uint32_t h[4];
        if (key.len == 16)
            expand_and_hash<4>(key, hd, te0, sb, h);
        else if (key.len == 24)
            expand_and_hash<6>(key, hd, te0, sb, h);
        else
            expand_and_hash<8>(key, hd, te0, sb, h);
        for (int i = 0; i < 4; ++i) {
            hd->h[i] = h[i];
            h_sh[i] = h[i];
        }
    }
    lds_barrier();
    write_hpow(hd, h_sh, frob);
}

// Fixed-multiplier tables.  Block b < kTab4Levels builds the nibble-position
// table of H^(2^b); the next sixteen build the byte-position table of
// H^(2^kStrideLevel) = H^64, the per-lane Horner multiplier of the tile
// kernel, one byte position each.
// a * b for one operand pair, all 64 lanes of the wave cooperating: lane i
// contributes the terms of bits i and i+64 of a (b * x^i, b * x^(i+64)), then
// an XOR across the wave sums them.  Every lane returns the product.
__device__ u32x4 gf_mul_wave(u32x4 a, u32x4 b)
{
    const int lane = threadIdx.x & 63;
    const uint32_t am[4] = {a.x, a.y, a.z, a.w};
    const P128 pa = mem_to_poly(am);
    const uint32_t bm[4] = {b.x, b.y, b.z, b.w};
    const P128 pb = mem_to_poly(bm);
    P128 acc;
    acc.lo = 0;
    acc.hi = 0;
    if ((pa.lo >> lane) & 1) {
        const P128 t = poly_mul_xi(pb, lane);
        acc.lo ^= t.lo;
        acc.hi ^= t.hi;
    }
    if ((pa.hi >> lane) & 1) {
        const P128 t = poly_mul_xi(pb, lane + 64);
        acc.lo ^= t.lo;
        acc.hi ^= t.hi;
    }
    const u32x4 r = poly_to_mem(acc);
    return u32x4{wave_xor_u32(r.x), wave_xor_u32(r.y), wave_xor_u32(r.z), wave_xor_u32(r.w)};
}

// Fixed-multiplier tables of one key (grid.y indexes the key).
//   blocks 0..39:   nibble-position table of H^(2^b)      (fix-ups, combine tree)
//   blocks 40..55:  byte-position table of H^64, position b - 40
//                   (per-lane Horner multiplier; one block per position, so
//                   that this table is not the launch's longest block)
//   blocks 56..119: H^e, e = 0..63, and its 4-bit window table for the lane
//                   l = 63 - e that multiplies by it in the tile fix-up
constexpr int kTab8Blocks = 16;
__global__ __launch_bounds__(256) void k_key_tables(SlotChunk chunk)
{
    __shared__ u32x4 basis[128];  // basis[i] = M * x^i, memory order
    __shared__ u32x4 m_sh;
    uint8_t *slot = reinterpret_cast<uint8_t *>(chunk.slots[blockIdx.y]);
    const KeySlotHdr *hd = reinterpret_cast<const KeySlotHdr *>(slot);
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    if (b < kTab4Levels + kTab8Blocks) {
        if (tid == 0) {
            const int lvl = b < kTab4Levels ? b : kStrideLevel;
            m_sh = u32x4{hd->hpow[lvl][0], hd->hpow[lvl][1], hd->hpow[lvl][2], hd->hpow[lvl][3]};
        }
    } else {
        // H^e as the product of H^(2^k) over the set bits of e (one wave),
        // then thread v < 16 writes (v * H^e) mod P for lane 63 - e
        if (tid < 64) {
            const int e = b - kTab4Levels - kTab8Blocks;
            u32x4 m = {0x80u, 0u, 0u, 0u};  // the field's one
            for (int k = 0; k < 6; ++k)
                if ((e >> k) & 1)
                    m = gf_mul_wave(m, u32x4{hd->hpow[k][0], hd->hpow[k][1], hd->hpow[k][2], hd->hpow[k][3]});
            if (tid < 16) {
                const uint32_t mm[4] = {m.x, m.y, m.z, m.w};
                const P128 pm = mem_to_poly(mm);
                P128 t;
                t.lo = 0;
                t.hi = 0;
                for (int i = 0; i < 4; ++i)
                    if ((tid >> i) & 1) {
                        const P128 sh = poly_mul_xi(pm, i);
                        t.lo ^= sh.lo;
                        t.hi ^= sh.hi;
                    }
                reinterpret_cast<u32x4 *>(slot + kSlotLaneWinOff)[kLanePows * tid + (63 - e)] =
                    u32x4{(uint32_t)t.lo, (uint32_t)(t.lo >> 32), (uint32_t)t.hi, (uint32_t)(t.hi >> 32)};
            }
        }
        return;
    }
    lds_barrier();
    if (tid < 128) {
        const uint32_t mm[4] = {m_sh.x, m_sh.y, m_sh.z, m_sh.w};
        basis[tid] = poly_to_mem(poly_mul_xi(mem_to_poly(mm), tid));
    }
    lds_barrier();
    if (b >= kTab4Levels) {
        // byte position k = b - kTab4Levels, value v = tid; entry-major:
        // (byte value v at position k) * M at index 16*v + k
        u32x4 *tab = reinterpret_cast<u32x4 *>(slot + kSlotTab8Off);
        const int k = b - kTab4Levels, v = tid;
        u32x4 acc = {0, 0, 0, 0};
        for (int t = 0; t < 8; ++t)
            if ((v >> t) & 1)
                acc ^= basis[8 * k + 7 - t];
        tab[16 * v + k] = acc;
        return;
    }
    u32x4 *tab = reinterpret_cast<u32x4 *>(slot + kSlotTab4Off + (uint64_t)b * kTab4Bytes);
    for (int e = tid; e < 512; e += 256) {
        const int j = e >> 4, nib = e & 15;
        const int byte = j >> 1, shift = (j & 1) ? 0 : 4;  // even j: high nibble
        u32x4 acc = {0, 0, 0, 0};
        for (int t = 0; t < 4; ++t)
            if ((nib >> t) & 1)
                acc ^= basis[8 * byte + 7 - (t + shift)];
        tab[e] = acc;
    }
}

// ---------------------------------------------------------------- GF(2^128) by table

// a * M with the nibble-position table of M (global memory, 32 gathers)
__device__ __forceinline__ u32x4 mul_tab4(u32x4 a, const u32x4 *__restrict__ tab)
{
    u32x4 r0 = {0, 0, 0, 0}, r1 = {0, 0, 0, 0};
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll 1
    for (int d = 0; d < 4; ++d) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t byte = (w[d] >> (8 * q)) & 0xffu;
            const int k = 4 * d + q;
            r0 ^= tab[(2 * k) * 16 + (byte >> 4)];
            r1 ^= tab[(2 * k + 1) * 16 + (byte & 15)];
        }
    }
    return r0 ^ r1;
}

// XOR over the 32 lanes of each half-wave (rows 0-1 and rows 2-3); every lane
// of the half-wave returns the sum.  All 64 lanes must execute it.
__device__ __forceinline__ uint32_t half_wave_xor_u32(uint32_t x)
{
    x ^= __builtin_amdgcn_update_dpp(0u, x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    x ^= __builtin_amdgcn_update_dpp(0u, x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    x ^= __builtin_amdgcn_update_dpp(0u, x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    x ^= __builtin_amdgcn_update_dpp(0u, x, 0x140, 0xF, 0xF, false);  // row_mirror
    const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);  // rows 0<->1, 2<->3
    return p[0] ^ p[1];
}

// v * M for a v that all 32 lanes of a half-wave hold, with M's
// nibble-position table: lane q (0..31) reads the entry of nibble position q
// (one lookup instead of 32), then an XOR across the half-wave.  Every lane of
// the half-wave returns the product; all 64 lanes of the wave must execute
// it (active == false: the lane's half-wave contributes zero).
__device__ __forceinline__ u32x4 mul_tab4_half(u32x4 v, const u32x4 *__restrict__ tab, uint32_t q, bool active)
{
    u32x4 t = {0, 0, 0, 0};
    if (active) {
        const uint32_t k = q >> 1;  // byte position; even q: its high nibble
        const uint32_t wsel = k >> 2;
        const uint32_t word = wsel == 0 ? v.x : wsel == 1 ? v.y : wsel == 2 ? v.z : v.w;
        const uint32_t byte = (word >> (8 * (k & 3))) & 0xffu;
        t = tab[q * 16 + ((q & 1) ? (byte & 15u) : (byte >> 4))];
    }
    return u32x4{half_wave_xor_u32(t.x), half_wave_xor_u32(t.y), half_wave_xor_u32(t.z), half_wave_xor_u32(t.w)};
}

__device__ __forceinline__ u32x4 wave_xor_reduce(u32x4 a)
{
    return u32x4{wave_xor_u32(a.x), wave_xor_u32(a.y), wave_xor_u32(a.z), wave_xor_u32(a.w)};
}

// ---------------------------------------------------------------- fused tile kernel
//
// LDS layout (144 KiB, one workgroup per CU):
//   [0, 64 KiB)        byte-position GHASH table of H^64 for the current key,
//                      entry-major: the product for byte value v at position
//                      k sits at byte 256*v + 16*k, so position k lives in
//                      bank group k (16 groups of four banks).
//   [64 KiB, 128 KiB)  AES T-tables: entry e of table t, copy c (c = 0..15)
//                      at 0x10000 + 256*e + 64*t + 4*c.
//   [128 KiB, 144 KiB) the key's lane fix-up window tables (slot layout).
//
// A wave64 ds_read_b32 takes two cycles when no two lanes of a half-wave
// share a bank; random indices into one 1 KiB table cost about three times
// that.  A ds_read_b128 serves 16 lanes per cycle, four banks each, so its
// 16 lanes must fall in 16 different bank groups.  The GHASH lookups get that
// from the schedule: in lookup j lane l reads position (j + l) & 15, with its
// accumulator held byte-rotated by l & 15 so that position is byte j of the
// rotated value; 16 consecutive lanes then read 16 different positions.
//  Here the bank of a T-table read depends only on
// (t, c): lane l uses copy c = l & 15, and lane group g = (l >> 4) & 3 keeps
// its AES state rotated left by 8g bits.  Because T_t = rotl(T_0, 8t), a
// rotated state turns "table r, byte r" into "table (r+g)&3, byte (r+g)&3",
// so in every lookup instruction the four lane groups read four different
// tables and each bank serves exactly two lanes.  One v_perm_b32 per lookup
// builds the address 0x10000 | byte << 8 | (64*table + 4*copy).

constexpr uint32_t kTeBase = 0x10000u;

struct LaneK {
    uint32_t sel[4];          // v_perm selectors: byte u_r of the state word into bits 8..15
    uint32_t off[4];          // 0x10000 | 64*u_r + 4*copy
    uint32_t rot;             // alignbit shift for rotl by 8g
    uint32_t fsel01, fsel23;  // last round: v_perm selectors of the S-box bytes
};

__device__ __forceinline__ LaneK lane_constants(int lane)
{
    LaneK k;
    const uint32_t g = (uint32_t)(lane >> 4) & 3u, copy = (uint32_t)lane & 15u;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t u = ((uint32_t)r + g) & 3u;
        k.sel[r] = 0x0c020000u | ((4u + u) << 8);
        k.off[r] = kTeBase | (u * 64u + copy * 4u);
    }
    {
        const uint32_t u0 = g & 3u, u1 = (1u + g) & 3u, u2 = (2u + g) & 3u, u3 = (3u + g) & 3u;
        // S(x) sits in byte (u+1)&3 of table u
        k.fsel01 = ((u0 + 1u) & 3u) | ((4u + ((u1 + 1u) & 3u)) << 8) | 0x0c0c0000u;
        k.fsel23 = 0x00000c0cu | (((u2 + 1u) & 3u) << 16) | ((4u + ((u3 + 1u) & 3u)) << 24);
    }
    k.rot = (32u - 8u * g) & 31u;
    return k;
}

__device__ __forceinline__ uint32_t lds_word(const uint8_t *lds, uint32_t byte_addr)
{
    return *reinterpret_cast<const uint32_t *>(lds + byte_addr);
}

__device__ __forceinline__ uint32_t rotr_by(uint32_t x, uint32_t n) { return __builtin_amdgcn_alignbit(x, x, n); }

#define B0(x) ((x) & 0xffu)
#define B1(x) (((x) >> 8) & 0xffu)
#define B2(x) (((x) >> 16) & 0xffu)
#define B3(x) ((x) >> 24)

// unrotated T_t[x] (uniform reads, used for the per-tile round-1 constants)
__device__ __forceinline__ uint32_t te_u(const uint8_t *lds, uint32_t t, uint32_t x)
{
    return lds_word(lds, kTeBase + x * 256u + t * 64u);
}

#define LK(r, w) lds_word(lds, __builtin_amdgcn_perm((w), lk.off[r], lk.sel[r]))

struct AesCtx {
    uint32_t u0, u1, u2, u3;  // round-1 columns with the 12 IV bytes folded in (unrotated, uniform)
    uint32_t rk3;             // round key 0, column 3
};

// Rounds R0..NR of AES on a lane-rotated state (rounds R0..NR-1 with the
// T-tables, the last with S-box bytes only).
template <int R0, int NR>
__device__ __forceinline__ u32x4 aes_rounds(uint32_t s0, uint32_t s1, uint32_t s2, uint32_t s3,
                                            const CONST_AS uint32_t *rk, const uint8_t *lds, const LaneK &lk)
{
    // fully unrolled: the scheduler issues each round's lookups as soon as
    // their addresses exist, across round boundaries
#pragma unroll
    for (int r = R0; r < NR; ++r) {
        const uint32_t k0 = rotr_by(rk[4 * r + 0], lk.rot), k1 = rotr_by(rk[4 * r + 1], lk.rot);
        const uint32_t k2 = rotr_by(rk[4 * r + 2], lk.rot), k3 = rotr_by(rk[4 * r + 3], lk.rot);
        const uint32_t t0 = xor3(xor3(LK(0, s0), LK(1, s1), LK(2, s2)), LK(3, s3), k0);
        const uint32_t t1 = xor3(xor3(LK(0, s1), LK(1, s2), LK(2, s3)), LK(3, s0), k1);
        const uint32_t t2 = xor3(xor3(LK(0, s2), LK(1, s3), LK(2, s0)), LK(3, s1), k2);
        const uint32_t t3 = xor3(xor3(LK(0, s3), LK(1, s0), LK(2, s1)), LK(3, s2), k3);
        s0 = t0;
        s1 = t1;
        s2 = t2;
        s3 = t3;
    }
    // last round: the round tables hold S(x) in byte (u+1)&3; two v_perm
    // pick the four S-box bytes into their unrotated positions, so the key
    // is added unrotated and the result needs no rotation back
    const uint32_t o0 = __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_perm(LK(1, s1), LK(0, s0), lk.fsel01),
                                                    __builtin_amdgcn_perm(LK(3, s3), LK(2, s2), lk.fsel23), rk[4 * NR + 0], 0x56);
    const uint32_t o1 = __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_perm(LK(1, s2), LK(0, s1), lk.fsel01),
                                                    __builtin_amdgcn_perm(LK(3, s0), LK(2, s3), lk.fsel23), rk[4 * NR + 1], 0x56);
    const uint32_t o2 = __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_perm(LK(1, s3), LK(0, s2), lk.fsel01),
                                                    __builtin_amdgcn_perm(LK(3, s1), LK(2, s0), lk.fsel23), rk[4 * NR + 2], 0x56);
    const uint32_t o3 = __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_perm(LK(1, s0), LK(0, s3), lk.fsel01),
                                                    __builtin_amdgcn_perm(LK(3, s2), LK(2, s1), lk.fsel23), rk[4 * NR + 3], 0x56);
    return u32x4{o0, o1, o2, o3};
}

// Keystream block for counter value `ctr` (big-endian in bytes 12..15).
// Only column 3 of the counter block varies, so round 1 needs four table
// lookups instead of sixteen (counter-mode caching).
template <int NR>
__device__ __forceinline__ u32x4 aes_ctr(uint32_t ctr, const AesCtx &c, const CONST_AS uint32_t *rk,
                                         const uint8_t *lds, const LaneK &lk)
{
    const uint32_t v = bswap32(ctr) ^ c.rk3;
    const uint32_t w3 = rotr_by(v, lk.rot);  // rotl(v, 8g)
    const uint32_t s0 = rotr_by(c.u0, lk.rot) ^ LK(3, w3);
    const uint32_t s1 = rotr_by(c.u1, lk.rot) ^ LK(2, w3);
    const uint32_t s2 = rotr_by(c.u2, lk.rot) ^ LK(1, w3);
    const uint32_t s3 = rotr_by(c.u3, lk.rot) ^ LK(0, w3);
    return aes_rounds<2, NR>(s0, s1, s2, s3, rk, lds, lk);
}

// Counter-mode caching through round 2.  With counter bytes 12..14 fixed,
// round 1 leaves state columns 1..3 fixed and only column 0 depends on the
// low counter byte; every round-2 output column then takes exactly one
// table entry indexed by a byte of that column, XOR a word that depends only
// on the upper 24 counter bits.  Ctr2 holds those four words (unrotated).
struct Ctr2 {
    uint32_t v0, v1, v2, v3;
};

// T_t[x] read through the scalar cache (uniform x): TE0 at word 0, TE1..TE3
// from word kTe1Off of the table block
__device__ __forceinline__ uint32_t te_s(const CONST_AS uint32_t *te, int t, uint32_t x)
{
    return t == 0 ? te[x] : te[kTe1Off + 256 * (t - 1) + x];
}

// the four round-2 words for upper counter bits `hi` (wave-uniform)
__device__ __forceinline__ Ctr2 ctr_round2(uint32_t hi, const AesCtx &c, const CONST_AS uint32_t *rk,
                                           const CONST_AS uint32_t *te)
{
    const uint32_t v = bswap32(hi << 8) ^ c.rk3;  // column 3 of the first state (byte 3 unused)
    const uint32_t u1 = c.u1 ^ te_s(te, 2, B2(v));
    const uint32_t u2 = c.u2 ^ te_s(te, 1, B1(v));
    const uint32_t u3 = c.u3 ^ te_s(te, 0, B0(v));
    Ctr2 q;
    q.v0 = te_s(te, 1, B1(u1)) ^ te_s(te, 2, B2(u2)) ^ te_s(te, 3, B3(u3)) ^ rk[8];
    q.v1 = te_s(te, 0, B0(u1)) ^ te_s(te, 1, B1(u2)) ^ te_s(te, 2, B2(u3)) ^ rk[9];
    q.v2 = te_s(te, 0, B0(u2)) ^ te_s(te, 1, B1(u3)) ^ te_s(te, 3, B3(u1)) ^ rk[10];
    q.v3 = te_s(te, 0, B0(u3)) ^ te_s(te, 2, B2(u1)) ^ te_s(te, 3, B3(u2)) ^ rk[11];
    return q;
}

// Keystream block for `ctr` whose upper 24 bits match `q`: one lookup in
// round 1 and four in round 2 instead of four and sixteen.
template <int NR>
__device__ __forceinline__ u32x4 aes_ctr2(uint32_t ctr, const Ctr2 &q, const AesCtx &c,
                                          const CONST_AS uint32_t *rk, const uint8_t *lds, const LaneK &lk)
{
    const uint32_t w3 = rotr_by((ctr << 24) ^ c.rk3, lk.rot);  // byte 3: low counter byte ^ key
    const uint32_t x0 = rotr_by(c.u0, lk.rot) ^ LK(3, w3);      // round-1 column 0
    const uint32_t s0 = rotr_by(q.v0, lk.rot) ^ LK(0, x0);
    const uint32_t s1 = rotr_by(q.v1, lk.rot) ^ LK(3, x0);
    const uint32_t s2 = rotr_by(q.v2, lk.rot) ^ LK(2, x0);
    const uint32_t s3 = rotr_by(q.v3, lk.rot) ^ LK(1, x0);
    return aes_rounds<3, NR>(s0, s1, s2, s3, rk, lds, lk);
}

// Per-lane constants of the GHASH lookup schedule (q = lane & 15):
// pos[m] byte t = 16 * ((4m + t + q) & 15), the bank-group offset of lookup
// j = 4m + t; the accumulator is rotated by q bytes as a dword rotation by
// q >> 2 (two conditional swaps) and a byte shift of 8 * (q & 3) bits.
struct GhK {
    uint32_t pos[4];
    uint32_t sh;
    bool s2, s1;
};

__device__ __forceinline__ GhK gh_constants(int lane)
{
    GhK g;
    const uint32_t q = (uint32_t)lane & 15u;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        uint32_t w = 0;
        for (int t = 0; t < 4; ++t)
            w |= (((4u * m + t + q) & 15u) << 4) << (8 * t);
        g.pos[m] = w;
    }
    g.sh = 8u * (q & 3u);
    g.s2 = (q & 8u) != 0;
    g.s1 = (q & 4u) != 0;
    return g;
}

// byte i of the result is byte (i + q) & 15 of a
__device__ __forceinline__ u32x4 rot_bytes_lane(u32x4 a, const GhK &g)
{
    const u32x4 c = g.s2 ? u32x4{a.z, a.w, a.x, a.y} : a;
    const u32x4 b = g.s1 ? u32x4{c.y, c.z, c.w, c.x} : c;
    return u32x4{__builtin_amdgcn_alignbit(b.y, b.x, g.sh), __builtin_amdgcn_alignbit(b.z, b.y, g.sh),
                 __builtin_amdgcn_alignbit(b.w, b.z, g.sh), __builtin_amdgcn_alignbit(b.x, b.w, g.sh)};
}

// a * H^64 + x with the entry-major byte-position table at LDS offset 0
// (16 lookups of 16 bytes, conflict-free across each 16-lane group)
__device__ __forceinline__ u32x4 ghash_mul8(u32x4 a, u32x4 x, const uint8_t *__restrict__ lds, const GhK &g)
{
    const u32x4 r = rot_bytes_lane(a, g);
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
    u32x4 acc = x;
    // two halves of eight lookups, so at most 32 result registers are live
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        u32x4 e[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = 8 * h + q;
            // address = 256 * (byte j of r) + 16 * position
            const uint32_t sel = 0x0c0c0000u | ((4u + (uint32_t)(j & 3)) << 8) | (uint32_t)(j & 3);
            const uint32_t addr = __builtin_amdgcn_perm(w[j >> 2], g.pos[j >> 2], sel);
            e[q] = *reinterpret_cast<const u32x4 *>(lds + addr);
        }
        acc = xor3v(xor3v(e[0], e[1], e[2]), xor3v(e[3], e[4], e[5]), xor3v(e[6], e[7], acc));
    }
    return acc;
}

// zero-padded load of block `blk` of a buffer of `total` bytes
__device__ __forceinline__ u32x4 load_block_partial(const uint8_t *p, uint64_t blk, uint64_t total)
{
    const uint64_t off = blk * 16;
    if (off + 16 <= total)
        return *reinterpret_cast<const u32x4 *>(p + off);
    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
    for (uint64_t k = off; k < total; ++k) {
        const uint32_t b = (uint32_t)p[k] << (8 * ((k - off) & 3));
        const uint64_t d = (k - off) >> 2;
        w0 |= d == 0 ? b : 0u;
        w1 |= d == 1 ? b : 0u;
        w2 |= d == 2 ? b : 0u;
        w3 |= d == 3 ? b : 0u;
    }
    return u32x4{w0, w1, w2, w3};
}

__device__ __forceinline__ uint32_t keep_bytes(uint32_t w, int nb)  // keep the low nb bytes (nb may be <=0 or >=4)
{
    return nb <= 0 ? 0u : nb >= 4 ? w : (w & ((1u << (8 * nb)) - 1u));
}

__device__ __forceinline__ u32x4 mask_block(u32x4 v, uint64_t blk, uint64_t total)
{
    const uint64_t off = blk * 16;
    if (off + 16 <= total)
        return v;
    const int nb = (int)(total - off);  // 1..15 valid bytes
    return u32x4{keep_bytes(v.x, nb), keep_bytes(v.y, nb - 4), keep_bytes(v.z, nb - 8), keep_bytes(v.w, nb - 12)};
}

__device__ __forceinline__ void store_block_partial(uint8_t *p, uint64_t blk, uint64_t total, u32x4 v)
{
    const uint64_t off = blk * 16;
    if (off + 16 <= total) {
        *reinterpret_cast<u32x4 *>(p + off) = v;
        return;
    }
    for (uint64_t k = off; k < total; ++k) {
        const uint64_t d = (k - off) >> 2;
        const uint32_t w = d == 0 ? v.x : d == 1 ? v.y : d == 2 ? v.z : v.w;
        p[k] = (uint8_t)(w >> (8 * ((k - off) & 3)));
    }
}

// LDS byte offset of the lane fix-up window table (after the GHASH table and
// the T-tables)
constexpr uint32_t kWinBase = 0x20000u;

// a * c_l for this lane's fixed multiplier c_l = H^(63 - lane), through its
// 4-bit window table in LDS (entry (v, l) = (v * c_l) mod P at
// kWinBase + 16 * (64 v + l)): a comb over the eight nibble positions of the
// four words of a, 256-bit accumulate with word-aligned XORs, one fold at the
// end.  32 conflict-free ds_read_b128 (16 consecutive lanes read 16
// different bank groups) and about 300 VALU instructions.
__device__ __forceinline__ u32x4 gf_mul_lanewin(u32x4 a, const uint8_t *__restrict__ lds, int lane)
{
    const uint32_t am[4] = {a.x, a.y, a.z, a.w};
    const P128 pa = mem_to_poly(am);
    const uint32_t aw[4] = {(uint32_t)pa.lo, (uint32_t)(pa.lo >> 32), (uint32_t)pa.hi, (uint32_t)(pa.hi >> 32)};
    const uint8_t *win = lds + kWinBase + 16u * (uint32_t)lane;
    uint32_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 7; q >= 0; --q) {
#pragma unroll
        for (int k = 7; k > 0; --k)
            acc[k] = __builtin_amdgcn_alignbit(acc[k], acc[k - 1], 28);  // acc <<= 4
        acc[0] <<= 4;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint32_t v = (aw[w] >> (4 * q)) & 15u;
            const u32x4 t = *reinterpret_cast<const u32x4 *>(win + 1024u * v);
            acc[w] ^= t.x;
            acc[w + 1] ^= t.y;
            acc[w + 2] ^= t.z;
            acc[w + 3] ^= t.w;
        }
    }
    const P128 r = poly_reduce((uint64_t)acc[0] | ((uint64_t)acc[1] << 32), (uint64_t)acc[2] | ((uint64_t)acc[3] << 32),
                               (uint64_t)acc[4] | ((uint64_t)acc[5] << 32), (uint64_t)acc[6] | ((uint64_t)acc[7] << 32));
    return poly_to_mem(r);
}

// One wave processes wave tile t of message d: rows of 64 consecutive
// blocks, lane l on block 64*r + l, so every load/store instruction moves one
// contiguous KiB.  a_l = sum_r X_(64r+l) * (H^64)^(R-1-r) by Horner; then
// p_t = sum_l a_l * H^(63-l) is formed by exponent-bit fix-ups and an XOR
// across the wave.  With GH false the tile is counter mode only (no GHASH,
// no partial).  AADROWS adds a GHASH-only pass over rows of whole AAD blocks,
// J0DEV reads J0 from device memory (IVs other than 96 bits) instead of
// forming IV || 0^31 || 1.  A streamed segment's counters start d.ctr_off
// blocks after J0 + 1 in every variant.  Both options cost the main loop its
// batching of LDS reads (a run-time counter base, or the extra loop, leaves
// it fewer registers), so each is compiled only into kernel variants of its
// own.
template <int NR, bool GH, bool AADROWS, bool J0DEV>
__device__ void wave_tile(const MsgDesc &d, uint64_t t, const uint8_t *__restrict__ lds, const LaneK &lk,
                          const GhK &gk, const uint32_t *__restrict__ te0g, u32x4 *__restrict__ partials)
{
    const int lane = threadIdx.x & 63;
    const CONST_AS uint32_t *te = cptr<uint32_t>(te0g);
    const CONST_AS uint32_t *rk_base = cptr<uint32_t>(reinterpret_cast<const void *>(d.slot));
    const CONST_AS uint32_t *rk = rk_base;
    // J0 = IV || 0^31 || 1, or a J0 computed from a longer or shorter IV;
    // E_K(J0) uses J0's own counter value cj0, data block j (of a streamed
    // segment that follows d.ctr_off earlier blocks) counter value c1 + j
    uint32_t iv0 = d.iv[0], iv1 = d.iv[1], iv2 = d.iv[2], cj0 = 1u;
    if (J0DEV) {
        const CONST_AS uint32_t *jw = cptr<uint32_t>(reinterpret_cast<const void *>(d.j0));
        iv0 = jw[0];
        iv1 = jw[1];
        iv2 = jw[2];
        cj0 = bswap32(jw[3]);
    }
    const uint32_t c1 = cj0 + 1u + d.ctr_off;
    AesCtx c;
    {
        const uint32_t s0 = iv0 ^ rk[0], s1 = iv1 ^ rk[1], s2 = iv2 ^ rk[2];
        c.u0 = uniform(te_u(lds, 0, B0(s0)) ^ te_u(lds, 1, B1(s1)) ^ te_u(lds, 2, B2(s2)) ^ rk[4]);
        c.u1 = uniform(te_u(lds, 0, B0(s1)) ^ te_u(lds, 1, B1(s2)) ^ te_u(lds, 3, B3(s0)) ^ rk[5]);
        c.u2 = uniform(te_u(lds, 0, B0(s2)) ^ te_u(lds, 2, B2(s0)) ^ te_u(lds, 3, B3(s1)) ^ rk[6]);
        c.u3 = uniform(te_u(lds, 1, B1(s0)) ^ te_u(lds, 2, B2(s1)) ^ te_u(lds, 3, B3(s2)) ^ rk[7]);
        c.rk3 = rk[3];
    }

    if (GH && t == 0) {
        // E_K(J0) is the keystream block of counter value 1; the wave that owns
        // tile 0 leaves it after the message's partials for the combine
        const u32x4 ek = aes_ctr<NR>(cj0, c, rk, lds, lk);
        if (lane == 0)
            partials[d.tile_base + d.n_tiles] = ek;
    }

    const uint64_t B = 1ull << d.log2B;
    const uint32_t R = (uint32_t)(B >> 6);
    const int64_t vbase = (int64_t)(t * B) - (int64_t)d.z;  // GHASH index of lane 0, row 0
    const uint32_t r0 = vbase < 0 ? (uint32_t)((uint64_t)(-vbase) >> 6) : 0u;
    const int64_t na = (int64_t)d.na;
    const int64_t nafull = (int64_t)(d.aad_len >> 4);
    const int64_t nfull = (int64_t)(d.len >> 4);
    const int64_t ndat = (int64_t)d.n;
    const bool enc = d.op == 0;
    const uint8_t *__restrict__ in = reinterpret_cast<const uint8_t *>(d.in);
    uint8_t *__restrict__ out = reinterpret_cast<uint8_t *>(d.out);
    const GLOBAL_AS u32x4 *in_g = gptr<const u32x4>(d.in);
    GLOBAL_AS u32x4 *out_g = gptr<u32x4>(d.out);
    const GLOBAL_AS u32x4 *aad_g = gptr<const u32x4>(d.aad);

    u32x4 a = {0, 0, 0, 0};
    // boundary row: zero padding, AAD, partial blocks or the length block
    auto boundary_row = [&](int64_t v0) {
        const int64_t v = v0 + lane;
        const uint64_t j = (uint64_t)(v - na);
        const u32x4 ks = aes_ctr<NR>((uint32_t)j + c1, c, rk, lds, lk);
        u32x4 X = {0, 0, 0, 0};
        if (GH && v >= 0 && v < na) {
            X = load_block_partial(reinterpret_cast<const uint8_t *>(d.aad), (uint64_t)v, d.aad_len);
        } else if (v >= na && v < na + ndat) {
            const u32x4 x = load_block_partial(in, j, d.len);
            const u32x4 o = x ^ ks;
            store_block_partial(out, j, d.len, o);
            X = enc ? mask_block(o, j, d.len) : x;
        } else if (GH && v == na + ndat) {
            const uint64_t abits = d.aad_len * 8, cbits = d.len * 8;
            X = u32x4{bswap32((uint32_t)(abits >> 32)), bswap32((uint32_t)abits), bswap32((uint32_t)(cbits >> 32)),
                      bswap32((uint32_t)cbits)};
        }
        if (GH)
            a = ghash_mul8(a, X, lds, gk);
    };

    uint32_t r = r0;
    if (GH && AADROWS) {
        // Rows of whole AAD blocks, [ra0, ra1), take the GHASH step only.  They
        // follow at most one boundary row (zero prefix and AAD start) and
        // precede every data row, so they are peeled off before the main loop.
        const int64_t vb = vbase;
        const int64_t rz = vb >= 0 ? 0 : (-vb + 63) >> 6;        // first row with v0 >= 0
        const int64_t fit = nafull - vb;                          // rows r with v0 + 64 <= nafull: r < fit / 64
        int64_t ra0 = rz > (int64_t)r0 ? rz : (int64_t)r0;
        int64_t ra1 = fit >= 64 ? fit >> 6 : 0;
        ra1 = ra1 < (int64_t)R ? ra1 : (int64_t)R;
        if (ra1 > ra0) {
            for (; (int64_t)r < ra0; ++r)
                boundary_row(vb + 64 * (int64_t)r);
            for (; (int64_t)r < ra1; ++r)
                a = ghash_mul8(a, aad_g[(uint64_t)(vb + 64 * (int64_t)r) + (uint64_t)lane], lds, gk);
        }
    }

    // Rows [fa, fb) hold 64 whole data blocks each and take the fast path
    // (v0 >= na and v0 + 64 <= na + nfull).  The range is computed once, so
    // the row loop keeps only scalar 32-bit bookkeeping and one uniform row
    // address.
    int64_t rf0, rf1;
    {
        const int64_t lo = na - vbase;                // 64 r >= lo
        const int64_t hi = na + nfull - vbase - 64;   // 64 r <= hi
        rf0 = lo <= 0 ? 0 : (lo + 63) >> 6;
        rf1 = hi < 0 ? 0 : (hi >> 6) + 1;
    }
    const uint32_t fa = (uint32_t)(rf0 > (int64_t)r ? (rf0 < (int64_t)R ? rf0 : (int64_t)R) : (int64_t)r);
    const uint32_t fb = (uint32_t)(rf1 > (int64_t)fa ? (rf1 < (int64_t)R ? rf1 : (int64_t)R) : (int64_t)fa);
    for (; r < fa; ++r)
        boundary_row(vbase + 64 * (int64_t)r);

    uint32_t hc = 0xffffffffu;  // upper counter bits `cur` belongs to (none yet)
    Ctr2 cur = {0, 0, 0, 0};
    const uint32_t loff = 16u * (uint32_t)lane;  // this lane's byte offset in a row
    // Issue priority falls as the wave gets through its rows (at 5/8, 3/4
    // and 7/8 of them), so that waves the arbiter has left behind catch up
    // and the compute unit stays full until its last tile ends.
    const uint32_t span = fb > r ? fb - r : 0u;
    const uint32_t q1 = r + 5 * (span / 8), q2 = r + 3 * (span / 4), q3 = r + 7 * (span / 8);
    __builtin_amdgcn_s_setprio(3);
    for (; r < fb; ++r) {
        if (r == q1)
            __builtin_amdgcn_s_setprio(2);
        if (r == q2)
            __builtin_amdgcn_s_setprio(1);
        if (r == q3)
            __builtin_amdgcn_s_setprio(0);
        // re-read the round keys with scalar loads each row instead of holding
        // 4*(Nr+1) of them (or their lane-rotated copies) in registers
        rk = rk_base;
        asm volatile("" : "+s"(rk));
        const uint64_t j0 = (uint64_t)(vbase + 64 * (int64_t)r - na);  // first data block of the row (uniform)
        const GLOBAL_AS uint8_t *src = reinterpret_cast<const GLOBAL_AS uint8_t *>(in_g + j0);
        GLOBAL_AS uint8_t *dst = reinterpret_cast<GLOBAL_AS uint8_t *>(out_g + j0);
        const u32x4 x = *reinterpret_cast<const GLOBAL_AS u32x4 *>(src + loff);
        // counters of this row: base + lane (mod 2^32); the upper 24 bits
        // change at most once inside a row, and then by one
        const uint32_t base = (uint32_t)j0 + c1;
        const uint32_t h = base >> 8;
        if (h != hc) {
            cur = ctr_round2(h, c, rk, te);
            hc = h;
        }
        const uint32_t ctr = base + (uint32_t)lane;
        Ctr2 q = cur;
        if ((base & 255u) > 192u) {
            const uint32_t h1 = (h + 1u) & 0xffffffu;
            const Ctr2 nxt = ctr_round2(h1, c, rk, te);
            // this lane's low counter byte wrapped inside the row; compared in
            // the top byte, as aes_ctr2 uses it, so that no per-lane constant
            // stays live across the loop
            const bool up = (ctr << 24) < (base << 24);
            q = Ctr2{up ? nxt.v0 : cur.v0, up ? nxt.v1 : cur.v1, up ? nxt.v2 : cur.v2, up ? nxt.v3 : cur.v3};
            cur = nxt;
            hc = h1;
        }
        const u32x4 ks = aes_ctr2<NR>(ctr, q, c, rk, lds, lk);
        const u32x4 o = x ^ ks;
        __builtin_nontemporal_store(o, reinterpret_cast<GLOBAL_AS u32x4 *>(dst + loff));
        if (GH)
            a = ghash_mul8(a, enc ? o : x, lds, gk);
    }
    for (; r < R; ++r)
        boundary_row(vbase + 64 * (int64_t)r);
    if (!GH)
        return;

    // fix-up: a * H^(63 - lane) through the lane's window table in LDS
    a = gf_mul_lanewin(a, lds, lane);
    a = wave_xor_reduce(a);
    if (lane == 0)
        partials[d.tile_base + t] = a;
}

// T-tables into LDS: dword 16384 + 64*e + 16*t + c holds rotl(TE0[e], 8t)
// for copy c = 0..15; thread q of NT writes the 16 copies of entries
// (e, t) = (q >> 2, q & 3), q + NT, ..., with all loads issued first.  The
// caller adds the barrier.
template <int NT>
__device__ __forceinline__ void stage_ttables(u32x4 *lds_v, const uint32_t *__restrict__ te0g)
{
    constexpr int kPer = (1024 + NT - 1) / NT;
    uint32_t v[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int q = (int)threadIdx.x + r * NT;
        v[r] = q < 1024 ? rotl32(te0g[q >> 2], 8 * (q & 3)) : 0u;
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int q = (int)threadIdx.x + r * NT;
        if (q >= 1024)
            break;
        u32x4 *dst = lds_v + 4096 + 4 * q;  // dword 16384 + 64*(q >> 2) + 16*(q & 3)
        const u32x4 x = {v[r], v[r], v[r], v[r]};
        dst[0] = x;
        dst[1] = x;
        dst[2] = x;
        dst[3] = x;
    }
}

// The key's GHASH table of H^64 (64 KiB, LDS bytes [0, 64 KiB)) and its
// lane fix-up windows (16 KiB, LDS bytes [128 KiB, 144 KiB)) from the key
// slot, all of a thread's loads issued before its stores.  In a workgroup
// of 16 waves (128 VGPRs a thread) the thread index goes through an empty
// asm so that the addresses are formed here: a caller that stages inside a
// loop would otherwise hold them across the whole loop, spilled, and each
// reload would wait for the previous load.  With fewer waves they stay in
// registers.  The caller adds the barriers.
template <int NT>
__device__ __forceinline__ void stage_key_tables(u32x4 *lds_v, uint64_t slot)
{
    const GLOBAL_AS u32x4 *tab = gptr<const u32x4>(slot + kSlotTab8Off);
    const GLOBAL_AS u32x4 *win = gptr<const u32x4>(slot + kSlotLaneWinOff);
    constexpr uint32_t kTab = 4096, kWin = 1024;
    constexpr int kPerT = (int)((kTab + NT - 1) / NT), kPerW = (int)((kWin + NT - 1) / NT);
    uint32_t tid = threadIdx.x;
    if (NT >= 1024)
        asm volatile("" : "+v"(tid));
    u32x4 a[kPerT], b[kPerW];
#pragma unroll
    for (int r = 0; r < kPerT; ++r) {
        const uint32_t q = tid + (uint32_t)(r * NT);
        if (kTab % NT == 0 || q < kTab)
            a[r] = tab[q];
    }
#pragma unroll
    for (int r = 0; r < kPerW; ++r) {
        const uint32_t q = tid + (uint32_t)(r * NT);
        if (kWin % NT == 0 || q < kWin)
            b[r] = win[q];
    }
#pragma unroll
    for (int r = 0; r < kPerT; ++r) {
        const uint32_t q = tid + (uint32_t)(r * NT);
        if (kTab % NT == 0 || q < kTab)
            lds_v[q] = a[r];
    }
#pragma unroll
    for (int r = 0; r < kPerW; ++r) {
        const uint32_t q = tid + (uint32_t)(r * NT);
        if (kWin % NT == 0 || q < kWin)
            lds_v[8192 + q] = b[r];
    }
}

// Kernel variants (each a kernel of its own, so that the extra work of one
// leaves the register allocation of the others alone): GCM; counter mode
// only; GCM with the GHASH-only pass over whole AAD rows, for single messages
// whose AAD spans at least 64 rows of blocks; GCM with J0 read from device
// memory, for single messages whose IV is not 96 bits (AAD rows then take the
// boundary path).
constexpr int kModeGcm = 0, kModeCtr = 1, kModeGcmAad = 2, kModeGcmJ0 = 3;
constexpr uint64_t kAadRowsMinBytes = 64 * 64 * 16;

template <int WAVES, bool BATCH, int MODE>
__global__ __launch_bounds__(WAVES * 64) void k_gcm_tiles(const MsgDesc *__restrict__ descs,
                                                          const WorkItem *__restrict__ items, uint32_t n_items,
                                                          MsgDesc single, const uint32_t *__restrict__ te0g,
                                                          u32x4 *__restrict__ partials, uint32_t *counters)
{
    constexpr bool GH = MODE != kModeCtr;
    constexpr bool AADROWS = MODE == kModeGcmAad;
    constexpr bool J0DEV = MODE == kModeGcmJ0;
    __shared__ u32x4 lds_v[9216];  // 144 KiB: GHASH table, replicated T-tables, fix-up windows
    const uint8_t *lds = reinterpret_cast<const uint8_t *>(lds_v);

    if (GH && blockIdx.x == 0 && threadIdx.x == 0)
        counters[0] = 0;  // reject count for this launch (read by the zero-fill)

    // A single message's key tables are staged here with the T-tables, while
    // little else is live; a batch stages the tables of each work item's key
    // in the loop (the first item's staging starts and ends with a barrier,
    // which also publishes the T-tables).
    stage_ttables<WAVES * 64>(lds_v, te0g);
    uint64_t cur_slot = 0;
    if (GH && !BATCH) {
        stage_key_tables<WAVES * 64>(lds_v, single.slot);
        cur_slot = single.slot;
    }
    if (!GH || !BATCH)
        lds_barrier();
    const LaneK lk = lane_constants(threadIdx.x & 63);
    const GhK gk = gh_constants(threadIdx.x & 63);

    const int wave = (int)uniform(threadIdx.x >> 6);  // wave-uniform: row bookkeeping stays scalar
    for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        MsgDesc d;
        uint32_t first;
        if (BATCH) {
            const WorkItem w = load_const<WorkItem>(items + it);
            d = load_const<MsgDesc>(descs + w.msg);
            first = w.first_tile;
        } else {
            // the descriptor's words pass through an empty asm on every item,
            // so that nothing derived from them is hoisted out of this loop
            // and held (or spilled) across all of it
            d = single;
            uint32_t *dw = reinterpret_cast<uint32_t *>(&d);
#pragma unroll
            for (unsigned i = 0; i < sizeof(MsgDesc) / 4; ++i)
                asm volatile("" : "+s"(dw[i]));
            first = (uint32_t)d.tile_lo + it * WAVES;
        }
        if (GH && BATCH && d.slot != cur_slot) {
            lds_barrier();
            stage_key_tables<WAVES * 64>(lds_v, d.slot);
            cur_slot = d.slot;
            lds_barrier();
        }
        const uint64_t t = (uint64_t)first + (uint64_t)wave;
        if (t < d.tile_hi) {
            if (d.nr == 10)
                wave_tile<10, GH, AADROWS, J0DEV>(d, t, lds, lk, gk, te0g, partials);
            else if (d.nr == 12)
                wave_tile<12, GH, AADROWS, J0DEV>(d, t, lds, lk, gk, te0g, partials);
            else
                wave_tile<14, GH, AADROWS, J0DEV>(d, t, lds, lk, gk, te0g, partials);
        }
    }
}

// ---------------------------------------------------------------- combine + tag

constexpr int kCombineThreads = 1024;
constexpr int kCombineLog2 = 10;

// S = sum_t p_t * H^((T-1-t)*B + 1); tag = S xor E_K(J0).  Thread i runs a
// Horner over partials i, i+1024, ... with the fixed multiplier H^(1024*B);
// its value then needs the weight H^((T-1-t_last)*B), and with N = 2^k >=
// min(T, 1024) leaves and r = T mod N that weight is H^((N-1-j)*B) for leaf
// j = (i - r) mod N.  A tree of fan-in F = 2^LOGF over the leaves closes the
// sum: a node whose F children each span w leaves is the Horner
// (((c_0*H^(B*w) ^ c_1)*H^(B*w) ^ c_2) ...) ^ c_(F-1), so the levels use the
// tables of H^(B*2^(LOGF*lev)) and the tree has ceil(k / LOGF) levels and
// N - 1 products in all (F = 2 is the binary tree L*H^(B*2^lev) ^ R); one
// more *H accounts for GHASH's final multiplication.  The nibble tables this needs
// (at most 12 of 8 KiB) are staged in LDS first, so every multiply is 32 LDS
// reads.  E_K(J0) was left by the tile kernel right after the message's T
// partials.
template <bool BATCH, int LOGF>
__global__ __launch_bounds__(kCombineThreads) void k_gcm_combine(const MsgDesc *__restrict__ descs, MsgDesc single,
                                                                 const u32x4 *__restrict__ partials,
                                                                 uint32_t *counters)
{
    __shared__ u32x4 tabs[kCombineLog2 + 2][512];  // [0]: H; [1+k]: H^(B*2^k), k = 0..10
    __shared__ u32x4 leaf[kCombineThreads];
    const MsgDesc d = BATCH ? load_const<MsgDesc>(descs + blockIdx.x) : single;
    const uint32_t i = threadIdx.x;
    const uint64_t T = d.n_tiles;

    // the first eight partials of this thread, loaded ahead of the table staging
    u32x4 pv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint64_t t = (uint64_t)i + (uint64_t)q * kCombineThreads;
        pv[q] = t < T ? partials[d.tile_base + t] : u32x4{0, 0, 0, 0};
    }

    // exponent bits needed for T-1-t_last < min(T, 1024), and whether any
    // thread owns more than one partial
    const uint64_t span = T < (uint64_t)kCombineThreads ? T : (uint64_t)kCombineThreads;
    int nbits = 0;
    while (nbits < kCombineLog2 && (1ull << nbits) < span)
        ++nbits;
    const bool horner = T > (uint64_t)kCombineThreads;
    {
        // all of a thread's table loads are issued before any is stored
        const GLOBAL_AS u32x4 *g = gptr<const u32x4>(d.slot + kSlotTab4Off);
        const int ntab = 1 + (horner ? kCombineLog2 + 1 : nbits);
        constexpr int kPer = ((kCombineLog2 + 2) * 512 + kCombineThreads - 1) / kCombineThreads;
        u32x4 st[kPer];
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int e = (int)i + r * kCombineThreads;
            const int tix = e >> 9;
            const int lvl = tix == 0 ? 0 : (int)d.log2B + tix - 1;
            if (e < ntab * 512)
                st[r] = g[(uint64_t)lvl * 512 + (e & 511)];
        }
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int e = (int)i + r * kCombineThreads;
            if (e < ntab * 512)
                tabs[e >> 9][e & 511] = st[r];
        }
    }
    lds_barrier();

    u32x4 acc = {0, 0, 0, 0};
    if (i < T) {
        for (uint64_t t0 = i; t0 < T; t0 += 8 * (uint64_t)kCombineThreads) {
            if (t0 != i) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint64_t t = t0 + (uint64_t)q * kCombineThreads;
                    pv[q] = t < T ? partials[d.tile_base + t] : u32x4{0, 0, 0, 0};
                }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint64_t t = t0 + (uint64_t)q * kCombineThreads;
                if (t < T)
                    acc = (horner ? mul_tab4(acc, tabs[1 + kCombineLog2]) : acc) ^ pv[q];
            }
        }
    }
    // leaves: thread i (< N) at (i - r) mod N; threads without partials hold 0
    const uint32_t N = 1u << nbits;
    const uint32_t r = (uint32_t)(T & (uint64_t)(N - 1));
    if (i < N)
        leaf[(i - r) & (N - 1)] = acc;
    lds_barrier();
    for (int lev = 0; lev < nbits; lev += LOGF) {
        const int span = nbits - lev < LOGF ? nbits - lev : LOGF;  // log2 of this level's children per node
        const uint32_t kids = 1u << span, w = 1u << lev;           // children, leaves per child
        const uint32_t nodes = N >> (lev + span);
        const u32x4 *tab = tabs[1 + lev];                            // H^(B*w)
        if (nodes > kCombineThreads / 32) {
            // wide levels: one thread per node (bound by LDS bandwidth)
            if (i < nodes) {
                const uint32_t a = i << (lev + span);
                u32x4 v = leaf[a];
                for (uint32_t c = 1; c < kids; ++c)
                    v = mul_tab4(v, tab) ^ leaf[a + c * w];
                leaf[a] = v;
            }
        } else {
            // narrow levels (bound by latency): 32 lanes per node, one lookup
            // each per product; node i / 32 is uniform across each half-wave,
            // whose reads of its leaves precede its write, and other nodes
            // touch other leaves
            const uint32_t pp = i >> 5;
            const bool act = pp < nodes;
            const uint32_t a = act ? pp << (lev + span) : 0u;
            u32x4 v = act ? leaf[a] : u32x4{0, 0, 0, 0};
            for (uint32_t c = 1; c < kids; ++c) {
                v = mul_tab4_half(v, tab, i & 31u, act);
                if (act)
                    v ^= leaf[a + c * w];
            }
            if (act && (i & 31u) == 0)
                leaf[a] = v;
        }
        lds_barrier();
    }
    // * H, by the first half-wave
    const u32x4 s = mul_tab4_half(i < 32 ? leaf[0] : u32x4{0, 0, 0, 0}, tabs[0], i & 31u, i < 32);
    if (d.yout) {
        // a streamed segment (or a POLYVAL pass): hand on its GHASH value,
        // first multiplied by H^lift (the blocks of the message that follow
        // the segment) with the key slot's nibble tables of H^(2^k), one
        // half-wave product per set bit
        if (i >= 64)
            return;
        u32x4 y = s;
        const u32x4 *g4 = reinterpret_cast<const u32x4 *>(d.slot + kSlotTab4Off);
        for (uint64_t e = d.lift, k = 0; e && k < (uint64_t)kTab4Levels; e >>= 1, ++k)
            if (e & 1u)
                y = mul_tab4_half(y, g4 + k * 512, i & 31u, i < 32);
        if (i == 0)
            *reinterpret_cast<u32x4 *>(d.yout) = y;
        return;
    }
    if (i == 0) {
        const u32x4 tag = s ^ partials[d.tile_base + T];
        const uint32_t tw[4] = {tag.x, tag.y, tag.z, tag.w};
        const int tl = (int)d.tag_len;  // T = MSB_t of the full tag
        if (d.op == 0) {
            uint8_t *dst = reinterpret_cast<uint8_t *>(d.tag);
            for (int k = 0; k < tl; ++k)
                dst[k] = (uint8_t)(tw[k >> 2] >> (8 * (k & 3)));
        } else {
            const uint8_t *exp = reinterpret_cast<const uint8_t *>(d.tag);
            uint32_t diff = 0;
            for (int k = 0; k < tl; ++k)
                diff |= ((tw[k >> 2] >> (8 * (k & 3))) & 0xffu) ^ exp[k];
            const int32_t ok = diff == 0 ? 1 : 0;
            *reinterpret_cast<int32_t *>(d.ok) = ok;
            if (!ok) {
                const uint32_t pos = atomicAdd(&counters[0], 1u);
                counters[1 + pos] = BATCH ? blockIdx.x : 0u;
            }
        }
    }
}

// ---------------------------------------------------------------- streamed message tag

// GHASH of a message fed in segments is the XOR of the segments' own GHASH
// values, each multiplied by H^(blocks after it) (the combine's lift); the
// tag adds E_K(J0).  One wave: lane l XORs values l, l + 64, ..., then an
// XOR across the wave.  Encrypt writes tag_len bytes of the tag; decrypt
// compares them without early exit and writes the accept flag.
__global__ __launch_bounds__(64) void k_gcm_fold(const u32x4 *__restrict__ vals, uint32_t k,
                                                 const u32x4 *__restrict__ ekj0, uint8_t *tag, int32_t *ok,
                                                 uint32_t op, uint32_t tag_len, uint64_t slot, u32x4 lenblk)
{
    const uint32_t lane = threadIdx.x;
    u32x4 acc = {0, 0, 0, 0};
    for (uint32_t j = lane; j < k; j += 64)
        acc ^= vals[j];
    acc = wave_xor_reduce(acc);
    if (slot) {
        // GHASH's last block, the length block L, enters as L * H (the
        // slot's nibble table of H^(2^0)); the values above were lifted past it
        const u32x4 *g4 = reinterpret_cast<const u32x4 *>(slot + kSlotTab4Off);
        acc ^= mul_tab4_half(lenblk, g4, lane & 31u, lane < 32);
    }
    if (lane != 0)
        return;
    const u32x4 t = acc ^ *ekj0;
    const uint32_t tw[4] = {t.x, t.y, t.z, t.w};
    if (op == 0) {
        for (uint32_t b = 0; b < tag_len; ++b)
            tag[b] = (uint8_t)(tw[b >> 2] >> (8 * (b & 3)));
    } else {
        uint32_t diff = 0;
        for (uint32_t b = 0; b < tag_len; ++b)
            diff |= ((tw[b >> 2] >> (8 * (b & 3))) & 0xffu) ^ tag[b];
        *ok = diff == 0 ? 1 : 0;
    }
}

// ---------------------------------------------------------------- J0 for other IV lengths

// J0 = GHASH_H(IV || 0^s || 0^64 || [8*len(IV)]_64) (SP 800-38D sec. 7.1,
// step 2), by Horner over the IV blocks with the nibble table of H staged in
// LDS; one workgroup, written to j0_out (16 bytes).
__global__ __launch_bounds__(64) void k_gcm_j0(IvArg iv, uint64_t slot, u32x4 *j0_out, u32x4 *y_zero)
{
    if (y_zero && threadIdx.x == 0)
        *y_zero = u32x4{0, 0, 0, 0};  // a new stream's GHASH value
    if (iv.len == 12) {  // J0 = IV || 0^31 || 1
        if (threadIdx.x == 0) {
            uint32_t w[3] = {0, 0, 0};
            for (int k = 0; k < 12; ++k)
                w[k >> 2] |= (uint32_t)iv.b[k] << (8 * (k & 3));
            *j0_out = u32x4{w[0], w[1], w[2], 0x01000000u};
        }
        return;
    }
    __shared__ u32x4 tab[512];
    const GLOBAL_AS u32x4 *src = gptr<const u32x4>(slot + kSlotTab4Off);  // level 0: H
    u32x4 st[8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
        st[r] = src[threadIdx.x + 64 * r];
#pragma unroll
    for (int r = 0; r < 8; ++r)
        tab[threadIdx.x + 64 * r] = st[r];
    lds_barrier();
    if (threadIdx.x != 0)
        return;
    u32x4 y = {0, 0, 0, 0};
    const uint32_t n = iv.len;
    for (uint32_t off = 0; off < n; off += 16) {
        uint32_t w[4] = {0, 0, 0, 0};
        for (uint32_t k = 0; k < 16 && off + k < n; ++k)
            w[k >> 2] |= (uint32_t)iv.b[off + k] << (8 * (k & 3));
        y = mul_tab4(y ^ u32x4{w[0], w[1], w[2], w[3]}, tab);
    }
    const uint64_t bits = (uint64_t)n * 8;
    y = mul_tab4(y ^ u32x4{0u, 0u, bswap32((uint32_t)(bits >> 32)), bswap32((uint32_t)bits)}, tab);
    *j0_out = y;
}

// ---------------------------------------------------------------- zero-fill on reject

template <bool BATCH>
__global__ __launch_bounds__(256) void k_gcm_zerofill(const MsgDesc *__restrict__ descs, MsgDesc single,
                                                      const uint32_t *__restrict__ counters)
{
    const uint32_t n_rej = counters[0];
    for (uint32_t q = 0; q < n_rej; ++q) {
        const MsgDesc d = BATCH ? descs[counters[1 + q]] : single;
        uint8_t *out = reinterpret_cast<uint8_t *>(d.out);
        const uint64_t nfull = d.len >> 4;
        const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
        for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nfull; j += stride)
            __builtin_nontemporal_store(u32x4{0, 0, 0, 0}, reinterpret_cast<u32x4 *>(out) + j);
        if (blockIdx.x == 0 && threadIdx.x < (d.len & 15))
            out[nfull * 16 + threadIdx.x] = 0;
    }
}

// ---------------------------------------------------------------- AES-GCM-SIV (RFC 8452)
//
// POLYVAL through GHASH: with BR the reversal of a block's 16 bytes,
// POLYVAL(H, X_1..X_s) = BR(GHASH_H'(BR(X_1), ..., BR(X_s))) where H' is
// BR(H) times x in GHASH's field (RFC 8452 appendix A).  A per-message slot
// holds the derived encryption key's round keys and H' with every GHASH table
// of an ordinary key slot, so the tiles, the lane fix-ups and the combine
// tree run unchanged on byte-reversed blocks.  The counter block is the tag
// with the top bit of byte 15 set; its bytes 0..3 (memory-order dword 0) are
// a little-endian 32-bit counter, so dword 0 is the column that varies, where
// GCM's counter varies column 3.

struct SivArg {
    uint32_t nonce[3];
    uint32_t pad;
};

__device__ __forceinline__ u32x4 rev_block(u32x4 x) { return u32x4{bswap32(x.w), bswap32(x.z), bswap32(x.y), bswap32(x.x)}; }

// One wave: the message keys from the key-generating key in slot `kgk`
// (first halves of AES_KGK(LE32(i) || nonce): i = 0, 1 the authentication
// key, i = 2, 3 (and 4, 5 for a 256-bit key) the encryption key), expanded
// into slot `out` with H' and its powers H'^(2^k).  With `tag_in` (decrypt)
// the counter block is also formed from the received tag at `ctr_out`.
__global__ __launch_bounds__(64) void k_siv_derive(uint64_t kgk, SivArg na, uint64_t out, const uint8_t *tag_in,
                                                   u32x4 *ctr_out, const uint32_t *te0g, const uint32_t *sbg,
                                                   const u32x4 *__restrict__ frob)
{
    __shared__ uint32_t te0[256], sb[256];
    __shared__ uint32_t h_sh[4];
    __shared__ uint32_t half_sh[12];
    stage_aes_tables64(te0, sb, te0g, sbg);
    lds_barrier();
    KeySlotHdr *hd = reinterpret_cast<KeySlotHdr *>(out);
    const KeySlotHdr *kh = reinterpret_cast<const KeySlotHdr *>(kgk);
    const bool k128 = kh->nr == 10;
    const int nblk = k128 ? 4 : 6;
    // the nblk key-generating blocks are independent: thread i encrypts
    // block i, thread 0 then expands the message key from their halves
    if ((int)threadIdx.x < nblk) {
        const int i = (int)threadIdx.x;
        uint32_t rkw[4 * (kMaxNr + 1)];
        for (int j = 0; j < 4 * (kMaxNr + 1); ++j)
            rkw[j] = kh->rk[j];
        const uint32_t in[4] = {(uint32_t)i, na.nonce[0], na.nonce[1], na.nonce[2]};
        uint32_t o[4];
        if (k128)
            aes_block<10>(rkw, te0, sb, in, o);
        else
            aes_block<14>(rkw, te0, sb, in, o);
        half_sh[2 * i] = o[0];
        half_sh[2 * i + 1] = o[1];
    }
    lds_barrier();
    if (threadIdx.x == 0) {
        uint32_t half[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int i = 0; i < 2 * nblk; ++i)
            half[i] = half_sh[i];
        uint32_t w[4 * (kMaxNr + 1)];
        if (k128)
            expand_key<4>(half + 4, hd, sb, w);
        else
            expand_key<8>(half + 4, hd, sb, w);
        const uint32_t br[4] = {bswap32(half[3]), bswap32(half[2]), bswap32(half[1]), bswap32(half[0])};
        const u32x4 hp = poly_to_mem(poly_mul_xi(mem_to_poly(br), 1));
        const uint32_t hw[4] = {hp.x, hp.y, hp.z, hp.w};
        for (int i = 0; i < 4; ++i) {
            hd->h[i] = hw[i];
            h_sh[i] = hw[i];
        }
        if (tag_in) {
            uint32_t c[4] = {0, 0, 0, 0};
            for (int k = 0; k < 16; ++k)
                c[k >> 2] |= (uint32_t)tag_in[k] << (8 * (k & 3));
            *ctr_out = u32x4{c[0], c[1], c[2], c[3] | 0x80000000u};
        }
    }
    lds_barrier();
    write_hpow(hd, h_sh, frob);
}

// One wave: S = BR(*g) is the POLYVAL value; S ^= nonce in bytes 0..11, top
// bit of byte 15 cleared; tag = AES(S) under the slot's encryption key.
// Encrypt (tag_out): write the tag and the counter block.  Decrypt: compare
// all 16 bytes with tag_in without early exit, write the accept flag and the
// reject count the zero-fill reads.
__global__ __launch_bounds__(64) void k_siv_tag(uint64_t slot, const u32x4 *g, SivArg na, uint8_t *tag_out,
                                                u32x4 *ctr_out, const uint8_t *tag_in, int32_t *ok,
                                                uint32_t *counters, const uint32_t *te0g, const uint32_t *sbg)
{
    __shared__ uint32_t te0[256], sb[256];
    stage_aes_tables64(te0, sb, te0g, sbg);
    lds_barrier();
    if (threadIdx.x != 0)
        return;
    const KeySlotHdr *hd = reinterpret_cast<const KeySlotHdr *>(slot);
    uint32_t rkw[4 * (kMaxNr + 1)];
    for (int i = 0; i < 4 * (kMaxNr + 1); ++i)
        rkw[i] = hd->rk[i];
    const u32x4 sv = rev_block(*g);
    const uint32_t in[4] = {sv.x ^ na.nonce[0], sv.y ^ na.nonce[1], sv.z ^ na.nonce[2], sv.w & 0x7fffffffu};
    uint32_t t[4];
    if (hd->nr == 10)
        aes_block<10>(rkw, te0, sb, in, t);
    else
        aes_block<14>(rkw, te0, sb, in, t);
    if (tag_out) {
        for (int k = 0; k < 16; ++k)
            tag_out[k] = (uint8_t)(t[k >> 2] >> (8 * (k & 3)));
        *ctr_out = u32x4{t[0], t[1], t[2], t[3] | 0x80000000u};
        return;
    }
    uint32_t diff = 0;
    for (int k = 0; k < 16; ++k)
        diff |= ((t[k >> 2] >> (8 * (k & 3))) & 0xffu) ^ tag_in[k];
    const int32_t accept = diff == 0 ? 1 : 0;
    *ok = accept;
    counters[0] = accept ? 0u : 1u;
    counters[1] = 0u;
}

struct SivCtx {
    uint32_t u0, u1, u2, u3;  // round-1 columns without the counter dword's bytes (unrotated, uniform)
    uint32_t rk0;             // round key 0, column 0
};

// Keystream block for LE counter value `ctr` in dword 0: round 1 needs the
// four lookups of the counter dword's bytes only.
template <int NR>
__device__ __forceinline__ u32x4 aes_siv_ctr(uint32_t ctr, const SivCtx &c, const CONST_AS uint32_t *rk,
                                             const uint8_t *lds, const LaneK &lk)
{
    const uint32_t w0 = rotr_by(ctr ^ c.rk0, lk.rot);
    const uint32_t s0 = rotr_by(c.u0, lk.rot) ^ LK(0, w0);
    const uint32_t s1 = rotr_by(c.u1, lk.rot) ^ LK(3, w0);
    const uint32_t s2 = rotr_by(c.u2, lk.rot) ^ LK(2, w0);
    const uint32_t s3 = rotr_by(c.u3, lk.rot) ^ LK(1, w0);
    return aes_rounds<2, NR>(s0, s1, s2, s3, rk, lds, lk);
}

// Counter-mode caching through round 2, as for GCM: with counter bytes 1..3
// fixed, round 1 leaves columns 1..3 fixed and column 0 depends on the low
// counter byte only, so round 2 takes one lookup per column.
__device__ __forceinline__ Ctr2 siv_round2(uint32_t hi, const SivCtx &c, const CONST_AS uint32_t *rk,
                                           const CONST_AS uint32_t *te)
{
    const uint32_t v = (hi << 8) ^ c.rk0;  // counter bytes 1..3 with the key (byte 0 unused)
    const uint32_t u1 = c.u1 ^ te_s(te, 3, B3(v));
    const uint32_t u2 = c.u2 ^ te_s(te, 2, B2(v));
    const uint32_t u3 = c.u3 ^ te_s(te, 1, B1(v));
    Ctr2 q;
    q.v0 = te_s(te, 1, B1(u1)) ^ te_s(te, 2, B2(u2)) ^ te_s(te, 3, B3(u3)) ^ rk[8];
    q.v1 = te_s(te, 0, B0(u1)) ^ te_s(te, 1, B1(u2)) ^ te_s(te, 2, B2(u3)) ^ rk[9];
    q.v2 = te_s(te, 0, B0(u2)) ^ te_s(te, 1, B1(u3)) ^ te_s(te, 3, B3(u1)) ^ rk[10];
    q.v3 = te_s(te, 0, B0(u3)) ^ te_s(te, 2, B2(u1)) ^ te_s(te, 3, B3(u2)) ^ rk[11];
    return q;
}

template <int NR>
__device__ __forceinline__ u32x4 aes_siv_ctr2(uint32_t ctr, const Ctr2 &q, const SivCtx &c,
                                              const CONST_AS uint32_t *rk, const uint8_t *lds, const LaneK &lk)
{
    const uint32_t w0 = rotr_by(ctr ^ c.rk0, lk.rot);       // byte 0: low counter byte ^ key
    const uint32_t x0 = rotr_by(c.u0, lk.rot) ^ LK(0, w0);  // round-1 column 0
    const uint32_t s0 = rotr_by(q.v0, lk.rot) ^ LK(0, x0);
    const uint32_t s1 = rotr_by(q.v1, lk.rot) ^ LK(3, x0);
    const uint32_t s2 = rotr_by(q.v2, lk.rot) ^ LK(2, x0);
    const uint32_t s3 = rotr_by(q.v3, lk.rot) ^ LK(1, x0);
    return aes_rounds<3, NR>(s0, s1, s2, s3, rk, lds, lk);
}

// The three tile passes: the POLYVAL of AAD and plaintext (encrypt, first
// pass), counter mode alone (encrypt, second pass, once the tag is known),
// and counter mode fused with the POLYVAL of its output (decrypt-verify).
constexpr int kSivHash = 0, kSivCtr = 1, kSivDec = 2;

// Wave tile t of one message, laid out as in wave_tile: rows of 64 blocks,
// lane l on block 64r + l, per-lane Horner with H'^64 over byte-reversed
// blocks, fix-up by H'^(63 - l), XOR across the wave.  The GHASH sequence is
// AAD blocks, data blocks and the length block LE64(8|A|) || LE64(8|P|),
// each zero-padded and reversed.
template <int NR, int PASS>
__device__ void wave_tile_siv(const MsgDesc &d, uint64_t t, const uint8_t *__restrict__ lds, const LaneK &lk,
                              const GhK &gk, const uint32_t *__restrict__ te0g, u32x4 *__restrict__ partials)
{
    constexpr bool GH = PASS != kSivCtr, AES = PASS != kSivHash;
    const int lane = threadIdx.x & 63;
    const CONST_AS uint32_t *te = cptr<uint32_t>(te0g);
    const CONST_AS uint32_t *rk_base = cptr<uint32_t>(reinterpret_cast<const void *>(d.slot));
    const CONST_AS uint32_t *rk = rk_base;
    SivCtx c = {0, 0, 0, 0, 0};
    uint32_t c0 = 0;
    if (AES) {
        const CONST_AS uint32_t *cw = cptr<uint32_t>(reinterpret_cast<const void *>(d.j0));
        c0 = cw[0];
        const uint32_t s1 = cw[1] ^ rk[1], s2 = cw[2] ^ rk[2], s3 = cw[3] ^ rk[3];
        c.u0 = uniform(te_u(lds, 1, B1(s1)) ^ te_u(lds, 2, B2(s2)) ^ te_u(lds, 3, B3(s3)) ^ rk[4]);
        c.u1 = uniform(te_u(lds, 0, B0(s1)) ^ te_u(lds, 1, B1(s2)) ^ te_u(lds, 2, B2(s3)) ^ rk[5]);
        c.u2 = uniform(te_u(lds, 0, B0(s2)) ^ te_u(lds, 1, B1(s3)) ^ te_u(lds, 3, B3(s1)) ^ rk[6]);
        c.u3 = uniform(te_u(lds, 0, B0(s3)) ^ te_u(lds, 2, B2(s1)) ^ te_u(lds, 3, B3(s2)) ^ rk[7]);
        c.rk0 = rk[0];
    }

    const uint64_t B = 1ull << d.log2B;
    const uint32_t R = (uint32_t)(B >> 6);
    const int64_t vbase = (int64_t)(t * B) - (int64_t)d.z;  // sequence index of lane 0, row 0
    const uint32_t r0 = vbase < 0 ? (uint32_t)((uint64_t)(-vbase) >> 6) : 0u;
    const int64_t na = (int64_t)d.na;
    const int64_t nfull = (int64_t)(d.len >> 4);
    const int64_t ndat = (int64_t)d.n;
    const uint8_t *__restrict__ in = reinterpret_cast<const uint8_t *>(d.in);
    uint8_t *__restrict__ out = reinterpret_cast<uint8_t *>(d.out);
    const GLOBAL_AS u32x4 *in_g = gptr<const u32x4>(d.in);
    GLOBAL_AS u32x4 *out_g = gptr<u32x4>(d.out);

    u32x4 a = {0, 0, 0, 0};
    auto boundary_row = [&](int64_t v0) {
        const int64_t v = v0 + lane;
        const uint64_t j = (uint64_t)(v - na);
        u32x4 ks = {0, 0, 0, 0};
        if (AES)
            ks = aes_siv_ctr<NR>((uint32_t)j + c0, c, rk, lds, lk);
        u32x4 X = {0, 0, 0, 0};
        if (GH && v >= 0 && v < na) {
            X = load_block_partial(reinterpret_cast<const uint8_t *>(d.aad), (uint64_t)v, d.aad_len);
        } else if (v >= na && v < na + ndat) {
            const u32x4 x = load_block_partial(in, j, d.len);
            if (AES) {
                const u32x4 o = x ^ ks;
                store_block_partial(out, j, d.len, o);
                X = mask_block(o, j, d.len);
            } else {
                X = x;
            }
        } else if (GH && v == na + ndat) {
            const uint64_t abits = d.aad_len * 8, pbits = d.len * 8;
            X = u32x4{(uint32_t)abits, (uint32_t)(abits >> 32), (uint32_t)pbits, (uint32_t)(pbits >> 32)};
        }
        if (GH)
            a = ghash_mul8(a, rev_block(X), lds, gk);
    };

    // rows [fa, fb) hold 64 whole data blocks (as in wave_tile), with the
    // same falling issue priority over them
    int64_t rf0, rf1;
    {
        const int64_t lo = na - vbase, hi = na + nfull - vbase - 64;
        rf0 = lo <= 0 ? 0 : (lo + 63) >> 6;
        rf1 = hi < 0 ? 0 : (hi >> 6) + 1;
    }
    const uint32_t fa = (uint32_t)(rf0 > (int64_t)r0 ? (rf0 < (int64_t)R ? rf0 : (int64_t)R) : (int64_t)r0);
    const uint32_t fb = (uint32_t)(rf1 > (int64_t)fa ? (rf1 < (int64_t)R ? rf1 : (int64_t)R) : (int64_t)fa);
    uint32_t r = r0;
    for (; r < fa; ++r)
        boundary_row(vbase + 64 * (int64_t)r);
    uint32_t hc = 0xffffffffu;
    Ctr2 cur = {0, 0, 0, 0};
    const uint32_t loff = 16u * (uint32_t)lane;
    const uint32_t span = fb - r;
    const uint32_t q1 = r + span / 4, q2 = r + span / 2, q3 = r + 3 * (span / 4);
    __builtin_amdgcn_s_setprio(3);
    for (; r < fb; ++r) {
        if (r == q1)
            __builtin_amdgcn_s_setprio(2);
        if (r == q2)
            __builtin_amdgcn_s_setprio(1);
        if (r == q3)
            __builtin_amdgcn_s_setprio(0);
        rk = rk_base;
        asm volatile("" : "+s"(rk));
        const uint64_t j0 = (uint64_t)(vbase + 64 * (int64_t)r - na);  // first data block of the row (uniform)
        {
            const u32x4 x = *reinterpret_cast<const GLOBAL_AS u32x4 *>(
                reinterpret_cast<const GLOBAL_AS uint8_t *>(in_g + j0) + loff);
            if (AES) {
                const uint32_t base = (uint32_t)j0 + c0;
                const uint32_t h = base >> 8;
                if (h != hc) {
                    cur = siv_round2(h, c, rk, te);
                    hc = h;
                }
                const uint32_t ctr = base + (uint32_t)lane;
                Ctr2 q = cur;
                if ((base & 255u) > 192u) {
                    const uint32_t h1 = (h + 1u) & 0xffffffu;
                    const Ctr2 nxt = siv_round2(h1, c, rk, te);
                    const bool up = (ctr << 24) < (base << 24);  // low counter byte wrapped in the row
                    q = Ctr2{up ? nxt.v0 : cur.v0, up ? nxt.v1 : cur.v1, up ? nxt.v2 : cur.v2, up ? nxt.v3 : cur.v3};
                    cur = nxt;
                    hc = h1;
                }
                const u32x4 o = x ^ aes_siv_ctr2<NR>(ctr, q, c, rk, lds, lk);
                __builtin_nontemporal_store(
                    o, reinterpret_cast<GLOBAL_AS u32x4 *>(reinterpret_cast<GLOBAL_AS uint8_t *>(out_g + j0) + loff));
                if (GH)
                    a = ghash_mul8(a, rev_block(o), lds, gk);
            } else {
                a = ghash_mul8(a, rev_block(x), lds, gk);
            }
        }
    }
    for (; r < R; ++r)
        boundary_row(vbase + 64 * (int64_t)r);
    if (!GH)
        return;
    a = gf_mul_lanewin(a, lds, lane);
    a = wave_xor_reduce(a);
    if (lane == 0)
        partials[d.tile_base + t] = a;
}

// One message, tiles [d.tile_lo, d.tile_hi): workgroup item it covers WAVES
// consecutive tiles.  LDS as in k_gcm_tiles (GHASH table of the message slot,
// T-tables), each staged only by the passes that read it.
template <int WAVES, int PASS>
__global__ __launch_bounds__(WAVES * 64) void k_siv_tiles(MsgDesc d, uint32_t n_items,
                                                          const uint32_t *__restrict__ te0g,
                                                          u32x4 *__restrict__ partials)
{
    constexpr bool GH = PASS != kSivCtr, AES = PASS != kSivHash;
    __shared__ u32x4 lds_v[9216];
    const uint8_t *lds = reinterpret_cast<const uint8_t *>(lds_v);
    if (AES)
        stage_ttables<WAVES * 64>(lds_v, te0g);
    if (GH)
        stage_key_tables<WAVES * 64>(lds_v, d.slot);
    lds_barrier();
    const LaneK lk = lane_constants(threadIdx.x & 63);
    const GhK gk = gh_constants(threadIdx.x & 63);
    const uint32_t wave = uniform(threadIdx.x >> 6);
    for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const uint64_t t = d.tile_lo + (uint64_t)it * WAVES + wave;
        if (t < d.tile_hi) {
            if (d.nr == 10)
                wave_tile_siv<10, PASS>(d, t, lds, lk, gk, te0g, partials);
            else
                wave_tile_siv<14, PASS>(d, t, lds, lk, gk, te0g, partials);
        }
    }
}

// ---------------------------------------------------------------- host-side launchers

hipError_t launch_init_tables(uint32_t *te0, uint32_t *sbox, void *frob, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_tables, dim3(1), dim3(256), 0, s, te0, sbox);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_frob_tables, dim3(kPowLevels - 1), dim3(256), 0, s, reinterpret_cast<u32x4 *>(frob));
    return hipGetLastError();
}

size_t frob_table_bytes() { return (size_t)(kPowLevels - 1) * 4096 * 16; }

// Expand n keys (key i: key_lens[i] bytes at keys + key_off[i]) into the
// slots at slot_addrs[i], in launches of kKeyChunk keys.
hipError_t launch_key_setup(const uint8_t *const *keys, const uint32_t *key_lens, const uint64_t *slot_addrs,
                            uint32_t n, const uint32_t *te0, const uint32_t *sbox, const void *frob, hipStream_t s)
{
    for (uint32_t base = 0; base < n; base += kKeyChunk) {
        const uint32_t m = n - base < (uint32_t)kKeyChunk ? n - base : (uint32_t)kKeyChunk;
        KeyChunk kc{};
        SlotChunk sc{};
        for (uint32_t j = 0; j < m; ++j) {
            const uint8_t *key = keys[base + j];
            const uint32_t len = key_lens[base + j];
            for (uint32_t i = 0; i < len / 4; ++i)
                kc.keys[j].w[i] = (uint32_t)key[4 * i] | ((uint32_t)key[4 * i + 1] << 8) |
                                  ((uint32_t)key[4 * i + 2] << 16) | ((uint32_t)key[4 * i + 3] << 24);
            kc.keys[j].len = len;
            kc.slots[j] = slot_addrs[base + j];
            sc.slots[j] = slot_addrs[base + j];
        }
        hipLaunchKernelGGL(k_key_setup, dim3(m), dim3(64), 0, s, kc, te0, sbox, reinterpret_cast<const u32x4 *>(frob));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_key_tables, dim3(kTab4Levels + kTab8Blocks + kLanePows, m), dim3(256), 0, s, sc);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <int WAVES>
static hipError_t launch_tiles_w(const MsgDesc *descs, const WorkItem *items, uint32_t n_items, const MsgDesc *single,
                                 const uint32_t *te0, u32x4 *partials, uint32_t *counters, uint32_t grid,
                                 hipStream_t s)
{
    if (descs)
        hipLaunchKernelGGL((k_gcm_tiles<WAVES, true, kModeGcm>), dim3(grid), dim3(WAVES * 64), 0, s, descs, items,
                           n_items, MsgDesc{}, te0, partials, counters);
    else if (single->op == 2)
        hipLaunchKernelGGL((k_gcm_tiles<WAVES, false, kModeCtr>), dim3(grid), dim3(WAVES * 64), 0, s, nullptr,
                           nullptr, n_items, *single, te0, partials, counters);
    else if (single->j0)
        hipLaunchKernelGGL((k_gcm_tiles<WAVES, false, kModeGcmJ0>), dim3(grid), dim3(WAVES * 64), 0, s, nullptr,
                           nullptr, n_items, *single, te0, partials, counters);
    else if (single->aad_len >= kAadRowsMinBytes)
        hipLaunchKernelGGL((k_gcm_tiles<WAVES, false, kModeGcmAad>), dim3(grid), dim3(WAVES * 64), 0, s, nullptr,
                           nullptr, n_items, *single, te0, partials, counters);
    else
        hipLaunchKernelGGL((k_gcm_tiles<WAVES, false, kModeGcm>), dim3(grid), dim3(WAVES * 64), 0, s, nullptr,
                           nullptr, n_items, *single, te0, partials, counters);
    return hipGetLastError();
}

hipError_t launch_tiles(int waves, const MsgDesc *descs, const WorkItem *items, uint32_t n_items,
                        const MsgDesc *single, const uint32_t *te0, void *partials, uint32_t *counters, uint32_t grid,
                        hipStream_t s)
{
    u32x4 *p = reinterpret_cast<u32x4 *>(partials);
    switch (waves) {
    case 8:
        return launch_tiles_w<8>(descs, items, n_items, single, te0, p, counters, grid, s);
    case 12:
        return launch_tiles_w<12>(descs, items, n_items, single, te0, p, counters, grid, s);
    case 16:
        return launch_tiles_w<16>(descs, items, n_items, single, te0, p, counters, grid, s);
    default:
        return hipErrorInvalidValue;
    }
}

int max_groups_per_cu(int waves)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (waves) {
    case 8:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gcm_tiles<8, false, kModeGcm>, 8 * 64, 0);
        break;
    case 12:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gcm_tiles<12, false, kModeGcm>, 12 * 64, 0);
        break;
    case 16:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gcm_tiles<16, false, kModeGcm>, 16 * 64, 0);
        break;
    }
    return (e == hipSuccess && n > 0) ? n : 1;
}

template <int LOGF>
static void launch_combine_f(const MsgDesc *descs, uint32_t n_msgs, const MsgDesc *single, const u32x4 *p,
                             uint32_t *counters, hipStream_t s)
{
    if (descs)
        hipLaunchKernelGGL((k_gcm_combine<true, LOGF>), dim3(n_msgs), dim3(kCombineThreads), 0, s, descs, MsgDesc{},
                           p, counters);
    else
        hipLaunchKernelGGL((k_gcm_combine<false, LOGF>), dim3(1), dim3(kCombineThreads), 0, s, nullptr, *single, p,
                           counters);
}

hipError_t launch_combine(const MsgDesc *descs, uint32_t n_msgs, const MsgDesc *single, const void *partials,
                          uint32_t *counters, uint32_t fanin, hipStream_t s)
{
    const u32x4 *p = reinterpret_cast<const u32x4 *>(partials);
    switch (fanin) {
    case 2:
        launch_combine_f<1>(descs, n_msgs, single, p, counters, s);
        break;
    case 4:
        launch_combine_f<2>(descs, n_msgs, single, p, counters, s);
        break;
    case 8:
        launch_combine_f<3>(descs, n_msgs, single, p, counters, s);
        break;
    case 16:
        launch_combine_f<4>(descs, n_msgs, single, p, counters, s);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fold(const void *vals, uint32_t k, const void *ekj0, uint8_t *tag, int32_t *ok, uint32_t op,
                       uint32_t tag_len, uint64_t slot, const uint32_t lenblk[4], hipStream_t s)
{
    const u32x4 l = lenblk ? u32x4{lenblk[0], lenblk[1], lenblk[2], lenblk[3]} : u32x4{0, 0, 0, 0};
    hipLaunchKernelGGL(k_gcm_fold, dim3(1), dim3(64), 0, s, reinterpret_cast<const u32x4 *>(vals), k,
                       reinterpret_cast<const u32x4 *>(ekj0), tag, ok, op, tag_len, lenblk ? slot : 0, l);
    return hipGetLastError();
}

hipError_t launch_j0(const IvArg &iv, uint64_t slot, void *j0_out, void *y_zero, hipStream_t s)
{
    hipLaunchKernelGGL(k_gcm_j0, dim3(1), dim3(64), 0, s, iv, slot, reinterpret_cast<u32x4 *>(j0_out),
                       reinterpret_cast<u32x4 *>(y_zero));
    return hipGetLastError();
}

hipError_t launch_zerofill(const MsgDesc *descs, const MsgDesc *single, const uint32_t *counters, uint32_t grid,
                           hipStream_t s)
{
    if (descs)
        hipLaunchKernelGGL(k_gcm_zerofill<true>, dim3(grid), dim3(256), 0, s, descs, MsgDesc{}, counters);
    else
        hipLaunchKernelGGL(k_gcm_zerofill<false>, dim3(grid), dim3(256), 0, s, nullptr, *single, counters);
    return hipGetLastError();
}

hipError_t launch_siv_derive(uint64_t kgk_slot, const uint8_t nonce[12], uint64_t out_slot, const uint8_t *tag_in,
                             void *ctr_out, const uint32_t *te0, const uint32_t *sbox, const void *frob, hipStream_t s)
{
    SivArg a{};
    for (int i = 0; i < 3; ++i)
        a.nonce[i] = (uint32_t)nonce[4 * i] | ((uint32_t)nonce[4 * i + 1] << 8) | ((uint32_t)nonce[4 * i + 2] << 16) |
                     ((uint32_t)nonce[4 * i + 3] << 24);
    hipLaunchKernelGGL(k_siv_derive, dim3(1), dim3(64), 0, s, kgk_slot, a, out_slot, tag_in,
                       reinterpret_cast<u32x4 *>(ctr_out), te0, sbox, reinterpret_cast<const u32x4 *>(frob));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    SlotChunk sc{};
    sc.slots[0] = out_slot;
    hipLaunchKernelGGL(k_key_tables, dim3(kTab4Levels + kTab8Blocks + kLanePows, 1), dim3(256), 0, s, sc);
    return hipGetLastError();
}

hipError_t launch_siv_tag(uint64_t slot, const void *g, const uint8_t nonce[12], uint8_t *tag_out, void *ctr_out,
                          const uint8_t *tag_in, int32_t *ok, uint32_t *counters, const uint32_t *te0,
                          const uint32_t *sbox, hipStream_t s)
{
    SivArg a{};
    for (int i = 0; i < 3; ++i)
        a.nonce[i] = (uint32_t)nonce[4 * i] | ((uint32_t)nonce[4 * i + 1] << 8) | ((uint32_t)nonce[4 * i + 2] << 16) |
                     ((uint32_t)nonce[4 * i + 3] << 24);
    hipLaunchKernelGGL(k_siv_tag, dim3(1), dim3(64), 0, s, slot, reinterpret_cast<const u32x4 *>(g), a, tag_out,
                       reinterpret_cast<u32x4 *>(ctr_out), tag_in, ok, counters, te0, sbox);
    return hipGetLastError();
}

template <int WAVES>
static hipError_t launch_siv_tiles_w(int pass, const MsgDesc &d, uint32_t n_items, const uint32_t *te0, u32x4 *p,
                                     uint32_t grid, hipStream_t s)
{
    if (pass == kSivHash)
        hipLaunchKernelGGL((k_siv_tiles<WAVES, kSivHash>), dim3(grid), dim3(WAVES * 64), 0, s, d, n_items, te0, p);
    else if (pass == kSivCtr)
        hipLaunchKernelGGL((k_siv_tiles<WAVES, kSivCtr>), dim3(grid), dim3(WAVES * 64), 0, s, d, n_items, te0, p);
    else
        hipLaunchKernelGGL((k_siv_tiles<WAVES, kSivDec>), dim3(grid), dim3(WAVES * 64), 0, s, d, n_items, te0, p);
    return hipGetLastError();
}

hipError_t launch_siv_tiles(int waves, int pass, const MsgDesc &d, uint32_t n_items, const uint32_t *te0,
                            void *partials, uint32_t grid, hipStream_t s)
{
    u32x4 *p = reinterpret_cast<u32x4 *>(partials);
    if (pass < kSivHash || pass > kSivDec)
        return hipErrorInvalidValue;
    switch (waves) {
    case 8:
        return launch_siv_tiles_w<8>(pass, d, n_items, te0, p, grid, s);
    case 12:
        return launch_siv_tiles_w<12>(pass, d, n_items, te0, p, grid, s);
    case 16:
        return launch_siv_tiles_w<16>(pass, d, n_items, te0, p, grid, s);
    default:
        return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- fixed device scratch

// Workspace of the allocation-free entry point: a module-scope array that
// every device the library runs on holds until the process ends.  Host code
// never passes its name to a kernel (on the host it is only a stand-in
// symbol); it passes the device address looked up below.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

// Device address of `scratch` on `device`, looked up once per device with
// that device current and kept for every later context on it.
hipError_t scratch_address(int device, void **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess)
            return e;
        if (cur != device) {
            e = hipSetDevice(device);
            if (e != hipSuccess)
                return e;
        }
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device)
            (void)hipSetDevice(cur);
        if (e != hipSuccess)
            return e;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

}  // namespace gcm
