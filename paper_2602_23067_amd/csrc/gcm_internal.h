// gcm_internal.h -- layouts shared by the host runtime and the gfx950 kernels.
//
// Byte/bit conventions (NIST SP 800-38D sec. 6.3, FIPS-197 sec. 3):
//  * A 16-byte block is held as four little-endian dwords in memory order:
//    byte j sits in dword j/4, bits 8*(j%4)..+7.  AES column c is dword c,
//    AES row r is byte r of a column.
//  * A GF(2^128) element is held in the same memory order.  Byte j bit s
//    (value 1<<s) is the coefficient of x^(8j + 7 - s), so the field's one is
//    byte 0 = 0x80.  Multiplication by a fixed element M is GF(2)-linear, so
//    X*M = XOR over byte positions j of TAB_j[X_j] with TAB_j[b] = (b at
//    position j)*M; the tables already contain the reduction, and the hot
//    loop never swaps bytes or reverses bits.
#pragma once
#include <stdint.h>

namespace gcm {

// ---- AES tables (device memory, one block per context) ----
// words [0, 256): TE0, the MixColumns column (2s, s, s, 3s) of S(x);
// [256, 512): the S-box as words; [512, 1280): TE1..TE3 = TE0 rotated left by
// 8, 16 and 24 bits.
constexpr uint32_t kTe1Off = 512;
constexpr uint32_t kAesTableWords = 1280;

// ---- key slot (device memory, one per resident key) ----
constexpr int kMaxNr = 14;
constexpr int kPowLevels = 48;      // H^(2^k), k = 0..47
constexpr int kTab4Levels = 40;     // nibble tables for H^(2^k), k = 0..39
constexpr int kStrideLevel = 6;     // the per-lane Horner multiplier is H^64 = H^(2^6)
constexpr int kKeyChunk = 56;       // keys per key-setup launch (by-value kernel arguments)

struct KeySlotHdr {
    uint32_t rk[4 * (kMaxNr + 1)];  // round keys, memory-order column words
    uint32_t nr;                    // 10, 12 or 14
    uint32_t key_len;
    uint32_t pad0[2];
    uint32_t h[4];                  // H = AES_K(0^128)
    uint32_t hpow[kPowLevels][4];   // H^(2^k)
};

constexpr uint64_t kSlotHdrBytes = 2048;
constexpr uint64_t kTab8Bytes = 16ull * 256 * 16;             // byte-position table, 64 KiB
constexpr uint64_t kTab4Bytes = 32ull * 16 * 16;              // nibble-position table, 8 KiB
constexpr uint64_t kSlotTab8Off = kSlotHdrBytes;
constexpr uint64_t kSlotTab4Off = kSlotTab8Off + kTab8Bytes;
// Tile fix-up tables: lane l of a wave multiplies its Horner value by
// c_l = H^(63 - l); entry (v, l) = (v * c_l) mod P for the 4-bit polynomial v
// sits at byte 16 * (64 * v + l), as polynomial-order words (bit i of the
// 128-bit value is the coefficient of x^i), 16 KiB in all.
constexpr uint64_t kSlotLaneWinOff = kSlotTab4Off + kTab4Levels * kTab4Bytes;
constexpr int kLanePows = 64;
constexpr uint64_t kLaneWinBytes = 16ull * kLanePows * 16;
constexpr uint64_t kSlotBytes = kSlotLaneWinOff + kLaneWinBytes;
static_assert(sizeof(KeySlotHdr) <= kSlotHdrBytes, "slot header too large");

// ---- per-message descriptor ----
// GHASH input X = A || 0-pad || C || 0-pad || L has m = nA + n + 1 blocks.
// It is left-padded with z zero blocks (GHASH(0^z || X) = GHASH(X)) so that
// m + z = T * B with B = 2^log2B blocks per wave tile; tile t covers padded
// positions [t*B, (t+1)*B).
struct MsgDesc {
    uint64_t in;       // device address of input payload
    uint64_t out;      // device address of output payload
    uint64_t aad;      // device address of AAD
    uint64_t tag;      // encrypt: where the tag goes; decrypt: expected tag (device)
    uint64_t ok;       // decrypt: int32 accept flag (device); unused for encrypt
    uint64_t len;      // payload bytes
    uint64_t aad_len;  // AAD bytes
    uint64_t slot;     // device address of the key slot
    uint64_t n;        // data blocks = ceil(len/16)
    uint64_t na;       // AAD blocks = ceil(aad_len/16)
    uint64_t m;        // na + n + 1
    uint64_t z;        // zero-block left padding
    uint64_t tile_base;  // first wave tile of this message in the partials array
    uint64_t n_tiles;    // T
    uint64_t tile_lo;    // this launch covers message tiles [tile_lo, tile_hi)
    uint64_t tile_hi;    //   (0 and T except for chunked host-pipeline launches)
    uint32_t iv[3];      // IV as memory-order dwords
    uint32_t op;         // 0 encrypt, 1 decrypt-verify, 2 CTR only (no GHASH, no tag)
    uint32_t log2B;      // wave tile = 2^log2B blocks (>= 6)
    uint32_t nr;         // AES rounds
    uint32_t groups;     // workgroup items for this message
    uint32_t pad0;
    uint64_t j0;         // device address of J0 (16 bytes) for IVs other than 96 bits; 0: J0 = IV || 0^31 || 1
    uint32_t tag_len;    // tag bytes written (encrypt) or compared (decrypt): 16, or 15, 14, 13, 12, 8, 4
    uint32_t ctr_off;    // a streamed segment: data blocks that precede it, added to the counters
    uint64_t lift;       // with yout: the combine multiplies the segment's GHASH value by H^lift (< 2^40)
    uint64_t yout;       // the combine writes the segment's GHASH value here instead of forming a tag
};

// Bytes of the fixed device scratch behind the allocation-free entry point:
// with tiles of up to 2^16 blocks its 65774 tile partials cover every
// message length SP 800-38D allows together with up to 238 MiB of AAD.
constexpr uint64_t kNoAllocScratchBytes = (1ull << 20) + 4096;  // GCM_NOALLOC_SCRATCH_BYTES

// IVs other than 96 bits: J0 = GHASH_H(IV || 0-pad || 0^64 || [len(IV)]_64),
// computed on the device from IV bytes passed by value
constexpr int kMaxIvBytes = 1024;
struct IvArg {
    uint32_t len;
    uint32_t pad[3];
    uint8_t b[kMaxIvBytes];
};

// One unit of work for a workgroup: `waves` consecutive wave tiles of one message.
struct WorkItem {
    uint32_t msg;
    uint32_t first_tile;  // first wave tile (message-local)
};

}  // namespace gcm
