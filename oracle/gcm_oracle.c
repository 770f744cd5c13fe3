/*
 * gcm_oracle.c -- plain, slow, deliberately literal CPU AES-GCM.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, tables or constants with the
 * GPU path: every table here is derived at start-up from the definitions.
 *
 * What it computes (the paper's "Cryptographic Protocol: AES-GCM" section
 * fixes AES-GCM per NIST SP 800-38D; the serial GHASH recurrence is the
 * paper's equation for Y_i in "Parallel GHASH Reduction"):
 *
 *   GF(2^8)    -- FIPS-197 sec. 4: polynomial basis mod x^8+x^4+x^3+x+1.
 *   S-box      -- FIPS-197 sec. 5.1.1: multiplicative inverse, then affine map.
 *   KeyExpansion, Cipher, InvCipher -- FIPS-197 sec. 5.2, 5.1, 5.3.
 *   GF(2^128)  -- SP 800-38D sec. 6.3, bit-serial product (Algorithm 1).
 *   GHASH      -- SP 800-38D sec. 6.4, sequential Horner: Y_i = (Y_{i-1}^X_i)*H.
 *   GCTR       -- SP 800-38D sec. 6.5 with inc32 (sec. 6.2).
 *   GCM-AE/AD  -- SP 800-38D sec. 7.1 / 7.2: any IV length (J0 = IV||0^31||1
 *                 for 96 bits, else GHASH of the padded IV and its length,
 *                 sec. 7.1 step 2); tags of t = 128, 120, 112, 104, 96, 64
 *                 or 32 bits (sec. 5.2.1.2), T = MSB_t of the full tag.
 *   AES-GCM-SIV -- RFC 8452 sec. 3-5 (the misuse-resistant alternative the
 *                 paper names under future directions): POLYVAL from its own
 *                 field definition, per-nonce key derivation, tag, and the
 *                 little-endian 32-bit counter; 16- or 32-byte keys, 12-byte
 *                 nonces.
 *
 * Readings where the paper is silent (listed in full in the design notes):
 *   - key sizes 16/24/32 bytes accepted (the paper uses AES-128 only);
 *   - IVs are whole bytes, 1 .. 2^61 - 1 of them (the paper uses 96-bit
 *     nonces; SP 800-38D allows any length from 1 bit); tags are 16 bytes
 *     unless a truncated length is given;
 *   - on a tag mismatch the plaintext output is zero-filled (the paper's
 *     payload-suppression behaviour) and *accept is 0;
 *   - tags are compared over all t bytes without early exit.
 *
 * Parity pins (all in tests/test_oracle_*.py): exhaustive GF(2^8) inverse,
 * S-box invariants, single-block equality with OpenSSL's AES-ECB, the
 * GF(2^128) product on all 128x128 basis pairs against an independent
 * polynomial formulation, field axioms, Horner == closed form == every tree
 * bracketing, full GCM equality with OpenSSL's EVP AES-GCM, round trip and
 * single-bit-flip rejection; for GCM-SIV (tests/test_oracle_siv_pins.py):
 * POLYVAL's product against an integer formulation and closed forms,
 * POLYVAL against OpenSSL's GHASH through RFC 8452 appendix A's byte
 * reversal identity, derivation / tag / counter keystream (including a
 * counter wrap) against OpenSSL's AES-ECB, and the AEAD properties.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <pthread.h>

/* ------------------------------------------------------------------ */
/* GF(2^8), FIPS-197 sec. 4.2                                          */
/* ------------------------------------------------------------------ */

/* multiplication by x: shift left, reduce by m(x) = x^8+x^4+x^3+x+1 (0x11B) */
static uint8_t gf8_xtime(uint8_t a)
{
    return (uint8_t)((a << 1) ^ ((a & 0x80) ? 0x1B : 0x00));
}

/* shift-and-add product: sum over set bits i of b of a * x^i */
static uint8_t gf8_mul(uint8_t a, uint8_t b)
{
    uint8_t p = 0;
    while (b) {
        if (b & 1)
            p ^= a;
        a = gf8_xtime(a);
        b >>= 1;
    }
    return p;
}

/* inverse as a^254 (a^255 = 1 for a != 0); gives 0 for a = 0 as FIPS-197 asks */
static uint8_t gf8_inv(uint8_t a)
{
    uint8_t result = 1, base = a;
    unsigned e = 254;
    while (e) {
        if (e & 1)
            result = gf8_mul(result, base);
        base = gf8_mul(base, base);
        e >>= 1;
    }
    return result;
}

/* FIPS-197 sec. 5.1.1 affine transform:
 * b'_i = b_i ^ b_{(i+4)%8} ^ b_{(i+5)%8} ^ b_{(i+6)%8} ^ b_{(i+7)%8} ^ c_i,  c = 0x63 */
static uint8_t aes_affine(uint8_t b)
{
    const uint8_t c = 0x63;
    uint8_t out = 0;
    for (int i = 0; i < 8; i++) {
        int bit = ((b >> i) & 1) ^ ((b >> ((i + 4) % 8)) & 1) ^ ((b >> ((i + 5) % 8)) & 1) ^
                  ((b >> ((i + 6) % 8)) & 1) ^ ((b >> ((i + 7) % 8)) & 1) ^ ((c >> i) & 1);
        out |= (uint8_t)(bit << i);
    }
    return out;
}

static uint8_t SBOX[256];
static uint8_t INV_SBOX[256];
static pthread_once_t sbox_once = PTHREAD_ONCE_INIT;

static void build_sbox(void)
{
    for (int a = 0; a < 256; a++) {
        uint8_t s = aes_affine(gf8_inv((uint8_t)a));
        SBOX[a] = s;
        INV_SBOX[s] = (uint8_t)a;
    }
}

static void ensure_sbox(void) { pthread_once(&sbox_once, build_sbox); }

/* ------------------------------------------------------------------ */
/* AES, FIPS-197 sec. 5                                                */
/* ------------------------------------------------------------------ */

#define AES_MAX_NR 14
#define AES_MAX_WORDS (4 * (AES_MAX_NR + 1))

/* returns Nr, or 0 for an unsupported key length.  w holds 4*(Nr+1) words of 4 bytes. */
static int key_expansion(const uint8_t *key, size_t key_len, uint8_t w[AES_MAX_WORDS][4])
{
    int nk;
    if (key_len == 16)
        nk = 4;
    else if (key_len == 24)
        nk = 6;
    else if (key_len == 32)
        nk = 8;
    else
        return 0;
    int nr = nk + 6;
    ensure_sbox();

    for (int i = 0; i < nk; i++)
        for (int j = 0; j < 4; j++)
            w[i][j] = key[4 * i + j];

    uint8_t rcon = 0x01; /* Rcon[i/Nk] = (x^(i/Nk - 1), 0, 0, 0) */
    for (int i = nk; i < 4 * (nr + 1); i++) {
        uint8_t temp[4];
        memcpy(temp, w[i - 1], 4);
        if (i % nk == 0) {
            /* RotWord then SubWord then xor Rcon */
            uint8_t t0 = temp[0];
            temp[0] = temp[1];
            temp[1] = temp[2];
            temp[2] = temp[3];
            temp[3] = t0;
            for (int j = 0; j < 4; j++)
                temp[j] = SBOX[temp[j]];
            temp[0] ^= rcon;
            rcon = gf8_xtime(rcon);
        } else if (nk > 6 && i % nk == 4) {
            for (int j = 0; j < 4; j++)
                temp[j] = SBOX[temp[j]];
        }
        for (int j = 0; j < 4; j++)
            w[i][j] = w[i - nk][j] ^ temp[j];
    }
    return nr;
}

/* state[r][c] = in[r + 4c] */
static void add_round_key(uint8_t st[4][4], uint8_t w[AES_MAX_WORDS][4], int round)
{
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            st[r][c] ^= w[4 * round + c][r];
}

static void sub_bytes(uint8_t st[4][4])
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            st[r][c] = SBOX[st[r][c]];
}

static void inv_sub_bytes(uint8_t st[4][4])
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            st[r][c] = INV_SBOX[st[r][c]];
}

/* row r is rotated left by r positions */
static void shift_rows(uint8_t st[4][4])
{
    for (int r = 1; r < 4; r++) {
        uint8_t row[4];
        for (int c = 0; c < 4; c++)
            row[c] = st[r][(c + r) % 4];
        memcpy(st[r], row, 4);
    }
}

static void inv_shift_rows(uint8_t st[4][4])
{
    for (int r = 1; r < 4; r++) {
        uint8_t row[4];
        for (int c = 0; c < 4; c++)
            row[(c + r) % 4] = st[r][c];
        memcpy(st[r], row, 4);
    }
}

/* each column times the circulant matrix with first row (02 03 01 01) */
static void mix_columns(uint8_t st[4][4])
{
    for (int c = 0; c < 4; c++) {
        uint8_t a0 = st[0][c], a1 = st[1][c], a2 = st[2][c], a3 = st[3][c];
        st[0][c] = gf8_mul(0x02, a0) ^ gf8_mul(0x03, a1) ^ a2 ^ a3;
        st[1][c] = a0 ^ gf8_mul(0x02, a1) ^ gf8_mul(0x03, a2) ^ a3;
        st[2][c] = a0 ^ a1 ^ gf8_mul(0x02, a2) ^ gf8_mul(0x03, a3);
        st[3][c] = gf8_mul(0x03, a0) ^ a1 ^ a2 ^ gf8_mul(0x02, a3);
    }
}

/* inverse circulant, first row (0e 0b 0d 09) */
static void inv_mix_columns(uint8_t st[4][4])
{
    for (int c = 0; c < 4; c++) {
        uint8_t a0 = st[0][c], a1 = st[1][c], a2 = st[2][c], a3 = st[3][c];
        st[0][c] = gf8_mul(0x0e, a0) ^ gf8_mul(0x0b, a1) ^ gf8_mul(0x0d, a2) ^ gf8_mul(0x09, a3);
        st[1][c] = gf8_mul(0x09, a0) ^ gf8_mul(0x0e, a1) ^ gf8_mul(0x0b, a2) ^ gf8_mul(0x0d, a3);
        st[2][c] = gf8_mul(0x0d, a0) ^ gf8_mul(0x09, a1) ^ gf8_mul(0x0e, a2) ^ gf8_mul(0x0b, a3);
        st[3][c] = gf8_mul(0x0b, a0) ^ gf8_mul(0x0d, a1) ^ gf8_mul(0x09, a2) ^ gf8_mul(0x0e, a3);
    }
}

/* FIPS-197 sec. 5.1 Cipher */
static void aes_cipher(uint8_t w[AES_MAX_WORDS][4], int nr, const uint8_t in[16], uint8_t out[16])
{
    uint8_t st[4][4];
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            st[r][c] = in[r + 4 * c];
    add_round_key(st, w, 0);
    for (int round = 1; round < nr; round++) {
        sub_bytes(st);
        shift_rows(st);
        mix_columns(st);
        add_round_key(st, w, round);
    }
    sub_bytes(st);
    shift_rows(st);
    add_round_key(st, w, nr);
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            out[r + 4 * c] = st[r][c];
}

/* FIPS-197 sec. 5.3 InvCipher -- only used by the round-trip pin */
static void aes_inv_cipher(uint8_t w[AES_MAX_WORDS][4], int nr, const uint8_t in[16], uint8_t out[16])
{
    uint8_t st[4][4];
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            st[r][c] = in[r + 4 * c];
    add_round_key(st, w, nr);
    for (int round = nr - 1; round >= 1; round--) {
        inv_shift_rows(st);
        inv_sub_bytes(st);
        add_round_key(st, w, round);
        inv_mix_columns(st);
    }
    inv_shift_rows(st);
    inv_sub_bytes(st);
    add_round_key(st, w, 0);
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            out[r + 4 * c] = st[r][c];
}

/* ------------------------------------------------------------------ */
/* GF(2^128), SP 800-38D sec. 6.3                                      */
/* bit i of a block is bit (7 - i%8) of byte i/8; bit 0 is the         */
/* coefficient of x^0.  R = 11100001 || 0^120.                         */
/* ------------------------------------------------------------------ */

static int block_bit(const uint8_t x[16], int i)
{
    return (x[i / 8] >> (7 - (i % 8))) & 1;
}

/* V >> 1 moves every bit to the next higher index (towards byte 15) */
static void block_shift_right1(uint8_t v[16])
{
    for (int k = 15; k > 0; k--)
        v[k] = (uint8_t)((v[k] >> 1) | (v[k - 1] << 7));
    v[0] >>= 1;
}

static void gf128_mul(const uint8_t x[16], const uint8_t y[16], uint8_t out[16])
{
    uint8_t z[16] = {0};
    uint8_t v[16];
    memcpy(v, y, 16);
    for (int i = 0; i < 128; i++) {
        if (block_bit(x, i))
            for (int k = 0; k < 16; k++)
                z[k] ^= v[k];
        int lsb = v[15] & 1; /* bit 127 of V */
        block_shift_right1(v);
        if (lsb)
            v[0] ^= 0xE1;
    }
    memcpy(out, z, 16);
}

/* ------------------------------------------------------------------ */
/* GHASH (sec. 6.4): Y_0 = 0, Y_i = (Y_{i-1} ^ X_i) * H                */
/* Here fed incrementally so that A, C and the length block can be    */
/* streamed without building the concatenation in memory.             */
/* ------------------------------------------------------------------ */

static void ghash_absorb_block(uint8_t y[16], const uint8_t h[16], const uint8_t x[16])
{
    uint8_t t[16];
    for (int k = 0; k < 16; k++)
        t[k] = y[k] ^ x[k];
    gf128_mul(t, h, y);
}

/* absorbs data zero-padded on the right to a whole number of blocks */
static void ghash_absorb_padded(uint8_t y[16], const uint8_t h[16], const uint8_t *data, uint64_t len)
{
    uint64_t off = 0;
    while (off < len) {
        uint8_t blk[16] = {0};
        uint64_t take = len - off < 16 ? len - off : 16;
        memcpy(blk, data + off, (size_t)take);
        ghash_absorb_block(y, h, blk);
        off += take;
    }
}

/* ------------------------------------------------------------------ */
/* inc32 and GCTR (sec. 6.2, 6.5)                                      */
/* ------------------------------------------------------------------ */

static void inc32(uint8_t cb[16])
{
    uint32_t c = ((uint32_t)cb[12] << 24) | ((uint32_t)cb[13] << 16) | ((uint32_t)cb[14] << 8) | cb[15];
    c += 1; /* mod 2^32 */
    cb[12] = (uint8_t)(c >> 24);
    cb[13] = (uint8_t)(c >> 16);
    cb[14] = (uint8_t)(c >> 8);
    cb[15] = (uint8_t)c;
}

static void gctr(uint8_t w[AES_MAX_WORDS][4], int nr, const uint8_t icb[16], const uint8_t *x, uint64_t len,
                 uint8_t *y)
{
    uint8_t cb[16];
    memcpy(cb, icb, 16);
    uint64_t off = 0;
    while (off < len) {
        uint8_t ks[16];
        aes_cipher(w, nr, cb, ks);
        uint64_t take = len - off < 16 ? len - off : 16; /* MSB_len of the last keystream block */
        for (uint64_t k = 0; k < take; k++)
            y[off + k] = x[off + k] ^ ks[k];
        inc32(cb);
        off += take;
    }
}

/* ------------------------------------------------------------------ */
/* GCM-AE / GCM-AD (sec. 7.1, 7.2), 96-bit IV only                     */
/* ------------------------------------------------------------------ */

enum {
    ORACLE_OK = 0,
    ORACLE_E_KEYLEN = -2,
    ORACLE_E_IVLEN = -3,
    ORACLE_E_TOOLONG = -4,
    ORACLE_E_ARG = -1,
};

/* |P| <= 2^39 - 256 bits  =>  len <= 2^36 - 32 bytes */
#define ORACLE_MAX_LEN ((((uint64_t)1) << 36) - 32)
/* |A| <= 2^64 - 1 bits  =>  aad_len < 2^61 bytes */
#define ORACLE_MAX_AAD ((((uint64_t)1) << 61) - 1)
/* 1 <= len(IV) <= 2^64 - 1 bits, in whole bytes */
#define ORACLE_MAX_IV ((((uint64_t)1) << 61) - 1)

static void put_be64(uint8_t *p, uint64_t v)
{
    for (int k = 0; k < 8; k++)
        p[k] = (uint8_t)(v >> (56 - 8 * k));
}

/* S = GHASH_H(A || 0^v || C || 0^u || [len(A)]_64 || [len(C)]_64), lengths in bits */
static void gcm_hash(const uint8_t h[16], const uint8_t *aad, uint64_t aad_len, const uint8_t *c, uint64_t len,
                     uint8_t s[16])
{
    uint8_t y[16] = {0};
    ghash_absorb_padded(y, h, aad, aad_len);
    ghash_absorb_padded(y, h, c, len);
    uint8_t lb[16];
    put_be64(lb, aad_len * 8);
    put_be64(lb + 8, len * 8);
    ghash_absorb_block(y, h, lb);
    memcpy(s, y, 16);
}

static int gcm_setup(const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len, uint64_t aad_len,
                     uint64_t len, uint8_t w[AES_MAX_WORDS][4], int *nr, uint8_t h[16], uint8_t j0[16])
{
    if (!key || !iv)
        return ORACLE_E_ARG;
    *nr = key_expansion(key, key_len, w);
    if (*nr == 0)
        return ORACLE_E_KEYLEN;
    if (iv_len == 0 || iv_len > ORACLE_MAX_IV)
        return ORACLE_E_IVLEN;
    if (len > ORACLE_MAX_LEN || aad_len > ORACLE_MAX_AAD)
        return ORACLE_E_TOOLONG;
    uint8_t zero[16] = {0};
    aes_cipher(w, *nr, zero, h); /* H = CIPH_K(0^128) */
    if (iv_len == 12) {
        memcpy(j0, iv, 12); /* J0 = IV || 0^31 || 1 */
        j0[12] = 0;
        j0[13] = 0;
        j0[14] = 0;
        j0[15] = 1;
    } else {
        /* J0 = GHASH_H(IV || 0^(s+64) || [len(IV)]_64), s pads IV to whole blocks */
        uint8_t y[16] = {0}, lb[16];
        ghash_absorb_padded(y, h, iv, iv_len);
        put_be64(lb, 0);
        put_be64(lb + 8, (uint64_t)iv_len * 8);
        ghash_absorb_block(y, h, lb);
        memcpy(j0, y, 16);
    }
    return ORACLE_OK;
}

int oracle_gcm_encrypt(const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len, const uint8_t *aad,
                       uint64_t aad_len, const uint8_t *pt, uint64_t len, uint8_t *ct, uint8_t tag[16])
{
    uint8_t w[AES_MAX_WORDS][4], h[16], j0[16];
    int nr;
    int rc = gcm_setup(key, key_len, iv, iv_len, aad_len, len, w, &nr, h, j0);
    if (rc)
        return rc;
    if ((len && (!pt || !ct)) || (aad_len && !aad) || !tag)
        return ORACLE_E_ARG;
    uint8_t icb[16];
    memcpy(icb, j0, 16);
    inc32(icb);
    gctr(w, nr, icb, pt, len, ct); /* C = GCTR_K(inc32(J0), P) */
    uint8_t s[16], ekj0[16];
    gcm_hash(h, aad, aad_len, ct, len, s);
    aes_cipher(w, nr, j0, ekj0);
    for (int k = 0; k < 16; k++)
        tag[k] = ekj0[k] ^ s[k]; /* T = MSB_128(GCTR_K(J0, S)) */
    return ORACLE_OK;
}

/* tag lengths of sec. 5.2.1.2, in bytes */
static int valid_tag_len(size_t t) { return t == 16 || t == 15 || t == 14 || t == 13 || t == 12 || t == 8 || t == 4; }

/* GCM-AD with a tag of tag_len bytes: accept iff T equals MSB_t(GCTR_K(J0, S)) */
int oracle_gcm_decrypt_verify_t(const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                                const uint8_t *aad, uint64_t aad_len, const uint8_t *ct, uint64_t len,
                                const uint8_t *tag, size_t tag_len, uint8_t *pt, int *accept)
{
    uint8_t w[AES_MAX_WORDS][4], h[16], j0[16];
    int nr;
    int rc = gcm_setup(key, key_len, iv, iv_len, aad_len, len, w, &nr, h, j0);
    if (rc)
        return rc;
    if ((len && (!pt || !ct)) || (aad_len && !aad) || !tag || !accept || !valid_tag_len(tag_len))
        return ORACLE_E_ARG;
    uint8_t s[16], ekj0[16];
    gcm_hash(h, aad, aad_len, ct, len, s);
    aes_cipher(w, nr, j0, ekj0);
    uint8_t diff = 0;
    for (size_t k = 0; k < tag_len; k++)
        diff |= (uint8_t)((ekj0[k] ^ s[k]) ^ tag[k]);
    if (diff == 0) {
        uint8_t icb[16];
        memcpy(icb, j0, 16);
        inc32(icb);
        gctr(w, nr, icb, ct, len, pt);
        *accept = 1;
    } else {
        if (len)
            memset(pt, 0, (size_t)len);
        *accept = 0;
    }
    return ORACLE_OK;
}

int oracle_gcm_decrypt_verify(const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                              const uint8_t *aad, uint64_t aad_len, const uint8_t *ct, uint64_t len,
                              const uint8_t tag[16], uint8_t *pt, int *accept)
{
    return oracle_gcm_decrypt_verify_t(key, key_len, iv, iv_len, aad, aad_len, ct, len, tag, 16, pt, accept);
}

/* J0 for an IV (sec. 7.1 step 2), exposed for the pins */
int oracle_gcm_j0(const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len, uint8_t out[16])
{
    uint8_t w[AES_MAX_WORDS][4], h[16];
    int nr;
    return gcm_setup(key, key_len, iv, iv_len, 0, 0, w, &nr, h, out);
}

/* ------------------------------------------------------------------ */
/* Primitive entry points exposed for the pins                         */
/* ------------------------------------------------------------------ */

uint8_t oracle_gf8_mul(uint8_t a, uint8_t b) { return gf8_mul(a, b); }
uint8_t oracle_gf8_inv(uint8_t a) { return gf8_inv(a); }
uint8_t oracle_gf8_xtime(uint8_t a) { return gf8_xtime(a); }

void oracle_sbox(uint8_t out[256])
{
    ensure_sbox();
    memcpy(out, SBOX, 256);
}

void oracle_inv_sbox(uint8_t out[256])
{
    ensure_sbox();
    memcpy(out, INV_SBOX, 256);
}

/* writes 16*(Nr+1) bytes of round keys (word i at bytes 4i..4i+3); returns Nr or 0 */
int oracle_key_expand(const uint8_t *key, size_t key_len, uint8_t *w_out)
{
    uint8_t w[AES_MAX_WORDS][4];
    int nr = key_expansion(key, key_len, w);
    if (nr)
        memcpy(w_out, w, (size_t)(16 * (nr + 1)));
    return nr;
}

int oracle_aes_encrypt_block(const uint8_t *key, size_t key_len, const uint8_t in[16], uint8_t out[16])
{
    uint8_t w[AES_MAX_WORDS][4];
    int nr = key_expansion(key, key_len, w);
    if (!nr)
        return ORACLE_E_KEYLEN;
    aes_cipher(w, nr, in, out);
    return ORACLE_OK;
}

int oracle_aes_decrypt_block(const uint8_t *key, size_t key_len, const uint8_t in[16], uint8_t out[16])
{
    uint8_t w[AES_MAX_WORDS][4];
    int nr = key_expansion(key, key_len, w);
    if (!nr)
        return ORACLE_E_KEYLEN;
    aes_inv_cipher(w, nr, in, out);
    return ORACLE_OK;
}

void oracle_gf128_mul(const uint8_t x[16], const uint8_t y[16], uint8_t out[16]) { gf128_mul(x, y, out); }

/* GHASH over nblocks whole blocks (the paper's serial recurrence) */
void oracle_ghash(const uint8_t h[16], const uint8_t *x, uint64_t nblocks, uint8_t out[16])
{
    uint8_t y[16] = {0};
    for (uint64_t i = 0; i < nblocks; i++)
        ghash_absorb_block(y, h, x + 16 * i);
    memcpy(out, y, 16);
}

/* the full GCM hash input string is not materialised; this returns S for (A, C) */
void oracle_gcm_hash(const uint8_t h[16], const uint8_t *aad, uint64_t aad_len, const uint8_t *c, uint64_t len,
                     uint8_t s[16])
{
    gcm_hash(h, aad, aad_len, c, len, s);
}

/* raw GCTR keystream application from an arbitrary initial counter block */
int oracle_gctr(const uint8_t *key, size_t key_len, const uint8_t icb[16], const uint8_t *x, uint64_t len,
                uint8_t *y)
{
    uint8_t w[AES_MAX_WORDS][4];
    int nr = key_expansion(key, key_len, w);
    if (!nr)
        return ORACLE_E_KEYLEN;
    gctr(w, nr, icb, x, len, y);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* AES-GCM-SIV (RFC 8452), the nonce-misuse-resistant AEAD the paper   */
/* names as an alternative (Discussion and Future Work, "Future        */
/* Directions", item 4).                                               */
/*                                                                     */
/* POLYVAL (RFC 8452 sec. 3): blocks are little-endian polynomials --  */
/* byte k bit j (value 1<<j) is the coefficient of x^(8k+j) -- in      */
/* GF(2)[x] / P, P = x^128 + x^127 + x^126 + x^121 + 1;                */
/* dot(a, b) = a * b * x^-128; S_0 = 0, S_j = dot(S_(j-1) ^ X_j, H).   */
/* ------------------------------------------------------------------ */

/* v * x mod P: shift towards byte 15; the x^128 carry folds back as   */
/* x^127 + x^126 + x^121 + 1                                           */
static void pv_mul_x(uint8_t v[16])
{
    int carry = v[15] >> 7;
    for (int k = 15; k > 0; k--)
        v[k] = (uint8_t)((v[k] << 1) | (v[k - 1] >> 7));
    v[0] = (uint8_t)(v[0] << 1);
    if (carry) {
        v[0] ^= 0x01;
        v[15] ^= 0xC2;
    }
}

/* v * x^-1 mod P: if the x^0 coefficient is set, add P first (making  */
/* v divisible by x), then shift towards byte 0; P / x contributes     */
/* x^127 + x^126 + x^125 + x^120                                       */
static void pv_mul_xinv(uint8_t v[16])
{
    int low = v[0] & 1;
    for (int k = 0; k < 15; k++)
        v[k] = (uint8_t)((v[k] >> 1) | (v[k + 1] << 7));
    v[15] >>= 1;
    if (low)
        v[15] ^= 0xE1;
}

/* a * b mod P, shift-and-add over the bits of a */
static void pv_mul(const uint8_t a[16], const uint8_t b[16], uint8_t out[16])
{
    uint8_t z[16] = {0}, v[16];
    memcpy(v, b, 16);
    for (int i = 0; i < 128; i++) {
        if ((a[i / 8] >> (i % 8)) & 1)
            for (int k = 0; k < 16; k++)
                z[k] ^= v[k];
        pv_mul_x(v);
    }
    memcpy(out, z, 16);
}

static void pv_dot(const uint8_t a[16], const uint8_t b[16], uint8_t out[16])
{
    uint8_t t[16];
    pv_mul(a, b, t);
    for (int i = 0; i < 128; i++)
        pv_mul_xinv(t);
    memcpy(out, t, 16);
}

static void polyval_absorb_block(uint8_t s[16], const uint8_t h[16], const uint8_t x[16])
{
    uint8_t t[16];
    for (int k = 0; k < 16; k++)
        t[k] = s[k] ^ x[k];
    pv_dot(t, h, s);
}

static void polyval_absorb_padded(uint8_t s[16], const uint8_t h[16], const uint8_t *data, uint64_t len)
{
    uint64_t off = 0;
    while (off < len) {
        uint8_t blk[16] = {0};
        uint64_t take = len - off < 16 ? len - off : 16;
        memcpy(blk, data + off, (size_t)take);
        polyval_absorb_block(s, h, blk);
        off += take;
    }
}

static void put_le64(uint8_t *p, uint64_t v)
{
    for (int k = 0; k < 8; k++)
        p[k] = (uint8_t)(v >> (8 * k));
}

/* RFC 8452 sec. 6: P_MAX = A_MAX = 2^36 bytes */
#define ORACLE_SIV_MAX ((((uint64_t)1) << 36))

/* sec. 4: message_authentication_key = first halves of AES_KGK(LE32(0)||N),
 * AES_KGK(LE32(1)||N); message_encryption_key = those of LE32(2), LE32(3)
 * (and LE32(4), LE32(5) for a 256-bit key-generating key) */
static int siv_derive(const uint8_t *kgk, size_t kgk_len, const uint8_t nonce[12], uint8_t auth[16], uint8_t *enc)
{
    if (kgk_len != 16 && kgk_len != 32)
        return ORACLE_E_KEYLEN;
    uint8_t w[AES_MAX_WORDS][4];
    int nr = key_expansion(kgk, kgk_len, w);
    int nblk = kgk_len == 16 ? 4 : 6;
    for (int i = 0; i < nblk; i++) {
        uint8_t in[16], out[16];
        put_le64(in, (uint64_t)i); /* LE32(i); bytes 4..7 are overwritten by the nonce */
        memcpy(in + 4, nonce, 12);
        aes_cipher(w, nr, in, out);
        memcpy(i < 2 ? auth + 8 * i : enc + 8 * (i - 2), out, 8);
    }
    return ORACLE_OK;
}

/* S_s = POLYVAL(auth, pad(A) || pad(P) || LE64(8|A|) || LE64(8|P|)), then
 * the nonce XORed into bytes 0..11 and the top bit of byte 15 cleared;
 * tag = AES_enc(S_s) */
static void siv_tag(const uint8_t auth[16], uint8_t we[AES_MAX_WORDS][4], int nre, const uint8_t nonce[12],
                    const uint8_t *aad, uint64_t aad_len, const uint8_t *pt, uint64_t len, uint8_t tag[16])
{
    uint8_t s[16] = {0}, lb[16];
    polyval_absorb_padded(s, auth, aad, aad_len);
    polyval_absorb_padded(s, auth, pt, len);
    put_le64(lb, aad_len * 8);
    put_le64(lb + 8, len * 8);
    polyval_absorb_block(s, auth, lb);
    for (int k = 0; k < 12; k++)
        s[k] ^= nonce[k];
    s[15] &= 0x7F;
    aes_cipher(we, nre, s, tag);
}

/* counter block = tag with the top bit of byte 15 set; bytes 0..3 are a
 * little-endian 32-bit counter incremented mod 2^32 per block */
static void siv_ctr(uint8_t we[AES_MAX_WORDS][4], int nre, const uint8_t tag[16], const uint8_t *x, uint64_t len,
                    uint8_t *y)
{
    uint8_t cb[16];
    memcpy(cb, tag, 16);
    cb[15] |= 0x80;
    uint64_t off = 0;
    while (off < len) {
        uint8_t ks[16];
        aes_cipher(we, nre, cb, ks);
        uint64_t take = len - off < 16 ? len - off : 16;
        for (uint64_t k = 0; k < take; k++)
            y[off + k] = x[off + k] ^ ks[k];
        uint32_t c = (uint32_t)cb[0] | ((uint32_t)cb[1] << 8) | ((uint32_t)cb[2] << 16) | ((uint32_t)cb[3] << 24);
        c += 1;
        cb[0] = (uint8_t)c;
        cb[1] = (uint8_t)(c >> 8);
        cb[2] = (uint8_t)(c >> 16);
        cb[3] = (uint8_t)(c >> 24);
        off += take;
    }
}

static int siv_setup(const uint8_t *kgk, size_t kgk_len, const uint8_t *nonce, size_t nonce_len, uint64_t aad_len,
                     uint64_t len, uint8_t auth[16], uint8_t we[AES_MAX_WORDS][4], int *nre)
{
    if (!kgk || !nonce)
        return ORACLE_E_ARG;
    if (kgk_len != 16 && kgk_len != 32)
        return ORACLE_E_KEYLEN;
    if (nonce_len != 12)
        return ORACLE_E_IVLEN;
    if (len > ORACLE_SIV_MAX || aad_len > ORACLE_SIV_MAX)
        return ORACLE_E_TOOLONG;
    uint8_t enc[32];
    siv_derive(kgk, kgk_len, nonce, auth, enc);
    *nre = key_expansion(enc, kgk_len, we);
    return ORACLE_OK;
}

int oracle_gcm_siv_encrypt(const uint8_t *kgk, size_t kgk_len, const uint8_t *nonce, size_t nonce_len,
                           const uint8_t *aad, uint64_t aad_len, const uint8_t *pt, uint64_t len, uint8_t *ct,
                           uint8_t tag[16])
{
    uint8_t auth[16], we[AES_MAX_WORDS][4];
    int nre;
    int rc = siv_setup(kgk, kgk_len, nonce, nonce_len, aad_len, len, auth, we, &nre);
    if (rc)
        return rc;
    if ((len && (!pt || !ct)) || (aad_len && !aad) || !tag)
        return ORACLE_E_ARG;
    siv_tag(auth, we, nre, nonce, aad, aad_len, pt, len, tag);
    siv_ctr(we, nre, tag, pt, len, ct);
    return ORACLE_OK;
}

/* decrypt with the counter taken from the received tag, recompute the tag
 * over the recovered plaintext, compare all 16 bytes; on mismatch the
 * plaintext output is zero-filled and *accept is 0 */
int oracle_gcm_siv_decrypt_verify(const uint8_t *kgk, size_t kgk_len, const uint8_t *nonce, size_t nonce_len,
                                  const uint8_t *aad, uint64_t aad_len, const uint8_t *ct, uint64_t len,
                                  const uint8_t tag[16], uint8_t *pt, int *accept)
{
    uint8_t auth[16], we[AES_MAX_WORDS][4];
    int nre;
    int rc = siv_setup(kgk, kgk_len, nonce, nonce_len, aad_len, len, auth, we, &nre);
    if (rc)
        return rc;
    if ((len && (!pt || !ct)) || (aad_len && !aad) || !tag || !accept)
        return ORACLE_E_ARG;
    siv_ctr(we, nre, tag, ct, len, pt);
    uint8_t want[16];
    siv_tag(auth, we, nre, nonce, aad, aad_len, pt, len, want);
    uint8_t diff = 0;
    for (int k = 0; k < 16; k++)
        diff |= (uint8_t)(want[k] ^ tag[k]);
    *accept = diff == 0;
    if (!*accept && len)
        memset(pt, 0, (size_t)len);
    return ORACLE_OK;
}

/* the derived per-nonce keys (enc gets kgk_len bytes) */
int oracle_gcm_siv_derive(const uint8_t *kgk, size_t kgk_len, const uint8_t nonce[12], uint8_t auth[16],
                          uint8_t *enc)
{
    if (!kgk || !nonce || !auth || !enc)
        return ORACLE_E_ARG;
    return siv_derive(kgk, kgk_len, nonce, auth, enc);
}

void oracle_polyval(const uint8_t h[16], const uint8_t *x, uint64_t nblocks, uint8_t out[16])
{
    uint8_t s[16] = {0};
    for (uint64_t i = 0; i < nblocks; i++)
        polyval_absorb_block(s, h, x + 16 * i);
    memcpy(out, s, 16);
}

void oracle_pv_mul(const uint8_t a[16], const uint8_t b[16], uint8_t out[16]) { pv_mul(a, b, out); }
