/*
 * gcm_mi355.h -- C ABI of the MI355X (gfx950) AES-GCM library.
 *
 * The library computes AES-GCM authenticated encryption and decryption with
 * verification, as fixed by NIST SP 800-38D over FIPS-197 AES (the paper's
 * "Cryptographic Protocol: AES-GCM" section), with the GHASH recurrence
 * (the paper's serial equation for Y_i) re-bracketed as a reduction tree over
 * GF(2^128) ("Parallel GHASH Reduction" section, its tree figure, and the
 * two-phase map-reduce of "Scalable MapReduce for Massive Files").
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Return value: GCM_OK (0) on success, a negative GCM_E_* code otherwise
 *    (the paper's API table: 0 success, < 0 system error).  A failed
 *    authentication is NOT an error: decrypt-verify returns GCM_OK with the
 *    accept flag 0 and the plaintext output zero-filled (the paper's payload
 *    suppression in "Policy Enforcement and Granular Access").
 *  - On an error return nothing has been launched and no output was touched.
 *    gcm_last_error() returns a thread-local message for the last error.
 *  - Pointers named *_d are DEVICE pointers on the context's device (for
 *    example torch.Tensor.data_ptr()); all other pointers are HOST pointers.
 *    Device payload pointers (aad_d, in, out) must be 16-byte aligned.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    it in stream order.
 *  - Keys are 16, 24 or 32 bytes (AES-128/192/256).  IVs are 12 bytes (the
 *    paper's 96-bit nonces, J0 = IV || 0^31 || 1) or, on the single-message
 *    GCM calls (one-shot, asynchronous, host pipeline), any length from 1 to
 *    1024 bytes (SP 800-38D sec. 7.1 step 2: J0 = GHASH_H(IV || 0-pad ||
 *    0^64 || [len(IV)]_64), computed on the device); batches, the serving
 *    loop and the counter-mode-only calls take 12-byte IVs.  Data block i
 *    (0-based) uses counter inc32^(i+1)(J0), independent of launch geometry
 *    (the paper's geometry-agnostic counter mapping).  Tags are 16 bytes
 *    except on the _ex calls (truncated tags).
 *  - Limits (SP 800-38D): len <= 2^36 - 32 bytes, aad_len < 2^61 bytes,
 *    else GCM_E_TOOLONG.
 *  - in == out is allowed (in place); partially overlapping in/out is
 *    GCM_E_ALIAS, and so is an output that overlaps the AAD, the tag or the
 *    accept flag (these are read or written while the output is written).
 *  - The caller owns every buffer.  The context owns its key table and its
 *    internal scratch.  No call keeps a caller pointer after it returns.
 *  - No C++ exception crosses this interface: a failed host allocation inside
 *    the runtime returns GCM_E_NOMEM, any other host runtime failure
 *    GCM_E_INTERNAL, with the message in gcm_last_error().
 */
#ifndef GCM_MI355_H
#define GCM_MI355_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GCM_OK 0
#define GCM_E_ARG (-1)     /* null pointer, bad size, bad op, misaligned pointer */
#define GCM_E_KEYLEN (-2)  /* key length not 16, 24 or 32 */
#define GCM_E_IVLEN (-3)   /* IV length not allowed by the call (see the conventions above) */
#define GCM_E_TOOLONG (-4) /* len or aad_len beyond the SP 800-38D limits */
#define GCM_E_NOMEM (-5)   /* device or pinned allocation failed / budget exceeded */
#define GCM_E_HIP (-6)     /* a HIP runtime call failed */
#define GCM_E_BUSY (-7)    /* no free key slot / serving queue full */
#define GCM_E_ALIAS (-8)   /* in and out overlap without being equal, or out overlaps AAD / tag / flag */
#define GCM_E_SLOT (-9)    /* key slot index not registered */
#define GCM_E_INTERNAL (-10) /* a host runtime failure other than memory (e.g. a thread that cannot start) */

typedef struct gcm_ctx gcm_ctx;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.
 *   hbm_budget_bytes: upper bound on device memory the context itself may
 *     allocate for key slots and scratch (0 = no bound).
 *   key_slots: number of resident key slots (each holds the round keys, H,
 *     the H^(2^k) power table and the GHASH multiplication tables, about
 *     403 KiB; the paper's precomputed table of powers of H).
 * Builds the AES tables on the device.  *out receives the context. */
int gcm_ctx_create(gcm_ctx **out, int device, uint64_t hbm_budget_bytes, uint32_t key_slots);

/* Wait for all work of the context, then free everything it owns. */
int gcm_ctx_destroy(gcm_ctx *ctx);

/* Thread-local message describing the last error on this thread ("" if none). */
const char *gcm_last_error(void);

/* ---------------------------------------------------------------- keys */

/* Expand `key` into a resident slot on `stream`: AES round keys, H =
 * AES_K(0^128), H^(2^k) for k = 0..47 and the GHASH tables (the paper's
 * H-power precompute, done on the GPU).  *slot_out receives the slot index.
 * The slot is usable by later work on the same stream (or after a sync).
 * GCM_E_BUSY if every slot is taken. */
int gcm_key_register(gcm_ctx *ctx, const uint8_t *key, size_t key_len, uint32_t *slot_out, void *stream);

/* Register n keys with as few launches as possible (the paper's H-power
 * precompute for a whole batch of keys).  keys: the n keys concatenated
 * (host); key_lens[i]: 16, 24 or 32; slots_out[i] receives key i's slot.
 * Either every key gets a slot or none does (GCM_E_BUSY). */
int gcm_key_register_many(gcm_ctx *ctx, const uint8_t *keys, const uint32_t *key_lens, uint32_t n,
                          uint32_t *slots_out, void *stream);

/* Return a slot to the free list.  The caller guarantees no queued work
 * still uses it. */
int gcm_key_release(gcm_ctx *ctx, uint32_t slot);

/* ---------------------------------------------------------------- one-shot, blocking */

/* AES-GCM authenticated encryption (SP 800-38D GCM-AE).
 * key, iv: host.  aad_d (aad_len bytes), pt_d (len bytes), ct_d (len bytes): device.
 * tag_out: host, 16 bytes.  Keys are cached in the context's key table, so a
 * repeated key costs no re-expansion.  Blocks until the tag is on the host. */
int gcm_encrypt(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                const uint8_t *aad_d, uint64_t aad_len, const uint8_t *pt_d, uint64_t len, uint8_t *ct_d,
                uint8_t tag_out[16], void *stream);

/* AES-GCM authenticated decryption (SP 800-38D GCM-AD) with verification.
 * tag: host, 16 bytes (expected tag).  *accept (host) receives 1 if the tag
 * matches (pt_d then holds the plaintext) and 0 otherwise (pt_d is then all
 * zeros).  Tags are compared over all 16 bytes without early exit.  Blocks
 * until the flag is on the host. */
int gcm_decrypt_verify(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                       const uint8_t *aad_d, uint64_t aad_len, const uint8_t *ct_d, uint64_t len,
                       const uint8_t tag[16], uint8_t *pt_d, int *accept, void *stream);

/* gcm_encrypt / gcm_decrypt_verify with a truncated tag of tag_len bytes
 * (SP 800-38D sec. 5.2.1.2: t = 128, 120, 112, 104, 96, or, for the uses
 * its Appendix C allows, 64 or 32 bits; tag_len 16, 15, 14, 13, 12, 8 or 4,
 * else GCM_E_ARG).  Encrypt writes T = MSB_t(full tag) to tag_out (tag_len
 * bytes, host); decrypt-verify compares tag_len bytes (host) without early
 * exit. */
int gcm_encrypt_ex(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                   const uint8_t *aad_d, uint64_t aad_len, const uint8_t *pt_d, uint64_t len, uint8_t *ct_d,
                   uint8_t *tag_out, size_t tag_len, void *stream);
int gcm_decrypt_verify_ex(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                          const uint8_t *aad_d, uint64_t aad_len, const uint8_t *ct_d, uint64_t len,
                          const uint8_t *tag, size_t tag_len, uint8_t *pt_d, int *accept, void *stream);

/* ---------------------------------------------------------------- asynchronous, resident key */

/* Device scratch bytes an asynchronous call on a message of up to `len` data
 * bytes and up to `aad_len` AAD bytes needs (the per-tile partial hashes of
 * the map phase, the block E_K(J0) that the reduce phase adds, and J0 itself
 * for IVs other than 96 bits), under the context's current launch settings:
 * enough for every shorter message as well (the tile count itself is not
 * monotonic in the length).  A workspace may be reused by calls that are
 * ordered on one stream. */
uint64_t gcm_workspace_size(gcm_ctx *ctx, uint64_t len, uint64_t aad_len);

/* Same computation as gcm_encrypt, fully on the device and without host
 * synchronisation: the key comes from a registered slot, the tag is written
 * to tag_d (device, 16 bytes).  workspace_d: device scratch of at least
 * gcm_workspace_size() bytes, 16-byte aligned.  The call enqueues kernels
 * only (no allocation, copy, memset or host wait), so it and
 * gcm_decrypt_verify_async may be captured into a HIP graph once the kernels
 * have been launched eagerly (their code is loaded on first use); a replay
 * reads the buffers' contents at replay time. */
int gcm_encrypt_async(gcm_ctx *ctx, uint32_t slot, const uint8_t *iv, size_t iv_len, const uint8_t *aad_d,
                      uint64_t aad_len, const uint8_t *pt_d, uint64_t len, uint8_t *ct_d, uint8_t *tag_d,
                      void *workspace_d, uint64_t workspace_bytes, void *stream);

/* Same computation as gcm_decrypt_verify on the device: expected tag read
 * from tag_d (device), the accept flag written to accept_d (device int32:
 * 1 accept, 0 reject; on reject pt_d is zero-filled by a later kernel on the
 * same stream). */
int gcm_decrypt_verify_async(gcm_ctx *ctx, uint32_t slot, const uint8_t *iv, size_t iv_len,
                             const uint8_t *aad_d, uint64_t aad_len, const uint8_t *ct_d, uint64_t len,
                             const uint8_t *tag_d, uint8_t *pt_d, int32_t *accept_d, void *workspace_d,
                             uint64_t workspace_bytes, void *stream);

/* gcm_encrypt_async without a workspace argument, for callers that cannot
 * allocate device memory around the call: code being captured into a HIP
 * graph, tight serving loops, harnesses that forbid hipMalloc.  The tile
 * partials, E_K(J0) and J0 live in a fixed device array of
 * GCM_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends (its address is looked up once per device, when the
 * first context on that device is created).  The call itself performs no
 * device or host allocation and no memset: it enqueues the same kernels as
 * gcm_encrypt_async, with tiles enlarged (up to 2^16 blocks, results
 * unchanged) until the partials fit.  A message whose partials still do not
 * fit (beyond every length SP 800-38D allows combined with about 238 MiB of
 * AAD) is GCM_E_NOMEM with nothing launched.  Every call on one device shares
 * that device's array and every value in it is written before it is read
 * within a call, so a call depends on nothing an earlier call left there;
 * but two calls whose work overlaps on one device (different streams, or
 * different contexts) race on it and may produce wrong tags: order them on
 * one stream or synchronise between them.  Arguments, layout and the other
 * errors are those of gcm_encrypt_async. */
#define GCM_NOALLOC_SCRATCH_BYTES ((1ull << 20) + 4096)
int gcm_encrypt_async_noalloc(gcm_ctx *ctx, uint32_t slot, const uint8_t *iv, size_t iv_len, const uint8_t *aad_d,
                              uint64_t aad_len, const uint8_t *pt_d, uint64_t len, uint8_t *ct_d, uint8_t *tag_d,
                              void *stream);

/* ---------------------------------------------------------------- counter mode only, GMAC */

/* AES-CTR without authentication (the paper's CTR-only baseline, the "E2E CTR"
 * column of its GCM-vs-CTR comparison table; "Choice of Cryptographic Mode").
 * out_d = in_d XOR keystream, where data block i (0-based) uses counter
 * inc32^(i+1)(J0) with J0 = IV || 0^31 || 1: the GCTR step of SP 800-38D
 * GCM-AE, so out_d equals gcm_encrypt's ciphertext and the same call
 * decrypts.  No tag, no workspace.  key, iv: host; in_d, out_d: device
 * (len bytes, 16-byte aligned, in_d == out_d allowed).  Blocks until the
 * output is written (the key may come from the context's key cache). */
int gcm_ctr_xcrypt(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                   const uint8_t *in_d, uint64_t len, uint8_t *out_d, void *stream);

/* gcm_ctr_xcrypt with a registered key slot, enqueued on `stream` without
 * host synchronisation. */
int gcm_ctr_async(gcm_ctx *ctx, uint32_t slot, const uint8_t *iv, size_t iv_len, const uint8_t *in_d, uint64_t len,
                  uint8_t *out_d, void *stream);

/* GMAC (SP 800-38D: GCM-AE with an empty plaintext): tag_out (host, 16 B) =
 * GHASH_H(A || 0-pad || [8|A|]_64 || 0^64) XOR E_K(J0) over aad_d (device,
 * aad_len bytes, 16-byte aligned).  Runs only the GHASH map and reduce
 * phases (the scope of the paper's GHASH-only throughput table); whole rows
 * of AAD blocks take no AES work.  Blocks until the tag is on the host. */
int gcm_gmac(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
             const uint8_t *aad_d, uint64_t aad_len, uint8_t tag_out[16], void *stream);

/* ---------------------------------------------------------------- host-to-host pipeline */

/* gcm_encrypt / gcm_decrypt_verify on HOST buffers (the paper's
 * "Asynchronous Streams Pipeline" and "Optimized Memory Pipeline":
 * page-locked host memory and concurrent streams overlapping PCIe transfers
 * with the kernels).  The message moves through a ring of three device chunk
 * buffers: the host-to-device copy of chunk c+1, the fused tile kernel on
 * chunk c and the device-to-host copy of chunk c-1 run concurrently on three
 * streams of the context; one combine after the last chunk forms the tag, so
 * results are bit-identical to the device-resident calls.  aad_h, pt_h/ct_h
 * and the outputs are host pointers (any alignment); pass page-locked memory
 * (hipHostMalloc, torch pin_memory) for the copies to overlap, pageable
 * memory works but serialises.  in == out is allowed.  Decrypt-verify writes
 * plaintext chunks as they are done and zero-fills the whole output before
 * returning when the tag does not match (accept 0).  Blocking.  If a HIP
 * error occurs after copies started, the output may be partly written. */
int gcm_encrypt_host(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                     const uint8_t *aad_h, uint64_t aad_len, const uint8_t *pt_h, uint64_t len, uint8_t *ct_h,
                     uint8_t tag_out[16]);
int gcm_decrypt_verify_host(gcm_ctx *ctx, const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                            const uint8_t *aad_h, uint64_t aad_len, const uint8_t *ct_h, uint64_t len,
                            const uint8_t tag[16], uint8_t *pt_h, int *accept);

/* Chunk size of the host pipeline in bytes (rounded down to whole wave tiles,
 * at least one tile); 0 restores the default of 64 MiB.  Three chunk buffers
 * are allocated from the context's budget on first use.  4 KiB..16 GiB. */
int gcm_set_pipeline(gcm_ctx *ctx, uint64_t chunk_bytes);

/* ---------------------------------------------------------------- streamed messages */

/* One message fed in segments (inputs larger than HBM, or arriving over
 * time): each segment's tile partials stay on the device, and the final call
 * reduces them all, each segment's GHASH value multiplied by H^(blocks after
 * it) (GHASH is linear in its input), so the ciphertext and tag equal
 * gcm_encrypt's on the concatenated input (the paper's map-reduce across
 * segments, "Scalable MapReduce for Massive Files").  All calls of one stream object are enqueued
 * on the given HIP stream in call order without host synchronisation; give
 * them one stream (or order them).  Key: a registered slot.  IV: 1..1024
 * bytes.  Decrypt-verify releases plaintext segment by segment; the caller
 * must not act on it before the final call's flag reads 1 (no zero-fill). */
typedef struct gcm_stream gcm_stream;

/* op 0 encrypt / 1 decrypt-verify; the AAD (device, 16-byte aligned, may be
 * empty) is hashed here.  The stream's partials buffer (at least 4 MiB, 16
 * bytes per wave tile of every segment) and the pinned staging of its final
 * call's descriptors are taken from those of an earlier destroyed stream of
 * this context, else allocated (the device buffer from the context budget)
 * when first needed; an update or final that outgrows the buffer doubles
 * it, and that call waits for the stream once (the partials written so far
 * move to the new buffer). */
int gcm_stream_begin(gcm_ctx *ctx, uint32_t op, uint32_t slot, const uint8_t *iv, size_t iv_len,
                     const uint8_t *aad_d, uint64_t aad_len, gcm_stream **out, void *stream);

/* The next `len` bytes of the message: in_d -> out_d (device, 16-byte
 * aligned, in place allowed).  Every segment but the last must be a multiple
 * of 16 bytes (GCM_E_ARG afterwards otherwise).  len 0 is a no-op. */
int gcm_stream_update(gcm_stream *st, const uint8_t *in_d, uint64_t len, uint8_t *out_d, void *stream);

/* Close the message: encrypt writes the 16-byte tag to tag_d (device);
 * decrypt-verify reads the expected tag from tag_d and writes the int32
 * accept flag (1/0) to accept_d (device). */
int gcm_stream_final(gcm_stream *st, uint8_t *tag_d, int32_t *accept_d, void *stream);

/* Free the stream's state.  Its buffers stay with the context for later
 * streams (up to four sets; released when an allocation would exceed the
 * context budget, and by gcm_ctx_destroy), with an event recorded after its
 * final call's kernels: a later stream's work waits for that event, so after
 * a final call this returns without waiting.  A stream destroyed before its
 * final call waits for the device first. */
int gcm_stream_destroy(gcm_stream *st);

/* ---------------------------------------------------------------- authenticated FITS container */

/* The paper's container ("Authenticated FITS File Format", "Context Binding
 * via Associated Data (AAD)", "Policy Enforcement and Granular Access") for a
 * 2-D FITS image (primary HDU, BITPIX 8/16/32/64/-32/-64, NAXIS = 2):
 *   HDU 0, NAXIS = 0: NONCE_H, NONCE_D (hex), ORIG_BPX, ORIG_NAX, ORIG_NA1,
 *     ORIG_NA2 (the original BITPIX, NAXIS, NAXIS1, NAXIS2), HIERARCH
 *     AUTHTAG_H / AUTHTAG_D (hex; the names exceed eight characters), and
 *     ENCHDR: the original header blocks (2880-byte multiple, END included)
 *     encrypted under the header key with AAD = NONCE_H, base64, in a long
 *     string continued over CONTINUE cards (LONGSTRN = 'OGIP 1.0');
 *   HDU 1: a one-row BINTABLE, TFORM1 = '<N>B', whose cell is the N pixel
 *     bytes encrypted under the data key with
 *     AAD_D = NONCE_D || dec(BITPIX) || dec(NAXIS) || dec(NAXIS1) || dec(NAXIS2)
 *     (raw nonce bytes, then each value in strict ASCII decimal, e.g. -32 ->
 *     the three bytes "-32", without separators).
 * Both GCM computations run on the GPU (through the host pipeline).  No
 * CHECKSUM/DATASUM cards are written. */
typedef struct gcm_fits_result {
    uint8_t *data;        /* FITS bytes (malloc'd by the library; gcm_fits_free) */
    uint64_t size;
    int32_t error_code;   /* GCM_OK, or the negative code the call returned */
    int32_t warning_code; /* decrypt: 0 full access; 1 header fallback (header key missing or wrong:
                             a minimal header rebuilt from ORIG_*); 2 payload suppressed (data key
                             missing or wrong, or pixels / ORIG_* / NONCE_D tampered: pixels zeroed);
                             3 both */
} gcm_fits_result;

/* Encrypt FITS file bytes (host) into a container (out->data, host).  Keys:
 * 16, 24 or 32 bytes each; nonces: 12 bytes each (see gcm_fits_nonce).
 * Returns GCM_OK or a negative code (also stored in out->error_code). */
int gcm_fits_encrypt(gcm_ctx *ctx, const uint8_t *fits, uint64_t fits_len, const uint8_t *key_h, size_t key_h_len,
                     const uint8_t *key_d, size_t key_d_len, const uint8_t nonce_h[12], const uint8_t nonce_d[12],
                     gcm_fits_result *out);

/* Decrypt a container with the keys the caller holds (either may be NULL):
 * out->data receives a FITS file whose header is the authenticated original
 * (else the minimal ORIG_* header) and whose pixels are the authenticated
 * plaintext (else zeros), with out->warning_code as above (the paper's
 * FitsOperationResult).  A malformed container is GCM_E_ARG. */
int gcm_fits_decrypt(gcm_ctx *ctx, const uint8_t *container, uint64_t len, const uint8_t *key_h, size_t key_h_len,
                     const uint8_t *key_d, size_t key_d_len, gcm_fits_result *out);

/* Free out->data of a result. */
void gcm_fits_free(gcm_fits_result *r);

/* 12 bytes from the kernel's entropy pool (getrandom), for NONCE_H / NONCE_D. */
int gcm_fits_nonce(uint8_t out[12]);

/* ---------------------------------------------------------------- AES-GCM-SIV */

/* AES-GCM-SIV (RFC 8452): the nonce-misuse-resistant AEAD that the paper
 * names as the alternative to GCM where several operators may share a key
 * (Discussion and Future Work, "Future Directions", item 4).  A repeated
 * nonce then reveals only whether two messages are equal.
 *
 * The key-generating key is a registered slot of 16 or 32 bytes (24 is
 * GCM_E_KEYLEN); nonces are 12 bytes (else GCM_E_IVLEN); AAD and data are at
 * most 2^36 bytes each (else GCM_E_TOOLONG).  Per message the device derives
 * the authentication and encryption keys from the nonce, computes the tag
 * over POLYVAL(AAD, data) and encrypts in counter mode from the tag, so
 * encryption reads the plaintext twice; decryption is one fused pass.
 * Buffers: device memory, data and AAD 16-byte aligned, input and output
 * identical or disjoint; the tag may sit anywhere in device memory.
 *
 * Device scratch for a message of up to `len` data and up to `aad_len` AAD
 * bytes: a key slot for the derived keys (about 403 KiB), the POLYVAL value
 * and counter block, and the per-tile partial hashes (enough for every
 * shorter message too, as for gcm_workspace_size).  A workspace may be
 * reused by calls that are ordered on one stream. */
uint64_t gcm_siv_workspace_size(gcm_ctx *ctx, uint64_t len, uint64_t aad_len);

/* Encrypt: ct_d = the ciphertext, tag_d (device, 16 bytes) = the tag, both
 * written by kernels on `stream`; workspace_d: at least
 * gcm_siv_workspace_size() bytes, 256-byte aligned.  The call returns once
 * the kernels are enqueued. */
int gcm_siv_encrypt_async(gcm_ctx *ctx, uint32_t slot, const uint8_t *nonce, size_t nonce_len,
                          const uint8_t *aad_d, uint64_t aad_len, const uint8_t *pt_d, uint64_t len, uint8_t *ct_d,
                          uint8_t *tag_d, void *workspace_d, uint64_t workspace_bytes, void *stream);

/* Decrypt-verify: counter mode from the received tag (device, 16 bytes),
 * the tag recomputed over the recovered plaintext and compared in all 16
 * bytes; accept_d (device int32) = 1 accept, 0 reject, and on reject pt_d is
 * zero-filled by a later kernel on the same stream. */
int gcm_siv_decrypt_verify_async(gcm_ctx *ctx, uint32_t slot, const uint8_t *nonce, size_t nonce_len,
                                 const uint8_t *aad_d, uint64_t aad_len, const uint8_t *ct_d, uint64_t len,
                                 const uint8_t *tag_d, uint8_t *pt_d, int32_t *accept_d, void *workspace_d,
                                 uint64_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------- batches */

/* One message of a batch.  All offsets are byte offsets into one device
 * allocation `base_d` (256-byte aligned) of `base_bytes` bytes. */
typedef struct gcm_job {
    uint32_t op;        /* 0 = encrypt, 1 = decrypt-verify */
    uint32_t key_slot;  /* a registered key slot */
    uint8_t iv[12];     /* 96-bit IV */
    uint32_t reserved;  /* must be 0 */
    uint64_t aad_off;   /* AAD (16-byte aligned offset) */
    uint64_t aad_len;
    uint64_t in_off;    /* input payload (16-byte aligned) */
    uint64_t out_off;   /* output payload (16-byte aligned; == in_off for in place) */
    uint64_t len;       /* payload bytes, any length */
    uint64_t tag_off;   /* encrypt: tag written here; decrypt: expected tag read here */
    uint64_t ok_off;    /* decrypt: int32 accept flag written here (4-byte aligned) */
} gcm_job;

typedef struct gcm_batch gcm_batch;

/* Plan a batch: validates every job (bounds, alignment, aliasing, key slots),
 * builds per-message descriptors, the tile prefix table and the work list of
 * the persistent launch (the paper's map phase spread over many messages) and
 * uploads them (blocking).  The plan binds base_d; jobs may be freed after. */
int gcm_batch_create(gcm_ctx *ctx, const gcm_job *jobs, uint32_t n, uint8_t *base_d, uint64_t base_bytes,
                     gcm_batch **out);

/* Enqueue one pass over the batch on `stream`: the fused tile kernel over all
 * messages in one persistent launch, the per-message combine (tags / accept
 * flags written to base_d) and the zero-fill of rejected outputs.  Allocates
 * nothing; results are identical to running each message alone. */
int gcm_batch_launch(gcm_batch *b, void *stream);

/* Same as gcm_batch_launch, but the kernels are captured once into a hipGraph
 * (on a private stream) and every call replays the graph on `stream`. */
int gcm_batch_graph_launch(gcm_batch *b, void *stream);

/* Payload bytes, total wave tiles and workgroup items of a plan (any may be NULL). */
int gcm_batch_info(const gcm_batch *b, uint64_t *payload_bytes, uint64_t *total_tiles, uint32_t *work_items);

/* Wait for the device, then free the plan's device tables and graph. */
int gcm_batch_destroy(gcm_batch *b);

/* Convenience: create, launch, synchronise `stream`, destroy. */
int gcm_batch_run(gcm_ctx *ctx, const gcm_job *jobs, uint32_t n, uint8_t *base_d, uint64_t base_bytes, void *stream);

/* ---------------------------------------------------------------- serving */

/* One request of the serving loop; every buffer is already in HBM. */
typedef struct gcm_request {
    uint32_t op;          /* 0 = encrypt, 1 = decrypt-verify */
    uint32_t key_slot;    /* a registered (resident) key slot */
    uint8_t iv[12];
    uint32_t reserved;    /* must be 0 */
    const uint8_t *aad_d; /* device, 16-byte aligned */
    uint64_t aad_len;
    const uint8_t *in_d;  /* device, 16-byte aligned */
    uint8_t *out_d;       /* device, 16-byte aligned (== in_d for in place) */
    uint64_t len;
    uint8_t *tag_d;       /* device, 16 bytes: encrypt writes the tag, decrypt reads the expected tag */
} gcm_request;

typedef struct gcm_serve_config {
    uint32_t n_streams;       /* batches in flight at once (0 = 4, at most 16) */
    uint32_t max_batch_reqs;  /* requests per batch (0 = 256) */
    uint64_t hbm_budget;      /* device bytes of admitted requests (in + out + AAD + their share of a
                                 batch's descriptors and tile partials) plus the loop's retained
                                 stream-slot memory (0 = 64 GiB) */
    uint64_t max_batch_bytes; /* payload bytes per batch; a larger request runs alone (0 = 256 MiB) */
    uint32_t max_queue;       /* waiting + admitted requests before submit says GCM_E_BUSY (0 = 65536) */
    uint32_t reserved;
} gcm_serve_config;

typedef struct gcm_serve_stats {
    uint64_t submitted, completed, rejected, batches;
    uint64_t bytes_completed;        /* payload bytes of requests completed without failure */
    uint64_t budget_high_water;      /* most device bytes ever held at once, as hbm_budget counts them
                                        (<= hbm_budget) */
    uint64_t overlapped_admissions;  /* requests admitted while another batch was on the GPU */
    uint64_t max_inflight_batches;
    uint64_t failed;                 /* requests completed with a failure status (their batch could not
                                        be launched or reported a device error); counted in completed */
    double p50_ms, p99_ms, mean_ms, max_ms;  /* latency: submit -> result known on the host */
    double wall_s;                           /* first submit -> last completion */
} gcm_serve_stats;

typedef struct gcm_serve gcm_serve;

/* Start the serving loop (a scheduler thread and n_streams HIP streams) over
 * the context's resident key table.  cfg may be NULL for the defaults.
 * Continuous batching: requests are admitted in arrival order while their
 * bytes fit the HBM budget, packed into batches (the persistent launch of
 * gcm_batch_launch) and launched on free streams while earlier batches still
 * run.  A request's result does not depend on what it was batched with. */
int gcm_serve_start(gcm_ctx *ctx, const gcm_serve_config *cfg, gcm_serve **out);

/* Queue a request (thread-safe, non-blocking).  GCM_E_NOMEM if it alone needs
 * more than the budget, GCM_E_BUSY if the queue is full, GCM_E_ALIAS if the
 * output overlaps the input (other than in place), the AAD or the tag.  The
 * caller keeps the buffers untouched until the request is reported done. */
int gcm_serve_submit(gcm_serve *s, const gcm_request *req, uint64_t *id_out);

/* Non-blocking status.  When *done is 1 the request is collected: *accept is
 * the decrypt verdict (1 for encrypt) and *latency_ns its latency.  A request
 * whose batch failed (launch or device error) is collected with *accept 0 and
 * the call returns that failure's status (its outputs are undefined: a
 * decrypt's plaintext may not have been zero-filled, so it must not be used). */
int gcm_serve_poll(gcm_serve *s, uint64_t id, int *done, int *accept, uint64_t *latency_ns);

/* Block until the request is done, then collect it as gcm_serve_poll does. */
int gcm_serve_wait(gcm_serve *s, uint64_t id, int *accept, uint64_t *latency_ns);

/* Block until every submitted request is done. */
int gcm_serve_drain(gcm_serve *s);

/* Counters and latency percentiles so far. */
int gcm_serve_get_stats(gcm_serve *s, gcm_serve_stats *out);

/* Finish queued work, stop the thread, free the serving state. */
int gcm_serve_stop(gcm_serve *s);

/* ---------------------------------------------------------------- tuning */

/* Launch shape of the fused tile kernel.  Results never depend on it (the
 * counter and GHASH exponents derive from block indices only); only speed
 * does.  log2_tile_blocks: blocks per wave tile (6..20, 0 = automatic);
 * waves_per_group: 8, 12 or 16 (0 = automatic); groups_per_cu: resident
 * workgroups per compute unit (0 = automatic). */
int gcm_set_launch(gcm_ctx *ctx, uint32_t log2_tile_blocks, uint32_t waves_per_group, uint32_t groups_per_cu);

/* Fan-in of the reduction tree over tile partials (the paper's combine of
 * partial GHASH values): 2, 4, 8 or 16 children per node; 0 = automatic
 * (the autotune cache, else 2).  Results never depend on it. */
int gcm_set_combine(gcm_ctx *ctx, uint32_t fanin);

/* Result of an autotune search (also the answer of gcm_launch_plan). */
typedef struct gcm_tune_result {
    uint32_t log2_tile_blocks; /* chosen blocks per wave tile (log2); for a batch, the cap on its tiles */
    uint32_t waves_per_group;  /* chosen workgroup size in waves */
    uint32_t candidates;       /* shapes timed */
    float best_ms;             /* mean time of the chosen shape (one encrypt pass / one batch pass) */
    double gbs;                /* payload GB/s of the chosen shape */
    uint32_t groups_per_cu;    /* chosen resident workgroups per compute unit */
    uint32_t combine_fanin;    /* chosen fan-in of the reduction tree */
} gcm_tune_result;

/* Exhaustive launch-shape search for messages of about `len` bytes under
 * `key_len`-byte keys (the paper's per-GPU parameter sweep): every candidate
 * tile size (blocks per lane), workgroup size, groups per CU (1 up to the
 * occupancy limit) and reduction fan-in is timed `reps` times with HIP events
 * on a scratch message, all candidates must produce the identical tag
 * (GCM_E_INTERNAL otherwise), and the fastest shape is cached for that (key
 * size, floor(log2 len)) and used by every later single-message call
 * (one-shot, asynchronous, counter mode, host pipeline, streamed segments;
 * gcm_workspace_size sizes for it) without an explicit gcm_set_launch.
 * Allocates scratch for the duration of the call; blocks until done. */
int gcm_autotune(gcm_ctx *ctx, uint32_t key_len, uint64_t len, uint32_t reps, gcm_tune_result *out, void *stream);

/* The same search for a batch, run on the caller's jobs (gcm_batch_create's
 * arguments): workgroup size x groups per CU x cap on the messages' tile
 * sizes (2^8..2^12 blocks) x fan-in, each point a full pass over the batch
 * timed `reps` times, every point's tags and accept flags required equal to
 * the first point's (GCM_E_INTERNAL otherwise).  The winner is cached for
 * (floor(log2 n), floor(log2 payload bytes)) and used by later
 * gcm_batch_create calls and serving batches of that shape.  Every pass
 * rewrites the jobs' outputs, tags and flags, so jobs may not run in place
 * (GCM_E_ARG) and one job's output may not overlap another's input.
 * Blocks until done. */
int gcm_batch_autotune(gcm_ctx *ctx, const gcm_job *jobs, uint32_t n, uint8_t *base_d, uint64_t base_bytes,
                       uint32_t reps, gcm_tune_result *out, void *stream);

/* The launch an asynchronous single-message call on a message of `len` data
 * bytes and `aad_len` AAD bytes under a `key_len`-byte key would use now
 * (explicit settings, else the autotune cache, else the heuristics):
 * log2_tile_blocks, waves_per_group, groups_per_cu and combine_fanin are
 * filled, candidates = its number of wave tiles (the message's GHASH blocks
 * over the tile size, rounded up), best_ms and gbs = 0.  Host only; for
 * introspection and for figures that need the tile count. */
int gcm_launch_plan(gcm_ctx *ctx, uint32_t key_len, uint64_t len, uint64_t aad_len, gcm_tune_result *out);

/* Persist / restore both autotune caches as JSON (restoring rejects a cache
 * written on another GPU architecture). */
int gcm_autotune_save(gcm_ctx *ctx, const char *path);
int gcm_autotune_load(gcm_ctx *ctx, const char *path);

/* ---------------------------------------------------------------- measurement */

/* Kernel timing for benchmarks.  While enabled, every launch of the fused
 * CTR+GHASH tile kernel is bracketed by a pair of HIP events recorded on the
 * stream the kernel runs on (the paper's kernel-only timing scope). */
int gcm_profile_enable(gcm_ctx *ctx, int enable);

/* Waits for the recorded events, returns the number of timed tile-kernel
 * launches and their summed duration in milliseconds, and resets both. */
int gcm_profile_read(gcm_ctx *ctx, uint64_t *launches, double *tile_ms_total);

#ifdef __cplusplus
}
#endif

#endif /* GCM_MI355_H */
