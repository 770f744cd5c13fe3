"""Test helper: an AAD block that makes an AES-GCM-SIV counter wrap.

POLYVAL is linear in its blocks, so with the nonce, the plaintext and the
AAD length fixed, the POLYVAL value for a first AAD block A is
S0 ^ POLYVAL(c, A), with S0 the value for A = 0 and c = POLYVAL over
(x^128 mod P, 0, ..., 0) -- one long oracle call each, then one block per
candidate.  The tag, and so the first counter, follows with one AES call."""
import random

import numpy as np

import oracle

ONE_X128 = bytes([1] + [0] * 14 + [0xC2])


def wrapping_aad(kgk: bytes, nonce: bytes, pt: np.ndarray, seed: int = 0, tries: int = 2_000_000):
    """(16-byte AAD, first counter) such that the message's counters pass
    2^32 inside its blocks (first counter > 2^32 - number of blocks)."""
    auth, enc = oracle.gcm_siv_derive(kgk, nonce)
    n = (pt.size + 15) // 16
    assert n >= 2
    padded = np.zeros(16 * n, np.uint8)
    padded[:pt.size] = pt
    lb = (8 * 16).to_bytes(8, "little") + (8 * pt.size).to_bytes(8, "little")
    body = np.concatenate([np.zeros(16, np.uint8), padded, np.frombuffer(lb, np.uint8)])
    s0 = oracle.polyval(auth, body)
    unit = np.zeros(body.size, np.uint8)
    unit[:16] = np.frombuffer(ONE_X128, np.uint8)
    c = oracle.polyval(auth, unit)
    r = random.Random(seed)
    for _ in range(tries):
        a = r.randbytes(16)
        s = bytearray(x ^ y for x, y in zip(s0, oracle.polyval(c, a)))
        for k in range(12):
            s[k] ^= nonce[k]
        s[15] &= 0x7F
        tag = oracle.aes_encrypt_block(enc, bytes(s))
        c0 = int.from_bytes(tag[:4], "little")
        if c0 > 2**32 - n + 1:
            return a, c0
    raise AssertionError("no wrapping AAD found")
