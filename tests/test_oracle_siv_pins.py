"""Pins for the oracle's AES-GCM-SIV (RFC 8452) and POLYVAL (no GPU).

The OpenSSL here has no GCM-SIV, so the construction is pinned step by step
against things other than the oracle: POLYVAL's field product against an
independent integer formulation and closed forms, POLYVAL against OpenSSL's
GHASH through the byte-reversal identity of RFC 8452 appendix A, the key
derivation, tag encryption and counter keystream against OpenSSL's AES-ECB,
and the AEAD properties (round trip, rejection of every single-field change,
nonce sensitivity, determinism)."""
import random

import numpy as np
import pytest

import oracle
import referee_openssl as ref
import siv_util

pytestmark = pytest.mark.skipif(not ref.available(), reason="libcrypto not loadable")

P_POLY = (1 << 128) | (1 << 127) | (1 << 126) | (1 << 121) | 1
ONE_X128 = bytes([1] + [0] * 14 + [0xC2])  # x^128 mod P, little-endian polynomial


def _int(b: bytes) -> int:  # little-endian polynomial: byte k bit j = x^(8k+j)
    return int.from_bytes(b, "little")


def _bytes(v: int) -> bytes:
    return v.to_bytes(16, "little")


def _pv_mul_int(a: int, b: int) -> int:
    """Independent product: carry-less integer product, then long division by P."""
    p = 0
    for i in range(128):
        if (b >> i) & 1:
            p ^= a << i
    for deg in range(254, 127, -1):
        if (p >> deg) & 1:
            p ^= P_POLY << (deg - 128)
    return p


def _br(b: bytes) -> bytes:
    return bytes(reversed(b))


def _ghash_div_x(h: bytes) -> bytes:
    """Inverse of GHASH's multiplication by x (SP 800-38D bit order: a right
    shift of the 128-bit big-endian string, folding 0xE1 into byte 0 when the
    last bit falls off).  The fold is visible as the top bit of the result."""
    v = int.from_bytes(h, "big")
    if v >> 127:
        v = ((v ^ (0xE1 << 120)) << 1) | 1
    else:
        v <<= 1
    return (v & ((1 << 128) - 1)).to_bytes(16, "big")


def test_pv_mul_matches_integer_formulation():
    r = random.Random(81)
    pairs = [(1 << i, 1 << j) for i in range(0, 128, 9) for j in range(0, 128, 11)]
    pairs += [(r.getrandbits(128), r.getrandbits(128)) for _ in range(200)]
    for a, b in pairs:
        assert oracle.pv_mul(_bytes(a), _bytes(b)) == _bytes(_pv_mul_int(a, b))


def test_x128_closed_form():
    x64 = _bytes(1 << 64)
    assert oracle.pv_mul(x64, x64) == ONE_X128  # x^128 = x^127 + x^126 + x^121 + 1 mod P


def test_polyval_closed_forms():
    r = random.Random(82)
    blocks = [r.randbytes(16) for _ in range(5)]
    # H = x^128 mod P makes dot(a, H) = a, so POLYVAL is the XOR of the blocks
    acc = bytes(16)
    for k, blk in enumerate(blocks):
        acc = bytes(x ^ y for x, y in zip(acc, blk))
        assert oracle.polyval(ONE_X128, b"".join(blocks[:k + 1])) == acc
    # one block: POLYVAL(H, X) * x^128 = X * H
    for _ in range(20):
        h, x = r.randbytes(16), r.randbytes(16)
        assert oracle.pv_mul(oracle.polyval(h, x), ONE_X128) == oracle.pv_mul(x, h)
    assert oracle.polyval(r.randbytes(16), b"") == bytes(16)
    assert oracle.polyval(bytes(16), b"".join(blocks)) == bytes(16)


def test_polyval_against_openssl_ghash():
    """POLYVAL(H, X_1..X_s) = BR(GHASH(mulX(BR(H)), BR(X_1), ..., BR(X_s))):
    with H_g = AES_K(0) from OpenSSL and H = BR(H_g / x), the GHASH side is
    OpenSSL's GMAC over AAD = BR(X_1)..BR(X_s-1) with X_s = BR(length block),
    minus E_K(J0)."""
    r = random.Random(83)
    for s in (1, 2, 7, 40):
        key, iv = r.randbytes(16), r.randbytes(12)
        hg = ref.aes_ecb_encrypt(key, bytes(16))
        h = _br(_ghash_div_x(hg))
        ys = [r.randbytes(16) for _ in range(s)]
        _, tag = ref.gcm_encrypt(key, iv, b"".join(ys), b"")
        ek_j0 = ref.aes_ecb_encrypt(key, iv + b"\x00\x00\x00\x01")
        length = (128 * s).to_bytes(8, "big") + bytes(8)
        ghash = bytes(a ^ b for a, b in zip(tag, ek_j0))
        xs = [_br(y) for y in ys] + [_br(length)]
        assert oracle.polyval(h, b"".join(xs)) == _br(ghash), s


@pytest.mark.parametrize("klen", [16, 32])
def test_derivation_tag_and_counter_against_openssl_ecb(klen):
    r = random.Random(84 + klen)
    for trial in range(6):
        kgk, nonce = r.randbytes(klen), r.randbytes(12)
        aad = r.randbytes(r.choice([0, 1, 16, 33]))
        pt = r.randbytes(r.choice([0, 5, 16, 47, 300]))
        # key derivation: first 8 bytes of AES_KGK(LE32(i) || nonce)
        halves = [ref.aes_ecb_encrypt(kgk, i.to_bytes(4, "little") + nonce)[:8] for i in range(klen // 8 + 2)]
        auth, enc = oracle.gcm_siv_derive(kgk, nonce)
        assert auth == halves[0] + halves[1]
        assert enc == b"".join(halves[2:])
        # tag = AES_enc(POLYVAL(...) ^ nonce, top bit of byte 15 cleared)
        pad = lambda b: b + bytes(-len(b) % 16)  # noqa: E731
        lb = (8 * len(aad)).to_bytes(8, "little") + (8 * len(pt)).to_bytes(8, "little")
        s = bytearray(oracle.polyval(auth, pad(aad) + pad(pt) + lb))
        for k in range(12):
            s[k] ^= nonce[k]
        s[15] &= 0x7F
        tag = ref.aes_ecb_encrypt(enc, bytes(s))
        # counter blocks: the tag with byte 15's top bit set, LE32 counter in bytes 0..3
        cb = bytearray(tag)
        cb[15] |= 0x80
        c0 = int.from_bytes(cb[:4], "little")
        ks = b"".join(ref.aes_ecb_encrypt(enc, ((c0 + i) % 2**32).to_bytes(4, "little") + bytes(cb[4:]))
                      for i in range((len(pt) + 15) // 16))
        ct = bytes(a ^ b for a, b in zip(pt, ks))
        got_ct, got_tag = oracle.gcm_siv_encrypt(kgk, nonce, aad, np.frombuffer(pt, np.uint8))
        assert got_tag == tag and got_ct.tobytes() == ct, trial


def test_counter_wraps_mod_2_32():
    """A message whose counters pass 2^32 (found through POLYVAL's
    linearity): the keystream continues at counter 0 in bytes 0..3, the
    other twelve bytes unchanged, against OpenSSL's AES-ECB."""
    r = np.random.default_rng(85)
    kgk, nonce = r.bytes(16), r.bytes(12)
    pt = r.integers(0, 256, 16 * 65536 + 5, dtype=np.uint8)
    aad, c0 = siv_util.wrapping_aad(kgk, nonce, pt, seed=85)
    ct, tag = oracle.gcm_siv_encrypt(kgk, nonce, aad, pt)
    assert int.from_bytes(tag[:4], "little") == c0
    _, enc = oracle.gcm_siv_derive(kgk, nonce)
    rest = bytes(tag[4:15]) + bytes([tag[15] | 0x80])
    nblk = (pt.size + 15) // 16
    wrap = 2**32 - c0  # blocks before the counter reaches 0
    assert 0 < wrap < nblk
    for i in (0, wrap - 1, wrap, wrap + 1, nblk - 1):
        ks = ref.aes_ecb_encrypt(enc, ((c0 + i) % 2**32).to_bytes(4, "little") + rest)
        got = ct[16 * i:16 * i + 16]
        want = np.frombuffer(ks[:got.size], np.uint8) ^ pt[16 * i:16 * i + got.size]
        assert np.array_equal(got, want), i
    back, ok = oracle.gcm_siv_decrypt_verify(kgk, nonce, aad, ct, tag)
    assert ok and np.array_equal(back, pt)


def test_round_trip_and_rejection():
    r = np.random.default_rng(86)
    for klen in (16, 32):
        for n, na in [(0, 0), (1, 0), (15, 7), (16, 16), (17, 100), (1000, 3), (4096 + 5, 0)]:
            kgk, nonce = r.bytes(klen), r.bytes(12)
            aad = r.integers(0, 256, na, dtype=np.uint8)
            pt = r.integers(0, 256, n, dtype=np.uint8)
            ct, tag = oracle.gcm_siv_encrypt(kgk, nonce, aad, pt)
            back, ok = oracle.gcm_siv_decrypt_verify(kgk, nonce, aad, ct, tag)
            assert ok and np.array_equal(back, pt)
            # deterministic; a different nonce changes the tag
            assert oracle.gcm_siv_encrypt(kgk, nonce, aad, pt)[1] == tag
            assert oracle.gcm_siv_encrypt(kgk, bytes(12) if nonce != bytes(12) else b"\1" * 12, aad, pt)[1] != tag
            bad_tag = bytes([tag[0] ^ 1]) + tag[1:]
            cases = [(kgk, nonce, aad, ct, bad_tag)]
            if n:
                c2 = ct.copy()
                c2[n // 2] ^= 0x40
                cases.append((kgk, nonce, aad, c2, tag))
            if na:
                a2 = aad.copy()
                a2[-1] ^= 1
                cases.append((kgk, nonce, a2, ct, tag))
            n2 = bytearray(nonce)
            n2[11] ^= 0x80
            cases.append((kgk, bytes(n2), aad, ct, tag))
            for args in cases:
                out, ok = oracle.gcm_siv_decrypt_verify(*args)
                assert not ok and not out.any()


def test_argument_errors():
    assert oracle.gcm_siv_derive(bytes(32), bytes(12))[1] == oracle.gcm_siv_derive(bytes(32), bytes(12))[1]
    for kgk, nonce, code in [(bytes(24), bytes(12), oracle.E_KEYLEN), (bytes(16), bytes(16), oracle.E_IVLEN),
                             (bytes(16), bytes(8), oracle.E_IVLEN)]:
        with pytest.raises(oracle.OracleError) as e:
            oracle.gcm_siv_encrypt(kgk, nonce, b"", b"abc")
        assert e.value.code == code
