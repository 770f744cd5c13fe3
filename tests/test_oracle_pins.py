"""Pins for the CPU oracle (no GPU).

Each test checks the oracle against something other than itself: brute
force over a whole finite field, an independent polynomial formulation,
algebraic invariants, the tree re-bracketing the paper proposes, and an
independent host library (OpenSSL EVP) standing in for the standards'
worked examples, which are not reproduced here.
"""
import random

import numpy as np
import pytest

import oracle
import referee_openssl as ref

pytestmark = pytest.mark.skipif(not ref.available(), reason="libcrypto not loadable")


# ---------------------------------------------------------------- GF(2^8)

def _clmul_mod_11b(a: int, b: int) -> int:
    """Independent GF(2^8) product: carry-less integer product, then
    polynomial remainder modulo x^8+x^4+x^3+x+1."""
    p = 0
    for i in range(8):
        if (b >> i) & 1:
            p ^= a << i
    for deg in range(14, 7, -1):
        if (p >> deg) & 1:
            p ^= 0x11B << (deg - 8)
    return p


def test_gf8_product_exhaustive():
    for a in range(256):
        for b in range(256):
            assert oracle.gf8_mul(a, b) == _clmul_mod_11b(a, b)


def test_gf8_inverse_exhaustive():
    assert oracle.gf8_inv(0) == 0
    for a in range(1, 256):
        assert oracle.gf8_mul(a, oracle.gf8_inv(a)) == 1


def test_gf8_xtime_is_times_x():
    for a in range(256):
        assert oracle.gf8_xtime(a) == _clmul_mod_11b(a, 2)


# ---------------------------------------------------------------- S-box

def test_sbox_invariants():
    s = oracle.sbox()
    inv = oracle.inv_sbox()
    assert sorted(s) == list(range(256))  # bijective
    assert s[0] == 0x63  # inverse(0) = 0, so S(0) is the affine constant
    for a in range(256):
        assert s[a] != a  # no fixed points
        assert s[a] != a ^ 0xFF  # no opposite fixed points
        assert inv[s[a]] == a


def test_sbox_is_affine_of_inverse():
    """S(a) xor 0x63 must be a GF(2)-linear function of inverse(a): check
    additivity of L(y) = S(inv(y)) ^ 0x63 over all pairs of basis vectors."""
    s = oracle.sbox()
    inv = {oracle.gf8_inv(a): a for a in range(256)}  # y -> a with inv(a) = y

    def L(y):
        return s[inv[y]] ^ 0x63

    assert L(0) == 0
    for y1 in range(256):
        for y2 in (1, 2, 4, 8, 16, 32, 64, 128):
            assert L(y1 ^ y2) == L(y1) ^ L(y2)


# ---------------------------------------------------------------- AES block

@pytest.mark.parametrize("key_len", [16, 24, 32])
def test_aes_block_matches_openssl(key_len):
    rng = random.Random(1000 + key_len)
    for _ in range(150):
        key = rng.randbytes(key_len)
        blk = rng.randbytes(16)
        assert oracle.aes_encrypt_block(key, blk) == ref.aes_ecb_encrypt(key, blk)


@pytest.mark.parametrize("key_len", [16, 24, 32])
def test_aes_inverse_round_trip(key_len):
    rng = random.Random(2000 + key_len)
    for _ in range(50):
        key = rng.randbytes(key_len)
        blk = rng.randbytes(16)
        assert oracle.aes_decrypt_block(key, oracle.aes_encrypt_block(key, blk)) == blk


def test_key_expansion_first_words_are_key():
    rng = random.Random(7)
    for key_len, nr in ((16, 10), (24, 12), (32, 14)):
        key = rng.randbytes(key_len)
        w = oracle.key_expand(key)
        assert len(w) == 16 * (nr + 1)
        assert w[:key_len] == key


def test_bad_key_length_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.aes_encrypt_block(bytes(20), bytes(16))


# ---------------------------------------------------------------- GF(2^128)

def _to_poly(b: bytes) -> int:
    """Independent representation: coefficient of x^i at integer bit i,
    where block bit i is bit (7 - i%8) of byte i//8."""
    v = 0
    for k in range(16):
        for t in range(8):
            if (b[k] >> (7 - t)) & 1:
                v |= 1 << (8 * k + t)
    return v


def _from_poly(v: int) -> bytes:
    out = bytearray(16)
    for i in range(128):
        if (v >> i) & 1:
            out[i // 8] |= 1 << (7 - i % 8)
    return bytes(out)


_P128 = (1 << 128) | 0x87  # x^128 + x^7 + x^2 + x + 1


def _poly_mulmod(a: int, b: int) -> int:
    p = 0
    while b:
        if b & 1:
            p ^= a
        a <<= 1
        b >>= 1
    for deg in range(p.bit_length() - 1, 127, -1):
        if (p >> deg) & 1:
            p ^= _P128 << (deg - 128)
    return p


def _basis(i: int) -> bytes:
    return _from_poly(1 << i)


def test_gf128_basis_pairs_exhaustive():
    """The product is bilinear, so agreement on all 128x128 basis pairs
    with an independent formulation proves agreement on every operand pair."""
    basis = [_basis(i) for i in range(128)]
    for i in range(128):
        for j in range(128):
            got = oracle.gf128_mul(basis[i], basis[j])
            assert got == _from_poly(_poly_mulmod(1 << i, 1 << j)), (i, j)


def test_gf128_random_operands_match_polynomial_form():
    rng = random.Random(11)
    for _ in range(300):
        a, b = rng.randbytes(16), rng.randbytes(16)
        assert oracle.gf128_mul(a, b) == _from_poly(_poly_mulmod(_to_poly(a), _to_poly(b)))


def test_gf128_field_axioms():
    rng = random.Random(12)
    one = oracle.GF128_ONE
    for _ in range(100):
        a, b, c = rng.randbytes(16), rng.randbytes(16), rng.randbytes(16)
        m = oracle.gf128_mul
        assert m(a, b) == m(b, a)
        assert m(m(a, b), c) == m(a, m(b, c))
        assert m(a, oracle.xor16(b, c)) == oracle.xor16(m(a, b), m(a, c))
        assert m(a, one) == a
        assert m(a, bytes(16)) == bytes(16)


def test_gf128_frobenius_and_group_order():
    rng = random.Random(13)
    for _ in range(3):
        a = rng.randbytes(16)
        x = a
        for _ in range(128):
            x = oracle.gf128_mul(x, x)
        assert x == a  # a^(2^128) = a
        assert oracle.gf128_pow(a, (1 << 128) - 1) == oracle.GF128_ONE  # a != 0 w.p. 1


# ---------------------------------------------------------------- GHASH

def _closed_form(h: bytes, blocks):
    """GHASH = sum_i X_i * H^(m-i+1) (1-based), from the recurrence unrolled."""
    m = len(blocks)
    acc = bytes(16)
    for i, x in enumerate(blocks, start=1):
        acc = oracle.xor16(acc, oracle.gf128_mul(x, oracle.gf128_pow(h, m - i + 1)))
    return acc


def _every_bracketing_value(h, blocks, lo, hi):
    """Set of node values over every binary bracketing of [lo, hi)."""
    if hi - lo == 1:
        return {bytes(blocks[lo])}
    vals = set()
    for mid in range(lo + 1, hi):
        for left in _every_bracketing_value(h, blocks, lo, mid):
            for right in _every_bracketing_value(h, blocks, mid, hi):
                vals.add(oracle.xor16(oracle.gf128_mul(left, oracle.gf128_pow(h, hi - mid)), right))
    return vals


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
def test_ghash_horner_equals_closed_form_and_every_tree(m):
    rng = random.Random(100 + m)
    h = rng.randbytes(16)
    blocks = [rng.randbytes(16) for _ in range(m)]
    horner = oracle.ghash(h, b"".join(blocks))
    assert horner == _closed_form(h, blocks)
    roots = _every_bracketing_value(h, blocks, 0, m)
    assert {oracle.gf128_mul(r, h) for r in roots} == {horner}


def test_ghash_paper_tree_power_of_two():
    """The paper's figure: level k combines with H^(2^k), then a final *H."""
    rng = random.Random(21)
    h = rng.randbytes(16)
    for m in (2, 4, 8, 16, 64):
        blocks = [rng.randbytes(16) for _ in range(m)]
        tree = oracle.ghash_tree(h, blocks, lambda lo, hi: (lo + hi) // 2)
        assert tree == oracle.ghash(h, b"".join(blocks))


def test_ghash_random_brackets_large():
    rng = random.Random(22)
    h = rng.randbytes(16)
    m = 257
    blocks = [rng.randbytes(16) for _ in range(m)]
    horner = oracle.ghash(h, b"".join(blocks))
    for _ in range(3):
        tree = oracle.ghash_tree(h, blocks, lambda lo, hi: rng.randrange(lo + 1, hi))
        assert tree == horner


def test_ghash_zero_prefix_invariance_and_linearity():
    rng = random.Random(23)
    h = rng.randbytes(16)
    x = rng.randbytes(16 * 37)
    y = rng.randbytes(16 * 37)
    gx = oracle.ghash(h, x)
    for z in (1, 5, 64):
        assert oracle.ghash(h, bytes(16 * z) + x) == gx
    assert oracle.ghash(h, x + bytes(16)) != gx  # right padding is not harmless
    xy = bytes(p ^ q for p, q in zip(x, y))
    assert oracle.ghash(h, xy) == oracle.xor16(gx, oracle.ghash(h, y))


# ---------------------------------------------------------------- GCM

def _rand_case(rng, key_len, plen, alen):
    return rng.randbytes(key_len), rng.randbytes(12), rng.randbytes(alen), rng.randbytes(plen)


@pytest.mark.parametrize("key_len", [16, 24, 32])
def test_gcm_matches_openssl_all_tails(key_len):
    rng = random.Random(300 + key_len)
    for plen in list(range(0, 97)) + [255, 256, 257, 1023, 1024, 1025, 4095, 4096, 4097]:
        alen = rng.choice([0, 1, 13, 16, 17, 31, 32, 80])
        key, iv, aad, pt = _rand_case(rng, key_len, plen, alen)
        ct, tag = oracle.gcm_encrypt(key, iv, aad, pt)
        rct, rtag = ref.gcm_encrypt(key, iv, aad, pt)
        assert ct.tobytes() == rct and tag == rtag, (plen, alen)


def test_gcm_aad_tails_match_openssl():
    rng = random.Random(310)
    for alen in range(0, 70):
        key, iv, aad, pt = _rand_case(rng, 16, rng.choice([0, 5, 16, 40]), alen)
        ct, tag = oracle.gcm_encrypt(key, iv, aad, pt)
        assert (ct.tobytes(), tag) == ref.gcm_encrypt(key, iv, aad, pt)


def test_gcm_large_message_matches_openssl():
    rng = np.random.default_rng(320)
    key = rng.integers(0, 256, 32, dtype=np.uint8).tobytes()
    iv = rng.integers(0, 256, 12, dtype=np.uint8).tobytes()
    aad = rng.integers(0, 256, 2880, dtype=np.uint8).tobytes()
    pt = rng.integers(0, 256, (1 << 20) + 11, dtype=np.uint8)
    ct, tag = oracle.gcm_encrypt(key, iv, aad, pt)
    rct, rtag = ref.gcm_encrypt(key, iv, aad, pt.tobytes())
    assert ct.tobytes() == rct and tag == rtag


def test_gcm_empty_empty_tag_is_ek_j0():
    rng = random.Random(330)
    for key_len in (16, 32):
        key, iv = rng.randbytes(key_len), rng.randbytes(12)
        _, tag = oracle.gcm_encrypt(key, iv, b"", b"")
        assert tag == ref.aes_ecb_encrypt(key, iv + b"\x00\x00\x00\x01")


def test_gcm_round_trip_and_decrypt_matches_openssl():
    rng = random.Random(340)
    for plen in (0, 1, 15, 16, 17, 100, 1000):
        key, iv, aad, pt = _rand_case(rng, rng.choice([16, 32]), plen, rng.choice([0, 7, 16]))
        ct, tag = oracle.gcm_encrypt(key, iv, aad, pt)
        back, ok = oracle.gcm_decrypt_verify(key, iv, aad, ct, tag)
        assert ok and back.tobytes() == pt
        rpt, rok = ref.gcm_decrypt(key, iv, aad, ct.tobytes(), tag)
        assert rok and rpt == pt


def test_gcm_every_single_bit_flip_rejected_and_zero_filled():
    rng = random.Random(350)
    key, iv, aad, pt = _rand_case(rng, 16, 37, 9)
    ct, tag = oracle.gcm_encrypt(key, iv, aad, pt)
    ctb = ct.tobytes()
    for pos in range(len(ctb) * 8):
        bad = bytearray(ctb)
        bad[pos // 8] ^= 1 << (pos % 8)
        out, ok = oracle.gcm_decrypt_verify(key, iv, aad, bytes(bad), tag)
        assert not ok and not out.any()
    for pos in range(128):
        bad = bytearray(tag)
        bad[pos // 8] ^= 1 << (pos % 8)
        out, ok = oracle.gcm_decrypt_verify(key, iv, aad, ctb, bytes(bad))
        assert not ok and not out.any()
    for pos in range(len(aad) * 8):
        bad = bytearray(aad)
        bad[pos // 8] ^= 1 << (pos % 8)
        _, ok = oracle.gcm_decrypt_verify(key, iv, bytes(bad), ctb, tag)
        assert not ok
    _, ok = oracle.gcm_decrypt_verify(bytes(16), iv, aad, ctb, tag)  # wrong key
    assert not ok


@pytest.mark.parametrize("iv_len", [1, 2, 7, 8, 11, 13, 15, 16, 17, 31, 32, 33, 60, 64, 100, 127, 128])
def test_gcm_other_iv_lengths_match_openssl(iv_len):
    """SP 800-38D sec. 7.1 step 2: J0 = GHASH_H(IV || 0^(s+64) || [len(IV)]_64) for IVs other than 96 bits.
    OpenSSL accepts IVs of up to 128 bytes (eight GHASH blocks); longer IVs take the same oracle code
    over more blocks."""
    rng = random.Random(360 + iv_len)
    for plen, alen in ((0, 0), (1, 0), (37, 13), (1000, 80), (4097, 2880)):
        key = rng.randbytes(rng.choice([16, 24, 32]))
        iv, aad, pt = rng.randbytes(iv_len), rng.randbytes(alen), rng.randbytes(plen)
        ct, tag = oracle.gcm_encrypt(key, iv, aad, pt)
        rct, rtag = ref.gcm_encrypt(key, iv, aad, pt)
        assert ct.tobytes() == rct and tag == rtag, (iv_len, plen, alen)
        back, ok = oracle.gcm_decrypt_verify(key, iv, aad, ct, tag)
        assert ok and back.tobytes() == pt


def test_gcm_j0_against_openssl_block_cipher():
    """J0 pinned without the oracle's GHASH: with P and A empty the tag is
    E_K(J0) (S = GHASH of the all-zero length block = 0), so OpenSSL's GCM tag
    must equal OpenSSL's AES-ECB of the oracle's J0."""
    rng = random.Random(370)
    for iv_len in (1, 8, 12, 16, 20, 60, 128):
        key, iv = rng.randbytes(16), rng.randbytes(iv_len)
        j0 = oracle.gcm_j0(key, iv)
        if iv_len == 12:
            assert j0 == iv + b"\x00\x00\x00\x01"
        _, rtag = ref.gcm_encrypt(key, iv, b"", b"")
        assert ref.aes_ecb_encrypt(key, j0) == rtag, iv_len


@pytest.mark.parametrize("tag_len", [4, 8, 12, 13, 14, 15, 16])
def test_gcm_truncated_tags(tag_len):
    """SP 800-38D sec. 5.2.1.2 / 7.2: T = MSB_t(full tag); verification compares t bits."""
    rng = random.Random(380 + tag_len)
    key, iv, aad, pt = _rand_case(rng, 32, 45, 11)
    ct, tag = oracle.gcm_encrypt(key, iv, aad, pt)
    t = tag[:tag_len]
    back, ok = oracle.gcm_decrypt_verify_t(key, iv, aad, ct, t)
    assert ok and back.tobytes() == pt
    assert ref.gcm_decrypt(key, iv, aad, ct.tobytes(), t) == (pt, True)
    for pos in range(tag_len * 8):
        bad = bytearray(t)
        bad[pos // 8] ^= 1 << (pos % 8)
        out, ok = oracle.gcm_decrypt_verify_t(key, iv, aad, ct, bytes(bad))
        assert not ok and not out.any()
        assert not ref.gcm_decrypt(key, iv, aad, ct.tobytes(), bytes(bad))[1]


def test_gcm_truncated_tag_lengths_outside_the_standard_rejected():
    key, iv = bytes(16), bytes(12)
    ct, tag = oracle.gcm_encrypt(key, iv, b"", b"abc")
    for bad_len in (0, 1, 3, 5, 7, 9, 11):
        with pytest.raises(oracle.OracleError) as e:
            oracle.gcm_decrypt_verify_t(key, iv, b"", ct, tag[:bad_len])
        assert e.value.code == oracle.E_ARG


def test_gcm_argument_errors():
    assert oracle.gcm_status(bytes(20), bytes(12), 0, 0) == oracle.E_KEYLEN
    assert oracle.gcm_status(bytes(16), b"", 0, 0) == oracle.E_IVLEN
    assert oracle.gcm_status(bytes(16), bytes(8), 0, 0) == oracle.OK
    assert oracle.gcm_status(bytes(16), bytes(16), 0, 0) == oracle.OK
    assert oracle.gcm_status(bytes(16), bytes(12), 0, (1 << 36) - 31) == oracle.E_TOOLONG
    assert oracle.gcm_status(bytes(16), bytes(12), 1 << 61, 0) == oracle.E_TOOLONG


def test_gctr_counter_wraps_mod_2_32():
    """inc32 wraps in the low 32 bits only: compare against OpenSSL's ECB on
    the explicitly wrapped counter blocks."""
    key = bytes(range(16))
    icb = bytes(range(12)) + b"\xff\xff\xff\xfe"
    out = oracle.gctr(key, icb, bytes(48))
    expect = b"".join(ref.aes_ecb_encrypt(key, bytes(range(12)) + c)
                      for c in (b"\xff\xff\xff\xfe", b"\xff\xff\xff\xff", b"\x00\x00\x00\x00"))
    assert out.tobytes() == expect
