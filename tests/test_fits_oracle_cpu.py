"""CPU pins of the oracle's authenticated FITS container (the paper's
"Authenticated FITS File Format", "Context Binding via Associated Data (AAD)"
and "Policy Enforcement and Granular Access")."""
import base64
import os
import random

import numpy as np
import pytest

import oracle
from oracle import fits_container as fc
from paper_2602_23067_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def _image(seed=1, ny=64, nx=48, bitpix=-32):
    return workloads.fits_file(workloads.rng_for(7000, seed), ny, nx, bitpix)


def _keys(seed=0):
    r = random.Random(seed)
    return r.randbytes(16), r.randbytes(32), r.randbytes(12), r.randbytes(12)


def test_serialize_matches_the_papers_example():
    for line in open(os.path.join(HERE, "golden", "fits_serialize.txt")):
        if line.startswith("#") or not line.strip():
            continue
        value, printed = line.rstrip("\n").split("\t")
        assert fc.serialize(int(value)) == printed.strip("'").encode("ascii")


def test_data_aad_layout():
    nonce = bytes(range(12))
    assert fc.data_aad(nonce, -32, 2, 256, 256) == nonce + b"-322256256"
    assert fc.data_aad(nonce, 16, 2, 100, 7) == nonce + b"162100" + b"7"


def test_base64_encoder_matches_the_standard_library():
    r = random.Random(3)
    for n in list(range(0, 70)) + [2880, 5760]:
        b = r.randbytes(n)
        assert fc._b64(b) == base64.b64encode(b).decode("ascii")


def test_container_structure():
    """FITS rules (cards of 80 printable ASCII characters, 2880-byte blocks,
    mandatory keywords first and in order) and the paper's keyword set."""
    f = _image()
    kh, kd, nh, nd = _keys()
    c = fc.encrypt(f, kh, kd, nh, nd)
    assert len(c) % 2880 == 0
    cards0, size0 = fc.parse_header(c)
    cards1, size1 = fc.parse_header(c, size0)
    for card in cards0 + cards1:
        assert len(card) == 80 and all(0x20 <= ord(ch) <= 0x7E for ch in card)
    assert [k[:8].strip() for k in cards0[:4]] == ["SIMPLE", "BITPIX", "NAXIS", "EXTEND"]
    assert int(fc._value(cards0, "NAXIS")) == 0
    assert [k[:8].strip() for k in cards1[:8]] == ["XTENSION", "BITPIX", "NAXIS", "NAXIS1", "NAXIS2", "PCOUNT",
                                                  "GCOUNT", "TFIELDS"]
    _, hsize, bitpix, naxis, n1, n2 = fc.image_structure(f)
    nbytes = 4 * n1 * n2
    assert int(fc._value(cards1, "NAXIS1")) == nbytes and fc._string(cards1, "TFORM1") == f"{nbytes}B"
    assert [int(fc._value(cards0, k)) for k in ("ORIG_BPX", "ORIG_NAX", "ORIG_NA1", "ORIG_NA2")] == \
        [bitpix, naxis, n1, n2]
    assert bytes.fromhex(fc._string(cards0, "NONCE_H")) == nh
    assert bytes.fromhex(fc._string(cards0, "NONCE_D")) == nd
    # ENCHDR is the GCM encryption of the original header blocks (AAD = NONCE_H)
    ct_h = base64.b64decode(fc._long_string(cards0, "ENCHDR"))
    want_ct, want_tag = oracle.gcm_encrypt(kh, nh, nh, np.frombuffer(f[:hsize], np.uint8))
    assert ct_h == want_ct.tobytes() and bytes.fromhex(fc._hierarch(cards0, "AUTHTAG_H")) == want_tag
    # the blob is the GCM encryption of the pixels under AAD_D
    ct_d, tag_d = oracle.gcm_encrypt(kd, nd, fc.data_aad(nd, bitpix, naxis, n1, n2),
                                     np.frombuffer(f[hsize:hsize + nbytes], np.uint8))
    assert c[size0 + size1:size0 + size1 + nbytes] == ct_d.tobytes()
    assert bytes.fromhex(fc._hierarch(cards0, "AUTHTAG_D")) == tag_d
    assert not any(c[size0 + size1 + nbytes:])


@pytest.mark.parametrize("bitpix", [8, 16, 32, 64, -32, -64])
def test_full_access_round_trip(bitpix):
    f = _image(2, 37, 101, bitpix)
    kh, kd, nh, nd = _keys(1)
    out, warn = fc.decrypt(fc.encrypt(f, kh, kd, nh, nd), kh, kd)
    assert warn == 0 and out == f


def test_access_scenarios():
    """The paper's policy table: header key only -> payload suppressed;
    data key only -> header fallback; neither / wrong keys -> both."""
    f = _image(3)
    kh, kd, nh, nd = _keys(2)
    c = fc.encrypt(f, kh, kd, nh, nd)
    _, hsize, bitpix, naxis, n1, n2 = fc.image_structure(f)
    nbytes = 4 * n1 * n2
    out, warn = fc.decrypt(c, kh, None)
    assert warn == 2 and out[:hsize] == f[:hsize] and not any(out[hsize:])
    out, warn = fc.decrypt(c, None, kd)
    fallback, fsize = fc.parse_header(out)
    assert warn == 1 and fsize == 2880
    assert [k[:8].strip() for k in fallback] == ["SIMPLE", "BITPIX", "NAXIS", "NAXIS1", "NAXIS2", "END"]
    assert out[2880:2880 + nbytes] == f[hsize:hsize + nbytes]
    out, warn = fc.decrypt(c, kd, kh)  # keys swapped: both wrong
    assert warn == 3 and not any(out[2880:])


def test_context_binding_detects_tampered_structure_and_payload():
    f = _image(4)
    kh, kd, nh, nd = _keys(3)
    c = bytearray(fc.encrypt(f, kh, kd, nh, nd))
    cards0, size0 = fc.parse_header(bytes(c))
    # an edited ORIG_NA2 (same card layout, one row fewer) -> AAD_D differs
    i = next(k for k, card in enumerate(cards0) if card.startswith("ORIG_NA2"))
    old = int(fc._value(cards0, "ORIG_NA2"))
    edited = bytearray(c)
    edited[i * 80:(i + 1) * 80] = fc._int("ORIG_NA2", old - 1).encode("ascii")
    out, warn = fc.decrypt(bytes(edited), kh, kd)
    hsize = fc.image_structure(f)[1]
    assert warn == 2 and out[:hsize] == f[:hsize]  # the authenticated header, zero pixels of its shape
    assert len(out) == len(f) and not any(out[hsize:])
    # one flipped ciphertext bit in the blob
    _, size1 = fc.parse_header(bytes(c), size0)
    bad = bytearray(c)
    bad[size0 + size1 + 5] ^= 0x10
    out, warn = fc.decrypt(bytes(bad), kh, kd)
    assert warn == 2
    # a flipped tag digit of AUTHTAG_H -> header fallback only
    j = next(k for k, card in enumerate(cards0) if card.startswith("HIERARCH AUTHTAG_H"))
    bad = bytearray(c)
    pos = j * 80 + len("HIERARCH AUTHTAG_H = '")
    bad[pos] = ord("0") if bad[pos] != ord("0") else ord("1")
    _, warn = fc.decrypt(bytes(bad), kh, kd)
    assert warn == 1


def test_data_aad_concatenation_is_not_prefix_free():
    """The paper's literal AAD_D admits equal-size reshapes (documented
    limitation of the format): 5 x 550 and 55 x 50 hash the same bytes."""
    nonce = bytes(12)
    assert fc.data_aad(nonce, -32, 2, 5, 550) == fc.data_aad(nonce, -32, 2, 55, 50)
    assert 5 * 550 == 55 * 50
