"""GPU parity of the authenticated FITS container: the library's container
bytes against the oracle's (same keys and nonces), and every access scenario
of the paper's policy table decrypted by both, byte for byte."""
import random

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fits_container as fc  # noqa: E402
from paper_2602_23067_amd import gcm, workloads  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gcm.Context(device=0, key_slots=32)
    yield c
    c.close()


def _keys(seed):
    r = random.Random(seed)
    return r.randbytes(16), r.randbytes(32), r.randbytes(12), r.randbytes(12)


SHAPES = [(256, 256, -32), (37, 101, 16), (1, 1, 8), (64, 64, -64), (33, 7, 32), (5, 3, 64), (2048, 2048, -32)]


@pytest.mark.parametrize("ny,nx,bitpix", SHAPES)
def test_container_matches_oracle(ctx, ny, nx, bitpix):
    f = workloads.fits_file(workloads.rng_for(7100, ny, nx, bitpix & 0xff), ny, nx, bitpix)
    kh, kd, nh, nd = _keys(ny * 131 + nx)
    print(f"fits {ny}x{nx} bitpix={bitpix} ({len(f)} B)", flush=True)
    want = fc.encrypt(f, kh, kd, nh, nd)
    got = ctx.fits_encrypt(f, kh, kd, nh, nd)
    assert got == want, "container bytes differ from the oracle's"
    out, warn = ctx.fits_decrypt(got, kh, kd)
    assert warn == 0 and out == f


def test_access_scenarios_match_oracle(ctx):
    f = workloads.fits_file(workloads.rng_for(7200), 256, 256)
    kh, kd, nh, nd = _keys(9)
    c = ctx.fits_encrypt(f, kh, kd, nh, nd)
    wrong = bytes(32)
    for key_h, key_d, expect in [(kh, kd, 0), (kh, None, 2), (None, kd, 1), (None, None, 3), (wrong, kd, 1),
                                 (kh, wrong, 2), (kd, kh, 3), (kh[:15], kd, 1)]:
        got, warn = ctx.fits_decrypt(c, key_h, key_d)
        want, want_warn = fc.decrypt(c, key_h, key_d)
        assert warn == want_warn == expect, (key_h is None, key_d is None, warn, want_warn)
        assert got == want


def test_tampering_matches_oracle(ctx):
    f = workloads.fits_file(workloads.rng_for(7300), 128, 96)
    kh, kd, nh, nd = _keys(10)
    c = ctx.fits_encrypt(f, kh, kd, nh, nd)
    cards0, size0 = fc.parse_header(c)
    _, size1 = fc.parse_header(c, size0)
    cases = []
    # an edited structure keyword (context binding), a blob bit, a tag digit, an ENCHDR character
    i = next(k for k, card in enumerate(cards0) if card.startswith("ORIG_NA1"))
    edited = bytearray(c)
    edited[i * 80:(i + 1) * 80] = fc._int("ORIG_NA1", 95).encode("ascii")
    cases.append((bytes(edited), 2))
    flipped = bytearray(c)
    flipped[size0 + size1 + 1000] ^= 1
    cases.append((bytes(flipped), 2))
    j = next(k for k, card in enumerate(cards0) if card.startswith("HIERARCH AUTHTAG_D"))
    tag = bytearray(c)
    p = j * 80 + len("HIERARCH AUTHTAG_D = '") + 31
    tag[p] = ord("A") if tag[p] != ord("A") else ord("B")
    cases.append((bytes(tag), 2))
    e = next(k for k, card in enumerate(cards0) if card.startswith("ENCHDR"))
    enc = bytearray(c)
    p = e * 80 + 11 + 20
    enc[p] = ord("Q") if enc[p] != ord("Q") else ord("R")
    cases.append((bytes(enc), 1))
    for blob, expect in cases:
        got, warn = ctx.fits_decrypt(blob, kh, kd)
        want, want_warn = fc.decrypt(blob, kh, kd)
        assert warn == want_warn == expect
        assert got == want


def test_nonces_and_errors(ctx):
    a, b = gcm.fits_nonce(), gcm.fits_nonce()
    assert len(a) == len(b) == 12 and a != b
    f = workloads.fits_file(workloads.rng_for(7400), 16, 16)
    kh, kd, _, _ = _keys(11)
    c1, c2 = ctx.fits_encrypt(f, kh, kd), ctx.fits_encrypt(f, kh, kd)
    assert c1 != c2  # fresh nonces each time
    assert ctx.fits_decrypt(c1, kh, kd) == (f, 0)
    with pytest.raises(gcm.GcmError) as e:
        ctx.fits_encrypt(b"not a fits file" * 300, kh, kd)
    assert e.value.code == gcm.GCM_E_ARG
    with pytest.raises(gcm.GcmError) as e:
        ctx.fits_decrypt(f, kh, kd)  # a plain FITS file is not a container
    assert e.value.code == gcm.GCM_E_ARG
    with pytest.raises(gcm.GcmError) as e:
        ctx.fits_decrypt(c1[:len(c1) - 2880], kh, kd)  # truncated blob
    assert e.value.code == gcm.GCM_E_ARG
    # sizes whose products overflow 64 bits, in an input image and in a container
    huge = f.replace(fc._int("NAXIS1", 16).encode(), fc._int("NAXIS1", 1 << 40).encode(), 1)
    with pytest.raises(gcm.GcmError) as e:
        ctx.fits_encrypt(huge, kh, kd)
    assert e.value.code == gcm.GCM_E_ARG
    cards0, size0 = fc.parse_header(c1)
    cards1, _ = fc.parse_header(c1, size0)
    big = c1.replace(fc._int("ORIG_NA1", 16).encode(), fc._int("ORIG_NA1", (1 << 62) + 1).encode(), 1)
    with pytest.raises(gcm.GcmError) as e:
        ctx.fits_decrypt(big, kh, kd)
    assert e.value.code == gcm.GCM_E_ARG
    n1 = int(fc._value(cards1, "NAXIS1"))
    blob = c1.replace(fc._int("NAXIS1", n1).encode(), fc._int("NAXIS1", (1 << 63) - 1).encode(), 1)
    blob = blob.replace(fc._str("TFORM1", f"{n1}B").encode(), fc._str("TFORM1", f"{(1 << 63) - 1}B").encode(), 1)
    with pytest.raises(gcm.GcmError) as e:
        ctx.fits_decrypt(blob, kh, kd)
    assert e.value.code == gcm.GCM_E_ARG
