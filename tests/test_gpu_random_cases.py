"""GPU parity on a seeded random sweep that mixes every parameter at once.

Each case draws a key size, an IV length (mostly 96 bits, else 1..80 bytes),
an AAD length, a payload length (biased towards row, tile and counter-byte
boundaries), a launch shape (the planner's own or a forced one), the one-shot
or the asynchronous resident-key path, and, for a third of the cases, one
flipped bit in the ciphertext, the tag or the AAD before decryption.  The
ciphertext and tag must equal the CPU oracle's bit for bit (SP 800-38D
GCM-AE), the decryption of the untouched ciphertext must return the
plaintext, and a tampered input must be rejected with a zero-filled output
(GCM-AD returns FAIL and no plaintext).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2602_23067_amd import gcm, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

from gpu_util import host, to_dev  # noqa: E402

N_CASES = 48
SHAPES = [(0, 0, 0), (0, 0, 0), (6, 8, 1), (7, 12, 1), (8, 16, 1), (9, 8, 2), (10, 16, 1), (12, 12, 1)]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gcm.Context(device=0, key_slots=16)
    yield c
    c.close()


def _payload_len(r) -> int:
    kind = int(r.integers(0, 4))
    if kind == 0:  # anywhere up to 1.5 MiB
        return int(r.integers(0, 3 << 19))
    if kind == 1:  # around a multiple of a 64-block row
        return max(0, 1024 * int(r.integers(1, 600)) + int(r.integers(-17, 18)))
    if kind == 2:  # around the point where the low counter byte wraps (256 blocks)
        return max(0, 4096 * int(r.integers(1, 200)) + int(r.integers(-40, 41)))
    return int(r.integers(0, 100))  # tiny


def _case(r):
    key_len = int(r.choice([16, 24, 32]))
    iv_len = 12 if r.random() < 0.7 else int(r.integers(1, 81))
    aad_len = int(r.choice([0, 1, 15, 16, 17, 2880, int(r.integers(0, 5000))]))
    n = _payload_len(r)
    shape = SHAPES[int(r.integers(0, len(SHAPES)))]
    path = "async" if (iv_len == 12 and r.random() < 0.5) else "oneshot"
    tamper = r.random() < 1 / 3
    where = str(r.choice(["ct", "tag", "aad"]))
    if where == "ct" and n == 0:
        where = "tag"
    if where == "aad" and aad_len == 0:
        where = "tag"
    return key_len, iv_len, aad_len, n, shape, path, tamper, where


def _encrypt(ctx, path, key, iv, aad, pt):
    aad_d = to_dev(aad) if len(aad) else None
    pt_d = to_dev(pt)
    ct_d = torch.empty_like(pt_d)
    if path == "oneshot":
        tag = ctx.encrypt(key, iv, aad_d, pt_d, ct_d)
        return host(ct_d), tag
    st = torch.cuda.current_stream()
    slot = ctx.key_register(key, st)
    try:
        ws = torch.zeros(max(1, ctx.workspace_size(len(pt), len(aad))), dtype=torch.uint8, device="cuda")
        tag_d = torch.zeros(16, dtype=torch.uint8, device="cuda")
        ctx.encrypt_async(slot, iv, aad_d, pt_d, ct_d, tag_d, ws, st)
        return host(ct_d), bytes(host(tag_d))
    finally:
        torch.cuda.synchronize()
        ctx.key_release(slot)


def _decrypt(ctx, key, iv, aad, ct, tag):
    aad_d = to_dev(aad) if len(aad) else None
    ct_d = to_dev(ct)
    out = torch.full_like(ct_d, 0x5A)
    ok = ctx.decrypt_verify(key, iv, aad_d, ct_d, tag, out)
    return host(out), ok


def test_random_cases_against_the_oracle(ctx):
    r = workloads.rng_for(90210)
    total = 0
    for i in range(N_CASES):
        key_len, iv_len, aad_len, n, shape, path, tamper, where = _case(r)
        key = workloads.random_bytes(r, key_len).tobytes()
        iv = workloads.random_bytes(r, iv_len).tobytes()
        aad = workloads.random_bytes(r, aad_len)
        pt = workloads.random_bytes(r, n)
        print(f"case {i}: key={8 * key_len} iv={iv_len} aad={aad_len} len={n} shape={shape} {path} "
              f"tamper={where if tamper else '-'}", flush=True)
        total += n
        ctx.set_launch(*shape)
        try:
            ct, tag = _encrypt(ctx, path, key, iv, aad, pt)
            rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
            assert np.array_equal(ct, rct), f"case {i}: ciphertext differs from the oracle"
            assert tag == rtag, f"case {i}: tag differs from the oracle"
            back, ok = _decrypt(ctx, key, iv, aad, ct, tag)
            assert ok and np.array_equal(back, pt), f"case {i}: round trip failed"
            if tamper:
                ct2, tag2, aad2 = ct.copy(), bytearray(tag), aad.copy()
                if where == "ct":
                    j = int(r.integers(0, n))
                    ct2[j] ^= np.uint8(1 << int(r.integers(0, 8)))
                elif where == "aad":
                    j = int(r.integers(0, aad_len))
                    aad2[j] ^= np.uint8(1 << int(r.integers(0, 8)))
                else:
                    tag2[int(r.integers(0, 16))] ^= 1 << int(r.integers(0, 8))
                bad, ok2 = _decrypt(ctx, key, iv, aad2, ct2, bytes(tag2))
                assert not ok2, f"case {i}: tampered {where} accepted"
                assert not bad.any(), f"case {i}: rejected output not zero-filled"
        finally:
            ctx.set_launch(0, 0, 0)
    assert total > 0
