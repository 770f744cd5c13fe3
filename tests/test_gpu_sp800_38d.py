"""GPU parity for the rest of the SP 800-38D surface: IVs other than 96 bits
(J0 from GHASH of the padded IV, computed on the device) and truncated tags,
against the CPU oracle bit for bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2602_23067_amd import gcm  # noqa: E402

pytestmark = pytest.mark.gpu

from gpu_util import canaries_intact, guarded, host, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gcm.Context(device=0, key_slots=64)
    yield c
    c.close()


def _case(seed, key_len, iv_len, n, aad_len):
    r = np.random.default_rng(seed)
    return (r.bytes(key_len), r.bytes(iv_len), r.integers(0, 256, aad_len, dtype=np.uint8),
            r.integers(0, 256, n, dtype=np.uint8))


@pytest.mark.parametrize("iv_len", [1, 8, 11, 13, 16, 17, 60, 64, 128, 1000, 1024])
def test_other_iv_lengths_one_shot(ctx, iv_len):
    key, iv, aad, pt = _case(5000 + iv_len, 16 if iv_len % 2 else 32, iv_len, 200_003, 77)
    rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
    print(f"iv_len={iv_len}", flush=True)
    for shape in [(0, 0, 0), (8, 16, 0)]:
        ctx.set_launch(*shape)
        try:
            pt_d = to_dev(pt)
            full, ct_d = guarded(pt.size)
            tag = ctx.encrypt(key, iv, to_dev(aad), pt_d, ct_d)
            assert np.array_equal(host(ct_d), rct), f"ciphertext, shape {shape}"
            assert tag == rtag, f"tag, shape {shape}"
            assert canaries_intact(full, pt.size)
            back = torch.empty_like(pt_d)
            assert ctx.decrypt_verify(key, iv, to_dev(aad), ct_d.contiguous(), tag, back)
            assert np.array_equal(host(back), pt)
        finally:
            ctx.set_launch(0, 0, 0)


def test_other_iv_length_async_and_host_pipeline(ctx):
    key, iv, aad, pt = _case(5100, 24, 20, 1_000_001, 5000)
    rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
    slot = ctx.key_register(key)
    try:
        pt_d = to_dev(pt)
        ct_d = torch.empty_like(pt_d)
        tag_d = torch.zeros(16, dtype=torch.uint8, device="cuda")
        ws = torch.zeros(ctx.workspace_size(pt.size, aad.size), dtype=torch.uint8, device="cuda")
        ctx.encrypt_async(slot, iv, to_dev(aad), pt_d, ct_d, tag_d, ws)
        assert np.array_equal(host(ct_d), rct) and bytes(host(tag_d)) == rtag
        ok_d = torch.zeros(1, dtype=torch.int32, device="cuda")
        back = torch.empty_like(pt_d)
        ctx.decrypt_verify_async(slot, iv, to_dev(aad), ct_d, tag_d, back, ok_d, ws)
        assert int(host(ok_d)[0]) == 1 and np.array_equal(host(back), pt)
    finally:
        ctx.key_release(slot)
    ctx.set_pipeline(64 * 1024)
    try:
        ct_h = np.empty_like(pt)
        assert ctx.encrypt_host(key, iv, aad, pt, ct_h) == rtag
        assert np.array_equal(ct_h, rct)
    finally:
        ctx.set_pipeline(0)


def test_j0_counter_wraps_inside_the_message(ctx):
    """A J0 whose 32-bit counter sits just below 2^32: inc32 wraps mod 2^32
    part-way through the message (inside a row, and inside the round-2 cache
    window), as SP 800-38D's inc32 prescribes."""
    r = np.random.default_rng(5200)
    key = r.bytes(16)
    for _ in range(400_000):
        iv = r.bytes(16)
        c0 = int.from_bytes(oracle.gcm_j0(key, iv)[12:], "big")
        if c0 > (1 << 32) - 60_000:
            break
    else:
        pytest.fail("no IV with a J0 counter near 2^32 found")
    n = 65536 * 16 + 9  # 65537 blocks: the counter wraps after at most 60000
    pt = r.integers(0, 256, n, dtype=np.uint8)
    aad = r.integers(0, 256, 33, dtype=np.uint8)
    rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
    print(f"J0 counter {c0:#x}", flush=True)
    for shape in [(0, 0, 0), (6, 16, 1), (12, 8, 0)]:
        ctx.set_launch(*shape)
        try:
            pt_d = to_dev(pt)
            ct_d = torch.empty_like(pt_d)
            tag = ctx.encrypt(key, iv, to_dev(aad), pt_d, ct_d)
            assert np.array_equal(host(ct_d), rct) and tag == rtag, f"shape {shape}"
        finally:
            ctx.set_launch(0, 0, 0)


def test_iv_length_errors(ctx):
    d = torch.zeros(32, dtype=torch.uint8, device="cuda")
    for bad in (b"", bytes(1025)):
        with pytest.raises(gcm.GcmError) as e:
            ctx.encrypt(bytes(16), bad, None, d, d)
        assert e.value.code == gcm.GCM_E_IVLEN
    with pytest.raises(gcm.GcmError) as e:
        ctx.ctr_xcrypt(bytes(16), bytes(16), d, d)  # counter mode only takes 96-bit IVs
    assert e.value.code == gcm.GCM_E_IVLEN


@pytest.mark.parametrize("tag_len", [4, 8, 12, 13, 14, 15, 16])
def test_truncated_tags(ctx, tag_len):
    key, iv, aad, pt = _case(5300 + tag_len, 32, 12 if tag_len != 13 else 7, 70_001, 19)
    rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
    pt_d = to_dev(pt)
    ct_d = torch.empty_like(pt_d)
    tag = ctx.encrypt_ex(key, iv, to_dev(aad), pt_d, ct_d, tag_len)
    assert len(tag) == tag_len and tag == rtag[:tag_len]
    assert np.array_equal(host(ct_d), rct)
    back = torch.empty_like(pt_d)
    assert ctx.decrypt_verify_ex(key, iv, to_dev(aad), ct_d, tag, back)
    assert np.array_equal(host(back), pt)
    for pos in (0, 8 * tag_len - 1, 5):
        bad = bytearray(tag)
        bad[pos // 8] ^= 1 << (pos % 8)
        back.fill_(0x5A)
        assert not ctx.decrypt_verify_ex(key, iv, to_dev(aad), ct_d, bytes(bad), back)
        assert not host(back).any()
        _, ok = oracle.gcm_decrypt_verify_t(key, iv, aad, rct, bytes(bad))
        assert not ok


def test_truncated_tag_length_errors(ctx):
    d = torch.zeros(32, dtype=torch.uint8, device="cuda")
    for bad in (0, 3, 5, 9, 11, 17):
        with pytest.raises(gcm.GcmError) as e:
            ctx.encrypt_ex(bytes(16), bytes(12), None, d, d, bad)
        assert e.value.code == gcm.GCM_E_ARG
