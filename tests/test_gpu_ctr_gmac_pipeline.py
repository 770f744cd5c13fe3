"""GPU parity of the counter-mode-only, GMAC and host-to-host pipeline entry
points against the CPU oracle, bit for bit.

- CTR only: the oracle's GCTR from inc32(J0) (SP 800-38D GCM-AE step 3).
- GMAC: the oracle's GCM-AE with an empty plaintext; AAD sizes that give
  whole AAD rows (the GHASH-only row path) and ragged AAD tails.
- Host pipeline: chunked host->device->host runs whose chunks are forced
  small, so one message crosses many chunks and all three chunk buffers.
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


def _rng(seed):
    return np.random.default_rng(seed)


def _icb(iv: bytes) -> bytes:
    return bytes(iv) + b"\x00\x00\x00\x02"  # inc32(J0), J0 = IV || 0^31 || 1


# ---------------------------------------------------------------- CTR only

@pytest.mark.parametrize("key_len", [16, 24, 32])
@pytest.mark.parametrize("n", [1, 15, 16, 17, 1023, 64 * 1024 + 5, 3 * (1 << 20) + 7])
def test_ctr_matches_oracle_gctr(ctx, key_len, n):
    r = _rng(1000 + n + key_len)
    key = r.bytes(key_len)
    iv = r.bytes(12)
    data = r.integers(0, 256, n, dtype=np.uint8)
    print(f"ctr key={8 * key_len} n={n}", flush=True)
    ctx.set_launch(8, 16, 0)  # 4 KiB tiles: even short inputs cross tiles
    try:
        src = to_dev(data)
        full, dst = guarded(n)
        ctx.ctr_xcrypt(key, iv, src, dst)
        out = host(dst)
        assert canaries_intact(full, n), "write outside the output"
    finally:
        ctx.set_launch(0, 0, 0)
    assert np.array_equal(out, oracle.gctr(key, _icb(iv), data))
    # the same call decrypts
    back = torch.empty_like(src)
    ctx.ctr_xcrypt(key, iv, dst.contiguous(), back)
    assert np.array_equal(host(back), data)


def test_ctr_equals_gcm_ciphertext_and_empty_input(ctx):
    r = _rng(7)
    key, iv = r.bytes(32), r.bytes(12)
    data = r.integers(0, 256, (1 << 20) + 9, dtype=np.uint8)
    src = to_dev(data)
    ct_gcm = torch.empty_like(src)
    ctx.encrypt(key, iv, None, src, ct_gcm)
    ct_ctr = torch.empty_like(src)
    ctx.ctr_xcrypt(key, iv, src, ct_ctr)
    assert torch.equal(ct_gcm, ct_ctr)
    empty = torch.empty(0, dtype=torch.uint8, device="cuda")
    ctx.ctr_xcrypt(key, iv, empty, empty)  # no work, no error


def test_ctr_async_in_place_on_a_stream(ctx):
    r = _rng(8)
    key, iv = r.bytes(16), r.bytes(12)
    data = r.integers(0, 256, 777_777, dtype=np.uint8)
    slot = ctx.key_register(key)
    try:
        buf = to_dev(data)
        s = torch.cuda.Stream()
        torch.cuda.current_stream().synchronize()
        ctx.ctr_async(slot, iv, buf, buf, stream=s)
        s.synchronize()
        assert np.array_equal(host(buf), oracle.gctr(key, _icb(iv), data))
    finally:
        ctx.key_release(slot)


def test_ctr_argument_errors(ctx):
    d = torch.zeros(32, dtype=torch.uint8, device="cuda")
    with pytest.raises(gcm.GcmError) as e:
        ctx.ctr_xcrypt(bytes(16), bytes(11), d, d)
    assert e.value.code == gcm.GCM_E_IVLEN
    with pytest.raises(gcm.GcmError) as e:
        ctx.ctr_xcrypt(bytes(20), bytes(12), d, d)
    assert e.value.code == gcm.GCM_E_KEYLEN
    with pytest.raises(gcm.GcmError) as e:
        ctx.ctr_xcrypt(bytes(16), bytes(12), d[:16], d[8:24])
    assert e.value.code in (gcm.GCM_E_ALIAS, gcm.GCM_E_ARG)
    with pytest.raises(gcm.GcmError) as e:
        ctx.ctr_async(63, bytes(12), d, d)
    assert e.value.code == gcm.GCM_E_SLOT


# ---------------------------------------------------------------- GMAC / whole AAD rows

@pytest.mark.parametrize("aad_len", [0, 1, 16, 4096, 65536 + 3, 1 << 20, (1 << 20) + 16 * 64 * 3 + 5])
def test_gmac_matches_oracle(ctx, aad_len):
    r = _rng(2000 + aad_len)
    key, iv = r.bytes(32), r.bytes(12)
    aad = r.integers(0, 256, aad_len, dtype=np.uint8)
    _, want = oracle.gcm_encrypt(key, iv, aad, np.zeros(0, np.uint8))
    print(f"gmac aad={aad_len}", flush=True)
    for shape in [(0, 0, 0), (8, 16, 0), (10, 8, 1)]:
        ctx.set_launch(*shape)
        try:
            tag = ctx.gmac(key, iv, to_dev(aad) if aad_len else None)
        finally:
            ctx.set_launch(0, 0, 0)
        assert tag == want, f"GMAC tag differs at launch shape {shape}"


@pytest.mark.parametrize("aad_len,n", [(200 * 1024 + 3, 300 * 1024 + 5), (64 * 16 * 5, 64 * 16 * 7),
                                       (4096 * 16 + 1, 17)])
def test_gcm_with_large_aad(ctx, aad_len, n):
    r = _rng(3000 + aad_len + n)
    key, iv = r.bytes(16), r.bytes(12)
    aad = r.integers(0, 256, aad_len, dtype=np.uint8)
    pt = r.integers(0, 256, n, dtype=np.uint8)
    rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
    for shape in [(0, 0, 0), (8, 8, 0), (6, 16, 1)]:
        ctx.set_launch(*shape)
        try:
            pt_d = to_dev(pt)
            ct_d = torch.empty_like(pt_d)
            tag = ctx.encrypt(key, iv, to_dev(aad), pt_d, ct_d)
            assert np.array_equal(host(ct_d), rct) and tag == rtag, f"shape {shape}"
            back = torch.empty_like(pt_d)
            assert ctx.decrypt_verify(key, iv, to_dev(aad), ct_d, tag, back)
            assert np.array_equal(host(back), pt)
        finally:
            ctx.set_launch(0, 0, 0)


# ---------------------------------------------------------------- host pipeline

def _pinned(a: np.ndarray) -> torch.Tensor:
    t = torch.empty(a.size, dtype=torch.uint8, pin_memory=True)
    t.numpy()[:] = a
    return t


@pytest.mark.parametrize("key_len,n,aad_len,chunk,log2B", [
    (32, (2 << 20) + 13, 5000, 64 * 1024, 8),    # 16 tiles per chunk, 33 chunks
    (16, (1 << 20), 0, 4096, 6),                  # 1 KiB tiles, four per chunk: 257 chunks
    (24, 300_001, 70_000, 64 * 1024, 10),         # AAD spans the first chunks
    (32, 3 * (1 << 20) + 1, 2880, 0, 0),          # default chunk and shape: a single chunk
])
def test_host_pipeline_matches_oracle(ctx, key_len, n, aad_len, chunk, log2B):
    r = _rng(4000 + n + aad_len + key_len)
    key, iv = r.bytes(key_len), r.bytes(12)
    aad = r.integers(0, 256, aad_len, dtype=np.uint8)
    pt = r.integers(0, 256, n, dtype=np.uint8)
    rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
    print(f"pipeline key={8 * key_len} n={n} aad={aad_len} chunk={chunk} log2B={log2B}", flush=True)
    ctx.set_pipeline(chunk)
    ctx.set_launch(log2B, 16 if log2B else 0, 0)
    try:
        pt_h = _pinned(pt)
        ct_h = torch.empty(n, dtype=torch.uint8, pin_memory=True)
        aad_h = _pinned(aad) if aad_len else None
        tag = ctx.encrypt_host(key, iv, aad_h, pt_h, ct_h)
        assert np.array_equal(ct_h.numpy(), rct), "ciphertext differs from the oracle"
        assert tag == rtag, "tag differs from the oracle"
        back = torch.empty(n, dtype=torch.uint8, pin_memory=True)
        assert ctx.decrypt_verify_host(key, iv, aad_h, ct_h, tag, back)
        assert np.array_equal(back.numpy(), pt)
        # a flipped tag bit is rejected and the whole output zero-filled
        bad = bytes([tag[0] ^ 1]) + tag[1:]
        back.fill_(0x5A)
        assert not ctx.decrypt_verify_host(key, iv, aad_h, ct_h, bad, back)
        assert not back.numpy().any()
    finally:
        ctx.set_pipeline(0)
        ctx.set_launch(0, 0, 0)


def test_host_pipeline_pageable_in_place_and_empty(ctx):
    r = _rng(5)
    key, iv = r.bytes(16), r.bytes(12)
    aad = r.integers(0, 256, 1234, dtype=np.uint8)
    pt = r.integers(0, 256, 900_000, dtype=np.uint8)
    rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
    ctx.set_pipeline(128 * 1024)
    try:
        buf = pt.copy()  # pageable numpy memory, encrypted in place
        tag = ctx.encrypt_host(key, iv, aad, buf, buf)
        assert tag == rtag and np.array_equal(buf, rct)
        # GMAC through the pipeline: no payload, AAD only
        _, want = oracle.gcm_encrypt(key, iv, aad, np.zeros(0, np.uint8))
        empty = np.zeros(0, np.uint8)
        assert ctx.encrypt_host(key, iv, aad, empty, empty) == want
    finally:
        ctx.set_pipeline(0)


def test_host_pipeline_argument_errors(ctx):
    a = np.zeros(64, np.uint8)
    with pytest.raises(gcm.GcmError) as e:
        ctx.encrypt_host(bytes(16), bytes(12), None, a[:32], a[16:48])
    assert e.value.code == gcm.GCM_E_ALIAS
    with pytest.raises(gcm.GcmError) as e:
        ctx.encrypt_host(bytes(15), bytes(12), None, a, a)
    assert e.value.code == gcm.GCM_E_KEYLEN
    with pytest.raises(gcm.GcmError) as e:
        ctx.set_pipeline(100)
    assert e.value.code == gcm.GCM_E_ARG
