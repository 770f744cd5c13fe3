"""The allocation-free encrypt entry point (gcm_encrypt_async_noalloc),
through the C ABI, against gcm_encrypt_async with a caller workspace on the
same inputs, bit for bit, and against the CPU oracle where it finishes in
seconds.  Consecutive calls share the device's fixed scratch, so the cases
run back to back with the later ones smaller than the earlier ones."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2602_23067_amd import gcm, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

from gpu_util import canaries_intact, guarded, host, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gcm.Context(device=0, key_slots=8)
    yield c
    c.close()


def _inputs(seed, key_len, iv_len, aad_len, n):
    r = workloads.rng_for(2602, 901, seed)
    key = workloads.random_bytes(r, key_len).tobytes()
    iv = workloads.random_bytes(r, iv_len).tobytes()
    aad = workloads.random_bytes(r, aad_len)
    pt = workloads.random_bytes(r, n)
    return key, iv, aad, pt


def _both(ctx, slot, iv, aad_d, pt_d):
    """(ciphertext, tag) from the workspace path and from the fixed-scratch path."""
    n = pt_d.numel()
    ws = torch.zeros(ctx.workspace_size(n, 0 if aad_d is None else aad_d.numel()), dtype=torch.uint8, device="cuda")
    ct_ref = torch.empty_like(pt_d)
    tag_ref = torch.zeros(16, dtype=torch.uint8, device="cuda")
    ctx.encrypt_async(slot, iv, aad_d, pt_d, ct_ref, tag_ref, ws)
    full, ct = guarded(n)
    tag = torch.zeros(16, dtype=torch.uint8, device="cuda")
    ctx.encrypt_async_noalloc(slot, iv, aad_d, pt_d, ct, tag)
    torch.cuda.synchronize()
    assert canaries_intact(full, n), "the fixed-scratch call wrote outside its output"
    return host(ct_ref), bytes(host(tag_ref)), host(ct), bytes(host(tag))


@pytest.mark.parametrize("key_len", [16, 32])
def test_two_calls_in_a_row_second_smaller(ctx, key_len):
    """A 5 MiB + 7 B message, then a 1000 B one: each equals the workspace
    path and the oracle, whatever the first call left in the scratch."""
    for k, (iv_len, aad_len, n) in enumerate([(12, 2880, (5 << 20) + 7), (12, 16, 1000)]):
        key, iv, aad, pt = _inputs(10 * key_len + k, key_len, iv_len, aad_len, n)
        print(f"noalloc: key={8 * key_len} len={n} aad={aad_len} iv={iv_len}", flush=True)
        slot = ctx.key_register(key)
        try:
            ct_ref, tag_ref, ct, tag = _both(ctx, slot, iv, to_dev(aad), to_dev(pt))
        finally:
            ctx.key_release(slot)
        assert tag == tag_ref, "tag differs from the workspace path"
        assert np.array_equal(ct, ct_ref), "ciphertext differs from the workspace path"
        rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
        assert tag == rtag and np.array_equal(ct, rct), "differs from the oracle"


def test_other_iv_length_and_empty_message(ctx):
    """A 60-byte IV (J0 computed on the device into the scratch), then an
    empty message with AAD only (a GMAC tag), then an empty message with no
    AAD (tag = E_K(J0))."""
    cases = [(60, 300, 70_001), (12, 100, 0), (12, 0, 0)]
    for k, (iv_len, aad_len, n) in enumerate(cases):
        key, iv, aad, pt = _inputs(500 + k, 24, iv_len, aad_len, n)
        print(f"noalloc: key=192 len={n} aad={aad_len} iv={iv_len}", flush=True)
        slot = ctx.key_register(key)
        try:
            aad_d = to_dev(aad) if aad_len else None
            pt_d = to_dev(pt) if n else torch.empty(0, dtype=torch.uint8, device="cuda")
            tag_ref = torch.zeros(16, dtype=torch.uint8, device="cuda")
            ws = torch.zeros(ctx.workspace_size(n, aad_len), dtype=torch.uint8, device="cuda")
            ct_ref = torch.empty_like(pt_d)
            ctx.encrypt_async(slot, iv, aad_d, pt_d if n else None, ct_ref if n else None, tag_ref, ws)
            ct = torch.empty_like(pt_d)
            tag = torch.zeros(16, dtype=torch.uint8, device="cuda")
            ctx.encrypt_async_noalloc(slot, iv, aad_d, pt_d if n else None, ct if n else None, tag)
            torch.cuda.synchronize()
        finally:
            ctx.key_release(slot)
        rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
        assert bytes(host(tag_ref)) == rtag, "the workspace path differs from the oracle"
        assert bytes(host(tag)) == rtag, "the fixed-scratch path differs from the oracle"
        if n:
            assert np.array_equal(host(ct_ref), rct)
            assert np.array_equal(host(ct), rct)


def test_small_tiles_are_enlarged_to_fit(ctx):
    """With 64-block tiles forced, a 96 MiB message has 1.5 M tile partials,
    more than the fixed scratch holds: the call enlarges its tiles until they
    fit, and its output equals the workspace path's at the forced size."""
    n = (96 << 20) + 3
    key, iv, aad, _ = _inputs(700, 32, 12, 2880, 0)
    g = torch.Generator(device="cuda")
    g.manual_seed(701)
    pt_d = torch.empty(n, dtype=torch.uint8, device="cuda").random_(0, 256, generator=g)
    slot = ctx.key_register(key)
    ctx.set_launch(6, 0, 0)
    try:
        print(f"noalloc: forced 64-block tiles, len={n}", flush=True)
        assert ctx.workspace_size(n, 2880) > gcm.NOALLOC_SCRATCH_BYTES
        ct_ref, tag_ref, ct, tag = _both(ctx, slot, iv, to_dev(aad), pt_d)
    finally:
        ctx.set_launch(0, 0, 0)
        ctx.key_release(slot)
    assert tag == tag_ref
    assert np.array_equal(ct, ct_ref)


def test_beyond_the_fixed_scratch_is_an_error(ctx):
    """AAD of 2^40 bytes needs 2^20 partials even with 2^16-block tiles: the
    call fails with GCM_E_NOMEM on the host before anything is launched (the
    AAD address is never read)."""
    key, iv, _, pt = _inputs(800, 16, 12, 0, 4096)
    slot = ctx.key_register(key)
    try:
        pt_d = to_dev(pt)
        ct = torch.zeros_like(pt_d)
        tag = torch.zeros(16, dtype=torch.uint8, device="cuda")
        lib = gcm.load()
        ivb = gcm._host(iv)
        rc = lib.gcm_encrypt_async_noalloc(ctx.handle, slot, ivb, 12, 16, 1 << 40, pt_d.data_ptr(), pt_d.numel(),
                                           ct.data_ptr(), tag.data_ptr(), 0)
        assert rc == gcm.GCM_E_NOMEM, rc
        assert b"fixed" in lib.gcm_last_error()
        torch.cuda.synchronize()
        assert not ct.any().item() and not tag.any().item(), "an error return must leave the outputs untouched"
    finally:
        ctx.key_release(slot)
