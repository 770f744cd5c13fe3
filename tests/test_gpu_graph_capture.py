"""The resident-key asynchronous calls (and the allocation-free one) captured
into a HIP graph.

gcm_encrypt_async and gcm_decrypt_verify_async with a 96-bit IV enqueue
kernels only (no allocation, copy, memset or host wait), so a caller may
capture them.  The graph is replayed several times with the program's own
eager work in between (new plaintext written into the captured input buffer,
a tampered tag for one replay); every replay must equal the eager calls on
the same bytes, and those equal the CPU oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2602_23067_amd import gcm, workloads  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gcm.Context(device=0, key_slots=8)
    yield c
    c.close()


def test_captured_async_calls_replay_like_eager(ctx):
    r = workloads.rng_for(4242)
    key = workloads.random_bytes(r, 32).tobytes()
    iv = workloads.random_bytes(r, 12).tobytes()
    n, na = 3 * (1 << 20) + 7, 2880
    aad_h = workloads.random_bytes(r, na)
    dev = torch.device("cuda:0")
    aad = torch.from_numpy(aad_h.copy()).to(dev)
    pt = torch.empty(n, dtype=torch.uint8, device=dev)
    ct = torch.empty(n, dtype=torch.uint8, device=dev)
    back = torch.empty(n, dtype=torch.uint8, device=dev)
    tag = torch.zeros(16, dtype=torch.uint8, device=dev)
    tag_in = torch.zeros(16, dtype=torch.uint8, device=dev)
    ok = torch.zeros(1, dtype=torch.int32, device=dev)

    side = torch.cuda.Stream()
    slot = ctx.key_register(key, side)
    ws_e = torch.zeros(ctx.workspace_size(n, na), dtype=torch.uint8, device=dev)
    ws_d = torch.zeros(ctx.workspace_size(n, na), dtype=torch.uint8, device=dev)
    side.synchronize()
    try:
        def calls(s):
            ctx.encrypt_async(slot, iv, aad, pt, ct, tag, ws_e, s)
            ctx.decrypt_verify_async(slot, iv, aad, ct, tag_in, back, ok, ws_d, s)

        # eager reference for the current contents of the buffers
        def eager():
            s = torch.cuda.current_stream()
            calls(s)
            torch.cuda.synchronize()
            return ct.cpu().numpy().copy(), bytes(tag.cpu().numpy()), back.cpu().numpy().copy(), int(ok.cpu()[0])

        # warm-up outside the capture (first launches load the kernels), then
        # capture once (the buffers' contents at capture time do not matter)
        pt.zero_()
        eager()
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=side):
            calls(side)
        torch.cuda.synchronize()

        for rep in range(4):
            pt_h = workloads.random_bytes(r, n)
            pt.copy_(torch.from_numpy(pt_h))
            rct, rtag = oracle.gcm_encrypt(key, iv, aad_h, pt_h)
            good = rep != 2  # replay 2 decrypts against a wrong tag
            t_in = bytearray(rtag)
            if not good:
                t_in[5] ^= 0x10
            tag_in.copy_(torch.frombuffer(bytearray(t_in), dtype=torch.uint8))
            back.fill_(0x5A)
            torch.cuda.synchronize()
            print(f"replay {rep}: len={n} tag {'good' if good else 'tampered'}", flush=True)
            g.replay()
            torch.cuda.synchronize()
            g_ct, g_tag = ct.cpu().numpy().copy(), bytes(tag.cpu().numpy())
            g_back, g_ok = back.cpu().numpy().copy(), int(ok.cpu()[0])
            assert np.array_equal(g_ct, rct), f"replay {rep}: ciphertext differs from the oracle"
            assert g_tag == rtag, f"replay {rep}: tag differs from the oracle"
            if good:
                assert g_ok == 1 and np.array_equal(g_back, pt_h), f"replay {rep}: round trip failed"
            else:
                assert g_ok == 0 and not g_back.any(), f"replay {rep}: tampered tag not rejected"
            # the same calls run eagerly on the same bytes
            back.fill_(0x5A)
            e_ct, e_tag, e_back, e_ok = eager()
            assert np.array_equal(e_ct, g_ct) and e_tag == g_tag
            assert e_ok == g_ok and np.array_equal(e_back, g_back)
    finally:
        torch.cuda.synchronize()
        ctx.key_release(slot)


def test_captured_allocation_free_call_replays_like_the_oracle(ctx):
    """The allocation-free entry point (the library's own fixed scratch) in a
    graph: two replays over different plaintexts, each equal to the oracle."""
    r = workloads.rng_for(4343)
    key = workloads.random_bytes(r, 16).tobytes()
    iv = workloads.random_bytes(r, 12).tobytes()
    n, na = (1 << 20) + 33, 100
    aad_h = workloads.random_bytes(r, na)
    dev = torch.device("cuda:0")
    aad = torch.from_numpy(aad_h.copy()).to(dev)
    pt = torch.zeros(n, dtype=torch.uint8, device=dev)
    ct = torch.empty(n, dtype=torch.uint8, device=dev)
    tag = torch.zeros(16, dtype=torch.uint8, device=dev)
    side = torch.cuda.Stream()
    slot = ctx.key_register(key, side)
    side.synchronize()
    try:
        ctx.encrypt_async_noalloc(slot, iv, aad, pt, ct, tag, torch.cuda.current_stream())  # warm-up
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            ctx.encrypt_async_noalloc(slot, iv, aad, pt, ct, tag, side)
        torch.cuda.synchronize()
        for rep in range(2):
            pt_h = workloads.random_bytes(r, n)
            pt.copy_(torch.from_numpy(pt_h))
            torch.cuda.synchronize()
            print(f"allocation-free replay {rep}: len={n}", flush=True)
            g.replay()
            torch.cuda.synchronize()
            rct, rtag = oracle.gcm_encrypt(key, iv, aad_h, pt_h)
            assert np.array_equal(ct.cpu().numpy(), rct), f"replay {rep}: ciphertext differs from the oracle"
            assert bytes(tag.cpu().numpy()) == rtag, f"replay {rep}: tag differs from the oracle"
    finally:
        torch.cuda.synchronize()
        ctx.key_release(slot)
