"""GPU parity of the streamed-message API: a message fed in device segments
must give the oracle's ciphertext and tag for the concatenated input, bit for
bit, for any segmentation."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2602_23067_amd import gcm  # noqa: E402

pytestmark = pytest.mark.gpu

from gpu_util import host, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gcm.Context(device=0, key_slots=16)
    yield c
    c.close()


def _stream_encrypt(ctx, slot, iv, aad, pt, cuts, stream=None):
    st = ctx.stream_begin(0, slot, iv, to_dev(aad) if aad.size else None, stream)
    try:
        outs = []
        for a, b in zip([0] + cuts, cuts + [pt.size]):
            src = to_dev(pt[a:b])
            dst = torch.empty_like(src)
            st.update(src, dst, stream)
            outs.append(dst)
        tag_d = torch.zeros(16, dtype=torch.uint8, device="cuda")
        st.final(tag_d, None, stream)
        torch.cuda.synchronize()
        ct = np.concatenate([host(o) for o in outs]) if outs else np.zeros(0, np.uint8)
        return ct, bytes(host(tag_d))
    finally:
        st.close()


CASES = [
    # (seed, key_len, iv_len, aad_len, segment lengths)
    (1, 16, 12, 0, [16]),
    (2, 32, 12, 5000, [1 << 20, (1 << 20) + 5]),
    (3, 24, 20, 77, [4096 * 3, 16, 1000 * 16, 777]),
    (4, 32, 12, 2880, [4096] * 50 + [33]),
    (5, 16, 7, 16, [64 * 16 * 5, 64 * 16 * 3, 15]),
    (6, 32, 12, 100_000, []),  # AAD only: a streamed GMAC
    (7, 16, 12, 0, []),  # nothing at all: T = E_K(J0)
]


@pytest.mark.parametrize("seed,key_len,iv_len,aad_len,segs", CASES)
def test_stream_encrypt_matches_oracle(ctx, seed, key_len, iv_len, aad_len, segs):
    r = np.random.default_rng(6000 + seed)
    key, iv = r.bytes(key_len), r.bytes(iv_len)
    aad = r.integers(0, 256, aad_len, dtype=np.uint8)
    pt = r.integers(0, 256, sum(segs), dtype=np.uint8)
    cuts = list(np.cumsum(segs)[:-1]) if segs else []
    rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
    print(f"stream seed={seed} segments={len(segs)} n={pt.size}", flush=True)
    slot = ctx.key_register(key)
    try:
        for shape in [(0, 0, 0), (8, 16, 0)]:
            ctx.set_launch(*shape)
            try:
                ct, tag = _stream_encrypt(ctx, slot, iv, aad, pt, [int(c) for c in cuts])
            finally:
                ctx.set_launch(0, 0, 0)
            assert np.array_equal(ct, rct), f"ciphertext, shape {shape}"
            assert tag == rtag, f"tag, shape {shape}"
    finally:
        ctx.key_release(slot)


def test_stream_decrypt_verify_and_tamper(ctx):
    r = np.random.default_rng(6100)
    key, iv = r.bytes(32), r.bytes(12)
    aad = r.integers(0, 256, 300, dtype=np.uint8)
    pt = r.integers(0, 256, 3 * (1 << 20) + 3, dtype=np.uint8)
    rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
    slot = ctx.key_register(key)
    s = torch.cuda.Stream()
    torch.cuda.current_stream().synchronize()
    try:
        for tag in (rtag, bytes([rtag[0] ^ 0x80]) + rtag[1:]):
            # every buffer is made on the current stream and kept alive until
            # `s` has finished with it
            aad_d = to_dev(aad)
            srcs = [to_dev(rct[a:b]) for a, b in ((0, 1 << 20), (1 << 20, 3 << 20), (3 << 20, pt.size))]
            outs = [torch.empty_like(x) for x in srcs]
            s.wait_stream(torch.cuda.current_stream())
            st = ctx.stream_begin(1, slot, iv, aad_d, stream=s)
            for src, dst in zip(srcs, outs):
                st.update(src, dst, stream=s)
            tag_d = to_dev(np.frombuffer(tag, np.uint8))
            ok_d = torch.full((1,), -1, dtype=torch.int32, device="cuda")
            s.wait_stream(torch.cuda.current_stream())
            st.final(tag_d, ok_d, stream=s)
            s.synchronize()
            st.close()
            ok = int(host(ok_d)[0])
            if tag == rtag:
                assert ok == 1
                assert np.array_equal(np.concatenate([host(o) for o in outs]), pt)
            else:
                assert ok == 0
    finally:
        ctx.key_release(slot)


def test_stream_counter_wraps_across_segments(ctx):
    r = np.random.default_rng(6200)
    key = r.bytes(16)
    for _ in range(400_000):
        iv = r.bytes(12 + 4)  # a 16-byte IV: J0 from GHASH, arbitrary counter
        c0 = int.from_bytes(oracle.gcm_j0(key, iv)[12:], "big")
        if c0 > (1 << 32) - 60_000:
            break
    else:
        pytest.fail("no IV with a J0 counter near 2^32 found")
    pt = r.integers(0, 256, 65536 * 16 + 1, dtype=np.uint8)
    rct, rtag = oracle.gcm_encrypt(key, iv, b"", pt)
    slot = ctx.key_register(key)
    try:
        ct, tag = _stream_encrypt(ctx, slot, iv, np.zeros(0, np.uint8), pt, [16 * 30_000, 16 * 61_000])
    finally:
        ctx.key_release(slot)
    assert np.array_equal(ct, rct) and tag == rtag


def test_stream_misuse_errors(ctx):
    slot = ctx.key_register(bytes(16))
    try:
        st = ctx.stream_begin(0, slot, bytes(12))
        buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
        st.update(buf[:32], buf[:32])
        st.update(buf[:17], buf[:17])  # a partial block: must be the last segment
        with pytest.raises(gcm.GcmError) as e:
            st.update(buf[:16], buf[:16])
        assert e.value.code == gcm.GCM_E_ARG
        tag_d = torch.zeros(16, dtype=torch.uint8, device="cuda")
        st.final(tag_d)
        with pytest.raises(gcm.GcmError) as e:
            st.final(tag_d)
        assert e.value.code == gcm.GCM_E_ARG
        st.close()
        with pytest.raises(gcm.GcmError) as e:
            ctx.stream_begin(2, slot, bytes(12))
        assert e.value.code == gcm.GCM_E_ARG
    finally:
        torch.cuda.synchronize()
        ctx.key_release(slot)


def test_stream_partials_buffer_grows_past_its_first_allocation(ctx):
    """300 segments of 1 MiB (+ a ragged last one) leave more tile partials
    than the stream's first 4 MiB partials buffer holds (with 64-block tiles
    forced, 1,025 slots per segment: 307,500 against 262,144), so the buffer
    is reallocated while segments are in flight; ciphertext and tag must
    equal one call of the asynchronous path on the concatenated message
    (itself checked against the oracle by the parity tests)."""
    r = np.random.default_rng(6300)
    key, iv = r.bytes(32), r.bytes(12)
    aad = to_dev(r.integers(0, 256, 2880, dtype=np.uint8))
    seg, nseg = 1 << 20, 300
    n = seg * nseg + 1234
    g = torch.Generator(device="cuda")
    g.manual_seed(6301)
    pt = torch.empty(n, dtype=torch.uint8, device="cuda").random_(0, 256, generator=g)
    slot = ctx.key_register(key)
    ctx.set_launch(6, 0, 0)
    try:
        print(f"stream: {nseg + 1} segments, {n} bytes, 64-block tiles", flush=True)
        st = ctx.stream_begin(0, slot, iv, aad)
        ct = torch.empty_like(pt)
        try:
            for off in range(0, n, seg):
                st.update(pt[off:off + seg], ct[off:off + seg])
            tag = torch.zeros(16, dtype=torch.uint8, device="cuda")
            st.final(tag, None)
            torch.cuda.synchronize()
        finally:
            st.close()
        ws = torch.zeros(ctx.workspace_size(n, aad.numel()), dtype=torch.uint8, device="cuda")
        ct1 = torch.empty_like(pt)
        tag1 = torch.zeros(16, dtype=torch.uint8, device="cuda")
        ctx.encrypt_async(slot, iv, aad, pt, ct1, tag1, ws)
        torch.cuda.synchronize()
    finally:
        ctx.set_launch(0, 0, 0)
        ctx.key_release(slot)
    assert torch.equal(tag, tag1), "tag differs from the one-call path"
    assert torch.equal(ct, ct1), "ciphertext differs from the one-call path"


def test_stream_buffers_are_reused_and_released_under_the_budget():
    """A destroyed stream's partials buffer stays with the context for the
    next stream and still counts against its budget; an allocation that would
    exceed the budget releases it first.  Budget: the context's own tables
    (AES tables, Frobenius tables, two key slots, the result block) plus one
    4 MiB partials buffer and half a MiB: the one-shot call's 1 MiB workspace
    fits only once the kept buffer is released, after which a new stream's
    4 MiB no longer fits (GCM_E_NOMEM, nothing launched)."""
    slot_bytes = 2048 + 65536 + 40 * 8192 + 16384
    base = 5 * 256 * 4 + 47 * 4096 * 16 + 2 * slot_bytes + 256
    c = gcm.Context(device=0, hbm_budget=base + (4 << 20) + (512 << 10), key_slots=2)
    try:
        r = np.random.default_rng(6400)
        key, iv = r.bytes(16), r.bytes(12)
        pt = r.integers(0, 256, 3 * 4096 + 5, dtype=np.uint8)
        rct, rtag = oracle.gcm_encrypt(key, iv, b"", pt)
        slot = c.key_register(key)
        for rep in range(2):  # the second stream runs on the first one's buffer
            print(f"stream rep {rep}", flush=True)
            ct, tag = _stream_encrypt(c, slot, iv, np.zeros(0, np.uint8), pt, [4096, 8192])
            assert np.array_equal(ct, rct) and tag == rtag
        x = to_dev(pt)
        y = torch.empty_like(x)
        tag1 = c.encrypt(key, iv, None, x, y)  # needs the kept buffer's budget
        torch.cuda.synchronize()
        assert tag1 == rtag and np.array_equal(host(y), rct)
        st = c.stream_begin(0, slot, iv)
        try:
            with pytest.raises(gcm.GcmError) as e:
                st.update(x, y)
            assert e.value.code == gcm.GCM_E_NOMEM
        finally:
            st.close()
    finally:
        torch.cuda.synchronize()
        c.close()


def test_stream_buffers_reused_across_hip_streams_without_waiting():
    """Message A (48 MiB, still running) is closed right after its final call;
    message B begins on another HIP stream at once and takes A's buffers from
    the context: B's kernels must wait for A's last work (the buffers' event),
    so both tags and ciphertexts equal one call of the asynchronous path on
    each message (itself checked against the oracle by the parity tests)."""
    r = np.random.default_rng(6500)
    key = r.bytes(32)
    n_a, n_b = 48 << 20, (3 << 20) + 100
    g = torch.Generator(device="cuda")
    g.manual_seed(6501)
    pa = torch.empty(n_a, dtype=torch.uint8, device="cuda").random_(0, 256, generator=g)
    pb = torch.empty(n_b, dtype=torch.uint8, device="cuda").random_(0, 256, generator=g)
    iv_a, iv_b = r.bytes(12), r.bytes(20)
    c = gcm.Context(device=0, key_slots=4)
    s2 = torch.cuda.Stream()
    try:
        slot = c.key_register(key)
        torch.cuda.synchronize()
        outs = []
        for _ in range(2):  # the second round reuses the buffers the first one left
            ca, cb = torch.empty_like(pa), torch.empty_like(pb)
            ta = torch.zeros(16, dtype=torch.uint8, device="cuda")
            tb = torch.zeros(16, dtype=torch.uint8, device="cuda")
            st = c.stream_begin(0, slot, iv_a)
            for off in range(0, n_a, 16 << 20):
                st.update(pa[off:off + (16 << 20)], ca[off:off + (16 << 20)])
            st.final(ta)
            st.close()
            s2.wait_stream(torch.cuda.current_stream())  # B's input was made on the default stream
            with torch.cuda.stream(s2):
                st = c.stream_begin(0, slot, iv_b, None, s2)
                st.update(pb[:1 << 20], cb[:1 << 20], s2)
                st.update(pb[1 << 20:], cb[1 << 20:], s2)
                st.final(tb, None, s2)
                st.close()
            outs.append((ca, cb, ta, tb))
        torch.cuda.synchronize()
        ws = torch.zeros(c.workspace_size(n_a, 0), dtype=torch.uint8, device="cuda")
        ra, rb = torch.empty_like(pa), torch.empty_like(pb)
        rta = torch.zeros(16, dtype=torch.uint8, device="cuda")
        rtb = torch.zeros(16, dtype=torch.uint8, device="cuda")
        c.encrypt_async(slot, iv_a, None, pa, ra, rta, ws)
        c.encrypt_async(slot, iv_b, None, pb, rb, rtb, ws)
        torch.cuda.synchronize()
        for ca, cb, ta, tb in outs:
            assert torch.equal(ta, rta) and torch.equal(ca, ra), "message A"
            assert torch.equal(tb, rtb) and torch.equal(cb, rb), "message B"
    finally:
        torch.cuda.synchronize()
        c.close()


def test_streams_from_several_host_threads_share_the_kept_buffers():
    """Four host threads, each on its own HIP stream, run five streamed
    messages each on one context: begin / update / final / destroy from the
    threads interleave on the context's lock and its kept buffers pass from
    thread to thread (each next user waiting on the previous one's event).
    Every ciphertext and tag must equal one call of the asynchronous path on
    the same message (itself checked against the oracle elsewhere)."""
    import threading

    r = np.random.default_rng(6600)
    key = r.bytes(32)
    c = gcm.Context(device=0, key_slots=4)
    try:
        slot = c.key_register(key)
        n_threads, per_thread = 4, 5
        jobs = []
        g = torch.Generator(device="cuda")
        g.manual_seed(6601)
        for t in range(n_threads):
            for k in range(per_thread):
                n = int(r.integers(1, 3 << 20))
                pt = torch.empty(n, dtype=torch.uint8, device="cuda").random_(0, 256, generator=g)
                aad = torch.empty(int(r.integers(0, 3000)) // 16 * 16, dtype=torch.uint8,
                                  device="cuda").random_(0, 256, generator=g)
                iv = r.bytes(12 if k % 2 == 0 else 20)
                jobs.append(dict(t=t, pt=pt, aad=aad, iv=iv, ct=torch.empty_like(pt),
                                 tag=torch.zeros(16, dtype=torch.uint8, device="cuda")))
        torch.cuda.synchronize()
        errors = []

        def run(t):
            s = torch.cuda.Stream()
            try:
                for j in [j for j in jobs if j["t"] == t]:
                    st = c.stream_begin(0, slot, j["iv"], j["aad"] if j["aad"].numel() else None, s)
                    try:
                        n = j["pt"].numel()
                        cut = (n // 3) // 16 * 16
                        st.update(j["pt"][:cut], j["ct"][:cut], s)
                        st.update(j["pt"][cut:], j["ct"][cut:], s)
                        st.final(j["tag"], None, s)
                    finally:
                        st.close()
                s.synchronize()
            except Exception as e:  # reported by the main thread
                errors.append(e)

        print(f"threads: {n_threads} x {per_thread} streamed messages", flush=True)
        threads = [threading.Thread(target=run, args=(t,)) for t in range(n_threads)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        torch.cuda.synchronize()
        assert not errors, errors
        ws = torch.zeros(c.workspace_size(3 << 20, 3000), dtype=torch.uint8, device="cuda")
        for j in jobs:
            ct1 = torch.empty_like(j["pt"])
            tag1 = torch.zeros(16, dtype=torch.uint8, device="cuda")
            c.encrypt_async(slot, j["iv"], j["aad"] if j["aad"].numel() else None, j["pt"], ct1, tag1, ws)
            torch.cuda.synchronize()
            assert torch.equal(j["tag"], tag1), "tag differs from the one-call path"
            assert torch.equal(j["ct"], ct1), "ciphertext differs from the one-call path"
    finally:
        torch.cuda.synchronize()
        c.close()
