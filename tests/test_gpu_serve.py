"""GPU tests of the continuous-batching serving loop.

Requests of mixed sizes, operations and resident keys arrive from another
thread in bursts, with exponential gaps between bursts, while earlier
batches run; every result is checked bit for bit against the CPU oracle (so it equals the same request
run alone), tampered decrypts are rejected and zero-filled, the admitted
bytes never exceed the HBM budget, and requests were admitted while other
batches were on the GPU."""
import threading
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2602_23067_amd import gcm, workloads  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gcm.Context(device=0, key_slots=80)
    yield c
    c.close()


def _requests(seed, n, n_keys):
    r = workloads.rng_for(seed, 55)
    keys = [workloads.random_bytes(r, 16 if i % 2 == 0 else 32).tobytes() for i in range(n_keys)]
    sizes = workloads.lognormal_lengths(r, n, 24_000.0, 1.5, 0, 400_000)
    ops = r.integers(0, 2, n)
    kidx = r.integers(0, n_keys, n)
    reqs = []
    for i in range(n):
        iv = workloads.random_bytes(r, 12).tobytes()
        aad = workloads.random_bytes(r, int(r.integers(0, 200)))
        pt = workloads.random_bytes(r, int(sizes[i]))
        ct, tag = oracle.gcm_encrypt(keys[kidx[i]], iv, aad, pt)
        tampered = bool(ops[i] == 1 and r.random() < 0.2)
        reqs.append(dict(op=int(ops[i]), k=int(kidx[i]), iv=iv, aad=aad, pt=pt, ct=ct, tag=tag, tampered=tampered))
    return keys, reqs


def _device_bufs(q):
    aad_d = torch.from_numpy(q["aad"]).cuda() if q["aad"].size else None
    src = q["pt"] if q["op"] == 0 else q["ct"]
    in_d = torch.from_numpy(np.ascontiguousarray(src)).cuda() if src.size else torch.empty(0, dtype=torch.uint8,
                                                                                          device="cuda")
    out_d = torch.full_like(in_d, 0x5A)
    tag = bytearray(q["tag"])
    if q["tampered"]:
        tag[3] ^= 0x20
    tag_d = torch.from_numpy(np.frombuffer(bytes(tag), np.uint8).copy()).cuda() if q["op"] == 1 else \
        torch.zeros(16, dtype=torch.uint8, device="cuda")
    return aad_d, in_d, out_d, tag_d


def test_serving_mixed_requests_match_oracle(ctx):
    keys, reqs = _requests(1, 120, 64)
    slots = ctx.key_register_many(keys)
    torch.cuda.synchronize()
    bufs = [_device_bufs(q) for q in reqs]
    torch.cuda.synchronize()
    budget = 3 << 20
    srv = gcm.Server(ctx, n_streams=4, hbm_budget=budget, max_batch_reqs=16, max_batch_bytes=512 << 10)
    ids = [None] * len(reqs)
    # bursts of 8 back-to-back submissions with exponential gaps between
    # bursts: inside a burst, later requests arrive while the burst's first
    # batch is on the GPU (a sleep cannot be shorter than one small batch's
    # ~50 us, so single submissions with short gaps do not reliably overlap)
    gaps = workloads.rng_for(1, 56).exponential(500e-6, len(reqs))

    def submitter():
        for i, q in enumerate(reqs):
            a, x, y, t = bufs[i]
            ids[i] = srv.submit(q["op"], slots[q["k"]], q["iv"], a, x, y, t)
            if i % 8 == 7:
                time.sleep(float(gaps[i]))

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    results = [srv.wait(i) for i in ids]
    st = srv.stats()
    srv.stop()
    print("serving stats:", st, flush=True)
    torch.cuda.synchronize()
    for q, (a, x, y, t), (acc, lat) in zip(reqs, bufs, results):
        out = y.cpu().numpy()
        assert lat > 0
        if q["op"] == 0:
            assert acc
            assert np.array_equal(out, q["ct"]), "ciphertext differs from the oracle"
            assert bytes(t.cpu().numpy()) == q["tag"], "tag differs from the oracle"
        elif q["tampered"]:
            assert not acc and not out.any()
        else:
            assert acc and np.array_equal(out, q["pt"])
    assert st["completed"] == len(reqs)
    assert st["budget_high_water"] <= budget
    assert st["rejected"] == sum(q["tampered"] for q in reqs)
    assert st["overlapped_admissions"] > 0, "no request was admitted while another batch ran"
    assert st["p99_ms"] >= st["p50_ms"] > 0
    for s in slots:
        ctx.key_release(s)


def test_serving_rejects_oversize_and_bad_slot(ctx):
    srv = gcm.Server(ctx, n_streams=2, hbm_budget=1 << 16)
    x = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    y = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    t = torch.zeros(16, dtype=torch.uint8, device="cuda")
    slot = ctx.key_register(bytes(16))
    try:
        with pytest.raises(gcm.GcmError) as e:
            srv.submit(0, slot, bytes(12), None, x, y, t)  # needs 128 KiB > 64 KiB budget
        assert e.value.code == gcm.GCM_E_NOMEM
        with pytest.raises(gcm.GcmError) as e:
            srv.submit(0, slot + 1, bytes(12), None, x[:256], y[:256], t)
        assert e.value.code == gcm.GCM_E_SLOT
        rid = srv.submit(0, slot, bytes(12), None, x[:4096], y[:4096], t)
        acc, lat = srv.wait(rid)
        assert acc
        ref_ct, ref_tag = oracle.gcm_encrypt(bytes(16), bytes(12), b"", bytes(4096))
        assert np.array_equal(y[:4096].cpu().numpy(), ref_ct) and bytes(t.cpu().numpy()) == ref_tag
    finally:
        srv.stop()
        ctx.key_release(slot)


def test_serving_batch_that_cannot_launch_fails_closed():
    """A batch whose device scratch cannot be allocated (the context's own
    memory budget is exhausted) completes its requests with that status: the
    wait reports GCM_E_NOMEM, a decrypt is never accepted, and the stats count
    the requests as completed and failed."""
    # budget: the context's AES tables (TE0, the S-box, TE1..TE3: 5 x 256
    # words), Frobenius tables, two key slots and the 256-byte result block,
    # and nothing for the serving loop's per-batch scratch
    slot_bytes = 2048 + 65536 + 40 * 8192 + 16384
    budget = 5 * 256 * 4 + 47 * 4096 * 16 + 2 * slot_bytes + 256
    c = gcm.Context(device=0, hbm_budget=budget, key_slots=2)
    try:
        key, iv = bytes(range(16)), bytes(12)
        slot = c.key_register(key)
        pt = workloads.random_bytes(workloads.rng_for(58), 4096)
        ct, tag = oracle.gcm_encrypt(key, iv, b"", pt)
        x = torch.from_numpy(ct).cuda()
        y = torch.full_like(x, 0x5A)
        t = torch.from_numpy(np.frombuffer(tag, np.uint8).copy()).cuda()
        srv = gcm.Server(c, n_streams=1, hbm_budget=1 << 20)
        try:
            rid = srv.submit(1, slot, iv, None, x, y, t)  # a valid tag: would be accepted
            with pytest.raises(gcm.GcmError) as e:
                srv.wait(rid)
            assert e.value.code == gcm.GCM_E_NOMEM
            st = srv.stats()
            assert st["completed"] == 1 and st["failed"] == 1 and st["rejected"] == 0
        finally:
            with pytest.raises(gcm.GcmError) as e:  # stop reports the loop's error
                srv.stop()
            assert e.value.code == gcm.GCM_E_NOMEM
    finally:
        c.close()
