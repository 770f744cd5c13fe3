"""GPU tests of the batched persistent launch: every message of a batch,
checked against the CPU oracle bit for bit, and against the same message run
alone; exact reject set on tampered decrypt batches; hipGraph replays."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2602_23067_amd import gcm, workloads  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gcm.Context(device=0, key_slots=256)
    yield c
    c.close()


class Packed:
    """A small seeded batch in one device buffer, with its oracle results."""

    def __init__(self, ctx, seed, n, median, lo, hi, max_aad=300, ops=None, tamper=None, in_place=False):
        r = workloads.rng_for(seed, 77)
        self.lengths = workloads.lognormal_lengths(r, n, median, 1.0, lo, hi)
        self.aad_lens = r.integers(0, max_aad + 1, n)
        self.keys = [workloads.random_bytes(r, int(r.choice([16, 32]))).tobytes() for _ in range(n)]
        self.ivs = [workloads.random_bytes(r, 12).tobytes() for _ in range(n)]
        self.aads = [workloads.random_bytes(r, int(a)) for a in self.aad_lens]
        self.pts = [workloads.random_bytes(r, int(ln)) for ln in self.lengths]
        self.ops = list(ops) if ops is not None else [0] * n
        self.ref = [oracle.gcm_encrypt(k, iv, a, p) for k, iv, a, p in zip(self.keys, self.ivs, self.aads, self.pts)]
        self.tamper = tamper or {}
        self.slots = ctx.key_register_many(self.keys)
        self.layout = gcm.BatchLayout(self.lengths, self.aad_lens, in_place=in_place)
        self.host = np.zeros(self.layout.total, dtype=np.uint8)
        self.fill()
        self.base = torch.from_numpy(self.host.copy()).cuda()
        self.jobs = self.layout.jobs(self.ops, self.slots, self.ivs)

    def fill(self):
        L = self.layout
        for i in range(L.n):
            self.host[L.aad_off[i]:L.aad_off[i] + L.aad_lens[i]] = self.aads[i]
            ct, tag = self.ref[i]
            if self.ops[i] == 0:
                self.host[L.in_off[i]:L.in_off[i] + L.lengths[i]] = self.pts[i]
            else:
                src = ct.copy()
                tag = bytearray(tag)
                t = self.tamper.get(i)
                if t is not None:
                    where, frac, bit = t
                    if where == "tag" or L.lengths[i] == 0:
                        tag[int(frac * 16)] ^= 1 << bit
                    else:
                        src[int(frac * L.lengths[i])] ^= 1 << bit
                self.host[L.in_off[i]:L.in_off[i] + L.lengths[i]] = src
                self.host[L.tag_base + 16 * i:L.tag_base + 16 * i + 16] = np.frombuffer(bytes(tag), np.uint8)

    def reset_device(self):
        self.base.copy_(torch.from_numpy(self.host))

    def check(self):
        torch.cuda.synchronize()
        out = self.base.cpu().numpy()
        L = self.layout
        rejected = set()
        for i in range(L.n):
            got = out[L.out_off[i]:L.out_off[i] + L.lengths[i]]
            ct, tag = self.ref[i]
            if self.ops[i] == 0:
                assert np.array_equal(got, ct), f"message {i}: ciphertext differs from the oracle"
                assert bytes(out[L.tag_base + 16 * i:L.tag_base + 16 * i + 16]) == tag, f"message {i}: tag"
            else:
                ok = int(out[L.ok_base + 4 * i:L.ok_base + 4 * i + 4].view(np.int32)[0])
                assert ok in (0, 1)
                if ok:
                    assert np.array_equal(got, self.pts[i]), f"message {i}: plaintext"
                else:
                    rejected.add(i)
                    assert not got.any(), f"message {i}: rejected output not zero-filled"
        return rejected

    def release(self, ctx):
        for s in self.slots:
            ctx.key_release(s)


def test_batch_encrypt_matches_oracle(ctx):
    p = Packed(ctx, 1, 48, median=20_000, lo=1, hi=90_001)
    print("lengths", list(p.lengths)[:10], flush=True)
    b = gcm.Batch(ctx, p.jobs, p.base)
    b.launch()
    assert p.check() == set()
    b.close()
    p.release(ctx)


def test_batch_decrypt_rejects_exactly_the_tampered_set(ctx):
    n = 40
    plan = workloads.tamper_plan(3, n, frac=0.2)
    p = Packed(ctx, 2, n, median=8_000, lo=0, hi=40_000, ops=[1] * n, tamper=plan)
    b = gcm.Batch(ctx, p.jobs, p.base)
    b.launch()
    assert p.check() == set(plan), "rejected set differs from the tampered set"
    b.close()
    p.release(ctx)


def test_batch_mixed_ops_in_place(ctx):
    n = 30
    ops = [i % 2 for i in range(n)]
    plan = {i: t for i, t in workloads.tamper_plan(4, n, frac=0.3).items() if ops[i] == 1}
    p = Packed(ctx, 5, n, median=5_000, lo=16, hi=30_000, ops=ops, tamper=plan, in_place=True)
    b = gcm.Batch(ctx, p.jobs, p.base)
    b.launch()
    assert p.check() == set(plan)
    b.close()
    p.release(ctx)


def test_batch_graph_replays_match_eager(ctx):
    n = 24
    ops = [i % 3 == 0 for i in range(n)]
    plan = {i: t for i, t in workloads.tamper_plan(6, n, frac=0.25).items() if ops[i]}
    p = Packed(ctx, 7, n, median=12_000, lo=1, hi=50_000, ops=[int(o) for o in ops], tamper=plan)
    b = gcm.Batch(ctx, p.jobs, p.base)
    b.launch()
    eager = p.check()
    assert eager == set(plan)
    for _ in range(3):
        p.base.zero_()  # eager work between replays
        torch.cuda.synchronize()
        p.reset_device()
        b.graph_launch()
        assert p.check() == eager
    b.close()
    p.release(ctx)


def test_batch_result_equals_message_alone(ctx):
    """The same message gives the same bits alone (async single-message path)
    and inside a batch."""
    p = Packed(ctx, 9, 16, median=30_000, lo=1, hi=70_000)
    b = gcm.Batch(ctx, p.jobs, p.base)
    b.launch()
    torch.cuda.synchronize()
    out = p.base.cpu().numpy()
    L = p.layout
    for i in range(L.n):
        pt_d = torch.from_numpy(p.pts[i]).cuda() if L.lengths[i] else torch.empty(0, dtype=torch.uint8, device="cuda")
        aad_d = torch.from_numpy(p.aads[i]).cuda() if L.aad_lens[i] else None
        ct_d = torch.empty_like(pt_d)
        tag_d = torch.zeros(16, dtype=torch.uint8, device="cuda")
        ws = torch.zeros(ctx.workspace_size(L.lengths[i], L.aad_lens[i]), dtype=torch.uint8, device="cuda")
        ctx.encrypt_async(p.slots[i], p.ivs[i], aad_d, pt_d, ct_d, tag_d, ws)
        torch.cuda.synchronize()
        assert np.array_equal(ct_d.cpu().numpy(), out[L.out_off[i]:L.out_off[i] + L.lengths[i]])
        assert bytes(tag_d.cpu().numpy()) == bytes(out[L.tag_base + 16 * i:L.tag_base + 16 * i + 16])
    b.close()
    p.release(ctx)


def test_batch_validation(ctx):
    slot = ctx.key_register(bytes(16))
    try:
        lay = gcm.BatchLayout([100], [0])
        base = torch.zeros(lay.total, dtype=torch.uint8, device="cuda")
        jobs = lay.jobs([0], [slot], [bytes(12)])
        jobs[0].len = lay.total  # runs past the buffer
        with pytest.raises(gcm.GcmError) as e:
            gcm.Batch(ctx, jobs, base)
        assert e.value.code == gcm.GCM_E_ARG
        jobs = lay.jobs([0], [slot], [bytes(12)])
        jobs[0].in_off += 8  # misaligned
        with pytest.raises(gcm.GcmError):
            gcm.Batch(ctx, jobs, base)
        jobs = lay.jobs([0], [slot], [bytes(12)])
        jobs[0].out_off = jobs[0].in_off + 16  # partial overlap
        with pytest.raises(gcm.GcmError) as e:
            gcm.Batch(ctx, jobs, base)
        assert e.value.code == gcm.GCM_E_ALIAS
        jobs = lay.jobs([0], [slot + 1], [bytes(12)])
        with pytest.raises(gcm.GcmError) as e:
            gcm.Batch(ctx, jobs, base)
        assert e.value.code == gcm.GCM_E_SLOT
        jobs = lay.jobs([2], [slot], [bytes(12)])
        with pytest.raises(gcm.GcmError):
            gcm.Batch(ctx, jobs, base)
    finally:
        ctx.key_release(slot)


def test_batch_autotune_then_batches_use_the_tuned_shape(ctx):
    """The exhaustive batch search (waves x groups per CU x tile cap x
    fan-in, every point's tags and flags required equal) on a mixed
    encrypt / decrypt batch; afterwards a batch of that shape is planned with
    the cached winner and every message still matches the oracle."""
    n = 36
    ops = [i % 2 for i in range(n)]
    plan = {i: t for i, t in workloads.tamper_plan(12, n, frac=0.3).items() if ops[i] == 1}
    p = Packed(ctx, 13, n, median=30_000, lo=1, hi=400_000, ops=ops, tamper=plan)
    res = ctx.batch_autotune(p.jobs, p.base, reps=1)
    print("batch autotune:", res, flush=True)
    assert res["candidates"] >= 3 * 5 * 4
    assert res["waves_per_group"] in (8, 12, 16) and 8 <= res["log2_tile_blocks"] <= 12
    assert res["combine_fanin"] in (2, 4, 8, 16)
    assert p.check() == set(plan)  # the outputs of the last point searched
    p.reset_device()
    b = gcm.Batch(ctx, p.jobs, p.base)
    b.graph_launch()
    assert p.check() == set(plan)
    b.close()
    p.release(ctx)


def test_batch_autotune_rejects_in_place_jobs(ctx):
    p = Packed(ctx, 14, 4, median=2_000, lo=16, hi=4_000, in_place=True)
    with pytest.raises(gcm.GcmError) as e:
        ctx.batch_autotune(p.jobs, p.base, reps=1)
    assert e.value.code == gcm.GCM_E_ARG
    p.release(ctx)
