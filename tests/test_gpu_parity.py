"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for bit.

Sizes here let the oracle finish in seconds while still spanning several
wave tiles and ragged tails; launch shapes are forced small so that even
short messages cross many tiles.
"""
import random

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
    c = gcm.Context(device=0, key_slots=64)
    yield c
    c.close()


def _enc(ctx, key, iv, aad, pt):
    aad_d = to_dev(aad) if len(aad) else None
    pt_d = to_dev(pt)
    ct_d = torch.empty_like(pt_d)
    tag = ctx.encrypt(key, iv, aad_d, pt_d, ct_d)
    return host(ct_d), tag


def _dec(ctx, key, iv, aad, ct, tag):
    aad_d = to_dev(aad) if len(aad) else None
    ct_d = to_dev(ct)
    pt_d = torch.full_like(ct_d, 0x5A)
    ok = ctx.decrypt_verify(key, iv, aad_d, ct_d, tag, pt_d)
    return host(pt_d), ok


def _check_case(ctx, key, iv, aad, pt):
    rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
    ct, tag = _enc(ctx, key, iv, aad, pt)
    assert np.array_equal(ct, rct), "ciphertext differs from the oracle"
    assert tag == rtag, "tag differs from the oracle"
    back, ok = _dec(ctx, key, iv, aad, ct, tag)
    assert ok and np.array_equal(back, np.asarray(pt, dtype=np.uint8))


def test_config1_parity(ctx):
    m = workloads.config1()
    print(f"config1: len={m.data.size} aad={m.aad.size}", flush=True)
    _check_case(ctx, m.key, m.iv, m.aad, m.data)


# the planner's own shapes for messages that do not fill the chip: 8- or
# 12-wave workgroups below a few MiB, 16 above (every one a distinct
# tile-size / wave-count choice on a 256-CU part), with ragged tails
@pytest.mark.parametrize("n", [(1 << 20) + 17, 2 << 20, (3 << 20) + 5, 4 << 20, (6 << 20) + 16, (12 << 20) + 1])
def test_default_shapes_by_size(ctx, n):
    r = workloads.rng_for(5000 + n % 997)
    key = workloads.random_bytes(r, 32).tobytes()
    iv = workloads.random_bytes(r, 12).tobytes()
    aad = workloads.random_bytes(r, 2880)
    pt = workloads.random_bytes(r, n)
    print(f"default shape: len={n}", flush=True)
    _check_case(ctx, key, iv, aad, pt)


@pytest.mark.parametrize("log2B", [6, 8])
def test_tail_sweep(ctx, log2B):
    ctx.set_launch(log2B, 8, 1)
    try:
        r = workloads.rng_for(7, log2B)
        sizes = list(range(0, 70)) + [255, 256, 257, 1023, 1024, 1025, 1040, 4095, 4096, 4097, 12345]
        for n in sizes:
            alen = int(r.choice([0, 1, 15, 16, 17, 100, 1024, 2880]))
            key = workloads.random_bytes(r, int(r.choice([16, 32]))).tobytes()
            iv = workloads.random_bytes(r, 12).tobytes()
            aad = workloads.random_bytes(r, alen)
            pt = workloads.random_bytes(r, n)
            _check_case(ctx, key, iv, aad, pt)
    finally:
        ctx.set_launch(0, 0, 0)


@pytest.mark.parametrize("key_len", [16, 24, 32])
def test_key_sizes(ctx, key_len):
    r = workloads.rng_for(11, key_len)
    key = workloads.random_bytes(r, key_len).tobytes()
    iv = workloads.random_bytes(r, 12).tobytes()
    _check_case(ctx, key, iv, workloads.random_bytes(r, 33), workloads.random_bytes(r, 70001))


@pytest.mark.parametrize("shape", [(6, 8, 1), (8, 12, 1), (7, 16, 1), (9, 16, 1), (10, 8, 2), (12, 8, 3), (0, 0, 0)])
def test_geometry_invariance(ctx, shape):
    """The paper's geometry-agnostic counter map: identical bits for every launch shape."""
    r = workloads.rng_for(13)
    key = workloads.random_bytes(r, 32).tobytes()
    iv = workloads.random_bytes(r, 12).tobytes()
    aad = workloads.random_bytes(r, 2880)
    pt = workloads.random_bytes(r, 300_007)
    ctx.set_launch(*shape)
    try:
        _check_case(ctx, key, iv, aad, pt)
    finally:
        ctx.set_launch(0, 0, 0)


def test_in_place_equals_out_of_place(ctx):
    r = workloads.rng_for(17)
    key, iv = workloads.random_bytes(r, 16).tobytes(), workloads.random_bytes(r, 12).tobytes()
    aad = to_dev(workloads.random_bytes(r, 20))
    pt = workloads.random_bytes(r, 100_003)
    rct, rtag = oracle.gcm_encrypt(key, iv, host(aad), pt)
    buf = to_dev(pt)
    tag = ctx.encrypt(key, iv, aad, buf, buf)
    assert tag == rtag and np.array_equal(host(buf), rct)
    ok = ctx.decrypt_verify(key, iv, aad, buf, tag, buf)
    assert ok and np.array_equal(host(buf), pt)


def test_no_write_outside_output(ctx):
    r = workloads.rng_for(19)
    key, iv = workloads.random_bytes(r, 32).tobytes(), workloads.random_bytes(r, 12).tobytes()
    for n in (1, 15, 17, 4097, 65541):
        pt = workloads.random_bytes(r, n)
        full, view = guarded(n)
        tag = ctx.encrypt(key, iv, None, to_dev(pt), view)
        assert canaries_intact(full, n)
        rct, rtag = oracle.gcm_encrypt(key, iv, b"", pt)
        assert tag == rtag and np.array_equal(host(view), rct)
        full2, view2 = guarded(n)
        bad = bytes([tag[0] ^ 1]) + tag[1:]
        ok = ctx.decrypt_verify(key, iv, None, to_dev(rct), bad, view2)
        assert not ok and canaries_intact(full2, n) and not host(view2).any()


def test_tampering_rejected_and_zero_filled(ctx):
    r = workloads.rng_for(23)
    key, iv = workloads.random_bytes(r, 16).tobytes(), workloads.random_bytes(r, 12).tobytes()
    aad = workloads.random_bytes(r, 45)
    pt = workloads.random_bytes(r, 200_001)
    ct, tag = oracle.gcm_encrypt(key, iv, aad, pt)
    rnd = random.Random(5)
    for _ in range(6):
        bad = ct.copy()
        pos = rnd.randrange(bad.size)
        bad[pos] ^= 1 << rnd.randrange(8)
        out, ok = _dec(ctx, key, iv, aad, bad, tag)
        assert not ok and not out.any()
    for bit in (0, 77, 127):
        t = bytearray(tag)
        t[bit // 8] ^= 1 << (bit % 8)
        out, ok = _dec(ctx, key, iv, aad, ct, bytes(t))
        assert not ok and not out.any()
    bad_aad = aad.copy()
    bad_aad[3] ^= 0x10
    out, ok = _dec(ctx, key, iv, bad_aad, ct, tag)
    assert not ok and not out.any()
    out, ok = _dec(ctx, bytes(16), iv, aad, ct, tag)
    assert not ok and not out.any()


def test_async_resident_key(ctx):
    r = workloads.rng_for(29)
    key, iv = workloads.random_bytes(r, 32).tobytes(), workloads.random_bytes(r, 12).tobytes()
    aad = workloads.random_bytes(r, 100)
    pt = workloads.random_bytes(r, 123_457)
    slot = ctx.key_register(key)
    try:
        ws = torch.zeros(ctx.workspace_size(pt.size, aad.size), dtype=torch.uint8, device="cuda")
        tag_d = torch.zeros(16, dtype=torch.uint8, device="cuda")
        aad_d, pt_d = to_dev(aad), to_dev(pt)
        ct_d = torch.empty_like(pt_d)
        ctx.encrypt_async(slot, iv, aad_d, pt_d, ct_d, tag_d, ws)
        rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
        assert bytes(host(tag_d)) == rtag and np.array_equal(host(ct_d), rct)
        acc = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        back = torch.empty_like(ct_d)
        ctx.decrypt_verify_async(slot, iv, aad_d, ct_d, tag_d, back, acc, ws)
        assert int(host(acc)[0]) == 1 and np.array_equal(host(back), pt)
        tag_d[0] ^= 1
        ctx.decrypt_verify_async(slot, iv, aad_d, ct_d, tag_d, back, acc, ws)
        assert int(host(acc)[0]) == 0 and not host(back).any()
    finally:
        ctx.key_release(slot)


def test_async_and_oneshot_calls_from_several_host_threads(ctx):
    """Four host threads on their own HIP streams share one context: two run
    asynchronous encrypt / decrypt-verify calls with a registered key and their
    own workspaces, two run one-shot calls (which share the context's own
    workspace and result block under its lock).  Every result equals the
    oracle's."""
    import threading

    r = workloads.rng_for(31)
    key = workloads.random_bytes(r, 32).tobytes()
    slot = ctx.key_register(key)
    cases = []
    for i in range(16):
        n = int(r.integers(1, 600_000))
        cases.append(dict(iv=workloads.random_bytes(r, 12).tobytes(), aad=workloads.random_bytes(r, int(r.integers(0, 300))),
                          pt=workloads.random_bytes(r, n)))
    for c in cases:
        c["rct"], c["rtag"] = oracle.gcm_encrypt(key, c["iv"], c["aad"], c["pt"])
    errors = []

    def run_async(mine):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                ws = torch.zeros(ctx.workspace_size(600_000, 300), dtype=torch.uint8, device="cuda")
                for c in mine:
                    aad_d = to_dev(c["aad"]) if c["aad"].size else None
                    pt_d = to_dev(c["pt"])
                    ct_d = torch.empty_like(pt_d)
                    tag_d = torch.zeros(16, dtype=torch.uint8, device="cuda")
                    ctx.encrypt_async(slot, c["iv"], aad_d, pt_d, ct_d, tag_d, ws, s)
                    back = torch.empty_like(ct_d)
                    acc = torch.full((1,), -1, dtype=torch.int32, device="cuda")
                    ctx.decrypt_verify_async(slot, c["iv"], aad_d, ct_d, tag_d, back, acc, ws, s)
                    s.synchronize()
                    if not (bytes(host(tag_d)) == c["rtag"] and np.array_equal(host(ct_d), c["rct"])
                            and int(host(acc)[0]) == 1 and np.array_equal(host(back), c["pt"])):
                        errors.append(f"async case of {c['pt'].size} bytes")
        except Exception as e:  # reported by the main thread
            errors.append(e)

    def run_oneshot(mine):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for c in mine:
                    aad_d = to_dev(c["aad"]) if c["aad"].size else None
                    pt_d = to_dev(c["pt"])
                    ct_d = torch.empty_like(pt_d)
                    tag = ctx.encrypt(key, c["iv"], aad_d, pt_d, ct_d, s)
                    if not (tag == c["rtag"] and np.array_equal(host(ct_d), c["rct"])):
                        errors.append(f"one-shot case of {c['pt'].size} bytes")
        except Exception as e:
            errors.append(e)

    print("threads: 2 asynchronous + 2 one-shot, 4 messages each", flush=True)
    try:
        ths = [threading.Thread(target=run_async, args=(cases[0:4],)),
               threading.Thread(target=run_async, args=(cases[4:8],)),
               threading.Thread(target=run_oneshot, args=(cases[8:12],)),
               threading.Thread(target=run_oneshot, args=(cases[12:16],))]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        torch.cuda.synchronize()
        assert not errors, errors
    finally:
        torch.cuda.synchronize()
        ctx.key_release(slot)


def test_empty_inputs(ctx):
    r = workloads.rng_for(31)
    key, iv = workloads.random_bytes(r, 16).tobytes(), workloads.random_bytes(r, 12).tobytes()
    empty = torch.empty(0, dtype=torch.uint8, device="cuda")
    tag = ctx.encrypt(key, iv, None, empty, empty)
    assert tag == oracle.gcm_encrypt(key, iv, b"", b"")[1]
    aad = workloads.random_bytes(r, 77)
    tag = ctx.encrypt(key, iv, to_dev(aad), empty, empty)
    assert tag == oracle.gcm_encrypt(key, iv, aad, b"")[1]
    assert ctx.decrypt_verify(key, iv, to_dev(aad), empty, tag, empty)


def test_argument_errors(ctx):
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(gcm.GcmError) as e:
        ctx.encrypt(bytes(20), bytes(12), None, buf, buf)
    assert e.value.code == gcm.GCM_E_KEYLEN
    for bad_iv in (b"", bytes(1025)):  # IVs of 1..1024 bytes are accepted
        with pytest.raises(gcm.GcmError) as e:
            ctx.encrypt(bytes(16), bad_iv, None, buf, buf)
        assert e.value.code == gcm.GCM_E_IVLEN
    with pytest.raises(gcm.GcmError) as e:
        ctx.encrypt(bytes(16), bytes(12), None, buf[1:33], buf[32:64])
    assert e.value.code == gcm.GCM_E_ARG  # misaligned
    big = torch.zeros(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(gcm.GcmError) as e:
        ctx.encrypt(bytes(16), bytes(12), None, big[0:128], big[16:144])
    assert e.value.code == gcm.GCM_E_ALIAS
    with pytest.raises(gcm.GcmError) as e:
        ctx.key_release(63)
    assert e.value.code == gcm.GCM_E_SLOT


def test_autotune_picks_a_shape_and_results_stay_exact(ctx, tmp_path):
    """Every candidate shape must give the identical tag (checked inside the
    search); afterwards the cached shape is used and results still match the
    oracle; the cache survives a save/load round trip."""
    res = ctx.autotune(32, 3 << 20, reps=2)
    print("autotune:", res, flush=True)
    assert res["candidates"] >= 2 and res["waves_per_group"] in (8, 12, 16) and 8 <= res["log2_tile_blocks"] <= 14
    assert res["combine_fanin"] in (2, 4, 8, 16) and res["groups_per_cu"] >= 1
    r = workloads.rng_for(37)
    key, iv = workloads.random_bytes(r, 32).tobytes(), workloads.random_bytes(r, 12).tobytes()
    _check_case(ctx, key, iv, workloads.random_bytes(r, 50), workloads.random_bytes(r, (3 << 20) + 5))
    path = str(tmp_path / "tune.json")
    ctx.autotune_save(path)
    c2 = gcm.Context(device=0, key_slots=4)
    try:
        c2.autotune_load(path)
        key2 = workloads.random_bytes(r, 32).tobytes()
        pt = workloads.random_bytes(r, 3 << 20)
        rct, rtag = oracle.gcm_encrypt(key2, iv, b"", pt)
        pt_d = to_dev(pt)
        ct_d = torch.empty_like(pt_d)
        assert c2.encrypt(key2, iv, None, pt_d, ct_d) == rtag and np.array_equal(host(ct_d), rct)
    finally:
        c2.close()


def test_workspace_size_covers_every_tuned_shape(ctx):
    """gcm_workspace_size and the asynchronous calls plan with the same shape
    function: after autotuning every key size at a message size, a workspace
    of exactly gcm_workspace_size bytes is enough for each key size, and the
    results match the oracle."""
    n = (1 << 20) + 3
    for kb in (16, 24, 32):
        ctx.autotune(kb, n, reps=1)
    r = workloads.rng_for(41)
    aad = workloads.random_bytes(r, 40)
    pt = workloads.random_bytes(r, n)
    ws = torch.zeros(ctx.workspace_size(n, aad.size), dtype=torch.uint8, device="cuda")
    for kb in (16, 24, 32):
        key, iv = workloads.random_bytes(r, kb).tobytes(), workloads.random_bytes(r, 12).tobytes()
        slot = ctx.key_register(key)
        try:
            rct, rtag = oracle.gcm_encrypt(key, iv, aad, pt)
            pt_d, aad_d = to_dev(pt), to_dev(aad)
            ct_d = torch.empty_like(pt_d)
            tag_d = torch.zeros(16, dtype=torch.uint8, device="cuda")
            ctx.encrypt_async(slot, iv, aad_d, pt_d, ct_d, tag_d, ws)
            assert bytes(host(tag_d)) == rtag and np.array_equal(host(ct_d), rct)
        finally:
            ctx.key_release(slot)


@pytest.mark.parametrize("fanin", [2, 4, 8, 16])
def test_reduction_fanin_does_not_change_results(ctx, fanin):
    """The tree over tile partials gives the same tag for every fan-in, with
    tile counts that are not powers of the fan-in, span one and several tree
    levels, and exceed the 1024 leaves (the strided Horner before the tree)."""
    r = workloads.rng_for(43, fanin)
    try:
        ctx.set_combine(fanin)
        for log2B, n in ((6, 16 * 64 * 5 + 7), (6, 16 * 64 * 37), (6, 16 * 64 * 300 + 1), (8, 16 * 256 * 1500 + 9)):
            ctx.set_launch(log2B, 16, 0)
            key, iv = workloads.random_bytes(r, 32).tobytes(), workloads.random_bytes(r, 12).tobytes()
            _check_case(ctx, key, iv, workloads.random_bytes(r, 33), workloads.random_bytes(r, n))
    finally:
        ctx.set_combine(0)
        ctx.set_launch(0, 0, 0)


def test_output_may_not_overlap_aad_tag_or_flag(ctx):
    slot = ctx.key_register(bytes(16))
    try:
        buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
        ws = torch.zeros(ctx.workspace_size(1024, 256), dtype=torch.uint8, device="cuda")
        with pytest.raises(gcm.GcmError) as e:  # ciphertext over the AAD
            ctx.encrypt_async(slot, bytes(12), buf[0:256], buf[1024:2048], buf[128:1152], buf[3000:3016], ws)
        assert e.value.code == gcm.GCM_E_ALIAS
        with pytest.raises(gcm.GcmError) as e:  # ciphertext over the tag
            ctx.encrypt_async(slot, bytes(12), None, buf[0:1024], buf[2048:3072], buf[2560:2576], ws)
        assert e.value.code == gcm.GCM_E_ALIAS
        ok = torch.zeros(1, dtype=torch.int32, device="cuda")
        with pytest.raises(gcm.GcmError) as e:  # plaintext over the expected tag
            ctx.decrypt_verify_async(slot, bytes(12), None, buf[0:1024], buf[1024:1040], buf[1024:2048], ok, ws)
        assert e.value.code == gcm.GCM_E_ALIAS
        with pytest.raises(gcm.GcmError) as e:  # one-shot: ciphertext over the AAD
            ctx.encrypt(bytes(16), bytes(12), buf[0:256], buf[1024:2048], buf[0:1024])
        assert e.value.code == gcm.GCM_E_ALIAS
    finally:
        ctx.key_release(slot)
