"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (default launch shape, resident keys, persistent
batches replayed from a hipGraph).

The oracle cannot encrypt gigabytes inside a test, so each test combines:
  * block-sampled ciphertext from the oracle (both ends of every checked
    message plus uniformly drawn blocks; the sampling helper is pinned to the
    oracle's whole-message encryption by the CPU tests);
  * whole-message ciphertext and tag from OpenSSL, the second referee the
    oracle is pinned to on every tail length;
  * properties that hold at any size: decrypt-verify returns the plaintext
    and accepts, a flipped tag bit is rejected with a zero-filled output, the
    rejected set of a tampered batch is exactly the tampered set.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import referee_openssl as ref  # noqa: E402
import sampled  # noqa: E402
from paper_2602_23067_amd import gcm, workloads  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gcm.Context(device=0, key_slots=4200)
    yield c
    c.close()
    torch.cuda.empty_cache()


def _check_sampled(key, iv, pt, ct, seed, label):
    nb = (pt.size + 15) // 16
    idx = sampled.sample_indices(nb, np.random.default_rng(seed))
    for j, want in sampled.oracle_blocks(key, iv, pt, idx).items():
        assert np.array_equal(ct[16 * j:16 * j + 16], want), f"{label}: block {j} differs from the oracle"


def test_config2_fits_1gib_aes256_full_size(ctx):
    """AES-256-GCM of the 16384x16384 float32 FITS-shaped buffer with its
    2880-byte header as AAD, through the resident-key path the benchmark
    times and through the one-shot call."""
    print("[fullsize] config 2: generating 1 GiB FITS-shaped input", flush=True)
    m = workloads.config2()
    n = m.data.size
    ref_ct, ref_tag = ref.gcm_encrypt_np(m.key, m.iv, m.aad.tobytes(), m.data)
    dev = torch.device("cuda:0")
    pt_d = torch.from_numpy(m.data).to(dev)
    aad_d = torch.from_numpy(m.aad).to(dev)
    ct_d = torch.empty_like(pt_d)
    tag_d = torch.zeros(16, dtype=torch.uint8, device=dev)
    ws = torch.zeros(ctx.workspace_size(n, m.aad.size), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    print("[fullsize] config 2: GPU encrypt (resident key)", flush=True)
    slot = ctx.key_register(m.key, stream)
    ctx.encrypt_async(slot, m.iv, aad_d, pt_d, ct_d, tag_d, ws, stream)
    torch.cuda.synchronize()
    ct = ct_d.cpu().numpy()
    assert bytes(tag_d.cpu().numpy()) == ref_tag, "tag differs from OpenSSL"
    assert np.array_equal(ct, ref_ct), "ciphertext differs from OpenSSL"
    _check_sampled(m.key, m.iv, m.data, ct, 21, "config 2")

    print("[fullsize] config 2: one-shot encrypt and decrypt-verify", flush=True)
    ct2_d = torch.empty_like(pt_d)
    assert ctx.encrypt(m.key, m.iv, aad_d, pt_d, ct2_d) == ref_tag
    assert torch.equal(ct2_d, ct_d)
    del ct2_d
    back_d = torch.full_like(pt_d, 0x5A)
    ok_d = torch.zeros(1, dtype=torch.int32, device=dev)
    ctx.decrypt_verify_async(slot, m.iv, aad_d, ct_d, tag_d, back_d, ok_d, ws, stream)
    torch.cuda.synchronize()
    assert int(ok_d.cpu()[0]) == 1 and torch.equal(back_d, pt_d)
    bad = bytearray(ref_tag)
    bad[15] ^= 0x80
    assert ctx.decrypt_verify(m.key, m.iv, aad_d, ct_d, bytes(bad), back_d) is False
    assert not bool(back_d.any()), "rejected output not zero-filled"
    ctx.key_release(slot)
    del pt_d, ct_d, back_d, ws
    torch.cuda.empty_cache()


def test_config3_batch_4096_messages_full_size(ctx):
    """4096 lognormal messages (~8 GiB) with per-message AES-128/256 keys and
    0..4 KiB AAD in one persistent launch replayed from a hipGraph: every
    tag and ciphertext against OpenSSL, sampled blocks of 32 messages and the
    16 shortest messages whole against the oracle."""
    spec = workloads.config3_spec()
    n_msgs = len(spec.lengths)
    lay = gcm.BatchLayout(spec.lengths, spec.aad_lens)
    dev = torch.device("cuda:0")
    print(f"[fullsize] config 3: {n_msgs} messages, {int(spec.lengths.sum())} payload bytes", flush=True)
    base = torch.empty(lay.total, dtype=torch.uint8, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(spec.seed)
    for i in range(n_msgs):  # the same seeded device bytes bench.py encrypts
        a, k = lay.aad_off[i], lay.aad_lens[i]
        if k:
            base[a:a + k].random_(0, 256, generator=g)
        o, k = lay.in_off[i], lay.lengths[i]
        if k:
            base[o:o + k].random_(0, 256, generator=g)
    stream = torch.cuda.current_stream()
    slots = ctx.key_register_many(spec.keys, stream)
    b = gcm.Batch(ctx, lay.jobs([0] * n_msgs, slots, spec.ivs), base)
    b.graph_launch(stream)
    b.graph_launch(stream)  # replays must give the same bytes
    torch.cuda.synchronize()
    host = base.cpu().numpy()
    b.close()
    for s in slots:
        ctx.key_release(s)
    del base
    torch.cuda.empty_cache()

    print("[fullsize] config 3: OpenSSL over every message", flush=True)
    r = np.random.default_rng(33)
    sample = set(int(x) for x in r.choice(n_msgs, 32, replace=False))
    shortest = set(int(x) for x in np.argsort(spec.lengths, kind="stable")[:16])
    import oracle

    for i in range(n_msgs):
        aad = host[lay.aad_off[i]:lay.aad_off[i] + lay.aad_lens[i]].tobytes()
        pt = host[lay.in_off[i]:lay.in_off[i] + lay.lengths[i]]
        got = host[lay.out_off[i]:lay.out_off[i] + lay.lengths[i]]
        tag = host[lay.tag_base + 16 * i:lay.tag_base + 16 * i + 16].tobytes()
        rct, rtag = ref.gcm_encrypt_np(spec.keys[i], spec.ivs[i], aad, pt)
        assert tag == rtag, f"message {i}: tag differs from OpenSSL"
        assert np.array_equal(got, rct), f"message {i}: ciphertext differs from OpenSSL"
        if i in sample:
            _check_sampled(spec.keys[i], spec.ivs[i], pt, got, 100 + i, f"config 3 message {i}")
        if i in shortest:
            oct_, otag = oracle.gcm_encrypt(spec.keys[i], spec.ivs[i], aad, pt)
            assert otag == tag and np.array_equal(oct_, got), f"message {i}: differs from the oracle"


def test_config4_decrypt_batch_1024_files_full_size(ctx):
    """1024 FITS-shaped 4096x4096 float32 files under per-file AES-256 keys,
    5% with one flipped tag or ciphertext bit, decrypt-verified in one
    persistent launch: the rejected set is exactly the tampered set, rejected
    outputs are zero, accepted outputs are the original images, and the
    ciphertexts of sampled files match OpenSSL and the oracle's blocks."""
    n_files, side, n_base = 1024, 4096, 8
    print("[fullsize] config 4: generating 8 distinct 64 MiB images", flush=True)
    imgs = [workloads.fits_image_bytes(workloads.rng_for(2602, 4, 10 + k), side, side, n_sources=100)
            for k in range(n_base)]
    hdrs = [np.frombuffer(workloads.fits_header(workloads.rng_for(2602, 4, 30 + k)), np.uint8).copy()
            for k in range(n_base)]
    size = imgs[0].size
    keys, ivs = workloads.config4_keys(n_files=n_files)
    lay = gcm.BatchLayout([size] * n_files, [2880] * n_files)
    dev = torch.device("cuda:0")
    base = torch.empty(lay.total, dtype=torch.uint8, device=dev)
    dimg = [torch.from_numpy(x).to(dev) for x in imgs]
    dhdr = [torch.from_numpy(h).to(dev) for h in hdrs]
    for i in range(n_files):
        base[lay.in_off[i]:lay.in_off[i] + size].copy_(dimg[i % n_base])
        base[lay.aad_off[i]:lay.aad_off[i] + 2880].copy_(dhdr[i % n_base])
    stream = torch.cuda.current_stream()
    slots = ctx.key_register_many(keys, stream)
    enc = lay.jobs([0] * n_files, slots, ivs)
    for j in enc:
        j.out_off = j.in_off  # encrypt in place: the ciphertexts become the decrypt inputs
    eb = gcm.Batch(ctx, enc, base)
    eb.launch(stream)
    torch.cuda.synchronize()
    eb.close()

    print("[fullsize] config 4: sampled files against OpenSSL and the oracle", flush=True)
    for f in (0, 1, 517, 1023):
        ct = base[lay.in_off[f]:lay.in_off[f] + size].cpu().numpy()
        tag = base[lay.tag_base + 16 * f:lay.tag_base + 16 * f + 16].cpu().numpy().tobytes()
        rct, rtag = ref.gcm_encrypt_np(keys[f], ivs[f], hdrs[f % n_base].tobytes(), imgs[f % n_base])
        assert tag == rtag and np.array_equal(ct, rct), f"file {f}: differs from OpenSSL"
        _check_sampled(keys[f], ivs[f], imgs[f % n_base], ct, 400 + f, f"config 4 file {f}")

    plan = workloads.tamper_plan(2602, n_files)
    for f, (where, frac, bit) in plan.items():
        pos = lay.tag_base + 16 * f + int(frac * 16) if where == "tag" else lay.in_off[f] + int(frac * size)
        base[pos] ^= (1 << bit)
    b = gcm.Batch(ctx, lay.jobs([1] * n_files, slots, ivs), base)
    b.graph_launch(stream)
    torch.cuda.synchronize()
    ok = base[lay.ok_base:lay.ok_base + 4 * n_files].view(torch.int32).cpu().numpy()
    assert set(np.unique(ok).tolist()) <= {0, 1}
    rejected = set(int(i) for i in np.nonzero(ok == 0)[0])
    assert rejected == set(plan), "rejected set differs from the tampered set"
    for f in range(n_files):
        out = base[lay.out_off[f]:lay.out_off[f] + size]
        if f in rejected:
            assert not bool(out.any()), f"file {f}: rejected output not zero-filled"
        else:
            assert torch.equal(out, dimg[f % n_base]), f"file {f}: plaintext differs from the original image"
    b.close()
    for s in slots:
        ctx.key_release(s)
    del base, dimg
    torch.cuda.empty_cache()
