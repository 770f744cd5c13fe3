"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (default launch shape, resident keys, persistent
batches replayed from a hipGraph).

Expected values come from the CPU oracle itself: tests/golden/
make_oracle_fullsize.py ran the oracle over the same seeded inputs and stored
each message's tag and the SHA-256 of its ciphertext (and digests of the
inputs, so a drifting generator fails loudly instead of comparing the wrong
thing).  OpenSSL, the second referee the oracle is pinned to, is checked as
well where it is cheap, and so are the properties that hold at any size:
decrypt-verify returns the plaintext and accepts, a flipped tag bit is
rejected with a zero-filled output, the rejected set of a tampered batch is
exactly the tampered set.
"""
import hashlib
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import referee_openssl as ref  # noqa: E402
from paper_2602_23067_amd import gcm, workloads  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gcm.Context(device=0, key_slots=4200)
    yield c
    c.close()
    torch.cuda.empty_cache()


def test_config2_fits_1gib_aes256_full_size(ctx):
    """AES-256-GCM of the 16384x16384 float32 FITS-shaped buffer with its
    2880-byte header as AAD, through the resident-key path the benchmark
    times and through the one-shot call."""
    print("[fullsize] config 2: generating 1 GiB FITS-shaped input", flush=True)
    m = workloads.config2()
    n = m.data.size
    want = golden("oracle_config2.json")
    assert (sha(m.data), sha(m.aad), m.iv.hex()) == (want["pt_sha256"], want["aad_sha256"], want["iv"]), \
        "config 2 input generator drifted from the oracle's expected values"
    ref_tag = bytes.fromhex(want["tag"])
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
    assert bytes(tag_d.cpu().numpy()) == ref_tag, "tag differs from the oracle's"
    assert sha(ct) == want["ct_sha256"], "ciphertext differs from the oracle's"
    rct, rtag = ref.gcm_encrypt_np(m.key, m.iv, m.aad.tobytes(), m.data)
    assert rtag == ref_tag and np.array_equal(ct, rct), "differs from OpenSSL"
    del rct

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
    tag and every ciphertext digest against the oracle's (and every message
    against OpenSSL)."""
    spec = workloads.config3_spec()
    n_msgs = len(spec.lengths)
    want = golden("oracle_config3.json")
    assert want["n"] == n_msgs and want["total_len"] == int(spec.lengths.sum())
    lay = gcm.BatchLayout(spec.lengths, spec.aad_lens)
    dev = torch.device("cuda:0")
    print(f"[fullsize] config 3: {n_msgs} messages, {int(spec.lengths.sum())} payload bytes", flush=True)
    base = torch.empty(lay.total, dtype=torch.uint8, device=dev)
    digests = []
    for i in range(n_msgs):  # the seeded host bytes the oracle encrypted
        aad = workloads.batch_payload(spec, i, aad=True)
        pt = workloads.batch_payload(spec, i)
        digests.append(sha(aad) + sha(pt))
        a, k = lay.aad_off[i], lay.aad_lens[i]
        if k:
            base[a:a + k].copy_(torch.from_numpy(aad))
        o, k = lay.in_off[i], lay.lengths[i]
        if k:
            base[o:o + k].copy_(torch.from_numpy(pt))
    assert hashlib.sha256("".join(digests).encode()).hexdigest() == want["inputs_sha256"], \
        "config 3 input generator drifted from the oracle's expected values"
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

    print("[fullsize] config 3: every message against the oracle's tags and digests, and OpenSSL", flush=True)
    for i in range(n_msgs):
        got = host[lay.out_off[i]:lay.out_off[i] + lay.lengths[i]]
        tag = host[lay.tag_base + 16 * i:lay.tag_base + 16 * i + 16].tobytes()
        assert tag.hex() == want["tags"][i], f"message {i}: tag differs from the oracle's"
        assert sha(got)[:32] == want["ct_sha256_128"][i], f"message {i}: ciphertext differs from the oracle's"
        aad = host[lay.aad_off[i]:lay.aad_off[i] + lay.aad_lens[i]].tobytes()
        pt = host[lay.in_off[i]:lay.in_off[i] + lay.lengths[i]]
        rct, rtag = ref.gcm_encrypt_np(spec.keys[i], spec.ivs[i], aad, pt)
        assert tag == rtag and np.array_equal(got, rct), f"message {i}: differs from OpenSSL"


def test_config4_decrypt_batch_1024_files_full_size(ctx):
    """1024 FITS-shaped 4096x4096 float32 files under per-file AES-256 keys,
    5% with one flipped tag or ciphertext bit, decrypt-verified in one
    persistent launch: the rejected set is exactly the tampered set, rejected
    outputs are zero, accepted outputs are the original images, and the
    ciphertexts of sampled files match the oracle's tags and digests and OpenSSL."""
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

    print("[fullsize] config 4: sampled files against the oracle's tags and digests, and OpenSSL", flush=True)
    want = golden("oracle_config4.json")["files"]
    for f in sorted(int(x) for x in want):
        k = f % n_base
        assert sha(imgs[k]) == want[str(f)]["pt_sha256"] and sha(hdrs[k]) == want[str(f)]["aad_sha256"], \
            "config 4 input generator drifted from the oracle's expected values"
    for f in sorted(int(x) for x in want):
        ct = base[lay.in_off[f]:lay.in_off[f] + size].cpu().numpy()
        tag = base[lay.tag_base + 16 * f:lay.tag_base + 16 * f + 16].cpu().numpy().tobytes()
        assert tag.hex() == want[str(f)]["tag"], f"file {f}: tag differs from the oracle's"
        assert sha(ct) == want[str(f)]["ct_sha256"], f"file {f}: ciphertext differs from the oracle's"
        rct, rtag = ref.gcm_encrypt_np(keys[f], ivs[f], hdrs[f % n_base].tobytes(), imgs[f % n_base])
        assert tag == rtag and np.array_equal(ct, rct), f"file {f}: differs from OpenSSL"

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
