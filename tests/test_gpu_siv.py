"""GPU parity of AES-GCM-SIV (RFC 8452): ciphertext and tag bit for bit
against the oracle, decrypt-verify of the oracle's output, every rejection
zero-filling the plaintext, a counter that wraps inside the message, writes
kept inside the output (canaries), and sampled keystream blocks at 1 GiB."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import siv_util  # noqa: E402
from paper_2602_23067_amd import gcm  # noqa: E402

pytestmark = pytest.mark.gpu

from gpu_util import canaries_intact, guarded, host, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gcm.Context(device=0, key_slots=16)
    yield c
    c.close()


def _enc(ctx, slot, nonce, aad, pt):
    aad_d = to_dev(aad) if aad.size else None
    full, ct_d = guarded(pt.size)
    pt_d = to_dev(pt) if pt.size else None
    tag_d = torch.zeros(16, dtype=torch.uint8, device="cuda")
    ws = ctx.siv_encrypt_async(slot, nonce, aad_d, pt_d, ct_d if pt.size else None, tag_d)
    torch.cuda.synchronize()
    del ws
    assert canaries_intact(full, pt.size)
    return host(ct_d), bytes(host(tag_d))


def _dec(ctx, slot, nonce, aad, ct, tag):
    aad_d = to_dev(aad) if aad.size else None
    full, pt_d = guarded(ct.size)
    ct_d = to_dev(ct) if ct.size else None
    tag_d = to_dev(np.frombuffer(tag, np.uint8))
    ok_d = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    ctx.siv_decrypt_verify_async(slot, nonce, aad_d, ct_d, tag_d, pt_d if ct.size else None, ok_d)
    torch.cuda.synchronize()
    assert canaries_intact(full, ct.size)
    return host(pt_d), int(host(ok_d)[0])


CASES = [
    # (seed, key bytes, AAD bytes, data bytes)
    (1, 16, 0, 0),
    (2, 32, 0, 1),
    (3, 16, 7, 15),
    (4, 32, 16, 16),
    (5, 16, 33, 17),
    (6, 32, 0, 64 * 16),
    (7, 16, 5000, 64 * 16 * 5 + 7),
    (8, 32, 100_000, (1 << 20) + 3),
    (9, 16, 0, 16 << 20),
    (10, 32, 3, (4 << 20) + 1),
    (11, 16, 70_000, 0),
]


@pytest.mark.parametrize("seed,klen,na,n", CASES)
def test_siv_matches_oracle(ctx, seed, klen, na, n):
    r = np.random.default_rng(9000 + seed)
    kgk, nonce = r.bytes(klen), r.bytes(12)
    aad = r.integers(0, 256, na, dtype=np.uint8)
    pt = r.integers(0, 256, n, dtype=np.uint8)
    print(f"siv seed={seed} key={klen} aad={na} n={n}", flush=True)
    rct, rtag = oracle.gcm_siv_encrypt(kgk, nonce, aad, pt)
    slot = ctx.key_register(kgk)
    try:
        for shape in [(0, 0, 0), (8, 16, 0), (6, 8, 0)]:
            ctx.set_launch(*shape)
            try:
                ct, tag = _enc(ctx, slot, nonce, aad, pt)
                assert np.array_equal(ct, rct), f"ciphertext, shape {shape}"
                assert tag == rtag, f"tag, shape {shape}"
                back, ok = _dec(ctx, slot, nonce, aad, rct, rtag)
                assert ok == 1 and np.array_equal(back, pt), f"decrypt, shape {shape}"
            finally:
                ctx.set_launch(0, 0, 0)
    finally:
        ctx.key_release(slot)


def test_siv_rejections_zero_fill(ctx):
    r = np.random.default_rng(9100)
    kgk, nonce = r.bytes(32), r.bytes(12)
    aad = r.integers(0, 256, 300, dtype=np.uint8)
    pt = r.integers(0, 256, (1 << 20) + 9, dtype=np.uint8)
    ct, tag = oracle.gcm_siv_encrypt(kgk, nonce, aad, pt)
    slot = ctx.key_register(kgk)
    try:
        bad_ct = ct.copy()
        bad_ct[777_777] ^= 4
        bad_aad = aad.copy()
        bad_aad[0] ^= 1
        bad_nonce = bytes([nonce[0] ^ 1]) + nonce[1:]
        for args in [(nonce, aad, ct, bytes([tag[0] ^ 0x80]) + tag[1:]), (nonce, aad, bad_ct, tag),
                     (nonce, bad_aad, ct, tag), (bad_nonce, aad, ct, tag), (nonce, aad[:299], ct, tag)]:
            got, ok = _dec(ctx, slot, *args)
            want, want_ok = oracle.gcm_siv_decrypt_verify(kgk, *args)
            assert ok == 0 and not want_ok
            assert not got.any() and np.array_equal(got, want)
    finally:
        ctx.key_release(slot)


def test_siv_in_place(ctx):
    r = np.random.default_rng(9200)
    kgk, nonce = r.bytes(16), r.bytes(12)
    pt = r.integers(0, 256, 3 * (1 << 20) + 1, dtype=np.uint8)
    rct, rtag = oracle.gcm_siv_encrypt(kgk, nonce, b"", pt)
    slot = ctx.key_register(kgk)
    try:
        buf = to_dev(pt)
        tag_d = torch.zeros(16, dtype=torch.uint8, device="cuda")
        ctx.siv_encrypt_async(slot, nonce, None, buf, buf, tag_d)
        assert np.array_equal(host(buf), rct) and bytes(host(tag_d)) == rtag
        ok_d = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        ctx.siv_decrypt_verify_async(slot, nonce, None, buf, tag_d, buf, ok_d)
        assert int(host(ok_d)[0]) == 1 and np.array_equal(host(buf), pt)
    finally:
        torch.cuda.synchronize()
        ctx.key_release(slot)


def test_siv_counter_wraps(ctx):
    r = np.random.default_rng(9300)
    kgk, nonce = r.bytes(32), r.bytes(12)
    pt = r.integers(0, 256, 16 * 65536 + 5, dtype=np.uint8)
    aad_b, c0 = siv_util.wrapping_aad(kgk, nonce, pt, seed=93)
    aad = np.frombuffer(aad_b, np.uint8)
    print(f"wrapping counter {c0:#x}", flush=True)
    rct, rtag = oracle.gcm_siv_encrypt(kgk, nonce, aad, pt)
    slot = ctx.key_register(kgk)
    try:
        ct, tag = _enc(ctx, slot, nonce, aad, pt)
        assert np.array_equal(ct, rct) and tag == rtag
        back, ok = _dec(ctx, slot, nonce, aad, rct, rtag)
        assert ok == 1 and np.array_equal(back, pt)
    finally:
        ctx.key_release(slot)


def test_siv_errors(ctx):
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    tag_d = torch.zeros(16, dtype=torch.uint8, device="cuda")
    s24 = ctx.key_register(bytes(24))
    s16 = ctx.key_register(bytes(16))
    try:
        with pytest.raises(gcm.GcmError) as e:
            ctx.siv_encrypt_async(s24, bytes(12), None, buf, buf, tag_d)
        assert e.value.code == gcm.GCM_E_KEYLEN
        with pytest.raises(gcm.GcmError) as e:
            ctx.siv_encrypt_async(s16, bytes(16), None, buf, buf, tag_d)
        assert e.value.code == gcm.GCM_E_IVLEN
        ws = torch.empty(ctx.siv_workspace_size(64, 0) + 256, dtype=torch.uint8, device="cuda")
        with pytest.raises(gcm.GcmError) as e:
            ctx.siv_encrypt_async(s16, bytes(12), None, buf, buf, tag_d, workspace=ws[16:])
        assert e.value.code == gcm.GCM_E_ARG
        with pytest.raises(gcm.GcmError) as e:
            ctx.siv_encrypt_async(s16, bytes(12), None, buf, buf, tag_d, workspace=ws[:1024])
        assert e.value.code == gcm.GCM_E_ARG
        with pytest.raises(gcm.GcmError) as e:
            ctx.siv_encrypt_async(s16, bytes(12), None, buf[:32], buf[16:48], tag_d)
        assert e.value.code == gcm.GCM_E_ALIAS
        with pytest.raises(gcm.GcmError) as e:
            ctx.siv_encrypt_async(15, bytes(12), None, buf, buf, tag_d)
        assert e.value.code == gcm.GCM_E_SLOT
    finally:
        torch.cuda.synchronize()
        ctx.key_release(s24)
        ctx.key_release(s16)


def test_siv_full_size_sampled(ctx):
    """1 GiB in the benchmark's launch shape: sampled ciphertext blocks
    against the oracle's keystream for the device tag (derived key, counter
    block from the tag), the round trip, and a rejection."""
    n = 1 << 30
    r = np.random.default_rng(9400)
    kgk, nonce = r.bytes(16), r.bytes(12)
    g = torch.Generator(device="cuda")
    g.manual_seed(94)
    pt_d = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda", generator=g)
    ct_d = torch.empty_like(pt_d)
    aad_d = to_dev(r.integers(0, 256, 4096, dtype=np.uint8))
    tag_d = torch.zeros(16, dtype=torch.uint8, device="cuda")
    slot = ctx.key_register(kgk)
    try:
        print("siv 1 GiB encrypt", flush=True)
        ws = ctx.siv_encrypt_async(slot, nonce, aad_d, pt_d, ct_d, tag_d)
        torch.cuda.synchronize()
        tag = bytes(host(tag_d))
        _, enc = oracle.gcm_siv_derive(kgk, nonce)
        c0 = int.from_bytes(tag[:4], "little")
        rest = tag[4:15] + bytes([tag[15] | 0x80])
        idx = np.unique(np.concatenate([[0, 1, 63, 64, n // 16 - 1], r.integers(0, n // 16, 200)]))
        blocks = torch.from_numpy(idx.astype(np.int64)).to("cuda")
        pt_s = host(pt_d.view(-1, 16)[blocks])
        ct_s = host(ct_d.view(-1, 16)[blocks])
        for k, i in enumerate(idx):
            ks = oracle.aes_encrypt_block(enc, ((c0 + int(i)) % 2**32).to_bytes(4, "little") + rest)
            assert np.array_equal(ct_s[k], pt_s[k] ^ np.frombuffer(ks, np.uint8)), int(i)
        print("siv 1 GiB decrypt", flush=True)
        back_d = torch.empty_like(pt_d)
        ok_d = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        ctx.siv_decrypt_verify_async(slot, nonce, aad_d, ct_d, tag_d, back_d, ok_d, workspace=ws)
        torch.cuda.synchronize()
        assert int(host(ok_d)[0]) == 1 and bool(torch.equal(back_d, pt_d))
        ct_d[n // 2] ^= 1
        ctx.siv_decrypt_verify_async(slot, nonce, aad_d, ct_d, tag_d, back_d, ok_d, workspace=ws)
        torch.cuda.synchronize()
        assert int(host(ok_d)[0]) == 0 and int(back_d.count_nonzero()) == 0
    finally:
        torch.cuda.synchronize()
        ctx.key_release(slot)


def test_siv_two_streams_and_odd_tag_offset(ctx):
    """Two messages in flight on two HIP streams at once, each with its own
    workspace (nothing else is shared but read-only key data), and tags at
    odd device offsets (the tag may sit anywhere)."""
    r = np.random.default_rng(9500)
    kgk, n1, n2 = r.bytes(32), r.bytes(12), r.bytes(12)
    p1 = r.integers(0, 256, (2 << 20) + 7, dtype=np.uint8)
    p2 = r.integers(0, 256, (3 << 20) + 1, dtype=np.uint8)
    a1 = r.integers(0, 256, 100, dtype=np.uint8)
    c1, t1 = oracle.gcm_siv_encrypt(kgk, n1, a1, p1)
    c2, t2 = oracle.gcm_siv_encrypt(kgk, n2, b"", p2)
    slot = ctx.key_register(kgk)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    try:
        pt1, pt2, aad1 = to_dev(p1), to_dev(p2), to_dev(a1)
        ct1, ct2 = torch.empty_like(pt1), torch.empty_like(pt2)
        tags = torch.zeros(64, dtype=torch.uint8, device="cuda")
        ws1 = torch.empty(ctx.siv_workspace_size(p1.size, a1.size), dtype=torch.uint8, device="cuda")
        ws2 = torch.empty(ctx.siv_workspace_size(p2.size, 0), dtype=torch.uint8, device="cuda")
        torch.cuda.current_stream().synchronize()
        ctx.siv_encrypt_async(slot, n1, aad1, pt1, ct1, tags[3:19], workspace=ws1, stream=s1)
        ctx.siv_encrypt_async(slot, n2, None, pt2, ct2, tags[37:53], workspace=ws2, stream=s2)
        s1.synchronize()
        s2.synchronize()
        assert np.array_equal(host(ct1), c1) and bytes(host(tags[3:19])) == t1
        assert np.array_equal(host(ct2), c2) and bytes(host(tags[37:53])) == t2
        ok = torch.full((2,), -1, dtype=torch.int32, device="cuda")
        b1, b2 = torch.empty_like(pt1), torch.empty_like(pt2)
        ctx.siv_decrypt_verify_async(slot, n1, aad1, ct1, tags[3:19], b1, ok[0:1], workspace=ws1, stream=s1)
        ctx.siv_decrypt_verify_async(slot, n2, None, ct2, tags[37:53], b2, ok[1:2], workspace=ws2, stream=s2)
        s1.synchronize()
        s2.synchronize()
        assert host(ok).tolist() == [1, 1]
        assert np.array_equal(host(b1), p1) and np.array_equal(host(b2), p2)
    finally:
        torch.cuda.synchronize()
        ctx.key_release(slot)
