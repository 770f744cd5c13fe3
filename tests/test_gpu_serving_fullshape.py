"""Serving parity at the serving workload's own shape: requests drawn from
its size distribution (lognormal, median 4 MiB, two of 256 MiB), FITS-shaped
payloads with 2880-byte header AAD, keys from a resident 1024-entry table,
a 64 GiB HBM budget, mixed encrypt and decrypt-verify with tampered
decrypts, submitted with exponential gaps while earlier batches run.

Every encrypt's tag and ciphertext digest equal the CPU oracle's (written by
tests/golden/make_oracle_fullsize.py over the same seeded inputs), every
decrypt input is OpenSSL's encryption of the payload whose tag equals the
oracle's, untampered decrypts return the payload and tampered ones are
rejected and zero-filled, and every result equals the same request run
alone through the one-launch-per-message asynchronous call."""
import hashlib
import json
import os
import threading
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import referee_openssl as ref  # noqa: E402
from paper_2602_23067_amd import gcm, workloads  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

SEED = 2602
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_serving.json")


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8).tobytes()).hexdigest()


def test_serving_workload_shape_matches_oracle_and_alone():
    cases = workloads.serving_parity_spec(SEED)
    keys = workloads.serving_key_table(SEED)
    want = json.load(open(GOLDEN))["requests"]
    assert len(want) == len(cases)
    assert max(c.size for c in cases) >= 256 << 20 and len(keys) == 1024
    dev = torch.device("cuda:0")
    ctx = gcm.Context(device=0, key_slots=1024)
    try:
        slots = ctx.key_register_many(keys)
        print(f"[serving] {len(cases)} requests, {sum(c.size for c in cases)} payload bytes", flush=True)
        reqs = []
        for i, c in enumerate(cases):
            aad, pt = workloads.serving_case_data(SEED, i, c)
            w = want[i]
            assert (sha(aad), sha(pt), w["size"], w["op"]) == (w["aad_sha256"], w["pt_sha256"], c.size, c.op), \
                f"request {i}: input generator drifted from the oracle's expected values"
            tag = bytes.fromhex(w["tag"])
            if c.op == 0:
                src = pt
            else:
                ct, rtag = ref.gcm_encrypt_np(keys[c.key_index], c.iv, aad.tobytes(), pt)
                assert rtag == tag and sha(ct) == w["ct_sha256"], f"request {i}: OpenSSL differs from the oracle"
                src = ct
                if c.tamper:
                    where, frac, bit = c.tamper
                    if where == "tag":
                        t = bytearray(tag)
                        t[int(frac * 16)] ^= 1 << bit
                        tag = bytes(t)
                    else:
                        src = ct.copy()
                        src[int(frac * c.size)] ^= 1 << bit
            tag_d = torch.from_numpy(np.frombuffer(tag if c.op == 1 else bytes(16), np.uint8).copy()).to(dev)
            reqs.append(dict(aad=torch.from_numpy(aad).to(dev), inp=torch.from_numpy(src).to(dev),
                             out=torch.full((c.size,), 0x5A, dtype=torch.uint8, device=dev), tag=tag_d,
                             pt_sha=w["pt_sha256"]))
        torch.cuda.synchronize()

        srv = gcm.Server(ctx, n_streams=4, hbm_budget=64 << 30)
        ids = [None] * len(cases)
        gaps = workloads.rng_for(SEED, 5, 9).exponential(40e-6, len(cases))

        def submitter():
            for i, (c, q) in enumerate(zip(cases, reqs)):
                ids[i] = srv.submit(c.op, slots[c.key_index], c.iv, q["aad"], q["inp"], q["out"], q["tag"])
                t_end = time.perf_counter() + float(gaps[i])
                while time.perf_counter() < t_end:
                    pass

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        results = [srv.wait(i) for i in ids]
        st = srv.stats()
        srv.stop()
        print("[serving] stats:", st, flush=True)
        torch.cuda.synchronize()
        assert st["completed"] == len(cases) and st["failed"] == 0
        assert st["budget_high_water"] <= 64 << 30
        assert st["rejected"] == sum(1 for c in cases if c.tamper)

        print("[serving] every result against the oracle and against the request run alone", flush=True)
        ws = torch.zeros(max(ctx.workspace_size(c.size, 2880) for c in cases), dtype=torch.uint8, device=dev)
        ok_d = torch.zeros(1, dtype=torch.int32, device=dev)
        for i, (c, q, (acc, lat)) in enumerate(zip(cases, reqs, results)):
            out = q["out"].cpu().numpy()
            assert lat > 0
            if c.op == 0:
                assert acc and q["tag"].cpu().numpy().tobytes().hex() == want[i]["tag"], f"request {i}: tag"
                assert sha(out) == want[i]["ct_sha256"], f"request {i}: ciphertext differs from the oracle's"
            elif c.tamper:
                assert not acc and not out.any(), f"request {i}: tampered decrypt not rejected and zero-filled"
            else:
                assert acc and sha(out) == q["pt_sha"], f"request {i}: plaintext differs from the payload"
            # the same request alone, one launch sequence of its own
            alone = torch.full_like(q["out"], 0x33)
            if c.op == 0:
                tag2 = torch.zeros(16, dtype=torch.uint8, device=dev)
                ctx.encrypt_async(slots[c.key_index], c.iv, q["aad"], q["inp"], alone, tag2, ws)
                torch.cuda.synchronize()
                assert torch.equal(tag2, q["tag"]), f"request {i}: tag alone differs from the served tag"
            else:
                ctx.decrypt_verify_async(slots[c.key_index], c.iv, q["aad"], q["inp"], q["tag"], alone, ok_d, ws)
                torch.cuda.synchronize()
                assert int(ok_d.cpu()[0]) == int(acc), f"request {i}: verdict alone differs"
            assert torch.equal(alone, q["out"]), f"request {i}: output alone differs from the served output"
    finally:
        ctx.close()
        torch.cuda.empty_cache()
