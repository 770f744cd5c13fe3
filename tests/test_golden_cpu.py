"""The stored full-size expected values are the oracle's: a sample of them
is recomputed here with the oracle from the same seeded inputs (the smallest
messages of the uneven batch, the smallest serving requests) and must match
bit for bit, and the files are complete and well formed."""
import hashlib
import json
import os

import numpy as np

import oracle
from paper_2602_23067_amd import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SEED = 2602


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8).tobytes()).hexdigest()


def test_config3_golden_is_the_oracles():
    g = load("oracle_config3.json")
    spec = workloads.config3_spec(SEED)
    assert g["n"] == len(spec.lengths) == len(g["tags"]) == len(g["ct_sha256_128"])
    assert g["total_len"] == int(spec.lengths.sum())
    assert g["lengths_sha256"] == sha(spec.lengths.astype("<i8"))
    for i in np.argsort(spec.lengths, kind="stable")[:12]:
        i = int(i)
        aad = workloads.batch_payload(spec, i, aad=True)
        pt = workloads.batch_payload(spec, i)
        ct, tag = oracle.gcm_encrypt(spec.keys[i], spec.ivs[i], aad, pt)
        assert tag.hex() == g["tags"][i] and sha(ct)[:32] == g["ct_sha256_128"][i], f"message {i}"


def test_serving_golden_is_the_oracles():
    g = load("oracle_serving.json")
    cases = workloads.serving_parity_spec(SEED)
    keys = workloads.serving_key_table(SEED)
    assert g["n"] == len(cases) == len(g["requests"])
    for i in sorted(range(len(cases)), key=lambda k: cases[k].size)[:6]:
        c, w = cases[i], g["requests"][i]
        aad, pt = workloads.serving_case_data(SEED, i, c)
        assert (w["op"], w["size"], w["aad_sha256"], w["pt_sha256"]) == (c.op, c.size, sha(aad), sha(pt))
        ct, tag = oracle.gcm_encrypt(keys[c.key_index], c.iv, aad, pt)
        assert tag.hex() == w["tag"] and sha(ct) == w["ct_sha256"], f"request {i}"


def test_serving_spec_has_the_workload_shape():
    cases = workloads.serving_parity_spec(SEED)
    sizes = [c.size for c in cases]
    assert max(sizes) >= 256 << 20 and min(sizes) >= 16 << 10
    assert all(s % 2880 == 0 for s in sizes)
    assert {c.op for c in cases} == {0, 1}
    assert any(c.tamper for c in cases) and all(c.op == 1 for c in cases if c.tamper)
    assert len(workloads.serving_key_table(SEED)) == 1024


def test_config2_and_config4_golden_are_well_formed():
    g2 = load("oracle_config2.json")
    m = workloads.config2(SEED, ny=16, nx=16, n_sources=0)  # key, IV and header only depend on the seed
    assert g2["iv"] == m.iv.hex() and g2["key_sha256"] == sha(np.frombuffer(m.key, np.uint8))
    assert g2["aad_sha256"] == sha(m.aad) and g2["len"] == 1_073_744_640 and g2["aad_len"] == 2880
    assert len(bytes.fromhex(g2["tag"])) == 16 and len(g2["ct_sha256"]) == 64
    g4 = load("oracle_config4.json")["files"]
    assert len(g4) >= 8 and {"0", "1023"} <= set(g4)
    for f in g4.values():
        assert len(bytes.fromhex(f["tag"])) == 16
