"""Write the oracle's expected results for the full-size workloads.

The CPU oracle (``oracle/``) encrypts every seeded input of the full-size
GPU tests here, once, and this script stores what it produced: per message
the 16-byte tag and the SHA-256 of the ciphertext, plus SHA-256 digests of
the inputs so that a test notices when a generator no longer produces the
bytes the expected values were computed from.  Nothing here comes from the
GPU path: inputs come from ``paper_2602_23067_amd.workloads`` (seeded numpy
generators, no cryptographic arithmetic) and results from ``oracle`` only.

    python tests/golden/make_oracle_fullsize.py [config2 config3 config4 serving] [--threads N]

Outputs (JSON, next to this script):
    oracle_config2.json   AES-256-GCM of the 1 GiB FITS-shaped buffer
    oracle_config3.json   all 4096 messages of the uneven batch
    oracle_config4.json   eight of the 1024 FITS-shaped 64 MiB files
    oracle_serving.json   every request of the serving parity test

The oracle runs at a few MB/s per core, so the full set takes tens of
minutes of CPU time; messages are spread over a thread pool (the oracle's
C calls release the interpreter lock).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2602_23067_amd import workloads  # noqa: E402

SEED = 2602
CONFIG4_FILES = (0, 1, 2, 3, 517, 1020, 1022, 1023)
CONFIG4_SIDE, CONFIG4_BASES = 4096, 8


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8).tobytes() if isinstance(a, np.ndarray) else a).hexdigest()


def config4_inputs(k: int):
    """Base image k and its header (the config-4 files reuse eight bases)."""
    img = workloads.fits_image_bytes(workloads.rng_for(SEED, 4, 10 + k), CONFIG4_SIDE, CONFIG4_SIDE, n_sources=100)
    hdr = np.frombuffer(workloads.fits_header(workloads.rng_for(SEED, 4, 30 + k)), np.uint8).copy()
    return img, hdr


def write(name: str, doc: dict) -> None:
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(f"wrote {path}", flush=True)


def header(what: str) -> dict:
    return {"what": what, "seed": SEED, "written_by": "tests/golden/make_oracle_fullsize.py (oracle/ only)"}


def run_config2(pool) -> None:
    m = workloads.config2(SEED)
    t = time.time()
    ct, tag = oracle.gcm_encrypt(m.key, m.iv, m.aad, m.data)
    doc = header("config 2: AES-256-GCM of the 16384x16384 float32 FITS-shaped buffer, 2880-byte header AAD")
    doc.update(len=int(m.data.size), aad_len=int(m.aad.size), pt_sha256=sha(m.data), aad_sha256=sha(m.aad),
               key_sha256=sha(m.key), iv=m.iv.hex(), tag=tag.hex(), ct_sha256=sha(ct),
               oracle_seconds=round(time.time() - t, 1))
    write("oracle_config2.json", doc)


def run_config3(pool) -> None:
    spec = workloads.config3_spec(SEED)
    n = len(spec.lengths)

    def one(i):
        aad = workloads.batch_payload(spec, i, aad=True)
        pt = workloads.batch_payload(spec, i)
        ct, tag = oracle.gcm_encrypt(spec.keys[i], spec.ivs[i], aad, pt)
        return i, sha(aad), sha(pt), tag.hex(), sha(ct)

    rows = [None] * n
    t = time.time()
    for k, (i, ah, ph, tag, ch) in enumerate(pool.map(one, range(n))):
        rows[i] = (ah, ph, tag, ch)
        if k % 256 == 255:
            print(f"config 3: {k + 1}/{n} messages ({time.time() - t:.0f} s)", flush=True)
    write_config3(spec, rows, round(time.time() - t, 1))


def config3_inputs_digest(rows) -> str:
    """SHA-256 over the concatenated hex digests (AAD, then payload) of every message."""
    return hashlib.sha256("".join(ah + ph for ah, ph, _, _ in rows).encode()).hexdigest()


def write_config3(spec, rows, seconds) -> None:
    # per message: the tag and the first 128 bits of the ciphertext's SHA-256
    doc = header("config 3: 4096 uneven messages, per-message AES-128/256 keys, IVs and 0..4 KiB AAD; payload and "
                 "AAD of message i from workloads.batch_payload")
    doc.update(n=len(rows), total_len=int(spec.lengths.sum()), lengths_sha256=sha(spec.lengths.astype("<i8")),
               inputs_sha256=config3_inputs_digest(rows), tags=[r[2] for r in rows],
               ct_sha256_128=[r[3][:32] for r in rows], oracle_seconds=seconds)
    path = os.path.join(HERE, "oracle_config3.json")
    with open(path, "w") as f:
        json.dump(doc, f)
        f.write("\n")
    print(f"wrote {path}", flush=True)


def run_config4(pool) -> None:
    keys, ivs = workloads.config4_keys(SEED, 1024)

    def one(f):
        img, hdr = config4_inputs(f % CONFIG4_BASES)
        ct, tag = oracle.gcm_encrypt(keys[f], ivs[f], hdr, img)
        return f, sha(hdr), sha(img), tag.hex(), sha(ct)

    rows = {}
    t = time.time()
    for f, hh, ih, tag, ch in pool.map(one, CONFIG4_FILES):
        rows[str(f)] = {"aad_sha256": hh, "pt_sha256": ih, "tag": tag, "ct_sha256": ch}
    doc = header("config 4: AES-256-GCM of sampled FITS-shaped 4096x4096 float32 files (file f uses base image "
                 "f mod 8 and its header), before tampering")
    doc.update(files=rows, oracle_seconds=round(time.time() - t, 1))
    write("oracle_config4.json", doc)


def run_serving(pool) -> None:
    cases = workloads.serving_parity_spec(SEED)
    keys = workloads.serving_key_table(SEED)

    def one(i):
        c = cases[i]
        aad, pt = workloads.serving_case_data(SEED, i, c)
        ct, tag = oracle.gcm_encrypt(keys[c.key_index], c.iv, aad, pt)
        return i, sha(aad), sha(pt), tag.hex(), sha(ct)

    rows = [None] * len(cases)
    t = time.time()
    # largest first, so the two 256 MiB requests do not finish last
    order = sorted(range(len(cases)), key=lambda i: -cases[i].size)
    for i, ah, ph, tag, ch in pool.map(one, order):
        rows[i] = {"op": cases[i].op, "size": cases[i].size, "aad_sha256": ah, "pt_sha256": ph, "tag": tag,
                   "ct_sha256": ch}
    doc = header("serving parity requests: sizes from the serving workload's lognormal (two of 256 MiB), "
                 "FITS-shaped noise payloads, 2880-byte header AAD, keys from the 1024-entry table; tag and "
                 "ciphertext digest of each payload's encryption (a decrypt request's input is that ciphertext)")
    doc.update(n=len(cases), requests=rows, oracle_seconds=round(time.time() - t, 1))
    write("oracle_serving.json", doc)


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", default=["config2", "config3", "config4", "serving"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 4)
    a = ap.parse_args()
    oracle.build(force=False)
    jobs = {"config2": run_config2, "config3": run_config3, "config4": run_config4, "serving": run_serving}
    with cf.ThreadPoolExecutor(a.threads) as pool:
        for w in a.which:
            jobs[w](pool)


if __name__ == "__main__":
    main()
