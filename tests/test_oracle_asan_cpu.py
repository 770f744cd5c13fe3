"""The CPU oracle built with AddressSanitizer and UBSan and run on exact-size
buffers (every tail length 0..70, several key, IV, AAD and truncated tag
lengths); its outputs must equal the normally built oracle's."""
import os
import subprocess

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _filled(n, seed):
    out = bytearray()
    for _ in range(n):
        seed = (seed * 1664525 + 1013904223) & 0xFFFFFFFF
        out.append(seed >> 24)
    return bytes(out)


def _fnv(b):
    h = 1469598103934665603
    for x in b:
        h = ((h ^ x) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_asan"
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-D_POSIX_C_SOURCE=200112L", "-pthread",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "oracle", "gcm_oracle.c"), os.path.join(ROOT, "tests", "oracle_asan_driver.c"),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = out.stdout.strip().split("\n")
    assert len(lines) == 71
    for line in lines:
        ln, kl, il, al, h, tag = line.split()
        ln, kl, il, al = int(ln), int(kl), int(il), int(al)
        key, iv = _filled(kl, 1 + ln), _filled(il, 2 + ln)
        aad, pt = _filled(al, 3 + ln), _filled(ln, 4 + ln)
        ct, want = oracle.gcm_encrypt(key, iv, aad, np.frombuffer(pt, np.uint8))
        assert int(h, 16) == _fnv(ct.tobytes()) and bytes.fromhex(tag) == want, line
