"""Block-sampled expected ciphertext from the oracle, for messages too large
for the oracle to encrypt whole in a test.

GCM's ciphertext block j is P_j xor CIPH_K(inc32^j(ICB)) with ICB = inc32(J0)
(SP 800-38D, GCTR function, and the GCM-AE steps that set ICB), and for a
96-bit IV J0 = IV || 0^31 || 1 (same standard, J0 definition).  So block j is
the oracle's GCTR function applied to P_j alone with the counter block
IV || [(2 + j) mod 2^32]_32.  The CPU tests pin this against the oracle's
whole-message encryption.
"""
from __future__ import annotations

from typing import Dict, Iterable

import numpy as np

import oracle


def counter_block(iv: bytes, j: int) -> bytes:
    assert len(iv) == 12, "only 96-bit IVs have J0 = IV || 0^31 || 1"
    return iv + ((2 + j) % (1 << 32)).to_bytes(4, "big")


def oracle_blocks(key: bytes, iv: bytes, pt: np.ndarray, idx: Iterable[int]) -> Dict[int, np.ndarray]:
    """{j: expected ciphertext bytes of block j} (the last block may be short)."""
    out = {}
    for j in idx:
        chunk = pt[16 * j:16 * j + 16]
        out[int(j)] = oracle.gctr(key, counter_block(iv, int(j)), chunk)
    return out


def sample_indices(n_blocks: int, rng: np.random.Generator, edge: int = 64, k: int = 256):
    """Both ends of the message plus k uniformly drawn blocks."""
    s = set(range(min(edge, n_blocks))) | set(range(max(0, n_blocks - edge), n_blocks))
    if n_blocks:
        s |= set(int(x) for x in rng.integers(0, n_blocks, k))
    return sorted(s)
