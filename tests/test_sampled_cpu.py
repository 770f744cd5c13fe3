"""CPU pins of the block-sampling helper used by the full-size GPU tests:
every sampled block equals the oracle's whole-message ciphertext, including a
ragged final block and a counter that wraps past 2^32 - 1."""
import numpy as np

import oracle
import referee_openssl as ref
import sampled


def test_sampled_blocks_equal_whole_message_encryption():
    r = np.random.default_rng(11)
    key, iv = r.bytes(32), r.bytes(12)
    pt = r.integers(0, 256, 16 * 300 + 7, dtype=np.uint8)
    ct, _ = oracle.gcm_encrypt(key, iv, b"hdr", pt)
    nb = (pt.size + 15) // 16
    idx = sampled.sample_indices(nb, r, edge=5, k=40)
    assert idx[0] == 0 and idx[-1] == nb - 1
    for j, blk in sampled.oracle_blocks(key, iv, pt, idx).items():
        assert np.array_equal(blk, ct[16 * j:16 * j + 16]), j


def test_sampled_counter_wraps_like_the_oracle():
    # block j = 2^32 - 3 has counter 0xFFFFFFFF; the oracle's GCTR steps the
    # next block to counter 0 (inc32), which is what block j + 1 must use
    key, iv = bytes(range(16)), bytes(range(12))
    j = 2**32 - 3
    assert sampled.counter_block(iv, j) == iv + b"\xff\xff\xff\xff"
    assert sampled.counter_block(iv, j + 1) == iv + bytes(4)
    two = oracle.gctr(key, sampled.counter_block(iv, j), bytes(32))
    assert np.array_equal(two[16:], oracle.gctr(key, sampled.counter_block(iv, j + 1), bytes(16)))


def test_numpy_referee_equals_bytes_referee():
    r = np.random.default_rng(12)
    key, iv, aad = r.bytes(32), r.bytes(12), r.bytes(2880)
    pt = r.integers(0, 256, 100_003, dtype=np.uint8)
    ct1, tag1 = ref.gcm_encrypt(key, iv, aad, pt.tobytes())
    ct2, tag2 = ref.gcm_encrypt_np(key, iv, aad, pt)
    assert tag1 == tag2 and ct1 == ct2.tobytes()
    ct3, tag3 = oracle.gcm_encrypt(key, iv, aad, pt)
    assert tag3 == tag2 and np.array_equal(ct3, ct2)
