"""CPU oracle for AES-GCM -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.

The arithmetic lives in ``gcm_oracle.c`` (plain C, built with gcc -O2, no
intrinsics).  This module builds it, loads it with ctypes and wraps each entry
point with numpy/bytes marshalling.  The only arithmetic written here is the
test helper :func:`ghash_tree`, which re-brackets GHASH as the paper's binary
reduction tree ("Parallel GHASH Reduction" section and its tree figure) on top
of the oracle's own GF(2^128) product.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Callable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gcm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_gcm.so")

_lib: Optional[ctypes.CDLL] = None

OK = 0
E_ARG = -1
E_KEYLEN = -2
E_IVLEN = -3
E_TOOLONG = -4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no SIMD intrinsics)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200112L", "-Wall", "-Wextra",
               "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u8p = ctypes.c_void_p
        sz = ctypes.c_size_t
        u64 = ctypes.c_uint64
        L.oracle_gcm_encrypt.argtypes = [u8p, sz, u8p, sz, u8p, u64, u8p, u64, u8p, u8p]
        L.oracle_gcm_encrypt.restype = ctypes.c_int
        L.oracle_gcm_decrypt_verify.argtypes = [u8p, sz, u8p, sz, u8p, u64, u8p, u64, u8p, u8p,
                                                ctypes.POINTER(ctypes.c_int)]
        L.oracle_gcm_decrypt_verify.restype = ctypes.c_int
        L.oracle_gcm_decrypt_verify_t.argtypes = [u8p, sz, u8p, sz, u8p, u64, u8p, u64, u8p, sz, u8p,
                                                  ctypes.POINTER(ctypes.c_int)]
        L.oracle_gcm_decrypt_verify_t.restype = ctypes.c_int
        L.oracle_gcm_j0.argtypes = [u8p, sz, u8p, sz, u8p]
        L.oracle_gcm_j0.restype = ctypes.c_int
        L.oracle_gf8_mul.argtypes = [ctypes.c_uint8, ctypes.c_uint8]
        L.oracle_gf8_mul.restype = ctypes.c_uint8
        L.oracle_gf8_inv.argtypes = [ctypes.c_uint8]
        L.oracle_gf8_inv.restype = ctypes.c_uint8
        L.oracle_gf8_xtime.argtypes = [ctypes.c_uint8]
        L.oracle_gf8_xtime.restype = ctypes.c_uint8
        L.oracle_sbox.argtypes = [u8p]
        L.oracle_inv_sbox.argtypes = [u8p]
        L.oracle_key_expand.argtypes = [u8p, sz, u8p]
        L.oracle_key_expand.restype = ctypes.c_int
        L.oracle_aes_encrypt_block.argtypes = [u8p, sz, u8p, u8p]
        L.oracle_aes_encrypt_block.restype = ctypes.c_int
        L.oracle_aes_decrypt_block.argtypes = [u8p, sz, u8p, u8p]
        L.oracle_aes_decrypt_block.restype = ctypes.c_int
        L.oracle_gf128_mul.argtypes = [u8p, u8p, u8p]
        L.oracle_ghash.argtypes = [u8p, u8p, u64, u8p]
        L.oracle_gcm_hash.argtypes = [u8p, u8p, u64, u8p, u64, u8p]
        L.oracle_gctr.argtypes = [u8p, sz, u8p, u8p, u64, u8p]
        L.oracle_gctr.restype = ctypes.c_int
        L.oracle_gcm_siv_encrypt.argtypes = [u8p, sz, u8p, sz, u8p, u64, u8p, u64, u8p, u8p]
        L.oracle_gcm_siv_encrypt.restype = ctypes.c_int
        L.oracle_gcm_siv_decrypt_verify.argtypes = [u8p, sz, u8p, sz, u8p, u64, u8p, u64, u8p, u8p,
                                                    ctypes.POINTER(ctypes.c_int)]
        L.oracle_gcm_siv_decrypt_verify.restype = ctypes.c_int
        L.oracle_gcm_siv_derive.argtypes = [u8p, sz, u8p, u8p, u8p]
        L.oracle_gcm_siv_derive.restype = ctypes.c_int
        L.oracle_polyval.argtypes = [u8p, u8p, u64, u8p]
        L.oracle_pv_mul.argtypes = [u8p, u8p, u8p]
        _lib = L
    return _lib


# ---------------------------------------------------------------- helpers

def _buf(data) -> np.ndarray:
    """Read-only view of bytes-like / numpy input as a contiguous uint8 array."""
    if isinstance(data, np.ndarray):
        return np.ascontiguousarray(data).view(np.uint8).reshape(-1)
    return np.frombuffer(bytes(data), dtype=np.uint8)


def _ptr(a: np.ndarray):
    return a.ctypes.data if a.size else None


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle returned status {code}")
        self.code = code


# ---------------------------------------------------------------- GF(2^8) / AES

def gf8_mul(a: int, b: int) -> int:
    return lib().oracle_gf8_mul(a, b)


def gf8_inv(a: int) -> int:
    return lib().oracle_gf8_inv(a)


def gf8_xtime(a: int) -> int:
    return lib().oracle_gf8_xtime(a)


def sbox() -> bytes:
    out = ctypes.create_string_buffer(256)
    lib().oracle_sbox(out)
    return out.raw


def inv_sbox() -> bytes:
    out = ctypes.create_string_buffer(256)
    lib().oracle_inv_sbox(out)
    return out.raw


def key_expand(key: bytes) -> bytes:
    out = ctypes.create_string_buffer(240)
    nr = lib().oracle_key_expand(key, len(key), out)
    if nr == 0:
        raise OracleError(E_KEYLEN)
    return out.raw[: 16 * (nr + 1)]


def aes_encrypt_block(key: bytes, block: bytes) -> bytes:
    out = ctypes.create_string_buffer(16)
    rc = lib().oracle_aes_encrypt_block(key, len(key), bytes(block), out)
    if rc:
        raise OracleError(rc)
    return out.raw


def aes_decrypt_block(key: bytes, block: bytes) -> bytes:
    out = ctypes.create_string_buffer(16)
    rc = lib().oracle_aes_decrypt_block(key, len(key), bytes(block), out)
    if rc:
        raise OracleError(rc)
    return out.raw


# ---------------------------------------------------------------- GF(2^128) / GHASH

def gf128_mul(x: bytes, y: bytes) -> bytes:
    out = ctypes.create_string_buffer(16)
    lib().oracle_gf128_mul(bytes(x), bytes(y), out)
    return out.raw


GF128_ONE = bytes([0x80]) + bytes(15)


def gf128_pow(x: bytes, e: int) -> bytes:
    """x^e by square-and-multiply over the oracle's product (test helper)."""
    result = GF128_ONE
    base = bytes(x)
    while e:
        if e & 1:
            result = gf128_mul(result, base)
        base = gf128_mul(base, base)
        e >>= 1
    return result


def xor16(a: bytes, b: bytes) -> bytes:
    return bytes(p ^ q for p, q in zip(a, b))


def ghash(h: bytes, data) -> bytes:
    """Sequential Horner GHASH over whole 16-byte blocks."""
    d = _buf(data)
    assert d.size % 16 == 0
    out = ctypes.create_string_buffer(16)
    lib().oracle_ghash(bytes(h), _ptr(d), d.size // 16, out)
    return out.raw


def gcm_hash(h: bytes, aad, ct) -> bytes:
    """S = GHASH_H(A || pad || C || pad || [8|A|]_64 || [8|C|]_64)."""
    a = _buf(aad)
    c = _buf(ct)
    out = ctypes.create_string_buffer(16)
    lib().oracle_gcm_hash(bytes(h), _ptr(a), a.size, _ptr(c), c.size, out)
    return out.raw


def ghash_tree(h: bytes, blocks: Sequence[bytes], split: Callable[[int, int], int]) -> bytes:
    """GHASH re-bracketed as a reduction tree (test helper for the pins).

    node(lo, hi) = sum_{i in [lo, hi)} X_i * H^(hi-1-i); a node is split at
    ``split(lo, hi)`` and combined as node(lo, mid) * H^(hi-mid) + node(mid, hi).
    The GHASH value is node(0, m) * H.  With ``split`` halving power-of-two
    ranges this is the paper's tree: level k multiplies by H^(2^k) and a
    final multiplication by H closes it.
    """

    def node(lo: int, hi: int) -> bytes:
        if hi - lo == 1:
            return bytes(blocks[lo])
        mid = split(lo, hi)
        assert lo < mid < hi
        left = node(lo, mid)
        right = node(mid, hi)
        return xor16(gf128_mul(left, gf128_pow(h, hi - mid)), right)

    if len(blocks) == 0:
        return bytes(16)
    return gf128_mul(node(0, len(blocks)), h)


# ---------------------------------------------------------------- GCM

def gcm_encrypt(key: bytes, iv: bytes, aad, pt, out: Optional[np.ndarray] = None):
    """Returns (ciphertext as np.uint8 array, 16-byte tag)."""
    a = _buf(aad)
    p = _buf(pt)
    ct = out if out is not None else np.empty(p.size, dtype=np.uint8)
    tag = ctypes.create_string_buffer(16)
    rc = lib().oracle_gcm_encrypt(bytes(key), len(key), bytes(iv), len(iv), _ptr(a), a.size,
                                  _ptr(p), p.size, _ptr(ct), tag)
    if rc:
        raise OracleError(rc)
    return ct, tag.raw


def gcm_decrypt_verify(key: bytes, iv: bytes, aad, ct, tag: bytes, out: Optional[np.ndarray] = None):
    """Returns (plaintext or zeros as np.uint8 array, accept flag)."""
    a = _buf(aad)
    c = _buf(ct)
    pt = out if out is not None else np.empty(c.size, dtype=np.uint8)
    acc = ctypes.c_int(-1)
    rc = lib().oracle_gcm_decrypt_verify(bytes(key), len(key), bytes(iv), len(iv), _ptr(a), a.size,
                                         _ptr(c), c.size, bytes(tag), _ptr(pt), ctypes.byref(acc))
    if rc:
        raise OracleError(rc)
    return pt, bool(acc.value)


def gcm_decrypt_verify_t(key: bytes, iv: bytes, aad, ct, tag: bytes, out: Optional[np.ndarray] = None):
    """GCM-AD with a truncated tag (len(tag) bytes): (plaintext or zeros, accept)."""
    a = _buf(aad)
    c = _buf(ct)
    pt = out if out is not None else np.empty(c.size, dtype=np.uint8)
    acc = ctypes.c_int(-1)
    t = bytes(tag)
    rc = lib().oracle_gcm_decrypt_verify_t(bytes(key), len(key), bytes(iv), len(iv), _ptr(a), a.size,
                                           _ptr(c), c.size, t, len(t), _ptr(pt), ctypes.byref(acc))
    if rc:
        raise OracleError(rc)
    return pt, bool(acc.value)


def gcm_j0(key: bytes, iv: bytes) -> bytes:
    out = ctypes.create_string_buffer(16)
    rc = lib().oracle_gcm_j0(bytes(key), len(key), bytes(iv), len(iv), out)
    if rc:
        raise OracleError(rc)
    return out.raw


def gcm_status(key: bytes, iv: bytes, aad_len: int, length: int) -> int:
    """Status the oracle returns for these argument sizes (no data is touched
    when the sizes are rejected)."""
    a = np.zeros(1, np.uint8)
    tag = ctypes.create_string_buffer(16)
    # sizes beyond the limits are rejected before any pointer is read
    return lib().oracle_gcm_encrypt(bytes(key), len(key), bytes(iv), len(iv), _ptr(a), aad_len,
                                    _ptr(a), length, _ptr(a), tag)


def gctr(key: bytes, icb: bytes, data) -> np.ndarray:
    d = _buf(data)
    out = np.empty(d.size, dtype=np.uint8)
    rc = lib().oracle_gctr(bytes(key), len(key), bytes(icb), _ptr(d), d.size, _ptr(out))
    if rc:
        raise OracleError(rc)
    return out


# ---------------------------------------------------------------- AES-GCM-SIV (RFC 8452)

def polyval(h: bytes, data) -> bytes:
    """POLYVAL(H, X_1..X_s) over whole 16-byte blocks."""
    d = _buf(data)
    assert d.size % 16 == 0
    out = ctypes.create_string_buffer(16)
    lib().oracle_polyval(bytes(h), _ptr(d), d.size // 16, out)
    return out.raw


def pv_mul(a: bytes, b: bytes) -> bytes:
    """a * b mod x^128 + x^127 + x^126 + x^121 + 1 (POLYVAL's field, no x^-128)."""
    out = ctypes.create_string_buffer(16)
    lib().oracle_pv_mul(bytes(a), bytes(b), out)
    return out.raw


def gcm_siv_derive(kgk: bytes, nonce: bytes):
    """(message authentication key, message encryption key) for this nonce."""
    auth = ctypes.create_string_buffer(16)
    enc = ctypes.create_string_buffer(32)
    rc = lib().oracle_gcm_siv_derive(bytes(kgk), len(kgk), bytes(nonce), auth, enc)
    if rc:
        raise OracleError(rc)
    return auth.raw, enc.raw[:len(kgk)]


def gcm_siv_encrypt(kgk: bytes, nonce: bytes, aad, pt, out: Optional[np.ndarray] = None):
    """Returns (ciphertext as np.uint8 array, 16-byte tag)."""
    a = _buf(aad)
    p = _buf(pt)
    ct = out if out is not None else np.empty(p.size, dtype=np.uint8)
    tag = ctypes.create_string_buffer(16)
    rc = lib().oracle_gcm_siv_encrypt(bytes(kgk), len(kgk), bytes(nonce), len(nonce), _ptr(a), a.size,
                                      _ptr(p), p.size, _ptr(ct), tag)
    if rc:
        raise OracleError(rc)
    return ct, tag.raw


def gcm_siv_decrypt_verify(kgk: bytes, nonce: bytes, aad, ct, tag: bytes, out: Optional[np.ndarray] = None):
    """Returns (plaintext or zeros as np.uint8 array, accept flag)."""
    a = _buf(aad)
    c = _buf(ct)
    pt = out if out is not None else np.empty(c.size, dtype=np.uint8)
    acc = ctypes.c_int(-1)
    rc = lib().oracle_gcm_siv_decrypt_verify(bytes(kgk), len(kgk), bytes(nonce), len(nonce), _ptr(a), a.size,
                                             _ptr(c), c.size, bytes(tag), _ptr(pt), ctypes.byref(acc))
    if rc:
        raise OracleError(rc)
    return pt, bool(acc.value)
