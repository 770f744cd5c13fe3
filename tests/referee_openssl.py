"""Second referee: OpenSSL's EVP AES-ECB / AES-GCM through its public C API.

Used by the CPU pins to check the oracle's conventions (byte order, bit order
of GF(2^128), counter increment, length block) against an independent, widely
deployed implementation.  Only the documented EVP entry points are called.
"""
from __future__ import annotations

import ctypes
import ctypes.util
from typing import Optional

import numpy as np

_EVP_CTRL_GCM_SET_IVLEN = 0x9
_EVP_CTRL_GCM_GET_TAG = 0x10
_EVP_CTRL_GCM_SET_TAG = 0x11

_lib: Optional[ctypes.CDLL] = None


def available() -> bool:
    try:
        _load()
        return True
    except OSError:
        return False


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        name = ctypes.util.find_library("crypto") or "libcrypto.so.3"
        L = ctypes.CDLL(name)
        vp = ctypes.c_void_p
        ip = ctypes.POINTER(ctypes.c_int)
        L.EVP_CIPHER_CTX_new.restype = vp
        L.EVP_CIPHER_CTX_free.argtypes = [vp]
        for fn in ("EVP_aes_128_gcm", "EVP_aes_192_gcm", "EVP_aes_256_gcm",
                   "EVP_aes_128_ecb", "EVP_aes_192_ecb", "EVP_aes_256_ecb"):
            getattr(L, fn).restype = vp
        L.EVP_EncryptInit_ex.argtypes = [vp, vp, vp, ctypes.c_char_p, ctypes.c_char_p]
        L.EVP_DecryptInit_ex.argtypes = [vp, vp, vp, ctypes.c_char_p, ctypes.c_char_p]
        L.EVP_EncryptUpdate.argtypes = [vp, vp, ip, vp, ctypes.c_int]
        L.EVP_DecryptUpdate.argtypes = [vp, vp, ip, vp, ctypes.c_int]
        L.EVP_EncryptFinal_ex.argtypes = [vp, vp, ip]
        L.EVP_DecryptFinal_ex.argtypes = [vp, vp, ip]
        L.EVP_CIPHER_CTX_ctrl.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
        L.EVP_CIPHER_CTX_set_padding.argtypes = [vp, ctypes.c_int]
        _lib = L
    return _lib


def _cipher(mode: str, key_len: int):
    L = _load()
    bits = {16: 128, 24: 192, 32: 256}[key_len]
    return getattr(L, f"EVP_aes_{bits}_{mode}")()


def aes_ecb_encrypt(key: bytes, block: bytes) -> bytes:
    L = _load()
    ctx = L.EVP_CIPHER_CTX_new()
    try:
        assert L.EVP_EncryptInit_ex(ctx, _cipher("ecb", len(key)), None, key, None) == 1
        L.EVP_CIPHER_CTX_set_padding(ctx, 0)
        out = ctypes.create_string_buffer(32)
        n = ctypes.c_int(0)
        assert L.EVP_EncryptUpdate(ctx, out, ctypes.byref(n), block, 16) == 1
        return out.raw[:16]
    finally:
        L.EVP_CIPHER_CTX_free(ctx)


def _chunks(data: bytes, step: int = 1 << 30):
    for off in range(0, len(data), step):
        yield off, data[off:off + step]


def gcm_encrypt(key: bytes, iv: bytes, aad: bytes, pt: bytes):
    L = _load()
    ctx = L.EVP_CIPHER_CTX_new()
    try:
        assert L.EVP_EncryptInit_ex(ctx, _cipher("gcm", len(key)), None, None, None) == 1
        assert L.EVP_CIPHER_CTX_ctrl(ctx, _EVP_CTRL_GCM_SET_IVLEN, len(iv), None) == 1
        assert L.EVP_EncryptInit_ex(ctx, None, None, key, iv) == 1
        n = ctypes.c_int(0)
        if aad:
            assert L.EVP_EncryptUpdate(ctx, None, ctypes.byref(n), aad, len(aad)) == 1
        out = ctypes.create_string_buffer(len(pt) + 16)
        for off, chunk in _chunks(pt):
            assert L.EVP_EncryptUpdate(ctx, ctypes.byref(out, off), ctypes.byref(n), chunk, len(chunk)) == 1
        assert L.EVP_EncryptFinal_ex(ctx, None, ctypes.byref(n)) == 1
        tag = ctypes.create_string_buffer(16)
        assert L.EVP_CIPHER_CTX_ctrl(ctx, _EVP_CTRL_GCM_GET_TAG, 16, tag) == 1
        return out.raw[: len(pt)], tag.raw
    finally:
        L.EVP_CIPHER_CTX_free(ctx)


def gcm_decrypt(key: bytes, iv: bytes, aad: bytes, ct: bytes, tag: bytes):
    """Returns (plaintext, accepted); a tag shorter than 16 bytes is checked
    as a truncated tag of that length."""
    L = _load()
    ctx = L.EVP_CIPHER_CTX_new()
    try:
        assert L.EVP_DecryptInit_ex(ctx, _cipher("gcm", len(key)), None, None, None) == 1
        assert L.EVP_CIPHER_CTX_ctrl(ctx, _EVP_CTRL_GCM_SET_IVLEN, len(iv), None) == 1
        assert L.EVP_DecryptInit_ex(ctx, None, None, key, iv) == 1
        n = ctypes.c_int(0)
        if aad:
            assert L.EVP_DecryptUpdate(ctx, None, ctypes.byref(n), aad, len(aad)) == 1
        out = ctypes.create_string_buffer(len(ct) + 16)
        for off, chunk in _chunks(ct):
            assert L.EVP_DecryptUpdate(ctx, ctypes.byref(out, off), ctypes.byref(n), chunk, len(chunk)) == 1
        tbuf = ctypes.create_string_buffer(bytes(tag), len(tag))
        assert L.EVP_CIPHER_CTX_ctrl(ctx, _EVP_CTRL_GCM_SET_TAG, len(tag), tbuf) == 1
        ok = L.EVP_DecryptFinal_ex(ctx, None, ctypes.byref(n)) == 1
        return out.raw[: len(ct)], ok
    finally:
        L.EVP_CIPHER_CTX_free(ctx)


def gcm_encrypt_np(key: bytes, iv: bytes, aad: bytes, pt: np.ndarray):
    """AES-GCM of a large contiguous uint8 array without Python-level copies:
    returns (ciphertext array, 16-byte tag)."""
    L = _load()
    pt = np.ascontiguousarray(pt, dtype=np.uint8).reshape(-1)
    out = np.empty_like(pt)
    ctx = L.EVP_CIPHER_CTX_new()
    try:
        assert L.EVP_EncryptInit_ex(ctx, _cipher("gcm", len(key)), None, None, None) == 1
        assert L.EVP_CIPHER_CTX_ctrl(ctx, _EVP_CTRL_GCM_SET_IVLEN, len(iv), None) == 1
        assert L.EVP_EncryptInit_ex(ctx, None, None, key, iv) == 1
        n = ctypes.c_int(0)
        if aad:
            assert L.EVP_EncryptUpdate(ctx, None, ctypes.byref(n), aad, len(aad)) == 1
        step = 1 << 28
        for off in range(0, pt.size, step):
            m = min(step, pt.size - off)
            assert L.EVP_EncryptUpdate(ctx, ctypes.c_void_p(out.ctypes.data + off), ctypes.byref(n),
                                       ctypes.c_void_p(pt.ctypes.data + off), m) == 1
        assert L.EVP_EncryptFinal_ex(ctx, None, ctypes.byref(n)) == 1
        tag = ctypes.create_string_buffer(16)
        assert L.EVP_CIPHER_CTX_ctrl(ctx, _EVP_CTRL_GCM_GET_TAG, 16, tag) == 1
        return out, tag.raw
    finally:
        L.EVP_CIPHER_CTX_free(ctx)
