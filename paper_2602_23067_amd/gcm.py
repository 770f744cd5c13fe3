"""Thin ctypes binding over ``libgcm_mi355.so`` (argument marshalling only).

Every step of AES-GCM runs in the library's HIP kernels; this module only
turns torch tensors into device pointers and HIP stream handles and checks
return codes.  It raises ``ImportError`` when the library has not been
built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgcm_mi355.so")

GCM_OK = 0
GCM_E_ARG = -1
GCM_E_KEYLEN = -2
GCM_E_IVLEN = -3
GCM_E_TOOLONG = -4
GCM_E_NOMEM = -5
GCM_E_HIP = -6
GCM_E_BUSY = -7
GCM_E_ALIAS = -8
GCM_E_SLOT = -9
GCM_E_INTERNAL = -10

# bytes of the fixed device scratch behind encrypt_async_noalloc (GCM_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = (1 << 20) + 4096

_lib: Optional[ctypes.CDLL] = None


class Request(ctypes.Structure):
    """Mirror of ``gcm_request``."""

    _fields_ = [
        ("op", ctypes.c_uint32),
        ("key_slot", ctypes.c_uint32),
        ("iv", ctypes.c_uint8 * 12),
        ("reserved", ctypes.c_uint32),
        ("aad_d", ctypes.c_void_p),
        ("aad_len", ctypes.c_uint64),
        ("in_d", ctypes.c_void_p),
        ("out_d", ctypes.c_void_p),
        ("len", ctypes.c_uint64),
        ("tag_d", ctypes.c_void_p),
    ]


class ServeConfig(ctypes.Structure):
    _fields_ = [
        ("n_streams", ctypes.c_uint32),
        ("max_batch_reqs", ctypes.c_uint32),
        ("hbm_budget", ctypes.c_uint64),
        ("max_batch_bytes", ctypes.c_uint64),
        ("max_queue", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class ServeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "rejected", "batches", "bytes_completed",
                                               "budget_high_water", "overlapped_admissions",
                                               "max_inflight_batches", "failed")] + \
               [(n, ctypes.c_double) for n in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "wall_s")]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [("log2_tile_blocks", ctypes.c_uint32), ("waves_per_group", ctypes.c_uint32),
                ("candidates", ctypes.c_uint32), ("best_ms", ctypes.c_float), ("gbs", ctypes.c_double),
                ("groups_per_cu", ctypes.c_uint32), ("combine_fanin", ctypes.c_uint32)]


class Job(ctypes.Structure):
    """Mirror of ``gcm_job`` (include/gcm_mi355.h)."""

    _fields_ = [
        ("op", ctypes.c_uint32),
        ("key_slot", ctypes.c_uint32),
        ("iv", ctypes.c_uint8 * 12),
        ("reserved", ctypes.c_uint32),
        ("aad_off", ctypes.c_uint64),
        ("aad_len", ctypes.c_uint64),
        ("in_off", ctypes.c_uint64),
        ("out_off", ctypes.c_uint64),
        ("len", ctypes.c_uint64),
        ("tag_off", ctypes.c_uint64),
        ("ok_off", ctypes.c_uint64),
    ]


class FitsResult(ctypes.Structure):
    """Mirror of ``gcm_fits_result``."""

    _fields_ = [("data", ctypes.c_void_p), ("size", ctypes.c_uint64), ("error_code", ctypes.c_int32),
                ("warning_code", ctypes.c_int32)]


class GcmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2602_23067_amd.build.build() "
                          "(there is no non-GPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, u64, u32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_uint32
    i32p = ctypes.POINTER(ctypes.c_int)
    sig = {
        "gcm_ctx_create": ([ctypes.POINTER(vp), ctypes.c_int, u64, u32], ctypes.c_int),
        "gcm_ctx_destroy": ([vp], ctypes.c_int),
        "gcm_last_error": ([], ctypes.c_char_p),
        "gcm_key_register": ([vp, vp, sz, ctypes.POINTER(u32), vp], ctypes.c_int),
        "gcm_key_release": ([vp, u32], ctypes.c_int),
        "gcm_encrypt": ([vp, vp, sz, vp, sz, vp, u64, vp, u64, vp, vp, vp], ctypes.c_int),
        "gcm_decrypt_verify": ([vp, vp, sz, vp, sz, vp, u64, vp, u64, vp, vp, i32p, vp], ctypes.c_int),
        "gcm_workspace_size": ([vp, u64, u64], u64),
        "gcm_encrypt_async": ([vp, u32, vp, sz, vp, u64, vp, u64, vp, vp, vp, u64, vp], ctypes.c_int),
        "gcm_decrypt_verify_async": ([vp, u32, vp, sz, vp, u64, vp, u64, vp, vp, vp, vp, u64, vp], ctypes.c_int),
        "gcm_encrypt_async_noalloc": ([vp, u32, vp, sz, vp, u64, vp, u64, vp, vp, vp], ctypes.c_int),
        "gcm_set_launch": ([vp, u32, u32, u32], ctypes.c_int),
        "gcm_key_register_many": ([vp, vp, vp, u32, vp, vp], ctypes.c_int),
        "gcm_batch_create": ([vp, vp, u32, vp, u64, ctypes.POINTER(vp)], ctypes.c_int),
        "gcm_batch_launch": ([vp, vp], ctypes.c_int),
        "gcm_batch_graph_launch": ([vp, vp], ctypes.c_int),
        "gcm_batch_info": ([vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u32)], ctypes.c_int),
        "gcm_batch_destroy": ([vp], ctypes.c_int),
        "gcm_batch_run": ([vp, vp, u32, vp, u64, vp], ctypes.c_int),
        "gcm_serve_start": ([vp, vp, ctypes.POINTER(vp)], ctypes.c_int),
        "gcm_serve_submit": ([vp, vp, ctypes.POINTER(u64)], ctypes.c_int),
        "gcm_serve_poll": ([vp, u64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                            ctypes.POINTER(u64)], ctypes.c_int),
        "gcm_serve_wait": ([vp, u64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(u64)], ctypes.c_int),
        "gcm_serve_drain": ([vp], ctypes.c_int),
        "gcm_serve_get_stats": ([vp, vp], ctypes.c_int),
        "gcm_serve_stop": ([vp], ctypes.c_int),
        "gcm_autotune": ([vp, u32, u64, u32, vp, vp], ctypes.c_int),
        "gcm_batch_autotune": ([vp, vp, u32, vp, u64, u32, vp, vp], ctypes.c_int),
        "gcm_set_combine": ([vp, u32], ctypes.c_int),
        "gcm_launch_plan": ([vp, u32, u64, u64, ctypes.POINTER(TuneResult)], ctypes.c_int),
        "gcm_autotune_save": ([vp, ctypes.c_char_p], ctypes.c_int),
        "gcm_autotune_load": ([vp, ctypes.c_char_p], ctypes.c_int),
        "gcm_profile_enable": ([vp, ctypes.c_int], ctypes.c_int),
        "gcm_profile_read": ([vp, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "gcm_ctr_xcrypt": ([vp, vp, sz, vp, sz, vp, u64, vp, vp], ctypes.c_int),
        "gcm_ctr_async": ([vp, u32, vp, sz, vp, u64, vp, vp], ctypes.c_int),
        "gcm_gmac": ([vp, vp, sz, vp, sz, vp, u64, vp, vp], ctypes.c_int),
        "gcm_encrypt_host": ([vp, vp, sz, vp, sz, vp, u64, vp, u64, vp, vp], ctypes.c_int),
        "gcm_decrypt_verify_host": ([vp, vp, sz, vp, sz, vp, u64, vp, u64, vp, vp, i32p], ctypes.c_int),
        "gcm_set_pipeline": ([vp, u64], ctypes.c_int),
        "gcm_encrypt_ex": ([vp, vp, sz, vp, sz, vp, u64, vp, u64, vp, vp, sz, vp], ctypes.c_int),
        "gcm_stream_begin": ([vp, u32, u32, vp, sz, vp, u64, ctypes.POINTER(vp), vp], ctypes.c_int),
        "gcm_fits_encrypt": ([vp, vp, u64, vp, sz, vp, sz, vp, vp, ctypes.POINTER(FitsResult)], ctypes.c_int),
        "gcm_fits_decrypt": ([vp, vp, u64, vp, sz, vp, sz, ctypes.POINTER(FitsResult)], ctypes.c_int),
        "gcm_fits_free": ([ctypes.POINTER(FitsResult)], None),
        "gcm_fits_nonce": ([vp], ctypes.c_int),
        "gcm_stream_update": ([vp, vp, u64, vp, vp], ctypes.c_int),
        "gcm_stream_final": ([vp, vp, vp, vp], ctypes.c_int),
        "gcm_stream_destroy": ([vp], ctypes.c_int),
        "gcm_decrypt_verify_ex": ([vp, vp, sz, vp, sz, vp, u64, vp, u64, vp, sz, vp, i32p, vp], ctypes.c_int),
        "gcm_siv_workspace_size": ([vp, u64, u64], u64),
        "gcm_siv_encrypt_async": ([vp, u32, vp, sz, vp, u64, vp, u64, vp, vp, vp, u64, vp], ctypes.c_int),
        "gcm_siv_decrypt_verify_async": ([vp, u32, vp, sz, vp, u64, vp, u64, vp, vp, vp, vp, u64, vp],
                                         ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(rc: int) -> int:
    if rc != GCM_OK:
        raise GcmError(rc, load().gcm_last_error().decode(errors="replace"))
    return rc


def _dev(t) -> int:
    """Device address of a contiguous uint8 CUDA tensor (0 for None/empty)."""
    if t is None:
        return 0
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if not t.is_cuda:
        raise ValueError("payload tensors must live on the GPU")
    if t.dtype != torch.uint8:
        raise TypeError("payload tensors must be uint8")
    if not t.is_contiguous():
        raise ValueError("payload tensors must be contiguous")
    return t.data_ptr() if t.numel() else 0


def _stream(stream) -> int:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _host(b: bytes) -> ctypes.Array:
    return ctypes.create_string_buffer(bytes(b), len(b))


def _hostbuf(t):
    """(address, bytes) of a contiguous host uint8 buffer: a CPU torch tensor
    (pinned or not) or a numpy array; (0, 0) for None/empty."""
    if t is None:
        return 0, 0
    try:
        import torch

        if isinstance(t, torch.Tensor):
            if t.is_cuda:
                raise ValueError("host-pipeline buffers must be in host memory")
            if t.dtype != torch.uint8 or not t.is_contiguous():
                raise TypeError("host buffers must be contiguous uint8")
            return (t.data_ptr() if t.numel() else 0), t.numel()
    except ImportError:
        pass
    import numpy as np

    if isinstance(t, np.ndarray):
        if t.dtype != np.uint8 or not t.flags["C_CONTIGUOUS"]:
            raise TypeError("host buffers must be contiguous uint8")
        return (t.ctypes.data if t.size else 0), t.size
    raise TypeError("expected a CPU torch.Tensor or a numpy array")


class Context:
    """An AES-GCM context on one GPU (key table, scratch, tuning)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, key_slots: int = 64):
        L = load()
        h = ctypes.c_void_p()
        _check(L.gcm_ctx_create(ctypes.byref(h), device, hbm_budget, key_slots))
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            load().gcm_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    # -------------------------------------------------------- keys
    def key_register(self, key: bytes, stream=None) -> int:
        slot = ctypes.c_uint32()
        _check(load().gcm_key_register(self._h, _host(key), len(key), ctypes.byref(slot), _stream(stream)))
        return slot.value

    def key_register_many(self, keys, stream=None):
        """Register a list of keys in as few launches as possible; returns slots."""
        import numpy as np

        lens = np.asarray([len(k) for k in keys], dtype=np.uint32)
        blob = b"".join(bytes(k) for k in keys)
        slots = np.zeros(len(keys), dtype=np.uint32)
        _check(load().gcm_key_register_many(self._h, _host(blob) if blob else None, lens.ctypes.data,
                                            len(keys), slots.ctypes.data, _stream(stream)))
        return [int(x) for x in slots]

    def key_release(self, slot: int) -> None:
        _check(load().gcm_key_release(self._h, slot))

    # -------------------------------------------------------- one-shot
    def encrypt(self, key: bytes, iv: bytes, aad, pt, ct, stream=None) -> bytes:
        tag = ctypes.create_string_buffer(16)
        _check(load().gcm_encrypt(self._h, _host(key), len(key), _host(iv), len(iv), _dev(aad),
                                  0 if aad is None else aad.numel(), _dev(pt), pt.numel(), _dev(ct), tag,
                                  _stream(stream)))
        return tag.raw

    def decrypt_verify(self, key: bytes, iv: bytes, aad, ct, tag: bytes, pt, stream=None) -> bool:
        acc = ctypes.c_int(-1)
        _check(load().gcm_decrypt_verify(self._h, _host(key), len(key), _host(iv), len(iv), _dev(aad),
                                         0 if aad is None else aad.numel(), _dev(ct), ct.numel(), _host(tag),
                                         _dev(pt), ctypes.byref(acc), _stream(stream)))
        return acc.value == 1

    def encrypt_ex(self, key: bytes, iv: bytes, aad, pt, ct, tag_len: int = 16, stream=None) -> bytes:
        """gcm_encrypt with a truncated tag (16, 15, 14, 13, 12, 8 or 4 bytes)."""
        tag = ctypes.create_string_buffer(16)
        _check(load().gcm_encrypt_ex(self._h, _host(key), len(key), _host(iv), len(iv), _dev(aad),
                                     0 if aad is None else aad.numel(), _dev(pt), 0 if pt is None else pt.numel(),
                                     _dev(ct), tag, tag_len, _stream(stream)))
        return tag.raw[:tag_len]

    def decrypt_verify_ex(self, key: bytes, iv: bytes, aad, ct, tag: bytes, pt, stream=None) -> bool:
        """gcm_decrypt_verify against a truncated tag of len(tag) bytes."""
        acc = ctypes.c_int(-1)
        _check(load().gcm_decrypt_verify_ex(self._h, _host(key), len(key), _host(iv), len(iv), _dev(aad),
                                            0 if aad is None else aad.numel(), _dev(ct),
                                            0 if ct is None else ct.numel(), _host(tag) if tag else None,
                                            len(tag), _dev(pt), ctypes.byref(acc), _stream(stream)))
        return acc.value == 1

    # -------------------------------------------------------- authenticated FITS container
    def fits_encrypt(self, fits_bytes: bytes, key_h: bytes, key_d: bytes, nonce_h: bytes = None,
                     nonce_d: bytes = None) -> bytes:
        """The paper's two-HDU container for a 2-D FITS image (nonces drawn
        from the entropy pool when not given)."""
        nonce_h = nonce_h if nonce_h is not None else fits_nonce()
        nonce_d = nonce_d if nonce_d is not None else fits_nonce()
        r = FitsResult()
        src = fits_bytes if isinstance(fits_bytes, bytes) else bytes(fits_bytes)  # passed without a copy
        try:
            _check(load().gcm_fits_encrypt(self._h, src, len(src), _host(key_h), len(key_h), _host(key_d),
                                           len(key_d), _host(nonce_h), _host(nonce_d), ctypes.byref(r)))
            return ctypes.string_at(r.data, r.size)
        finally:
            load().gcm_fits_free(ctypes.byref(r))

    def fits_decrypt(self, container: bytes, key_h: bytes = None, key_d: bytes = None):
        """(FITS bytes, warning_code): 0 full, 1 header fallback, 2 payload suppressed, 3 both."""
        r = FitsResult()
        src = container if isinstance(container, bytes) else bytes(container)  # passed without a copy
        try:
            _check(load().gcm_fits_decrypt(self._h, src, len(src), _host(key_h) if key_h else None,
                                           len(key_h) if key_h else 0, _host(key_d) if key_d else None,
                                           len(key_d) if key_d else 0, ctypes.byref(r)))
            return ctypes.string_at(r.data, r.size), r.warning_code
        finally:
            load().gcm_fits_free(ctypes.byref(r))

    # -------------------------------------------------------- streamed messages
    def stream_begin(self, op: int, slot: int, iv: bytes, aad=None, stream=None) -> "GcmStream":
        h = ctypes.c_void_p()
        _check(load().gcm_stream_begin(self._h, op, slot, _host(iv), len(iv), _dev(aad),
                                       0 if aad is None else aad.numel(), ctypes.byref(h), _stream(stream)))
        return GcmStream(h)

    # -------------------------------------------------------- counter mode only, GMAC
    def ctr_xcrypt(self, key: bytes, iv: bytes, src, dst, stream=None) -> None:
        """AES-CTR with GCM's counters (no tag); encrypts and decrypts."""
        _check(load().gcm_ctr_xcrypt(self._h, _host(key), len(key), _host(iv), len(iv), _dev(src), src.numel(),
                                     _dev(dst), _stream(stream)))

    def ctr_async(self, slot: int, iv: bytes, src, dst, stream=None) -> None:
        _check(load().gcm_ctr_async(self._h, slot, _host(iv), len(iv), _dev(src), src.numel(), _dev(dst),
                                    _stream(stream)))

    def gmac(self, key: bytes, iv: bytes, aad, stream=None) -> bytes:
        """GMAC tag over the device buffer `aad` (GCM with an empty plaintext)."""
        tag = ctypes.create_string_buffer(16)
        _check(load().gcm_gmac(self._h, _host(key), len(key), _host(iv), len(iv), _dev(aad),
                               0 if aad is None else aad.numel(), tag, _stream(stream)))
        return tag.raw

    # -------------------------------------------------------- host-to-host pipeline
    def set_pipeline(self, chunk_bytes: int = 0) -> None:
        _check(load().gcm_set_pipeline(self._h, chunk_bytes))

    def encrypt_host(self, key: bytes, iv: bytes, aad, pt, ct) -> bytes:
        """GCM-AE on host buffers (CPU tensors, ideally pinned, or numpy arrays)."""
        a, alen = _hostbuf(aad)
        p, plen = _hostbuf(pt)
        c, clen = _hostbuf(ct)
        if clen != plen:
            raise ValueError("pt and ct must have the same length")
        tag = ctypes.create_string_buffer(16)
        _check(load().gcm_encrypt_host(self._h, _host(key), len(key), _host(iv), len(iv), a, alen, p, plen, c, tag))
        return tag.raw

    def decrypt_verify_host(self, key: bytes, iv: bytes, aad, ct, tag: bytes, pt) -> bool:
        a, alen = _hostbuf(aad)
        c, clen = _hostbuf(ct)
        p, plen = _hostbuf(pt)
        if clen != plen:
            raise ValueError("ct and pt must have the same length")
        acc = ctypes.c_int(-1)
        _check(load().gcm_decrypt_verify_host(self._h, _host(key), len(key), _host(iv), len(iv), a, alen, c, clen,
                                              _host(tag), p, ctypes.byref(acc)))
        return acc.value == 1

    # -------------------------------------------------------- async, resident key
    def workspace_size(self, length: int, aad_len: int) -> int:
        return int(load().gcm_workspace_size(self._h, length, aad_len))

    def encrypt_async(self, slot: int, iv: bytes, aad, pt, ct, tag_d, workspace, stream=None) -> None:
        _check(load().gcm_encrypt_async(self._h, slot, _host(iv), len(iv), _dev(aad),
                                        0 if aad is None else aad.numel(), _dev(pt),
                                        0 if pt is None else pt.numel(), _dev(ct), _dev(tag_d), _dev(workspace),
                                        workspace.numel(), _stream(stream)))

    def encrypt_async_noalloc(self, slot: int, iv: bytes, aad, pt, ct, tag_d, stream=None) -> None:
        """encrypt_async with the library's fixed device scratch instead of a workspace."""
        _check(load().gcm_encrypt_async_noalloc(self._h, slot, _host(iv), len(iv), _dev(aad),
                                                0 if aad is None else aad.numel(), _dev(pt),
                                                0 if pt is None else pt.numel(), _dev(ct), _dev(tag_d),
                                                _stream(stream)))

    def decrypt_verify_async(self, slot: int, iv: bytes, aad, ct, tag_d, pt, accept_d, workspace,
                             stream=None) -> None:
        _check(load().gcm_decrypt_verify_async(self._h, slot, _host(iv), len(iv), _dev(aad),
                                               0 if aad is None else aad.numel(), _dev(ct), ct.numel(),
                                               _dev(tag_d), _dev(pt), accept_d.data_ptr(), _dev(workspace),
                                               workspace.numel(), _stream(stream)))

    # -------------------------------------------------------- AES-GCM-SIV (RFC 8452)
    def siv_workspace_size(self, length: int, aad_len: int) -> int:
        return int(load().gcm_siv_workspace_size(self._h, length, aad_len))

    def _siv_ws(self, length: int, aad_len: int, workspace):
        if workspace is not None:
            return workspace
        import torch
        n = self.siv_workspace_size(length, aad_len)
        return torch.empty(n, dtype=torch.uint8, device=f"cuda:{self.device}")

    def siv_encrypt_async(self, slot: int, nonce: bytes, aad, pt, ct, tag_d, workspace=None, stream=None):
        """Enqueue GCM-SIV encryption of device tensors; returns the workspace
        used (keep it alive until the stream has passed the call)."""
        n = 0 if pt is None else pt.numel()
        na = 0 if aad is None else aad.numel()
        ws = self._siv_ws(n, na, workspace)
        _check(load().gcm_siv_encrypt_async(self._h, slot, _host(nonce), len(nonce), _dev(aad), na, _dev(pt), n,
                                            _dev(ct), _dev(tag_d), _dev(ws), ws.numel(), _stream(stream)))
        return ws

    def siv_decrypt_verify_async(self, slot: int, nonce: bytes, aad, ct, tag_d, pt, accept_d, workspace=None,
                                 stream=None):
        n = 0 if ct is None else ct.numel()
        na = 0 if aad is None else aad.numel()
        ws = self._siv_ws(n, na, workspace)
        _check(load().gcm_siv_decrypt_verify_async(self._h, slot, _host(nonce), len(nonce), _dev(aad), na,
                                                   _dev(ct), n, _dev(tag_d), _dev(pt), accept_d.data_ptr(),
                                                   _dev(ws), ws.numel(), _stream(stream)))
        return ws

    # -------------------------------------------------------- measurement
    def profile_enable(self, on: bool = True) -> None:
        _check(load().gcm_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """(tile-kernel launches, summed tile-kernel milliseconds) since the last read."""
        n = ctypes.c_uint64()
        ms = ctypes.c_double()
        _check(load().gcm_profile_read(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    # -------------------------------------------------------- tuning
    def autotune(self, key_len: int, length: int, reps: int = 3, stream=None) -> dict:
        r = TuneResult()
        _check(load().gcm_autotune(self._h, key_len, length, reps, ctypes.byref(r), _stream(stream)))
        return _tune_dict(r)

    def autotune_save(self, path: str) -> None:
        _check(load().gcm_autotune_save(self._h, path.encode()))

    def autotune_load(self, path: str) -> None:
        _check(load().gcm_autotune_load(self._h, path.encode()))

    def set_launch(self, log2_tile_blocks: int = 0, waves_per_group: int = 0, groups_per_cu: int = 0) -> None:
        _check(load().gcm_set_launch(self._h, log2_tile_blocks, waves_per_group, groups_per_cu))

    def set_combine(self, fanin: int = 0) -> None:
        _check(load().gcm_set_combine(self._h, fanin))

    def launch_plan(self, key_len: int, length: int, aad_len: int = 0) -> dict:
        """The launch an asynchronous call would use for such a message (see
        gcm_launch_plan): log2_tile_blocks, waves_per_group, groups_per_cu,
        combine_fanin and `tiles`."""
        r = TuneResult()
        _check(load().gcm_launch_plan(self._h, key_len, length, aad_len, ctypes.byref(r)))
        return {"log2_tile_blocks": r.log2_tile_blocks, "waves_per_group": r.waves_per_group,
                "groups_per_cu": r.groups_per_cu, "combine_fanin": r.combine_fanin, "tiles": r.candidates}

    def batch_autotune(self, jobs, base, reps: int = 3, stream=None) -> dict:
        """Launch-shape search on a batch (see gcm_batch_autotune); `jobs` and
        `base` as for Batch."""
        r = TuneResult()
        _check(load().gcm_batch_autotune(self._h, ctypes.cast(jobs, ctypes.c_void_p), len(jobs), _dev(base),
                                         base.numel(), reps, ctypes.byref(r), _stream(stream)))
        return _tune_dict(r)


def _tune_dict(r: TuneResult) -> dict:
    return {"log2_tile_blocks": r.log2_tile_blocks, "waves_per_group": r.waves_per_group,
            "candidates": r.candidates, "best_ms": r.best_ms, "gbs": r.gbs, "groups_per_cu": r.groups_per_cu,
            "combine_fanin": r.combine_fanin}


def fits_nonce() -> bytes:
    """12 bytes from the kernel's entropy pool."""
    b = ctypes.create_string_buffer(12)
    _check(load().gcm_fits_nonce(b))
    return b.raw


class GcmStream:
    """A message fed in segments (see gcm_stream_* in the C header)."""

    def __init__(self, h):
        self._h = h

    def update(self, src, dst, stream=None) -> None:
        _check(load().gcm_stream_update(self._h, _dev(src), src.numel(), _dev(dst), _stream(stream)))

    def final(self, tag_d, accept_d=None, stream=None) -> None:
        _check(load().gcm_stream_final(self._h, _dev(tag_d), None if accept_d is None else accept_d.data_ptr(),
                                       _stream(stream)))

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().gcm_stream_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ batches

def align_up(x: int, a: int = 256) -> int:
    return (x + a - 1) // a * a


class BatchLayout:
    """Byte offsets of a packed batch inside one device buffer.

    Each message gets its AAD, input and output (or input only when in
    place) at 256-byte aligned offsets; the 16-byte tags and 4-byte accept
    flags sit in two arrays after the payloads.  Only offsets are computed
    here; callers fill the buffer."""

    def __init__(self, lengths, aad_lens, in_place: bool = False):
        self.n = len(lengths)
        self.aad_off, self.in_off, self.out_off = [], [], []
        off = 0
        for ln, al in zip(lengths, aad_lens):
            self.aad_off.append(off)
            off = align_up(off + int(al))
            self.in_off.append(off)
            off = align_up(off + int(ln))
            if in_place:
                self.out_off.append(self.in_off[-1])
            else:
                self.out_off.append(off)
                off = align_up(off + int(ln))
        self.tag_base = off
        off = align_up(off + 16 * self.n)
        self.ok_base = off
        off = align_up(off + 4 * self.n)
        self.total = max(off, 256)
        self.lengths = [int(x) for x in lengths]
        self.aad_lens = [int(x) for x in aad_lens]

    def jobs(self, ops, slots, ivs):
        arr = (Job * self.n)()
        for i in range(self.n):
            j = arr[i]
            j.op = int(ops[i])
            j.key_slot = int(slots[i])
            j.iv[:] = list(bytes(ivs[i]))
            j.reserved = 0
            j.aad_off = self.aad_off[i]
            j.aad_len = self.aad_lens[i]
            j.in_off = self.in_off[i]
            j.out_off = self.out_off[i]
            j.len = self.lengths[i]
            j.tag_off = self.tag_base + 16 * i
            j.ok_off = self.ok_base + 4 * i
        return arr


class Batch:
    """A planned batch bound to one device buffer (see gcm_batch_create)."""

    def __init__(self, ctx: Context, jobs, base):
        self._ctx = ctx
        self._base = base  # keep the buffer alive
        h = ctypes.c_void_p()
        _check(load().gcm_batch_create(ctx.handle, ctypes.cast(jobs, ctypes.c_void_p), len(jobs), _dev(base),
                                       base.numel(), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None) -> None:
        _check(load().gcm_batch_launch(self._h, _stream(stream)))

    def graph_launch(self, stream=None) -> None:
        _check(load().gcm_batch_graph_launch(self._h, _stream(stream)))

    def info(self):
        pb, tt, wi = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32()
        _check(load().gcm_batch_info(self._h, ctypes.byref(pb), ctypes.byref(tt), ctypes.byref(wi)))
        return {"payload_bytes": pb.value, "total_tiles": tt.value, "work_items": wi.value}

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().gcm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving

class Server:
    """Continuous-batching serving loop over a context's resident keys."""

    def __init__(self, ctx: Context, n_streams: int = 4, hbm_budget: int = 64 << 30, max_batch_reqs: int = 256,
                 max_batch_bytes: int = 256 << 20, max_queue: int = 1 << 16):
        self._ctx = ctx
        cfg = ServeConfig(n_streams, max_batch_reqs, hbm_budget, max_batch_bytes, max_queue, 0)
        h = ctypes.c_void_p()
        _check(load().gcm_serve_start(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, op: int, slot: int, iv: bytes, aad, inp, out, tag_d) -> int:
        r = self.prepare(op, slot, iv, aad, inp, out, tag_d)
        rid = self.submit_prepared(r)
        self._keep[rid] = (aad, inp, out, tag_d)
        return rid

    @staticmethod
    def prepare(op: int, slot: int, iv: bytes, aad, inp, out, tag_d) -> Request:
        """The request record for submit_prepared (argument marshalling done
        ahead of time); the caller keeps the tensors alive until the request
        completes."""
        r = Request()
        r.op = op
        r.key_slot = slot
        r.iv[:] = list(bytes(iv))
        r.reserved = 0
        r.aad_d = _dev(aad) or None
        r.aad_len = 0 if aad is None else aad.numel()
        r.in_d = _dev(inp) or None
        r.out_d = _dev(out) or None
        r.len = inp.numel()
        r.tag_d = _dev(tag_d)
        return r

    def submit_prepared(self, r: Request) -> int:
        rid = ctypes.c_uint64()
        _check(load().gcm_serve_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        return rid.value

    def poll(self, rid: int):
        """None while running, else (accept, latency_ns)."""
        done, acc, lat = ctypes.c_int(), ctypes.c_int(), ctypes.c_uint64()
        _check(load().gcm_serve_poll(self._h, rid, ctypes.byref(done), ctypes.byref(acc), ctypes.byref(lat)))
        if not done.value:
            return None
        self._keep.pop(rid, None)
        return bool(acc.value), lat.value

    def wait(self, rid: int):
        acc, lat = ctypes.c_int(), ctypes.c_uint64()
        _check(load().gcm_serve_wait(self._h, rid, ctypes.byref(acc), ctypes.byref(lat)))
        self._keep.pop(rid, None)
        return bool(acc.value), lat.value

    def drain(self) -> None:
        _check(load().gcm_serve_drain(self._h))

    def stats(self) -> dict:
        st = ServeStats()
        _check(load().gcm_serve_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def stop(self) -> None:
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check(load().gcm_serve_stop(h))
            self._keep.clear()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
