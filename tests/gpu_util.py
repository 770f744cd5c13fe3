"""Shared helpers for the GPU tests (device buffers, canaries)."""
from __future__ import annotations

import numpy as np
import torch

CANARY = 0xA5
PAD = 4096


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a).view(np.uint8).reshape(-1).copy()).to("cuda")


def guarded(n: int):
    """(full buffer, view of n bytes starting PAD bytes in) pre-filled with the canary."""
    full = torch.full((n + 2 * PAD,), CANARY, dtype=torch.uint8, device="cuda")
    return full, full[PAD:PAD + n]


def canaries_intact(full: torch.Tensor, n: int) -> bool:
    head = full[:PAD].cpu().numpy()
    tail = full[PAD + n:].cpu().numpy()
    return bool((head == CANARY).all() and (tail == CANARY).all())


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()
