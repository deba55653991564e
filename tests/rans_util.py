"""Helpers shared by the GPU tests: move numpy arrays through librans."""
from __future__ import annotations

import numpy as np


def dev(arr: np.ndarray):
    import torch
    raw = np.ascontiguousarray(arr).view(np.uint8).reshape(-1)
    t = torch.empty(max(raw.size, 16), dtype=torch.uint8, device="cuda")
    if raw.size:
        t[: raw.size].copy_(torch.from_numpy(raw.copy()))
    return t


def host(t, nbytes: int) -> np.ndarray:
    return t[:nbytes].cpu().numpy().copy()


def gpu_encode(lr, table, params, syms: np.ndarray) -> np.ndarray:
    """Encodes on the GPU; returns the container as a host uint8 array."""
    import torch
    p = lr.rans_params.make(*params)
    n = syms.size
    cap = lr.rans_encode_bound(n, p)
    d_in = dev(syms)
    d_out = torch.full((cap + 64,), 0xA5, dtype=torch.uint8, device="cuda")
    olen = lr.rans_encode(table, p, d_in, n, d_out, cap)
    torch.cuda.synchronize()
    return host(d_out, olen)


def gpu_decode(lr, table, container: np.ndarray, n: int, w: int) -> np.ndarray:
    import torch
    d_in = dev(container)
    d_out = torch.full((n * w + 64,), 0x5A, dtype=torch.uint8, device="cuda")
    got = lr.rans_decode(table, d_in, container.size, d_out, n)
    torch.cuda.synchronize()
    assert got == n
    tail = d_out[n * w: n * w + 64].cpu().numpy()
    assert (tail == 0x5A).all(), "decode wrote past the symbol count"
    raw = host(d_out, n * w)
    return raw.view(np.uint8 if w == 1 else np.uint16)


def first_diff(a: np.ndarray, b: np.ndarray) -> str:
    if a.size != b.size:
        return f"length {a.size} vs {b.size}"
    idx = np.flatnonzero(a != b)
    return "equal" if idx.size == 0 else f"first diff at byte {idx[0]} of {a.size}"
