"""CPU oracle for interleaved streaming rANS -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The product library neither imports nor links it, and
it shares no code with it.  The arithmetic lives in ``rans_oracle.c`` (plain
C, 64-bit integers, '/' and '%'); this module only builds that file with gcc
and marshals numpy arrays through ctypes.

Paper: F. Giesen, "Interleaved entropy coders" (arXiv:1402.3392):
coding pair C/D (Section 2, example in Section 2.1), Algorithm 1 streaming
renormalisation, interleaving of N coders in one stream (Sections 3-4),
depth-first / breadth-first digit order (Section 5).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rans_oracle.c")
_LIB = os.path.join(_HERE, "librans_oracle.so")

OK, EINVAL, EPREC, ENOSYM, ENOSPC, ECORRUPT, ENOMEM = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "OK", -1: "EINVAL", -2: "EPREC", -3: "ENOSYM", -4: "ENOSPC",
          -5: "ECORRUPT", -6: "ENOMEM"}

_lib = None


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle error {code} ({_NAMES.get(code, '?')})")
        self.code = code


def build(force: bool = True) -> str:
    """Compiles rans_oracle.c into librans_oracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                               "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def use_library(path: str | None) -> None:
    """Points the wrapper at another build of rans_oracle.c (the mutation test
    compiles deliberately broken copies); None returns to the default."""
    global _lib
    _lib = None if path is None else _bind(ct.CDLL(path))


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    _lib = _bind(ct.CDLL(_LIB))
    return _lib


def _bind(lib):
    u32p = ct.POINTER(ct.c_uint32)
    u64p = ct.POINTER(ct.c_uint64)
    u8p = ct.POINTER(ct.c_uint8)
    u32, u64, i32 = ct.c_uint32, ct.c_uint64, ct.c_int
    lib.orc_quantize.argtypes = [u64p, u32, u32, u32p]
    lib.orc_C.argtypes = [u32p, u32, u32, u32, u64]
    lib.orc_C.restype = u64
    lib.orc_D.argtypes = [u32p, u32, u32, u64, u32p, u64p]
    lib.orc_encode_digits.argtypes = [u32p, u32, u32, u32, u32, u32, i32, u32p, u64,
                                      u64p, u32p, u64, u64p, u64p]
    lib.orc_decode_digits.argtypes = [u32p, u32, u32, u32, u32, u32, i32, u64p, u32p, u64,
                                      u32p, u64, u64p]
    lib.orc_encode_bound.argtypes = [u64, u32, u32, u32, u32]
    lib.orc_encode_bound.restype = u64
    lib.orc_encode.argtypes = [u32p, u32, u32, u32, u32, u32, u32, u32, u8p, u64, u8p, u64,
                               u64p, i32]
    lib.orc_encode_order.argtypes = [u32p, u32, u32, u32, u32, u32, u32, u32, i32, u8p, u64, u8p,
                                     u64, u64p, i32]
    lib.orc_encode_flags.argtypes = [u32p, u32, u32, u32, u32, u32, u32, u32, i32, u8p, u64, u8p,
                                     u64, u64p, i32]
    lib.orc_encode_bound_raw.argtypes = [u64, u32, u32, u32, u32, u32]
    lib.orc_encode_bound_raw.restype = u64
    lib.orc_pfx_code.argtypes = [u32p, u32, u32, u32p, u32p]
    lib.orc_decode.argtypes = [u32p, u32, u8p, u64, u8p, u64, u64p, i32]
    lib.orc_header.argtypes = [u8p, u64, u64p]
    return lib


def _p(a: np.ndarray, ctype):
    return a.ctypes.data_as(ct.POINTER(ctype))


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def _check(rc: int, what: str):
    if rc != OK:
        raise OracleError(rc, what)


# ---------------------------------------------------------------- model ----

def quantize(counts, k: int) -> np.ndarray:
    """Quantises symbol counts to frequencies summing to 2^k (reading Q2)."""
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint64))
    f = np.zeros(len(c), dtype=np.uint32)
    _check(_load().orc_quantize(_p(c, ct.c_uint64), len(c), k, _p(f, ct.c_uint32)),
           "quantize")
    return f


def C(f, k: int, s: int, x: int) -> int:
    """rANS coding function C(s, x) (Section 2)."""
    f = _u32(f)
    y = _load().orc_C(_p(f, ct.c_uint32), len(f), k, s, x)
    if y == 2**64 - 1:
        raise OracleError(EINVAL, "C")
    return int(y)


def D(f, k: int, x: int) -> tuple[int, int]:
    """rANS decoding function D(x) = (s, x') (Section 2)."""
    f = _u32(f)
    s = ct.c_uint32()
    xo = ct.c_uint64()
    _check(_load().orc_D(_p(f, ct.c_uint32), len(f), k, x, ct.byref(s), ct.byref(xo)), "D")
    return int(s.value), int(xo.value)


# ------------------------------------------------------- digit streams ----

def encode_digits(f, k: int, r: int, l: int, N: int, syms, order: str = "df",
                  trace: bool = False):
    """Interleaved encode of one chunk into a digit stream.

    Returns (states[N], digits, trace-or-None); digits are in decoder order.
    order 'df' = depth-first (N scalar Algorithm-1 coders sharing a buffer),
    'bf' = breadth-first renormalisation rounds (Section 5)."""
    f = _u32(f)
    s = _u32(syms)
    n = len(s)
    cap = ((k + r - 1) // r) * n + 1
    states = np.zeros(N, dtype=np.uint64)
    dig = np.zeros(cap, dtype=np.uint32)
    nd = ct.c_uint64()
    tr = np.zeros(max(n, 1), dtype=np.uint64)
    rc = _load().orc_encode_digits(_p(f, ct.c_uint32), len(f), k, r, l, N,
                                   1 if order == "bf" else 0, _p(s, ct.c_uint32), n,
                                   _p(states, ct.c_uint64), _p(dig, ct.c_uint32), cap,
                                   ct.byref(nd), _p(tr, ct.c_uint64) if trace else None)
    _check(rc, "encode_digits")
    return states, dig[:nd.value].copy(), (tr[:n] if trace else None)


def decode_digits(f, k: int, r: int, l: int, N: int, states, digits, n: int,
                  order: str = "df", trace: bool = False):
    """Interleaved decode of one chunk; raises OracleError(ECORRUPT) when the
    coders do not end in state L with the stream fully consumed."""
    f = _u32(f)
    st = np.ascontiguousarray(np.asarray(states, dtype=np.uint64))
    dg = _u32(digits)
    out = np.zeros(max(n, 1), dtype=np.uint32)
    tr = np.zeros(max(n, 1), dtype=np.uint64)
    rc = _load().orc_decode_digits(_p(f, ct.c_uint32), len(f), k, r, l, N,
                                   1 if order == "bf" else 0, _p(st, ct.c_uint64),
                                   _p(dg, ct.c_uint32), len(dg), _p(out, ct.c_uint32), n,
                                   _p(tr, ct.c_uint64) if trace else None)
    _check(rc, "decode_digits")
    return (out[:n], tr[:n]) if trace else out[:n]


# ------------------------------------------------------------ container ----

def encode_bound(n: int, k: int, r: int, N: int, C: int) -> int:
    return int(_load().orc_encode_bound(n, k, r, N, C))


def prefix_code(f, k: int) -> tuple[np.ndarray, np.ndarray]:
    """(lengths, codes) of the canonical prefix code for frequencies f."""
    f = _u32(f)
    ln = np.zeros(len(f), np.uint32)
    cd = np.zeros(len(f), np.uint32)
    _check(_load().orc_pfx_code(_p(f, ct.c_uint32), len(f), k, _p(ln, ct.c_uint32),
                                _p(cd, ct.c_uint32)), "prefix_code")
    return ln, cd


def encode(f, syms: np.ndarray, k: int, r: int, l: int, N: int, C: int,
           threads: int = 1, order: str = "df", escape: bool = False,
           coder: str = "rans") -> np.ndarray:
    """Encodes a symbol array (uint8 or uint16) into a container (uint8 array).
    order: digit order of the chunk streams, 'df' depth-first or 'bf'
    breadth-first (Section 5).  escape: escape coding with raw digits
    (uint16 symbols, depth-first; the last symbol of f is the escape).
    coder 'prefix': the prefix-code family multiplexed by the instrumented
    decoder (Section 4; r must be 16, l is recorded but unused).  All three
    are recorded in header byte 9."""
    f = _u32(f)
    syms = np.ascontiguousarray(syms)
    w = syms.dtype.itemsize
    if syms.dtype not in (np.uint8, np.uint16):
        raise ValueError("symbols must be uint8 or uint16")
    n = syms.size
    nraw = (8 * w + r - 1) // r if escape else 0
    cap = int(_load().orc_encode_bound_raw(n, k, r, N, C, nraw))
    if coder == "prefix":  # a word per symbol at most, plus one per coder and chunk
        cap = encode_bound(n, 16, 16, N, C) + 2 * N * (n // max(C, 1) + 2)
    elif coder != "rans":
        raise ValueError("coder must be 'rans' or 'prefix'")
    out = np.zeros(cap, dtype=np.uint8)
    olen = ct.c_uint64()
    raw = syms.view(np.uint8).reshape(-1) if n else np.zeros(1, dtype=np.uint8)
    if order not in ("df", "bf"):
        raise ValueError("order must be 'df' or 'bf'")
    flags = (1 if order == "bf" else 0) | (2 if escape else 0) | (4 if coder == "prefix" else 0)
    rc = _load().orc_encode_flags(_p(f, ct.c_uint32), len(f), k, r, l, w, N, C, flags,
                                  _p(raw, ct.c_uint8), n, _p(out, ct.c_uint8), cap,
                                  ct.byref(olen), threads)
    _check(rc, "encode")
    return out[:olen.value]


def header(container: np.ndarray) -> dict:
    buf = np.ascontiguousarray(container, dtype=np.uint8)
    h = np.zeros(11, dtype=np.uint64)
    _check(_load().orc_header(_p(buf, ct.c_uint8), buf.size, _p(h, ct.c_uint64)), "header")
    keys = ("k", "r", "l", "w", "N", "C", "n", "n_chunks", "order", "nraw", "prefix")
    d = {kk: int(v) for kk, v in zip(keys, h)}
    d["order"] = "bf" if d["order"] else "df"
    d["escape"] = d["nraw"] > 0
    d["coder"] = "prefix" if d.pop("prefix") else "rans"
    return d


def decode(f, container: np.ndarray, threads: int = 1) -> np.ndarray:
    """Decodes a container back into its symbol array (uint8 or uint16)."""
    f = _u32(f)
    buf = np.ascontiguousarray(container, dtype=np.uint8)
    h = header(buf)
    dt = np.uint8 if h["w"] == 1 else np.uint16
    out = np.zeros(max(h["n"], 1), dtype=dt)
    n = ct.c_uint64()
    rc = _load().orc_decode(_p(f, ct.c_uint32), len(f), _p(buf, ct.c_uint8), buf.size,
                            _p(out.view(np.uint8), ct.c_uint8), h["n"], ct.byref(n), threads)
    _check(rc, "decode")
    return out[:n.value]
