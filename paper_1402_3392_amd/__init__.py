"""librans -- interleaved streaming rANS on MI355X: thin Python binding.

Argument marshalling only: every step of encoding and decoding runs in the
HIP kernels of ``librans.so`` (built from ``csrc/`` by ``_build.py``).  There
is no CPU fallback: importing this package without the built library raises.

The functions carry the C ABI's names (``include/librans.h``).  Device
buffers are torch tensors on a ROCm device (only their ``data_ptr()`` is
used) and streams are torch streams (``cuda_stream`` handle); torch is here
for device memory and streams, nothing else.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY_PATH = os.path.join(_HERE, "librans.so")

RANS_OK, RANS_EINVAL, RANS_EPREC, RANS_ENOSYM = 0, -1, -2, -3
RANS_ENOSPC, RANS_ECORRUPT, RANS_EDEVICE, RANS_ENOMEM = -4, -5, -6, -7

if not os.path.exists(LIBRARY_PATH):
    raise ImportError(f"{LIBRARY_PATH} is not built; run __graft_entry__.build() "
                      "(hipcc --offload-arch=gfx950) first")

_lib = ct.CDLL(LIBRARY_PATH)


class rans_params(ct.Structure):
    """Mirror of the C struct rans_params."""
    _fields_ = [("prob_bits", ct.c_uint8), ("radix_bits", ct.c_uint8),
                ("state_lbits", ct.c_uint8), ("sym_bytes", ct.c_uint8),
                ("interleave", ct.c_uint16), ("digit_order", ct.c_uint8),
                ("escape", ct.c_uint8), ("chunk_syms", ct.c_uint32)]

    @classmethod
    def make(cls, k, r, l, w, N, C, order="df", escape=False):
        """order: "df" (depth-first) or "bf" (breadth-first) digit order;
        escape: escape coding with raw digits (16-bit symbols)."""
        if order not in ("df", "bf"):
            raise ValueError(f"digit order {order!r}: expected 'df' or 'bf'")
        return cls(k, r, l, w, N, 1 if order == "bf" else 0, 1 if escape else 0, C)


class rans_batch_config(ct.Structure):
    """Mirror of the C struct rans_batch_config."""
    _fields_ = [("waves_per_group", ct.c_uint32), ("groups_per_cu", ct.c_uint32),
                ("table_layout", ct.c_uint32), ("use_graph", ct.c_uint32)]


class rans_tune_result(ct.Structure):
    _fields_ = [("chunk_syms", ct.c_uint32), ("waves_per_group", ct.c_uint32),
                ("groups_per_cu", ct.c_uint32), ("table_layout", ct.c_uint32),
                ("encode_gbps", ct.c_double), ("decode_gbps", ct.c_double),
                ("use_graph", ct.c_uint32), ("interleave", ct.c_uint32),
                ("lanes_per_stream", ct.c_uint32), ("chunks_per_wave", ct.c_uint32)]


class rans_job(ct.Structure):
    """Mirror of the C struct rans_job."""
    _fields_ = [("table", ct.c_void_p), ("in_", ct.c_void_p), ("in_len", ct.c_uint64),
                ("out", ct.c_void_p), ("out_cap", ct.c_uint64),
                ("d_out_len", ct.c_void_p), ("d_status", ct.c_void_p)]


class rans_server_config(ct.Structure):
    _fields_ = [("hbm_budget", ct.c_uint64), ("streams", ct.c_uint32), ("max_batch", ct.c_uint32),
                ("params", rans_params)]


class rans_completion(ct.Structure):
    _fields_ = [("id", ct.c_uint64), ("status", ct.c_int32), ("op", ct.c_int32),
                ("in_len", ct.c_uint64), ("out_len", ct.c_uint64), ("d_out", ct.c_void_p),
                ("latency_us", ct.c_double), ("queue_us", ct.c_double)]


class rans_server_stats_t(ct.Structure):
    _fields_ = [("budget", ct.c_uint64), ("used", ct.c_uint64), ("peak", ct.c_uint64),
                ("waiting", ct.c_uint32), ("ready", ct.c_uint32), ("busy_streams", ct.c_uint32),
                ("peak_busy_streams", ct.c_uint32), ("launches", ct.c_uint64),
                ("multi_request_launches", ct.c_uint64), ("fixed", ct.c_uint64),
                ("max_launch_requests", ct.c_uint32), ("reserved", ct.c_uint32)]


class rans_server_request(ct.Structure):
    _fields_ = [("op", ct.c_int32), ("reserved", ct.c_uint32), ("table", ct.c_void_p),
                ("d_in", ct.c_void_p), ("in_len", ct.c_uint64), ("out_cap", ct.c_uint64),
                ("arrival_us", ct.c_double)]


RANS_OP_ENCODE, RANS_OP_DECODE = 0, 1

_u64p = ct.POINTER(ct.c_uint64)
_u32p = ct.POINTER(ct.c_uint32)
_P = ct.POINTER(rans_params)
_sig = {
    "rans_quantize": (ct.c_int, [_u64p, ct.c_uint32, ct.c_uint32, _u32p]),
    "rans_tables_build": (ct.c_int, [_u64p, ct.c_uint32, ct.c_uint32, ct.POINTER(ct.c_void_p)]),
    "rans_table_freqs": (ct.c_int, [ct.c_void_p, _u32p]),
    "rans_table_alphabet": (ct.c_uint32, [ct.c_void_p]),
    "rans_table_prob_bits": (ct.c_uint32, [ct.c_void_p]),
    "rans_table_destroy": (None, [ct.c_void_p]),
    "rans_params_check": (ct.c_int, [_P]),
    "rans_encode_bound": (ct.c_uint64, [ct.c_uint64, _P]),
    "rans_encode": (ct.c_int, [ct.c_void_p, _P, ct.c_void_p, ct.c_uint64, ct.c_void_p,
                               ct.c_uint64, _u64p, ct.c_void_p]),
    "rans_decode": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_uint64, ct.c_void_p,
                               ct.c_uint64, _u64p, ct.c_void_p]),
    "rans_encode_async": (ct.c_int, [ct.c_void_p, _P, ct.c_void_p, ct.c_uint64, ct.c_void_p,
                                     ct.c_uint64, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "rans_encode_async_noalloc": (ct.c_int, [ct.c_void_p, _P, ct.c_void_p, ct.c_uint64, ct.c_void_p,
                                             ct.c_uint64, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "rans_decode_async": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_uint64, ct.c_char_p,
                                     ct.c_void_p, ct.c_uint64, ct.c_void_p, ct.c_void_p]),
    "rans_pfx_encode": (ct.c_int, [ct.c_void_p, _P, ct.c_void_p, ct.c_uint64, ct.c_void_p,
                                   ct.c_uint64, _u64p, ct.c_void_p]),
    "rans_pfx_encode_async": (ct.c_int, [ct.c_void_p, _P, ct.c_void_p, ct.c_uint64, ct.c_void_p,
                                         ct.c_uint64, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "rans_decode_lut": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_uint64, ct.c_void_p, ct.c_uint32,
                                   ct.c_void_p, ct.c_uint64, _u64p, ct.c_void_p]),
    "rans_decode_lut_async": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_uint64, ct.c_char_p,
                                         ct.c_void_p, ct.c_uint32, ct.c_void_p, ct.c_uint64,
                                         ct.c_void_p, ct.c_void_p]),
    "rans_encode_batch": (ct.c_int, [ct.POINTER(rans_job), ct.c_uint32, _P, ct.c_void_p]),
    "rans_decode_batch": (ct.c_int, [ct.POINTER(rans_job), ct.c_uint32, _P, ct.c_void_p]),
    "rans_strerror": (ct.c_char_p, [ct.c_int]),
    "rans_batch_set_config": (ct.c_int, [ct.POINTER(rans_batch_config)]),
    "rans_autotune": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_uint64, _P, ct.c_char_p,
                                 ct.POINTER(rans_tune_result)]),
    "rans_autotune_batch": (ct.c_int, [ct.POINTER(rans_job), ct.c_uint32, _P, ct.c_char_p,
                                       ct.POINTER(rans_tune_result)]),
    "rans_server_create": (ct.c_int, [ct.POINTER(rans_server_config), ct.POINTER(ct.c_void_p)]),
    "rans_server_destroy": (None, [ct.c_void_p]),
    "rans_server_submit": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_uint64,
                                      ct.c_uint64, _u64p]),
    "rans_server_poll": (ct.c_int, [ct.c_void_p, ct.c_int, ct.POINTER(rans_completion), ct.c_uint32,
                                    ct.POINTER(ct.c_uint32)]),
    "rans_server_release": (ct.c_int, [ct.c_void_p, ct.c_uint64]),
    "rans_server_stats": (ct.c_int, [ct.c_void_p, ct.POINTER(rans_server_stats_t)]),
    "rans_server_replay": (ct.c_int, [ct.c_void_p, ct.POINTER(rans_server_request), ct.c_uint32,
                                      ct.c_int, ct.POINTER(rans_completion),
                                      ct.POINTER(ct.c_double)]),
    "rans_batch_get_config": (ct.c_int, [ct.POINTER(rans_batch_config)]),
    "rans_workspace_release": (ct.c_int, [ct.c_void_p]),
    "rans_timing_enable": (ct.c_int, [ct.c_int]),
    "rans_timing_reset": (ct.c_int, []),
    "rans_timing_read": (ct.c_int, [ct.c_int, _u64p, ct.POINTER(ct.c_double)]),
}
for _name, (_res, _args) in _sig.items():
    if hasattr(_lib, _name):
        _fn = getattr(_lib, _name)
        _fn.restype = _res
        _fn.argtypes = _args


class RansError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {rans_strerror(code)} ({code})")
        self.code = code


def _check(rc: int, what: str):
    if rc != RANS_OK:
        raise RansError(rc, what)


def rans_strerror(code: int) -> str:
    return _lib.rans_strerror(code).decode()


def _ptr(buf) -> int:
    """Device address of a torch tensor (or an int address)."""
    if buf is None:
        return 0
    if isinstance(buf, int):
        return buf
    return int(buf.data_ptr())


def _stream(stream) -> int:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _params(p) -> rans_params:
    if isinstance(p, rans_params):
        return p
    if isinstance(p, dict):
        return rans_params.make(p["k"], p["r"], p["l"], p["w"], p["N"], p["C"], p.get("order", "df"),
                                p.get("escape", False))
    if hasattr(p, "astuple"):
        return rans_params.make(*p.astuple())
    return rans_params.make(*p)


# ------------------------------------------------------------------ tables --

def rans_quantize(counts, prob_bits: int) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint64))
    f = np.zeros(len(c), dtype=np.uint32)
    _check(_lib.rans_quantize(c.ctypes.data_as(_u64p), len(c), prob_bits,
                              f.ctypes.data_as(_u32p)), "rans_quantize")
    return f


class Table:
    """Owning handle of a device-resident rans_table."""

    def __init__(self, handle: int):
        self.handle = handle

    @property
    def alphabet(self) -> int:
        return int(_lib.rans_table_alphabet(self.handle))

    @property
    def prob_bits(self) -> int:
        return int(_lib.rans_table_prob_bits(self.handle))

    def close(self):
        if self.handle:
            _lib.rans_table_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rans_tables_build(counts, prob_bits: int) -> Table:
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint64))
    h = ct.c_void_p()
    _check(_lib.rans_tables_build(c.ctypes.data_as(_u64p), len(c), prob_bits, ct.byref(h)),
           "rans_tables_build")
    return Table(h.value)


def rans_table_freqs(table: Table) -> np.ndarray:
    f = np.zeros(table.alphabet, dtype=np.uint32)
    _check(_lib.rans_table_freqs(table.handle, f.ctypes.data_as(_u32p)), "rans_table_freqs")
    return f


def rans_params_check(params) -> int:
    p = _params(params)
    return int(_lib.rans_params_check(ct.byref(p)))


def rans_encode_bound(n_syms: int, params) -> int:
    p = _params(params)
    return int(_lib.rans_encode_bound(n_syms, ct.byref(p)))


# ------------------------------------------------------- single buffers ----

def rans_encode(table: Table, params, d_syms, n_syms: int, d_out, out_cap: int,
                stream=None) -> int:
    """Encodes n_syms symbols at d_syms into d_out; returns the container length."""
    p = _params(params)
    olen = ct.c_uint64()
    rc = _lib.rans_encode(table.handle, ct.byref(p), _ptr(d_syms), n_syms, _ptr(d_out), out_cap,
                          ct.byref(olen), _stream(stream))
    _check(rc, "rans_encode")
    return int(olen.value)


def rans_decode(table: Table, d_in, in_len: int, d_syms, syms_cap: int, stream=None) -> int:
    """Decodes the container d_in[in_len] into d_syms; returns the symbol count."""
    n = ct.c_uint64()
    rc = _lib.rans_decode(table.handle, _ptr(d_in), in_len, _ptr(d_syms), syms_cap, ct.byref(n),
                          _stream(stream))
    _check(rc, "rans_decode")
    return int(n.value)


def rans_encode_async(table: Table, params, d_syms, n_syms: int, d_out, out_cap: int,
                      d_out_len, d_status, stream=None):
    """Stream-ordered encode; *d_status (device int32) must be 0 beforehand."""
    p = _params(params)
    _check(_lib.rans_encode_async(table.handle, ct.byref(p), _ptr(d_syms), n_syms, _ptr(d_out),
                                  out_cap, _ptr(d_out_len), _ptr(d_status), _stream(stream)),
           "rans_encode_async")


def rans_encode_async_noalloc(table: Table, params, d_syms, n_syms: int, d_out, out_cap: int,
                              d_out_len, d_status, stream=None):
    """rans_encode_async with its scratch in the library's fixed device array
    (allocates nothing; calls overlapping on one GPU race)."""
    p = _params(params)
    _check(_lib.rans_encode_async_noalloc(table.handle, ct.byref(p), _ptr(d_syms), n_syms,
                                          _ptr(d_out), out_cap, _ptr(d_out_len), _ptr(d_status),
                                          _stream(stream)),
           "rans_encode_async_noalloc")


def rans_decode_async(table: Table, d_in, in_len: int, header: bytes, d_syms, syms_cap: int,
                      d_status, stream=None):
    """Stream-ordered decode given a host copy of the 32-byte header."""
    hb = bytes(header[:32])
    _check(_lib.rans_decode_async(table.handle, _ptr(d_in), in_len, hb, _ptr(d_syms), syms_cap,
                                  _ptr(d_status), _stream(stream)), "rans_decode_async")


def rans_pfx_encode(table: Table, params, d_syms, n_syms: int, d_out, out_cap: int,
                    stream=None) -> int:
    """Encodes with the prefix-code family multiplexed as Section 4 describes;
    returns the container length (decode with rans_decode)."""
    p = _params(params)
    out_len = ct.c_uint64()
    rc = _lib.rans_pfx_encode(table.handle, ct.byref(p), _ptr(d_syms), n_syms, _ptr(d_out), out_cap,
                              ct.byref(out_len), _stream(stream))
    _check(rc, "rans_pfx_encode")
    return int(out_len.value)


def rans_pfx_encode_async(table: Table, params, d_syms, n_syms: int, d_out, out_cap: int,
                          d_out_len, d_status, stream=None):
    p = _params(params)
    _check(_lib.rans_pfx_encode_async(table.handle, ct.byref(p), _ptr(d_syms), n_syms, _ptr(d_out),
                                      out_cap, _ptr(d_out_len), _ptr(d_status), _stream(stream)),
           "rans_pfx_encode_async")


def rans_decode_lut(table: Table, d_in, in_len: int, d_lut, lut_bytes: int, d_out, out_cap: int,
                    stream=None) -> int:
    """Decode fused with a lookup: d_out[i] = d_lut[symbol i] (lut_bytes = 2 or 4 bytes per
    element); returns the element count."""
    n = ct.c_uint64()
    rc = _lib.rans_decode_lut(table.handle, _ptr(d_in), in_len, _ptr(d_lut), lut_bytes, _ptr(d_out),
                              out_cap, ct.byref(n), _stream(stream))
    _check(rc, "rans_decode_lut")
    return int(n.value)


def rans_decode_lut_async(table: Table, d_in, in_len: int, header: bytes, d_lut, lut_bytes: int,
                          d_out, out_cap: int, d_status, stream=None):
    """Stream-ordered rans_decode_lut given a host copy of the 32-byte header."""
    hb = bytes(header[:32])
    _check(_lib.rans_decode_lut_async(table.handle, _ptr(d_in), in_len, hb, _ptr(d_lut), lut_bytes,
                                      _ptr(d_out), out_cap, _ptr(d_status), _stream(stream)),
           "rans_decode_lut_async")


# ---------------------------------------------------------------- batches --

def make_jobs(specs) -> ct.Array:
    """specs: iterable of (table, d_in, in_len, d_out, out_cap, d_out_len_addr, d_status_addr)."""
    specs = list(specs)
    arr = (rans_job * max(1, len(specs)))()
    for i, (tab, din, inl, dout, cap, dlen, dst) in enumerate(specs):
        arr[i] = rans_job(tab.handle, _ptr(din), inl, _ptr(dout), cap, _ptr(dlen), _ptr(dst))
    return arr


def rans_encode_batch(jobs, njobs: int, params, stream=None):
    p = _params(params)
    _check(_lib.rans_encode_batch(jobs, njobs, ct.byref(p), _stream(stream)), "rans_encode_batch")


def rans_decode_batch(jobs, njobs: int, params, stream=None):
    p = _params(params)
    _check(_lib.rans_decode_batch(jobs, njobs, ct.byref(p), _stream(stream)), "rans_decode_batch")


def rans_batch_set_config(waves_per_group: int = 16, groups_per_cu: int = 1,
                          table_layout: int = 0, use_graph: int = 1):
    cfg = rans_batch_config(waves_per_group, groups_per_cu, table_layout, use_graph)
    _check(_lib.rans_batch_set_config(ct.byref(cfg)), "rans_batch_set_config")


def rans_batch_get_config() -> dict:
    cfg = rans_batch_config()
    _check(_lib.rans_batch_get_config(ct.byref(cfg)), "rans_batch_get_config")
    return {f: int(getattr(cfg, f)) for f, _ in cfg._fields_}


def rans_autotune(table: Table, d_syms, n_syms: int, params, cache_path: str | None = None):
    """Tunes chunk size and batched decode shape on a device sample; returns a dict."""
    p = _params(params)
    r = rans_tune_result()
    cp = cache_path.encode() if cache_path else None
    _check(_lib.rans_autotune(table.handle, _ptr(d_syms), n_syms, ct.byref(p), cp, ct.byref(r)),
           "rans_autotune")
    return {f: getattr(r, f) for f, _ in r._fields_}


def rans_autotune_batch(jobs, njobs: int, params, cache_path: str | None = None):
    """Tunes on a whole batch of encode jobs (make_jobs); returns a dict."""
    p = _params(params)
    r = rans_tune_result()
    cp = cache_path.encode() if cache_path else None
    _check(_lib.rans_autotune_batch(jobs, njobs, ct.byref(p), cp, ct.byref(r)), "rans_autotune_batch")
    return {f: getattr(r, f) for f, _ in r._fields_}


# ---------------------------------------------------------------- serving --

def rans_server_create(hbm_budget: int, streams: int, max_batch: int, params):
    cfg = rans_server_config(hbm_budget, streams, max_batch, _params(params))
    h = ct.c_void_p()
    _check(_lib.rans_server_create(ct.byref(cfg), ct.byref(h)), "rans_server_create")
    return h.value


def rans_server_destroy(server):
    _lib.rans_server_destroy(server)


def rans_server_submit(server, op: int, table: Table, d_in, in_len: int, out_cap: int) -> int:
    rid = ct.c_uint64()
    _check(_lib.rans_server_submit(server, op, table.handle, _ptr(d_in), in_len, out_cap,
                                   ct.byref(rid)), "rans_server_submit")
    return int(rid.value)


def rans_server_poll(server, keep_outputs: bool = False, max_out: int = 256):
    arr = (rans_completion * max_out)()
    n = ct.c_uint32()
    _check(_lib.rans_server_poll(server, 1 if keep_outputs else 0, arr, max_out, ct.byref(n)),
           "rans_server_poll")
    return [arr[i] for i in range(n.value)]


def rans_server_release(server, rid: int):
    _check(_lib.rans_server_release(server, rid), "rans_server_release")


def rans_server_stats(server) -> dict:
    st = rans_server_stats_t()
    _check(_lib.rans_server_stats(server, ct.byref(st)), "rans_server_stats")
    return {f: int(getattr(st, f)) for f, _ in st._fields_}


def rans_server_replay(server, requests, keep_outputs: bool = False):
    """requests: list of (op, table, d_in, in_len, out_cap, arrival_us).
    Returns (list of rans_completion in request order, makespan_us)."""
    n = len(requests)
    arr = (rans_server_request * max(n, 1))()
    for i, (op, tab, din, inl, cap, t) in enumerate(requests):
        arr[i] = rans_server_request(op, 0, tab.handle, _ptr(din), inl, cap, float(t))
    res = (rans_completion * max(n, 1))()
    mk = ct.c_double()
    _check(_lib.rans_server_replay(server, arr, n, 1 if keep_outputs else 0, res, ct.byref(mk)),
           "rans_server_replay")
    return [res[i] for i in range(n)], float(mk.value)


# ------------------------------------------------------------------ timing --

RANS_KERNEL_DECODE, RANS_KERNEL_ENCODE, RANS_KERNEL_SCAN, RANS_KERNEL_COMPACT = 0, 1, 2, 3
RANS_KERNEL_BATCH_DECODE, RANS_KERNEL_BATCH_ENCODE, RANS_KERNEL_BATCH_PLAN = 4, 5, 6


def rans_workspace_release(stream=None):
    _check(_lib.rans_workspace_release(_stream(stream)), "rans_workspace_release")


def rans_timing_enable(on: bool = True):
    _check(_lib.rans_timing_enable(1 if on else 0), "rans_timing_enable")


def rans_timing_reset():
    _check(_lib.rans_timing_reset(), "rans_timing_reset")


def rans_timing_read(kind: int):
    """Returns (launches, total milliseconds) of one kernel kind."""
    n = ct.c_uint64()
    ms = ct.c_double()
    _check(_lib.rans_timing_read(kind, ct.byref(n), ct.byref(ms)), "rans_timing_read")
    return int(n.value), float(ms.value)


# --------------------------------------------------- torch conveniences ----

def encode(table: Table, params, syms, stream=None):
    """syms: device uint8 tensor of n*w bytes.  Returns (container tensor, length)."""
    import torch
    p = _params(params)
    n = syms.numel() * syms.element_size() // p.sym_bytes
    cap = rans_encode_bound(n, p)
    out = torch.empty(max(cap, 16), dtype=torch.uint8, device=syms.device)
    olen = rans_encode(table, p, syms, n, out, cap, stream)
    return out, olen


def decode(table: Table, container, in_len: int, n_syms: int, sym_bytes: int = 1, stream=None):
    """Returns a device uint8 tensor holding n_syms*sym_bytes decoded bytes."""
    import torch
    out = torch.empty(max(n_syms * sym_bytes, 16), dtype=torch.uint8, device=container.device)
    n = rans_decode(table, container, in_len, out, n_syms, stream)
    return out[: n * sym_bytes]
