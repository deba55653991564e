"""Serving: continuous batching under an HBM budget.

Each request's result is the same alone and in the mix (tolerance 0 bytes:
the coder is lossless and its bitstream is unique for a given table and
parameters), the admission ledger never exceeds the budget, and latencies
are complete and consistent.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

K, R, L, W, N, C = 14, 16, 16, 1, 64, 65536


@pytest.fixture(scope="module")
def lr():
    import torch
    assert torch.cuda.is_available()
    import paper_1402_3392_amd as m
    return m


def make_requests(lr, nreq, seed, lo=12, hi=20):
    """Small mixed requests: payloads staged in device memory beforehand."""
    import torch
    reqs = datagen.serving_requests(nreq=nreq, seed=seed, lo_log2=lo, hi_log2=hi)
    params = lr.rans_params.make(K, R, L, W, N, C)
    out = []
    for q in reqs:
        syms = datagen.request_data(q, seed=seed)
        counts = datagen.counts(syms, 256)
        table = lr.rans_tables_build(counts, K)
        f = oracle.quantize(counts, K)
        if q["op"] == "encode":
            d_in = torch.from_numpy(syms).cuda()
            out.append(dict(op=lr.RANS_OP_ENCODE, table=table, d_in=d_in, in_len=syms.size,
                            out_cap=lr.rans_encode_bound(syms.size, params), syms=syms, f=f))
        else:
            cont = oracle.encode(f, syms, K, R, L, N, C)
            d_in = torch.from_numpy(cont).cuda()
            out.append(dict(op=lr.RANS_OP_DECODE, table=table, d_in=d_in, in_len=cont.size,
                            out_cap=syms.size, syms=syms, f=f, cont=cont))
    return out, params


def poisson(n, rate_per_us, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_per_us, n))


def device_bytes(addr, n):
    import torch
    t = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
    import ctypes
    torch.cuda.synchronize()
    # copy through the HIP runtime that torch already loaded
    hip = ctypes.CDLL("libamdhip64.so")
    assert hip.hipMemcpy(ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(addr), ctypes.c_size_t(n),
                         3) == 0  # device to device
    return t[:n].cpu().numpy()


def alone(lr, req, params):
    """The same request through the single-buffer entry points."""
    import torch
    if req["op"] == lr.RANS_OP_ENCODE:
        cap = req["out_cap"]
        d = torch.empty(cap, dtype=torch.uint8, device="cuda")
        n = lr.rans_encode(req["table"], params, req["d_in"], req["in_len"], d, cap)
        return d[:n].cpu().numpy()
    d = torch.empty(max(req["out_cap"], 16), dtype=torch.uint8, device="cuda")
    n = lr.rans_decode(req["table"], req["d_in"], req["in_len"], d, req["out_cap"])
    return d[:n].cpu().numpy()


def check_result(lr, q, c, params, solo=True):
    """A completion's output equals the request run alone and the oracle."""
    assert c.status == 0, c.status
    assert c.latency_us >= c.queue_us >= 0
    got = device_bytes(c.d_out, c.out_len)
    if q["op"] == lr.RANS_OP_ENCODE:
        ref = oracle.encode(q["f"], q["syms"], K, R, L, N, C)
        assert got.size == ref.size and (got == ref).all()
    else:
        assert got.size == q["syms"].size and (got == q["syms"]).all()
    if solo:
        alone_out = alone(lr, q, params)
        assert got.size == alone_out.size and (got == alone_out).all()


@pytest.mark.parametrize("budget_mib,streams,max_batch", [(512, 4, 16), (8, 2, 4)])
def test_same_alone_and_in_the_mix(lr, budget_mib, streams, max_batch):
    """A burst of every request at once, polled from here: each output,
    checked (and released) as soon as it completes while the others run,
    equals the request run alone and the oracle, and the server's counters
    show that launches held several requests and that several streams ran at
    once.  Then Poisson arrivals through the replay loop: every request
    completes with the oracle's output length, and free device memory is the
    same before and after (the server allocates nothing while serving)."""
    import torch
    reqs, params = make_requests(lr, 60, seed=5101)
    srv = lr.rans_server_create(budget_mib << 20, streams, max_batch, params)
    try:
        ids = {lr.rans_server_submit(srv, q["op"], q["table"], q["d_in"], q["in_len"],
                                     q["out_cap"]): q for q in reqs}
        done = 0
        for _ in range(1000000):
            for c in lr.rans_server_poll(srv, keep_outputs=True):
                check_result(lr, ids[c.id], c, params, solo=done % 3 == 0)
                lr.rans_server_release(srv, c.id)
                done += 1
            if done == len(reqs):
                break
        assert done == len(reqs)
        st = lr.rans_server_stats(srv)
        assert st["peak"] <= st["budget"] and st["used"] == st["fixed"]
        assert st["max_launch_requests"] > 1 and st["multi_request_launches"] >= 1, st
        assert st["peak_busy_streams"] > 1, st

        arrivals = poisson(len(reqs), rate_per_us=1 / 30.0, seed=7)
        spec = [(q["op"], q["table"], q["d_in"], q["in_len"], q["out_cap"], t)
                for q, t in zip(reqs, arrivals)]
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        res, mk = lr.rans_server_replay(srv, spec, keep_outputs=False)
        free1 = torch.cuda.mem_get_info()[0]
        assert free1 == free0, (free0, free1)
        st2 = lr.rans_server_stats(srv)
        assert st2["peak"] <= st2["budget"] and st2["used"] == st2["fixed"]
        assert st2["launches"] > st["launches"] and mk > 0
        for q, c in zip(reqs, res):
            assert c.status == 0, c.status
            assert c.latency_us >= c.queue_us >= 0
            if q["op"] == lr.RANS_OP_ENCODE:
                assert c.out_len == oracle.encode(q["f"], q["syms"], K, R, L, N, C).size
            else:
                assert c.out_len == q["syms"].size
    finally:
        lr.rans_server_destroy(srv)


def test_submit_poll_api_and_oversized_request(lr):
    import torch
    reqs, params = make_requests(lr, 6, seed=5202, lo=12, hi=14)
    srv = lr.rans_server_create(1 << 20, 2, 8, params)
    try:
        big = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
        with pytest.raises(lr.RansError) as e:
            lr.rans_server_submit(srv, lr.RANS_OP_ENCODE, reqs[0]["table"], big, big.numel(),
                                  2 << 20)
        assert e.value.code == lr.RANS_ENOMEM
        ids = [lr.rans_server_submit(srv, q["op"], q["table"], q["d_in"], q["in_len"], q["out_cap"])
               for q in reqs]
        done = {}
        for _ in range(200000):
            for c in lr.rans_server_poll(srv):
                done[c.id] = c
            if len(done) == len(ids):
                break
        assert sorted(done) == sorted(ids)
        assert all(c.status == 0 for c in done.values())
    finally:
        lr.rans_server_destroy(srv)
