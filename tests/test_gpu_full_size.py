"""GPU parity at the workloads' real sizes (through the C ABI).

The containers the GPU writes are compared byte for byte with the oracle's
and the GPU decodes the oracle's containers back to the input: the 1 MiB
four-coder stream in one chunk, the three 256 MiB Zipf buffers, points of the
64 MiB radix/precision sweep (plain and batched paths), uneven streams from
the batched workload's generator in one batched launch, and serving requests
drawn from the serving workload's size distribution.
"""
import numpy as np
import pytest

import datagen
import oracle
from rans_util import first_diff, gpu_decode, gpu_encode

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
THREADS = 16


@pytest.fixture(scope="module")
def lr():
    import torch
    assert torch.cuda.is_available()
    import paper_1402_3392_amd as m
    return m


def check_roundtrip(lr, syms, alphabet, k, r, l, N, C):
    w = syms.dtype.itemsize
    counts = datagen.counts(syms, alphabet)
    f = oracle.quantize(counts, k)
    table = lr.rans_tables_build(counts, k)
    assert (lr.rans_table_freqs(table) == f).all()
    ref = oracle.encode(f, syms, k, r, l, N, C, threads=THREADS)
    got = gpu_encode(lr, table, (k, r, l, w, N, C), syms)
    assert got.size == ref.size and (got == ref).all(), first_diff(got, ref)
    dec = gpu_decode(lr, table, ref, syms.size, w)
    assert (dec.view(syms.dtype) == syms).all()
    return table, ref


def test_one_chunk_four_coders_1MiB(lr):
    w = datagen.tiny_zipf()
    check_roundtrip(lr, w.syms, 256, *w.params.astuple()[:3], w.params.N, w.params.C)


@pytest.mark.parametrize("s", datagen.ZIPF_S)
def test_256MiB_zipf(lr, s):
    w = datagen.zipf_buffer(s)
    k, r, l, _, N, C = w.params.astuple()
    check_roundtrip(lr, w.syms, 256, k, r, l, N, C)


# sweep points (alphabet, distribution, k, (r, l), N), at 64 MiB of symbol
# bytes, with 16 KiB chunks
SWEEP = [(2, "dominant", 11, (8, 23), 64), (16, "zipf1.1", 15, (16, 16), 32),
         (256, "near_uniform", 11, (16, 16), 64), (256, "zipf1.1", 15, (8, 23), 32),
         (4096, "dominant", 15, (16, 16), 64), (4096, "near_uniform", 15, (8, 23), 64)]


@pytest.mark.parametrize("pt", SWEEP, ids=[f"a{p[0]}-{p[1]}-k{p[2]}-r{p[3][0]}-N{p[4]}" for p in SWEEP])
def test_sweep_point_64MiB_plain_and_batched(lr, pt):
    import torch
    alphabet, dist, k, (r, l), N = pt
    syms = datagen.sweep_data(alphabet, dist)[0]
    w = syms.dtype.itemsize
    C = 16384 // w
    table, ref = check_roundtrip(lr, syms, alphabet, k, r, l, N, C)
    # the batched persistent kernel decodes the same container
    params = lr.rans_params.make(k, r, l, w, N, 0)
    d_in = torch.from_numpy(ref).cuda()
    out = torch.zeros(syms.size * w, dtype=torch.uint8, device="cuda")
    lens = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    jobs = lr.make_jobs([(table, d_in, ref.size, out, syms.size * w, int(lens.data_ptr()),
                          int(st.data_ptr()))])
    lr.rans_decode_batch(jobs, 1, params)
    torch.cuda.synchronize()
    assert int(st[0]) == 0 and int(lens[0]) == syms.size
    assert (out.cpu().numpy().view(syms.dtype) == syms).all()


def test_uneven_streams_one_batched_launch(lr):
    """192 streams from the batched workload's generator (1 KiB .. 4 MiB,
    Dirichlet tables), encoded and decoded in one batched call each."""
    import torch
    from test_gpu_batch import run_decode_batch, run_encode_batch
    data = datagen.dirichlet_streams(nstreams=192, seed=4001)
    k, r, l, C = 14, 16, 16, 8192
    tables, outs, st, lens = run_encode_batch(lr, data, k, r, l, C)
    assert (st == 0).all()
    for i, (s, _) in enumerate(data):
        ref = oracle.encode(oracle.quantize(datagen.counts(s, 256), k), s, k, r, l, 64, C,
                            threads=THREADS)
        assert outs[i].size == ref.size and (outs[i] == ref).all(), (i, first_diff(outs[i], ref))
    dec, st2, n2 = run_decode_batch(lr, tables, outs, [s.size for s, _ in data], k, r, l)
    assert (st2 == 0).all()
    for i, (s, _) in enumerate(data):
        assert n2[i] == s.size and (dec[i] == s).all(), i
    torch.cuda.synchronize()


def test_serving_requests_at_full_size_range(lr):
    """40 requests from the serving workload's distribution (4 KiB .. 64 MiB),
    replayed with Poisson arrivals under the 8 GiB budget: every encode result
    equals the oracle's container, every decode result the input."""
    import torch
    from test_gpu_serve import device_bytes
    K, R, L, W, N, C = 14, 16, 16, 1, 64, 65536
    params = lr.rans_params.make(K, R, L, W, N, C)
    reqs = datagen.serving_requests(nreq=40, seed=5201)
    staged, want = [], []
    for q in reqs:
        syms = datagen.request_data(q, seed=5201)
        counts = datagen.counts(syms, 256)
        table = lr.rans_tables_build(counts, K)
        ref = oracle.encode(oracle.quantize(counts, K), syms, K, R, L, N, C, threads=THREADS)
        if q["op"] == "encode":
            d = torch.from_numpy(syms).cuda()
            staged.append((lr.RANS_OP_ENCODE, table, d, syms.size, lr.rans_encode_bound(syms.size, params)))
            want.append(ref)
        else:
            d = torch.from_numpy(ref).cuda()
            staged.append((lr.RANS_OP_DECODE, table, d, ref.size, syms.size))
            want.append(syms)
    rng = np.random.Generator(np.random.PCG64(11))
    arrivals = np.cumsum(rng.exponential(200.0, len(staged)))
    srv = lr.rans_server_create(8 << 30, 4, 64, params)
    try:
        res, _ = lr.rans_server_replay(srv, [s + (float(t),) for s, t in zip(staged, arrivals)],
                                       keep_outputs=True)
        for c, ref in zip(res, want):
            assert c.status == 0 and c.out_len == ref.size
            got = device_bytes(c.d_out, c.out_len)
            assert (got == ref).all()
            lr.rans_server_release(srv, c.id)
    finally:
        lr.rans_server_destroy(srv)


@pytest.mark.parametrize("s", datagen.ZIPF_S)
def test_prefix_family_256MiB(lr, s):
    """The prefix-code family at the round-trip size: the GPU container equals
    the oracle's (its instrumented-decoder multiplexer) and decodes back."""
    import torch
    from rans_util import dev
    w = datagen.zipf_buffer(s)
    k, _, _, W, N, C = w.params.astuple()
    f = oracle.quantize(w.counts, k)
    table = lr.rans_tables_build(w.counts, k)
    ref = oracle.encode(f, w.syms, k, 16, 16, N, C, threads=THREADS, coder="prefix")
    p = lr.rans_params.make(k, 16, 16, W, N, C)
    cap = lr.rans_encode_bound(w.syms.size, p) + 4096
    d_out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    olen = lr.rans_pfx_encode(table, p, dev(w.syms), w.syms.size, d_out, cap)
    got = d_out[:olen].cpu().numpy()
    assert got.size == ref.size and (got == ref).all(), first_diff(got, ref)
    dec = gpu_decode(lr, table, ref, w.syms.size, 1)
    assert (dec == w.syms).all()


def test_escape_64MiB_laplace(lr):
    """Escape coding at the escape workload's size: 2^25 zigzag Laplace
    values, 1024-symbol table, about 18% escaped."""
    rng = np.random.Generator(np.random.PCG64(7001))
    v = datagen.sample(datagen.laplace_u16_probs(300.0), 1 << 25, rng, np.uint16)
    T = 1024
    counts = np.bincount(np.minimum(v, T - 1), minlength=T).astype(np.uint64)
    f = oracle.quantize(counts, 15)
    table = lr.rans_tables_build(counts, 15)
    for r, l in [(16, 16), (8, 23)]:
        ref = oracle.encode(f, v, 15, r, l, 64, 32768, threads=THREADS, escape=True)
        got = gpu_encode(lr, table, (15, r, l, 2, 64, 32768, "df", True), v)
        assert got.size == ref.size and (got == ref).all(), first_diff(got, ref)
        assert (gpu_decode(lr, table, ref, v.size, 2) == v).all()


def test_lookup_decode_256MiB(lr):
    """The fused lookup decode at the dequantisation workload's size: every
    output element equals lut[the oracle's decoded symbol]."""
    import torch
    from rans_util import dev
    rng = np.random.Generator(np.random.PCG64(6001))
    syms = datagen.sample(datagen.gaussian_codes_probs(256, 24.0), 1 << 28, rng)
    counts = datagen.counts(syms, 256)
    f = oracle.quantize(counts, 14)
    table = lr.rans_tables_build(counts, 14)
    ref = oracle.encode(f, syms, 14, 16, 16, 64, 65536, threads=THREADS)
    lut = ((np.arange(256, dtype=np.int64) - 128) * 977 % 65536).astype(np.uint16)
    want = lut[oracle.decode(f, ref, threads=THREADS)]
    d_out = torch.empty(syms.size * 2, dtype=torch.uint8, device="cuda")
    n = lr.rans_decode_lut(table, dev(ref), ref.size, dev(lut), 2, d_out, syms.size)
    assert n == syms.size
    got = d_out.cpu().numpy().view(np.uint16)
    assert (got == want).all(), first_diff(got.view(np.uint8), want.view(np.uint8))
