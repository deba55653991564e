"""GPU parity at the workloads' real sizes (through the C ABI).

The containers the GPU writes are compared byte for byte with the oracle's
and the GPU decodes the oracle's containers back to the input: the 1 MiB
four-coder stream in one chunk, the three 256 MiB Zipf buffers, every one of
the 84 feasible 64 MiB points of the radix/precision sweep (batched and
plain paths, in the configuration the benchmark times), the 4096 uneven
streams of the batched workload in one batched launch each way, and the
1000 requests of the serving workload through one server.
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


def tuned(lr, tmp_path, jobs, njobs, base):
    """The autotuner's choice for these jobs from the tuning results that ship
    with the library (the configuration bench.py times); a copy of the cache
    is used, so a miss tunes without touching the shipped file."""
    import os
    import shutil
    src = os.path.join(os.path.dirname(lr.__file__), "tune_mi355x.txt")
    cache = str(tmp_path / "tune.txt")
    if os.path.exists(src):
        shutil.copy(src, cache)
    return lr.rans_autotune_batch(jobs, njobs, base, cache)


def sweep_groups():
    groups = {}
    for p in datagen.sweep_points():
        if p["feasible"]:
            groups.setdefault((p["k"], p["r"], p["l"], p["w"], p["N"]), []).append(p)
    return sorted(groups.items())


SWEEP_GROUPS = sweep_groups()


@pytest.mark.parametrize("group", SWEEP_GROUPS, ids=[f"k{g[0][0]}-r{g[0][1]}-w{g[0][3]}-N{g[0][4]}"
                                                     for g in SWEEP_GROUPS])
def test_sweep_group_64MiB_every_point(lr, group, tmp_path):
    """Every feasible point of the radix/precision sweep (84 in 12 groups
    sharing k, r, l, w, N; 64 MiB of symbol bytes each, its own table), in
    the configuration bench.py times: one batched encode of the group at the
    tuned chunk size and launch shape writes the oracle's containers byte for
    byte; the plain encoder writes them too; the plain decoder and one
    batched decode of the group return every input from the oracle's
    containers."""
    import torch
    from rans_util import dev
    (k, r, l, w, N), pts = group
    data = [datagen.sweep_data(p["alphabet"], p["dist"])[0] for p in pts]
    counts = [datagen.counts(x, p["alphabet"]) for p, x in zip(pts, data)]
    tables = [lr.rans_tables_build(c, k) for c in counts]
    d_in = [dev(x) for x in data]
    sizes = [x.nbytes for x in data]
    jobs = lr.make_jobs((tables[i], d_in[i], sizes[i], 0, 0, 0, 0) for i in range(len(pts)))
    tune = tuned(lr, tmp_path, jobs, len(pts), lr.rans_params.make(k, r, l, w, N, 65536 // w))
    C = int(tune["chunk_syms"])
    assert int(tune["interleave"]) == N
    print(f"[sweep-group] k={k} r={r} w={w} N={N} C={C} shape={tune['waves_per_group']},"
          f"{tune['groups_per_cu']},{tune['table_layout']}", flush=True)
    params = lr.rans_params.make(k, r, l, w, N, C)
    refs = [oracle.encode(oracle.quantize(c, k), x, k, r, l, N, C, threads=THREADS)
            for c, x in zip(counts, data)]
    caps = [lr.rans_encode_bound(x.size, params) for x in data]
    d_cont = [torch.full((cap,), 0xA5, dtype=torch.uint8, device="cuda") for cap in caps]
    lens = torch.zeros(len(pts), dtype=torch.int64, device="cuda")
    st = torch.full((len(pts),), 99, dtype=torch.int32, device="cuda")
    enc = lr.make_jobs((tables[i], d_in[i], sizes[i], d_cont[i], caps[i], int(lens.data_ptr()) + 8 * i,
                        int(st.data_ptr()) + 4 * i) for i in range(len(pts)))
    lr.rans_encode_batch(enc, len(pts), params)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all(), st.tolist()
    for i, ref in enumerate(refs):
        got = d_cont[i][: int(lens[i])].cpu().numpy()
        assert got.size == ref.size and (got == ref).all(), (i, first_diff(got, ref))
        plain = gpu_encode(lr, tables[i], (k, r, l, w, N, C), data[i])
        assert plain.size == ref.size and (plain == ref).all(), (i, "plain", first_diff(plain, ref))
        dec = gpu_decode(lr, tables[i], ref, data[i].size, w)
        assert (dec.view(data[i].dtype) == data[i]).all(), (i, "plain decode")
    # one batched decode of the oracle's containers
    d_ref = [dev(ref) for ref in refs]
    d_out = [torch.zeros(n, dtype=torch.uint8, device="cuda") for n in sizes]
    st.fill_(99)
    dj = lr.make_jobs((tables[i], d_ref[i], refs[i].size, d_out[i], sizes[i], int(lens.data_ptr()) + 8 * i,
                       int(st.data_ptr()) + 4 * i) for i in range(len(pts)))
    lr.rans_decode_batch(dj, len(pts), params)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all(), st.tolist()
    for i, x in enumerate(data):
        assert int(lens[i]) == x.size
        assert (d_out[i].cpu().numpy().view(x.dtype) == x).all(), (i, "batched decode")


def test_4096_uneven_streams_one_batched_launch(lr, tmp_path):
    """The batched workload at full size: 4096 streams of 2^U(10,22) bytes
    (about 2 GiB) with Dirichlet tables, at the tuned interleave factor, chunk
    size and launch shape (as bench.py times them): one batched encode writes
    every stream's oracle container byte for byte, one batched decode of the
    oracle's containers returns every stream."""
    import torch
    from test_gpu_batch import Pool
    k, r, l = 14, 16, 16
    data = datagen.dirichlet_streams(nstreams=4096, seed=4001)
    sizes = [s.size for s, _ in data]
    # containers of any tuned shape fit the 64-coder, 4096-symbol-chunk bound
    bound = sum(lr.rans_encode_bound(n, lr.rans_params.make(k, r, l, 1, 64, 4096)) for n in sizes)
    pool = Pool(2 * sum(sizes) + 2 * bound + 4 * 256 * len(data))
    tables = [lr.rans_tables_build(datagen.counts(s, 256), k) for s, _ in data]
    d_in = []
    for s, _ in data:
        a = pool.take(s.size)
        pool.put(a, s)
        d_in.append(a)
    jobs = lr.make_jobs((tables[i], d_in[i], sizes[i], 0, 0, 0, 0) for i in range(len(data)))
    tune = tuned(lr, tmp_path, jobs, len(data), lr.rans_params.make(k, r, l, 1, 0, 65536))
    N, C = int(tune["interleave"]), int(tune["chunk_syms"])
    print(f"[4096-streams] N={N} C={C}", flush=True)
    params = lr.rans_params.make(k, r, l, 1, N, C)
    caps = [lr.rans_encode_bound(n, params) for n in sizes]
    d_cont = [pool.take(c) for c in caps]
    lens = torch.zeros(len(data), dtype=torch.int64, device="cuda")
    st = torch.full((len(data),), 99, dtype=torch.int32, device="cuda")
    enc = lr.make_jobs((tables[i], d_in[i], sizes[i], d_cont[i], caps[i], int(lens.data_ptr()) + 8 * i,
                        int(st.data_ptr()) + 4 * i) for i in range(len(data)))
    lr.rans_encode_batch(enc, len(data), params)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    clen = lens.cpu().numpy()
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(THREADS) as ex:  # one oracle call per stream, streams in parallel
        refs = list(ex.map(lambda sp: oracle.encode(oracle.quantize(datagen.counts(sp[0], 256), k), sp[0],
                                                    k, r, l, N, C), data))
    for i, ref in enumerate(refs):
        got = pool.get(d_cont[i], int(clen[i]))
        assert got.size == ref.size and (got == ref).all(), (i, first_diff(got, ref))
    d_ref, d_out = [], []
    for ref, n in zip(refs, sizes):
        a = pool.take(ref.size)
        pool.put(a, ref)
        d_ref.append(a)
        d_out.append(pool.take(n))
    st.fill_(99)
    dj = lr.make_jobs((tables[i], d_ref[i], refs[i].size, d_out[i], sizes[i], int(lens.data_ptr()) + 8 * i,
                       int(st.data_ptr()) + 4 * i) for i in range(len(data)))
    lr.rans_decode_batch(dj, len(data), params)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    n2 = lens.cpu().numpy()
    for i, (s, _) in enumerate(data):
        assert n2[i] == s.size and (pool.get(d_out[i], s.size) == s).all(), i


def test_serving_1000_requests_full_size_range(lr):
    """The serving workload at full size, as bench.py runs it: 1000 requests
    of 2^U(12,26) bytes (encode/decode 50/50, Zipf tables; about 6.8 GiB),
    one server with the 8 GiB budget, 4 streams and up to 64 requests per
    launch.  All requests arrive at once; each output is checked as soon as it
    completes (every encode result is the oracle's container, every decode
    result the input) and released, so requests keep being admitted as
    memory frees up.  The server's counters show launches of several
    requests and several streams busy at once, and the budget held.  Then the
    same requests under Poisson arrivals complete with the oracle's lengths."""
    import torch
    from test_gpu_serve import device_bytes
    K, R, L, W, N, C = 14, 16, 16, 1, 64, 65536
    params = lr.rans_params.make(K, R, L, W, N, C)
    reqs = datagen.serving_requests(nreq=1000, seed=5001)
    staged, want = [], []
    for q, syms in zip(reqs, datagen.requests_data(reqs, seed=5001)):
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
    print(f"[serving] {len(staged)} requests staged", flush=True)
    srv = lr.rans_server_create(8 << 30, 4, 64, params)
    try:
        ids = {}
        for i, (op, table, d, inl, cap) in enumerate(staged):
            ids[lr.rans_server_submit(srv, op, table, d, inl, cap)] = i
        done = 0
        while done < len(staged):
            for c in lr.rans_server_poll(srv, keep_outputs=True, max_out=64):
                i = ids[c.id]
                assert c.status == 0 and c.out_len == want[i].size, (i, c.status)
                assert (device_bytes(c.d_out, c.out_len) == want[i]).all(), i
                lr.rans_server_release(srv, c.id)
                done += 1
        st = lr.rans_server_stats(srv)
        print(f"[serving] {st}", flush=True)
        assert st["peak"] <= st["budget"] and st["used"] == st["fixed"]
        assert st["max_launch_requests"] > 1 and st["multi_request_launches"] > 0
        assert st["peak_busy_streams"] > 1
        rng = np.random.Generator(np.random.PCG64(11))
        arrivals = np.cumsum(rng.exponential(5.0, len(staged)))
        res, _ = lr.rans_server_replay(srv, [s + (float(t),) for s, t in zip(staged, arrivals)])
        for c, ref in zip(res, want):
            assert c.status == 0 and c.out_len == ref.size
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
