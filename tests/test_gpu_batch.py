"""GPU parity of the batched entry points (persistent kernel + HIP graph).

Every job of a batch is checked against the oracle byte for byte (encode)
and symbol for symbol (decode); a failing job must fail alone; graph replays
with new data in the same shapes must stay exact.
"""
import numpy as np
import pytest

import datagen
import oracle
from rans_util import first_diff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lr():
    import torch
    assert torch.cuda.is_available()
    import paper_1402_3392_amd as m
    m.rans_batch_set_config(16, 1, 0, 1)
    return m


def streams(nstreams, seed, lo=10, hi=17):
    """Uint8 streams of log-uniform length with Dirichlet(alpha) tables."""
    return datagen.dirichlet_streams(nstreams=nstreams, lo_log2=lo, hi_log2=hi, seed=seed)


class Pool:
    """Carves 256-byte aligned pieces out of one device allocation."""

    def __init__(self, nbytes):
        import torch
        self.buf = torch.zeros(nbytes + 4096, dtype=torch.uint8, device="cuda")
        self.base = int(self.buf.data_ptr())
        self.off = 0

    def take(self, nbytes):
        a = self.base + self.off
        self.off += (max(nbytes, 1) + 255) // 256 * 256
        assert self.off <= self.buf.numel()
        return a

    def put(self, addr, arr):
        raw = np.ascontiguousarray(arr).view(np.uint8).reshape(-1)
        import torch
        o = addr - self.base
        self.buf[o:o + raw.size].copy_(torch.from_numpy(raw.copy()))

    def get(self, addr, nbytes):
        o = addr - self.base
        return self.buf[o:o + nbytes].cpu().numpy()


def run_encode_batch(lr, data, k, r, l, C, cap_override=None, N=64, order="df", counts=None):
    import torch
    params = lr.rans_params.make(k, r, l, 1, N, C, order)
    tables, specs = [], []
    total = sum(s.size for s, _ in data)
    pool = Pool(sum(lr.rans_encode_bound(s.size, params) + s.size + 1024 for s, _ in data))
    lens = torch.zeros(len(data), dtype=torch.int64, device="cuda")
    st = torch.full((len(data),), 99, dtype=torch.int32, device="cuda")
    for i, (s, _) in enumerate(data):
        t = lr.rans_tables_build(datagen.counts(s, 256) if counts is None else counts[i], k)
        tables.append(t)
        din = pool.take(s.size)
        pool.put(din, s)
        cap = lr.rans_encode_bound(s.size, params)
        if cap_override and i in cap_override:
            cap = cap_override[i]
        dout = pool.take(cap)
        specs.append((t, din, s.size, dout, cap, int(lens.data_ptr()) + 8 * i,
                      int(st.data_ptr()) + 4 * i))
    jobs = lr.make_jobs(specs)
    lr.rans_encode_batch(jobs, len(data), params)
    torch.cuda.synchronize()
    outs = [pool.get(specs[i][3], int(lens[i])) for i in range(len(data))]
    assert total > 0
    return tables, outs, st.cpu().numpy(), lens.cpu().numpy()


def run_decode_batch(lr, tables, containers, sizes, k, r, l, corrupt=None, N=64, order="df"):
    import torch
    params = lr.rans_params.make(k, r, l, 1, N, 0, order)
    pool = Pool(sum(c.size + n + 1024 for c, n in zip(containers, sizes)))
    lens = torch.zeros(len(containers), dtype=torch.int64, device="cuda")
    st = torch.full((len(containers),), 99, dtype=torch.int32, device="cuda")
    specs = []
    for i, (c, n) in enumerate(zip(containers, sizes)):
        din = pool.take(c.size)
        pool.put(din, c)
        dout = pool.take(n)
        specs.append((tables[i], din, c.size, dout, n, int(lens.data_ptr()) + 8 * i,
                      int(st.data_ptr()) + 4 * i))
    jobs = lr.make_jobs(specs)
    lr.rans_decode_batch(jobs, len(containers), params)
    torch.cuda.synchronize()
    outs = [pool.get(specs[i][3], sizes[i]) for i in range(len(containers))]
    return outs, st.cpu().numpy(), lens.cpu().numpy()


@pytest.mark.parametrize("k,r,l,C,N", [(14, 16, 16, 4096, 64), (14, 16, 16, 65536, 64),
                                       (12, 8, 23, 8192, 64), (14, 16, 16, 4096, 32),
                                       (12, 8, 23, 2048, 32)])
def test_batch_encode_decode_match_oracle(lr, k, r, l, C, N):
    data = streams(40, seed=4100 + k + r + N)
    tables, outs, st, lens = run_encode_batch(lr, data, k, r, l, C, N=N)
    assert (st == 0).all(), st
    refs = []
    for i, (s, _) in enumerate(data):
        f = oracle.quantize(datagen.counts(s, 256), k)
        ref = oracle.encode(f, s, k, r, l, N, C)
        refs.append(ref)
        assert outs[i].size == ref.size and (outs[i] == ref).all(), (i, first_diff(outs[i], ref))
    dec, st2, n2 = run_decode_batch(lr, tables, refs, [s.size for s, _ in data], k, r, l, N=N)
    assert (st2 == 0).all(), st2
    for i, (s, _) in enumerate(data):
        assert n2[i] == s.size
        assert (dec[i] == s).all(), i


def _zipf_stream(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return datagen.sample(datagen.zipf_probs(256, 1.1), n, rng, np.uint8)


@pytest.mark.parametrize("N", [64, 32])
def test_batch_edge_jobs(lr, N):
    """Jobs the batched encoder places specially: empty (a header-only
    container written by the planning kernel), one symbol, exactly 64 and 65
    chunks (the look-back's group level), a ragged last chunk; then the same
    batch with one job 16 bytes short of its container and an empty job
    with room for less than a header (RANS_ENOSPC for those two alone, the
    needed length reported)."""
    k, r, l, C = 12, 16, 16, 1024
    sizes = [0, 1, 64 * C, 65 * C, 3 * C + 17, 0, 5 * C]
    data = [(_zipf_stream(n, 4700 + i), None) for i, n in enumerate(sizes)]
    counts = []
    for s, _ in data:
        c = datagen.counts(s, 256)
        c[0] += 1  # a non-empty histogram for the empty jobs
        counts.append(c)
    refs = [oracle.encode(oracle.quantize(c, k), s, k, r, l, N, C) for c, (s, _) in zip(counts, data)]
    assert refs[0].size == 32 and refs[5].size == 32
    tables, outs, st, lens = run_encode_batch(lr, data, k, r, l, C, N=N, counts=counts)
    assert (st == 0).all(), st
    for i in range(len(sizes)):
        assert lens[i] == refs[i].size and (outs[i] == refs[i]).all(), (i, first_diff(outs[i], refs[i]))
    dec, st2, n2 = run_decode_batch(lr, tables, refs, sizes, k, r, l, N=N)
    assert (st2 == 0).all(), st2
    for i, (s, _) in enumerate(data):
        assert n2[i] == s.size and (dec[i][:s.size] == s).all(), i
    short = {3: refs[3].size - 16, 5: 16}
    _, _, st3, lens3 = run_encode_batch(lr, data, k, r, l, C, cap_override=short, N=N, counts=counts)
    assert st3[3] == lr.RANS_ENOSPC and st3[5] == lr.RANS_ENOSPC, st3
    assert lens3[3] == refs[3].size and lens3[5] == 32
    assert (np.delete(st3, [3, 5]) == 0).all(), st3


@pytest.mark.parametrize("N,C,layout", [(64, 8192, 1), (64, 2048, 2), (32, 4096, 3), (32, 1024, 0)])
def test_batch_breadth_first_match_oracle(lr, N, C, layout):
    """Breadth-first containers (Section 5) through the batched kernels, on
    every decoder table layout; a depth-first decode of them fails per job."""
    lr.rans_batch_set_config(16, 1, layout, 1)
    try:
        k, r, l = 12, 8, 23
        data = streams(24, seed=4600 + N + layout)
        tables, outs, st, _ = run_encode_batch(lr, data, k, r, l, C, N=N, order="bf")
        assert (st == 0).all(), st
        refs = []
        for i, (s, _) in enumerate(data):
            ref = oracle.encode(oracle.quantize(datagen.counts(s, 256), k), s, k, r, l, N, C,
                                order="bf")
            refs.append(ref)
            assert outs[i].size == ref.size and (outs[i] == ref).all(), (i, first_diff(outs[i], ref))
        sizes = [s.size for s, _ in data]
        dec, st2, n2 = run_decode_batch(lr, tables, refs, sizes, k, r, l, N=N, order="bf")
        assert (st2 == 0).all(), st2
        for i, (s, _) in enumerate(data):
            assert n2[i] == s.size and (dec[i] == s).all(), i
        _, st3, _ = run_decode_batch(lr, tables, refs, sizes, k, r, l, N=N, order="df")
        assert (st3 == lr.RANS_EINVAL).all(), st3
    finally:
        lr.rans_batch_set_config(16, 1, 0, 1)


def test_batch_failures_are_isolated(lr):
    k, r, l, C = 14, 16, 16, 4096
    data = streams(12, seed=4200)
    # job 3 gets a container capacity of 40 bytes: ENOSPC for it alone
    tables, outs, st, lens = run_encode_batch(lr, data, k, r, l, C, cap_override={3: 40})
    assert st[3] == lr.RANS_ENOSPC
    assert (np.delete(st, 3) == 0).all()
    refs = [oracle.encode(oracle.quantize(datagen.counts(s, 256), k), s, k, r, l, 64, C)
            for s, _ in data]
    for i in range(len(data)):
        if i != 3:
            assert (outs[i] == refs[i]).all()
    # job 5's container is corrupted, job 7's header claims another radix
    bad = [c.copy() for c in refs]
    first = int(np.frombuffer(bad[5][32:40].tobytes(), "<u8")[0])
    bad[5][first + 300] ^= 0x22
    bad[7][6] = 8
    dec, st2, _ = run_decode_batch(lr, tables, bad, [s.size for s, _ in data], k, r, l)
    assert st2[5] == lr.RANS_ECORRUPT
    assert st2[7] == lr.RANS_EINVAL
    for i, (s, _) in enumerate(data):
        if i not in (5, 7):
            assert st2[i] == 0 and (dec[i] == s).all(), i


@pytest.mark.parametrize("use_graph", [1, 0])
def test_batch_replays_stay_exact(lr, use_graph):
    """Same shapes, new data: the captured graph is replayed; every replay is
    checked, with host work and synchronisation in between."""
    lr.rans_batch_set_config(16, 1, 0, use_graph)
    try:
        k, r, l, C = 14, 16, 16, 4096
        for rep in range(3):
            data = streams(16, seed=4300 + rep, lo=12, hi=15)
            # equal lengths across replays keep the launch image identical
            data = [(s[: 1 << 12], p) for s, p in data]
            tables, outs, st, _ = run_encode_batch(lr, data, k, r, l, C)
            assert (st == 0).all()
            for i, (s, _) in enumerate(data):
                ref = oracle.encode(oracle.quantize(datagen.counts(s, 256), k), s, k, r, l, 64, C)
                assert (outs[i] == ref).all(), (rep, i)
            dec, st2, _ = run_decode_batch(lr, tables, outs, [s.size for s, _ in data], k, r, l)
            assert (st2 == 0).all()
            for i, (s, _) in enumerate(data):
                assert (dec[i] == s).all(), (rep, i)
    finally:
        lr.rans_batch_set_config(16, 1, 0, 1)


def test_batch_config_validation(lr):
    with pytest.raises(lr.RansError):
        lr.rans_batch_set_config(0, 1, 0, 1)
    with pytest.raises(lr.RansError):
        lr.rans_batch_set_config(16, 17, 0, 1)
    lr.rans_batch_set_config(8, 2, 2, 1)
    assert lr.rans_batch_get_config() == {"waves_per_group": 8, "groups_per_cu": 2,
                                          "table_layout": 2, "use_graph": 1}
    lr.rans_batch_set_config(16, 1, 0, 1)


@pytest.mark.parametrize("G,gpc,layout", [(4, 2, 0), (8, 2, 2), (16, 1, 1)])
def test_batch_launch_shapes(lr, G, gpc, layout):
    lr.rans_batch_set_config(G, gpc, layout, 1)
    try:
        k, r, l, C = 14, 16, 16, 8192
        data = streams(20, seed=4400 + G)
        tables, outs, st, _ = run_encode_batch(lr, data, k, r, l, C)
        assert (st == 0).all()
        dec, st2, _ = run_decode_batch(lr, tables, outs, [s.size for s, _ in data], k, r, l)
        assert (st2 == 0).all()
        for i, (s, _) in enumerate(data):
            ref = oracle.encode(oracle.quantize(datagen.counts(s, 256), k), s, k, r, l, 64, C)
            assert (outs[i] == ref).all() and (dec[i] == s).all(), i
    finally:
        lr.rans_batch_set_config(16, 1, 0, 1)


def test_autotune_result_is_valid_applied_and_cached(lr, tmp_path):
    import torch
    k, r, l = 14, 16, 16
    s, _ = streams(1, seed=4500, lo=20, hi=20.5)[0]
    table = lr.rans_tables_build(datagen.counts(s, 256), k)
    d = torch.from_numpy(s).cuda()
    cache = str(tmp_path / "tune.txt")
    base = lr.rans_params.make(k, r, l, 1, 64, 65536)  # N fixed at 64
    res = lr.rans_autotune(table, d, s.size, base, cache)
    assert res["chunk_syms"] in (65536, 32768, 16384, 8192, 4096)
    N = res["interleave"]
    assert N == 64 and res["lanes_per_stream"] == N and res["chunks_per_wave"] == 1
    assert res["waves_per_group"] in (16, 8, 4) and res["groups_per_cu"] in (1, 2, 4)
    assert res["table_layout"] in (1, 2, 3) and res["use_graph"] in (0, 1)
    assert res["encode_gbps"] > 0 and res["decode_gbps"] > 0
    cfg = lr.rans_batch_get_config()
    assert (cfg["waves_per_group"], cfg["groups_per_cu"], cfg["table_layout"], cfg["use_graph"]) == \
        (res["waves_per_group"], res["groups_per_cu"], res["table_layout"], res["use_graph"])
    lines = open(cache).read().splitlines()
    assert len(lines) == 1
    lr.rans_batch_set_config(16, 1, 0, 1)
    again = lr.rans_autotune(table, d, s.size, base, cache)  # a cache hit: same answer, no new line
    assert again["chunk_syms"] == res["chunk_syms"] and len(open(cache).read().splitlines()) == 1
    # the tuned shape codes bit-exactly
    C = res["chunk_syms"]
    tables, outs, st, _ = run_encode_batch(lr, [(s, None)], k, r, l, C, N=N)
    assert (st == 0).all()
    ref = oracle.encode(oracle.quantize(datagen.counts(s, 256), k), s, k, r, l, N, C)
    assert outs[0].size == ref.size and (outs[0] == ref).all()
    dec, st2, _ = run_decode_batch(lr, tables, outs, [s.size], k, r, l, N=N)
    assert (st2 == 0).all() and (dec[0] == s).all()
    lr.rans_batch_set_config(16, 1, 0, 1)


def test_batch_autotune_on_the_batch(lr, tmp_path):
    """The tuner times candidates on the whole batch; its choice is applied,
    cached, and codes the batch bit-exactly."""
    import torch
    k, r, l = 14, 16, 16
    data = streams(24, seed=4700, lo=10, hi=16)
    tables = [lr.rans_tables_build(datagen.counts(s, 256), k) for s, _ in data]
    pool = Pool(sum(s.size + 256 for s, _ in data))
    ins = []
    for s, _ in data:
        a = pool.take(s.size)
        pool.put(a, s)
        ins.append(a)
    jobs = lr.make_jobs((tables[i], ins[i], data[i][0].size, 0, 0, 0, 0) for i in range(len(data)))
    cache = str(tmp_path / "tune.txt")
    base = lr.rans_params.make(k, r, l, 1, 0, 65536)  # N searched over 32 and 64
    res = lr.rans_autotune_batch(jobs, len(data), base, cache)
    assert res["chunk_syms"] in (65536, 32768, 16384, 8192, 4096)
    N = res["interleave"]
    assert N in (32, 64) and res["lanes_per_stream"] == N and res["chunks_per_wave"] == 64 // N
    assert res["waves_per_group"] in (16, 8, 4) and res["groups_per_cu"] in (1, 2, 4)
    assert res["table_layout"] in (1, 2, 3) and res["decode_gbps"] > 0
    cfg = lr.rans_batch_get_config()
    assert (cfg["waves_per_group"], cfg["groups_per_cu"], cfg["table_layout"]) == \
        (res["waves_per_group"], res["groups_per_cu"], res["table_layout"])
    assert len(open(cache).read().splitlines()) == 1
    again = lr.rans_autotune_batch(jobs, len(data), base, cache)
    assert again["chunk_syms"] == res["chunk_syms"] and len(open(cache).read().splitlines()) == 1
    try:
        C = res["chunk_syms"]
        tabs, outs, st, _ = run_encode_batch(lr, data, k, r, l, C, N=N)
        assert (st == 0).all()
        for i, (s, _) in enumerate(data):
            ref = oracle.encode(oracle.quantize(datagen.counts(s, 256), k), s, k, r, l, N, C)
            assert (outs[i] == ref).all(), i
        dec, st2, _ = run_decode_batch(lr, tabs, outs, [s.size for s, _ in data], k, r, l, N=N)
        assert (st2 == 0).all() and all((dec[i] == s).all() for i, (s, _) in enumerate(data))
    finally:
        lr.rans_batch_set_config(16, 1, 0, 1)
    torch.cuda.synchronize()


@pytest.mark.parametrize("G", [16, 1])
def test_batch_decode_many_small_low_entropy_chunks(lr, G):
    """N = 32 chunks of 4096 bytes of a two-symbol source with p0 = 0.995
    cost about 170 bytes each (16 directory bytes, 128 of states, a few
    digits): more chunks per
    container byte than a 64-coder chunk can have.  A batch of such
    containers decodes every chunk of every job, with one wave per work item
    (G = 1: the most work items) too."""
    import torch
    k, r, l, N, C = 11, 16, 16, 32, 4096
    data = []
    for i in range(3):
        rng = np.random.Generator(np.random.PCG64(4800 + i))
        data.append(datagen.sample(datagen.dominant_probs(2, 0.995), (1 << 20) + 77 * i, rng))
    refs, tables = [], []
    for s in data:
        c = datagen.counts(s, 256)
        refs.append(oracle.encode(oracle.quantize(c, k), s, k, r, l, N, C))
        tables.append(lr.rans_tables_build(c, k))
    # more chunks than a 16 + 4 * 64 byte per chunk bound would allow
    for s, ref in zip(data, refs):
        assert (s.size + C - 1) // C > (ref.size - 32) // (16 + 4 * 64)
    cfg = lr.rans_batch_get_config()
    lr.rans_batch_set_config(G, 1, 0, 1)
    try:
        dec, st, n = run_decode_batch(lr, tables, refs, [s.size for s in data], k, r, l, N=N)
    finally:
        lr.rans_batch_set_config(cfg["waves_per_group"], cfg["groups_per_cu"], cfg["table_layout"],
                                 cfg["use_graph"])
    torch.cuda.synchronize()
    assert (st == 0).all(), st
    for i, s in enumerate(data):
        assert n[i] == s.size and (dec[i] == s).all(), i
