"""GPU parity of escape coding with raw digits (Section 3), through the C ABI.

16-bit values are coded with a table of the frequent ones whose last symbol
is an escape; the other values travel as raw digits in the interleaved
stream.  The GPU container must equal the oracle's byte for byte, and the
GPU must decode the oracle's container to the input.
"""
import zlib

import numpy as np
import pytest

import datagen
import oracle
from rans_util import dev, first_diff, gpu_decode, gpu_encode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1402_3392_amd as m
    return m


def make_values(table, p_wild, n, seed, zero=()):
    """Values drawn from Zipf(1.1) over table - 1 symbols, a fraction p_wild
    replaced by uniform 16-bit values; counts over the table (the escape
    counts every value at or above table - 1), with `zero` forced to 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = datagen.sample(datagen.zipf_probs(table - 1, 1.1), n, rng, np.uint16)
    wild = rng.random(n) < p_wild
    v[wild] = rng.integers(0, 65536, int(wild.sum()))
    counts = np.bincount(np.minimum(v, table - 1), minlength=table).astype(np.uint64)
    counts[table - 1] += 1
    for z in zero:
        counts[z] = 0
    return v, counts


# (table, p_wild, k, r, l, N, C, n)
CASES = [
    (256, 0.05, 12, 16, 16, 64, 4096, 200_003),
    (256, 0.30, 14, 16, 16, 64, 8192, 150_001),
    (256, 0.90, 12, 16, 16, 32, 2048, 3 * 2048 + 31 * 32 + 17),
    (4096, 0.05, 15, 16, 16, 64, 8192, 100_001),
    (256, 0.05, 12, 8, 23, 64, 4096, 200_003),
    (256, 0.50, 11, 8, 23, 32, 8192, 100_000),
    (4096, 0.20, 15, 8, 23, 64, 1024, 7 * 1024 + 999),
    (256, 0.95, 12, 8, 23, 64, 4096, 50_000),
    # generic kernels (N < 32)
    (256, 0.10, 12, 16, 16, 16, 1000, 20_011),
    (256, 0.10, 12, 8, 23, 4, 999, 20_011),
    (4096, 0.10, 15, 8, 22, 1, 0, 20_011),
]


def ids(c):
    return f"t{c[0]}-w{c[1]}-k{c[2]}-r{c[3]}-l{c[4]}-N{c[5]}-C{c[6]}-n{c[7]}"


@pytest.mark.parametrize("case", CASES, ids=[ids(c) for c in CASES])
def test_escape_matches_oracle(lr, case):
    table, p_wild, k, r, l, N, C, n = case
    v, counts = make_values(table, p_wild, n, zlib.crc32(ids(case).encode()), zero=(2, 5))
    f = oracle.quantize(counts, k)
    t = lr.rans_tables_build(counts, k)
    print(f"[escape] {ids(case)}", flush=True)
    ref = oracle.encode(f, v, k, r, l, N, C, threads=4, escape=True)
    assert ref[9] == 2
    got = gpu_encode(lr, t, (k, r, l, 2, N, C, "df", True), v)
    assert got.size == ref.size and (got == ref).all(), first_diff(got, ref)
    dec = gpu_decode(lr, t, ref, n, 2)
    assert (dec == v).all(), first_diff(dec.view(np.uint8), v.view(np.uint8))


@pytest.mark.parametrize("r,l,N", [(16, 16, 64), (8, 23, 32), (16, 16, 8)])
def test_one_symbol_table_stores_raw_values(lr, r, l, N):
    """Every value escapes and nothing renormalises: the payload is the
    values themselves (the oracle's closed form, checked by its pins)."""
    rng = np.random.Generator(np.random.PCG64(91))
    v = rng.integers(0, 65536, 30_001).astype(np.uint16)
    counts = np.array([1], np.uint64)
    f = oracle.quantize(counts, 10)
    t = lr.rans_tables_build(counts, 10)
    ref = oracle.encode(f, v, 10, r, l, N, 4096, escape=True)
    got = gpu_encode(lr, t, (10, r, l, 2, N, 4096, "df", True), v)
    assert (got == ref).all(), first_diff(got, ref)
    assert (gpu_decode(lr, t, ref, v.size, 2) == v).all()


def test_escape_errors(lr):
    import torch
    v, counts = make_values(256, 0.2, 20_000, 92)
    counts[255] = 0  # the escape itself has frequency 0: escaped values cannot be coded
    counts[0] += 1
    t = lr.rans_tables_build(counts, 12)
    p = lr.rans_params.make(12, 16, 16, 2, 64, 4096, "df", True)
    cap = lr.rans_encode_bound(v.size, p)
    d_out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    with pytest.raises(lr.RansError) as e:
        lr.rans_encode(t, p, dev(v), v.size, d_out, cap)
    assert e.value.code == lr.RANS_ENOSYM
    # 8-bit symbols, breadth-first order: not defined with escapes
    assert lr.rans_params_check(lr.rans_params.make(12, 16, 16, 1, 64, 4096, "df", True)) \
        == lr.RANS_EINVAL
    assert lr.rans_params_check(lr.rans_params.make(12, 8, 23, 2, 64, 4096, "bf", True)) \
        == lr.RANS_EINVAL
    # the batched entry points and the fused lookup decode reject escape coding
    v2, counts2 = make_values(256, 0.2, 20_000, 93)
    t2 = lr.rans_tables_build(counts2, 12)
    f2 = oracle.quantize(counts2, 12)
    cont = oracle.encode(f2, v2, 12, 16, 16, 64, 4096, escape=True)
    lens = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    d_dec = torch.empty(v2.size * 2, dtype=torch.uint8, device="cuda")
    jobs = lr.make_jobs([(t2, dev(cont), cont.size, d_dec, v2.size * 2, int(lens.data_ptr()),
                          int(st.data_ptr()))])
    with pytest.raises(lr.RansError) as e:
        lr.rans_decode_batch(jobs, 1, p)
    assert e.value.code == lr.RANS_EINVAL
    lut = np.zeros(256, np.uint16)
    with pytest.raises(lr.RansError) as e:
        lr.rans_decode_lut(t2, dev(cont), cont.size, dev(lut), 2, d_dec, v2.size)
    assert e.value.code == lr.RANS_EINVAL
    # a flipped raw digit changes exactly its value (raw digits carry no check)
    onesym = np.array([1], np.uint64)
    t1 = lr.rans_tables_build(onesym, 10)
    v3 = np.arange(5000, dtype=np.uint16) * 13
    c3 = oracle.encode(oracle.quantize(onesym, 10), v3, 10, 16, 16, 64, 4096, escape=True)
    off = int(np.frombuffer(c3[32:40].tobytes(), "<u8")[0])
    c3[off + 4 * 64 + 2 * 777] ^= 0x40
    out = gpu_decode(lr, t1, c3, v3.size, 2)
    assert np.flatnonzero(out != v3).tolist() == [777]
