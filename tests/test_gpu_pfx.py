"""GPU parity of the prefix-code family multiplexed as Section 4 describes.

rans_pfx_encode must produce the oracle's container byte for byte (the
oracle builds it by running an instrumented decoder over per-coder streams);
rans_decode must return the input from the oracle's container.
"""
import zlib

import numpy as np
import pytest

import datagen
import oracle
from rans_util import dev, first_diff, gpu_decode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1402_3392_amd as m
    return m


def pfx_encode(lr, table, params, syms):
    import torch
    p = lr.rans_params.make(*params)
    cap = lr.rans_encode_bound(syms.size, p) + 4096
    d_out = torch.full((cap + 64,), 0xA5, dtype=torch.uint8, device="cuda")
    olen = lr.rans_pfx_encode(table, p, dev(syms), syms.size, d_out, cap)
    torch.cuda.synchronize()
    return d_out[:olen].cpu().numpy()


def make_syms(alphabet, dist, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    if dist == "zipf":
        p = datagen.zipf_probs(alphabet, 1.1)
    elif dist == "near_uniform":
        p = datagen.near_uniform_probs(alphabet, rng)
    else:
        p = datagen.dominant_probs(alphabet, 0.995)
    return datagen.sample(p, n, rng, np.uint8 if alphabet <= 256 else np.uint16)


# (alphabet, dist, k, N, C, n)
CASES = [
    (256, "zipf", 12, 64, 4096, 200_003),
    (256, "zipf", 14, 64, 65536, 3 * 65536 + 12345),
    (256, "near_uniform", 15, 64, 8192, 100_001),
    (256, "dominant", 12, 64, 4096, 150_000),
    (256, "zipf", 11, 32, 8192, 150_001),
    (4096, "near_uniform", 15, 64, 8192, 70_001),
    (4096, "zipf", 15, 32, 2048, 2 * 2048 + 15 * 32 + 5),
    (256, "zipf", 12, 64, 1024, 5 * 1024 + 992),
    (16, "zipf", 10, 64, 16, 1_001),
    (2, "dominant", 15, 32, 4096, 300_000),
]


def ids(c):
    return f"a{c[0]}-{c[1]}-k{c[2]}-N{c[3]}-C{c[4]}-n{c[5]}"


@pytest.mark.parametrize("case", CASES, ids=[ids(c) for c in CASES])
def test_pfx_matches_oracle(lr, case):
    alphabet, dist, k, N, C, n = case
    syms = make_syms(alphabet, dist, n, zlib.crc32(ids(case).encode()))
    w = syms.dtype.itemsize
    counts = datagen.counts(syms, alphabet)
    f = oracle.quantize(counts, k)
    table = lr.rans_tables_build(counts, k)
    print(f"[pfx] {ids(case)}", flush=True)
    ref = oracle.encode(f, syms, k, 16, 16, N, C, threads=4, coder="prefix")
    assert ref[9] == 4
    got = pfx_encode(lr, table, (k, 16, 16, w, N, C), syms)
    assert got.size == ref.size and (got == ref).all(), first_diff(got, ref)
    dec = gpu_decode(lr, table, ref, n, w)
    assert (dec == syms).all(), first_diff(dec.view(np.uint8), syms.view(np.uint8))


def test_pfx_single_symbol_and_tiny(lr):
    for n in (1, 63, 64, 65, 1000):
        syms = np.zeros(n, np.uint8)
        counts = np.zeros(256, np.uint64)
        counts[0] = n
        f = oracle.quantize(counts, 12)
        table = lr.rans_tables_build(counts, 12)
        ref = oracle.encode(f, syms, 12, 16, 16, 64, 4096, coder="prefix")
        got = pfx_encode(lr, table, (12, 16, 16, 1, 64, 4096), syms)
        assert (got == ref).all(), (n, first_diff(got, ref))
        assert (gpu_decode(lr, table, ref, n, 1) == syms).all()


def test_pfx_errors(lr):
    import torch
    syms = make_syms(256, "zipf", 50_000, 95)
    counts = datagen.counts(syms, 256)
    table = lr.rans_tables_build(counts, 12)
    d_out = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")

    def code(fn):
        try:
            fn()
            return 0
        except lr.RansError as e:
            return e.code

    for bad in [(12, 8, 23, 1, 64, 4096), (12, 16, 16, 1, 4, 4096), (12, 16, 16, 1, 64, 4100)]:
        assert code(lambda: lr.rans_pfx_encode(table, lr.rans_params.make(*bad), dev(syms),
                                               syms.size, d_out, d_out.numel())) == lr.RANS_EINVAL, bad
    c2 = counts.copy()
    c2[syms[7]] = 0  # a symbol the code cannot express
    t2 = lr.rans_tables_build(c2, 12)
    assert code(lambda: lr.rans_pfx_encode(t2, lr.rans_params.make(12, 16, 16, 1, 64, 4096),
                                           dev(syms), syms.size, d_out, d_out.numel())) == lr.RANS_ENOSYM
    f = oracle.quantize(counts, 12)
    ref = oracle.encode(f, syms, 12, 16, 16, 64, 4096, coder="prefix")
    bad = ref.copy()
    off = int(np.frombuffer(bad[48:56].tobytes(), "<u8")[0])
    bad[off + 4] ^= 1  # coder 1's bit count
    d_dec = torch.empty(syms.size + 64, dtype=torch.uint8, device="cuda")
    assert code(lambda: lr.rans_decode(table, dev(bad), bad.size, d_dec, syms.size)) == lr.RANS_ECORRUPT
    # a container of the family does not decode on the batched path
    lens = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    jobs = lr.make_jobs([(table, dev(ref), ref.size, d_dec, syms.size, int(lens.data_ptr()),
                          int(st.data_ptr()))])
    lr.rans_decode_batch(jobs, 1, lr.rans_params.make(12, 16, 16, 1, 64, 0))
    torch.cuda.synchronize()
    assert int(st[0]) in (lr.RANS_EINVAL, lr.RANS_ECORRUPT)
