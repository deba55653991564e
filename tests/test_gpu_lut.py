"""GPU parity of the decode fused with a table-lookup consumer.

rans_decode_lut writes lut[symbol i] for every decoded symbol.  The expected
output is the oracle's decode of the oracle's container, mapped through the
same lookup table on the host; the comparison is bit for bit, and the bytes
after the last element must be untouched.
"""
import zlib

import numpy as np
import pytest

import datagen
import oracle
from rans_util import dev, first_diff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1402_3392_amd as m
    return m


def make_syms(alphabet, dist, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    if dist == "zipf":
        p = datagen.zipf_probs(alphabet, 1.1)
    elif dist == "near_uniform":
        p = datagen.near_uniform_probs(alphabet, rng)
    else:
        p = datagen.dominant_probs(alphabet, 0.995)
    return datagen.sample(p, n, rng, np.uint8 if alphabet <= 256 else np.uint16)


def run_lut(lr, table, cont, n, lut, lut_w, cap=None, guard=64):
    import torch
    cap = n if cap is None else cap
    d_lut = dev(lut)
    d_out = torch.full((cap * lut_w + guard,), 0xC3, dtype=torch.uint8, device="cuda")
    got = lr.rans_decode_lut(table, dev(cont), cont.size, d_lut, lut_w, d_out, cap)
    torch.cuda.synchronize()
    raw = d_out.cpu().numpy()
    assert (raw[n * lut_w:] == 0xC3).all(), "wrote past the last element"
    return got, raw[: n * lut_w].view(np.uint16 if lut_w == 2 else np.uint32)


# (alphabet, dist, k, r, l, N, C, n, lut_w, order); the decoder table layout
# follows from (alphabet, k): fused for 8-bit alphabets with k <= 14, packed
# or two-level otherwise
CASES = [
    (256, "zipf", 12, 16, 16, 64, 4096, 200_003, 2, "df"),
    (256, "zipf", 14, 16, 16, 64, 65536, 3 * 65536 + 12345, 4, "df"),
    (256, "near_uniform", 15, 16, 16, 64, 8192, 100_001, 2, "df"),
    (256, "zipf", 11, 8, 23, 32, 8192, 150_001, 4, "df"),
    (256, "zipf", 15, 8, 23, 64, 4096, 100_000, 2, "bf"),
    (4096, "near_uniform", 15, 16, 16, 64, 8192, 70_001, 4, "df"),
    (4096, "zipf", 15, 8, 23, 32, 2048, 2 * 2048 + 15 * 32 + 5, 2, "bf"),
    (4096, "near_uniform", 15, 8, 23, 64, 1024, 7 * 1024 + 999, 4, "df"),
    # ragged last steps and partial output blocks on N = 64 and 32
    (256, "zipf", 12, 16, 16, 64, 1024, 5 * 1024 + 992, 4, "df"),
    (256, "zipf", 14, 16, 16, 32, 2048, 3 * 2048 + 31 * 32 + 17, 2, "df"),
    (2, "dominant", 15, 16, 16, 64, 4096, 300_000, 2, "df"),
    (256, "zipf", 14, 16, 16, 64, 8, 1_001, 2, "df"),
    (256, "zipf", 14, 16, 16, 64, 4, 333, 4, "df"),
]


def ids(c):
    return f"a{c[0]}-{c[1]}-k{c[2]}-r{c[3]}-l{c[4]}-N{c[5]}-C{c[6]}-n{c[7]}-e{c[8]}-{c[9]}"


@pytest.mark.parametrize("case", CASES, ids=[ids(c) for c in CASES])
def test_lut_decode_matches_oracle(lr, case):
    alphabet, dist, k, r, l, N, C, n, lut_w, order = case
    seed = zlib.crc32(ids(case).encode())
    syms = make_syms(alphabet, dist, n, seed)
    counts = datagen.counts(syms, alphabet)
    f = oracle.quantize(counts, k)
    table = lr.rans_tables_build(counts, k)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    lut = rng.integers(0, 1 << (8 * lut_w), alphabet, dtype=np.uint64).astype(
        np.uint16 if lut_w == 2 else np.uint32)
    print(f"[lut] {ids(case)}", flush=True)
    cont = oracle.encode(f, syms, k, r, l, N, C, threads=4, order=order)
    ref = lut[oracle.decode(f, cont, threads=4)]
    got_n, got = run_lut(lr, table, cont, n, lut, lut_w)
    assert got_n == n
    assert (got == ref).all(), first_diff(got.view(np.uint8), ref.view(np.uint8))


def test_lut_decode_async_matches(lr):
    import torch
    syms = make_syms(256, "zipf", 123_457, 77)
    counts = datagen.counts(syms, 256)
    f = oracle.quantize(counts, 13)
    table = lr.rans_tables_build(counts, 13)
    cont = oracle.encode(f, syms, 13, 16, 16, 64, 4096)
    lut = (np.arange(256, dtype=np.uint64) * 2654435761 % (1 << 32)).astype(np.uint32)
    d_out = torch.zeros(syms.size * 4, dtype=torch.uint8, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    lr.rans_decode_lut_async(table, dev(cont), cont.size, cont[:32].tobytes(), dev(lut), 4, d_out,
                             syms.size, st)
    torch.cuda.synchronize()
    assert int(st[0]) == 0
    assert (d_out.cpu().numpy().view(np.uint32) == lut[syms]).all()


def test_lut_decode_rejects(lr):
    import torch
    syms = make_syms(256, "zipf", 50_000, 78)
    counts = datagen.counts(syms, 256)
    f = oracle.quantize(counts, 12)
    table = lr.rans_tables_build(counts, 12)
    lut = np.arange(256, dtype=np.uint16)
    d_in_ok = dev(oracle.encode(f, syms, 12, 16, 16, 64, 4096))
    n_ok = d_in_ok.numel()
    cont4 = oracle.encode(f, syms, 12, 16, 16, 4, 4096)  # N = 4: no one-wave-per-chunk kernel
    d_out = torch.zeros(syms.size * 4 + 64, dtype=torch.uint8, device="cuda")

    def code(fn):
        try:
            fn()
            return 0
        except lr.RansError as e:
            return e.code

    ok = oracle.encode(f, syms, 12, 16, 16, 64, 4096)
    assert code(lambda: lr.rans_decode_lut(table, dev(ok), ok.size, dev(lut), 3, d_out, syms.size)) \
        == lr.RANS_EINVAL
    assert code(lambda: lr.rans_decode_lut(table, dev(ok), ok.size, dev(lut), 0, d_out, syms.size)) \
        == lr.RANS_EINVAL
    assert code(lambda: lr.rans_decode_lut(table, dev(cont4), cont4.size, dev(lut), 2, d_out,
                                           syms.size)) == lr.RANS_EINVAL
    assert code(lambda: lr.rans_decode_lut(table, dev(ok), ok.size, dev(lut), 2, d_out[2:],
                                           syms.size)) == lr.RANS_EINVAL  # output not 16-byte aligned
    assert code(lambda: lr.rans_decode_lut(table, dev(ok), ok.size, dev(lut), 2, d_out,
                                           syms.size - 1)) == lr.RANS_ENOSPC
    bad = ok.copy()
    first = int(np.frombuffer(bad[32:40].tobytes(), "<u8")[0])
    bad[first + 4 * 64 + 100] ^= 0x5A
    assert code(lambda: lr.rans_decode_lut(table, dev(bad), bad.size, dev(lut), 2, d_out,
                                           syms.size)) == lr.RANS_ECORRUPT
    assert n_ok > 0
