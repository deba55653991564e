"""GPU parity: librans (HIP, gfx950) against the CPU oracle, through the C ABI.

The bar is bit-exactness: the GPU container must equal the oracle's byte for
byte, the GPU must decode the oracle's container to the input, and the
quantised tables must agree.  Inputs are seeded synthetic symbol arrays
(datagen) sized so the oracle finishes in seconds while spanning several
chunks, several waves and ragged tails.
"""
import zlib

import numpy as np
import pytest

import datagen
import oracle
from rans_util import first_diff, gpu_decode, gpu_encode

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
    elif dist == "dominant":
        p = datagen.dominant_probs(alphabet, 0.995)
    elif dist == "uniform":
        p = np.full(alphabet, 1.0 / alphabet)
    elif dist == "near_uniform":
        p = datagen.near_uniform_probs(alphabet, rng)
    else:
        raise ValueError(dist)
    dt = np.uint8 if alphabet <= 256 else np.uint16
    return datagen.sample(p, n, rng, dt)


# (alphabet, dist, k, r, l, N, C, n)
CASES = [
    (256, "zipf", 12, 16, 16, 4, 0, 100_003),
    (256, "zipf", 14, 16, 16, 64, 65536, 3 * 65536 + 12345),
    (256, "zipf", 14, 16, 16, 64, 4096, 200_007),
    (256, "zipf", 11, 8, 23, 32, 8192, 150_001),
    (256, "zipf", 15, 8, 23, 64, 4096, 100_000),
    (256, "zipf", 12, 16, 16, 1, 1000, 20_011),
    (256, "zipf", 12, 16, 16, 2, 1000, 20_011),
    (256, "zipf", 12, 16, 16, 8, 999, 20_011),
    (256, "zipf", 12, 8, 20, 16, 1000, 20_011),
    (256, "uniform", 8, 16, 16, 64, 4096, 50_000),
    (256, "uniform", 8, 8, 16, 64, 4096, 50_000),
    (4096, "near_uniform", 15, 16, 16, 64, 8192, 70_001),
    (4096, "near_uniform", 15, 8, 23, 32, 8192, 70_001),
    (4096, "dominant", 15, 16, 16, 64, 4096, 60_000),
    (16, "zipf", 11, 16, 16, 64, 4096, 50_000),
    (2, "dominant", 15, 16, 16, 64, 4096, 300_000),
    (2, "dominant", 15, 8, 23, 32, 4096, 300_000),
    (256, "zipf", 14, 16, 16, 64, 1, 300),
    (256, "zipf", 14, 16, 16, 64, 100, 1_001),
    # last chunk = 15 full steps + a partial one: the ragged step closes an
    # output block of the N = 64 decoder
    (256, "zipf", 12, 16, 16, 64, 1024, 5 * 1024 + 992),
    (4096, "near_uniform", 15, 16, 16, 64, 2048, 3 * 2048 + 480),
    (256, "zipf", 12, 8, 23, 64, 1024, 5 * 1024 + 960),
    # N = 32 on the one-wave-per-chunk kernels (lanes 32..63 idle): the last
    # chunk is 31 full steps + a partial one (w = 1: 32 steps per block,
    # w = 2: 16), and a high-entropy case that refills on most steps
    (256, "zipf", 14, 16, 16, 32, 2048, 3 * 2048 + 31 * 32 + 17),
    (4096, "near_uniform", 15, 16, 16, 32, 2048, 2 * 2048 + 15 * 32 + 5),
    (256, "uniform", 8, 16, 16, 32, 4096, 50_000),
    (16, "zipf", 11, 8, 23, 32, 1024, 7 * 1024 + 999),
]


def ids(c):
    return f"a{c[0]}-{c[1]}-k{c[2]}-r{c[3]}-l{c[4]}-N{c[5]}-C{c[6]}-n{c[7]}"


@pytest.mark.parametrize("case", CASES, ids=[ids(c) for c in CASES])
def test_bitstream_and_symbols_match_oracle(lr, case):
    alphabet, dist, k, r, l, N, C, n = case
    syms = make_syms(alphabet, dist, n, seed=zlib.crc32(ids(case).encode()))
    w = syms.dtype.itemsize
    counts = datagen.counts(syms, alphabet)
    f_or = oracle.quantize(counts, k)
    table = lr.rans_tables_build(counts, k)
    assert (lr.rans_table_freqs(table) == f_or).all()
    params = (k, r, l, w, N, C)
    print(f"[parity] {ids(case)}", flush=True)
    ref = oracle.encode(f_or, syms, k, r, l, N, C, threads=4)
    got = gpu_encode(lr, table, params, syms)
    assert got.size == ref.size and (got == ref).all(), first_diff(got, ref)
    dec = gpu_decode(lr, table, ref, n, w)
    assert (dec == syms).all(), first_diff(dec.view(np.uint8), syms.view(np.uint8))


# Breadth-first digit order (Section 5).  It differs from depth-first only
# when a step can read two digits (b = 2^8 < M): one-wave-per-chunk kernels
# (N = 32, 64; w = 1 and 2; sparse and dense refills; ragged last chunks) and
# the generic kernels (N < 32); a 16-bit-digit case must give the depth-first
# payload.
BF_CASES = [
    (256, "zipf", 15, 8, 23, 64, 4096, 100_000),
    (256, "zipf", 12, 8, 23, 32, 8192, 150_001),
    (256, "zipf", 12, 8, 23, 64, 1024, 5 * 1024 + 960),
    (4096, "near_uniform", 15, 8, 23, 64, 8192, 70_001),
    (4096, "near_uniform", 15, 8, 23, 32, 2048, 2 * 2048 + 15 * 32 + 5),
    (256, "dominant", 15, 8, 23, 32, 4096, 300_000),
    (4096, "near_uniform", 14, 8, 22, 64, 1024, 7 * 1024 + 999),
    (256, "zipf", 12, 8, 20, 16, 1000, 20_011),
    (256, "zipf", 14, 8, 23, 4, 999, 20_011),
    (256, "zipf", 13, 8, 23, 1, 0, 20_011),
    (256, "zipf", 14, 16, 16, 64, 4096, 200_007),
]


@pytest.mark.parametrize("case", BF_CASES, ids=[ids(c) for c in BF_CASES])
def test_breadth_first_matches_oracle(lr, case):
    alphabet, dist, k, r, l, N, C, n = case
    syms = make_syms(alphabet, dist, n, seed=zlib.crc32(("bf" + ids(case)).encode()))
    w = syms.dtype.itemsize
    counts = datagen.counts(syms, alphabet)
    f_or = oracle.quantize(counts, k)
    table = lr.rans_tables_build(counts, k)
    print(f"[parity-bf] {ids(case)}", flush=True)
    ref = oracle.encode(f_or, syms, k, r, l, N, C, threads=4, order="bf")
    df = oracle.encode(f_or, syms, k, r, l, N, C, threads=4)
    if r == 16 or N == 1:
        assert (ref[10:] == df[10:]).all()   # one digit per step, or one coder
    else:
        assert (ref[32:] != df[32:]).any()   # the case exercises the order
    got = gpu_encode(lr, table, (k, r, l, w, N, C, "bf"), syms)
    assert got[9] == 1
    assert got.size == ref.size and (got == ref).all(), first_diff(got, ref)
    dec = gpu_decode(lr, table, ref, n, w)
    assert (dec == syms).all(), first_diff(dec.view(np.uint8), syms.view(np.uint8))
    if r == 8 and N > 1:
        # read in the other order, the streams fail the end-of-chunk check
        flipped = ref.copy()
        flipped[9] = 0
        assert _decode_rc(lr, table, flipped, n) == lr.RANS_ECORRUPT
        flipped = df.copy()
        flipped[9] = 1
        assert _decode_rc(lr, table, flipped, n) == lr.RANS_ECORRUPT


def test_unknown_digit_order_rejected(lr):
    syms, table, ref = _container(lr)
    bad = ref.copy()
    bad[9] = 2
    assert _decode_rc(lr, table, bad, syms.size) == lr.RANS_ECORRUPT


def test_single_symbol_alphabet(lr):
    """f = M: C and D are the identity and nothing is ever emitted."""
    syms = np.zeros(10_000, dtype=np.uint8)
    counts = datagen.counts(syms, 256)
    for k, r, l in [(14, 16, 16), (12, 8, 23)]:
        table = lr.rans_tables_build(counts, k)
        f = oracle.quantize(counts, k)
        ref = oracle.encode(f, syms, k, r, l, 64, 4096)
        got = gpu_encode(lr, table, (k, r, l, 1, 64, 4096), syms)
        assert (got == ref).all()
        assert (gpu_decode(lr, table, ref, syms.size, 1) == syms).all()


@pytest.mark.parametrize("n", [0, 1, 5, 63, 64, 65, 129])
def test_tiny_inputs(lr, n):
    syms = (np.arange(n) % 3).astype(np.uint8)
    counts = datagen.counts(np.arange(3).astype(np.uint8), 256)  # every symbol used present
    f = oracle.quantize(counts, 12)
    table = lr.rans_tables_build(counts, 12)
    for N, C in [(64, 0), (4, 7), (64, 64)]:
        ref = oracle.encode(f, syms, 12, 16, 16, N, C)
        got = gpu_encode(lr, table, (12, 16, 16, 1, N, C), syms)
        assert (got == ref).all(), (N, C, first_diff(got, ref))
        if n:
            assert (gpu_decode(lr, table, ref, n, 1) == syms).all()


# ------------------------------------------------------ failure handling --

def _container(lr, n=60_000, N=64, C=8192, seed=5):
    syms = make_syms(256, "zipf", n, seed)
    counts = datagen.counts(syms, 256)
    table = lr.rans_tables_build(counts, 12)
    ref = oracle.encode(oracle.quantize(counts, 12), syms, 12, 16, 16, N, C)
    return syms, table, ref


def _decode_rc(lr, table, buf, n, in_len=None):
    import torch
    from rans_util import dev
    d_in = dev(buf)
    d_out = torch.empty(n + 64, dtype=torch.uint8, device="cuda")
    try:
        lr.rans_decode(table, d_in, buf.size if in_len is None else in_len, d_out, n)
        return lr.RANS_OK
    except lr.RansError as e:
        return e.code


def test_corrupt_payload_detected(lr):
    syms, table, ref = _container(lr)
    first = int(np.frombuffer(ref[32:40].tobytes(), "<u8")[0])
    for delta in (4 * 64 + 10, 4 * 64 + 1000, 3):
        bad = ref.copy()
        bad[first + delta] ^= 0x41
        assert _decode_rc(lr, table, bad, syms.size) == lr.RANS_ECORRUPT


def test_truncated_and_bad_header(lr):
    syms, table, ref = _container(lr)
    assert _decode_rc(lr, table, ref, syms.size, in_len=ref.size - 32) == lr.RANS_ECORRUPT
    assert _decode_rc(lr, table, ref, syms.size, in_len=20) == lr.RANS_ECORRUPT
    bad = ref.copy()
    bad[0] ^= 1
    assert _decode_rc(lr, table, bad, syms.size) == lr.RANS_ECORRUPT
    bad = ref.copy()
    bad[32:40] = np.frombuffer(np.uint64(ref.size + 4096).tobytes(), np.uint8)
    assert _decode_rc(lr, table, bad, syms.size) == lr.RANS_ECORRUPT
    assert _decode_rc(lr, table, ref, syms.size - 1) == lr.RANS_ENOSPC


def test_other_chunks_still_decode_after_corruption(lr):
    """A corrupted chunk fails the end check; the others are bit-exact."""
    import torch
    from rans_util import dev
    syms, table, ref = _container(lr)
    off1 = int(np.frombuffer(ref[48:56].tobytes(), "<u8")[0])
    bad = ref.copy()
    bad[off1 + 300] ^= 0x10
    d_out = torch.zeros(syms.size + 64, dtype=torch.uint8, device="cuda")
    with pytest.raises(lr.RansError):
        lr.rans_decode(table, dev(bad), bad.size, d_out, syms.size)
    out = d_out[: syms.size].cpu().numpy()
    assert (out[:8192] == syms[:8192]).all()
    assert (out[2 * 8192:] == syms[2 * 8192:]).all()


@pytest.mark.parametrize("N", [64, 32, 4])
def test_symbol_beyond_small_alphabet(lr, N):
    """8-bit symbols coded with a 16-symbol table: a value at or above the
    alphabet has no entry (the one-wave kernels stage all 256 entries, those
    past the table marked not encodable) and fails with RANS_ENOSYM, planted
    inside a chunk's whole symbol blocks and in the ragged tail; the clean
    input matches the oracle."""
    import torch
    from rans_util import dev
    syms = make_syms(16, "zipf", 50_001, 31)
    counts = datagen.counts(syms, 16)
    f = oracle.quantize(counts, 11)
    table = lr.rans_tables_build(counts, 11)
    p = lr.rans_params.make(11, 16, 16, 1, N, 4096)
    cap = lr.rans_encode_bound(syms.size, p)
    d_out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    n = lr.rans_encode(table, p, dev(syms), syms.size, d_out, cap)
    ref = oracle.encode(f, syms, 11, 16, 16, N, 4096)
    got = d_out[:n].cpu().numpy()
    assert got.size == ref.size and (got == ref).all(), first_diff(got, ref)
    for pos, v in ((5000, 16), (5001, 17), (syms.size - 3, 255)):
        bad = syms.copy()
        bad[pos] = v
        with pytest.raises(lr.RansError) as e:
            lr.rans_encode(table, p, dev(bad), bad.size, d_out, cap)
        assert e.value.code == lr.RANS_ENOSYM, (pos, v)


def test_encode_errors(lr):
    import torch
    from rans_util import dev
    syms = make_syms(256, "zipf", 10_000, 9)
    counts = datagen.counts(syms, 256)
    counts[syms[123]] = 0  # that symbol now has frequency 0
    table = lr.rans_tables_build(counts, 12)
    d_in = dev(syms)
    p = lr.rans_params.make(12, 16, 16, 1, 64, 4096)
    cap = lr.rans_encode_bound(syms.size, p)
    d_out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    with pytest.raises(lr.RansError) as e:
        lr.rans_encode(table, p, d_in, syms.size, d_out, cap)
    assert e.value.code == lr.RANS_ENOSYM
    good = lr.rans_tables_build(datagen.counts(syms, 256), 12)
    with pytest.raises(lr.RansError) as e:
        lr.rans_encode(good, p, d_in, syms.size, d_out, 100)
    assert e.value.code == lr.RANS_ENOSPC
    with pytest.raises(lr.RansError) as e:
        lr.rans_encode(good, lr.rans_params.make(13, 16, 16, 1, 64, 4096), d_in, syms.size,
                       d_out, cap)
    assert e.value.code == lr.RANS_EINVAL
    with pytest.raises(lr.RansError) as e:
        lr.rans_tables_build(np.ones(4096, dtype=np.uint64), 11)
    assert e.value.code == lr.RANS_EPREC


@pytest.mark.parametrize("name", ["digit_order_two_coders.txt", "digit_order_packed_load.txt"])
def test_digit_orders_equal_hand_derived_streams(lr, name):
    """The GPU coder on Section 5's hand-derived digit-order messages: both
    orders' states and digits equal the fixtures (not the oracle's output),
    and both containers decode back to the message."""
    from conftest import load_golden
    g = load_golden(name)
    k, r, l, N = g["k"][0], g["radix_bits"][0], g["L_bits"][0], g["N"][0]
    msg = np.array(g["message"], dtype=np.uint8)
    table = lr.rans_tables_build(np.array(g["freq"], dtype=np.uint64), k)
    assert [int(v) for v in lr.rans_table_freqs(table)] == g["freq"]
    off = 32 + 16  # one chunk: header, one directory entry, 16-byte aligned stream
    for order, key in (("df", "depth_first"), ("bf", "breadth_first")):
        print(f"[golden-order] {name} {order}", flush=True)
        got = gpu_encode(lr, table, (k, r, l, 1, N, 0, order), msg)
        states = got[off:off + 4 * N].view("<u4")
        assert [int(v) for v in states] == g["states"], order
        # the chunk's digits, then zero padding to the container's 16-byte end
        digits = g[key]
        end = off + 4 * N + len(digits)
        assert [int(v) for v in got[off + 4 * N:end]] == digits, order
        assert got.size == (end + 15) // 16 * 16 and not got[end:].any(), order
        assert (gpu_decode(lr, table, got, msg.size, 1) == msg).all(), order


@pytest.mark.parametrize("order", ["df", "bf"])
def test_byte_digit_steps_with_and_without_second_digits(lr, order):
    """Byte digits (b = 2^8, L = 2^23) with 64 coders per chunk.  Most of each
    chunk holds symbols with f >= M / 256, so no lane can need a second digit
    in a step (the renormalised state stays below b L); short bursts of one
    symbol with f < M / 256 give steps in which some lanes emit two.  The
    encoder takes a shorter path for steps without second digits; either way
    the container must equal the oracle's in both digit orders, and decode."""
    k, r, l, N, C = 12, 8, 23, 64, 16384
    rng = np.random.Generator(np.random.PCG64(4242))
    n = 8 * C + 777
    syms = rng.integers(0, 16, n, dtype=np.uint8)
    for c0 in range(0, n, C):
        burst = c0 + 4096 + np.arange(0, 1024, 32)
        syms[burst[burst < n]] = 200
    counts = datagen.counts(syms, 256)
    f_or = oracle.quantize(counts, k)
    assert 0 < f_or[200] < (1 << k) // 256 <= int(f_or[:16].min())
    table = lr.rans_tables_build(counts, k)
    print(f"[parity-digits] order={order} n={n}", flush=True)
    ref = oracle.encode(f_or, syms, k, r, l, N, C, threads=4, order=order)
    other = oracle.encode(f_or, syms, k, r, l, N, C, threads=4, order="bf" if order == "df" else "df")
    assert (ref[32:] != other[32:]).any()  # the orders differ: some steps do emit second digits
    got = gpu_encode(lr, table, (k, r, l, 1, N, C, order), syms)
    assert got.size == ref.size and (got == ref).all(), first_diff(got, ref)
    dec = gpu_decode(lr, table, ref, n, 1)
    assert (dec == syms).all(), first_diff(dec, syms)


@pytest.mark.parametrize("N", [32, 64])
@pytest.mark.parametrize("order", ["df", "bf"])
def test_byte_digits_one_digit_table(lr, N, order):
    """A table whose every nonzero f is at least M / 256 never needs two byte
    digits in one step (b = 2^8), and the coders then take their single-digit
    encode and refill paths: containers equal the oracle's in both digit
    orders (which coincide here), and decode, through the single-buffer and
    the batched kernels."""
    from test_gpu_batch import run_decode_batch, run_encode_batch
    k, r, l, C = 12, 8, 23, 8192
    rng = np.random.Generator(np.random.PCG64(5150 + N))
    syms = rng.integers(0, 16, 5 * C + 333, dtype=np.uint8)
    counts = datagen.counts(syms, 256)
    f_or = oracle.quantize(counts, k)
    assert int(f_or[f_or > 0].min()) >= (1 << k) // 256
    table = lr.rans_tables_build(counts, k)
    print(f"[parity-one-digit] N={N} order={order}", flush=True)
    ref = oracle.encode(f_or, syms, k, r, l, N, C, threads=4, order=order)
    other = oracle.encode(f_or, syms, k, r, l, N, C, threads=4, order="bf" if order == "df" else "df")
    assert (ref[32:] == other[32:]).all()  # one digit per step: the orders agree
    got = gpu_encode(lr, table, (k, r, l, 1, N, C, order), syms)
    assert got.size == ref.size and (got == ref).all(), first_diff(got, ref)
    dec = gpu_decode(lr, table, ref, syms.size, 1)
    assert (dec == syms).all(), first_diff(dec, syms)
    data = [(syms, None), (syms[: 2 * C + 77].copy(), None)]
    tables, outs, st, _ = run_encode_batch(lr, data, k, r, l, C, N=N, order=order)
    assert (st == 0).all(), st
    refs = [ref, oracle.encode(oracle.quantize(datagen.counts(data[1][0], 256), k),
                               data[1][0], k, r, l, N, C, threads=4, order=order)]
    for i in range(2):
        assert outs[i].size == refs[i].size and (outs[i] == refs[i]).all(), (i, first_diff(outs[i], refs[i]))
    sizes = [s.size for s, _ in data]
    dec2, st2, n2 = run_decode_batch(lr, tables, refs, sizes, k, r, l, N=N, order=order)
    assert (st2 == 0).all(), st2
    for i, (s, _) in enumerate(data):
        assert n2[i] == s.size and (dec2[i] == s).all(), i
