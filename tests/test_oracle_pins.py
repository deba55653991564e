"""Pins the CPU oracle to what the paper and the mathematics fix.

None of these checks re-runs the oracle's own formulas: they compare it with
values printed in the paper (worked example, Section 2.1 / Section 3), with
the example's own, differently written coding function, with brute-force
enumerations of the stated properties (C and D inverse, precursor sets of the
b-unique form, x stays in I, last-in-first-out, encoder/decoder lockstep), with
an independent construction of the interleaved stream (Section 4's
instrumented-decoder multiplexer), and with the entropy bound on the size.
"""
import itertools

import numpy as np
import pytest

import oracle


# --------------------------------------------------------- worked example --

def example_C(s, x):
    """The example coding function exactly as Section 2.1 prints it."""
    return 4 * x if s == 0 else 4 * (x // 3) + (x % 3) + 1


def example_D(x):
    """The example decoding function exactly as Section 2.1 prints it."""
    return (0, x // 4) if x % 4 == 0 else (1, 3 * (x // 4) + (x % 4) - 1)


def test_example_C_and_D_equal_paper_formulas(golden_example):
    f = golden_example["freq"]
    for x in range(0, 3000):
        assert oracle.C(f, 2, 0, x) == example_C(0, x)
        assert oracle.C(f, 2, 1, x) == example_C(1, x)
        assert oracle.D(f, 2, x) == example_D(x)


def test_example_precursor_sets_match_paper(golden_example):
    f = golden_example["freq"]
    L = golden_example["L"][0]
    b = golden_example["radix"][0]
    for s, key in ((0, "I_a"), (1, "I_b")):
        # C(s,x) >= x, so no x >= bL can land in I: scanning [0, bL) is complete.
        pre = [x for x in range(0, b * L) if L <= oracle.C(f, 2, s, x) < b * L]
        assert pre == golden_example[key]


def test_example_decoder_passes_printed_state(golden_example):
    f = golden_example["freq"]
    msg = golden_example["message"]
    L, b = golden_example["L"][0], golden_example["radix"][0]
    l, r = L.bit_length() - 1, b.bit_length() - 1
    states, digits, _ = oracle.encode_digits(f, 2, r, l, 1, msg)
    out, trace = oracle.decode_digits(f, 2, r, l, 1, states, digits, len(msg), trace=True)
    assert list(out) == msg
    first_a = msg.index(0)
    assert int(trace[first_a]) == golden_example["state_after_first_a"][0]
    assert all(L <= int(x) < b * L for x in trace)


def test_example_encoder_decoder_lockstep(golden_example):
    """Decoder state after symbol i equals the encoder state after it coded
    symbol i+1 (the encoder runs backwards); the last one is the start L."""
    f = golden_example["freq"]
    msg = golden_example["message"]
    states, digits, etr = oracle.encode_digits(f, 2, 1, 4, 1, msg, trace=True)
    _, dtr = oracle.decode_digits(f, 2, 1, 4, 1, states, digits, len(msg), trace=True)
    assert int(states[0]) == int(etr[0])
    for i in range(len(msg) - 1):
        assert dtr[i] == etr[i + 1]
    assert int(dtr[-1]) == 16


def test_example_against_scalar_algorithm_with_paper_functions(golden_example):
    """Algorithm 1 run with the example's printed C and D (not the oracle's
    general rANS) gives the same stream, final state and decode."""
    msg = golden_example["message"]
    L, b = 16, 2
    x, stream = L, []
    for s in reversed(msg):
        while not (L <= example_C(s, x) < b * L):
            stream.insert(0, x % b)
            x //= b
        x = example_C(s, x)
    states, digits, _ = oracle.encode_digits(golden_example["freq"], 2, 1, 4, 1, msg)
    assert int(states[0]) == x
    assert list(digits) == stream


# ------------------------------------------------------------ brute force --

def random_models(seed, count=24):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        k = int(rng.integers(2, 5))
        M = 1 << k
        n = int(rng.integers(2, min(M, 4) + 1))
        cuts = np.sort(rng.choice(np.arange(1, M), n - 1, replace=False))
        f = np.diff(np.concatenate([[0], cuts, [M]])).astype(np.uint32)
        l = k + int(rng.integers(0, 3))
        r = int(rng.integers(1, 4))
        yield f, k, l, r


def test_C_D_are_inverse_bruteforce():
    for f, k, l, r in random_models(1):
        b, L = 1 << r, 1 << l
        for x in range(1, 4 * b * L):
            s, xp = oracle.D(f, k, x)
            assert f[s] > 0
            assert oracle.C(f, k, s, xp) == x
        for s in range(len(f)):
            for x in range(0, 2 * b * L):
                assert oracle.D(f, k, oracle.C(f, k, s, x)) == (s, x)


def test_precursor_sets_are_b_unique_bruteforce():
    """I_s = {x : C(s,x) in I} has the form {m, ..., bm-1}, m >= 1."""
    for f, k, l, r in random_models(2):
        b, L = 1 << r, 1 << l
        for s in range(len(f)):
            pre = [x for x in range(0, b * L) if L <= oracle.C(f, k, s, x) < b * L]
            m = pre[0]
            assert m >= 1
            assert pre == list(range(m, b * m))


def test_lifo_property():
    rng = np.random.default_rng(3)
    for f, k, l, r in random_models(3, 8):
        for _ in range(50):
            a, c = rng.integers(0, len(f), 2)
            x = int(rng.integers(0, 1000))
            inner = oracle.C(f, k, int(a), x)
            assert oracle.D(f, k, oracle.C(f, k, int(c), inner)) == (int(c), inner)


def enumerate_messages(n_alpha, max_len):
    for length in range(0, max_len + 1):
        yield from itertools.product(range(n_alpha), repeat=length)


@pytest.mark.parametrize("N", [1, 2, 3])
def test_exhaustive_roundtrip_and_injectivity(N):
    cases = [([1, 3], 2, 4, 1), ([2, 1, 1], 2, 2, 2), ([1, 2, 5], 3, 3, 3), ([3, 5], 3, 4, 2)]
    for f, k, l, r in cases:
        b, L = 1 << r, 1 << l
        seen = {}
        for msg in enumerate_messages(len(f), 6):
            states, digits, etr = oracle.encode_digits(f, k, r, l, N, list(msg), trace=True)
            out, dtr = oracle.decode_digits(f, k, r, l, N, states, digits, len(msg),
                                            trace=True)
            assert tuple(int(v) for v in out) == msg
            assert all(L <= int(x) < b * L for x in etr)
            assert all(L <= int(x) < b * L for x in dtr)
            key = (len(msg), tuple(int(v) for v in states), tuple(int(v) for v in digits))
            assert key not in seen, (msg, seen.get(key))
            seen[key] = msg


def test_lockstep_per_coder():
    """Coder j's decoder state after symbol i equals its encoder state after
    symbol i+N (or L when there is none)."""
    rng = np.random.default_rng(4)
    f, k, l, r, N = [5, 7, 3, 1], 4, 8, 4, 3
    msg = rng.integers(0, 4, 200).tolist()
    st, dg, etr = oracle.encode_digits(f, k, r, l, N, msg, trace=True)
    _, dtr = oracle.decode_digits(f, k, r, l, N, st, dg, len(msg), trace=True)
    for i in range(len(msg)):
        want = int(etr[i + N]) if i + N < len(msg) else 1 << l
        assert int(dtr[i]) == want


# ----------------------------------------------------------- interleaving --

def instrumented_mux(f, k, r, l, N, msg):
    """Section 4's construction: code each coder's subsequence into its own
    stream with a single-coder encoder, then run the decoders in the
    interleaved order, appending every digit read to the shared stream."""
    b, L = 1 << r, 1 << l
    lanes = []
    for j in range(N):
        sub = msg[j::N]
        st, dg, _ = oracle.encode_digits(f, k, r, l, 1, sub)
        lanes.append([int(st[0]), [int(d) for d in dg], 0])
    mux = []
    for i, s in enumerate(msg):
        lane = lanes[i % N]
        got, x = oracle.D(f, k, lane[0])
        assert got == s
        while x < L:
            d = lane[1][lane[2]]
            lane[2] += 1
            mux.append(d)
            x = b * x + d
        lane[0] = x
    return [ln_[0] for ln_ in lanes], mux


@pytest.mark.parametrize("N", [2, 3, 5])
def test_interleaved_stream_equals_instrumented_mux(N):
    rng = np.random.default_rng(10 + N)
    for f, k, l, r in [([1, 3], 2, 4, 1), ([9, 1, 4, 2], 4, 6, 3), ([200, 40, 16], 8, 16, 16),
                       ([100, 50, 106], 8, 23, 8)]:
        msg = rng.integers(0, len(f), 301).tolist()
        st, dg, _ = oracle.encode_digits(f, k, r, l, N, msg)
        final_states, mux = instrumented_mux(f, k, r, l, N, msg)
        assert [int(v) for v in dg] == mux
        # after the instrumented decode every coder is back at L
        assert final_states == [1 << l] * N
        # the coders' initial decoder states are the single-coder final states
        for j in range(N):
            st1, _, _ = oracle.encode_digits(f, k, r, l, 1, msg[j::N])
            assert int(st[j]) == int(st1[0])


def test_wrong_interleave_or_order_fails_end_check():
    rng = np.random.default_rng(5)
    f, k, l, r = [30, 20, 14], 6, 16, 16
    msg = rng.integers(0, 3, 999).tolist()
    st, dg, _ = oracle.encode_digits(f, k, r, l, 4, msg)
    with pytest.raises(oracle.OracleError) as e:
        oracle.decode_digits(f, k, r, l, 2, st[:2], dg, len(msg))
    assert e.value.code == oracle.ECORRUPT
    with pytest.raises(oracle.OracleError):
        oracle.decode_digits(f, k, r, l, 4, st[::-1].copy(), dg, len(msg))


def test_single_step_rule_and_order_independence_when_b_ge_M():
    """With b >= M no symbol needs more than one digit, and depth-first and
    breadth-first streams coincide (Section 5)."""
    rng = np.random.default_rng(6)
    for f, k, l, r in [([100, 50, 106], 8, 16, 8), ([1000, 3000, 96], 12, 16, 16)]:
        for N in (1, 4, 7, 64):
            msg = rng.integers(0, 3, 777).tolist()
            s1, d1, _ = oracle.encode_digits(f, k, r, l, N, msg, order="df")
            s2, d2, _ = oracle.encode_digits(f, k, r, l, N, msg, order="bf")
            assert (s1 == s2).all() and (d1 == d2).all()
            assert len(d1) <= len(msg)
            out = oracle.decode_digits(f, k, r, l, N, s2, d2, len(msg), order="df")
            assert list(out) == msg


def test_depth_first_and_breadth_first_differ_when_b_lt_M():
    rng = np.random.default_rng(7)
    f, k, l, r, N = [1, 2, 13], 4, 8, 1, 4
    differ = 0
    for _ in range(20):
        msg = rng.integers(0, 3, 64).tolist()
        s1, d1, _ = oracle.encode_digits(f, k, r, l, N, msg, order="df")
        s2, d2, _ = oracle.encode_digits(f, k, r, l, N, msg, order="bf")
        assert (s1 == s2).all()               # states do not depend on the layout
        assert sorted(d1) == sorted(d2)        # same digits, different order
        assert list(oracle.decode_digits(f, k, r, l, N, s2, d2, 64, order="bf")) == msg
        if list(d1) != list(d2):
            differ += 1
    assert differ > 0


def _digit_order_case(name):
    from conftest import load_golden
    g = load_golden(name)
    return (g["freq"], g["k"][0], g["radix_bits"][0], g["L_bits"][0], g["N"][0], g["message"],
            g["states"], g["depth_first"], g["breadth_first"], g)


@pytest.mark.parametrize("name", ["digit_order_two_coders.txt", "digit_order_packed_load.txt"])
def test_digit_orders_equal_hand_derived_streams(name):
    """Section 5's two orders on hand-derived messages: the two-coder case the
    paper describes in words (coder 0 reads two bytes, coder 1 one) and the
    paper's packed-load mask {1, 0, 1, 1} followed by a second round with
    two coders, ascending in both rounds; the last step is ragged."""
    f, k, r, l, N, msg, states, df, bf, _ = _digit_order_case(name)
    for order, want in (("df", df), ("bf", bf)):
        st, dig, _ = oracle.encode_digits(f, k, r, l, N, msg, order=order)
        assert [int(v) for v in st] == states, order
        assert [int(v) for v in dig] == want, order
        assert [int(v) for v in oracle.decode_digits(f, k, r, l, N, states, want, len(msg),
                                                     order=order)] == msg, order
    # read in the other order the streams fail the end check (same digits,
    # other coders)
    for order, other in (("df", bf), ("bf", df)):
        with pytest.raises(oracle.OracleError):
            oracle.decode_digits(f, k, r, l, N, states, other, len(msg), order=order)


def test_breadth_first_rounds_read_lanes_ascending():
    """After step 0 of the packed-load message, the coders hold the states
    the hand derivation gives: round 1 feeds coders 0, 2, 3 the bytes at
    ptr[0], ptr[1], ptr[2]; round 2 feeds coders 0, 3 the next two."""
    f, k, r, l, N, msg, states, _, bf, g = _digit_order_case("digit_order_packed_load.txt")
    _, tr = oracle.decode_digits(f, k, r, l, N, states, bf, len(msg), order="bf", trace=True)
    assert [int(v) for v in tr[:N]] == g["after_step0"]


def test_quantizer_hand_computed_ties_and_excess():
    """The quantiser rule on hand-computed cases: deficits by remainder with
    ties to the lower index, forced symbols left out of the deficit, absent
    symbols at 0, an excess taken from the largest f with ties to the lower
    index."""
    from conftest import load_golden
    g = load_golden("quantizer_ties.txt")
    names = [key[len("counts_"):] for key in g if key.startswith("counts_")]
    assert len(names) >= 7
    for nm in names:
        c = np.array(g["counts_" + nm], dtype=np.uint64)
        assert [int(v) for v in oracle.quantize(c, g["k_" + nm][0])] == g["expect_" + nm], nm


# ------------------------------------------------------------------ sizes --

def test_size_close_to_cross_entropy():
    """Coding s grows the state by about M/f_s (Section 2.1), so the payload
    is close to sum_s c_s log2(M/f_s) bits."""
    import datagen
    rng = np.random.Generator(np.random.PCG64(11))
    for s_exp, k, r, l, N in [(1.1, 12, 16, 16, 4), (0.8, 14, 8, 23, 64), (1.5, 11, 16, 16, 32)]:
        p = datagen.zipf_probs(256, s_exp)
        syms = datagen.sample(p, 200_000, rng)
        f = oracle.quantize(datagen.counts(syms, 256), k)
        st, dg, _ = oracle.encode_digits(f, k, r, l, N, syms)
        payload_bits = len(dg) * r
        c = datagen.counts(syms, 256).astype(np.float64)
        nz = c > 0
        hx = float((c[nz] * np.log2((1 << k) / f[nz].astype(np.float64))).sum())
        assert abs(payload_bits - hx) <= 0.01 * len(syms) + 32 * N + r * N


# -------------------------------------------------------------- quantiser --

def test_quantizer_properties():
    rng = np.random.default_rng(8)
    for trial in range(300):
        n = int(rng.integers(1, 300))
        k = int(rng.integers(max(1, int(np.ceil(np.log2(n)))), 17))
        c = rng.integers(0, 1000, n).astype(np.uint64)
        if trial % 3 == 0:
            c[rng.random(n) < 0.5] = 0
        if c.sum() == 0:
            c[0] = 1
        f = oracle.quantize(c, k)
        M = 1 << k
        assert int(f.sum()) == M
        assert ((f > 0) == (c > 0)).all()
        exact = c.astype(np.float64) * M / float(c.sum())
        if not ((exact < 1) & (c > 0)).any():
            assert (np.abs(f - exact) < 1).all()


def test_quantizer_identity_and_errors():
    f0 = np.array([1, 3, 0, 12], dtype=np.uint64)
    assert list(oracle.quantize(f0, 4)) == [1, 3, 0, 12]
    with pytest.raises(oracle.OracleError) as e:
        oracle.quantize(np.ones(5, dtype=np.uint64), 2)
    assert e.value.code == oracle.EPREC
    with pytest.raises(oracle.OracleError) as e:
        oracle.quantize(np.zeros(5, dtype=np.uint64), 8)
    assert e.value.code == oracle.EINVAL


# -------------------------------------------------------------- container --

def test_container_layout_and_roundtrip():
    import struct
    rng = np.random.default_rng(9)
    syms = rng.integers(0, 7, 10_001).astype(np.uint8)
    f = oracle.quantize(np.bincount(syms, minlength=256).astype(np.uint64), 12)
    for r, l, N, C in [(16, 16, 4, 0), (16, 16, 64, 1000), (8, 23, 32, 333), (8, 20, 7, 4096)]:
        buf = oracle.encode(f, syms, 12, r, l, N, C)
        magic, ver, k_, r_, l_, w_, z, N_, C_, n_, nch, z2 = struct.unpack_from(
            "<IBBBBBBHIQII", buf.tobytes(), 0)
        assert (magic, ver, k_, r_, l_, w_, z, N_, n_) == (0x534E4172, 1, 12, r, l, 1, 0, N,
                                                           len(syms))
        Ceff = C or len(syms)
        assert C_ == Ceff and nch == -(-len(syms) // Ceff) and z2 == 0
        end = 32 + 16 * nch
        for c in range(nch):
            off, ln, z3 = struct.unpack_from("<QII", buf.tobytes(), 32 + 16 * c)
            assert off % 16 == 0 and z3 == 0 and off >= end
            assert not buf[end:off].any()  # zero padding
            end = off + ln
        assert len(buf) == (end + 15) // 16 * 16
        assert (oracle.decode(f, buf) == syms).all()


@pytest.mark.parametrize("n", [0, 1, 3, 63, 64, 65])
def test_container_small_and_ragged(n):
    f = [3, 1] + [0] * 254
    syms = (np.arange(n) % 2).astype(np.uint8)
    for N in (1, 4, 64):
        buf = oracle.encode(f, syms, 2, 16, 16, N, 0)
        assert (oracle.decode(f, buf) == syms).all()


def test_container_corruption_detected():
    rng = np.random.default_rng(12)
    syms = rng.integers(0, 200, 50_000).astype(np.uint8)
    f = oracle.quantize(np.bincount(syms, minlength=256).astype(np.uint64), 12)
    buf = oracle.encode(f, syms, 12, 16, 16, 64, 8192)
    hdr = oracle.header(buf)
    first = int(np.frombuffer(buf[32:40].tobytes(), "<u8")[0])
    bad = buf.copy()
    bad[first + 4 * 64 + 100] ^= 0x5A
    with pytest.raises(oracle.OracleError) as e:
        oracle.decode(f, bad)
    assert e.value.code == oracle.ECORRUPT
    with pytest.raises(oracle.OracleError):
        oracle.decode(f, buf[:len(buf) - 200])
    assert hdr["n_chunks"] == 7


def test_encode_rejects_absent_symbol():
    f = [4, 0, 0, 12]
    with pytest.raises(oracle.OracleError) as e:
        oracle.encode(f, np.array([0, 1, 3], dtype=np.uint8), 4, 16, 16, 1, 0)
    assert e.value.code == oracle.ENOSYM


def test_uint16_symbols_large_alphabet():
    rng = np.random.default_rng(13)
    syms = rng.integers(0, 4096, 20_000).astype(np.uint16)
    f = oracle.quantize(np.bincount(syms, minlength=4096).astype(np.uint64), 15)
    for r, l in [(16, 16), (8, 23)]:
        buf = oracle.encode(f, syms, 15, r, l, 32, 4096)
        assert (oracle.decode(f, buf, threads=3) == syms).all()


# ------------------------------------------------- breadth-first containers --

def _chunk_streams(buf):
    """(states, digit bytes) of every chunk of a container, from its directory."""
    import struct
    raw = buf.tobytes()
    N = struct.unpack_from("<H", raw, 10)[0]
    nch = struct.unpack_from("<I", raw, 24)[0]
    out = []
    for c in range(nch):
        off, ln, _ = struct.unpack_from("<QII", raw, 32 + 16 * c)
        out.append((np.frombuffer(raw[off:off + 4 * N], "<u4"), buf[off + 4 * N:off + ln]))
    return out


def test_breadth_first_container_roundtrip_and_order_byte():
    rng = np.random.default_rng(21)
    # half the mass on one symbol, the rest spread over 255 symbols of
    # frequency below M/b = 16, so many steps emit two 8-bit digits
    syms = np.where(rng.random(20_000) < 0.5, 0, rng.integers(1, 256, 20_000)).astype(np.uint8)
    f = oracle.quantize(np.bincount(syms, minlength=256).astype(np.uint64), 12)
    for r, l, N, C in [(8, 23, 64, 4096), (8, 20, 7, 1000), (16, 16, 32, 2048)]:
        bf = oracle.encode(f, syms, 12, r, l, N, C, order="bf")
        assert bf[9] == 1 and oracle.header(bf)["order"] == "bf"
        assert (oracle.decode(f, bf) == syms).all()
        df = oracle.encode(f, syms, 12, r, l, N, C)
        assert df[9] == 0 and bf.size == df.size
        assert (df[:9] == bf[:9]).all() and (df[10:] == bf[10:]).all() if r == 16 else True
        if r == 8:
            # b < M: same chunk lengths and states, digits in another order
            assert (df[32:32 + 16] == bf[32:32 + 16]).all()
            assert any((a[1] != b[1]).any() for a, b in zip(_chunk_streams(df), _chunk_streams(bf)))
            # read with the other order the streams fail the end check
            flipped = bf.copy()
            flipped[9] = 0
            with pytest.raises(oracle.OracleError):
                oracle.decode(f, flipped)


def test_breadth_first_container_chunks_equal_digit_level_coder():
    """Each chunk of a breadth-first container is the digit-level
    breadth-first coder's stream for that chunk's symbols."""
    rng = np.random.default_rng(22)
    syms = rng.integers(0, 60, 5_000).astype(np.uint8)
    f = oracle.quantize(np.bincount(syms, minlength=256).astype(np.uint64), 10)
    k, r, l, N, C = 10, 8, 23, 16, 1500
    buf = oracle.encode(f, syms, k, r, l, N, C, order="bf")
    for c, (states, digs) in enumerate(_chunk_streams(buf)):
        s, d, _ = oracle.encode_digits(f, k, r, l, N, syms[c * C:(c + 1) * C].tolist(), order="bf")
        assert (states == s).all() and (digs == np.asarray(d, np.uint8)).all()


def test_order_byte_values_above_one_rejected():
    syms = (np.arange(1000) % 3).astype(np.uint8)
    f = oracle.quantize(np.bincount(syms, minlength=256).astype(np.uint64), 8)
    buf = oracle.encode(f, syms, 8, 8, 23, 4, 0)
    buf[9] = 2  # escape coding, which 8-bit symbols cannot use
    with pytest.raises(oracle.OracleError):
        oracle.decode(f, buf)
    with pytest.raises(ValueError):
        oracle.encode(f, syms, 8, 8, 23, 4, 0, order="xx")


# ----------------------------------------------------- escape / raw digits --

def _escape_case(seed, n=6000, alpha=300, k=12):
    """uint16 values: most drawn from a Zipf table over `alpha` symbols (the
    last of which is the escape), the rest anywhere in 0..65535; the table
    gives two frequent values frequency 0."""
    rng = np.random.default_rng(seed)
    p = 1.0 / np.arange(1, alpha + 1) ** 1.1
    v = rng.choice(alpha, size=n, p=p / p.sum()).astype(np.uint16)
    wild = rng.random(n) < 0.1
    v[wild] = rng.integers(0, 65536, int(wild.sum()))
    counts = np.bincount(np.minimum(v, alpha - 1), minlength=alpha).astype(np.uint64)
    counts[alpha - 1] += 1
    counts[[3, 7]] = 0  # values the table leaves out escape too
    return v, oracle.quantize(counts, k)


def _tokens(v, f):
    E = len(f) - 1
    vi = v.astype(np.int64)
    esc = (vi >= E) | (np.asarray(f)[np.minimum(vi, E)] == 0)
    return np.where(esc, E, vi).astype(np.uint16), esc


@pytest.mark.parametrize("r,l", [(16, 16), (8, 23)])
@pytest.mark.parametrize("N,C", [(1, 0), (4, 1000), (64, 2048), (32, 777)])
def test_escape_roundtrip_and_states_equal_token_stream(r, l, N, C):
    """Raw digits never touch a coder state (Section 3): the states of an
    escape container are those of the plain container of the token
    sequence, and each escape adds exactly 16/r raw digits."""
    v, f = _escape_case(31 + N + r)
    buf = oracle.encode(f, v, 12, r, l, N, C, escape=True)
    h = oracle.header(buf)
    assert buf[9] == 2 and h["escape"] and h["nraw"] == 16 // r
    assert (oracle.decode(f, buf) == v).all()
    tok, esc = _tokens(v, f)
    plain = oracle.encode(f, tok, 12, r, l, N, C)
    Ce = C or v.size
    for c, (a, b) in enumerate(zip(_chunk_streams(buf), _chunk_streams(plain))):
        assert (a[0] == b[0]).all(), c
        nesc = int(esc[c * Ce:(c + 1) * Ce].sum())
        assert a[1].size == b[1].size + nesc * 2, c  # 16 raw bits per escape


def test_escape_without_escapes_is_the_plain_stream():
    rng = np.random.default_rng(33)
    v = rng.integers(0, 40, 5000).astype(np.uint16)
    f = oracle.quantize(np.bincount(np.r_[v, [40]], minlength=41).astype(np.uint64), 11)
    assert (f[:40] > 0).all() and f[40] > 0
    for r, l in [(16, 16), (8, 23)]:
        a = oracle.encode(f, v, 11, r, l, 16, 1000, escape=True)
        b = oracle.encode(f, v, 11, r, l, 16, 1000)
        assert a[9] == 2 and b[9] == 0
        assert (a[:9] == b[:9]).all() and (a[10:] == b[10:]).all()


@pytest.mark.parametrize("r,l", [(16, 16), (8, 23)])
def test_escape_with_one_symbol_table_is_raw_storage(r, l):
    """With f = (M): C and D are the identity and nothing renormalises, so every
    value escapes and each chunk stream is the states (all L) followed by the
    values themselves in message order, 16 bits each, high digit first."""
    rng = np.random.default_rng(34)
    v = rng.integers(0, 65536, 3001).astype(np.uint16)
    f = np.array([1 << 10], np.uint32)
    N, C = 8, 1000
    buf = oracle.encode(f, v, 10, r, l, N, C, escape=True)
    for c, (st, dig) in enumerate(_chunk_streams(buf)):
        assert (st == (1 << l)).all()
        part = v[c * C:(c + 1) * C]
        want = (part.astype("<u2").view(np.uint8) if r == 16
                else part.astype(">u2").view(np.uint8))
        assert (dig == want).all(), c
    # a raw digit sits where that closed form says: flipping the one of value
    # 1234 changes that value only, and the end check still passes
    bad = buf.copy()
    off = int(np.frombuffer(bad[32 + 16:32 + 24].tobytes(), "<u8")[0])  # chunk 1
    bad[off + 4 * N + 2 * (1234 - C) + (1 if r == 8 else 0)] ^= 0x81
    out = oracle.decode(f, bad)
    diff = np.flatnonzero(out != v)
    assert diff.tolist() == [1234] and int(out[1234]) == int(v[1234]) ^ 0x81


def test_escape_flags_checked():
    v, f = _escape_case(35, n=500)
    buf = oracle.encode(f, v, 12, 16, 16, 4, 0, escape=True)
    plainread = buf.copy()
    plainread[9] = 0  # raw digits read as renormalisation digits
    try:
        out = oracle.decode(f, plainread)
        assert (out != v).any()
    except oracle.OracleError:
        pass
    for bad_flags in (3, 4, 0x80):
        b = buf.copy()
        b[9] = bad_flags
        with pytest.raises(oracle.OracleError):
            oracle.decode(f, b)
    w1 = (np.arange(100) % 3).astype(np.uint8)
    f1 = oracle.quantize(np.array([40, 30, 30, 1], np.uint64), 8)
    with pytest.raises(oracle.OracleError):
        oracle.encode(f1, w1, 8, 16, 16, 4, 0, escape=True)  # 16-bit symbols only
    with pytest.raises(oracle.OracleError):
        oracle.encode(f, v, 12, 16, 16, 4, 0, order="bf", escape=True)


# ------------------------------------ prefix-code family and its multiplexer --

def _pfx_case(seed, n=5000, alpha=40, k=11):
    rng = np.random.default_rng(seed)
    p = 1.0 / np.arange(1, alpha + 1) ** 1.3
    syms = rng.choice(alpha, size=n, p=p / p.sum()).astype(np.uint8)
    f = oracle.quantize(np.bincount(syms, minlength=alpha).astype(np.uint64), k)
    return syms, f


def test_prefix_code_is_a_valid_canonical_code():
    """Kraft, prefix-freedom by brute force, canonical order, and the Shannon
    bound len < log2(M/f) + 1."""
    for seed, alpha, k in [(41, 40, 11), (42, 256, 12), (43, 3, 8), (44, 1, 9)]:
        _, f = _pfx_case(seed, alpha=alpha, k=k)
        ln, cd = oracle.prefix_code(f, k)
        used = [s for s in range(len(f)) if f[s] > 0]
        assert all(ln[s] == 0 for s in range(len(f)) if f[s] == 0)
        assert sum(2.0 ** -int(ln[s]) for s in used) <= 1.0
        bits = {s: format(int(cd[s]), "0%db" % int(ln[s])) for s in used}
        for a in used:
            for b in used:
                if a != b:
                    assert not bits[b].startswith(bits[a]), (a, b)
        order = sorted(used, key=lambda s: (int(ln[s]), s))
        vals = [int(cd[s]) << (int(ln.max()) - int(ln[s])) for s in order]
        assert vals == sorted(vals) and len(set(vals)) == len(vals)
        M = 1 << k
        for s in used:
            assert 1 <= ln[s] <= k and 2.0 ** (int(ln[s]) - 1) < max(2.0, M / f[s]) * (1 + 1e-12)


def _lane_streams(f, k, syms, N):
    """Each coder's own word stream, built by concatenating code strings."""
    ln, cd = oracle.prefix_code(f, k)
    out = []
    for j in range(N):
        b = "".join(format(int(cd[s]), "0%db" % int(ln[s])) for s in syms[j::N])
        b += "0" * ((-len(b)) % 16) + "0" * 16  # zero padding and the possible extra word
        out.append([int(b[i:i + 16], 2) for i in range(0, len(b), 16)])
    return out, ln


def _read_schedule(ln, syms, N):
    """Which coder reads at each read, from code lengths alone: a coder reads
    a word before a symbol whenever it holds fewer than 16 bits."""
    nb = [0] * N
    order = []
    for i, s in enumerate(syms):
        j = i % N
        if nb[j] < 16:
            order.append(j)
            nb[j] += 16
        nb[j] -= int(ln[s])
    return order


@pytest.mark.parametrize("N", [1, 3, 32, 64])
def test_prefix_mux_is_the_decoders_read_order(N):
    """Section 4: the multiplexed stream is every coder's own stream, merged
    in the order the decoders read it -- derived here from the code lengths
    alone -- and decodes back to the input."""
    syms, f = _pfx_case(45 + N)
    k = 11
    buf = oracle.encode(f, syms, k, 16, 16, N, 0, coder="prefix")
    h = oracle.header(buf)
    assert buf[9] == 4 and h["coder"] == "prefix"
    assert (oracle.decode(f, buf) == syms).all()
    (states, dig), = _chunk_streams(buf)
    words = dig.view("<u2")
    streams, ln = _lane_streams(f, k, syms, N)
    order = _read_schedule(ln, syms, N)
    pos = [0] * N
    want = []
    for j in order:
        want.append(streams[j][pos[j]])
        pos[j] += 1
    assert words.tolist() == want
    assert states.tolist() == [int(sum(int(ln[s]) for s in syms[j::N])) for j in range(N)]


def test_prefix_mux_roundtrip_chunks_and_checks():
    syms, f = _pfx_case(50, n=20_000, alpha=200, k=12)
    for N, C in [(4, 1000), (64, 4096), (32, 777)]:
        buf = oracle.encode(f, syms, 12, 16, 16, N, C, coder="prefix", threads=2)
        assert (oracle.decode(f, buf) == syms).all()
        (states, dig) = _chunk_streams(buf)[1]
        # a wrong bit count fails the end check; a flipped bit is caught or decodes wrongly
        bad = buf.copy()
        off = int(np.frombuffer(bad[48:56].tobytes(), "<u8")[0])
        bad[off] ^= 1
        with pytest.raises(oracle.OracleError):
            oracle.decode(f, bad)
        bad = buf.copy()
        bad[off + 4 * N + 7] ^= 0x10
        try:
            assert (oracle.decode(f, bad) != syms).any()
        except oracle.OracleError:
            pass
    with pytest.raises(oracle.OracleError):
        oracle.encode(f, syms, 12, 8, 23, 4, 0, coder="prefix")  # 16-bit words only
    for flags in (3, 5, 6, 7, 8):
        b = oracle.encode(f, syms[:100], 12, 16, 16, 4, 0, coder="prefix")
        b[9] = flags
        with pytest.raises(oracle.OracleError):
            oracle.decode(f, b)
