"""Host model of the fast decoder's stream schedule (CPU).

The N = 32/64 decode kernel copies a chunk's digit stream into an S-slot LDS
ring of 256-byte windows (S = 8 tested every 4 steps, or S = 4 tested every
2 steps next to the large fused table) with direct-to-LDS loads issued up to
S - 1 windows ahead, and waits whenever its read position enters a new
window, leaving in flight exactly the operations issued after the newest
window a test block may read (S - 1 - TB/2 window loads plus the output
stores and slot-0 copies among them, counted as the kernel counts them; 0
near the end).  This model replays that schedule lane by
lane on the oracle's containers, with loads that land only when a wait
guarantees them (until then their ring bytes hold random garbage), output
stores counted as memory operations, and the same refill addressing.  It
decodes correctly only if no read ever touches a window that may still be in
flight, and if lane addresses stay inside the container.
"""
import numpy as np
import pytest

import datagen
import oracle

KWIN = 256


def model_decode_chunk(cont, nch, chunk, C, n, k, l, R, f, NL, rng, S=8, TB=4, OB=1024, OW=1,
                       esc=False):
    """OW: output bytes per symbol (the fused lookup writes 2 or 4); esc:
    escape coding, a step then reads up to 4 digit bytes per coder."""
    RES = 1 + TB * (256 if esc else 128) // KWIN
    AHEAD = S - RES
    in_len = cont.size
    M = 1 << k
    cum = np.concatenate([[0], np.cumsum(f)])
    slot2sym = np.repeat(np.arange(len(f)), f)
    de = 32 + 16 * chunk
    off = int(np.frombuffer(cont[de:de + 8].tobytes(), "<u8")[0])
    ln = int(np.frombuffer(cont[de + 8:de + 12].tobytes(), "<u4")[0])
    first = chunk * C
    nsym = min(n - first, C)
    plen = ln - 4 * NL
    room = (in_len - 4) & ~3
    lds = rng.integers(0, 256, OB + (S + 1) * KWIN, dtype=np.uint8)
    pending = []  # oldest first; None = an output store

    def fetch(src, dst):
        vo = np.arange(64) * 4
        if src + KWIN > room + 4:
            src = min(src, room)
            vo = np.minimum(vo, room - src)
        assert src + int(vo.max()) + 4 <= in_len
        pending.append((dst, np.concatenate([cont[src + v:src + v + 4] for v in vo])))

    def wait(keep):
        while len(pending) > keep:
            op = pending.pop(0)
            if op is not None:
                lds[op[0]:op[0] + len(op[1])] = op[1]

    pay, nwin = off + 4 * NL, (plen + KWIN - 1) // KWIN

    cnt = {"hist": [0] * AHEAD, "cur": 0}

    def issue(w):
        if w % S == 0:  # the copy of slot 0 first, as the kernel does
            fetch(pay + w * KWIN, OB + S * KWIN)
            cnt["cur"] += 1
        fetch(pay + w * KWIN, OB + (w % S) * KWIN)
        cnt["hist"] = cnt["hist"][1:] + [cnt["cur"]]
        cnt["cur"] = 0

    fetch(off, 0)
    for w in range(min(S, nwin)):
        issue(w)
    wait(AHEAD if nwin >= S else 0)
    cnt["hist"], cnt["cur"] = [0] * AHEAD, 0
    L = 1 << l
    live = np.arange(64) < NL
    x = np.frombuffer(lds[:256].tobytes(), "<u4").astype(np.int64).copy()
    x[~live] = L
    SPB = OB // (NL * OW)
    E = len(f) - 1
    full, steps = nsym // NL, (nsym + NL - 1) // NL
    out = np.zeros(nsym, np.int64)
    st = {"bpos": 0, "kw": 0, "wend": KWIN, "t": 0, "x": x}

    def step(act):
        x = st["x"]
        slot = x & (M - 1)
        sym = slot2sym[slot]
        x = np.where(act, f[sym] * (x >> k) + slot - cum[sym], x)
        base = OB + (st["bpos"] & (S * KWIN - 1))
        ne = act & (sym == E) if esc else np.zeros(64, bool)
        if R == 16:
            n1 = act & (x < L)
            if n1.any() or ne.any():
                at = base + 2 * (np.cumsum(n1) - n1 + np.cumsum(ne) - ne)
                v = lds[at].astype(np.int64) | (lds[at + 1].astype(np.int64) << 8)
                v1 = lds[at + 2].astype(np.int64) | (lds[at + 3].astype(np.int64) << 8)
                x = np.where(n1, (x << 16) | v, x)
                sym = np.where(ne, np.where(n1, v1, v), sym)
                st["bpos"] += 2 * int(n1.sum() + ne.sum())
        else:
            n1, n2 = act & (x < L), act & (x < (L >> 8))
            if n1.any() or ne.any():
                at = base + np.cumsum(n1) - n1 + np.cumsum(n2) - n2 + 2 * (np.cumsum(ne) - ne)
                b = [lds[at + q].astype(np.int64) for q in range(4)]
                x1 = (x << 8) | b[0]
                x2 = (x1 << 8) | b[1]
                x = np.where(n1, np.where(n2, x2, x1), x)
                nren = n1.astype(int) + n2.astype(int)
                raw = np.choose(nren, [(b[0] << 8) | b[1], (b[1] << 8) | b[2], (b[2] << 8) | b[3]])
                sym = np.where(ne, raw, sym)
                st["bpos"] += int(n1.sum() + n2.sum() + 2 * ne.sum())
        st["x"] = x
        t = st["t"]
        m = max(0, min(NL, nsym - t * NL))
        out[t * NL:t * NL + m] = np.where(act, sym, 0)[:m]
        st["t"] = t + 1
        if st["t"] % SPB == 0:
            pending.append(None)
            cnt["cur"] += 1

    def advance():
        while st["bpos"] >= st["wend"]:
            st["kw"] += 1
            st["wend"] += KWIN
            if st["kw"] + S - 1 < nwin:
                issue(st["kw"] + S - 1)
                wait(min(AHEAD + cnt["cur"] + sum(cnt["hist"]), AHEAD + 6))
            else:
                wait(0)

    while st["t"] + TB <= full:
        advance()
        for _ in range(TB):
            step(live)
    advance()
    while st["t"] < full:
        step(live)
    if st["t"] < steps:
        step(np.arange(64) < nsym - st["t"] * NL)
    wait(0)
    return out, bool((st["x"] == L).all() and st["bpos"] == plen)


CASES = [  # k, r, l, N, C, n, zipf s (small s: high entropy, many windows per step)
    (14, 16, 16, 64, 4096, 4096 * 3 + 77, 1.1),
    (14, 16, 16, 64, 16384, 16384 + 1000, 0.05),
    (12, 8, 23, 64, 8192, 8192 + 63, 0.01),
    (14, 16, 16, 64, 1024, 5 * 1024 + 992, 1.1),
    (14, 16, 16, 64, 64, 64 * 7 + 1, 1.0),
    (10, 8, 23, 64, 2048, 5000, 3.0),
    (14, 16, 16, 32, 2048, 3 * 2048 + 31 * 32 + 17, 1.1),
    (12, 8, 23, 32, 4096, 4096 + 5, 0.01),
    (14, 16, 16, 32, 8192, 8192, 0.05),
]


@pytest.mark.parametrize("geometry", [(8, 4, 1024), (4, 2, 512)], ids=["S8", "S4"])
@pytest.mark.parametrize("case", CASES, ids=[f"k{c[0]}-r{c[1]}-N{c[3]}-C{c[4]}-n{c[5]}-s{c[6]}"
                                             for c in CASES])
def test_ring_schedule_decodes_oracle_containers(case, geometry):
    k, r, l, N, C, n, s = case
    S, TB, OB = geometry
    rng = np.random.default_rng(n + k)
    syms = rng.choice(256, size=n, p=datagen.zipf_probs(256, s)).astype(np.uint8)
    f = oracle.quantize(np.bincount(syms, minlength=256).astype(np.uint64), k)
    cont = oracle.encode(f, syms, k, r, l, N, C)
    f = np.asarray(f, np.int64)
    nch = (n + C - 1) // C
    for c in range(nch):
        out, ok = model_decode_chunk(cont, nch, c, C, n, k, l, r, f, N, rng, S=S, TB=TB, OB=OB)
        assert ok, (c, "end check")
        assert (out == syms[c * C:c * C + C]).all(), c


# lookup output (2 or 4 bytes per symbol: more output stores per window) and
# escape coding (up to 4 digit bytes per coder and step: a wider wait)
MORE = [  # kind, k, r, l, N, C, n, zipf s
    ("lut2", 14, 16, 16, 64, 4096, 4096 * 2 + 77, 0.05),
    ("lut4", 12, 8, 23, 64, 8192, 8192 + 63, 0.01),
    ("lut4", 14, 16, 16, 32, 2048, 2 * 2048 + 31 * 32 + 17, 0.05),
    ("esc", 12, 16, 16, 64, 4096, 4096 * 2 + 77, 0.3),
    ("esc", 12, 8, 23, 64, 8192, 8192 + 63, 0.3),
    ("esc", 13, 8, 23, 32, 4096, 4096 + 5, 0.3),
    ("esc", 12, 16, 16, 32, 2048, 2 * 2048 + 31 * 32 + 17, 0.3),
    # nearly every value escapes: steps read close to 4 bytes per coder
    ("esc95", 12, 16, 16, 64, 8192, 8192 * 2 + 77, 0.3),
    ("esc95", 12, 8, 23, 64, 8192, 8192 + 63, 0.01),
]


@pytest.mark.parametrize("geometry", [(8, 4, 1024), (4, 2, 512)], ids=["S8", "S4"])
@pytest.mark.parametrize("case", MORE, ids=[f"{c[0]}-k{c[1]}-r{c[2]}-N{c[4]}-C{c[5]}-n{c[6]}"
                                            for c in MORE])
def test_ring_schedule_lookup_and_escape(case, geometry):
    kind, k, r, l, N, C, n, s = case
    S, TB, OB = geometry
    rng = np.random.default_rng(n + k + r)
    if kind.startswith("esc"):
        # 16-bit values: a 255-symbol table plus the escape; about 30% (95%)
        # of the values escape
        v = rng.choice(255, size=n, p=datagen.zipf_probs(255, s)).astype(np.uint16)
        wild = rng.random(n) < (0.95 if kind == "esc95" else 0.3)
        v[wild] = rng.integers(0, 65536, int(wild.sum()))
        cnt = np.bincount(np.minimum(v, 255), minlength=256).astype(np.uint64)
        f = oracle.quantize(cnt, k)
        cont = oracle.encode(f, v, k, r, l, N, C, escape=True)
        want, OW = v, 2
    else:
        want = rng.choice(256, size=n, p=datagen.zipf_probs(256, s)).astype(np.uint8)
        f = oracle.quantize(np.bincount(want, minlength=256).astype(np.uint64), k)
        cont = oracle.encode(f, want, k, r, l, N, C)
        OW = int(kind[3])
    f = np.asarray(f, np.int64)
    nch = (n + C - 1) // C
    for c in range(nch):
        out, ok = model_decode_chunk(cont, nch, c, C, n, k, l, r, f, N, rng, S=S, TB=TB, OB=OB,
                                     OW=OW, esc=kind.startswith("esc"))
        assert ok, (c, "end check")
        assert (out == want[c * C:c * C + C]).all(), c
