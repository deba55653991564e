"""Host model of the segment decoder's stream schedule (CPU).

The N = 32/64 decoder codes 64 / N chunks per wave ("segments": lanes
0-31 and 32-63 with N = 32).  Each segment copies its chunk's digit stream
into its own S-slot LDS ring of 256-byte windows with direct-to-LDS loads
issued up to S - 1 windows ahead; every vector-memory operation of the wave
is numbered, and entering a window waits until at most (issued - number of
the newest window the next test block may read) operations are pending.
This model replays that schedule lane by lane on the oracle's containers:
loads land only when a wait guarantees them (until then their ring bytes
hold random garbage), output stores count as operations, the refill reads
use the kernel's addressing (one prefix count over the whole wave, the upper
segment's lanes moved to their own ring by a per-lane offset, 32-bit
wrap-around included), and every read must stay inside its own segment's
ring.  It decodes correctly only if no read touches a window that may still
be in flight.
"""
import numpy as np
import pytest

import datagen
import oracle

KWIN = 256
U32 = 0xFFFFFFFF


def model_decode_pair(cont, nch, chunk0, C, n, k, l, R, f, NL, rng, S=8, TB=4, OB=1024, bf=False):
    SEG = 64 // NL
    DB = R // 8
    MAXB = 2 * NL
    RES = 1 + (TB * MAXB + KWIN - 1) // KWIN
    RING = (S + 1) * KWIN
    DMASK = S * KWIN // DB - 1
    WD = KWIN // DB
    OBS = OB // SEG
    SPB = OBS // NL  # one output byte per symbol
    PIECE = OB // 64
    RBD = RING // DB
    assert SPB % TB == 0 and RES < S
    in_len = cont.size
    M = 1 << k
    L = 1 << l
    cum = np.concatenate([[0], np.cumsum(f)])
    slot2sym = np.repeat(np.arange(len(f)), f)
    room = (in_len - 4) & ~3
    data0 = (32 + 16 * nch + 15) & ~15
    lds = rng.integers(0, 256, OB + SEG * RING, dtype=np.uint8)
    pending = []  # oldest first: (dst, bytes) for loads, None for stores
    st = {"nops": 0}
    wseq = {}
    lane = np.arange(64)
    seg = lane // NL
    jl = lane % NL

    pay, nsym, nwin, wfast, ndig = [0] * SEG, [0] * SEG, [0] * SEG, [0] * SEG, [0] * SEG
    exists = [False] * SEG
    for s in range(SEG):
        c = chunk0 + s
        if c >= nch:
            continue
        de = 32 + 16 * c
        off = int(np.frombuffer(cont[de:de + 8].tobytes(), "<u8")[0])
        ln = int(np.frombuffer(cont[de + 8:de + 12].tobytes(), "<u4")[0])
        assert off % 16 == 0 and off >= data0 and off + ln <= in_len and ln >= 4 * NL
        nsym[s] = min(n - c * C, C)
        plen = ln - 4 * NL
        pay[s] = off + 4 * NL
        nwin[s] = (plen + KWIN - 1) // KWIN
        ndig[s] = plen // DB
        wfast[s] = (room + 4 - pay[s] - KWIN) // KWIN + 1 if room + 4 >= pay[s] + KWIN else 0
        exists[s] = True

    def dma(src_addrs, dst, active):
        # lane i (active) moves 4 bytes at src_addrs[i] to LDS dst + 4 i
        data = []
        for i in range(64):
            if active[i]:
                a = int(src_addrs[i])
                assert 0 <= a and a + 4 <= in_len, "load outside the container"
                data.append((dst + 4 * i, cont[a:a + 4].copy()))
        pending.append(data)
        st["nops"] += 1

    def fetch(src, dst, fast):
        vo = lane * 4
        if not fast and src + KWIN > room + 4:
            src = min(src, room)
            vo = np.minimum(vo, room - src)
        dma(src + vo, dst, np.ones(64, bool))

    def issue(s, w):
        src = pay[s] + w * KWIN
        ring = OB + s * RING
        slot = w % S
        if slot == 0:
            fetch(src, ring + S * KWIN, w < wfast[s])
        fetch(src, ring + slot * KWIN, w < wfast[s])
        wseq[(s, slot)] = st["nops"]

    def wait(keep):
        keep = min(keep, 31)
        while len(pending) > keep:
            op = pending.pop(0)
            if op is not None:
                for dst, b in op:
                    lds[dst:dst + 4] = b

    def need(s, w):
        wait(st["nops"] - wseq[(s, w % S)])

    state_seq = 0
    for s in range(SEG):
        if exists[s]:
            dma(pay[s] - 4 * NL - 4 * NL * s + lane * 4, 0, seg == s)
            state_seq = st["nops"]
    for w in range(S):
        for s in range(SEG):
            if w < nwin[s]:
                issue(s, w)
    q = state_seq
    for s in range(SEG):
        if nwin[s]:
            q = max(q, wseq[(s, min(nwin[s], RES) - 1)])
    wait(st["nops"] - q)
    live = np.array([exists[s] for s in seg])
    x = np.frombuffer(lds[:256].tobytes(), "<u4").astype(np.int64).copy()
    x[~live] = L
    pos = [0] * SEG
    kw = [0] * SEG
    wend = [WD] * SEG
    vhi = np.where(lane >= NL, U32, 0) if SEG == 2 else np.zeros(64, np.int64)
    out = {s: np.zeros(nsym[s], np.int64) for s in range(SEG)}
    ob = np.zeros(OB, np.int64)  # output block (symbols)

    def mbcnt(m, acc):  # count of set lanes below each lane, plus acc (mod 2^32)
        return (np.cumsum(m) - m + acc) & U32

    def pos_off(lower):
        if SEG == 1:
            return np.zeros(64, np.int64)
        d = (RBD + (pos[1] & DMASK) - (pos[0] & DMASK) - lower) & U32
        return vhi & d

    def read(addr_bytes, nbytes=1):
        # LDS byte reads of every lane: each inside its own segment's ring
        out_ = []
        for i in range(64):
            a = int(addr_bytes[i]) & U32
            lo = OB + seg[i] * RING
            assert lo <= a and a + nbytes <= lo + RING, ("read outside the ring", i, a)
            out_.append(int.from_bytes(lds[a:a + nbytes].tobytes(), "little"))
        return np.array(out_, np.int64)

    def step(act):
        nonlocal x
        slot = x & (M - 1)
        sym = slot2sym[slot]
        xd = np.where(act, f[sym] * (x >> k) + slot - cum[sym], x)
        base0 = OB + DB * (pos[0] & DMASK)
        if R == 16:
            n1 = act & (xd < L)
            m1 = n1.astype(np.int64)
            lo1, hi1 = int(m1[:32].sum()), int(m1[32:].sum())
            if n1.any():
                idx = mbcnt(m1, pos_off(lo1))
                v = read(base0 + 2 * idx, 2)
                xd = np.where(n1, (xd << 16) | v, xd)
                if SEG == 1:
                    pos[0] += lo1 + hi1
                else:
                    pos[0] += lo1
                    pos[1] += hi1
        else:
            n1, n2 = act & (xd < L), act & (xd < (L >> 8))
            m1, m2 = n1.astype(np.int64), n2.astype(np.int64)
            lo1, hi1 = int(m1[:32].sum()), int(m1[32:].sum())
            lo2, hi2 = int(m2[:32].sum()), int(m2[32:].sum())
            if n1.any():
                if bf:
                    if SEG == 2:
                        o2 = vhi & ((RBD + (pos[1] & DMASK) + hi1 - (pos[0] & DMASK) - lo1 - lo2) & U32)
                        r2 = base0 + lo1
                    else:
                        o2 = np.zeros(64, np.int64)
                        r2 = base0 + lo1 + hi1
                    b0 = read(base0 + mbcnt(m1, pos_off(lo1)))
                    b1 = read(r2 + mbcnt(m2, o2))
                else:
                    q = base0 + ((mbcnt(m1, pos_off(lo1 + lo2)) + mbcnt(m2, 0)) & U32)
                    b0, b1 = read(q), read(q + 1)
                x1 = (xd << 8) | b0
                x2 = (x1 << 8) | b1
                xd = np.where(n1, np.where(n2, x2, x1), xd)
                if SEG == 1:
                    pos[0] += lo1 + hi1 + lo2 + hi2
                else:
                    pos[0] += lo1 + lo2
                    pos[1] += hi1 + hi2
        x = xd
        return sym

    def advance():
        for s in range(SEG):
            while pos[s] >= wend[s]:
                kw[s] += 1
                wend[s] += WD
                if kw[s] + S - 1 < nwin[s]:
                    issue(s, kw[s] + S - 1)
                w = min(kw[s] + RES - 1, nwin[s] - 1)
                if kw[s] < nwin[s]:
                    need(s, w)

    full = min(nsym[s] // NL for s in range(SEG) if exists[s])
    steps = max((nsym[s] + NL - 1) // NL for s in range(SEG) if exists[s])
    t = 0

    def store_piece(tb, lanes_mask):
        for i in range(64):
            if lanes_mask[i]:
                s = seg[i]
                start = tb * NL + jl[i] * PIECE
                vals = ob[s * OBS + jl[i] * PIECE: s * OBS + (jl[i] + 1) * PIECE]
                m = min(PIECE, nsym[s] - start)
                out[s][start:start + m] = vals[:m]

    while t + SPB <= full:
        for b in range(SPB // TB):
            advance()
            for i in range(TB):
                sym = step(live)
                tt = (b * TB + i)
                for ln in range(64):
                    ob[seg[ln] * OBS + tt * NL + jl[ln]] = sym[ln]
        t += SPB
        store_piece(t - SPB, live)
        pending.append(None)
        st["nops"] += 1

    def tail_flush(tb):
        valid = np.array([max(0, min(PIECE, nsym[seg[i]] - (tb * NL + jl[i] * PIECE))) if live[i] else 0
                          for i in range(64)])
        if (valid == PIECE).any():
            store_piece(tb, valid == PIECE)
            pending.append(None)
            st["nops"] += 1
        part = (valid != 0) & (valid != PIECE)
        if part.any():
            wait(0)
            store_piece(tb, part)

    while t < steps:
        advance()
        act = np.array([live[i] and t * NL + jl[i] < nsym[seg[i]] for i in range(64)])
        sym = step(act)
        tt = t % SPB
        for ln in range(64):
            if act[ln]:
                ob[seg[ln] * OBS + tt * NL + jl[ln]] = sym[ln]
        t += 1
        if t % SPB == 0:
            tail_flush(t - SPB)
    if t % SPB != 0:
        tail_flush(t - t % SPB)
    wait(0)
    ok = {}
    for s in range(SEG):
        if exists[s]:
            lanes = seg == s
            ok[s] = bool((x[lanes] == L).all() and pos[s] == ndig[s])
    return out, ok


CASES = [  # k, r, l, N, C, n, zipf s, order
    (14, 16, 16, 32, 4096, 4096 * 3 + 77, 1.1, "df"),
    (14, 16, 16, 32, 8192, 8192 * 2, 0.05, "df"),
    (12, 8, 23, 32, 4096, 4096 * 3 + 5, 0.01, "df"),
    (12, 8, 23, 32, 4096, 4096 * 2 + 4000, 0.3, "bf"),
    (11, 8, 23, 32, 2048, 2048 * 4 + 33, 3.0, "bf"),
    (14, 16, 16, 32, 1024, 1024 * 5 + 992, 1.1, "df"),
    (14, 16, 16, 32, 2048, 2048 + 31, 1.1, "df"),  # the second chunk has 31 symbols
    (14, 16, 16, 64, 4096, 4096 * 3 + 77, 1.1, "df"),
    (12, 8, 23, 64, 8192, 8192 + 63, 0.01, "df"),
    (12, 8, 23, 64, 8192, 8192 + 1000, 0.3, "bf"),
    (14, 16, 16, 64, 64, 64 * 7 + 1, 1.0, "df"),
]


@pytest.mark.parametrize("geometry", [(8, 4, 1024), (4, 2, 512)], ids=["S8", "S4"])
@pytest.mark.parametrize("case", CASES, ids=[f"k{c[0]}-r{c[1]}-N{c[3]}-C{c[4]}-n{c[5]}-s{c[6]}-{c[7]}"
                                             for c in CASES])
def test_segment_schedule_decodes_oracle_containers(case, geometry):
    k, r, l, N, C, n, s, order = case
    S, TB, OB = geometry
    rng = np.random.default_rng(n + k + N)
    syms = rng.choice(256, size=n, p=datagen.zipf_probs(256, s)).astype(np.uint8)
    f = oracle.quantize(np.bincount(syms, minlength=256).astype(np.uint64), k)
    cont = oracle.encode(f, syms, k, r, l, N, C, order=order)
    f = np.asarray(f, np.int64)
    nch = (n + C - 1) // C
    SEG = 64 // N
    for c0 in range(0, nch, SEG):
        out, ok = model_decode_pair(cont, nch, c0, C, n, k, l, r, f, N, rng, S=S, TB=TB, OB=OB,
                                    bf=order == "bf")
        for sg, good in ok.items():
            c = c0 + sg
            assert good, (c, "end check")
            assert (out[sg] == syms[c * C:c * C + C]).all(), c


def test_segment_schedule_fails_with_the_wrong_coder_count():
    """A container coded with 64 coders per chunk, read as if it had 32 (the
    chunk geometry agrees, the states and digits do not): the end check
    fails, as it must."""
    k, r, l, C, n = 14, 16, 16, 4096, 4096 * 2
    rng = np.random.default_rng(3)
    syms = rng.choice(256, size=n, p=datagen.zipf_probs(256, 1.1)).astype(np.uint8)
    f = oracle.quantize(np.bincount(syms, minlength=256).astype(np.uint64), k)
    cont = oracle.encode(f, syms, k, r, l, 64, C)
    _, ok = model_decode_pair(cont, 2, 0, C, n, k, l, r, np.asarray(f, np.int64), 32, rng)
    assert not all(ok.values())
