"""Host model of the fast decoder's stream schedule (CPU).

The N = 32/64 decode kernel copies a chunk's digit stream into an 8-slot LDS
ring of 256-byte windows with direct-to-LDS loads issued up to seven windows
ahead, and waits with `s_waitcnt vmcnt(5)` (or 0 near the end) whenever its
read position enters a new window.  This model replays that schedule lane by
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

KWIN, KSLOTS = 256, 8


def model_decode_chunk(cont, nch, chunk, C, n, k, l, R, f, NL, rng, OB=1024):
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
    lds = rng.integers(0, 256, OB + (KSLOTS + 1) * KWIN, dtype=np.uint8)
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

    def issue(w):
        fetch(pay + w * KWIN, OB + (w % KSLOTS) * KWIN)
        if w % KSLOTS == 0:
            fetch(pay + w * KWIN, OB + KSLOTS * KWIN)

    fetch(off, 0)
    for w in range(min(KSLOTS, nwin)):
        issue(w)
    wait(5 if nwin >= KSLOTS else 0)
    L = 1 << l
    live = np.arange(64) < NL
    x = np.frombuffer(lds[:256].tobytes(), "<u4").astype(np.int64).copy()
    x[~live] = L
    SPB = OB // NL
    full, steps = nsym // NL, (nsym + NL - 1) // NL
    out = np.zeros(nsym, np.int64)
    st = {"bpos": 0, "kw": 0, "wend": KWIN, "t": 0, "x": x}

    def step(act):
        x = st["x"]
        slot = x & (M - 1)
        sym = slot2sym[slot]
        x = np.where(act, f[sym] * (x >> k) + slot - cum[sym], x)
        base = OB + (st["bpos"] & (KSLOTS * KWIN - 1))
        if R == 16:
            n1 = act & (x < L)
            if n1.any():
                at = base + 2 * (np.cumsum(n1) - n1)
                v = lds[at].astype(np.int64) | (lds[at + 1].astype(np.int64) << 8)
                x = np.where(n1, (x << 16) | v, x)
                st["bpos"] += 2 * int(n1.sum())
        else:
            n1, n2 = act & (x < L), act & (x < (L >> 8))
            if n1.any():
                at = base + np.cumsum(n1) - n1 + np.cumsum(n2) - n2
                x1 = (x << 8) | lds[at].astype(np.int64)
                x2 = (x1 << 8) | lds[at + 1].astype(np.int64)
                x = np.where(n1, np.where(n2, x2, x1), x)
                st["bpos"] += int(n1.sum() + n2.sum())
        st["x"] = x
        t = st["t"]
        m = max(0, min(NL, nsym - t * NL))
        out[t * NL:t * NL + m] = np.where(act, sym, 0)[:m]
        st["t"] = t + 1
        if st["t"] % SPB == 0:
            pending.append(None)

    def advance():
        while st["bpos"] >= st["wend"]:
            st["kw"] += 1
            st["wend"] += KWIN
            if st["kw"] + KSLOTS - 1 < nwin:
                issue(st["kw"] + KSLOTS - 1)
                wait(5)
            else:
                wait(0)

    while st["t"] + 4 <= full:
        advance()
        for _ in range(4):
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


@pytest.mark.parametrize("case", CASES, ids=[f"k{c[0]}-r{c[1]}-N{c[3]}-C{c[4]}-n{c[5]}-s{c[6]}"
                                             for c in CASES])
def test_ring_schedule_decodes_oracle_containers(case):
    k, r, l, N, C, n, s = case
    rng = np.random.default_rng(n + k)
    syms = rng.choice(256, size=n, p=datagen.zipf_probs(256, s)).astype(np.uint8)
    f = oracle.quantize(np.bincount(syms, minlength=256).astype(np.uint64), k)
    cont = oracle.encode(f, syms, k, r, l, N, C)
    f = np.asarray(f, np.int64)
    nch = (n + C - 1) // C
    for c in range(nch):
        out, ok = model_decode_chunk(cont, nch, c, C, n, k, l, r, f, N, rng)
        assert ok, (c, "end check")
        assert (out == syms[c * C:c * C + C]).all(), c
