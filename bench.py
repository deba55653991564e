#!/usr/bin/env python3
"""Benchmark of interleaved streaming rANS on one MI355X.

Default line (the metric: decode/encode GB/s, batched vs plain, p99 decode
latency): the radix/precision sweep -- 84 feasible points of 64 MiB of
symbol bytes (alphabets 2, 16, 256 as uint8 and 4096 as uint16; M = 2^11 or
2^15; one dominant symbol, Zipf(1.1) or near-uniform; byte or 16-bit
digits; 32 or 64 coders per chunk), each point with its own table -- coded
by batched persistent launches, one per group of points sharing (k, r, l,
w, N).  One step = batched encode + batched decode of every point (inputs
resident in HBM; tables built once before timing, as the paper's static
order-0 model is fixed once per input).

value = uncompressed bytes encoded-and-decoded per second (GB = 1e9 B).
Also reported: the batched kernels' roofline fractions from HIP events
recorded on the launch stream, one plain launch per point at its own best
chunk size (the speedup), the 4096-stream batch against plain per-stream
calls, the serving loop's p50/p99 latency, the plain 256 MiB round trip,
and the CPU oracle on a bounded sample (one thread and every host thread).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, AMD published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of every source file the kernels are built from: a traffic figure
    measured on other sources does not describe these kernels."""
    import hashlib
    d = os.path.join(ROOT, "paper_1402_3392_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".h", ".hip", ".cpp")):
            with open(os.path.join(d, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` on this workload, from the committed
    counter summary (profiles/traffic.txt: FETCH_SIZE and WRITE_SIZE scaled by
    the copy-kernel calibration), or None when it was taken on other sources."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    src = kernel_source_hash()
    for line in open(path):
        if line.startswith("#") or "=" not in line:
            continue
        kv = dict(tok.split("=", 1) for tok in line.split())
        if kv.get("kernel") == kernel and kv.get("source") == src:
            return int(kv["traffic_bytes"])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size-log2", type=int, default=28, help="symbols per buffer (log2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "roundtrip", "batched", "sweep", "serving", "dequant", "escape",
                             "prefix"],
                    help="headline: the metric's line (the radix/precision sweep encoded and decoded "
                         "by batched launches, with the 4096-stream batch, serving and the round trip "
                         "beside it); "
                         "roundtrip: 3 x 256 MiB encode+decode by the plain entry points; "
                         "batched: 4096 uneven streams, one persistent launch vs plain calls; "
                         "sweep: radix/precision/alphabet sweep, batched vs plain decode; "
                         "serving: Poisson request loop, p50/p99 latency; "
                         "dequant: decode fused with a codebook lookup vs decode + gather; "
                         "escape: escape coding with raw digits vs the clipped stream; "
                         "prefix: prefix-code family multiplexed by the decoder read rule vs rANS")
    ap.add_argument("--streams", type=int, default=4096, help="batched: number of streams")
    ap.add_argument("--requests", type=int, default=1000, help="serving: requests per rate")
    ap.add_argument("--points", default="", help="sweep: comma-separated point indices")
    ap.add_argument("--grouped", action="store_true",
                    help="sweep: batch the points sharing (k, r, l, w, N) into one launch each")
    ap.add_argument("--chunk-syms", type=int, default=0,
                    help="sweep: fixed chunk size in symbols (0: autotune per point)")
    ap.add_argument("--order", default="df", choices=["df", "bf"],
                    help="sweep: digit order within a step, depth-first or breadth-first "
                         "(differs only with byte digits)")
    ap.add_argument("--source-hash", action="store_true", help="print the kernels' source hash")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1402_3392_amd", "tune_mi355x.txt"),
                    help="autotuner cache file (results measured on MI355X; '' disables it)")
    ap.add_argument("--headline-only", action="store_true",
                    help="headline: only the sweep line (no 4096-stream, serving, round-trip extras)")
    ap.add_argument("--groups", default="",
                    help="headline: only these sweep groups (comma-separated indices in (k, r, l, w, N) "
                         "order; for profiling one kernel instance)")
    ap.add_argument("--batched-only", action="store_true",
                    help="headline: only the timed batched steps and their roofline (no per-group "
                         "times, plain launches or extras; the profiling passes run this)")
    return ap.parse_args()


def copy_probe():
    """A plain copy of known size: what FETCH_SIZE / WRITE_SIZE read for
    1 GiB in and 1 GiB out calibrates the counters used for traffic."""
    import torch
    src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        dst.copy_(src)
    torch.cuda.synchronize()
    gbps = 10 * 2 * src.numel() / (time.perf_counter() - t0) / 1e9
    print(json.dumps({"copy_probe_bytes": src.numel(), "copy_gbps": round(gbps, 1)}), flush=True)


def cpu_baseline(work, threads):
    """The oracle, as it is, on a bounded sample: the first 64 MiB of each
    buffer, encoded and decoded with `threads` threads over chunks."""
    import numpy as np

    import oracle
    sample = 64 << 20
    tot_bytes, tot_s = 0, 0.0
    for w, f in work:
        s = np.ascontiguousarray(w.syms[:sample])
        k, r, l, _, N, C = w.params.astuple()
        t0 = time.perf_counter()
        c = oracle.encode(f, s, k, r, l, N, C, threads=threads)
        t1 = time.perf_counter()
        d = oracle.decode(f, c, threads=threads)
        t2 = time.perf_counter()
        assert (d == s).all()
        tot_bytes += s.nbytes
        tot_s += t2 - t0
    return {"value": round(tot_bytes / tot_s / 1e9, 4), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {sample >> 20} MiB of each of the 3 buffers, encode+decode, "
                      f"{threads} threads over 64 KiB chunks"}


class DevPool:
    """Carves 256-byte aligned pieces out of one device allocation."""

    def __init__(self, nbytes):
        import torch
        self.buf = torch.empty(nbytes + 4096, dtype=torch.uint8, device="cuda")
        self.base = int(self.buf.data_ptr())
        self.off = 0

    def take(self, nbytes):
        a = self.base + self.off
        self.off += (max(nbytes, 1) + 255) // 256 * 256
        assert self.off <= self.buf.numel(), "pool exhausted"
        return a

    def view(self, addr, nbytes):
        o = addr - self.base
        return self.buf[o:o + nbytes]


def timed(fn, reps):
    """Median wall time (s) of fn() over reps runs on the current stream,
    measured with events recorded on that stream."""
    import torch
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def base_result(metric, value, unit, args, config, higher=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": higher, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic", "config": config}


def run_batched(args, emit=True):
    """Many independent streams of uneven length, each with its own table:
    one persistent batched launch (a graph replay; interleave factor, chunk
    size and launch shape from the autotuner on the whole batch) against one
    plain rans_decode_async / rans_encode_async call per stream on the same
    stream, the plain calls at the chunk size that suits them best."""
    import numpy as np
    import torch

    import datagen
    import paper_1402_3392_amd as lr

    K, R, L = 14, 16, 16
    log(f"generating {args.streams} streams")
    data = datagen.dirichlet_streams(nstreams=args.streams)
    sizes = [int(s.size) for s, _ in data]
    total = sum(sizes)
    log(f"{total / 2**30:.2f} GiB in {len(data)} streams; building tables")
    tables = [lr.rans_tables_build(datagen.counts(s, 256), K) for s, _ in data]

    # 64 coders and the smallest chunk size bound every container the tuner may choose
    caps = [lr.rans_encode_bound(n, lr.rans_params.make(K, R, L, 1, 64, 4096)) for n in sizes]
    pool = DevPool(sum((n + 255) // 256 * 256 for n in sizes) * 2 + sum(caps) + 256 * len(sizes))
    d_in = [pool.take(n) for n in sizes]
    for a, (s, _) in zip(d_in, data):
        pool.view(a, s.size).copy_(torch.from_numpy(s))
    # chunk size and launch shape from the autotuner, timed on the whole batch
    tune_jobs = lr.make_jobs((tables[i], d_in[i], sizes[i], 0, 0, 0, 0) for i in range(len(data)))
    log("autotuning on the batch")
    tune = lr.rans_autotune_batch(tune_jobs, len(data), lr.rans_params.make(K, R, L, 1, 0, 65536),
                                  args.tune_cache or None)
    C, N = int(tune["chunk_syms"]), int(tune["interleave"])
    params = lr.rans_params.make(K, R, L, 1, N, C)
    d_cont = [pool.take(c) for c in caps]
    d_dec = [pool.take(n) for n in sizes]
    lens = torch.zeros(len(data), dtype=torch.int64, device="cuda")
    st = torch.zeros(len(data), dtype=torch.int32, device="cuda")
    enc_jobs = lr.make_jobs((tables[i], d_in[i], sizes[i], d_cont[i], caps[i],
                             int(lens.data_ptr()) + 8 * i, int(st.data_ptr()) + 4 * i)
                            for i in range(len(data)))
    log("batched encode (containers for decode)")
    lr.rans_encode_batch(enc_jobs, len(data), params)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0, "batched encode failed"
    clen = [int(v) for v in lens.cpu().tolist()]
    headers = [bytes(pool.view(d_cont[i], 32).cpu().numpy().tobytes()) for i in range(len(data))]
    comp = sum(clen)
    dec_jobs = lr.make_jobs((tables[i], d_cont[i], clen[i], d_dec[i], sizes[i],
                             int(lens.data_ptr()) + 8 * i, int(st.data_ptr()) + 4 * i)
                            for i in range(len(data)))
    lens_enc = lens.clone()

    def batched_decode():
        lr.rans_decode_batch(dec_jobs, len(data), params)

    def batched_encode():
        lr.rans_encode_batch(enc_jobs, len(data), params)

    def plain_decode():
        for i in range(len(data)):
            lr.rans_decode_async(tables[i], pool.view(d_cont[i], clen[i]), clen[i], headers[i],
                                 pool.view(d_dec[i], sizes[i]), sizes[i], st[i:i + 1])

    def plain_encode():
        for i in range(len(data)):
            lr.rans_encode_async(tables[i], params, pool.view(d_in[i], sizes[i]), sizes[i],
                                 pool.view(d_cont[i], caps[i]), caps[i], lens[i:i + 1], st[i:i + 1])

    reps = max(3, args.steps)
    res = {}
    lr.rans_timing_reset()
    lr.rans_timing_enable(True)
    for name, fn in [("batched_decode", batched_decode), ("batched_encode", batched_encode)]:
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        st.zero_()
        t = timed(fn, reps)
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0, f"{name}: status {st.nonzero()[:4].tolist()}"
        if name.endswith("decode"):
            for i in range(0, len(data), max(1, len(data) // 64)):
                assert torch.equal(pool.view(d_dec[i], sizes[i]), pool.view(d_in[i], sizes[i])), name
        else:
            assert torch.equal(lens, lens_enc), name
        res[name] = t
        log(f"{name}: {t * 1e3:.2f} ms, {total / t / 1e9:.1f} GB/s")
    lr.rans_timing_enable(False)
    kt = {name: lr.rans_timing_read(kind) for name, kind in
          (("decode", lr.RANS_KERNEL_BATCH_DECODE), ("encode", lr.RANS_KERNEL_BATCH_ENCODE))}
    lr.rans_timing_reset()

    # plain per-stream calls at each candidate chunk size (and N = 64, 32):
    # the fastest decode and the fastest encode count as the plain baseline
    plain = {}
    for pn in (64, 32):
        for pc in (65536, 16384, 4096):
            pp = lr.rans_params.make(K, R, L, 1, pn, pc)

            def penc(pp=pp):
                for i in range(len(data)):
                    lr.rans_encode_async(tables[i], pp, pool.view(d_in[i], sizes[i]), sizes[i],
                                         pool.view(d_cont[i], caps[i]), caps[i], lens[i:i + 1], st[i:i + 1])
            st.zero_()
            penc()
            torch.cuda.synchronize()
            assert int(st.abs().sum()) == 0, "plain encode failed"
            plen = [int(v) for v in lens.cpu().tolist()]
            phdr = [bytes(pool.view(d_cont[i], 32).cpu().numpy().tobytes()) for i in range(len(data))]

            def pdec(plen=plen, phdr=phdr):
                for i in range(len(data)):
                    lr.rans_decode_async(tables[i], pool.view(d_cont[i], plen[i]), plen[i], phdr[i],
                                         pool.view(d_dec[i], sizes[i]), sizes[i], st[i:i + 1])
            te, td = timed(penc, 2), timed(pdec, 2)
            torch.cuda.synchronize()
            assert int(st.abs().sum()) == 0, "plain decode failed"
            plain[(pn, pc)] = (te, td)
            log(f"plain N={pn} C={pc}: encode {total / te / 1e9:.1f} GB/s, decode {total / td / 1e9:.1f} GB/s")
    best_dec = min(plain, key=lambda q: plain[q][1])
    best_enc = min(plain, key=lambda q: plain[q][0])
    res["plain_decode"], res["plain_encode"] = plain[best_dec][1], plain[best_enc][0]
    # the batched containers again (the plain runs overwrote them)
    lr.rans_encode_batch(enc_jobs, len(data), params)
    lr.rans_decode_batch(dec_jobs, len(data), params)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    alg = comp + total + 4 * 256 * len(data)
    dec_us = 1e3 * kt["decode"][1] / max(kt["decode"][0], 1)
    out = base_result("rANS decode/encode GB/s on 1 MI355X, batched vs plain; p99 decode latency",
                      round(total / res["batched_decode"] / 1e9, 3), "GB/s", args,
                      {"workload": f"{len(data)} uint8 streams, lengths 2^U(10,22) B "
                                   f"({total / 2**30:.2f} GiB), Dirichlet(alpha in 0.05..5) tables, "
                                   f"M=2^14, b=L=2^16, N={N}, C={C} (autotuned), batched decode"})
    out.update({
        "batched_decode_gbps": round(total / res["batched_decode"] / 1e9, 2),
        "plain_decode_gbps": round(total / res["plain_decode"] / 1e9, 2),
        "plain_decode_choice": {"N": best_dec[0], "C": best_dec[1]},
        "decode_speedup": round(res["plain_decode"] / res["batched_decode"], 2),
        "batched_encode_gbps": round(total / res["batched_encode"] / 1e9, 2),
        "plain_encode_gbps": round(total / res["plain_encode"] / 1e9, 2),
        "plain_encode_choice": {"N": best_enc[0], "C": best_enc[1]},
        "encode_speedup": round(res["plain_encode"] / res["batched_encode"], 2),
        "compression_ratio": round(comp / total, 4),
        "autotune": {k: (round(v, 2) if isinstance(v, float) else v) for k, v in tune.items()},
        "roofline": {"bound": "hbm", "kernel": "k_batch_decode64", "unit": "GB/s",
                     "achieved": round(alg / (dec_us * 1e-6) / 1e9, 1), "peak": HBM_PEAK_GBPS,
                     "frac": round(alg / (dec_us * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4),
                     "traffic": None, "avg_us": round(dec_us, 1),
                     "note": "events around each launch (planning kernel included)"},
    })
    if emit:
        print(json.dumps(out), flush=True)
    return out


def run_sweep(args):
    """Radix / precision / alphabet / entropy sweep: per point, GPU encode
    (container compared byte for byte with the oracle's), then plain and
    batched persistent decode of the oracle's container, timed."""
    import numpy as np
    import torch

    import datagen
    import oracle
    import paper_1402_3392_amd as lr

    pts = datagen.sweep_points()
    sel = [int(x) for x in args.points.split(",") if x] if args.points else range(len(pts))
    threads = min(16, os.cpu_count() or 1)
    cache = {}
    rows = []
    for idx in sel:
        p = pts[idx]
        key = (p["alphabet"], p["dist"])
        if key not in cache:
            cache.clear()
            cache[key] = datagen.sweep_data(p["alphabet"], p["dist"])[0]
        syms = cache[key]
        w = 1 if p["alphabet"] <= 256 else 2
        row = {"idx": idx, "alphabet": p["alphabet"], "dist": p["dist"], "k": p["k"], "r": p["r"],
               "l": p["l"], "N": p["N"], "order": args.order}
        if not p["feasible"]:
            row["status"] = "n/a (more symbols present than 2^k)"
            rows.append(row)
            log(json.dumps(row))
            continue
        counts = datagen.counts(syms, p["alphabet"])
        f = oracle.quantize(counts, p["k"])
        table = lr.rans_tables_build(counts, p["k"])
        d_syms = torch.from_numpy(syms.view(np.uint8)).cuda()
        if args.chunk_syms:
            C = args.chunk_syms
            cfg = lr.rans_batch_get_config()
            row.update(C=C, G=cfg["waves_per_group"], gpc=cfg["groups_per_cu"],
                       layout=cfg["table_layout"])
        else:
            # chunk size and batched launch shape from the autotuner, on this buffer
            tune = lr.rans_autotune(table, d_syms, syms.size,
                                    lr.rans_params.make(p["k"], p["r"], p["l"], w, 64, 65536 // w,
                                                        args.order))
            C = int(tune["chunk_syms"])
            row.update(C=C, G=int(tune["waves_per_group"]), gpc=int(tune["groups_per_cu"]),
                       layout=int(tune["table_layout"]))
        params = lr.rans_params.make(p["k"], p["r"], p["l"], w, p["N"], C, args.order)
        cont = oracle.encode(f, syms, p["k"], p["r"], p["l"], p["N"], C, threads=threads,
                             order=args.order)
        cap = lr.rans_encode_bound(syms.size, params)
        d_enc = torch.empty(cap, dtype=torch.uint8, device="cuda")
        nb = lr.rans_encode(table, params, d_syms, syms.size, d_enc, cap)
        row["encode_bit_exact"] = bool(nb == cont.size and np.array_equal(d_enc[:nb].cpu().numpy(), cont))
        d_cont = torch.from_numpy(cont).cuda()
        d_out = torch.empty(syms.size * w, dtype=torch.uint8, device="cuda")
        hdr = bytes(cont[:32].tobytes())
        st = torch.zeros(2, dtype=torch.int32, device="cuda")
        lens = torch.zeros(1, dtype=torch.int64, device="cuda")

        def plain():
            lr.rans_decode_async(table, d_cont, cont.size, hdr, d_out, syms.size, st[0:1])

        def enc():
            lr.rans_encode_async(table, params, d_syms, syms.size, d_enc, cap, lens, st[0:1])

        jobs = lr.make_jobs([(table, d_cont, cont.size, d_out, syms.size * w,
                              int(lens.data_ptr()), int(st.data_ptr()) + 4)])

        def batched():
            lr.rans_decode_batch(jobs, 1, params)

        nbytes = syms.size * w
        for name, fn in [("plain_decode", plain), ("batched_decode", batched), ("encode", enc)]:
            try:
                fn()
                torch.cuda.synchronize()
            except lr.RansError as e:
                row[name] = f"n/a ({e})"
                continue
            t = timed(fn, max(5, args.steps))
            row[name + "_gbps"] = round(nbytes / t / 1e9, 2)
            if name != "encode":
                row[name + "_ok"] = bool(torch.equal(d_out, d_syms)) and int(st.abs().sum()) == 0
                d_out.fill_(0)
            if name == "batched_decode":
                alg = cont.size + nbytes + 4 * p["alphabet"]
                row["batched_roofline_frac"] = round(alg / t / 1e9 / HBM_PEAK_GBPS, 4)
        row["ratio"] = round(cont.size / nbytes, 4)
        rows.append(row)
        log(json.dumps(row))
        table.close()
    ok = [r for r in rows if "batched_decode_gbps" in r]
    best = max((r["batched_decode_gbps"] for r in ok), default=0.0)
    out = base_result("rANS decode/encode GB/s on 1 MI355X, batched vs plain; p99 decode latency",
                      best, "GB/s", args,
                      {"workload": "64 MiB symbol bytes per point; alphabets 2/16/256/4096, "
                                   "M=2^11/2^15, p0=0.995 / Zipf(1.1) / near-uniform, "
                                   "(b,L)=(2^8,2^23)/(2^16,2^16), N=32/64, autotuned chunk size",
                                   "digit_order": args.order})
    out["points"] = rows
    print(json.dumps(out), flush=True)


def run_dequant(args):
    """Decode fused with a codebook lookup (a consumer in the same kernel):
    256 MiB of 8-bit quantisation codes of a normally distributed tensor,
    decoded straight to bf16 (or fp32) values, against the unfused pair
    decode-to-codes + a separate gather."""
    import numpy as np
    import torch

    import datagen
    import paper_1402_3392_amd as lr

    K, R, L, W, N, C = 14, 16, 16, 1, 64, 65536
    n = 1 << args.size_log2
    log(f"generating {n >> 20} MiB of Gaussian 8-bit codes")
    rng = np.random.Generator(np.random.PCG64(6001))
    syms = datagen.sample(datagen.gaussian_codes_probs(256, 24.0), n, rng)
    counts = datagen.counts(syms, 256)
    table = lr.rans_tables_build(counts, K)
    params = lr.rans_params.make(K, R, L, W, N, C)
    d_in = torch.from_numpy(syms).cuda()
    cap = lr.rans_encode_bound(n, params)
    d_cont = torch.empty(cap, dtype=torch.uint8, device="cuda")
    clen = lr.rans_encode(table, params, d_in, n, d_cont, cap)
    hdr = bytes(d_cont[:32].cpu().numpy().tobytes())
    vals = (torch.arange(256, dtype=torch.float32) - 128.0) / 64.0
    lut2 = vals.to(torch.bfloat16).cuda()
    lut4 = vals.cuda()
    out2 = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    out4 = torch.empty(n, dtype=torch.float32, device="cuda")
    codes = torch.empty(n, dtype=torch.uint8, device="cuda")
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    out_u = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    st = torch.zeros(4, dtype=torch.int32, device="cuda")

    def fused2():
        lr.rans_decode_lut_async(table, d_cont, clen, hdr, lut2, 2, out2, n, st[0:1])

    def fused4():
        lr.rans_decode_lut_async(table, d_cont, clen, hdr, lut4, 4, out4, n, st[1:2])

    def decode():
        lr.rans_decode_async(table, d_cont, clen, hdr, codes, n, st[2:3])

    def gather():
        torch.index_select(lut2, 0, idx.copy_(codes), out=out_u)

    def unfused():
        decode()
        gather()

    def copy():  # device copy of the bf16 output: 2n bytes read, 2n written
        out_u.copy_(out2)

    reps = max(5, args.steps)
    res = {}
    for name, fn in [("fused_bf16", fused2), ("fused_fp32", fused4), ("decode_codes", decode),
                     ("gather", gather), ("unfused_bf16", unfused), ("copy_bf16", copy)]:
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        res[name] = timed(fn, reps)
        log(f"{name}: {res[name] * 1e6:.1f} us")
    assert int(st.abs().sum()) == 0, f"status {st.tolist()}"
    ref = lut2[d_in.long()]
    assert torch.equal(out2.view(torch.int16), ref.view(torch.int16)), "fused bf16 output"
    assert torch.equal(out4, lut4[d_in.long()]), "fused fp32 output"
    assert torch.equal(out_u.view(torch.int16), ref.view(torch.int16)), "unfused output"
    t = res["fused_bf16"]
    alg = clen + 2 * n + 2 * 256 + 8 * (1 << K)
    # the best a separate gather pass could do: n bytes of codes in, 2n out,
    # at the rate of a plain device copy
    copy_rate = 4 * n / res["copy_bf16"]
    unfused_bound = res["decode_codes"] + 3 * n / copy_rate
    out = base_result("rANS decode fused with a codebook lookup, GB/s of codes", round(n / t / 1e9, 2),
                      "GB/s", args,
                      {"workload": f"{n >> 20} MiB of 8-bit codes, discretised normal (sigma 24 codes), "
                                   f"M=2^{K}, b=L=2^16, N=64, 64 KiB chunks, bf16 codebook"})
    out.update({
        "fused_bf16_us": round(t * 1e6, 1),
        "fused_fp32_us": round(res["fused_fp32"] * 1e6, 1),
        "unfused_bf16_us": round(res["unfused_bf16"] * 1e6, 1),
        "decode_codes_us": round(res["decode_codes"] * 1e6, 1),
        "gather_us": round(res["gather"] * 1e6, 1),
        "fused_speedup": round(res["unfused_bf16"] / t, 3),
        "unfused_bound_us": round(unfused_bound * 1e6, 1),
        "fused_speedup_vs_bound": round(unfused_bound / t, 3),
        "copy_gbps": round(copy_rate / 1e9, 1),
        "unfused_note": "gather = torch index_select after a uint8->int32 index copy; "
                        "bound = decode + 3 bytes per code at the device-copy rate",
        "compression_ratio": round(clen / n, 4),
        "roofline": {"bound": "hbm", "kernel": "k_decode64 (LUT output)", "unit": "GB/s",
                     "achieved": round(alg / t / 1e9, 1), "peak": HBM_PEAK_GBPS,
                     "frac": round(alg / t / 1e9 / HBM_PEAK_GBPS, 4), "traffic": None},
    })
    print(json.dumps(out), flush=True)


def cpu_model():
    """The host CPU's model name (as /proc/cpuinfo gives it), or ''."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def host_threads():
    """Threads the CPU baseline may use: the cores this process may run on,
    at most 16 (one GPU's share of the host on the GPU machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline_points(points, one_bytes, many_bytes):
    """The oracle, as it is, on a bounded sample of the sweep: encode + decode
    of the first one_bytes of every point with one thread, and of the first
    many_bytes of every point with every host thread (over chunks)."""
    import numpy as np

    import oracle

    def run(nbytes, threads):
        tot_b, tot_s = 0, 0.0
        for p, syms, f, C in points:
            s = np.ascontiguousarray(syms[: nbytes // syms.itemsize])
            t0 = time.perf_counter()
            c = oracle.encode(f, s, p["k"], p["r"], p["l"], p["N"], C, threads=threads)
            d = oracle.decode(f, c, threads=threads)
            tot_s += time.perf_counter() - t0
            assert (d == s).all()
            tot_b += s.nbytes
        return tot_b / tot_s / 1e9

    many = host_threads()
    single = run(one_bytes, 1)
    multi = run(many_bytes, many)
    return {"value": round(multi, 4), "unit": "GB/s", "cores": many, "kind": "oracle",
            "single_thread_gbps": round(single, 4), "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(),
            "sample": f"encode+decode of the first {many_bytes >> 20} MiB of each of the "
                      f"{len(points)} sweep points with {many} threads over chunks; single-thread "
                      f"figure on the first {one_bytes >> 20} MiB of each point"}


class SweepGroups:
    """The radix/precision sweep as batches: the points sharing (k, r, l, w,
    N) -- the three distributions of every alphabet of one symbol width --
    form one job list, each point with its own table; all stay resident."""

    def __init__(self, args, tune_cache):
        import numpy as np
        import torch

        import datagen
        import paper_1402_3392_amd as lr

        self.lr = lr
        pts = [p for p in datagen.sweep_points() if p["feasible"]]
        groups = {}
        for p in pts:
            groups.setdefault((p["k"], p["r"], p["l"], p["w"], p["N"]), []).append(p)
        keys = sorted(groups)
        if getattr(args, "groups", ""):
            keys = [keys[int(i)] for i in args.groups.split(",")]
        data = {}
        for key in keys:
            for p in groups[key]:
                dk = (p["alphabet"], p["dist"])
                if dk not in data:
                    data[dk] = datagen.sweep_data(p["alphabet"], p["dist"])[0]
        self.groups = []
        self.points = []  # (point, symbols, quantised frequencies, C) for the CPU baseline
        for (k, r, l, w, N) in keys:
            gp = groups[(k, r, l, w, N)]
            syms = [data[(p["alphabet"], p["dist"])] for p in gp]
            sizes = [int(x.nbytes) for x in syms]
            tables = [lr.rans_tables_build(datagen.counts(x, p["alphabet"]), k) for p, x in zip(gp, syms)]
            d_in = [torch.from_numpy(x.view(np.uint8)).cuda() for x in syms]
            # the largest container any tuned chunk size can give
            cap_params = lr.rans_params.make(k, r, l, w, N, 4096 // w)
            caps = [lr.rans_encode_bound(x.size, cap_params) for x in syms]
            d_cont = [torch.empty(c, dtype=torch.uint8, device="cuda") for c in caps]
            d_dec = [torch.empty_like(x) for x in d_in]
            lens = torch.zeros(len(gp), dtype=torch.int64, device="cuda")
            st = torch.zeros(len(gp), dtype=torch.int32, device="cuda")
            tune_jobs = lr.make_jobs((tables[i], d_in[i], sizes[i], 0, 0, 0, 0) for i in range(len(gp)))
            tune = lr.rans_autotune_batch(tune_jobs, len(gp), lr.rans_params.make(k, r, l, w, N, 65536 // w),
                                          tune_cache)
            C = int(tune["chunk_syms"])
            params = lr.rans_params.make(k, r, l, w, N, C)
            cfg = (int(tune["waves_per_group"]), int(tune["groups_per_cu"]), int(tune["table_layout"]),
                   int(tune["use_graph"]))
            enc_jobs = lr.make_jobs((tables[i], d_in[i], sizes[i], d_cont[i], caps[i],
                                     int(lens.data_ptr()) + 8 * i, int(st.data_ptr()) + 4 * i)
                                    for i in range(len(gp)))
            lr.rans_batch_set_config(*cfg)
            lr.rans_encode_batch(enc_jobs, len(gp), params)
            torch.cuda.synchronize()
            assert int(st.abs().sum()) == 0, f"batched encode status {st.tolist()}"
            clen = [int(v) for v in lens.cpu().tolist()]
            dec_jobs = lr.make_jobs((tables[i], d_cont[i], clen[i], d_dec[i], sizes[i],
                                     int(lens.data_ptr()) + 8 * i, int(st.data_ptr()) + 4 * i)
                                    for i in range(len(gp)))
            g = dict(key=(k, r, l, w, N), points=gp, syms=syms, sizes=sizes, tables=tables, d_in=d_in,
                     d_cont=d_cont, d_dec=d_dec, caps=caps, lens=lens, st=st, clen=clen, C=C, cfg=cfg,
                     params=params, enc_jobs=enc_jobs, dec_jobs=dec_jobs,
                     alg=sum(clen) + sum(sizes) + sum(4 * p["alphabet"] for p in gp))
            self.groups.append(g)
            import oracle
            for p, x in zip(gp, syms):
                self.points.append((p, x, oracle.quantize(datagen.counts(x, p["alphabet"]), k), C))
            log(f"group k={k} r={r} w={w} N={N}: {len(gp)} points, C={C}, shape {cfg}, "
                f"ratio {sum(clen) / sum(sizes):.4f}")
        self.total = sum(sum(g["sizes"]) for g in self.groups)
        self.alg = sum(g["alg"] for g in self.groups)

    def encode(self, g):
        self.lr.rans_batch_set_config(*g["cfg"])
        self.lr.rans_encode_batch(g["enc_jobs"], len(g["points"]), g["params"])

    def decode(self, g):
        self.lr.rans_batch_set_config(*g["cfg"])
        self.lr.rans_decode_batch(g["dec_jobs"], len(g["points"]), g["params"])

    def step(self):
        # (the planning kernel of every launch sets each job's status word)
        for g in self.groups:
            self.encode(g)
            self.decode(g)

    def check(self):
        import torch
        for g in self.groups:
            assert int(g["st"].abs().sum()) == 0, (g["key"], g["st"].tolist())
            assert [int(v) for v in g["lens"].cpu().tolist()] == [x.size for x in g["syms"]]
            for a, b in zip(g["d_dec"], g["d_in"]):
                assert torch.equal(a, b), g["key"]

    def group_times(self, reps):
        """Batched decode and encode of each group alone (median of reps)."""
        rows = []
        for g in self.groups:
            td = timed(lambda: self.decode(g), reps)
            te = timed(lambda: self.encode(g), reps)
            k, r, l, w, N = g["key"]
            rows.append({"k": k, "r": r, "w": w, "N": N, "points": len(g["points"]), "C": g["C"],
                         "shape": list(g["cfg"]), "ratio": round(sum(g["clen"]) / sum(g["sizes"]), 4),
                         "batched_decode_gbps": round(sum(g["sizes"]) / td / 1e9, 1),
                         "batched_encode_gbps": round(sum(g["sizes"]) / te / 1e9, 1),
                         "decode_roofline_frac": round(g["alg"] / td / 1e9 / HBM_PEAK_GBPS, 4),
                         "encode_roofline_frac": round(g["alg"] / te / 1e9 / HBM_PEAK_GBPS, 4),
                         "t_decode": td, "t_encode": te})
        return rows

    def plain_best(self, reps):
        """One plain launch per point, each at the chunk size that suits it
        best (the fastest of 64, 32, 16, 8 and 4 KiB chunks, separately for
        decode and encode); returns the total times over all points."""
        import torch
        lr = self.lr
        t_dec, t_enc = 0.0, 0.0
        for g in self.groups:
            k, r, l, w, N = g["key"]
            for i, p in enumerate(g["points"]):
                n = g["syms"][i].size
                st = torch.zeros(1, dtype=torch.int32, device="cuda")
                olen = torch.zeros(1, dtype=torch.int64, device="cuda")
                best_d, best_e = 1e30, 1e30
                for C in (65536, 32768, 16384, 8192, 4096):
                    Cw = C // w
                    pp = lr.rans_params.make(k, r, l, w, N, Cw)
                    cap = lr.rans_encode_bound(n, pp)
                    out = g["d_cont"][i]
                    assert cap <= out.numel()
                    enc = lambda: lr.rans_encode_async(g["tables"][i], pp, g["d_in"][i], n, out, cap, olen, st)
                    te = timed(enc, reps)
                    torch.cuda.synchronize()
                    nb = int(olen)
                    hdr = bytes(out[:32].cpu().numpy().tobytes())
                    dec = lambda: lr.rans_decode_async(g["tables"][i], out, nb, hdr, g["d_dec"][i], n, st)
                    td = timed(dec, reps)
                    torch.cuda.synchronize()
                    assert int(st) == 0 and torch.equal(g["d_dec"][i], g["d_in"][i])
                    best_d, best_e = min(best_d, td), min(best_e, te)
                t_dec += best_d
                t_enc += best_e
        # the batched containers again (the plain runs overwrote them)
        for g in self.groups:
            g["st"].zero_()
            self.encode(g)
        torch.cuda.synchronize()
        return t_dec, t_enc


def traffic_for(kernel, workload):
    """HBM bytes per step of `kernel` on `workload` from profiles/traffic.txt
    (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration), or None
    when they were taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    src = kernel_source_hash()
    for line in open(path):
        if line.startswith("#") or "=" not in line:
            continue
        kv = dict(tok.split("=", 1) for tok in line.split())
        if kv.get("kernel") == kernel and kv.get("source") == src and kv.get("workload") == workload:
            return int(kv["traffic_bytes"])
    return None


def run_headline(args):
    """The metric's line.  Value: the radix/precision sweep (84 feasible
    points of 64 MiB each) encoded and decoded by batched persistent launches,
    one per group of points sharing (k, r, l, w, N), in uncompressed GB/s.
    Beside it: the batched kernels' roofline fractions, one plain launch per
    point at its own best chunk size (the speedup), the 4096-stream batch
    against plain per-stream calls, the serving loop's p50/p99, the plain
    256 MiB round trip, and the CPU oracle."""
    import torch

    import paper_1402_3392_amd as lr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    tune_cache = args.tune_cache or None
    log("sweep: generating 12 x 64 MiB, building 84 tables, batching by (k, r, l, w, N)")
    sw = SweepGroups(args, tune_cache)
    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        sw.step()
    torch.cuda.synchronize()
    if args.warmup:
        sw.check()  # the decoded lengths are in place only after a step
    log(f"timing {args.steps} steps")
    lr.rans_timing_reset()
    lr.rans_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sw.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lr.rans_timing_enable(False)
    sw.check()
    kt = {name: lr.rans_timing_read(kind) for name, kind in
          (("decode", lr.RANS_KERNEL_BATCH_DECODE), ("encode", lr.RANS_KERNEL_BATCH_ENCODE))}
    lr.rans_timing_reset()
    elapsed = t1 - t0
    value = args.steps * sw.total / elapsed / 1e9
    nlaunch = len(sw.groups)

    def roof(name, kname):
        cnt, ms = kt[name]
        avg_us = 1e3 * ms / max(cnt, 1)
        alg_launch = sw.alg / nlaunch
        ach = args.steps * sw.alg / (ms / 1e3) / 1e9
        tr = None if args.groups else traffic_for(kname, "sweep84")
        return {"bound": "hbm", "kernel": kname, "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4),
                "traffic": None if tr is None else int(tr / nlaunch),
                "alg_bytes_per_launch": int(alg_launch), "launches": cnt, "avg_us": round(avg_us, 1),
                "note": "12 launches per step (one per group); events around each launch, "
                        "planning kernel included"}

    dom, other = ("encode", "decode") if kt["encode"][1] >= kt["decode"][1] else ("decode", "encode")
    knames = {"decode": "k_batch_decode64", "encode": "k_batch_encode64"}
    if args.batched_only:
        res = base_result("rANS decode/encode GB/s on 1 MI355X, batched", round(value, 2), "GB/s", args,
                          {"workload": f"radix/precision sweep, {len(sw.points)} points of 64 MiB, batched by "
                                       f"(k,r,l,w,N)" + (f" (groups {args.groups} only)" if args.groups else ""),
                           "points": len(sw.points), "launches_per_step": 2 * nlaunch,
                           "symbol_bytes_per_step": sw.total, "parallelism": "none"})
        res["ms_per_step"] = round(1e3 * elapsed / args.steps, 3)
        res["roofline"] = roof(dom, knames[dom])
        res[f"roofline_{other}"] = roof(other, knames[other])
        print(json.dumps(res), flush=True)
        return
    log("per-group times")
    rows = sw.group_times(max(3, args.steps))
    log("plain launches per point at their best chunk size")
    plain_dec, plain_enc = sw.plain_best(3)
    bat_dec = sum(r["t_decode"] for r in rows)
    bat_enc = sum(r["t_encode"] for r in rows)
    for r in rows:
        del r["t_decode"], r["t_encode"]
    res = base_result("rANS decode/encode GB/s on 1 MI355X, batched vs plain; p99 decode latency",
                      round(value, 2), "GB/s", args,
                      {"workload": "radix/precision sweep: 84 feasible points of 64 MiB of symbol bytes "
                                   "(alphabets 2/16/256 uint8 and 4096 uint16; M=2^11/2^15; p0=0.995, "
                                   "Zipf(1.1), near-uniform; (b,L)=(2^8,2^23)/(2^16,2^16); N=32/64), "
                                   "each with its own table, batched by (k,r,l,w,N): 12 persistent "
                                   "launches per direction, chunk size and launch shape autotuned per "
                                   "batch; one step = batched encode + batched decode of every point",
                       "points": len(sw.points), "launches_per_step": 2 * nlaunch,
                       "symbol_bytes_per_step": sw.total, "parallelism": "none"})
    res["ms_per_step"] = round(1e3 * elapsed / args.steps, 3)
    res["batched_decode_gbps"] = round(sw.total / bat_dec / 1e9, 1)
    res["batched_encode_gbps"] = round(sw.total / bat_enc / 1e9, 1)
    res["plain_decode_gbps"] = round(sw.total / plain_dec / 1e9, 1)
    res["plain_encode_gbps"] = round(sw.total / plain_enc / 1e9, 1)
    res["decode_speedup_vs_plain"] = round(plain_dec / bat_dec, 2)
    res["encode_speedup_vs_plain"] = round(plain_enc / bat_enc, 2)
    res["plain_note"] = "one launch per point, each at its fastest of 64/32/16/8/4 KiB chunks"
    res["roofline"] = roof(dom, knames[dom])
    res[f"roofline_{other}"] = roof(other, knames[other])
    res["groups"] = rows
    if not args.headline_only:
        log("4096 streams: batched vs plain")
        b = run_batched(args, emit=False)
        res["batched_4096_streams"] = {k: b[k] for k in (
            "value", "batched_decode_gbps", "plain_decode_gbps", "plain_decode_choice", "decode_speedup",
            "batched_encode_gbps", "plain_encode_gbps", "plain_encode_choice", "encode_speedup",
            "compression_ratio", "autotune", "roofline")}
        res["batched_4096_streams"]["workload"] = b["config"]["workload"]
        log("serving")
        sv = run_serving(args, emit=False, rates=(0.5, 1.0))
        at1 = [r for r in sv["rates"] if r["rate_frac"] == 1.0][0]
        res["serving"] = {"workload": sv["config"]["workload"], "saturated_gbps": sv["saturated_gbps"],
                          "decode_p50_ms": at1.get("decode_p50_ms"), "decode_p99_ms": at1.get("decode_p99_ms"),
                          "encode_p50_ms": at1.get("encode_p50_ms"), "encode_p99_ms": at1.get("encode_p99_ms"),
                          "rates": sv["rates"]}
        log("256 MiB round trip")
        rt = run_roundtrip(args, emit=False)
        res["roundtrip_3x256MiB"] = {k: rt[k] for k in ("value", "decode_gbps_kernel", "encode_gbps_kernels",
                                                        "kernels", "roofline", "roofline_decode")}
    if not args.no_cpu_baseline:
        log(f"cpu baseline: 1 thread and {host_threads()} threads")
        res["cpu_baseline"] = cpu_baseline_points(sw.points, 1 << 20, 8 << 20)
    print(json.dumps(res), flush=True)


def run_sweep_grouped(args):
    """The sweep's points as batches: the points that share (k, r, l, w, N)
    -- the three distributions of every alphabet with the same symbol width --
    go through one persistent batched launch, each with its own table, tuned
    on that batch; against one plain launch per point.  Every container is
    compared with the oracle's."""
    import numpy as np
    import torch

    import datagen
    import oracle
    import paper_1402_3392_amd as lr

    pts = [p for p in datagen.sweep_points() if p["feasible"]]
    if args.points:
        keep = {int(x) for x in args.points.split(",") if x}
        pts = [p for i, p in enumerate(datagen.sweep_points()) if i in keep and p["feasible"]]
    groups = {}
    for p in pts:
        groups.setdefault((p["k"], p["r"], p["l"], p["w"], p["N"]), []).append(p)
    threads = min(16, os.cpu_count() or 1)
    rows = []
    cache = {}
    for (k, r, l, w, N), gp in sorted(groups.items()):
        data = []
        for p in gp:
            key = (p["alphabet"], p["dist"])
            if key not in cache:
                if len(cache) > 12:
                    cache.clear()
                cache[key] = datagen.sweep_data(p["alphabet"], p["dist"])[0]
            data.append((p, cache[key]))
        sizes = [int(s.size) * w for _, s in data]
        total = sum(sizes)
        tables = [lr.rans_tables_build(datagen.counts(s, p["alphabet"]), k) for p, s in data]
        cap_params = lr.rans_params.make(k, r, l, w, N, 4096 // w)
        caps = [lr.rans_encode_bound(s.size, cap_params) for _, s in data]
        pool = DevPool(sum((n + 255) // 256 * 256 for n in sizes) * 2 + sum(caps) + 256 * len(data))
        d_in = [pool.take(n) for n in sizes]
        for a, (_, s) in zip(d_in, data):
            pool.view(a, s.nbytes).copy_(torch.from_numpy(s.view(np.uint8)))
        d_cont = [pool.take(c) for c in caps]
        d_dec = [pool.take(n) for n in sizes]
        lens = torch.zeros(len(data), dtype=torch.int64, device="cuda")
        st = torch.zeros(len(data), dtype=torch.int32, device="cuda")
        tune_jobs = lr.make_jobs((tables[i], d_in[i], sizes[i], 0, 0, 0, 0) for i in range(len(data)))
        tune = lr.rans_autotune_batch(tune_jobs, len(data), lr.rans_params.make(k, r, l, w, 64, 65536 // w))
        C = int(tune["chunk_syms"])
        params = lr.rans_params.make(k, r, l, w, N, C)
        enc_jobs = lr.make_jobs((tables[i], d_in[i], sizes[i], d_cont[i], caps[i],
                                 int(lens.data_ptr()) + 8 * i, int(st.data_ptr()) + 4 * i)
                                for i in range(len(data)))
        lr.rans_encode_batch(enc_jobs, len(data), params)
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0, f"batched encode status {st.tolist()}"
        clen = [int(v) for v in lens.cpu().tolist()]
        exact = True
        for i, (p, s) in enumerate(data):
            f = oracle.quantize(datagen.counts(s, p["alphabet"]), k)
            ref = oracle.encode(f, s, k, r, l, N, C, threads=threads)
            exact &= clen[i] == ref.size and np.array_equal(pool.view(d_cont[i], clen[i]).cpu().numpy(), ref)
        headers = [bytes(pool.view(d_cont[i], 32).cpu().numpy().tobytes()) for i in range(len(data))]
        dec_jobs = lr.make_jobs((tables[i], d_cont[i], clen[i], d_dec[i], sizes[i],
                                 int(lens.data_ptr()) + 8 * i, int(st.data_ptr()) + 4 * i)
                                for i in range(len(data)))

        def batched():
            lr.rans_decode_batch(dec_jobs, len(data), params)

        def plain():
            for i in range(len(data)):
                lr.rans_decode_async(tables[i], pool.view(d_cont[i], clen[i]), clen[i], headers[i],
                                     pool.view(d_dec[i], sizes[i]), sizes[i] // w, st[i:i + 1])

        res = {}
        for name, fn in (("batched", batched), ("plain", plain)):
            fn()
            torch.cuda.synchronize()
            st.zero_()
            res[name] = timed(fn, max(5, args.steps))
            torch.cuda.synchronize()
            assert int(st.abs().sum()) == 0, name
            for i in range(len(data)):
                assert torch.equal(pool.view(d_dec[i], sizes[i]), pool.view(d_in[i], sizes[i])), name
        alg = sum(clen) + total + sum(4 * p["alphabet"] for p, _ in data)
        row = {"k": k, "r": r, "l": l, "w": w, "N": N, "points": len(data), "bytes": total, "C": C,
               "G": tune["waves_per_group"], "gpc": tune["groups_per_cu"], "layout": tune["table_layout"],
               "bit_exact": bool(exact),
               "batched_decode_gbps": round(total / res["batched"] / 1e9, 1),
               "plain_decode_gbps": round(total / res["plain"] / 1e9, 1),
               "speedup": round(res["plain"] / res["batched"], 2),
               "ratio": round(sum(clen) / total, 4),
               "batched_roofline_frac": round(alg / res["batched"] / 1e9 / HBM_PEAK_GBPS, 4)}
        rows.append(row)
        log(json.dumps(row))
        for t in tables:
            t.close()
        del pool
        torch.cuda.empty_cache()
    best = max(rows, key=lambda r_: r_["batched_roofline_frac"])
    out = base_result("rANS decode/encode GB/s on 1 MI355X, batched vs plain; p99 decode latency",
                      best["batched_decode_gbps"], "GB/s", args,
                      {"workload": "sweep points batched by (k, r, l, w, N): 64 MiB of symbol bytes "
                                   "per point, each with its own table; batched decode vs one plain "
                                   "launch per point"})
    out["groups"] = rows
    out["roofline"] = {"bound": "hbm", "kernel": "k_batch_decode64", "unit": "GB/s",
                       "achieved": round(best["batched_roofline_frac"] * HBM_PEAK_GBPS, 1),
                       "peak": HBM_PEAK_GBPS, "frac": best["batched_roofline_frac"], "traffic": None,
                       "note": f"best group: k={best['k']} r={best['r']} w={best['w']} N={best['N']}"}
    print(json.dumps(out), flush=True)


def run_escape(args):
    """Escape coding (raw digits in the interleaved stream): 64 MiB of 16-bit
    zigzag Laplace values (scale 300), coded with a 1024-symbol table whose
    last symbol is the escape, against the same stream without the raw
    digits (every value clipped to the table)."""
    import numpy as np
    import torch

    import datagen
    import paper_1402_3392_amd as lr

    K, R, L, W, N, C, T = 15, 16, 16, 2, 64, 32768, 1024
    n = (1 << 26) // W
    log(f"generating {n} zigzag Laplace values")
    rng = np.random.Generator(np.random.PCG64(7001))
    v = datagen.sample(datagen.laplace_u16_probs(300.0), n, rng, np.uint16)
    counts = np.bincount(np.minimum(v, T - 1), minlength=T).astype(np.uint64)
    table = lr.rans_tables_build(counts, K)
    esc_frac = float((v >= T - 1).mean())
    res, sizes = {}, {}
    d_in = torch.from_numpy(v.view(np.uint8)).cuda()
    d_clip = torch.from_numpy(np.minimum(v, T - 2).astype(np.uint16).view(np.uint8)).cuda()
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    lens = torch.zeros(2, dtype=torch.int64, device="cuda")
    for name, src, esc in (("escape", d_in, True), ("clipped", d_clip, False)):
        params = lr.rans_params.make(K, R, L, W, N, C, "df", esc)
        cap = lr.rans_encode_bound(n, params)
        cont = torch.empty(cap, dtype=torch.uint8, device="cuda")
        clen = lr.rans_encode(table, params, src, n, cont, cap)
        hdr = bytes(cont[:32].cpu().numpy().tobytes())
        out = torch.empty(n * W, dtype=torch.uint8, device="cuda")
        i = 0 if esc else 1

        def enc():
            lr.rans_encode_async(table, params, src, n, cont, cap, lens[i:i + 1], st[2 * i:2 * i + 1])

        def dec():
            lr.rans_decode_async(table, cont, clen, hdr, out, n, st[2 * i + 1:2 * i + 2])

        for fn_name, fn in (("encode", enc), ("decode", dec)):
            for _ in range(max(1, args.warmup)):
                fn()
            torch.cuda.synchronize()
            res[f"{name}_{fn_name}"] = timed(fn, max(5, args.steps))
        assert int(st.abs().sum()) == 0, f"status {st.tolist()}"
        assert torch.equal(out, src), f"{name}: decode mismatch"
        sizes[name] = clen
        log(f"{name}: {clen / (n * W):.4f} of input; encode {res[name + '_encode'] * 1e6:.1f} us, "
            f"decode {res[name + '_decode'] * 1e6:.1f} us")
    t = res["escape_decode"]
    alg = sizes["escape"] + n * W + 4 * T
    out = base_result("rANS escape-coded decode, GB/s of 16-bit symbols", round(n * W / t / 1e9, 2),
                      "GB/s", args,
                      {"workload": f"{n * W >> 20} MiB of uint16 zigzag Laplace(300) values, "
                                   f"{T}-symbol table with escape (16 raw bits), M=2^{K}, "
                                   f"b=L=2^16, N=64, 64 KiB chunks"})
    out.update({
        "escaped_fraction": round(esc_frac, 4),
        "escape_ratio": round(sizes["escape"] / (n * W), 4),
        "clipped_ratio": round(sizes["clipped"] / (n * W), 4),
        "escape_encode_gbps": round(n * W / res["escape_encode"] / 1e9, 2),
        "escape_decode_gbps": round(n * W / res["escape_decode"] / 1e9, 2),
        "clipped_encode_gbps": round(n * W / res["clipped_encode"] / 1e9, 2),
        "clipped_decode_gbps": round(n * W / res["clipped_decode"] / 1e9, 2),
        "roofline": {"bound": "hbm", "kernel": "k_decode64 (escape)", "unit": "GB/s",
                     "achieved": round(alg / t / 1e9, 1), "peak": HBM_PEAK_GBPS,
                     "frac": round(alg / t / 1e9 / HBM_PEAK_GBPS, 4), "traffic": None},
    })
    print(json.dumps(out), flush=True)


def run_prefix(args):
    """Section 4's multiplexer with a second coder family: the three 256 MiB
    Zipf buffers of the round trip coded with the canonical prefix code
    (N = 64 coder streams multiplexed in decoder read order), against rANS
    with the same table, chunking and interleave."""
    import numpy as np
    import torch

    import datagen
    import paper_1402_3392_amd as lr

    n = 1 << args.size_log2
    rows, res = [], {}
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    lens = torch.zeros(2, dtype=torch.int64, device="cuda")
    tot = {"pfx_enc": 0.0, "pfx_dec": 0.0, "rans_enc": 0.0, "rans_dec": 0.0, "pfx_bytes": 0}
    for s_ in datagen.ZIPF_S:
        w = datagen.zipf_buffer(s_, n=n)
        k, r, l, W, N, C = w.params.astuple()
        table = lr.rans_tables_build(w.counts, k)
        d_in = torch.from_numpy(w.syms).cuda()
        out = torch.empty_like(d_in)
        row = {"s": s_}
        for name, pfx in (("pfx", True), ("rans", False)):
            params = lr.rans_params.make(k, 16, 16, W, N, C)
            cap = lr.rans_encode_bound(n, params)
            cont = torch.empty(cap, dtype=torch.uint8, device="cuda")
            enc_fn = lr.rans_pfx_encode if pfx else lr.rans_encode
            clen = enc_fn(table, params, d_in, n, cont, cap)
            hdr = bytes(cont[:32].cpu().numpy().tobytes())
            i = 0 if pfx else 1
            enc_async = lr.rans_pfx_encode_async if pfx else lr.rans_encode_async

            def enc():
                enc_async(table, params, d_in, n, cont, cap, lens[i:i + 1], st[2 * i:2 * i + 1])

            def dec():
                lr.rans_decode_async(table, cont, clen, hdr, out, n, st[2 * i + 1:2 * i + 2])

            for fn_name, fn in (("enc", enc), ("dec", dec)):
                for _ in range(max(1, args.warmup)):
                    fn()
                torch.cuda.synchronize()
                t = timed(fn, max(5, args.steps))
                row[f"{name}_{fn_name}_us"] = round(t * 1e6, 1)
                tot[f"{name}_{fn_name}"] += t
            assert int(st.abs().sum()) == 0, f"status {st.tolist()}"
            assert torch.equal(out, d_in), f"{name}: decode mismatch"
            row[f"{name}_ratio"] = round(clen / n, 4)
            if pfx:
                tot["pfx_bytes"] += clen
        rows.append(row)
        log(json.dumps(row))
        table.close()
    total = 3 * n
    t = tot["pfx_dec"]
    alg = tot["pfx_bytes"] + total + 3 * 2 * (1 << 14)
    out = base_result("prefix-code family multiplexed by the decoder read rule: decode GB/s",
                      round(total / t / 1e9, 2), "GB/s", args,
                      {"workload": f"3 x {n >> 20} MiB uint8 Zipf(s in 0.8/1.1/1.5) over 256, "
                                   f"canonical prefix code from M=2^14 frequencies, 16-bit words, "
                                   f"N=64, 64 KiB chunks; rANS with the same table beside it"})
    out.update({
        "pfx_encode_gbps": round(total / tot["pfx_enc"] / 1e9, 2),
        "pfx_decode_gbps": round(total / tot["pfx_dec"] / 1e9, 2),
        "rans_encode_gbps": round(total / tot["rans_enc"] / 1e9, 2),
        "rans_decode_gbps": round(total / tot["rans_dec"] / 1e9, 2),
        "buffers": rows,
        "roofline": {"bound": "hbm", "kernel": "k_decode64 (prefix-code family)", "unit": "GB/s",
                     "achieved": round(alg / t / 1e9, 1), "peak": HBM_PEAK_GBPS,
                     "frac": round(alg / t / 1e9 / HBM_PEAK_GBPS, 4), "traffic": None},
    })
    print(json.dumps(out), flush=True)


def run_serving(args, emit=True, rates=(0.25, 0.5, 0.75, 0.9, 1.0, 1.2)):
    """Request loop: Poisson arrivals of mixed encode/decode requests under an
    8 GiB HBM budget, rates swept around the saturated throughput; p50/p99
    latency (arrival to completion) per operation and aggregate GB/s."""
    import numpy as np
    import torch

    import datagen
    import paper_1402_3392_amd as lr

    K, R, L, W, N, C = 14, 16, 16, 1, 64, 65536
    params = lr.rans_params.make(K, R, L, W, N, C)
    reqs = datagen.serving_requests(nreq=args.requests)
    log(f"{len(reqs)} requests, {sum(q['size'] for q in reqs) / 2**30:.2f} GiB; staging")
    staged = []
    for q, syms in zip(reqs, datagen.requests_data(reqs)):
        table = lr.rans_tables_build(datagen.counts(syms, 256), K)
        d = torch.from_numpy(syms).cuda()
        if q["op"] == "encode":
            staged.append((lr.RANS_OP_ENCODE, table, d, syms.size,
                           lr.rans_encode_bound(syms.size, params), syms.size))
        else:
            cap = lr.rans_encode_bound(syms.size, params)
            c = torch.empty(cap, dtype=torch.uint8, device="cuda")
            nb = lr.rans_encode(table, params, d, syms.size, c, cap)
            staged.append((lr.RANS_OP_DECODE, table, c[:nb].clone(), nb, syms.size, syms.size))
            del c
    torch.cuda.synchronize()
    total = sum(s[5] for s in staged)
    srv = lr.rans_server_create(8 << 30, 4, 64, params)

    def replay(arrivals):
        reqlist = [(op, tab, d, inl, cap, float(t))
                   for (op, tab, d, inl, cap, _), t in zip(staged, arrivals)]
        res, mk = lr.rans_server_replay(srv, reqlist)
        bad = [r.status for r in res if r.status != 0]
        assert not bad, f"serving failures: {bad[:4]}"
        return res, mk

    log("saturated replay")
    replay(np.zeros(len(staged)))  # warm: graphs, arena
    _, mk = replay(np.zeros(len(staged)))
    sat_rate = len(staged) / mk  # requests per microsecond
    rows = []
    for frac in rates:
        rng = np.random.Generator(np.random.PCG64(5001 + int(frac * 100)))
        arr = np.cumsum(rng.exponential(1.0 / (frac * sat_rate), len(staged)))
        arr -= arr[0]
        res, mk = replay(arr)
        lat = {op: np.array([r.latency_us for r in res if r.op == op]) for op in (0, 1)}
        row = {"rate_frac": frac, "req_per_s": round(frac * sat_rate * 1e6, 1),
               "gbps": round(total / (mk * 1e-6) / 1e9, 2)}
        for op, name in ((1, "decode"), (0, "encode")):
            if lat[op].size:
                row[f"{name}_p50_ms"] = round(float(np.percentile(lat[op], 50)) / 1e3, 3)
                row[f"{name}_p99_ms"] = round(float(np.percentile(lat[op], 99)) / 1e3, 3)
        rows.append(row)
        log(json.dumps(row))
    stats = lr.rans_server_stats(srv)
    lr.rans_server_destroy(srv)
    at1 = [r for r in rows if r["rate_frac"] == 1.0][0]
    out = base_result("rANS decode/encode GB/s on 1 MI355X, batched vs plain; p99 decode latency",
                      at1["decode_p99_ms"], "ms", args,
                      {"workload": f"{len(staged)} requests, sizes 2^U(12,26) B, encode/decode 50/50, "
                                   "Zipf(s~U(0.7,1.5)) tables, M=2^14, b=L=2^16, N=64, 64 KiB chunks, "
                                   "8 GiB HBM budget, Poisson arrivals"}, higher=False)
    out.update({"saturated_gbps": round(total / (len(staged) / sat_rate * 1e-6) / 1e9, 2),
                "rates": rows, "server": stats})
    if emit:
        print(json.dumps(out), flush=True)
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one MI355X only: the coder's work is independent per "
              "chunk and the library has no multi-GPU path (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    if args.source_hash:
        print(kernel_source_hash())
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.workload == "sweep" and args.grouped:
        run_sweep_grouped(args)
        return
    {"headline": run_headline, "roundtrip": run_roundtrip, "batched": run_batched, "sweep": run_sweep,
     "serving": run_serving, "dequant": run_dequant, "escape": run_escape,
     "prefix": run_prefix}[args.workload](args)


def run_roundtrip(args, emit=True):
    """Three 256 MiB Zipf buffers encoded and decoded by the plain
    single-buffer entry points (64 KiB chunks, 64 coders)."""
    import numpy as np
    import torch

    import datagen
    import paper_1402_3392_amd as lr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n = 1 << args.size_log2

    log(f"generating 3 x {n >> 20} MiB Zipf buffers")
    work = []
    for s in datagen.ZIPF_S:
        w = datagen.zipf_buffer(s, n=n)
        work.append(w)
    params = [lr.rans_params.make(*w.params.astuple()) for w in work]
    tables = [lr.rans_tables_build(w.counts, w.params.k) for w in work]
    freqs = [lr.rans_table_freqs(t) for t in tables]

    d_in = [torch.from_numpy(w.syms).to(dev) for w in work]
    caps = [lr.rans_encode_bound(n, p) for p in params]
    d_cont = [torch.empty(c, dtype=torch.uint8, device=dev) for c in caps]
    d_dec = [torch.empty(n, dtype=torch.uint8, device=dev) for _ in work]
    d_len = torch.zeros(len(work), dtype=torch.int64, device=dev)
    d_st = torch.zeros(2 * len(work), dtype=torch.int32, device=dev)

    def enc(i):
        lr.rans_encode_async(tables[i], params[i], d_in[i], n, d_cont[i], caps[i],
                             d_len[i:i + 1], d_st[2 * i:2 * i + 1])

    # the container length and header are fixed for a given input: learn them once
    for i in range(len(work)):
        enc(i)
    torch.cuda.synchronize()
    assert int(d_st.abs().sum()) == 0, f"encode status {d_st.tolist()}"
    lens = [int(v) for v in d_len.cpu().tolist()]
    headers = [bytes(d_cont[i][:32].cpu().numpy().tobytes()) for i in range(len(work))]

    def dec(i):
        lr.rans_decode_async(tables[i], d_cont[i], lens[i], headers[i], d_dec[i], n,
                             d_st[2 * i + 1:2 * i + 2])

    def step():
        d_st.zero_()
        for i in range(len(work)):
            enc(i)
            dec(i)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.warmup:
        for i in range(len(work)):
            assert torch.equal(d_dec[i], d_in[i]), f"round trip mismatch on buffer {i}"
        assert int(d_st.abs().sum()) == 0

    log(f"timing {args.steps} steps")
    lr.rans_timing_reset()
    lr.rans_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lr.rans_timing_enable(False)
    assert int(d_st.abs().sum()) == 0, f"status {d_st.tolist()}"
    for i in range(len(work)):
        assert torch.equal(d_dec[i], d_in[i])

    elapsed = t1 - t0
    sym_bytes = n * len(work)
    value = args.steps * sym_bytes / elapsed / 1e9
    kt = {}
    for kind, name in [(lr.RANS_KERNEL_DECODE, "decode"), (lr.RANS_KERNEL_ENCODE, "encode"),
                       (lr.RANS_KERNEL_SCAN, "scan"), (lr.RANS_KERNEL_COMPACT, "compact")]:
        cnt, ms = lr.rans_timing_read(kind)
        kt[name] = (cnt, ms)
    lr.rans_timing_reset()

    # algorithmic bytes per launch: container read (or written) + symbols
    # written (or read) + the static table (4 bytes per alphabet symbol)
    alg = [lens[i] + n + 4 * 256 for i in range(len(work))]
    alg_total = args.steps * sum(alg)
    per_kernel = {k: {"launches": c, "avg_us": round(1e3 * ms / max(c, 1), 2)}
                  for k, (c, ms) in kt.items()}
    dom = "decode" if kt["decode"][1] >= kt["encode"][1] else "encode"
    dom_gbps = alg_total / (kt[dom][1] / 1e3) / 1e9
    other = "encode" if dom == "decode" else "decode"
    kname = {"decode": "k_decode64", "encode": "k_encode64_place"}[dom]
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(dom_gbps, 1),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(dom_gbps / HBM_PEAK_GBPS, 4),
                "traffic": measured_traffic(kname),
                "alg_bytes_per_launch": int(sum(alg) / len(alg))}

    res = {
        "metric": "rANS decode/encode GB/s on 1 MI355X, batched vs plain; p99 decode latency",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"3 x {n >> 20} MiB uint8 Zipf(s in 0.8/1.1/1.5) over 256, "
                               "M=2^14, b=L=2^16, N=64, 64 KiB chunks, encode+decode round trip",
                   "global_batch": 3, "seq_len": n, "parallelism": "none"},
        "decode_gbps_kernel": round(sym_bytes * args.steps / (kt["decode"][1] / 1e3) / 1e9, 2),
        "encode_gbps_kernels": round(sym_bytes * args.steps / (
            (kt["encode"][1] + kt["scan"][1] + kt["compact"][1]) / 1e3) / 1e9, 2),
        "compression_ratio": [round(lens[i] / n, 4) for i in range(len(work))],
        "kernels": per_kernel,
        "roofline": roofline,
        f"roofline_{other}": {"achieved": round(alg_total / (kt[other][1] / 1e3) / 1e9, 1),
                              "frac": round(alg_total / (kt[other][1] / 1e3) / 1e9 /
                                            HBM_PEAK_GBPS, 4)},
    }
    if emit and not args.no_cpu_baseline:
        threads = args.cpu_threads or host_threads()
        log(f"cpu baseline with {threads} threads")
        res["cpu_baseline"] = cpu_baseline(list(zip(work, freqs)), threads)
    if emit:
        print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main()
