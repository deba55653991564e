"""Host-side checks of librans that need no GPU: every function the C header
declares is exported, the quantiser agrees with the oracle's, parameter
validation, the encode bound, and the encoder's division constants."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import datagen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lr():
    import paper_1402_3392_amd as m
    return m


def declared_functions():
    text = open(os.path.join(ROOT, "include", "librans.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(rans_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_symbols_are_exported(lr):
    names = declared_functions()
    assert len(names) >= 25, names
    lib = ct.CDLL(lr.LIBRARY_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_quantizer_matches_oracle(lr):
    rng = np.random.default_rng(21)
    for trial in range(400):
        n = int(rng.integers(1, 600))
        k = int(rng.integers(max(1, int(np.ceil(np.log2(n)))), 17))
        c = rng.integers(0, 5000, n).astype(np.uint64)
        if trial % 2:
            c[rng.random(n) < 0.6] = 0
        if trial % 5 == 0:
            c = (rng.pareto(0.7, n) * 10).astype(np.uint64)
        if c.sum() == 0:
            c[0] = 3
        assert (lr.rans_quantize(c, k) == oracle.quantize(c, k)).all(), trial


def test_quantizer_on_workload_histograms(lr):
    w = datagen.tiny_zipf(n=1 << 18)
    assert (lr.rans_quantize(w.counts, 12) == oracle.quantize(w.counts, 12)).all()
    for a in datagen.SWEEP_ALPHABETS:
        for dist in datagen.SWEEP_DISTS:
            syms, _ = datagen.sweep_data(a, dist, nbytes=1 << 18)
            c = datagen.counts(syms, a)
            for k in datagen.SWEEP_K:
                if int((c > 0).sum()) > (1 << k):
                    with pytest.raises(lr.RansError) as e:
                        lr.rans_quantize(c, k)
                    assert e.value.code == lr.RANS_EPREC
                    continue
                assert (lr.rans_quantize(c, k) == oracle.quantize(c, k)).all()


def test_params_check(lr):
    ok = [(12, 16, 16, 1, 64, 0), (8, 8, 16, 2, 1, 7), (15, 8, 23, 2, 32, 1 << 20),
          (11, 16, 16, 1, 4, 100)]
    bad = [(7, 16, 16, 1, 64, 0), (16, 16, 16, 1, 64, 0), (12, 12, 16, 1, 64, 0),
           (12, 16, 11, 1, 64, 0), (12, 16, 17, 1, 64, 0), (12, 16, 16, 3, 64, 0),
           (12, 16, 16, 1, 3, 0), (12, 16, 16, 1, 128, 0), (12, 8, 25, 1, 64, 0)]
    for p in ok:
        assert lr.rans_params_check(p) == 0, p
    for p in bad:
        assert lr.rans_params_check(p) == lr.RANS_EINVAL, p
    # digit order: 0 depth-first, 1 breadth-first, nothing else
    for order in ("df", "bf"):
        assert lr.rans_params_check(lr.rans_params.make(15, 8, 23, 1, 64, 4096, order)) == 0
    p = lr.rans_params.make(15, 8, 23, 1, 64, 4096)
    p.digit_order = 2
    assert lr.rans_params_check(p) == lr.RANS_EINVAL
    assert lr.rans_encode_bound(1000, p) == 0
    with pytest.raises(ValueError):
        lr.rans_params.make(15, 8, 23, 1, 64, 4096, "zz")
    # escape coding: 16-bit symbols, depth-first only
    assert lr.rans_params_check(lr.rans_params.make(15, 8, 23, 2, 64, 4096, "df", True)) == 0
    assert lr.rans_params_check(lr.rans_params.make(15, 8, 23, 1, 64, 4096, "df", True)) \
        == lr.RANS_EINVAL
    assert lr.rans_params_check(lr.rans_params.make(15, 8, 23, 2, 64, 4096, "bf", True)) \
        == lr.RANS_EINVAL
    p = lr.rans_params.make(15, 8, 23, 2, 64, 4096)
    p.escape = 2
    assert lr.rans_params_check(p) == lr.RANS_EINVAL


def test_encode_bound_covers_oracle(lr):
    rng = np.random.default_rng(22)
    for k, r, l, N, C in [(12, 16, 16, 64, 4096), (15, 8, 23, 32, 1000), (8, 8, 16, 4, 0)]:
        for n in (0, 1, 1000, 12345):
            syms = rng.integers(0, 256, n).astype(np.uint8)  # near-incompressible
            f = oracle.quantize(np.bincount(np.r_[syms, [0]], minlength=256).astype(np.uint64), k)
            p = (k, r, l, 1, N, C)
            bound = lr.rans_encode_bound(n, p)
            assert bound == oracle.encode_bound(n, k, r, N, C)
            assert oracle.encode(f, syms, k, r, l, N, C).size <= bound


def test_encode_bound_with_escapes_covers_oracle(lr):
    rng = np.random.default_rng(23)
    for k, r, l, N, C in [(12, 16, 16, 64, 4096), (15, 8, 23, 32, 1000), (10, 8, 16, 4, 0)]:
        v = rng.integers(0, 65536, 12345).astype(np.uint16)  # nearly every value escapes
        counts = np.bincount(np.minimum(v, 99), minlength=100).astype(np.uint64)
        f = oracle.quantize(counts, k)
        p = lr.rans_params.make(k, r, l, 2, N, C, "df", True)
        assert lr.rans_encode_bound(v.size, p) >= oracle.encode(f, v, k, r, l, N, C, escape=True).size


def test_division_constants(lr):
    lib = ct.CDLL(lr.LIBRARY_PATH)
    lib.rans_internal_check_division.restype = ct.c_uint64
    lib.rans_internal_check_division.argtypes = [ct.c_uint32, ct.c_uint32]
    assert lib.rans_internal_check_division(1 << 15, 64) == 0


def test_strerror(lr):
    for code in range(0, -8, -1):
        assert lr.rans_strerror(code)


def test_quantizer_hand_computed_cases(lr):
    """The library's own quantiser on the hand-computed tie, forced-symbol and
    excess cases (independent of the oracle)."""
    from conftest import load_golden
    g = load_golden("quantizer_ties.txt")
    for key in g:
        if key.startswith("counts_"):
            nm = key[len("counts_"):]
            got = lr.rans_quantize(np.array(g[key], dtype=np.uint64), g["k_" + nm][0])
            assert [int(v) for v in got] == g["expect_" + nm], nm


def test_struct_layouts_match_the_header(lr, tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's sizes
    and field offsets (a mismatch would shift every field after it)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"rans_params": lr.rans_params, "rans_batch_config": lr.rans_batch_config,
               "rans_tune_result": lr.rans_tune_result, "rans_job": lr.rans_job,
               "rans_server_config": lr.rans_server_config, "rans_completion": lr.rans_completion,
               "rans_server_stats_t": lr.rans_server_stats_t,
               "rans_server_request": lr.rans_server_request}
    # the binding names a field "in_" where C says "in"
    cname = {"in_": "in"}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "librans.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {cname.get(f, f)}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(out[name]) == ct.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(out[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)
