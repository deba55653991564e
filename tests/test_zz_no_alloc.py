"""The allocation-free encode entry point against rans_encode_async.

rans_encode_async_noalloc takes its scratch from the library's fixed device
array; its containers must equal rans_encode_async's byte for byte (and the
oracle's), on two calls in a row with the second input smaller, so stale
scratch from the first call cannot leak into the second.  Inputs beyond the
array's capacity are refused before anything is launched."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lr():
    import torch
    assert torch.cuda.is_available()
    import paper_1402_3392_amd as m
    return m


def _encode(lr, fn, table, params, d_syms, n, cap):
    import torch
    d_out = torch.full((cap,), 0xA5, dtype=torch.uint8, device="cuda")
    meta = torch.zeros(4, dtype=torch.int64, device="cuda")  # [len, status]
    fn(table, params, d_syms, n, d_out, cap, int(meta.data_ptr()), int(meta.data_ptr()) + 8)
    torch.cuda.synchronize()
    olen, st = int(meta[0]), int(meta.view(torch.int32)[2])
    assert st == 0, st
    return d_out[:olen].cpu().numpy()


@pytest.mark.parametrize("k,r,l,N,C", [(14, 16, 16, 64, 65536), (11, 8, 23, 32, 8192),
                                       (12, 16, 16, 4, 0)])
def test_noalloc_equals_workspace_encode(lr, k, r, l, N, C):
    import torch
    rng = np.random.Generator(np.random.PCG64(9100 + k + N))
    big = datagen.sample(datagen.zipf_probs(256, 1.1), (3 << 20) + 13, rng)
    small = big[: (1 << 20) - 7] if C else big[: 300_001]
    if not C:
        big = big[: 700_003]  # one chunk: n must fit one chunk's 32-bit count
    table = lr.rans_tables_build(datagen.counts(big, 256), k)
    f = oracle.quantize(datagen.counts(big, 256), k)
    params = lr.rans_params.make(k, r, l, 1, N, C)
    for syms in (big, small):  # the second call is smaller
        d = torch.from_numpy(syms).cuda()
        cap = lr.rans_encode_bound(syms.size, params)
        got = _encode(lr, lr.rans_encode_async_noalloc, table, params, d, syms.size, cap)
        ref = _encode(lr, lr.rans_encode_async, table, params, d, syms.size, cap)
        assert got.size == ref.size and (got == ref).all()
        want = oracle.encode(f, syms, k, r, l, N, C, threads=8)
        assert got.size == want.size and (got == want).all()


def test_noalloc_allocates_nothing_and_refuses_oversized_inputs(lr):
    import torch
    rng = np.random.Generator(np.random.PCG64(9200))
    syms = datagen.sample(datagen.zipf_probs(256, 0.9), 1 << 22, rng)
    table = lr.rans_tables_build(datagen.counts(syms, 256), 14)
    params = lr.rans_params.make(14, 16, 16, 1, 64, 65536)
    d = torch.from_numpy(syms).cuda()
    cap = lr.rans_encode_bound(syms.size, params)
    d_out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    meta = torch.zeros(4, dtype=torch.int64, device="cuda")
    lr.rans_encode_async_noalloc(table, params, d, syms.size, d_out, cap, int(meta.data_ptr()),
                                 int(meta.data_ptr()) + 8)  # warm-up: loads the kernels
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        meta.zero_()
        lr.rans_encode_async_noalloc(table, params, d, syms.size, d_out, cap,
                                     int(meta.data_ptr()), int(meta.data_ptr()) + 8)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert int(meta.view(torch.int32)[2]) == 0
    # 48 Mi symbols need about 96 MiB of digit slots: more than the array
    n = 48 << 20
    d_big = torch.zeros(n, dtype=torch.uint8, device="cuda")
    cap = lr.rans_encode_bound(n, params)
    d_out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    with pytest.raises(lr.RansError) as e:
        lr.rans_encode_async_noalloc(table, params, d_big, n, d_out, cap, int(meta.data_ptr()),
                                     int(meta.data_ptr()) + 8)
    assert e.value.code == lr.RANS_ENOMEM
