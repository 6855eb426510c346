"""The allocation-free transpose (lsq2l_transpose_noalloc) through the C ABI
against the allocating one (lsq2l_transpose): bit-exact on two calls in a
row, the second with a smaller input (the static work space keeps the first
call's contents), plus its size limit."""
import ctypes as C

import numpy as np
import pytest

from workloads import generators as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need a ROCm device"
    import paper_2107_09006_amd as lib
    lib.load_library()
    return lib


def _out(torch, n, nnz):
    return (torch.empty(n + 1, dtype=torch.int32, device="cuda"),
            torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda"),
            torch.empty(max(nnz, 1), dtype=torch.float64, device="cuda"),
            torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda"))


def test_noalloc_transpose_matches_allocating_one(L):
    import torch
    big = W.small_config("irregular")                 # 24,000 x 6,000, ragged rows
    small = W.random_banded(900, 2100, 4, seed=5)      # then a smaller one
    for p in (big, small):
        ref = L.transpose(p.m, p.n, p.indptr, p.indices, p.data)
        torch.cuda.synchronize()
        out = _out(torch, p.n, p.nnz)
        got = L.transpose(p.m, p.n, p.indptr, p.indices, p.data, noalloc=True, out=out)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
        A = p.scipy().T.tocsr()
        A.sort_indices()
        assert np.array_equal(got[0].cpu().numpy(), A.indptr)
        assert np.array_equal(got[1].cpu().numpy(), A.indices)


def test_noalloc_transpose_rejects_oversize_and_bad_columns(L):
    import torch
    lib = L.load_library()
    # 12.6M entries: the radix sort's ping-pong keys and values alone need
    # 100 MiB, so the 104 MiB work space cannot hold them; the call is
    # rejected on the host before any device work
    n, nnz = 1 << 24, (1 << 23) + (1 << 22)
    rp = torch.tensor([0, nnz], dtype=torch.int32, device="cuda")
    ci = torch.arange(nnz, dtype=torch.int32, device="cuda")
    trp = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    tr = torch.empty(nnz, dtype=torch.int32, device="cuda")
    st = lib.lsq2l_transpose_noalloc(1, n, nnz, C.c_void_p(rp.data_ptr()), C.c_void_p(ci.data_ptr()),
                                     None, C.c_void_p(trp.data_ptr()), C.c_void_p(tr.data_ptr()),
                                     None, None, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == L.EINVAL and b"work space" in lib.lsq2l_last_error()
    p = W.banded_1000()
    bad = p.indices.copy()
    bad[7] = -1
    with pytest.raises(L.Lsq2lError) as e:
        L.transpose(p.m, p.n, p.indptr, bad, p.data, noalloc=True, out=_out(torch, p.n, p.nnz))
    assert e.value.status == L.EINVAL
