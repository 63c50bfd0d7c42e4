"""The allocation-free modified Cholesky (afqmc_modified_cholesky_noalloc) against the entry
point that takes a caller workspace (afqmc_modified_cholesky), called through the C ABI: the
same vectors, count and convergence flag on two calls in a row, the second with a smaller
tensor (the library's static scratch keeps the first call's contents), and sizes beyond the
scratch's limit refused before any device work."""

import ctypes as C

import numpy as np
import pytest

from tests.parity_helpers import log

pytestmark = pytest.mark.gpu


def _eri(M, seed):
    rng = np.random.default_rng(seed)
    n = M * M
    B = rng.standard_normal((n, M, M))
    B = B + B.transpose(0, 2, 1)
    w = np.exp(-np.arange(n) / (0.8 * M)) / M
    return np.einsum("k,kpr,kqs->pqrs", w, B, B)


def _lib():
    import paper_1711_02242_amd as afq
    lib = afq.load()
    lib.afqmc_modified_cholesky_noalloc.argtypes = [
        C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.c_void_p, C.POINTER(C.c_int32),
        C.POINTER(C.c_int32), C.c_void_p]
    lib.afqmc_modified_cholesky_noalloc.restype = C.c_int
    return lib


def _run(lib, eri_np, delta, noalloc):
    import torch
    M = eri_np.shape[0]
    eri = torch.from_numpy(eri_np).cuda()
    out = torch.full((M * M, M, M), float("nan"), dtype=torch.float64, device="cuda")
    n, conv = C.c_int32(-1), C.c_int32(-1)
    stream = C.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    if noalloc:
        rc = lib.afqmc_modified_cholesky_noalloc(C.c_void_p(eri.data_ptr()), M, delta, M * M,
                                                 C.c_void_p(out.data_ptr()), C.byref(n),
                                                 C.byref(conv), stream)
    else:
        wb = C.c_size_t()
        assert lib.afqmc_mcd_workspace_bytes(M, C.byref(wb)) == 0
        raw = torch.empty(wb.value + 256, dtype=torch.uint8, device="cuda")
        off = (-int(raw.data_ptr())) % 256
        rc = lib.afqmc_modified_cholesky(C.c_void_p(eri.data_ptr()), M, delta, M * M,
                                         C.c_void_p(out.data_ptr()), C.byref(n), C.byref(conv),
                                         C.c_void_p(raw.data_ptr() + off), wb.value, stream)
    assert rc == 0, rc
    torch.cuda.synchronize()
    return out[: n.value].cpu().numpy(), n.value, conv.value


def test_noalloc_matches_workspace_entry_point_two_calls():
    lib = _lib()
    for M, delta, seed in ((14, 1e-6, 3), (9, 1e-5, 4)):    # second call smaller
        eri = _eri(M, seed)
        log(f"no-alloc mcd M={M} delta={delta}")
        ref, n_ref, c_ref = _run(lib, eri, delta, noalloc=False)
        got, n_got, c_got = _run(lib, eri, delta, noalloc=True)
        assert n_got == n_ref and c_got == c_ref == 1
        assert np.array_equal(got, ref)               # same kernels, same arithmetic
        V = eri.transpose(0, 2, 1, 3).reshape(M * M, M * M)
        R = V - got.reshape(n_got, -1).T @ got.reshape(n_got, -1)
        assert np.abs(R).max() <= delta * (1 + 1e-9)
        log(f"  {n_got} vectors, identical")


def test_noalloc_refuses_sizes_beyond_scratch():
    lib = _lib()
    n, conv = C.c_int32(-1), C.c_int32(-1)
    # M = 257 exceeds the scratch (M <= 256): refused on the host, before any device access
    rc = lib.afqmc_modified_cholesky_noalloc(C.c_void_p(8), 257, 1e-6, 1, C.c_void_p(8),
                                             C.byref(n), C.byref(conv), None)
    assert rc == -2 and n.value == -1
