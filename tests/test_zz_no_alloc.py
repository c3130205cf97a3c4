"""mm_demag_apply_static, the allocation-free variant of mm_demag_apply (its
half spectra in the library's fixed device array), against mm_demag_apply
through the C ABI: bitwise equal on two calls in a row, the second on a
smaller grid; grids beyond the array are rejected."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from gpucommon import rel_l2, say, to_dev, to_host
from paper_1406_7459_amd import workloads as W

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1406_7459_amd import mm
    L = mm.lib()
    L.mm_demag_apply_static.argtypes = [C.c_void_p] * 4
    L.mm_demag_apply_static.restype = C.c_int
    L.mm_demag_static_scratch_bytes.argtypes = []
    L.mm_demag_static_scratch_bytes.restype = C.c_size_t
    return mm, L


def test_static_apply_matches_workspace_apply_twice_then_smaller():
    mm, L = _lib()
    s = torch.cuda.current_stream().cuda_stream
    for grid, d, seed in (((48, 24, 6), (2e-9, 3e-9, 2e-9), 1), ((12, 8, 1), (4e-9, 4e-9, 3e-9), 2)):
        say("static apply", grid)
        plan = mm.Plan(*grid, *d)
        M = to_dev(8e5 * W.random_unit(*grid, seed=seed))
        ref = to_host(plan.demag(M))
        H = torch.full_like(M, float("nan"))
        assert L.mm_demag_apply_static(plan._h, M.data_ptr(), H.data_ptr(), s) == mm.MM_OK
        got = to_host(H)
        assert np.array_equal(got, ref)
        Ho = oracle.Demag(*grid, *d).apply(to_host(M))
        assert rel_l2(got, Ho) < 1e-5
        plan.close()


def test_static_apply_rejects_grids_beyond_the_array():
    mm, L = _lib()
    cap = L.mm_demag_static_scratch_bytes()
    assert cap == 64 << 20
    plan = mm.Plan(256, 256, 16, 2e-9, 2e-9, 2e-9)  # X1 + X2 = 80 MiB
    M = torch.zeros(plan.field_shape, dtype=torch.float32, device="cuda")
    H = torch.empty_like(M)
    assert L.mm_demag_apply_static(plan._h, M.data_ptr(), H.data_ptr(), None) == mm.MM_EINVAL
    assert L.mm_demag_apply_static(None, M.data_ptr(), H.data_ptr(), None) == mm.MM_EINVAL
    plan.close()
