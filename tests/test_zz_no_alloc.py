"""The allocation-free apply (stig_apply_Pinv_noalloc, intermediates in the library's
static per-GPU scratch array) against the workspace apply (stig_apply_Pinv) through the
C ABI: the same kernels, so the results must agree bit for bit, and both within 1e-12 of
the oracle in FP64.  Two calls in a row, the second with a smaller input; a size whose
intermediates exceed the static array is refused before any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import fd
from oracle.problems import CubeProblem

pytestmark = pytest.mark.gpu

PREC = {"fp64": 0, "fp32": 1, "bf16": 2}


def _vp(t):
    return C.c_void_p(t.data_ptr())


def _plan(name, n_el):
    from paper_1909_07309_amd.problem import CubeFactors
    w = wl.WORKLOADS[name] if n_el is None else wl.scaled(wl.WORKLOADS[name], n_el)
    return w, CubeFactors(w).make_plan()


def _both(plan, r, nrhs, prec, transpose):
    """(noalloc result, workspace result) through the C ABI."""
    from paper_1909_07309_amd._lib import lib
    L = lib()
    s_na = torch.full_like(r, float("nan"))
    s_ws = torch.full_like(r, float("nan"))
    plan._ensure_workspace(plan.workspace_bytes(nrhs, 0, prec), r.device)
    plan._sync_stream()
    assert L.stig_apply_Pinv_noalloc(plan._h, _vp(r), _vp(s_na), nrhs, transpose, PREC[prec]) == 0, \
        L.stig_last_error()
    assert L.stig_apply_Pinv(plan._h, _vp(r), _vp(s_ws), nrhs, transpose, PREC[prec]) == 0
    torch.cuda.synchronize()
    return s_na, s_ws


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_noalloc_apply_matches_workspace_apply(prec):
    # a cube with ragged tiles (n_s = 21, n_t = 22) and a batch of 3, then one right-hand
    # side of a smaller square grid (n_s = 15, n_t = 16) on another plan
    w, plan = _plan("cube_p3_n64", 20)
    r = torch.from_numpy(wl.random_tensor((3,) + w.shape, 21)).to("cuda")
    pr = CubeProblem(w)
    P = fd.FDPreconditioner(pr.K1d, pr.M1d, pr.Wt, pr.Mt)
    rh = r.cpu().numpy()
    for tr in (0, 1):
        s_na, s_ws = _both(plan, r, 3, prec, tr)
        assert torch.equal(s_na, s_ws), (prec, tr)
        if prec == "fp64":
            for b in range(3):
                ref = P.apply(rh[b], transpose=bool(tr))
                assert np.abs(s_na[b].cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    w2, plan2 = _plan("square_p2_n8", 15)
    r2 = torch.from_numpy(wl.random_tensor(w2.shape, 22)).to("cuda")
    s_na, s_ws = _both(plan2, r2, 1, prec, 0)
    assert torch.equal(s_na, s_ws)
    # and the first plan again with one right-hand side (smaller than its first call)
    s_na, s_ws = _both(plan, r[:1].contiguous(), 1, prec, 0)
    assert torch.equal(s_na, s_ws)


def test_noalloc_apply_full_size_batch_workload_and_limit():
    """The 48-element cube (5,882,450 unknowns, 94 MB of FP64 intermediates) fits; the
    64-element cube in FP64 (291 MB) is refused with STIG_EINVAL and a message."""
    from paper_1909_07309_amd._lib import lib
    L = lib()
    w, plan = _plan("cube_p3_n48_b32", None)
    r = torch.from_numpy(wl.random_tensor(w.shape, 23)).to("cuda")
    s_na, s_ws = _both(plan, r, 1, "fp64", 0)
    assert torch.equal(s_na, s_ws)
    w1, plan1 = _plan("cube_p3_n64", None)
    r1 = torch.zeros(w1.shape, dtype=torch.float64, device="cuda")
    s1 = torch.empty_like(r1)
    plan1._sync_stream()
    assert L.stig_apply_Pinv_noalloc(plan1._h, _vp(r1), _vp(s1), 1, 0, 0) == -1
    assert b"static scratch" in L.stig_last_error()
    # BF16 at the same size fits (two 2-byte intermediates)
    s_na, s_ws = _both(plan1, r1, 1, "bf16", 0)
    assert torch.equal(s_na, s_ws)
