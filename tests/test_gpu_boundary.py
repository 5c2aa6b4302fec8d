"""GPU tests of the C-ABI boundary itself: the caller-owned workspace (the hot-path
calls allocate nothing), the accumulate form of the initial-datum lifting,
bitwise repeatability of the apply, the matvec and the solves, and a breakdown
forced from the host (gamma = nu = 0 makes every shifted time system singular;
the setup's pivot pass reports it through a flag, every kernel exits normally)."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import fd
from oracle.problems import CubeProblem

pytestmark = pytest.mark.gpu


def _vp(t):
    return C.c_void_p(t.data_ptr())


def _setup(name, n_el):
    from paper_1909_07309_amd.problem import CubeFactors
    w = wl.WORKLOADS[name] if n_el is None else wl.scaled(wl.WORKLOADS[name], n_el)
    fac = CubeFactors(w)
    return w, fac, fac.make_plan()


def test_workspace_is_caller_owned_full_size():
    """The 64-element cube (18,125,250 unknowns): a workspace allocated by torch, then the
    FP64 apply, the matvec and a GMRES(30) solve through the C ABI.  The plan's own device
    bytes and the device's free memory do not change across those calls, and the results
    match the oracle."""
    from paper_1909_07309_amd._lib import StigInfo, lib
    from paper_1909_07309_amd.problem import source
    w, fac, plan = _setup("cube_p3_n64", None)
    f = source(w, plan)
    need = plan.workspace_bytes(1, 30, "fp64")
    assert need >= (3 * 30 + 3) * w.N * 8
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    plan.set_workspace(ws)
    s = torch.empty_like(f)
    y = torch.empty_like(f)
    u = torch.zeros_like(f)
    L = lib()
    h = plan._h
    plan._sync_stream()
    torch.cuda.synchronize()
    held = plan.device_bytes()
    free0 = torch.cuda.mem_get_info()[0]
    assert L.stig_apply_Pinv(h, _vp(f), _vp(s), 1, 0, 0) == 0
    assert L.stig_matvec_A(h, _vp(s), _vp(y), 1, 0) == 0
    info = StigInfo()
    assert L.stig_gmres_solve(h, _vp(f), _vp(u), 1, 30, 1e-8, 300, 0, 0, 0, C.byref(info)) == 0
    torch.cuda.synchronize()
    assert plan.device_bytes() == held
    assert torch.cuda.mem_get_info()[0] == free0
    pr = CubeProblem(w)
    f_ref = pr.source()
    ref = fd.FDPreconditioner(pr.K1d, pr.M1d, pr.Wt, pr.Mt).apply(f_ref)
    s_h = s.cpu().numpy()
    assert np.abs(s_h - ref).max() <= 1e-12 * np.abs(ref).max()
    # P = A on the cube: A s reproduces f
    assert np.abs(y.cpu().numpy() - f_ref).max() <= 1e-12 * np.abs(f_ref).max()
    u_h = u.cpu().numpy()
    r = f_ref - fd.kron_matvec(u_h, pr.Wt, pr.Mt, pr.K1d, pr.M1d)
    relres = np.linalg.norm(r) / np.linalg.norm(f_ref)
    assert relres <= 1e-8
    # the reported residual is a fresh product: it agrees with the oracle's
    assert abs(info.relres_true - relres) <= 1e-3 * relres + 1e-15
    # a workspace too small for the solve, then none: refused, nothing launched
    assert L.stig_set_workspace(h, _vp(ws), need // 2) == 0
    assert L.stig_gmres_solve(h, _vp(f), _vp(u), 1, 30, 1e-8, 300, 0, 0, 0, None) == -1
    assert b"workspace" in L.stig_last_error()
    assert L.stig_set_workspace(h, None, 0) == 0
    assert L.stig_apply_Pinv(h, _vp(f), _vp(s), 1, 0, 0) == -6
    assert b"workspace" in L.stig_last_error()
    assert L.stig_set_workspace(h, _vp(ws), need) == 0
    assert plan.device_bytes() == held


def test_lift_apply_accumulate_form():
    """y = f - A_{I,0} c0 in one call equals f minus the plain lifting product."""
    w, fac, plan = _setup("cube_p3_n48_b32", 6)
    nb = 3
    c0 = torch.from_numpy(wl.random_tensor((nb,) + w.shape[1:], 4)).to("cuda")
    f = torch.from_numpy(wl.random_tensor((nb,) + w.shape, 5)).to("cuda")
    lift = plan.lift_apply(fac.W_col0, fac.M_col0, c0)
    y = plan.lift_apply(fac.W_col0, fac.M_col0, c0, f=f)
    ref = (f - lift).cpu().numpy()
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-14 * np.abs(ref).max()
    # in place (f is y)
    g = f.clone()
    plan.lift_apply(fac.W_col0, fac.M_col0, c0, f=g, y=g)
    assert torch.equal(g, y)


@pytest.mark.parametrize("name,n_el", [("cube_p3_n64", 20), ("cube_p3_n64", None)])
def test_bitwise_repeatable(name, n_el):
    """Two identical applies (every precision, plain and transposed), matvecs and solves
    give bit-identical results: fixed grids and fixed reduction orders, no atomics."""
    from paper_1909_07309_amd.problem import source
    w, fac, plan = _setup(name, n_el)
    f = source(w, plan)
    for prec in ("fp64", "fp32", "bf16"):
        for tr in (False, True):
            a = plan.apply_Pinv(f, prec=prec, transpose=tr)
            b = plan.apply_Pinv(f, prec=prec, transpose=tr)
            assert torch.equal(a, b), (prec, tr)
    assert torch.equal(plan.matvec_A(f), plan.matvec_A(f))
    for prec, flex in (("fp64", False), ("fp32", True)):
        u1, i1 = plan.gmres_solve(f, restart=30, rtol=1e-8, maxit=300, prec=prec, flexible=flex)
        u2, i2 = plan.gmres_solve(f, restart=30, rtol=1e-8, maxit=300, prec=prec, flexible=flex)
        assert torch.equal(u1, u2) and i1["iters"] == i2["iters"]
        assert i1["relres_true"] == i2["relres_true"]


@pytest.mark.parametrize("name,n_el", [("square_p2_n8", None), ("cube_p3_n64", 5),
                                       ("cube_p3_n64", 64)])
def test_breakdown_forced_from_the_host(name, n_el):
    """gamma = nu = 0: every shifted system gamma W_t + nu lambda M_t is zero, so the setup's
    pivot pass (register-resident kernel for n_t = 9 and 66, generic one for n_t = 7) sets
    the breakdown flag and the setup returns STIG_EBREAKDOWN; the plan is then not usable
    until a valid setup."""
    from paper_1909_07309_amd import StigError
    from paper_1909_07309_amd.problem import CubeFactors
    w = wl.WORKLOADS[name] if n_el is None else wl.scaled(wl.WORKLOADS[name], n_el)
    fac = CubeFactors(w)
    from paper_1909_07309_amd.api import Plan
    plan = Plan([w.n_s] * w.d, w.n_t, w.p, w.p)
    with pytest.raises(StigError) as e:
        plan.setup_1d_pencils(fac.K1d, fac.M1d, fac.Wt, fac.Mt, 0.0, 0.0)
    assert e.value.code == -4
    x = torch.ones(w.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(StigError) as e:
        plan.apply_Pinv(x)
    assert e.value.code == -6
    plan.setup_1d_pencils(fac.K1d, fac.M1d, fac.Wt, fac.Mt, 1.0, 1.0)
    s = plan.apply_Pinv(x)
    assert bool(torch.isfinite(s).all())
