"""GPU parity for the quarter-annulus workload (variable conductivity and heat
capacity, p=4): full space-time CSR matvec, geometry-aware A-hat^G apply in FP64
and FP32, flexible GMRES solves, against the oracle's independent assembly."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import fd
from oracle.annulus import AnnulusProblem

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _setup(n_el):
    from paper_1909_07309_amd.annulus import AnnulusSetup
    w = wl.scaled(wl.WORKLOADS["annulus_p4_n128"], n_el) if n_el else wl.WORKLOADS["annulus_p4_n128"]
    a = AnnulusSetup(w)
    return w, a, a.make_plan(), AnnulusProblem(w)


def test_annulus_csr_matvec_and_preconditioner_match_oracle():
    w, a, plan, o = _setup(20)
    x = wl.random_tensor(w.shape, 3)
    y = plan.matvec_A(_dev(x)).cpu().numpy()
    ref = o.matvec(x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    P = o.preconditioner()
    ref_s = P.apply(x)
    ref_t = P.apply(x, transpose=True)
    s = plan.apply_Pinv(_dev(x)).cpu().numpy()
    assert np.abs(s - ref_s).max() <= 1e-12 * np.abs(ref_s).max()
    s32 = plan.apply_Pinv(_dev(x), prec="fp32").cpu().numpy()
    assert np.abs(s32 - ref_s).max() <= 1e-4 * np.abs(ref_s).max()
    # both forms of step 3 (the default picks the arrowhead form at n_t = 131:
    # MFMA products along t around the block-LU middle factor; the generic
    # banded elimination on request)
    for tk in ("arrowhead", "generic"):
        plan.set_option("time_kernel", tk)
        for tr, ref in ((False, ref_s), (True, ref_t)):
            sa = plan.apply_Pinv(_dev(x), transpose=tr).cpu().numpy()
            ea = np.abs(sa - ref).max() / np.abs(ref).max()
            sa32 = plan.apply_Pinv(_dev(x), transpose=tr, prec="fp32").cpu().numpy()
            ea32 = np.abs(sa32 - ref).max() / np.abs(ref).max()
            print(f"annulus {tk} apply (transpose={tr}): FP64 {ea:.2e}, FP32 {ea32:.2e}")
            assert ea <= 1e-12 and ea32 <= 1e-4
    plan.set_option("time_kernel", "right_looking")
    # diag(A-hat^G) = diag(A): D^{1/2} A-tilde D^{1/2} reproduces the diagonal exactly
    assert np.allclose(o.D().ravel() * o.diag_Atilde().ravel(), o.diag_A().ravel(), rtol=1e-13)


def test_annulus_solve_reduced_size():
    w, a, plan, o = _setup(20)
    f = a.source()
    f_ref = o.source()
    assert np.abs(f.cpu().numpy() - f_ref).max() <= 1e-13 * np.abs(f_ref).max()
    u, info = plan.gmres_solve(f, restart=30, rtol=1e-8, maxit=200, flexible=True, prec="fp32")
    u = u.cpu().numpy()
    A = o.dense_A()
    res = np.linalg.norm(f_ref.ravel() - A @ u.ravel()) / np.linalg.norm(f_ref)
    assert res <= 1e-8
    u_ref = np.linalg.solve(A, f_ref.ravel())
    assert np.linalg.norm(u.ravel() - u_ref) / np.linalg.norm(u_ref) <= 1e-6
    assert info["iters"] < 40


def test_annulus_full_size_csr_and_solve():
    """128 elements per direction, p = 4: 2,213,900 unknowns, ~1.5e9 CSR entries."""
    w, a, plan, o = _setup(None)
    x = wl.random_tensor(w.shape, 5)
    y = plan.matvec_A(_dev(x)).cpu().numpy()
    ref = o.matvec(x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    # the FP64 / FP32 A-hat^G apply at n_s = 130 (mode products split over
    # blocks of one XCD, diagonal scaling fused), against the oracle's fast
    # diagonalization, element by element, and through the residual
    # ||A-hat^G s - x|| / ||x|| with the oracle's factored product
    # A-hat^G = D^{1/2} (W_t (x) M-tilde_s + M_t' (x) K-tilde_s) D^{1/2}
    P = o.preconditioner()
    Dh = np.sqrt(o.D())

    def ahat(v, transpose=False):
        return Dh * fd.kron_matvec(Dh * v, o.Wt, o.Mt, o.Kt, o.Mtl, transpose=transpose)

    ref_s = P.apply(x)
    s64 = plan.apply_Pinv(_dev(x)).cpu().numpy()
    err = np.abs(s64 - ref_s).max() / np.abs(ref_s).max()
    res = np.linalg.norm(ahat(s64) - x) / np.linalg.norm(x)
    st = plan.apply_Pinv(_dev(x), transpose=True).cpu().numpy()
    ref_t = P.apply(x, transpose=True)
    err_t = np.abs(st - ref_t).max() / np.abs(ref_t).max()
    res_t = np.linalg.norm(ahat(st, True) - x) / np.linalg.norm(x)
    print(f"annulus FP64 apply: max rel err {err:.2e} / {err_t:.2e} (plain / transposed), "
          f"residual {res:.2e} / {res_t:.2e}")
    assert res <= 1e-13 and res_t <= 1e-13
    assert err <= 1e-12 and err_t <= 1e-12
    s32 = plan.apply_Pinv(_dev(x), prec="fp32").cpu().numpy()
    assert np.abs(s32 - ref_s).max() <= 1e-4 * np.abs(ref_s).max()
    f = a.source()
    u, info = plan.gmres_solve(f, restart=30, rtol=1e-8, maxit=300, flexible=True, prec="fp32")
    f_ref = o.source()
    r = f_ref - o.matvec(u.cpu().numpy())
    relres = np.linalg.norm(r) / np.linalg.norm(f_ref)
    print(f"annulus full size: {info['iters']} FGMRES iterations, oracle residual {relres:.2e}")
    assert relres <= 1e-8
