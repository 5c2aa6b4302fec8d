"""GPU parity for the extruded quarter annulus in 3D (variable conductivity and heat
capacity, p=2): full space-time CSR matvec, the 3D geometry-aware A-hat^G apply in
FP64 and FP32, flexible GMRES solves, against the oracle's independent assembly."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle.annulus3d import Annulus3DProblem

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _setup(n_el):
    from paper_1909_07309_amd.annulus3d import Annulus3DSetup
    base = wl.WORKLOADS["annulus3d_p2_n32"]
    w = wl.scaled(base, n_el) if n_el else base
    a = Annulus3DSetup(w)
    return w, a, a.make_plan(), Annulus3DProblem(w)


@pytest.mark.parametrize("n_el", [6, 12])
def test_annulus3d_csr_matvec_and_preconditioner_match_oracle(n_el):
    w, a, plan, o = _setup(n_el)
    x = wl.random_tensor(w.shape, 3)
    y = plan.matvec_A(_dev(x)).cpu().numpy()
    ref = o.matvec(x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    P = o.preconditioner()
    ref_s = P.apply(x)
    s = plan.apply_Pinv(_dev(x)).cpu().numpy()
    assert np.abs(s - ref_s).max() <= 1e-12 * np.abs(ref_s).max()
    s32 = plan.apply_Pinv(_dev(x), prec="fp32").cpu().numpy()
    assert np.abs(s32 - ref_s).max() <= 1e-4 * np.abs(ref_s).max()


def test_annulus3d_solve_reduced_size():
    w, a, plan, o = _setup(10)
    f = a.source()
    f_ref = o.source()
    assert np.abs(f.cpu().numpy() - f_ref).max() <= 1e-13 * np.abs(f_ref).max()
    u, info = plan.gmres_solve(f, restart=30, rtol=1e-8, maxit=300, flexible=True, prec="fp32")
    r = f_ref - o.matvec(u.cpu().numpy())
    assert np.linalg.norm(r) / np.linalg.norm(f_ref) <= 1e-8
    u64, info64 = plan.gmres_solve(f, restart=30, rtol=1e-8, maxit=300, flexible=True)
    u, u64 = u.cpu().numpy(), u64.cpu().numpy()
    assert np.linalg.norm(u - u64) / np.linalg.norm(u64) <= 1e-6
    assert info["iters"] < 60 and abs(info["iters"] - info64["iters"]) <= 2


def test_annulus3d_full_size_csr_and_solve():
    """32 elements per direction, p = 2: 32^3 x 33 = 1,081,344 unknowns, ~5.8e8 CSR entries."""
    w, a, plan, o = _setup(None)
    x = wl.random_tensor(w.shape, 5)
    y = plan.matvec_A(_dev(x)).cpu().numpy()
    ref = o.matvec(x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    # the 3D A-hat^G apply at n_s = 32 (compile-time mode products with the
    # diagonal scaling fused into the first and last), element by element
    # against the oracle, FP64 and FP32, plain and transposed, with both forms
    # of step 3 (the default at n_t = 33 is the arrowhead form, whose products
    # along t have a compile-time kernel; the generic banded elimination)
    P = o.preconditioner()
    for kernel in ("right_looking", "generic"):
        plan.set_option("time_kernel", kernel)
        for tr in (False, True):
            ref_s = P.apply(x, transpose=tr)
            s64 = plan.apply_Pinv(_dev(x), transpose=tr).cpu().numpy()
            s32 = plan.apply_Pinv(_dev(x), transpose=tr, prec="fp32").cpu().numpy()
            e64 = np.abs(s64 - ref_s).max() / np.abs(ref_s).max()
            e32 = np.abs(s32 - ref_s).max() / np.abs(ref_s).max()
            print(f"3D annulus apply ({kernel}, transpose={tr}): FP64 {e64:.2e}, FP32 {e32:.2e}")
            assert e64 <= 1e-12 and e32 <= 1e-4
    plan.set_option("time_kernel", "right_looking")
    f = a.source()
    u, info = plan.gmres_solve(f, restart=30, rtol=1e-8, maxit=300, flexible=True, prec="fp32")
    f_ref = o.source()
    r = f_ref - o.matvec(u.cpu().numpy())
    relres = np.linalg.norm(r) / np.linalg.norm(f_ref)
    print(f"3D annulus full size: {info['iters']} FGMRES iterations, oracle residual {relres:.2e}")
    assert relres <= 1e-8
