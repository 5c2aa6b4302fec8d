"""GPU parity for the matvec with sparse spatial factors (Section 4.5: only the
spatial and time factors of A are stored) on the quarter annulus (2D, p = 4)
and the extruded quarter annulus (3D, p = 2): plain and transposed products,
batches, the residual path inside (F)GMRES and the adjoint solve, against the
oracle's independent assembly.  Shapes span several 256-row blocks with a
ragged last block and time levels that are not a multiple of the 8-level
chunks of the spatial pass."""
import numpy as np
import pytest
import torch

import workloads as wl
from paper_1909_07309_amd._lib import StigError
from oracle.annulus import AnnulusProblem
from oracle.annulus3d import Annulus3DProblem

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _setup(d, n_el, matvec="factored"):
    if d == 2:
        from paper_1909_07309_amd.annulus import AnnulusSetup as Setup
        base, Oracle = wl.WORKLOADS["annulus_p4_n128"], AnnulusProblem
    else:
        from paper_1909_07309_amd.annulus3d import Annulus3DSetup as Setup
        base, Oracle = wl.WORKLOADS["annulus3d_p2_n32"], Annulus3DProblem
    w = wl.scaled(base, n_el) if n_el else base
    a = Setup(w)
    return w, a, a.make_plan(matvec=matvec), Oracle(w)


def _oracle_transposed(o, x):
    """A^T x = (W_t^T (x) M_s^T + M_t^T (x) K_s^T) x from the oracle's factor matrices."""
    X = np.asarray(x).reshape(o.w.n_t, -1)
    MX = (o.Ms.T @ X.T).T
    KX = (o.Ks.T @ X.T).T
    return (o.Wt.T @ MX + o.Mt.T @ KX).reshape(np.shape(x))


@pytest.mark.parametrize("d,n_el", [(2, 6), (2, 20), (3, 4), (3, 9)])
def test_factored_matvec_matches_dense_oracle(d, n_el):
    w, a, plan, o = _setup(d, n_el)
    x = wl.random_tensor((2,) + w.shape, 11)
    A = o.dense_A()
    y = plan.matvec_A(_dev(x)).cpu().numpy()
    yt = plan.matvec_A(_dev(x), transpose=True).cpu().numpy()
    for r in range(2):
        ref = A @ x[r].ravel()
        reft = A.T @ x[r].ravel()
        assert np.abs(y[r].ravel() - ref).max() <= 1e-13 * np.abs(ref).max()
        assert np.abs(yt[r].ravel() - reft).max() <= 1e-13 * np.abs(reft).max()


@pytest.mark.parametrize("d", [2, 3])
def test_factored_form_replaces_and_is_replaced_by_csr(d):
    w, a, plan, o = _setup(d, 6, matvec="csr")
    x = wl.random_tensor(w.shape, 2)
    ref = o.matvec(x)
    y_csr = plan.matvec_A(_dev(x)).cpu().numpy()
    with pytest.raises(StigError):
        plan.matvec_A(_dev(x), transpose=True)       # the CSR form has no transpose
    plan.set_spatial_factors(a.space)                 # clears the CSR
    y_fac = plan.matvec_A(_dev(x)).cpu().numpy()
    plan.matvec_A(_dev(x), transpose=True)
    rowptr, col, val = plan.kron_csr(a.space, a.Wt, a.Mt)
    plan.set_A_csr(rowptr, col, val)                  # clears the factors
    with pytest.raises(StigError):
        plan.matvec_A(_dev(x), transpose=True)
    plan.set_A_csr(None, None, None)
    plan.set_spatial_factors(None)                    # back to the plan's Kronecker factors
    y_kron = plan.matvec_A(_dev(x)).cpu().numpy()
    for y in (y_csr, y_fac):
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    # the Kronecker factors are the separated approximation, not A
    assert np.abs(y_kron - ref).max() > 1e-6 * np.abs(ref).max()


@pytest.mark.parametrize("d", [2, 3])
def test_factored_form_rejects_bad_pattern(d):
    w, a, plan, o = _setup(d, 6)
    rp, col, vK, vM = a.space
    bad = col.copy()
    bad[5] = plan.N_s
    with pytest.raises(StigError):
        plan.set_spatial_factors((rp, bad, vK, vM))
    # nothing changed: the factors set before still give A x
    x = wl.random_tensor(w.shape, 4)
    ref = o.matvec(x)
    y = plan.matvec_A(_dev(x)).cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("d", [2, 3])
def test_factored_full_size_matvec_transpose_and_solve(d):
    """2D: 130^2 x 131 = 2,213,900 unknowns; 3D: 32^3 x 33 = 1,081,344 unknowns."""
    w, a, plan, o = _setup(d, None)
    x = wl.random_tensor(w.shape, 5)
    y = plan.matvec_A(_dev(x)).cpu().numpy()
    ref = o.matvec(x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    yt = plan.matvec_A(_dev(x), transpose=True).cpu().numpy()
    reft = _oracle_transposed(o, x)
    assert np.abs(yt - reft).max() <= 1e-13 * np.abs(reft).max()
    f = a.source()
    f_ref = o.source()
    u, info = plan.gmres_solve(f, restart=30, rtol=1e-8, maxit=300, flexible=True, prec="fp32")
    r = f_ref - o.matvec(u.cpu().numpy())
    relres = np.linalg.norm(r) / np.linalg.norm(f_ref)
    print(f"d={d} factored matvec: {info['iters']} FGMRES iterations, oracle residual {relres:.2e}")
    assert relres <= 1e-8
    assert abs(info["relres_true"] - relres) <= 1e-3 * relres + 1e-15
    it_csr = 18 if d == 2 else 12     # iterations of the same solve with the space-time CSR
    assert abs(info["iters"] - it_csr) <= 1


@pytest.mark.parametrize("d,n_el", [(2, 12), (3, 6)])
def test_factored_adjoint_solve_matches_dense_oracle(d, n_el):
    w, a, plan, o = _setup(d, n_el)
    g = wl.random_tensor(w.shape, 8)
    lam, info = plan.gmres_solve(_dev(g), restart=30, rtol=1e-10, maxit=300, transpose=True)
    At = o.dense_A().T
    lam = lam.cpu().numpy().ravel()
    res = np.linalg.norm(g.ravel() - At @ lam) / np.linalg.norm(g)
    assert res <= 1e-10
    ref = np.linalg.solve(At, g.ravel())
    assert np.linalg.norm(lam - ref) / np.linalg.norm(ref) <= 1e-7


def _dense_kron(Wt, Mt, Ms, Ks):
    """W_t (x) M_s + M_t (x) K_s (eq. syst_mat with gamma = nu = 1), dense."""
    return np.kron(Wt, Ms) + np.kron(Mt, Ks)


def _csr_to_dense(rp, col, val, n):
    D = np.zeros((n, n))
    for r in range(n):
        for e in range(rp[r], rp[r + 1]):
            D[r, col[e]] += val[e]
    return D


@pytest.mark.parametrize("layout", ["diagonals", "rows"])
@pytest.mark.parametrize("n_el", [6, 20])
def test_nonsymmetric_spatial_factors_both_layouts(layout, n_el):
    """Random non-symmetric values, on the annulus pattern (stored by diagonals) or on a
    scattered random pattern (too many distinct offsets: stored by padded rows); plain
    and transposed products against the dense Kronecker sum."""
    w, a, plan, o = _setup(2, n_el, matvec=None)
    Ns = plan.N_s
    rng = np.random.default_rng(100 + n_el)
    if layout == "diagonals":
        rp, col = a.space[0], a.space[1]
    else:
        rows = [np.unique(rng.integers(0, Ns, size=1 + r % 9)) for r in range(Ns)]
        rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
        col = np.concatenate(rows).astype(np.int32)
    vK = rng.standard_normal(col.size)
    vM = rng.standard_normal(col.size)
    plan.set_spatial_factors((rp, col, vK, vM))
    A = _dense_kron(a.Wt, a.Mt, _csr_to_dense(rp, col, vM, Ns), _csr_to_dense(rp, col, vK, Ns))
    x = wl.random_tensor((2,) + w.shape, 21)
    y = plan.matvec_A(_dev(x)).cpu().numpy()
    yt = plan.matvec_A(_dev(x), transpose=True).cpu().numpy()
    for r in range(2):
        ref, reft = A @ x[r].ravel(), A.T @ x[r].ravel()
        assert np.abs(y[r].ravel() - ref).max() <= 1e-13 * np.abs(ref).max()
        assert np.abs(yt[r].ravel() - reft).max() <= 1e-13 * np.abs(reft).max()


@pytest.mark.parametrize("d,n_el", [(2, 12), (3, 8)])
def test_factored_batched_solve_matches_one_by_one(d, n_el):
    """Several right-hand sides in one FGMRES call with the sparse-factor matvec (first
    restart cycle in lockstep, restart length 4 so the one-by-one hand-over runs too)
    against separate calls, and the oracle's residual for each; one right-hand side
    starts from a nonzero guess."""
    w, a, plan, o = _setup(d, n_el)
    f1 = _dev(o.source())
    f = torch.stack([f1, _dev(wl.random_tensor(w.shape, 41)), 2.0 * f1])
    u0 = torch.zeros_like(f)
    u0[1] = _dev(wl.random_tensor(w.shape, 42))
    ub, info = plan.gmres_solve(f, u0.clone(), restart=4, rtol=1e-9, maxit=400, flexible=True,
                                prec="fp32")
    assert info["converged"]
    A = o.dense_A()
    fh = f.cpu().numpy()
    for r in range(3):
        ur, _ = plan.gmres_solve(f[r].clone(), u0[r].clone(), restart=4, rtol=1e-9, maxit=400,
                                 flexible=True, prec="fp32")
        x, y = ub[r].cpu().numpy().ravel(), ur.cpu().numpy().ravel()
        res = np.linalg.norm(fh[r].ravel() - A @ x) / np.linalg.norm(fh[r])
        assert res <= 1e-9
        assert np.linalg.norm(x - y) / np.linalg.norm(y) <= 1e-7


def _isolated_offsets_case(d, n_el, offsets, seed):
    """Random values on a pattern of isolated offsets (stored by diagonals, runs of length
    one), plain and transposed, against sparse Kronecker products of the plan's time
    factors."""
    import scipy.sparse as sp
    w, a, plan, o = _setup(d, n_el, matvec=None)
    Ns = plan.N_s
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for r in range(Ns):
        for off in offsets(Ns):
            if 0 <= r + off < Ns and (r * 7 + off) % 5 != 1:
                rows.append(r)
                cols.append(r + off)
    rows, cols = np.array(rows), np.array(cols)
    vK, vM = rng.standard_normal(rows.size), rng.standard_normal(rows.size)
    Ks = sp.csr_matrix((vK, (rows, cols)), shape=(Ns, Ns))
    Ms = sp.csr_matrix((vM, (rows, cols)), shape=(Ns, Ns))
    Ks.sort_indices()
    Ms.sort_indices()
    assert np.array_equal(Ks.indptr, Ms.indptr) and np.array_equal(Ks.indices, Ms.indices)
    plan.set_spatial_factors((Ks.indptr.astype(np.int64), Ks.indices.astype(np.int32), Ks.data,
                              Ms.data))
    A = (sp.kron(sp.csr_matrix(a.Wt), Ms) + sp.kron(sp.csr_matrix(a.Mt), Ks)).tocsr()
    x = wl.random_tensor((2,) + w.shape, seed + 16)
    y = plan.matvec_A(_dev(x)).cpu().numpy()
    yt = plan.matvec_A(_dev(x), transpose=True).cpu().numpy()
    for r in range(2):
        ref, reft = A @ x[r].ravel(), A.T @ x[r].ravel()
        assert np.abs(y[r].ravel() - ref).max() <= 1e-13 * np.abs(ref).max()
        assert np.abs(yt[r].ravel() - reft).max() <= 1e-13 * np.abs(reft).max()


def test_isolated_wide_offsets_plain_diagonal_form():
    """Five isolated offsets spanning most of a 12^3 grid: too wide to stage in LDS,
    plain gathers."""
    _isolated_offsets_case(3, 12, lambda Ns: (-(Ns // 2), -7, 0, 5, Ns // 3), 7)


def test_isolated_narrow_offsets_staged_diagonal_form():
    """Five isolated offsets within +-7 on a 22^2 grid: x staged in LDS."""
    _isolated_offsets_case(2, 20, lambda Ns: (-5, -2, 0, 3, 7), 9)
