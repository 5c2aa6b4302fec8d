"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: numbers the
paper prints (tests/golden/cond_numbers.json), closed forms, exact identities,
a library routine (scipy's B-spline design matrix), an independent brute-force
quadrature of the bilinear form, dense direct solves, and observed convergence
rates of a manufactured solution.  The last tests plant plausible mistakes in
the oracle and check that a pin catches each of them.
"""
import json
import os

import numpy as np
import pytest
import scipy.interpolate as si
import scipy.linalg as sla

import workloads as wl
from oracle import arrowhead as ah
from oracle import bsplines as bs
from oracle import dense
from oracle import fd
from oracle.convergence import manufactured_errors
from oracle.problems import CubeProblem

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cond_numbers.json")))


def round2(x):
    """Round to two significant digits, as the paper's tables print."""
    e = np.floor(np.log10(abs(x)))
    return round(x / 10 ** e, 1) * 10 ** e


# ------------------------------------------------------------- B-spline basis

@pytest.mark.parametrize("p,n_el", [(1, 5), (2, 8), (3, 7), (4, 6)])
def test_cox_de_boor_matches_scipy_design_matrix(p, n_el):
    xi = bs.open_uniform_knots(n_el, p)
    x = np.linspace(0.0, 1.0, 97)[:-1] + 0.003
    ours = bs.basis(xi, p, x)
    ref = si.BSpline.design_matrix(x, xi, p).toarray()
    assert np.abs(ours - ref).max() < 1e-14
    # derivative: scipy's BSpline with unit coefficient vectors
    m = len(xi) - p - 1
    dref = np.stack([si.BSpline(xi, np.eye(m)[i], p).derivative()(x) for i in range(m)], axis=1)
    assert np.abs(bs.basis_derivative(xi, p, x) - dref).max() < 1e-12


def test_partition_of_unity_and_open_ends():
    xi = bs.open_uniform_knots(9, 3)
    x = np.linspace(0, 1, 201)
    B = bs.basis(xi, 3, x)
    assert np.abs(B.sum(1) - 1).max() < 1e-14
    # open knot vector: interpolatory at both ends
    assert B[0, 0] == 1.0 and B[-1, -1] == 1.0


def test_linear_splines_closed_forms():
    """p = 1 (hat functions): M = h/6 tridiag(1, 4, 1), K = 1/h tridiag(-1, 2, -1) inside."""
    n = 10
    h = 1.0 / n
    K, M = bs.space_matrices(n, 1)
    Mref = h / 6 * (4 * np.eye(n - 1) + np.eye(n - 1, k=1) + np.eye(n - 1, k=-1))
    Kref = 1 / h * (2 * np.eye(n - 1) - np.eye(n - 1, k=1) - np.eye(n - 1, k=-1))
    assert np.abs(M - Mref).max() < 1e-15 and np.abs(K - Kref).max() < 1e-12


@pytest.mark.parametrize("p", [2, 3, 4])
def test_quadrature_is_exact(p):
    """p+1 Gauss points per element integrate all 1D products exactly: more points change nothing."""
    xi = bs.open_uniform_knots(7, p)
    for f in (bs.mass, bs.stiffness, bs.advection):
        assert np.abs(f(xi, p) - f(xi, p, nq=p + 6)).max() < 1e-13


# ------------------------------------------------ printed condition numbers

@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 7, 8])
def test_table1_kappa_spatial_eigvecs(p):
    t = GOLDEN["table1_space"]
    want = t["value"][t["p"].index(p)]
    for n_el in t["n_el"]:
        K, M = bs.space_matrices(n_el, p)
        lam, U = fd.space_eig(K, M)
        assert round2(np.linalg.cond(U)) == pytest.approx(want)


def test_table3_kappa_stable_time_factor():
    for row in GOLDEN["table3_time_stable"]["rows"]:
        for p, want in zip(row["p"], row["value"]):
            if p > 5 and row["n_el"] > 64:
                continue  # keeps the CPU suite short; same values as n_el = 64
            Wt, Mt = bs.time_matrices(row["n_el"], p)
            Ut = ah.time_arrowhead(Wt, Mt)[0]
            assert round2(np.linalg.cond(Ut)) == pytest.approx(want), (row["n_el"], p)


def test_table2_kappa_unstable_time_eig():
    """kappa2 of the M_t-normalised eigenvectors of (W_t, M_t): pins W_t."""
    for e in GOLDEN["table2_time_unstable"]["entries"]:
        Wt, Mt = bs.time_matrices(e["n_el"], e["p"])
        _, U = sla.eig(Wt, Mt)
        U = U / np.sqrt(np.real(np.einsum("ij,ik,kj->j", U.conj(), Mt, U)))
        assert round2(np.linalg.cond(U)) == pytest.approx(e["value"]), e


# ---------------------------------------------------------- exact identities

@pytest.mark.parametrize("p,n_el", [(2, 8), (3, 16), (4, 5)])
def test_time_matrix_identities(p, n_el):
    """eq. integral_W: W + W^T = b(T) b(T)^T = e_n e_n^T, so W-ring is skew and omega = 1/2."""
    Wt, Mt = bs.time_matrices(n_el, p)
    n = Wt.shape[0]
    E = np.zeros((n, n))
    E[-1, -1] = 1.0
    assert np.abs(Wt + Wt.T - E).max() < 1e-14
    assert Wt[-1, -1] == pytest.approx(0.5, abs=1e-14)
    Wf, Mf = bs.time_matrices_full(n_el, p, T=2.5)
    assert np.abs(Wf.sum(axis=1)).max() < 1e-14          # derivative of the constant 1
    assert Mf.sum() == pytest.approx(2.5, rel=1e-14)      # int_0^T 1 dt
    assert np.abs(bs.stiffness(bs.open_uniform_knots(n_el, p), p).sum(1)).max() < 1e-11
    # M_t = T * M-hat, W_t independent of T (Section 4)
    W2, M2 = bs.time_matrices(n_el, p, T=3.0)
    assert np.abs(W2 - Wt).max() < 1e-13 and np.abs(M2 - 3.0 * Mt).max() < 1e-13


def test_spatial_eigendecomposition_and_laplacian_limit():
    K, M = bs.space_matrices(64, 3)
    lam, U = fd.space_eig(K, M)
    assert np.abs(U.T @ M @ U - np.eye(len(lam))).max() < 1e-13
    assert np.abs(U.T @ K @ U - np.diag(lam)).max() < 1e-9 * lam.max()
    # smallest Dirichlet-Laplacian eigenvalue on (0,1) is pi^2
    assert lam[0] == pytest.approx(np.pi ** 2, rel=1e-10)
    assert np.all(np.diff(lam) > 0)


# ------------------------------------------------ Kronecker form of the system

@pytest.mark.parametrize("d,n_el,p,T,gamma,nu", [(1, 5, 3, 2.0, 0.7, 1.3), (2, 3, 2, 1.0, 1.0, 1.0),
                                                 (2, 3, 3, 0.5, 2.0, 0.3), (3, 2, 2, 1.0, 1.0, 1.0)])
def test_kronecker_system_matches_brute_force_quadrature(d, n_el, p, T, gamma, nu):
    A = dense.unit_cube_system(d, n_el, p, T, gamma, nu)
    Ab = dense.brute_force_system(d, n_el, p, T, gamma, nu)
    assert np.abs(A - Ab).max() < 1e-13 * max(1.0, np.abs(A).max())


def test_kron_matvec_and_mass_apply_match_dense():
    w = wl.scaled(wl.WORKLOADS["cube_p3_n64"], 3)
    pr = CubeProblem(w)
    A = dense.kron_system(pr.Wt, pr.Mt, pr.K1d, pr.M1d, 1.3, 0.6)
    x = wl.random_tensor(w.shape, 5)
    y = fd.kron_matvec(x, pr.Wt, pr.Mt, pr.K1d, pr.M1d, 1.3, 0.6)
    assert np.abs(y.ravel() - A @ x.ravel()).max() < 1e-14 * np.abs(A).max() * 50
    yt = fd.kron_matvec(x, pr.Wt, pr.Mt, pr.K1d, pr.M1d, 1.3, 0.6, transpose=True)
    assert np.abs(yt.ravel() - A.T @ x.ravel()).max() < 1e-14 * np.abs(A).max() * 50
    Ms = dense.kron_all([pr.Mt] + pr.M1d[::-1])
    assert np.abs(fd.mass_apply(x, pr.Mt, pr.M1d).ravel() - Ms @ x.ravel()).max() < 1e-16 * 50


# -------------------------------------------------- A-hat^{-1} by FD and arrowhead

@pytest.mark.parametrize("name,n_el", [("square_p2_n8", 8), ("cube_p3_n64", 3), ("cube_p3_n64", 4)])
def test_fd_apply_matches_dense_solve(name, n_el):
    w = wl.scaled(wl.WORKLOADS[name], n_el)
    pr = CubeProblem(w)
    for gamma, nu in [(1.0, 1.0), (0.3, 2.5)]:
        A = dense.kron_system(pr.Wt, pr.Mt, pr.K1d, pr.M1d, gamma, nu)
        r = wl.random_tensor(w.shape, 11)
        P = fd.FDPreconditioner(pr.K1d, pr.M1d, pr.Wt, pr.Mt, gamma, nu)
        s = P.apply(r)
        ref = dense.solve(A, r.ravel())
        assert np.abs(s.ravel() - ref).max() <= 1e-12 * np.abs(ref).max()
        st = P.apply(r, transpose=True)
        reft = dense.solve(A.T, r.ravel())
        assert np.abs(st.ravel() - reft).max() <= 1e-12 * np.abs(reft).max()


def test_arrowhead_factorization_properties():
    Wt, Mt = bs.time_matrices(16, 3)
    U, Delta, lam_ring, g, sigma = ah.time_arrowhead(Wt, Mt)
    n = Wt.shape[0]
    assert np.abs(U.conj().T @ Mt @ U - np.eye(n)).max() < 1e-12        # eq. Mt-orthogonality
    off = Delta.copy()
    off[np.arange(n - 1), np.arange(n - 1)] = 0
    off[-1, :] = 0
    off[:, -1] = 0
    assert np.abs(off).max() < 1e-12                                     # arrowhead
    assert np.abs(np.diag(Delta)[:-1] - lam_ring).max() < 1e-11
    assert np.abs(lam_ring.real).max() < 1e-12                            # purely imaginary
    assert np.abs(Delta[:-1, -1] - g).max() < 1e-12                       # g of eq. time_eig_2
    assert np.abs(Delta[-1, :-1] + g.conj()).max() < 1e-12                # lower arm is -g^*
    rho = U[-1, -1].real
    assert sigma == pytest.approx(rho ** 2 / 2, rel=1e-12)                # from eq. integral_W


@pytest.mark.parametrize("name,n_el", [("square_p2_n8", 8), ("cube_p3_n64", 3)])
def test_arrowhead_apply_matches_banded_fd_and_dense(name, n_el):
    w = wl.scaled(wl.WORKLOADS[name], n_el)
    pr = CubeProblem(w)
    r = wl.random_tensor(w.shape, 3)
    s_fd = fd.FDPreconditioner(pr.K1d, pr.M1d, pr.Wt, pr.Mt, 0.8, 1.7).apply(r)
    s_ah = ah.ArrowheadPreconditioner(pr.K1d, pr.M1d, pr.Wt, pr.Mt, 0.8, 1.7).apply(r)
    A = dense.kron_system(pr.Wt, pr.Mt, pr.K1d, pr.M1d, 0.8, 1.7)
    ref = dense.solve(A, r.ravel())
    assert np.abs(s_ah.ravel() - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(s_fd - s_ah).max() <= 1e-12 * np.abs(ref).max()


def test_banded_solve_rejects_zero_pivot():
    Wt, Mt = bs.time_matrices(4, 2)
    with pytest.raises(ZeroDivisionError):
        fd.banded_shifted_solve(Wt, Mt, np.ones(3), np.ones((Wt.shape[0], 3)), 0.0, 0.0)


# ------------------------------------------------------ discretisation error

@pytest.mark.parametrize("d,p,n_el", [(2, 1, 8), (2, 2, 8), (2, 3, 8),
                                       (3, 1, 6), (3, 2, 6), (3, 3, 6)])
def test_manufactured_solution_rates(d, p, n_el):
    """Section 5.1 and eq. a-riori-error-bound: L2 order p+1, X-type norm order p, on the
    unit square (d = 2) and cube (d = 3), from n_el to 2 n_el elements."""
    e1 = manufactured_errors(d, n_el, p)
    e2 = manufactured_errors(d, 2 * n_el, p)
    r_l2 = np.log2(e1[0] / e2[0])
    r_x = np.log2(e1[1] / e2[1])
    assert abs(r_l2 - (p + 1)) < 0.15, r_l2
    assert abs(r_x - p) < 0.15, r_x


def test_annulus_exact_solution_is_admissible_and_its_derivatives_are_right():
    """The annulus manufactured solution vanishes on the spatial boundary, and its hand-written
    gradient and Laplacian (and the conductivity's gradient) agree with central differences."""
    from oracle.convergence import annulus_conductivity_gradient, annulus_solution
    th = np.linspace(0, np.pi / 2, 7)
    for r in (1.0, 2.0):
        assert np.abs(annulus_solution(r * np.cos(th), r * np.sin(th))[0]).max() < 1e-14
    rr = np.linspace(1, 2, 7)
    assert np.abs(annulus_solution(0 * rr, rr)[0]).max() < 1e-14
    assert np.abs(annulus_solution(rr, 0 * rr)[0]).max() < 1e-14
    rng = np.random.default_rng(4)
    x, y = rng.uniform(0.3, 1.3, 20), rng.uniform(0.3, 1.3, 20)
    h = 1e-5
    u = lambda a, b: annulus_solution(a, b)[0]
    _, ux, uy, lap = annulus_solution(x, y)
    assert np.allclose(ux, (u(x + h, y) - u(x - h, y)) / (2 * h), rtol=0, atol=1e-8)
    assert np.allclose(uy, (u(x, y + h) - u(x, y - h)) / (2 * h), rtol=0, atol=1e-8)
    h2 = 1e-4
    lap_fd = (u(x + h2, y) + u(x - h2, y) + u(x, y + h2) + u(x, y - h2) - 4 * u(x, y)) / h2 ** 2
    assert np.allclose(lap, lap_fd, rtol=0, atol=1e-5)
    kx, ky = annulus_conductivity_gradient(x, y)
    k = wl.annulus_conductivity
    assert np.allclose(kx, (k(x + h, y) - k(x - h, y)) / (2 * h), rtol=0, atol=1e-8)
    assert np.allclose(ky, (k(x, y + h) - k(x, y - h)) / (2 * h), rtol=0, atol=1e-8)


def _annulus_p(n_el, p):
    from oracle.annulus import AnnulusProblem
    return AnnulusProblem(wl.scaled(wl.WORKLOADS["annulus_p4_n128"], n_el, p=p))


@pytest.mark.parametrize("p", [2, 3, 4])
def test_annulus_manufactured_solution_rates(p):
    """The annulus workload's own system (variable conductivity, 1/c-weighted M_t, polar
    map) solved for the 2D analogue of the paper's Section 5.1 solution: L2 order p+1 and
    X-type order p, 16 -> 32 elements.  This pins the variable-coefficient assembly."""
    from oracle.convergence import annulus_manufactured_errors
    e1 = annulus_manufactured_errors(_annulus_p(16, p))
    e2 = annulus_manufactured_errors(_annulus_p(32, p))
    r_l2, r_x = np.log2(e1[0] / e2[0]), np.log2(e1[1] / e2[1])
    assert abs(r_l2 - (p + 1)) < 0.15, r_l2
    assert abs(r_x - p) < 0.15, r_x


def _plant_annulus(kind, n_el, p, monkeypatch):
    import oracle.annulus as oa
    if kind == "kappa at parametric points":
        monkeypatch.setattr(oa, "physical_point", lambda e1, e2: (e1, e2))
    elif kind == "kappa at swapped parametric coordinates":
        orig = oa.physical_point
        monkeypatch.setattr(oa, "physical_point", lambda e1, e2: orig(e2, e1))
    elif kind == "radial and angular metric swapped":
        orig_c = oa.polar_coefficients
        monkeypatch.setattr(oa, "polar_coefficients",
                            lambda e1, e2: (lambda c: (c[1], c[0], c[2]))(orig_c(e1, e2)))
    o = _annulus_p(n_el, p)
    monkeypatch.undo()
    if kind == "M_t without the 1/c weight":
        o.Mt = bs.time_matrices(n_el, p)[1]
    elif kind == "M_t weighted by c":
        o.Mt = bs.time_matrices(n_el, p, mass_weight=wl.annulus_heat_capacity)[1]
    elif kind == "W_t weighted by c":
        xt = bs.open_uniform_knots(n_el, p)
        x, w = bs.gauss_points(xt, p + 3)
        B, D = bs.basis(xt, p, x), bs.basis_derivative(xt, p, x)
        o.Wt = bs.restrict_time(B.T @ ((w * wl.annulus_heat_capacity(x))[:, None] * D))
    return o


@pytest.mark.parametrize("kind", ["kappa at parametric points",
                                  "kappa at swapped parametric coordinates",
                                  "radial and angular metric swapped",
                                  "M_t without the 1/c weight", "M_t weighted by c",
                                  "W_t weighted by c"])
def test_pins_catch_annulus_coefficient_mistakes(kind, monkeypatch):
    """Each plausible misreading of the variable-coefficient assembly makes the discrete
    solution converge to the wrong limit: the L2 error stops falling."""
    from oracle.convergence import annulus_manufactured_errors
    e1 = annulus_manufactured_errors(_plant_annulus(kind, 8, 3, monkeypatch))
    e2 = annulus_manufactured_errors(_plant_annulus(kind, 16, 3, monkeypatch))
    assert np.log2(e1[0] / e2[0]) < 1.0 and e2[0] > 1e-3, (kind, e1, e2)


# ----------------------------------------------------------- planted mistakes

def test_pins_catch_transposed_time_derivative(monkeypatch):
    """If W were assembled with the derivative on the test index, the brute-force pin fails."""
    orig = bs.advection
    monkeypatch.setattr(bs, "advection", lambda xi, p, nq=None: orig(xi, p, nq).T)
    A = dense.unit_cube_system(2, 3, 2)
    monkeypatch.setattr(bs, "advection", orig)
    Ab = dense.brute_force_system(2, 3, 2)
    assert np.abs(A - Ab).max() > 1e-3


def test_pins_catch_untransposed_forward_transform(monkeypatch):
    """Step 2 with U_l instead of U_l^T breaks agreement with the dense solve."""
    w = wl.scaled(wl.WORKLOADS["cube_p3_n64"], 3)
    pr = CubeProblem(w)
    P = fd.FDPreconditioner(pr.K1d, pr.M1d, pr.Wt, pr.Mt)
    P.U = [U.T for U in P.U]       # apply() transposes them back the wrong way round
    r = wl.random_tensor(w.shape, 1)
    A = dense.kron_system(pr.Wt, pr.Mt, pr.K1d, pr.M1d)
    ref = dense.solve(A, r.ravel())
    assert np.abs(P.apply(r).ravel() - ref).max() > 1e-3 * np.abs(ref).max()


def test_pins_catch_dropped_spatial_stiffness_term():
    """Dropping one direction's stiffness term from K_s breaks the brute-force pin."""
    K, M = bs.space_matrices(3, 2)
    Wt, Mt = bs.time_matrices(3, 2)
    Ms = np.kron(M, M)
    Ks_wrong = np.kron(M, K)          # missing K (x) M
    A_wrong = np.kron(Wt, Ms) + np.kron(Mt, Ks_wrong)
    assert np.abs(A_wrong - dense.brute_force_system(2, 3, 2)).max() > 1e-3


# ------------------------------------------------------------------- adjoint

def test_lifting_block_matches_brute_force_quadrature():
    """A_{I,0} (the first time function's block column) from the unrestricted bilinear form."""
    from oracle.adjoint import DenseAdjoint
    d, n_el, p = 2, 3, 2
    adj = DenseAdjoint(d, n_el, p, gamma=0.7, nu=1.3)
    full = dense.brute_force_system(d, n_el, p, gamma=0.7, nu=1.3, full_time=True)
    Ns = adj.Ms.shape[0]
    assert np.abs(full[Ns:, :Ns] - adj.AI0).max() < 1e-13
    assert np.abs(full[Ns:, Ns:] - adj.A).max() < 1e-13


def test_adjoint_gradients_match_central_differences():
    """L is quadratic in (f, c0): central differences equal the directional derivative."""
    from oracle.adjoint import DenseAdjoint
    adj = DenseAdjoint(3, 2, 2)
    N, Ns = adj.A.shape[0], adj.Ms.shape[0]
    rng = np.random.default_rng(3)
    f, c0, tgt = rng.standard_normal(N), rng.standard_normal(Ns), rng.standard_normal(N)
    gf, gc = adj.gradients(f, c0, tgt)
    for _ in range(4):
        df, dc = rng.standard_normal(N), rng.standard_normal(Ns)
        h = 1e-3
        fd = (adj.loss(f + h * df, c0 + h * dc, tgt) - adj.loss(f - h * df, c0 - h * dc, tgt)) / (2 * h)
        an = gf @ df + gc @ dc
        assert abs(fd - an) <= 1e-9 * abs(an)


def test_pins_catch_wrong_lifting_sign():
    from oracle.adjoint import DenseAdjoint
    adj = DenseAdjoint(2, 3, 2)
    N, Ns = adj.A.shape[0], adj.Ms.shape[0]
    rng = np.random.default_rng(5)
    f, c0, tgt = rng.standard_normal(N), rng.standard_normal(Ns), rng.standard_normal(N)
    _, gc = adj.gradients(f, c0, tgt)
    dc = rng.standard_normal(Ns)
    h = 1e-3
    fd = (adj.loss(f, c0 + h * dc, tgt) - adj.loss(f, c0 - h * dc, tgt)) / (2 * h)
    assert abs(fd - (-gc) @ dc) > 1e-3 * abs(fd)      # the flipped sign is caught


# ------------------------------------------------------------------- annulus

def _annulus(n_el):
    from oracle.annulus import AnnulusProblem
    return AnnulusProblem(wl.scaled(wl.WORKLOADS["annulus_p4_n128"], n_el))


def test_annulus_mass_is_radially_weighted_kronecker_product():
    """M_s = int B_i B_j |det J| with |det J| = pi r / 2 depending on eta_1 only."""
    o = _annulus(6)
    xi = bs.open_uniform_knots(6, 4)
    Mr = bs.restrict_space(bs.mass(xi, 4, weight=lambda x: np.pi * (1 + x) / 2, nq=7))
    Mth = bs.restrict_space(bs.mass(xi, 4, nq=7))
    assert np.abs(o.Ms.toarray() - np.kron(Mth, Mr)).max() < 1e-15


def test_annulus_stiffness_separates_for_constant_conductivity(monkeypatch):
    """With kappa = 1 the polar-map stiffness is Mth (x) K_r[pi r/2] + K_th (x) M_r[2/(pi r)]."""
    monkeypatch.setattr(wl, "annulus_conductivity", lambda x, y: np.ones_like(x))
    o = _annulus(5)
    xi = bs.open_uniform_knots(5, 4)
    Kr = bs.restrict_space(bs.stiffness(xi, 4, weight=lambda x: np.pi * (1 + x) / 2, nq=7))
    Mr = bs.restrict_space(bs.mass(xi, 4, weight=lambda x: 2 / (np.pi * (1 + x)), nq=7))
    Kth = bs.restrict_space(bs.stiffness(xi, 4, nq=7))
    Mth = bs.restrict_space(bs.mass(xi, 4, nq=7))
    ref = np.kron(Mth, Kr) + np.kron(Kth, Mr)
    assert np.abs(o.Ks.toarray() - ref).max() < 1e-12 * np.abs(ref).max()
    # C33 and C11 are separable under the model of eq. separation, so those fits are exact.
    # (C22 = 2/(pi r) is not: the model pairs Phi_2 with the mass factor phi_1 ~ r, and
    # the diagonal scaling D of eq. prec_geo absorbs the mismatch.)
    n = 5
    mids = (np.arange(n) + 0.5) / n
    E1, E2 = np.meshgrid(mids, mids, indexing="xy")
    C33 = np.pi * (1 + E1) / 2
    phi1, phi2 = o.phi
    Phi1, Phi2 = o.Phi
    assert np.allclose(np.outer(phi2, phi1), C33, rtol=1e-13)
    assert np.allclose(np.outer(phi2, Phi1), np.pi * (1 + E1) / 2, rtol=1e-13)


def _sep_kappa_2d(x, y):
    """kappa = a(r) b(theta), separable in the polar coordinates (not in x and y)."""
    r, th = np.hypot(x, y), np.arctan2(y, x)
    return (1.0 + 0.3 * r * r) * (2.0 + np.sin(3.0 * th))


def test_annulus_stiffness_is_exact_for_polar_separable_conductivity(monkeypatch):
    """For kappa = a(r) b(theta) the polar-map stiffness is the Kronecker sum
    M_th[b] (x) K_r[a pi r/2] + K_th[b] (x) M_r[a 2/(pi r)] of weighted 1D matrices, assembled
    here by the 1D routines (same Gauss rule), independently of the 2D element assembly."""
    monkeypatch.setattr(wl, "annulus_conductivity", _sep_kappa_2d)
    n_el, p = 5, 4
    o = _annulus(n_el)
    xi = bs.open_uniform_knots(n_el, p)
    a = lambda e1: 1.0 + 0.3 * (1 + e1) ** 2
    b = lambda e2: 2.0 + np.sin(1.5 * np.pi * e2)
    Kr = bs.restrict_space(bs.stiffness(xi, p, weight=lambda x: a(x) * np.pi * (1 + x) / 2, nq=p + 3))
    Mr = bs.restrict_space(bs.mass(xi, p, weight=lambda x: a(x) * 2 / (np.pi * (1 + x)), nq=p + 3))
    Kth = bs.restrict_space(bs.stiffness(xi, p, weight=b, nq=p + 3))
    Mth = bs.restrict_space(bs.mass(xi, p, weight=b, nq=p + 3))
    ref = np.kron(Mth, Kr) + np.kron(Kth, Mr)
    assert np.abs(o.Ks.toarray() - ref).max() < 1e-13 * np.abs(ref).max()
    # the same conductivity sampled at swapped parametric coordinates is caught
    import oracle.annulus as oa
    orig = oa.physical_point
    monkeypatch.setattr(oa, "physical_point", lambda e1, e2: orig(e2, e1))
    bad = _annulus(n_el)
    assert np.abs(bad.Ks.toarray() - ref).max() > 1e-2 * np.abs(ref).max()


def test_annulus_geometry_preconditioner_matches_dense():
    """A-hat^G = D^{1/2} A-tilde D^{1/2} (eq. prec_geo): FD apply against a dense solve,
    and diag(A-hat^G) = diag(A)."""
    o = _annulus(5)
    Kt, Mtl = o.Kt, o.Mtl
    At = (np.kron(o.Wt, np.kron(Mtl[1], Mtl[0]))
          + np.kron(o.Mt, np.kron(Mtl[1], Kt[0]) + np.kron(Kt[1], Mtl[0])))
    D = o.D().ravel()
    AG = np.sqrt(D)[:, None] * At * np.sqrt(D)[None, :]
    A = o.dense_A()
    assert np.abs(np.diag(AG) - np.diag(A)).max() < 1e-13 * np.abs(np.diag(A)).max()
    r = wl.random_tensor(o.w.shape, 2)
    s = o.preconditioner().apply(r)
    ref = np.linalg.solve(AG, r.ravel())
    assert np.abs(s.ravel() - ref).max() <= 1e-12 * np.abs(ref).max()


# ------------------------------------------------------- extruded annulus (3D)

def _annulus3d(n_el, p=2):
    from oracle.annulus3d import Annulus3DProblem
    return Annulus3DProblem(wl.scaled(wl.WORKLOADS["annulus3d_p2_n32"], n_el, p=p))


def test_annulus3d_mass_is_radially_weighted_kronecker_product():
    """M_s = int B_i B_j |det J| with |det J| = pi r / 2 depending on eta_1 only:
    M-hat_3 (x) M-hat_2 (x) M_r[pi r / 2]."""
    o = _annulus3d(4, p=3)
    xi = bs.open_uniform_knots(4, 3)
    Mr = bs.restrict_space(bs.mass(xi, 3, weight=lambda x: np.pi * (1 + x) / 2, nq=6))
    Mh = bs.restrict_space(bs.mass(xi, 3, nq=6))
    assert np.abs(o.Ms.toarray() - np.kron(Mh, np.kron(Mh, Mr))).max() < 1e-15


def test_annulus3d_stiffness_separates_for_constant_conductivity(monkeypatch):
    """With kappa = 1 the extruded polar-map stiffness is
    M3 (x) M2 (x) K_r[pi r/2] + M3 (x) K2 (x) M_r[2/(pi r)] + K3 (x) M2 (x) M_r[pi r/2]
    (direction 1 radial, 2 angular, 3 along the extrusion)."""
    monkeypatch.setattr(wl, "annulus3d_conductivity", lambda x, y, z: np.ones_like(x))
    o = _annulus3d(4, p=2)
    xi = bs.open_uniform_knots(4, 2)
    Kr = bs.restrict_space(bs.stiffness(xi, 2, weight=lambda x: np.pi * (1 + x) / 2, nq=5))
    Mr1 = bs.restrict_space(bs.mass(xi, 2, weight=lambda x: 2 / (np.pi * (1 + x)), nq=5))
    Mr2 = bs.restrict_space(bs.mass(xi, 2, weight=lambda x: np.pi * (1 + x) / 2, nq=5))
    Kh = bs.restrict_space(bs.stiffness(xi, 2, nq=5))
    Mh = bs.restrict_space(bs.mass(xi, 2, nq=5))
    ref = (np.kron(Mh, np.kron(Mh, Kr)) + np.kron(Mh, np.kron(Kh, Mr1))
           + np.kron(Kh, np.kron(Mh, Mr2)))
    assert np.abs(o.Ks.toarray() - ref).max() < 1e-12 * np.abs(ref).max()
    # C00, C11 and C33 depend on eta_1 only: their separated fits are exact
    mids = (np.arange(4) + 0.5) / 4
    E3, E2, E1 = np.meshgrid(mids, mids, mids, indexing="ij")
    c = np.pi * (1 + E1) / 2
    phi1, phi2, phi3 = o.phi
    Phi1, Phi2, Phi3 = o.Phi
    prod = phi3[:, None, None] * phi2[None, :, None] * phi1[None, None, :]
    assert np.allclose(prod, c, rtol=1e-13)
    assert np.allclose(phi3[:, None, None] * phi2[None, :, None] * Phi1[None, None, :], c, rtol=1e-13)
    assert np.allclose(Phi3[:, None, None] * phi2[None, :, None] * phi1[None, None, :], c, rtol=1e-13)


def test_annulus3d_stiffness_is_exact_for_separable_conductivity(monkeypatch):
    """For kappa = a(r) b(theta) e(z) the extruded polar-map stiffness is the sum of three
    Kronecker products of weighted 1D matrices (same Gauss rule), and the 3D time mass
    matrix is the 1/c-weighted one of the 2D workload (pinned by the annulus rates)."""
    a = lambda e1: 1.0 + 0.3 * (1 + e1) ** 2
    b = lambda e2: 2.0 + np.sin(1.5 * np.pi * e2)
    e = lambda e3: 1.5 + np.cos(2.0 * e3)

    def kap(x, y, z):
        r, th = np.hypot(x, y), np.arctan2(y, x)
        return (1.0 + 0.3 * r * r) * (2.0 + np.sin(3.0 * th)) * (1.5 + np.cos(2.0 * z))
    monkeypatch.setattr(wl, "annulus3d_conductivity", kap)
    n_el, p = 4, 2
    o = _annulus3d(n_el, p=p)
    xi = bs.open_uniform_knots(n_el, p)
    nq = p + 3
    w1 = lambda f: bs.restrict_space(bs.mass(xi, p, weight=f, nq=nq))
    k1 = lambda f: bs.restrict_space(bs.stiffness(xi, p, weight=f, nq=nq))
    pr = lambda x: np.pi * (1 + x) / 2
    ref = (np.kron(w1(e), np.kron(w1(b), k1(lambda x: a(x) * pr(x))))
           + np.kron(w1(e), np.kron(k1(b), w1(lambda x: a(x) / pr(x))))
           + np.kron(k1(e), np.kron(w1(b), w1(lambda x: a(x) * pr(x)))))
    assert np.abs(o.Ks.toarray() - ref).max() < 1e-13 * np.abs(ref).max()
    o2 = _annulus_p(n_el, p)
    assert np.abs(o.Mt - o2.Mt).max() == 0.0


def test_annulus3d_separation_is_exact_for_separable_samples(monkeypatch):
    """The 3D fit of eq. separation reproduces samples that have the model's form:
    C00 = b1(e1) b2(e2) b3(e3) and C_ll = a_l(e_l) prod_{m != l} b_m(e_m)."""
    from oracle import annulus3d as a3
    b1 = lambda x: 1 + x
    b2 = lambda y: 1 + y ** 2
    b3 = lambda z: 3 - z
    coeffs = lambda e1, e2, e3: ((0.5 + e1) * b2(e2) * b3(e3), b1(e1) * (2 + e2) * b3(e3),
                                 b1(e1) * b2(e2) * (1 + e3), b1(e1) * b2(e2) * b3(e3))
    monkeypatch.setattr(a3, "extruded_polar_coefficients", coeffs)
    monkeypatch.setattr(wl, "annulus3d_conductivity", lambda x, y, z: np.ones_like(x))
    o = _annulus3d(5, p=2)
    mids = (np.arange(5) + 0.5) / 5
    E3, E2, E1 = np.meshgrid(mids, mids, mids, indexing="ij")
    C11, C22, C33, C00 = coeffs(E1, E2, E3)
    phi1, phi2, phi3 = o.phi
    Phi1, Phi2, Phi3 = o.Phi
    g = lambda f3, f2, f1: f3[:, None, None] * f2[None, :, None] * f1[None, None, :]
    assert np.allclose(g(phi3, phi2, phi1), C00, rtol=1e-13)
    assert np.allclose(g(phi3, phi2, Phi1), C11, rtol=1e-13)
    assert np.allclose(g(phi3, Phi2, phi1), C22, rtol=1e-13)
    assert np.allclose(g(Phi3, phi2, phi1), C33, rtol=1e-13)
    # and a dropped direction is caught: a fit without phi3 misses C00
    assert not np.allclose(g(np.ones(5), phi2, phi1), C00, rtol=1e-3)


def test_annulus3d_geometry_preconditioner_matches_dense():
    """A-hat^G = D^{1/2} A-tilde D^{1/2} in 3D: FD apply against a dense solve, and
    diag(A-hat^G) = diag(A)."""
    o = _annulus3d(3, p=2)
    Kt, Mtl = o.Kt, o.Mtl
    k3 = lambda a, b, c: np.kron(a, np.kron(b, c))
    Ms = k3(Mtl[2], Mtl[1], Mtl[0])
    Ks = k3(Mtl[2], Mtl[1], Kt[0]) + k3(Mtl[2], Kt[1], Mtl[0]) + k3(Kt[2], Mtl[1], Mtl[0])
    At = np.kron(o.Wt, Ms) + np.kron(o.Mt, Ks)
    D = o.D().ravel()
    AG = np.sqrt(D)[:, None] * At * np.sqrt(D)[None, :]
    A = o.dense_A()
    assert np.abs(np.diag(AG) - np.diag(A)).max() < 1e-13 * np.abs(np.diag(A)).max()
    r = wl.random_tensor(o.w.shape, 2)
    s = o.preconditioner().apply(r)
    ref = np.linalg.solve(AG, r.ravel())
    assert np.abs(s.ravel() - ref).max() <= 1e-12 * np.abs(ref).max()
