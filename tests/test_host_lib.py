"""CPU tests of libstig's host side: the library loads and exports every entry
point of include/stig.h, its host numerics (quadrature, B-spline assembly,
eigensolver) agree with the oracle, and argument validation returns the
documented codes.  No GPU call is made."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import bsplines as bs
from oracle import fd

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1909_07309_amd import _lib as L
    return L


def header_symbols():
    src = open(os.path.join(ROOT, "include", "stig.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stig_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = L.lib()
    syms = header_symbols()
    assert "stig_apply_Pinv" in syms and "stig_gmres_solve" in syms
    for s in syms:
        assert hasattr(lib, s), s
        assert s in L.SIGNATURES, f"{s} has no ctypes signature"


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("n_el", [1, 3, 8, 13])
def test_assembly_matches_oracle(p, n_el):
    from paper_1909_07309_amd import api
    for T in (1.0, 2.5):
        xi = bs.open_uniform_knots(n_el, p, T)
        for kind, ref in (("mass", bs.mass(xi, p)), ("stiffness", bs.stiffness(xi, p)),
                          ("advection", bs.advection(xi, p))):
            A = api.assemble_1d(n_el, p, kind, length=T)
            assert np.abs(A - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()), (kind, T)


def test_weighted_assembly_and_load_match_oracle():
    from paper_1909_07309_amd import api
    n_el, p, nq = 6, 3, 6
    x, w = api.quadrature(n_el, nq)
    xo, wo = bs.gauss_points(bs.open_uniform_knots(n_el, p), nq)
    assert np.abs(x - xo).max() < 1e-15 and np.abs(w - wo).max() < 1e-15
    c = 1.0 / (1.0 + 0.3 * np.cos(np.pi * x))
    A = api.assemble_1d(n_el, p, "mass", weight=c, nq=nq)
    ref = bs.mass(bs.open_uniform_knots(n_el, p), p,
                  weight=lambda t: 1.0 / (1.0 + 0.3 * np.cos(np.pi * t)), nq=nq)
    assert np.abs(A - ref).max() < 1e-15
    g = api.load_1d(n_el, p, np.sin(2 * np.pi * x), nq)
    go = bs.load(bs.open_uniform_knots(n_el, p), p, lambda t: np.sin(2 * np.pi * t), nq=nq)
    assert np.abs(g - go).max() < 1e-15


@pytest.mark.parametrize("n_el,p", [(8, 2), (64, 3), (128, 4)])
def test_host_eigensolver_matches_oracle(n_el, p):
    from paper_1909_07309_amd import api
    K, M = bs.space_matrices(n_el, p)
    lam, U = api.sym_eig(K, M)
    lo, _ = fd.space_eig(K, M)
    assert np.abs(lam - lo).max() <= 1e-12 * lo.max()
    n = len(lam)
    assert np.abs(U.T @ M @ U - np.eye(n)).max() < 1e-12
    assert np.abs(U.T @ K @ U - np.diag(lam)).max() < 1e-12 * lam.max()


@pytest.mark.parametrize("n_el,p", [(8, 2), (31, 3), (32, 3), (48, 3), (64, 3), (128, 4)])
def test_split_eigenbasis_is_an_exact_parity_eigenbasis(n_el, p):
    """Persymmetric pencils (uniform knots): the even/odd split basis is M-orthonormal,
    diagonalizes K, has exact parity, and its eigenvalues are the oracle's."""
    from paper_1909_07309_amd import api
    K, M = bs.space_matrices(n_el, p)
    n = K.shape[0]
    J = np.eye(n)[::-1]
    lam, U = api.split_eig(K, M)
    ne = n - n // 2
    assert np.abs(U.T @ M @ U - np.eye(n)).max() < 1e-12
    assert np.abs(U.T @ K @ U - np.diag(lam)).max() < 1e-12 * lam.max()
    assert np.array_equal(J @ U[:, :ne], U[:, :ne])          # even, bit for bit
    assert np.array_equal(J @ U[:, ne:], -U[:, ne:])         # odd
    assert np.all(np.diff(lam[:ne]) > 0) and np.all(np.diff(lam[ne:]) > 0)
    lo, _ = fd.space_eig(K, M)
    assert np.abs(np.sort(lam) - lo).max() <= 1e-12 * lo.max()


def test_split_eigenbasis_rejects_a_non_persymmetric_pencil():
    from paper_1909_07309_amd import api
    from paper_1909_07309_amd._lib import StigError
    K, M = bs.space_matrices(16, 3)
    K = K.copy()
    K[0, 0] *= 1.001
    with pytest.raises(StigError):
        api.split_eig(K, M)


@pytest.mark.parametrize("n_el,p", [(8, 2), (32, 3), (64, 3)])
def test_host_arrowhead_matches_the_oracle_factorization(n_el, p):
    """The real block form of the time pencil's arrowhead factorization: U^T M U = I,
    block structure of D, its 2 x 2 blocks carry the oracle's purely imaginary
    eigenvalues, and U (gamma D + nu lam I)^{-1} U^T solves the shifted system."""
    from paper_1909_07309_amd import api
    from oracle.arrowhead import time_arrowhead as oracle_arrowhead
    Wt, Mt = bs.time_matrices(n_el, p)
    U, D, nz = api.time_arrowhead(Wt, Mt)
    n = Wt.shape[0]
    assert np.abs(U.T @ Mt @ U - np.eye(n)).max() < 1e-12
    assert np.abs(U.T @ Wt @ U - D).max() < 1e-12 * np.abs(D).max()
    m = n - 1
    assert nz == m % 2
    if nz:
        assert abs(D[0, 0]) < 1e-12 * np.abs(D).max()
    blocks = []
    for a in range(nz, m, 2):
        B = D[a:a + 2, a:a + 2]
        assert abs(B[0, 0]) + abs(B[1, 1]) < 1e-11 * np.abs(D).max()
        assert abs(B[0, 1] + B[1, 0]) < 1e-11 * np.abs(D).max()
        blocks.append(abs(B[0, 1]))
    inner = D[:m, :m].copy()
    for a in range(nz, m, 2):
        inner[a:a + 2, a:a + 2] = 0
    assert np.abs(inner).max() < 1e-10 * np.abs(D).max()
    _, _, lam_ring, _, sigma = oracle_arrowhead(Wt, Mt)
    mu = np.sort(np.abs(lam_ring.imag))
    ours = np.sort(np.concatenate([[0.0] * nz, blocks, blocks]))
    assert np.abs(mu - ours).max() < 1e-10 * mu.max()
    assert abs(D[-1, -1] - sigma.real) < 1e-12 * abs(sigma)
    for lam in (3.0, 250.0):
        x = np.random.default_rng(1).standard_normal(n)
        ref = np.linalg.solve(Wt + lam * Mt, x)
        got = U @ np.linalg.solve(D + lam * np.eye(n), U.T @ x)
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_argument_validation_without_gpu():
    L = _lib()
    lib = L.lib()
    h = C.c_void_p()
    n = (C.c_int * 3)(65, 65, 65)
    assert lib.stig_plan_create(C.byref(h), 4, n, 66, 3, 3, None) == -1       # d > 3
    assert lib.stig_plan_create(C.byref(h), 3, n, 66, 9, 3, None) == -1       # degree too high
    assert lib.stig_plan_create(C.byref(h), 3, n, 66, 3, 3, None) == 0
    # apply before setup -> ESTATE; no device memory is touched
    assert lib.stig_apply_Pinv(h, C.c_void_p(8), C.c_void_p(16), 1, 0, 0) == -6
    assert b"setup" in lib.stig_last_error()
    assert lib.stig_gmres_solve(h, None, None, 1, 30, 1e-8, 10, 0, 0, 0, None) == -6
    # kernel options: known values accepted, anything else rejected
    assert lib.stig_set_option(h, 0, 0) == 0 and lib.stig_set_option(h, 0, 1) == 0
    assert lib.stig_set_option(h, 0, 2) == -1
    assert all(lib.stig_set_option(h, 1, v) == 0 for v in (0, 1, 2, 3, 4))
    assert lib.stig_set_option(h, 1, 5) == -1 and lib.stig_set_option(h, 1, -1) == -1
    assert lib.stig_set_option(h, 1, 0) == 0
    assert lib.stig_set_option(h, 2, 0) == 0 and lib.stig_set_option(h, 2, 1) == 0
    assert lib.stig_set_option(h, 2, 5) == -1
    assert lib.stig_set_option(h, 7, 0) == -1
    # workspace: a misaligned pointer is refused; NULL detaches
    assert lib.stig_set_workspace(h, C.c_void_p(8), 1 << 20) == -1
    assert b"aligned" in lib.stig_last_error()
    assert lib.stig_set_workspace(h, None, 0) == 0
    lib.stig_plan_destroy(h)
    assert lib.stig_status_string(-4) == b"breakdown (non-positive pivot)"
    # the arrowhead time kernel: any n_t up to 200 (three-pass form) or n_t = 32 q + 2
    # (fused kernel); n_t = 300 is refused
    n2 = (C.c_int * 2)(130, 130)
    assert lib.stig_plan_create(C.byref(h), 2, n2, 131, 4, 4, None) == 0
    assert lib.stig_set_option(h, 1, 4) == 0
    lib.stig_plan_destroy(h)
    assert lib.stig_plan_create(C.byref(h), 2, n2, 300, 4, 4, None) == 0
    assert lib.stig_set_option(h, 1, 4) == -1
    assert b"n_t" in lib.stig_last_error()
    assert lib.stig_set_option(h, 1, 2) == 0
    lib.stig_plan_destroy(h)


def _round256(b):
    return (b + 255) // 256 * 256


def test_workspace_bytes_cover_each_calls_tensors():
    """stig_workspace_bytes on the 64-element cube (65^3 x 66 unknowns): the FP64 apply keeps
    two intermediates with x/y planes padded to 128 bytes (65^2 = 4225 -> 4240 entries), the
    FP32 / BF16 ones to 4256 / 4288; GMRES(m) adds V (m+1 vectors), Z and A Z (m each) and one
    more vector of N doubles per right-hand side.  Sizes computed here from the tensor shapes."""
    L = _lib()
    lib = L.lib()
    h = C.c_void_p()
    n = (C.c_int * 3)(65, 65, 65)
    assert lib.stig_plan_create(C.byref(h), 3, n, 66, 3, 3, None) == 0
    N = 65 ** 3 * 66
    try:
        ws = lambda m, prec, nrhs: lib.stig_workspace_bytes(h, m, 0, prec, nrhs)
        vec = _round256(N * 8)
        for prec, size, plane in ((0, 8, 4240), (1, 4, 4256), (2, 2, 4288)):
            apply_b = 2 * _round256(65 * plane * 66 * size)
            op = max(apply_b, 2 * vec)  # matvec (fused stencil: a, b) and mass (two buffers)
            assert ws(0, prec, 1) == op, prec
            for m in (1, 30):
                gm = _round256((m + 1) * N * 8) + 2 * _round256(m * N * 8) + vec
                assert ws(m, prec, 1) == op + gm
        # batches: every part scales with the right-hand sides
        assert ws(0, 0, 3) == max(2 * _round256(3 * 65 * 4240 * 66 * 8), 2 * _round256(3 * N * 8))
        assert ws(31, 0, 1) > 0 and ws(33, 0, 1) == 0 and ws(0, 0, 0) == 0 and ws(0, 7, 1) == 0
    finally:
        lib.stig_plan_destroy(h)


@pytest.mark.parametrize("n_el,p", [(4, 2), (5, 3)])
def test_3d_assembly_separation_and_factors_match_oracle(n_el, p):
    """The extruded-annulus setup on the host: 3D CSR stiffness / mass, the 3D
    separation and the weighted 1D factors against the oracle's own code."""
    from oracle.annulus3d import Annulus3DProblem
    from paper_1909_07309_amd.annulus3d import Annulus3DSetup
    w = wl.scaled(wl.WORKLOADS["annulus3d_p2_n32"], n_el, p=p)
    a = Annulus3DSetup(w)
    o = Annulus3DProblem(w)
    rp, col, vK, vM = a.space
    n3 = (n_el + p - 2) ** 3
    assert rp.size == n3 + 1 and np.all(np.diff(rp) > 0)
    import scipy.sparse as sp
    K = sp.csr_matrix((vK, col, rp), shape=(n3, n3)).toarray()
    M = sp.csr_matrix((vM, col, rp), shape=(n3, n3)).toarray()
    assert np.abs(K - o.Ks.toarray()).max() <= 1e-13 * np.abs(K).max()
    assert np.abs(M - o.Ms.toarray()).max() <= 1e-13 * np.abs(M).max()
    assert np.abs(a.dKs - np.diag(K)).max() == 0 and np.abs(a.dMs - np.diag(M)).max() == 0
    for l in range(3):
        assert np.abs(a.Kt[l] - o.Kt[l]).max() <= 1e-13 * np.abs(o.Kt[l]).max()
        assert np.abs(a.Mtl[l] - o.Mtl[l]).max() <= 1e-13 * np.abs(o.Mtl[l]).max()
    assert np.abs(a.Wt - o.Wt).max() < 1e-14 and np.abs(a.Mt - o.Mt).max() < 1e-14
