"""B-splines and 1D Galerkin matrices (oracle; test infrastructure only).

Follows Section 2.1 (open knot vectors, Cox-de Boor recursion with the
convention 0/0 = 0) and Section 3.3 / Section 4 (the 1D factors of the system
matrix).  Integrals are computed with Gauss-Legendre quadrature, p+1 points
per element by default, which is exact for the products of two degree-p
piecewise polynomials that make up every 1D matrix.
"""
from __future__ import annotations

import numpy as np


def open_uniform_knots(n_el: int, p: int, length: float = 1.0) -> np.ndarray:
    """Open knot vector on [0, length]: p+1 repeated end knots, n_el-1 simple
    interior knots (maximal continuity C^{p-1}); Section 2.1 and Section 5.
    Has m + p + 1 entries with m = n_el + p basis functions."""
    interior = np.linspace(0.0, length, n_el + 1)[1:-1]
    return np.concatenate([np.zeros(p + 1), interior, np.full(p + 1, length)])


def _ratio(num, den):
    """num / den with the convention 0/0 = 0 (den == 0 only when num's term vanishes)."""
    den = np.asarray(den, dtype=float)
    safe = np.where(den == 0.0, 1.0, den)
    return np.where(den == 0.0, 0.0, num / safe)


def basis(knots: np.ndarray, p: int, x: np.ndarray) -> np.ndarray:
    """All B-splines of degree p at the points x, by the Cox-de Boor recursion.

    Returns B with B[q, i] = b_{i,p}(x_q), i = 0..m-1 (0-based).  Degree 0
    functions are indicators of half-open spans [xi_i, xi_{i+1}); the point
    x = knots[-1] is assigned to the last non-empty span so that the basis is
    right-continuous inside and left-continuous at the right end.
    """
    x = np.atleast_1d(np.asarray(x, dtype=float))
    xi = np.asarray(knots, dtype=float)
    nk = len(xi)
    B = np.zeros((len(x), nk - 1))
    for i in range(nk - 1):
        B[:, i] = (xi[i] <= x) & (x < xi[i + 1])
    # right end point: the last non-empty span owns it
    last = np.max(np.nonzero(xi[1:] > xi[:-1])[0])
    B[x == xi[-1], :] = 0.0
    B[x == xi[-1], last] = 1.0
    for k in range(1, p + 1):
        Bn = np.zeros((len(x), nk - 1 - k))
        for i in range(nk - 1 - k):
            left = _ratio(x - xi[i], xi[i + k] - xi[i])
            right = _ratio(xi[i + k + 1] - x, xi[i + k + 1] - xi[i + 1])
            Bn[:, i] = left * B[:, i] + right * B[:, i + 1]
        B = Bn
    return B


def basis_derivative(knots: np.ndarray, p: int, x: np.ndarray) -> np.ndarray:
    """First derivatives b'_{i,p}(x) (textbook B-spline derivative formula):
    b'_{i,p} = p/(xi_{i+p}-xi_i) b_{i,p-1} - p/(xi_{i+p+1}-xi_{i+1}) b_{i+1,p-1}, with 0/0 = 0."""
    xi = np.asarray(knots, dtype=float)
    Bm = basis(xi, p - 1, x)  # degree p-1 basis: m+1 functions
    m = len(xi) - p - 1
    D = np.zeros((Bm.shape[0], m))
    for i in range(m):
        a = _ratio(p, xi[i + p] - xi[i])
        b = _ratio(p, xi[i + p + 1] - xi[i + 1])
        D[:, i] = a * Bm[:, i] - b * Bm[:, i + 1]
    return D


def gauss_points(knots: np.ndarray, nq: int):
    """Gauss-Legendre points and weights, nq per non-empty knot span."""
    g, gw = np.polynomial.legendre.leggauss(nq)
    xi = np.unique(knots)
    a, b = xi[:-1], xi[1:]
    x = (0.5 * (b - a)[:, None] * (g[None, :] + 1.0) + a[:, None]).ravel()
    w = (0.5 * (b - a)[:, None] * gw[None, :]).ravel()
    return x, w


def mass(knots, p, weight=None, nq=None):
    """[M]_{ij} = int b_i b_j (times an optional weight function of x); full m x m."""
    x, w = gauss_points(knots, nq or p + 1)
    if weight is not None:
        w = w * weight(x)
    B = basis(knots, p, x)
    return B.T @ (w[:, None] * B)


def stiffness(knots, p, weight=None, nq=None):
    """[K]_{ij} = int b'_i b'_j (times an optional weight); full m x m."""
    x, w = gauss_points(knots, nq or p + 1)
    if weight is not None:
        w = w * weight(x)
    D = basis_derivative(knots, p, x)
    return D.T @ (w[:, None] * D)


def advection(knots, p, nq=None):
    """[W]_{ij} = int b'_j b_i (derivative on the trial index j), eq. time_mat; full m x m."""
    x, w = gauss_points(knots, nq or p + 1)
    B = basis(knots, p, x)
    D = basis_derivative(knots, p, x)
    return B.T @ (w[:, None] * D)


def load(knots, p, func, nq=None):
    """[g]_i = int func(x) b_i(x) dx with nq Gauss points per element (default p+3)."""
    x, w = gauss_points(knots, nq or p + 3)
    B = basis(knots, p, x)
    return B.T @ (w * func(x))


def restrict_space(A):
    """Homogeneous Dirichlet: keep functions 2..m-1 (1-based), Section 2.2."""
    return A[1:-1, 1:-1] if A.ndim == 2 else A[1:-1]


def restrict_time(A):
    """Zero initial datum: keep time functions 2..m (1-based), Section 2.2."""
    return A[1:, 1:] if A.ndim == 2 else A[1:]


def space_matrices(n_el: int, p: int):
    """Parametric 1D spatial factors (K-hat_l, M-hat_l) on (0,1) after the Dirichlet restriction."""
    xi = open_uniform_knots(n_el, p)
    return restrict_space(stiffness(xi, p)), restrict_space(mass(xi, p))


def time_matrices(n_el: int, p: int, T: float = 1.0, mass_weight=None):
    """Time factors (W_t, M_t) on (0,T) after removing the first function.

    W_t does not depend on T (eq. time_mat changes variables to tau = t/T);
    M_t = T * M-hat.  ``mass_weight`` (a function of t) weights M_t only, as
    in Section 4.3.1 for separable time-dependent coefficients."""
    xi = open_uniform_knots(n_el, p, T)
    W = advection(xi, p)
    M = mass(xi, p, weight=mass_weight)
    return restrict_time(W), restrict_time(M)


def time_matrices_full(n_el: int, p: int, T: float = 1.0):
    """Unrestricted time factors (W, M), m x m, used for the initial-datum lifting."""
    xi = open_uniform_knots(n_el, p, T)
    return advection(xi, p), mass(xi, p)
