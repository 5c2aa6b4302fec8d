"""Dense assembly and direct solves on tiny grids (oracle; test infrastructure only).

* ``kron_system``     - A = gamma W_t (x) M_s + nu M_t (x) K_s, eq. syst_mat, with
                        K_s, M_s the Kronecker sums/products of eq. space_univ_par_mat
                        (identity geometry, so A = A-hat of eq. prec_definition).
* ``brute_force_system`` - the same matrix from the bilinear form of Section 3.1,
                        int int (gamma d_t B_j B_i + nu grad B_j . grad B_i), by tensor
                        Gauss quadrature over every space-time element, never using
                        the Kronecker structure.  It pins eq. syst_mat itself.
* ``solve``           - LU with partial pivoting (numpy), for A^{-1} f, A-hat^{-1} r,
                        and A^{-T} for the adjoint.

Vectors follow the colexicographic ``vec`` of Section 2.3: a C-order array
[t][x_d]..[x_1] flattened, which matches np.kron(J_t, J_d, ..., J_1).
"""
from __future__ import annotations

from functools import reduce

import numpy as np

from . import bsplines as bs


def kron_all(mats):
    """mats = [J_{d+1}, ..., J_1] -> J_{d+1} (x) ... (x) J_1."""
    return reduce(np.kron, mats)


def spatial_kron(K1d, M1d):
    """K_s and M_s from 1D factors given in direction order l = 1..d (eq. space_univ_par_mat).

    M_s = M_d (x) ... (x) M_1;  K_s = sum_l M_d (x) .. (x) K_l (x) .. (x) M_1."""
    d = len(K1d)
    Ms = kron_all([M1d[l] for l in reversed(range(d))])
    Ks = 0
    for l in range(d):
        Ks = Ks + kron_all([K1d[j] if j == l else M1d[j] for j in reversed(range(d))])
    return Ks, Ms


def kron_system(Wt, Mt, K1d, M1d, gamma=1.0, nu=1.0):
    """A = gamma W_t (x) M_s + nu M_t (x) K_s (eq. syst_mat / prec_definition)."""
    Ks, Ms = spatial_kron(K1d, M1d)
    return gamma * np.kron(Wt, Ms) + nu * np.kron(Mt, Ks)


def unit_cube_system(d, n_el, p, T=1.0, gamma=1.0, nu=1.0):
    """Dense A on the unit cube (d spatial dims) with constant coefficients."""
    K, M = bs.space_matrices(n_el, p)
    Wt, Mt = bs.time_matrices(n_el, p, T)
    return kron_system(Wt, Mt, [K] * d, [M] * d, gamma, nu)


def brute_force_system(d, n_el, p, T=1.0, gamma=1.0, nu=1.0, nq=None, full_time=False):
    """A_{ij} = int_0^T int_Omega (gamma d_t B_j B_i + nu grad B_j . grad B_i) on Omega = (0,1)^d.

    B_i(x, t) is the product of the restricted 1D B-splines (eq. tens-prod-space-parametric,
    Section 2.2).  Every multivariate basis function and its partial derivatives are
    evaluated at every point of a tensor Gauss grid over the whole space-time domain;
    the integral is one weighted sum over those points.  No Kronecker identity is used.
    """
    nq = nq or p + 1
    xs = bs.open_uniform_knots(n_el, p)
    xt = bs.open_uniform_knots(n_el, p, T)
    qs, ws = bs.gauss_points(xs, nq)
    qt, wt = bs.gauss_points(xt, nq)
    # [q, i]: keep spatial functions 2..m-1 and time functions 2..m (Section 2.2)
    Bs = bs.basis(xs, p, qs)[:, 1:-1]
    Ds = bs.basis_derivative(xs, p, qs)[:, 1:-1]
    # full_time=True keeps the first time function too (its block column is the
    # initial-datum lifting operator)
    t0 = 0 if full_time else 1
    Bt = bs.basis(xt, p, qt)[:, t0:]
    Dt = bs.basis_derivative(xt, p, qt)[:, t0:]

    # Multivariate basis on the full tensor grid: for each factor (time, x_d, ..., x_1)
    # take either the value or the derivative of the 1D function, multiply them
    # pointwise (outer product over the grid), and flatten to [point, function].
    def tensor_eval(factors):
        out = factors[0]
        for f in factors[1:]:
            # out[q.., i..] (x) f[q, i] -> out[q.., q, i.., i]
            nqo, nio = out.shape
            out = (out[:, None, :, None] * f[None, :, None, :]).reshape(
                nqo * f.shape[0], nio * f.shape[1])
        return out

    val = tensor_eval([Bt] + [Bs] * d)
    dtv = tensor_eval([Dt] + [Bs] * d)
    wq = tensor_eval([wt[:, None]] + [ws[:, None]] * d)[:, 0]
    A = gamma * val.T @ (wq[:, None] * dtv)
    # spatial direction l (1-based) is factor position d+1-l in (t, x_d, ..., x_1)
    for l in range(1, d + 1):
        facs = [Bt] + [Ds if k == d + 1 - l else Bs for k in range(1, d + 1)]
        g = tensor_eval(facs)
        A += nu * g.T @ (wq[:, None] * g)
    return A


def solve(A, b):
    """Direct solve by LU with partial pivoting (LAPACK gesv); columns of b are right-hand sides."""
    return np.linalg.solve(A, b)
