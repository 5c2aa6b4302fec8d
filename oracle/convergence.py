"""Manufactured-solution error of the space-time Galerkin solution (oracle; test infrastructure only).

Exact solution u = sin(pi t) prod_l sin(pi x_l) on (0,1)^d x (0,1): zero on the
spatial boundary and at t = 0, as eq. problem requires.  Its source is
f = gamma pi cos(pi t) prod sin + nu d pi^2 sin(pi t) prod sin.  The discrete
solution of eq. sys_solve is computed with the oracle's FD apply (A-hat = A on
the unit cube); errors are measured by tensor Gauss quadrature in the
L2(0,T;L2) norm (observed order p+1, Section 5.1) and in the
L2(0,T;H1_0) + H1(0,T;L2) norm that bounds the X_h norm (order p, eq.
a-riori-error-bound and the remark after it).
"""
from __future__ import annotations

import numpy as np

from . import bsplines as bs
from .fd import FDPreconditioner, mode_product


def _kron_eval(coeff, mats):
    """Evaluate sum_i c_i prod_k B_k[q_k, i_k] on a tensor grid; mats in array-axis order."""
    X = coeff
    for ax, B in enumerate(mats):
        X = mode_product(X, B, ax)
    return X


def manufactured_errors(d, n_el, p, gamma=1.0, nu=1.0):
    xs = bs.open_uniform_knots(n_el, p)
    K, M = bs.space_matrices(n_el, p)
    Wt, Mt = bs.time_matrices(n_el, p)
    # load vector: two separable terms, each a Kronecker product of 1D loads
    s = bs.restrict_space(bs.load(xs, p, lambda x: np.sin(np.pi * x)))
    ts = bs.restrict_time(bs.load(xs, p, lambda t: np.sin(np.pi * t)))
    tc = bs.restrict_time(bs.load(xs, p, lambda t: np.cos(np.pi * t)))
    prod_s = s
    for _ in range(d - 1):
        prod_s = np.multiply.outer(prod_s, s)
    f = (gamma * np.pi * np.multiply.outer(tc, prod_s)
         + nu * d * np.pi ** 2 * np.multiply.outer(ts, prod_s))
    P = FDPreconditioner([K] * d, [M] * d, Wt, Mt, gamma, nu)
    c = P.apply(f)

    # quadrature grid, p+3 points per element
    q, w = bs.gauss_points(xs, p + 3)
    Bs = bs.basis(xs, p, q)[:, 1:-1]
    Ds = bs.basis_derivative(xs, p, q)[:, 1:-1]
    Bt = bs.basis(xs, p, q)[:, 1:]
    Dt = bs.basis_derivative(xs, p, q)[:, 1:]
    sq, cq = np.sin(np.pi * q), np.cos(np.pi * q)

    def outer_all(vecs):
        out = vecs[0]
        for v in vecs[1:]:
            out = np.multiply.outer(out, v)
        return out

    wgt = outer_all([w] * (d + 1))
    uh = _kron_eval(c, [Bt] + [Bs] * d)
    u = outer_all([sq] * (d + 1))
    l2 = np.sqrt(np.sum(wgt * (u - uh) ** 2))
    l2u = np.sqrt(np.sum(wgt * u ** 2))
    # time derivative and gradient
    dt_h = _kron_eval(c, [Dt] + [Bs] * d)
    dt_u = outer_all([np.pi * cq] + [sq] * d)
    err_x = np.sum(wgt * (dt_u - dt_h) ** 2)
    nrm_x = np.sum(wgt * dt_u ** 2)
    for ax in range(1, d + 1):
        mats = [Bt] + [Ds if k == ax else Bs for k in range(1, d + 1)]
        g_h = _kron_eval(c, mats)
        g_u = outer_all([sq] + [np.pi * cq if k == ax else sq for k in range(1, d + 1)])
        err_x += np.sum(wgt * (g_u - g_h) ** 2)
        nrm_x += np.sum(wgt * g_u ** 2)
    return l2 / l2u, np.sqrt(err_x / nrm_x)
