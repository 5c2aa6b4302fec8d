"""Manufactured-solution error of the space-time Galerkin solution (oracle; test infrastructure only).

Exact solution u = sin(pi t) prod_l sin(pi x_l) on (0,1)^d x (0,1): zero on the
spatial boundary and at t = 0, as eq. problem requires.  Its source is
f = gamma pi cos(pi t) prod sin + nu d pi^2 sin(pi t) prod sin.  The discrete
solution of eq. sys_solve is computed with the oracle's FD apply (A-hat = A on
the unit cube); errors are measured by tensor Gauss quadrature in the
L2(0,T;L2) norm (observed order p+1, Section 5.1) and in the
L2(0,T;H1_0) + H1(0,T;L2) norm that bounds the X_h norm (order p, eq.
a-riori-error-bound and the remark after it).

The second part does the same on the quarter annulus with the annulus
workload's variable conductivity and heat capacity (see the section below):
it is the check that pins the variable-coefficient assembly.
"""
from __future__ import annotations

import numpy as np

import workloads as wl

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


# ------------------------------------------------------------ quarter annulus
#
# The two-dimensional counterpart of the paper's manufactured example on the
# rotated quarter annulus (Section 5.1): u = -(r^2-1)(r^2-4) x y^2 sin t on the
# quarter annulus of radii 1 and 2 in the first quadrant, which vanishes on the
# whole spatial boundary (r = 1, r = 2, x = 0, y = 0) and at t = 0.  The
# equation is the variable-coefficient one of the annulus workload,
# c(t) d_t u - div(kappa grad u) = f, divided by c (Section 4.3.1), so the
# Galerkin right-hand side is the load of f / c.

def annulus_solution(x, y):
    """Spatial factor u_s of the exact solution, its gradient and its Laplacian,
    written out by hand: u_s = g h with g = -(s-1)(s-4), s = x^2 + y^2, h = x y^2."""
    s = x * x + y * y
    g = -(s - 1.0) * (s - 4.0)
    gx, gy = -(2.0 * s - 5.0) * 2.0 * x, -(2.0 * s - 5.0) * 2.0 * y
    gxx, gyy = -(8.0 * x * x + 4.0 * s - 10.0), -(8.0 * y * y + 4.0 * s - 10.0)
    h, hx, hy, hxx, hyy = x * y * y, y * y, 2.0 * x * y, 0.0, 2.0 * x
    u = g * h
    ux, uy = gx * h + g * hx, gy * h + g * hy
    lap = gxx * h + 2.0 * gx * hx + g * hxx + gyy * h + 2.0 * gy * hy + g * hyy
    return u, ux, uy, lap


def annulus_conductivity_gradient(x, y):
    """Gradient of the workload's kappa = 1 + 0.5 sin(2 pi x) sin(2 pi y)."""
    return (np.pi * np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y),
            np.pi * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y))


def annulus_manufactured_errors(problem, rtol=1e-13):
    """Relative L2(0,T;L2) and X-type (L2(0,T;H1_0) + H1(0,T;L2)) errors of the
    discrete solution of A u = F on the quarter annulus, where A is the problem's
    own space-time matrix (problem.Ms, Ks, Wt, Mt) and F the load of f / c for the
    manufactured solution above.

    The load and the errors use tensor Gauss quadrature with p+3 points per
    element on the parametric square and in time; physical points, |det J| and
    the polar gradient are computed here from the map, independently of the
    problem's assembly.  The system is solved by GMRES preconditioned with the
    problem's geometry-aware fast diagonalization, to the relative residual rtol
    (checked)."""
    import scipy.sparse.linalg as spl

    w = problem.w
    n_el, p, T = w.n_el, w.p, w.T
    nq = p + 3
    xs = bs.open_uniform_knots(n_el, p)
    xt = bs.open_uniform_knots(n_el, p, T)
    q, qw = bs.gauss_points(xs, nq)
    qt, qtw = bs.gauss_points(xt, nq)
    B = bs.basis(xs, p, q)[:, 1:-1]
    D = bs.basis_derivative(xs, p, q)[:, 1:-1]
    Bt = bs.basis(xt, p, qt)[:, 1:]
    Dt = bs.basis_derivative(xt, p, qt)[:, 1:]
    # parametric grid [q2][q1]; eta_1 radial, eta_2 angular
    E2, E1 = np.meshgrid(q, q, indexing="ij")
    r = 1.0 + E1
    th = 0.5 * np.pi * E2
    X, Y = r * np.cos(th), r * np.sin(th)
    jac = 0.5 * np.pi * r
    u, ux, uy, lap = annulus_solution(X, Y)
    kap = wl.annulus_conductivity(X, Y)
    kx, ky = annulus_conductivity_gradient(X, Y)
    div = kx * ux + ky * uy + kap * lap             # div(kappa grad u_s)
    c = wl.annulus_heat_capacity(qt)
    W2 = np.outer(qw, qw) * jac
    # F = load of f / c = u_s cos t - div sin t / c, a sum of two space-time products
    ls_u = B.T @ (W2 * u) @ B                        # [i2][i1]
    ls_d = B.T @ (W2 * div) @ B
    lt_c = Bt.T @ (qtw * np.cos(qt))
    lt_s = Bt.T @ (qtw * np.sin(qt) / c)
    F = np.multiply.outer(lt_c, ls_u) - np.multiply.outer(lt_s, ls_d)
    N = F.size
    P = problem.preconditioner()
    Aop = spl.LinearOperator((N, N), matvec=lambda v: problem.matvec(v.reshape(F.shape)).ravel())
    Mop = spl.LinearOperator((N, N), matvec=lambda v: P.apply(v.reshape(F.shape)).ravel())
    sol, _ = spl.gmres(Aop, F.ravel(), M=Mop, rtol=rtol, restart=80, maxiter=20)
    res = np.linalg.norm(F.ravel() - Aop @ sol) / np.linalg.norm(F)
    if not res <= 10 * rtol:
        raise RuntimeError(f"manufactured solve reached only {res:.2e}")
    Cf = sol.reshape(F.shape)                        # [t][i2][i1]

    def ev(Tm, S2, S1):
        return np.einsum("ta,aij->tij", Tm,
                         np.einsum("ib,abj->aij", S2, np.einsum("jc,abc->abj", S1, Cf)))

    Wq = np.multiply.outer(qtw, W2)
    sq, cq = np.sin(qt), np.cos(qt)
    U = np.multiply.outer(sq, u)
    l2 = np.sqrt(np.sum(Wq * (U - ev(Bt, B, B)) ** 2) / np.sum(Wq * U ** 2))
    # X-type norm: time derivative and the physical gradient.  For the polar map
    # d/d eta_1 = d/dr and d/d eta_2 = (pi/2) d/d theta, and
    # |grad v|^2 = (dv/dr)^2 + (dv/dtheta / r)^2.
    ur = ux * np.cos(th) + uy * np.sin(th)
    ut = -ux * np.sin(th) + uy * np.cos(th)          # (du/dtheta) / r
    e_t = np.multiply.outer(cq, u) - ev(Dt, B, B)
    e_r = np.multiply.outer(sq, ur) - ev(Bt, B, D)
    e_a = np.multiply.outer(sq, ut) - ev(Bt, D, B) / (0.5 * np.pi * r)[None]
    err_x = np.sum(Wq * (e_t ** 2 + e_r ** 2 + e_a ** 2))
    nrm_x = np.sum(Wq * (np.multiply.outer(cq, u) ** 2 + np.multiply.outer(sq, ur) ** 2
                         + np.multiply.outer(sq, ut) ** 2))
    return l2, np.sqrt(err_x / nrm_x)
