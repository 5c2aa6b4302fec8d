"""Extruded quarter annulus with variable coefficients, 3D (oracle; test infrastructure only).

Geometry: F(eta) = ((1+eta_1) cos(pi eta_2 / 2), (1+eta_1) sin(pi eta_2 / 2), eta_3), the
quarter annulus of radii 1 and 2 extruded over [0, 1]; eta_1 is the radial (fastest)
direction.  With r = 1 + eta_1: |det J| = pi r / 2 and
J^{-1} J^{-T} |det J| = diag(pi r / 2, 2 / (pi r), pi r / 2).

Equation c(t) d_t u - div(kappa(x) grad u) = f with
kappa(x) = 1 + 0.5 sin(2 pi x) sin(2 pi y) cos(pi z) and c(t) = 1 + 0.3 cos(pi t).  The
coefficients separate between space and time, so Section 4.3.1 gives
    A = W_t (x) M_s + M_t' (x) K_s,
with W_t unweighted, [M_t']_ij = int b_i b_j / c(t) dt, M_s = int B_i B_j |det J| and
K_s = int kappa grad-hat B_i^T (J^{-1} J^{-T} |det J|) grad-hat B_j.

Preconditioner (Section 4.3, in 3D): the diagonal entries of the coefficient matrix
(C11 = kappa pi r / 2, C22 = 2 kappa / (pi r), C33 = kappa pi r / 2) and the mass
coefficient C00 = pi r / 2 are sampled at element midpoints and approximated by products
of univariate piecewise-constant factors (eq. separation): C00 ~ phi_1 phi_2 phi_3 by a
rank-one fit in log space, C_ll ~ Phi_l prod_{m != l} phi_m.  The univariate factors
weight the 1D matrices, giving A-tilde (eq. over_A), and A-hat^G = D^{1/2} A-tilde D^{1/2}
with D_ii = A_ii / A-tilde_ii (eq. prec_geo).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

import workloads as wl

from . import bsplines as bs


def extruded_polar_coefficients(e1, e2, e3):
    """(C11 / kappa, C22 / kappa, C33 / kappa, C00) of the extruded polar map."""
    r = 1.0 + e1 + 0.0 * (e2 + e3)
    return np.pi * r / 2.0, 2.0 / (np.pi * r), np.pi * r / 2.0, np.pi * r / 2.0


def physical_point(e1, e2, e3):
    r = 1.0 + e1
    th = np.pi * e2 / 2.0
    return r * np.cos(th), r * np.sin(th), e3 + 0.0 * r


class Annulus3DProblem:
    def __init__(self, w: wl.Workload, nq=None):
        self.w = w
        n_el, p = w.n_el, w.p
        nq = nq or p + 3
        xi = bs.open_uniform_knots(n_el, p)
        q, qw = bs.gauss_points(xi, nq)                  # element-major: e*nq + k
        Bf = bs.basis(xi, p, q)                          # [q, m] unrestricted
        Df = bs.basis_derivative(xi, p, q)
        e_idx = np.arange(n_el)[:, None, None]
        k_idx = np.arange(nq)[None, :, None]
        a_idx = np.arange(p + 1)[None, None, :]
        rows = e_idx * nq + k_idx
        NB = Bf[rows, e_idx + a_idx]                     # [e, k, a]
        ND = Df[rows, e_idx + a_idx]
        QX = q.reshape(n_el, nq)                         # [e, k]
        QW = qw.reshape(n_el, nq)
        # parametric points and weights on the grid [e3, k3, e2, k2, e1, k1]
        X3 = QX[:, :, None, None, None, None]
        X2 = QX[None, None, :, :, None, None]
        X1 = QX[None, None, None, None, :, :]
        W = (QW[:, :, None, None, None, None] * QW[None, None, :, :, None, None]
             * QW[None, None, None, None, :, :])
        c11, c22, c33, c00 = extruded_polar_coefficients(X1, X2, X3)
        kap = wl.annulus3d_conductivity(*physical_point(X1, X2, X3))
        n = n_el + p - 2
        self.n = n

        def assemble(coef, F1, G1, F2, G2, F3, G3):
            # local[e3, e2, e1, a3, b3, a2, b2, a1, b1]: one parametric direction at a time
            t1 = np.einsum("ukvlxm,xma,xmb->ukvlxab", coef, F1, G1, optimize=True)
            t2 = np.einsum("ukvlxab,vlc,vld->ukvxcdab", t1, F2, G2, optimize=True)
            loc = np.einsum("ukvxcdab,uke,ukf->uvxefcdab", t2, F3, G3, optimize=True)
            sh = loc.shape
            ax = [np.arange(s) for s in sh]
            e3, e2, e1, a3, b3, a2, b2, a1, b1 = np.meshgrid(*ax, indexing="ij", sparse=True)
            # restricted (Dirichlet) indices: global function g -> g - 1, valid in [0, n)
            i1, j1 = e1 + a1 - 1, e1 + b1 - 1
            i2, j2 = e2 + a2 - 1, e2 + b2 - 1
            i3, j3 = e3 + a3 - 1, e3 + b3 - 1
            I1, J1, I2, J2, I3, J3 = (np.broadcast_to(v, sh).ravel() for v in (i1, j1, i2, j2, i3, j3))
            V = loc.ravel()
            ok = ((I1 >= 0) & (I1 < n) & (J1 >= 0) & (J1 < n) & (I2 >= 0) & (I2 < n)
                  & (J2 >= 0) & (J2 < n) & (I3 >= 0) & (I3 < n) & (J3 >= 0) & (J3 < n))
            r = ((I3 * n + I2) * n + I1)[ok]
            c = ((J3 * n + J2) * n + J1)[ok]
            return sp.csr_matrix((V[ok], (r, c)), shape=(n ** 3, n ** 3))

        self.Ms = assemble(W * c00, NB, NB, NB, NB, NB, NB)
        self.Ks = (assemble(W * kap * c11, ND, ND, NB, NB, NB, NB)
                   + assemble(W * kap * c22, NB, NB, ND, ND, NB, NB)
                   + assemble(W * kap * c33, NB, NB, NB, NB, ND, ND))
        # time matrices: W_t unweighted, M_t weighted by 1 / c(t)
        self.Wt, _ = bs.time_matrices(n_el, p, w.T)
        xt = bs.open_uniform_knots(n_el, p, w.T)
        self.Mt = bs.restrict_time(bs.mass(xt, p, weight=lambda t: 1.0 / wl.annulus_heat_capacity(t),
                                            nq=nq))
        self._separation(xi)

    # ------------------------------------------------------------ separation
    def _separation(self, xi):
        w, p = self.w, self.w.p
        mids = 0.5 * (np.unique(xi)[:-1] + np.unique(xi)[1:])
        E3, E2, E1 = np.meshgrid(mids, mids, mids, indexing="ij")   # [e3, e2, e1]
        c11, c22, c33, c00 = extruded_polar_coefficients(E1, E2, E3)
        kap = wl.annulus3d_conductivity(*physical_point(E1, E2, E3))
        C = (kap * c11, kap * c22, kap * c33)
        L00 = np.log(c00)
        g = L00.mean()
        lphi1 = L00.mean(axis=(0, 1))                     # function of e1
        lphi2 = L00.mean(axis=(0, 2)) - g                 # function of e2
        lphi3 = L00.mean(axis=(1, 2)) - g                 # function of e3
        phi = (np.exp(lphi1), np.exp(lphi2), np.exp(lphi3))
        grids = (phi[0][None, None, :], phi[1][None, :, None], phi[2][:, None, None])
        axes = ((0, 1), (0, 2), (1, 2))                  # average over the other two directions
        Phi = []
        for l in range(3):
            other = np.ones_like(C[l])
            for m in range(3):
                if m != l:
                    other = other * grids[m]
            Phi.append(np.exp(np.log(C[l] / other).mean(axis=axes[l])))
        self.phi, self.Phi = phi, tuple(Phi)
        n_el = w.n_el

        def pc(vals):  # piecewise-constant weight function on the element grid
            return lambda x: vals[np.minimum((x * n_el).astype(int), n_el - 1)]
        self.Kt = [bs.restrict_space(bs.stiffness(xi, p, weight=pc(Ph))) for Ph in self.Phi]
        self.Mtl = [bs.restrict_space(bs.mass(xi, p, weight=pc(ph))) for ph in self.phi]

    # ------------------------------------------------------------ operators
    def matvec(self, x):
        """A x with the factored form W_t (x) M_s + M_t' (x) K_s (exact: the coefficients
        separate between space and time)."""
        X = np.asarray(x).reshape(self.w.n_t, -1)          # [t][s]
        MX = (self.Ms @ X.T).T
        KX = (self.Ks @ X.T).T
        return (self.Wt @ MX + self.Mt @ KX).reshape(np.shape(x))

    def diag_A(self):
        return (np.outer(np.diag(self.Wt), self.Ms.diagonal())
                + np.outer(np.diag(self.Mt), self.Ks.diagonal()))

    def diag_Atilde(self):
        dM = [np.diag(m) for m in self.Mtl]
        dK = [np.diag(k) for k in self.Kt]
        kron3 = lambda a3, a2, a1: np.einsum("i,j,k->ijk", a3, a2, a1).ravel()
        dMs = kron3(dM[2], dM[1], dM[0])
        dKs = kron3(dM[2], dM[1], dK[0]) + kron3(dM[2], dK[1], dM[0]) + kron3(dK[2], dM[1], dM[0])
        return np.outer(np.diag(self.Wt), dMs) + np.outer(np.diag(self.Mt), dKs)

    def D(self):
        """D_ii = A_ii / A-tilde_ii, shaped [t][x_3][x_2][x_1]."""
        return (self.diag_A() / self.diag_Atilde()).reshape(self.w.shape)

    def preconditioner(self):
        from .fd import FDPreconditioner
        return FDPreconditioner(self.Kt, self.Mtl, self.Wt, self.Mt, 1.0, 1.0, D=self.D())

    def dense_A(self):
        return (np.kron(self.Wt, self.Ms.toarray()) + np.kron(self.Mt, self.Ks.toarray()))

    def source(self, seed=0):
        """f = (M_t (x) M-hat_3 (x) M-hat_2 (x) M-hat_1) z with the plain parametric 1D mass matrices."""
        from .fd import mass_apply
        K, M = bs.space_matrices(self.w.n_el, self.w.p)
        _, Mt = bs.time_matrices(self.w.n_el, self.w.p, self.w.T)
        return mass_apply(wl.source_coefficients(self.w, seed), Mt, [M, M, M])
