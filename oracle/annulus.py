"""Quarter annulus with variable coefficients (oracle; test infrastructure only).

Geometry: polar map F(eta) = ((1+eta_1) cos(pi eta_2 / 2), (1+eta_1) sin(pi eta_2 / 2))
onto the quarter annulus of radii 1 and 2; eta_1 is the radial (fastest) direction.
With r = 1 + eta_1: |det J| = pi r / 2 and J^{-1} J^{-T} |det J| = diag(pi r / 2, 2 / (pi r)).

Equation c(t) d_t u - div(kappa(x) grad u) = f with kappa(x) = 1 + 0.5 sin(2 pi x) sin(2 pi y)
and c(t) = 1 + 0.3 cos(pi t).  The coefficients are separable between space and time
(gamma_s = 1, gamma_t = c, nu_s = kappa, nu_t = 1), so Section 4.3.1 gives
    A = W_t (x) M_s + M_t' (x) K_s,
with W_t unweighted, [M_t']_ij = int b_i b_j / c(t) dt (nu_t / gamma_t), and the spatial
matrices M_s = int B_i B_j |det J|, K_s = int kappa grad-hat B_i^T (J^{-1}J^{-T}|det J|) grad-hat B_j.

Preconditioner (Section 4.3): the diagonal entries of the coefficient matrix
(C11 = kappa pi r / 2, C22 = 2 kappa / (pi r), C33 = pi r / 2) are sampled at element
midpoints and approximated by products of univariate piecewise-constant factors
(eq. separation); the separation is a rank-one fit in log space: phi_l from C33,
Phi_l from C_ll divided by the other direction's phi.  The univariate factors weight
the 1D matrices, giving A-tilde (eq. over_A), and A-hat^G = D^{1/2} A-tilde D^{1/2}
with D_ii = A_ii / A-tilde_ii (eq. prec_geo).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

import workloads as wl

from . import bsplines as bs


def polar_coefficients(e1, e2):
    """(C11 / kappa, C22 / kappa, C33) of the polar map at parametric points."""
    r = 1.0 + e1
    return np.pi * r / 2.0, 2.0 / (np.pi * r), np.pi * r / 2.0


def physical_point(e1, e2):
    r = 1.0 + e1
    th = np.pi * e2 / 2.0
    return r * np.cos(th), r * np.sin(th)


class AnnulusProblem:
    def __init__(self, w: wl.Workload, nq=None):
        self.w = w
        n_el, p = w.n_el, w.p
        nq = nq or p + 3
        xi = bs.open_uniform_knots(n_el, p)
        q, qw = bs.gauss_points(xi, nq)                  # element-major: e*nq + k
        Bf = bs.basis(xi, p, q)                          # [q, m] unrestricted
        Df = bs.basis_derivative(xi, p, q)
        # local values: element e, point k, local function a -> global function e + a
        e_idx = np.arange(n_el)[:, None, None]
        k_idx = np.arange(nq)[None, :, None]
        a_idx = np.arange(p + 1)[None, None, :]
        rows = e_idx * nq + k_idx
        NB = Bf[rows, e_idx + a_idx]                     # [e, k, a]
        ND = Df[rows, e_idx + a_idx]
        QX = q.reshape(n_el, nq)                         # [e, k]
        QW = qw.reshape(n_el, nq)
        # coefficients on the tensor grid [e2, k2, e1, k1]
        E1 = QX[None, None, :, :] + 0 * QX[:, :, None, None]
        E2 = QX[:, :, None, None] + 0 * QX[None, None, :, :]
        c11, c22, c33 = polar_coefficients(E1, E2)
        X, Y = physical_point(E1, E2)
        kap = wl.annulus_conductivity(X, Y)
        WW = QW[:, :, None, None] * QW[None, None, :, :]
        n = n_el + p - 2

        def assemble(coef, F1, G1, F2, G2):
            # local[e2, e1, a2, b2, a1, b1] = sum_{k2,k1} coef F1[e1,k1,a1] G1[e1,k1,b1] F2[e2,k2,a2] G2[e2,k2,b2]
            t = np.einsum("xkyl,yla,ylb->xkyab", coef, F1, G1, optimize=True)
            loc = np.einsum("xkyab,xkc,xkd->xycdab", t, F2, G2, optimize=True)
            e2 = np.arange(n_el)[:, None, None, None, None, None]
            e1 = np.arange(n_el)[None, :, None, None, None, None]
            a2 = np.arange(p + 1)[None, None, :, None, None, None]
            b2 = np.arange(p + 1)[None, None, None, :, None, None]
            a1 = np.arange(p + 1)[None, None, None, None, :, None]
            b1 = np.arange(p + 1)[None, None, None, None, None, :]
            # restricted (Dirichlet) indices: global function g -> g - 1, valid in [0, n)
            i1, j1, i2, j2 = e1 + a1 - 1, e1 + b1 - 1, e2 + a2 - 1, e2 + b2 - 1
            shape = loc.shape
            I1, J1, I2, J2 = (np.broadcast_to(v, shape).ravel() for v in (i1, j1, i2, j2))
            V = loc.ravel()
            ok = (I1 >= 0) & (I1 < n) & (J1 >= 0) & (J1 < n) & (I2 >= 0) & (I2 < n) & (J2 >= 0) & (J2 < n)
            r = (I2 * n + I1)[ok]
            c = (J2 * n + J1)[ok]
            return sp.csr_matrix((V[ok], (r, c)), shape=(n * n, n * n))

        self.Ms = assemble(WW * c33, NB, NB, NB, NB)
        self.Ks = (assemble(WW * kap * c11, ND, ND, NB, NB)
                   + assemble(WW * kap * c22, NB, NB, ND, ND))
        # time matrices: W_t unweighted, M_t weighted by 1 / c(t)
        self.Wt, _ = bs.time_matrices(n_el, p, w.T)
        xt = bs.open_uniform_knots(n_el, p, w.T)
        self.Mt = bs.restrict_time(bs.mass(xt, p, weight=lambda t: 1.0 / wl.annulus_heat_capacity(t),
                                            nq=nq))
        self.n = n
        self._separation(xi)

    # ------------------------------------------------------------ separation
    def _separation(self, xi):
        w, p = self.w, self.w.p
        mids = 0.5 * (np.unique(xi)[:-1] + np.unique(xi)[1:])
        E1, E2 = np.meshgrid(mids, mids, indexing="xy")   # [e2, e1]
        c11, c22, c33 = polar_coefficients(E1, E2)
        X, Y = physical_point(E1, E2)
        kap = wl.annulus_conductivity(X, Y)
        C11, C22, C33 = kap * c11, kap * c22, c33
        L33 = np.log(C33)
        lphi1 = L33.mean(axis=0)                          # function of e1
        lphi2 = L33.mean(axis=1) - L33.mean()              # function of e2
        phi1, phi2 = np.exp(lphi1), np.exp(lphi2)
        Phi1 = np.exp(np.log(C11 / phi2[:, None]).mean(axis=0))
        Phi2 = np.exp(np.log(C22 / phi1[None, :]).mean(axis=1))
        self.phi = (phi1, phi2)
        self.Phi = (Phi1, Phi2)
        n_el = w.n_el

        def pc(vals):  # piecewise-constant weight function on the element grid
            return lambda x: vals[np.minimum((x * n_el).astype(int), n_el - 1)]
        self.Kt = [bs.restrict_space(bs.stiffness(xi, p, weight=pc(Phi))) for Phi in self.Phi]
        self.Mtl = [bs.restrict_space(bs.mass(xi, p, weight=pc(phi))) for phi in self.phi]

    # ------------------------------------------------------------ operators
    def matvec(self, x):
        """A x with the factored form W_t (x) M_s + M_t' (x) K_s (exact for separable coefficients)."""
        X = np.asarray(x).reshape(self.w.n_t, -1)          # [t][s]
        MX = (self.Ms @ X.T).T
        KX = (self.Ks @ X.T).T
        return (self.Wt @ MX + self.Mt @ KX).reshape(np.shape(x))

    def diag_A(self):
        return (np.outer(np.diag(self.Wt), self.Ms.diagonal())
                + np.outer(np.diag(self.Mt), self.Ks.diagonal()))

    def diag_Atilde(self):
        M1, M2 = self.Mtl
        K1, K2 = self.Kt
        dMs = np.outer(np.diag(M2), np.diag(M1)).ravel()
        dKs = (np.outer(np.diag(M2), np.diag(K1)) + np.outer(np.diag(K2), np.diag(M1))).ravel()
        return np.outer(np.diag(self.Wt), dMs) + np.outer(np.diag(self.Mt), dKs)

    def D(self):
        """D_ii = A_ii / A-tilde_ii, shaped [t][x_2][x_1]."""
        return (self.diag_A() / self.diag_Atilde()).reshape(self.w.shape)

    def preconditioner(self):
        from .fd import FDPreconditioner
        return FDPreconditioner(self.Kt, self.Mtl, self.Wt, self.Mt, 1.0, 1.0, D=self.D())

    def dense_A(self):
        return (np.kron(self.Wt, self.Ms.toarray()) + np.kron(self.Mt, self.Ks.toarray()))

    def source(self, seed=0):
        """f = (M_t (x) M-hat_2 (x) M-hat_1) z with the plain parametric 1D mass matrices."""
        from .fd import mass_apply
        K, M = bs.space_matrices(self.w.n_el, self.w.p)
        _, Mt = bs.time_matrices(self.w.n_el, self.w.p, self.w.T)
        return mass_apply(wl.source_coefficients(self.w, seed), Mt, [M, M])
