"""The paper's stable arrowhead factorization of the time pencil and Algorithm 1
(oracle; test infrastructure only).

Section 4.2.2: split W_t and M_t into the leading (n_t-1) blocks, the last
column and the corner (eq. split).  The leading block of W_t is skew-symmetric
(from eq. integral_W), so the pencil (W-ring, M-ring) has an M-ring-orthonormal
eigenbasis U-ring with purely imaginary eigenvalues (eq. factorization_first_block).
The last column of U_t is [v; 1] normalised in the M_t norm, with M-ring v = -m
(eq. syst_v).  Then Delta_t = U_t^* W_t U_t is an arrowhead matrix
(eq. time_eig_2) and U_t^* M_t U_t = I (eq. Mt-orthogonality).

Section 4.4: with U_s, Lambda_s from eq. space_eig, A-hat factors as in
eq. preconditioner_str1, the middle factor has the block-arrowhead form
eq. syst-arr with diagonal blocks, and is solved by the block LU of
eq. block_LU with the diagonal Schur complement S = H_n + sum_i B_i^* H_i^{-1} B_i.

Algorithm 1 is read with input r and output s, i.e. it solves A-hat s = r
(eq. prec_appl): transform r with (U_t^* (x) U_s^T), apply the middle inverse,
transform back with (U_t (x) U_s).  Complex arithmetic throughout; the result's
imaginary part is rounding noise and is dropped.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .fd import axis_of, eigen_shift_tensor, mode_product, space_eig


def time_arrowhead(Wt, Mt):
    """Return (U_t, Delta_t, lam_ring, g, sigma) for the pencil (W_t, M_t)."""
    n = Wt.shape[0]
    Wr, w = Wt[:-1, :-1], Wt[:-1, -1]
    Mr, m = Mt[:-1, :-1], Mt[:-1, -1]
    # M-ring = L L^T; L^{-1} W-ring L^{-T} is real skew-symmetric, so i times it is
    # Hermitian and has a unitary eigenbasis Q: W-ring U = M-ring U Lambda with U = L^{-T} Q.
    L = np.linalg.cholesky(Mr)
    S = sla.solve_triangular(L, sla.solve_triangular(L, Wr.T, lower=True).T, lower=True)
    mu, Q = np.linalg.eigh(1j * S)
    lam_ring = -1j * mu                     # S Q = Q diag(-i mu)
    Ur = sla.solve_triangular(L.T, Q, lower=False)
    v = np.linalg.solve(Mr, -m)             # eq. syst_v
    col = np.concatenate([v, [1.0]])
    col = col / np.sqrt(col @ Mt @ col)
    U = np.zeros((n, n), dtype=complex)
    U[:-1, :-1] = Ur
    U[:, -1] = col
    # g and sigma as defined after eq. time_eig_2
    g = Ur.conj().T @ (np.hstack([Wr, w[:, None]]) @ col)
    sigma = col @ Wt @ col
    Delta = U.conj().T @ Wt @ U
    return U, Delta, lam_ring, g, sigma


class ArrowheadPreconditioner:
    """A-hat^{-1} r by Algorithm 1 with the paper's time factorization and block LU."""

    def __init__(self, K1d, M1d, Wt, Mt, gamma=1.0, nu=1.0):
        self.d = len(K1d)
        self.gamma, self.nu = gamma, nu
        eig = [space_eig(K1d[l], M1d[l]) for l in range(self.d)]
        self.U = [e[1] for e in eig]
        self.lam_s = eigen_shift_tensor([e[0] for e in eig])     # Lambda_s diagonal
        self.Ut, self.Delta, self.lam_ring, self.g, self.sigma = time_arrowhead(Wt, Mt)

    def apply(self, r):
        d, gam, nu = self.d, self.gamma, self.nu
        X = np.array(r, dtype=complex)
        # step 2: (U_t^* (x) U_s^T) r
        for l in range(1, d + 1):
            X = mode_product(X, self.U[l - 1].T, axis_of(l, d))
        X = mode_product(X, self.Ut.conj().T, 0)
        # step 3: block-arrowhead solve, eq. syst-arr and eq. block_LU
        n = X.shape[0]
        lam_s = self.lam_s
        H = [gam * self.lam_ring[i] + nu * lam_s for i in range(n - 1)]   # diagonals
        B = [gam * self.g[i] for i in range(n - 1)]                         # scalars
        Hn = gam * self.sigma + nu * lam_s
        Sch = Hn + sum(np.conj(B[i]) * B[i] / H[i] for i in range(n - 1))
        y_last = X[-1] + sum(np.conj(B[i]) * X[i] / H[i] for i in range(n - 1))
        Q = np.empty_like(X)
        Q[-1] = y_last / Sch
        for i in range(n - 1):
            Q[i] = (X[i] - B[i] * Q[-1]) / H[i]
        # step 4: (U_t (x) U_s) q
        Q = mode_product(Q, self.Ut, 0)
        for l in range(1, d + 1):
            Q = mode_product(Q, self.U[l - 1], axis_of(l, d))
        return Q.real
