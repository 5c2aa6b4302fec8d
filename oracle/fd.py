"""Fast-diagonalization apply of A-hat^{-1} and Kronecker matvec (oracle; test infrastructure only).

A-hat = gamma W_t (x) M_s + nu M_t (x) K_s (eq. prec_definition).  With the spatial
generalized eigendecompositions U_l^T K_l U_l = Lambda_l, U_l^T M_l U_l = I
(eq. space_eig) and U_s = U_d (x) ... (x) U_1,

    (I (x) U_s^T) A-hat (I (x) U_s) = gamma W_t (x) I + nu M_t (x) Lambda_s,

which is block diagonal after a permutation: one n_t x n_t system
(gamma W_t + nu lambda_k M_t) per spatial eigen-index k, lambda_k = sum_l lambda_{l,i_l}.
So A-hat^{-1} r = step 2 (forward spatial transform with U_l^T), step 3 (the shifted
time systems), step 4 (back transform with U_l) -- the structure of Algorithm 1 with
the time pencil left un-diagonalized.  The time systems are banded (bandwidth p_t)
and are solved by Gaussian elimination without pivoting: the symmetric part of
gamma W_t + nu lambda M_t is (gamma/2) e_n e_n^T + nu lambda M_t (eq. integral_W),
positive definite for lambda > 0, so every pivot is nonzero.

Mode products follow the definition of Section 2.3:
    [X x_m J]_{..., i_m, ...} = sum_j X_{..., j, ...} J_{i_m, j},
and the Kronecker-vector identity eq. kron_vec_multi.  Arrays are C-order
[t][x_d]..[x_1], so spatial direction l is array axis d+1-l (time is axis 0).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def space_eig(K, M):
    """Generalized symmetric eigendecomposition K U = M U Lambda with U^T M U = I (eq. space_eig).

    Eigenvalues ascending (LAPACK sygvd via scipy)."""
    lam, U = sla.eigh(K, M)
    return lam, U


def mode_product(X, J, axis):
    """X x_axis J: contracts array axis ``axis`` of X with the columns of J (Section 2.3)."""
    Y = np.tensordot(J, X, axes=([1], [axis]))   # new axis 0 = rows of J
    return np.moveaxis(Y, 0, axis)


def axis_of(l, d, batch=0):
    """Array axis of spatial direction l (1-based) in [batch..][t][x_d]..[x_1]."""
    return batch + d + 1 - l


def eigen_shift_tensor(lams):
    """lambda_k = sum_l lambda_{l, i_l}, shaped [x_d]..[x_1] (Lambda_s of Section 4.4)."""
    d = len(lams)
    out = np.zeros([len(lams[l]) for l in reversed(range(d))])
    for l in range(d):
        shape = [1] * d
        shape[d - 1 - l] = len(lams[l])
        out = out + lams[l].reshape(shape)
    return out


def band_width(A, tol=0.0):
    """Largest |i - j| with a nonzero entry."""
    i, j = np.nonzero(np.abs(A) > tol)
    return int(np.max(np.abs(i - j))) if len(i) else 0


def banded_shifted_solve(Wt, Mt, lam, R, gamma=1.0, nu=1.0, transpose=False):
    """Solve (gamma W + nu lam_k M) q_k = r_k for every k at once.

    R has shape [n_t, K] (time first); lam has shape [K].  With transpose=True the
    systems are (gamma W^T + nu lam_k M) q_k = r_k (the adjoint; M is symmetric).
    Gaussian elimination without pivoting on the band, vectorised over k.
    """
    W = Wt.T if transpose else Wt
    n = W.shape[0]
    p = max(band_width(W), band_width(Mt))
    K = R.shape[1]
    # band storage: Ab[i, p + (j - i), k] = A_k[i, j] for |i - j| <= p
    Ab = np.zeros((n, 2 * p + 1, K))
    for i in range(n):
        for j in range(max(0, i - p), min(n, i + p + 1)):
            Ab[i, p + j - i, :] = gamma * W[i, j] + nu * lam * Mt[i, j]
    b = np.array(R, dtype=float, copy=True)
    for i in range(n):                       # forward elimination
        piv = Ab[i, p, :]
        if np.any(piv <= 0.0):
            raise ZeroDivisionError("non-positive pivot in shifted time system")
        for r in range(1, p + 1):
            if i + r >= n:
                break
            l = Ab[i + r, p - r, :] / piv
            for c in range(0, p + 1):        # row i, columns i..i+p
                if i + c < n:
                    Ab[i + r, p - r + c, :] -= l * Ab[i, p + c, :]
            b[i + r] -= l * b[i]
    q = np.zeros_like(b)
    for i in range(n - 1, -1, -1):           # back substitution
        acc = b[i].copy()
        for c in range(1, p + 1):
            if i + c < n:
                acc -= Ab[i, p + c, :] * q[i + c]
        q[i] = acc / Ab[i, p, :]
    return q


class FDPreconditioner:
    """A-hat^{-1} by fast diagonalization with banded time solves.

    K1d, M1d: lists of 1D spatial factors in direction order l = 1..d.
    Wt, Mt:  time factors.  Optional D (shape of the unknown tensor) gives the
    geometry-aware variant A-hat^G = D^{1/2} A-tilde D^{1/2} of eq. prec_geo:
    (A-hat^G)^{-1} r = D^{-1/2} A-tilde^{-1} D^{-1/2} r.
    """

    def __init__(self, K1d, M1d, Wt, Mt, gamma=1.0, nu=1.0, D=None):
        self.d = len(K1d)
        self.Wt, self.Mt = np.asarray(Wt), np.asarray(Mt)
        self.gamma, self.nu = gamma, nu
        eig = [space_eig(K1d[l], M1d[l]) for l in range(self.d)]
        self.lams = [e[0] for e in eig]
        self.U = [e[1] for e in eig]
        self.lam = eigen_shift_tensor(self.lams)
        self.Dmh = None if D is None else 1.0 / np.sqrt(D)

    def apply(self, r, transpose=False):
        """s = A-hat^{-1} r (or A-hat^{-T} r); r has the unknown-tensor shape [t][x_d]..[x_1]."""
        d = self.d
        X = np.array(r, dtype=float)
        if self.Dmh is not None:
            X = X * self.Dmh
        for l in range(1, d + 1):                     # step 2: x_l U_l^T
            X = mode_product(X, self.U[l - 1].T, axis_of(l, d))
        n_t = X.shape[0]
        Q = banded_shifted_solve(self.Wt, self.Mt, self.lam.ravel(),
                                 X.reshape(n_t, -1), self.gamma, self.nu,
                                 transpose).reshape(X.shape)   # step 3
        for l in range(1, d + 1):                     # step 4: x_l U_l
            Q = mode_product(Q, self.U[l - 1], axis_of(l, d))
        if self.Dmh is not None:
            Q = Q * self.Dmh
        return Q


def kron_matvec(x, Wt, Mt, K1d, M1d, gamma=1.0, nu=1.0, transpose=False):
    """y = (gamma W_t (x) M_s + nu M_t (x) K_s) x by mode products (eq. kron_vec_multi).

    transpose=True gives A^T x = (gamma W_t^T (x) M_s + nu M_t (x) K_s) x."""
    d = len(K1d)
    W = Wt.T if transpose else Wt
    mass_part = np.array(x, dtype=float)
    for l in range(1, d + 1):
        mass_part = mode_product(mass_part, M1d[l - 1], axis_of(l, d))
    y = gamma * mode_product(mass_part, W, 0)
    for l in range(1, d + 1):
        term = np.array(x, dtype=float)
        for j in range(1, d + 1):
            term = mode_product(term, K1d[j - 1] if j == l else M1d[j - 1], axis_of(j, d))
        y = y + nu * mode_product(term, Mt, 0)
    return y


def mass_apply(z, Mt, M1d):
    """(M_t (x) M_d (x) ... (x) M_1) z: load vector of the spline function with coefficients z."""
    d = len(M1d)
    X = np.array(z, dtype=float)
    for l in range(1, d + 1):
        X = mode_product(X, M1d[l - 1], axis_of(l, d))
    return mode_product(X, Mt, 0)
