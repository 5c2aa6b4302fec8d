"""Dense adjoint of the space-time solve on tiny grids (oracle; test infrastructure only).

Forward: the initial datum u_0(x) = sum_i c0_i B_i(x) b_1(t) uses the removed first
time B-spline b_1 as a discrete lifting (Section 3.1 splits u into a lifting of u_0
plus a solution with zero initial datum).  Keeping the full time basis, the Galerkin
equations for the kept unknowns read A u + A_{I,0} c0 = f, where A_{I,0} is the
block column of the unrestricted space-time matrix that belongs to the first time
function: A_{I,0} = gamma W[1:, 0] (x) M_s + nu M[1:, 0] (x) K_s.
Loss L = 0.5 ||u - u*||^2 summed over right-hand sides.  With lambda = A^{-T}(u - u*):
    dL/df = lambda,   dL/dc0 = -A_{I,0}^T lambda.
"""
from __future__ import annotations

import numpy as np

from . import bsplines as bs
from . import dense


class DenseAdjoint:
    def __init__(self, d, n_el, p, T=1.0, gamma=1.0, nu=1.0):
        K, M = bs.space_matrices(n_el, p)
        Wt, Mt = bs.time_matrices(n_el, p, T)
        Wf, Mf = bs.time_matrices_full(n_el, p, T)
        self.Ks, self.Ms = dense.spatial_kron([K] * d, [M] * d)
        self.A = gamma * np.kron(Wt, self.Ms) + nu * np.kron(Mt, self.Ks)
        self.AI0 = (gamma * np.kron(Wf[1:, 0][:, None], self.Ms)
                    + nu * np.kron(Mf[1:, 0][:, None], self.Ks))
        self.a_col, self.b_col = Wf[1:, 0].copy(), Mf[1:, 0].copy()

    def solve(self, f, c0):
        """u for flattened f (N,) and c0 (N_s,)."""
        return np.linalg.solve(self.A, f - self.AI0 @ c0)

    def loss(self, f, c0, target):
        u = self.solve(f, c0)
        return 0.5 * np.sum((u - target) ** 2)

    def gradients(self, f, c0, target):
        u = self.solve(f, c0)
        lam = np.linalg.solve(self.A.T, u - target)
        return lam, -self.AI0.T @ lam
