"""Quarter-annulus workload on the HIP side: variable conductivity and heat capacity,
A x from the sparse spatial factors and the time bands (Section 4.5) or from the
full space-time CSR, geometry-aware preconditioner (Section 4.3).

Geometry (problem data): the polar map F(eta) = ((1+eta_1) cos(pi eta_2/2),
(1+eta_1) sin(pi eta_2/2)) onto the quarter annulus with radii 1 and 2.  Its
Jacobian gives |det J| = pi r / 2 and J^{-1} J^{-T} |det J| = diag(pi r / 2, 2/(pi r)),
r = 1 + eta_1.  The equation c(t) d_t u - div(kappa grad u) = f is divided by c(t)
(Section 4.3.1): A = W_t (x) M_s + M_t' (x) K_s with [M_t']_ij = int b_i b_j / c.
"""
from __future__ import annotations

import numpy as np
import torch

import workloads as wl

from .api import Plan, assemble_1d, assemble_2d, quadrature, separate_2d


def polar_map_coefficients(e1, e2):
    """kappa-free diagonal entries (C11, C22) and C33 = |det J| of the polar map."""
    r = 1.0 + e1
    return 0.5 * np.pi * r, 2.0 / (np.pi * r), 0.5 * np.pi * r


def physical(e1, e2):
    r = 1.0 + e1
    return r * np.cos(0.5 * np.pi * e2), r * np.sin(0.5 * np.pi * e2)


class AnnulusSetup:
    """Host-side setup (spatial CSR, time factors, separated 1D factors) and the plan."""

    def __init__(self, w: wl.Workload, nq=None):
        assert w.d == 2
        self.w = w
        n_el, p = w.n_el, w.p
        self.nq = nq = nq or p + 3
        x, _ = quadrature(n_el, nq)
        E1, E2 = np.meshgrid(x, x, indexing="xy")          # [q2][q1]
        c11, c22, c33 = polar_map_coefficients(E1, E2)
        kap = wl.annulus_conductivity(*physical(E1, E2))
        self.space = assemble_2d(n_el, p, nq, kap * c11, kap * c22, c33)
        rp, col, vK, vM = self.space
        diag_idx = [rp[s] + np.nonzero(col[rp[s]:rp[s + 1]] == s)[0][0] for s in range(rp.size - 1)]
        self.dKs, self.dMs = vK[diag_idx], vM[diag_idx]
        # time factors: W_t unweighted, M_t weighted by 1/c(t), first function removed
        xt, _ = quadrature(n_el, nq, w.T)
        Wf = assemble_1d(n_el, p, "advection", length=w.T)
        Mf = assemble_1d(n_el, p, "mass", length=w.T,
                         weight=1.0 / wl.annulus_heat_capacity(xt), nq=nq)
        self.Wt, self.Mt = Wf[1:, 1:].copy(), Mf[1:, 1:].copy()
        # separated coefficients at element midpoints -> weighted 1D factors
        mids = (np.arange(n_el) + 0.5) / n_el
        M1, M2 = np.meshgrid(mids, mids, indexing="xy")
        m11, m22, m33 = polar_map_coefficients(M1, M2)
        mk = wl.annulus_conductivity(*physical(M1, M2))
        phi1, phi2, Phi1, Phi2 = separate_2d(mk * m11, mk * m22, m33)
        elem = np.repeat(np.arange(n_el), nq)              # element of each quadrature point
        self.Kt = [assemble_1d(n_el, p, "stiffness", weight=Ph[elem], nq=nq)[1:-1, 1:-1].copy()
                   for Ph in (Phi1, Phi2)]
        self.Mtl = [assemble_1d(n_el, p, "mass", weight=ph[elem], nq=nq)[1:-1, 1:-1].copy()
                    for ph in (phi1, phi2)]

    def make_plan(self, matvec="csr", device="cuda"):
        """matvec: "csr" (the whole space-time matrix on the device), "factored" (only the
        sparse spatial factors, Section 4.5) or None (the plan's Kronecker factors)."""
        w = self.w
        plan = Plan([w.n_s, w.n_s], w.n_t, w.p, w.p)
        plan.setup_1d_pencils(self.Kt, self.Mtl, self.Wt, self.Mt, 1.0, 1.0)
        plan.set_diag_scaling_kron(self.dMs, self.dKs)
        if matvec == "csr":
            rowptr, col, val = plan.kron_csr(self.space, self.Wt, self.Mt, device)
            plan.set_A_csr(rowptr, col, val)
        elif matvec == "factored":
            plan.set_spatial_factors(self.space)
        else:
            assert matvec is None, matvec
        return plan

    def source(self, device="cuda", seed=0):
        """f = (M_t (x) M-hat_2 (x) M-hat_1) z with the plain parametric mass matrices."""
        from .problem import CubeFactors
        fac = CubeFactors(wl.Workload("plain", d=2, p=self.w.p, n_el=self.w.n_el, T=self.w.T))
        mplan = fac.make_plan()
        z = torch.from_numpy(wl.source_coefficients(self.w, seed)).to(device)
        return mplan.apply_mass(z)
