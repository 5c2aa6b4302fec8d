"""Extruded quarter-annulus workload on the HIP side: the 3D geometry-aware
preconditioner of Section 4.3 with variable conductivity and heat capacity, A x
from the sparse spatial factors (Section 4.5) or a full space-time CSR, and the
3D separation of the coefficients.

Geometry (problem data): F(eta) = ((1+eta_1) cos(pi eta_2/2), (1+eta_1)
sin(pi eta_2/2), eta_3), the quarter annulus with radii 1 and 2 extruded over
[0, 1].  With r = 1 + eta_1: |det J| = pi r / 2 and J^{-1} J^{-T} |det J| =
diag(pi r / 2, 2/(pi r), pi r / 2).  The equation c(t) d_t u - div(kappa grad u)
= f is divided by c(t) (Section 4.3.1): A = W_t (x) M_s + M_t' (x) K_s with
[M_t']_ij = int b_i b_j / c.  The preconditioner is A-hat^G = D^{1/2} A-tilde
D^{1/2} (eq. prec_geo) with A-tilde from 1D factors weighted by the separated
coefficients (eq. separation, eq. over_A) and D_ii = A_ii / A-tilde_ii.
"""
from __future__ import annotations

import numpy as np
import torch

import workloads as wl

from .api import Plan, assemble_1d, assemble_3d, quadrature, separate_3d


def extruded_polar_coefficients(e1, e2, e3):
    """kappa-free diagonal of J^{-1} J^{-T} |det J| (C11, C22, C33) and |det J| (C00)."""
    r = 1.0 + e1
    return 0.5 * np.pi * r, 2.0 / (np.pi * r), 0.5 * np.pi * r, 0.5 * np.pi * r


def physical(e1, e2, e3):
    r = 1.0 + e1
    return r * np.cos(0.5 * np.pi * e2), r * np.sin(0.5 * np.pi * e2), e3 + 0.0 * r


def _csr_diagonal(rowptr, col, val):
    rows = np.repeat(np.arange(rowptr.size - 1), np.diff(rowptr))
    on = col == rows
    out = np.zeros(rowptr.size - 1)
    out[rows[on]] = val[on]
    return out


class Annulus3DSetup:
    """Host-side setup (3D spatial CSR, time factors, separated 1D factors) and the plan."""

    def __init__(self, w: wl.Workload, nq=None):
        assert w.d == 3
        self.w = w
        n_el, p = w.n_el, w.p
        self.nq = nq = nq or p + 3
        x, _ = quadrature(n_el, nq)
        E3, E2, E1 = np.meshgrid(x, x, x, indexing="ij")      # [q3][q2][q1]
        c11, c22, c33, c00 = extruded_polar_coefficients(E1, E2, E3)
        kap = wl.annulus3d_conductivity(*physical(E1, E2, E3))
        self.space = assemble_3d(n_el, p, nq, kap * c11, kap * c22, kap * c33, c00)
        rp, col, vK, vM = self.space
        self.dKs, self.dMs = _csr_diagonal(rp, col, vK), _csr_diagonal(rp, col, vM)
        # time factors: W_t unweighted, M_t weighted by 1/c(t), first function removed
        xt, _ = quadrature(n_el, nq, w.T)
        Wf = assemble_1d(n_el, p, "advection", length=w.T)
        Mf = assemble_1d(n_el, p, "mass", length=w.T,
                         weight=1.0 / wl.annulus_heat_capacity(xt), nq=nq)
        self.Wt, self.Mt = Wf[1:, 1:].copy(), Mf[1:, 1:].copy()
        # separated coefficients at element midpoints -> weighted 1D factors
        mids = (np.arange(n_el) + 0.5) / n_el
        M3, M2, M1 = np.meshgrid(mids, mids, mids, indexing="ij")
        m11, m22, m33, m00 = extruded_polar_coefficients(M1, M2, M3)
        mk = wl.annulus3d_conductivity(*physical(M1, M2, M3))
        phi1, phi2, phi3, Phi1, Phi2, Phi3 = separate_3d(mk * m11, mk * m22, mk * m33, m00)
        elem = np.repeat(np.arange(n_el), nq)                 # element of each quadrature point
        self.Kt = [assemble_1d(n_el, p, "stiffness", weight=Ph[elem], nq=nq)[1:-1, 1:-1].copy()
                   for Ph in (Phi1, Phi2, Phi3)]
        self.Mtl = [assemble_1d(n_el, p, "mass", weight=ph[elem], nq=nq)[1:-1, 1:-1].copy()
                    for ph in (phi1, phi2, phi3)]

    def make_plan(self, matvec="csr", device="cuda"):
        """matvec: "csr" (the whole space-time matrix on the device), "factored" (only the
        sparse spatial factors, Section 4.5) or None (the plan's Kronecker factors)."""
        w = self.w
        plan = Plan([w.n_s] * 3, w.n_t, w.p, w.p)
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
        """f = (M_t (x) M-hat_3 (x) M-hat_2 (x) M-hat_1) z with the plain parametric mass matrices."""
        from .problem import CubeFactors
        fac = CubeFactors(wl.Workload("plain", d=3, p=self.w.p, n_el=self.w.n_el, T=self.w.T))
        mplan = fac.make_plan()
        z = torch.from_numpy(wl.source_coefficients(self.w, seed)).to(device)
        return mplan.apply_mass(z)
