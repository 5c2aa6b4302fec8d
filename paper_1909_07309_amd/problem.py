"""Problem construction on the HIP side: 1D factors from libstig's own B-spline
assembly, boundary/initial restrictions (Section 2.2) and synthetic load vectors.

Identity geometry (unit square / cube), constant gamma and nu: the spatial
factors are the parametric K-hat_l, M-hat_l (eq. space_univ_par_mat) and the
time factors W_t, M_t = T M-hat (eq. time_mat and Section 4).
"""
from __future__ import annotations

import numpy as np
import torch

import workloads as wl

from .api import Plan, assemble_1d, load_1d, quadrature


class CubeFactors:
    """Restricted 1D factors for a workload on (0,1)^d x (0,T)."""

    def __init__(self, w: wl.Workload):
        self.w = w
        n_el, p = w.n_el, w.p
        Kf = assemble_1d(n_el, p, "stiffness")
        Mf = assemble_1d(n_el, p, "mass")
        # homogeneous Dirichlet: drop the first and last spatial function
        self.K = Kf[1:-1, 1:-1].copy()
        self.M = Mf[1:-1, 1:-1].copy()
        Wf = assemble_1d(n_el, p, "advection", length=w.T)
        Mtf = assemble_1d(n_el, p, "mass", length=w.T)
        # zero initial datum: drop the first time function
        self.Wt = Wf[1:, 1:].copy()
        self.Mt = Mtf[1:, 1:].copy()
        # column of the removed first time function (initial-datum lifting)
        self.W_col0 = Wf[1:, 0].copy()
        self.M_col0 = Mtf[1:, 0].copy()
        self.K1d = [self.K] * w.d
        self.M1d = [self.M] * w.d

    def make_plan(self) -> Plan:
        w = self.w
        plan = Plan([w.n_s] * w.d, w.n_t, w.p, w.p)
        plan.setup_1d_pencils(self.K1d, self.M1d, self.Wt, self.Mt, w.gamma, w.nu)
        return plan


def sine_source(w: wl.Workload, a, kx, ky, kt) -> np.ndarray:
    """Load vector of f = sum_k a_k sin(kx pi x) sin(ky pi y) sin(kt pi t / T) (d = 2),
    as a sum of Kronecker products of 1D load vectors (p+3 Gauss points per element)."""
    assert w.d == 2
    nq = w.p + 3
    xs, _ = quadrature(w.n_el, nq)
    xt, _ = quadrature(w.n_el, nq, w.T)
    f = np.zeros(w.shape)
    for ak, ax, ay, at in zip(a, kx, ky, kt):
        gx = load_1d(w.n_el, w.p, np.sin(ax * np.pi * xs), nq)[1:-1]
        gy = load_1d(w.n_el, w.p, np.sin(ay * np.pi * xs), nq)[1:-1]
        gt = load_1d(w.n_el, w.p, np.sin(at * np.pi * xt / w.T), nq, w.T)[1:]
        f += ak * np.multiply.outer(gt, np.multiply.outer(gy, gx))
    return f


def smoothed_source(plan: Plan, z: torch.Tensor) -> torch.Tensor:
    """f = (M_t (x) M_d (x) ... (x) M_1) z on the device (libstig mass apply)."""
    return plan.apply_mass(z.contiguous())


def source(w: wl.Workload, plan: Plan, device="cuda", seed=0) -> torch.Tensor:
    if w.source == "sines":
        f = sine_source(w, *wl.sine_terms(seed))
        return torch.from_numpy(f).to(device)
    z = torch.from_numpy(wl.source_coefficients(w, seed)).to(device)
    return smoothed_source(plan, z)
