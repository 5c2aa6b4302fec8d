"""Oracle-side problem construction for the synthetic workloads (test infrastructure only).

Turns the seeded draws of ``workloads`` into 1D factors and load vectors with the
oracle's own B-spline code.  Identity geometry (unit square / cube), constant
coefficients: K_s, M_s are built from the parametric 1D factors (eq. space_univ_par_mat).
"""
from __future__ import annotations

import numpy as np

import workloads as wl

from . import bsplines as bs
from .fd import mass_apply


class CubeProblem:
    """1D factors of A on (0,1)^d x (0,T) for a workload with identity geometry."""

    def __init__(self, w: wl.Workload):
        self.w = w
        K, M = bs.space_matrices(w.n_el, w.p)
        self.K1d = [K] * w.d
        self.M1d = [M] * w.d
        self.Wt, self.Mt = bs.time_matrices(w.n_el, w.p, w.T)
        self.Wfull, self.Mfull = bs.time_matrices_full(w.n_el, w.p, w.T)

    def source_sines(self, a, kx, ky, kt):
        """Load vector of f = sum_k a_k sin(kx pi x) sin(ky pi y) sin(kt pi t / T) (d = 2).

        Each term is separable, so its load vector is the Kronecker product of
        three 1D load vectors int sin(k pi x) b_i(x) dx (Gauss, p+3 points per element)."""
        w = self.w
        assert w.d == 2
        xs = bs.open_uniform_knots(w.n_el, w.p)
        xt = bs.open_uniform_knots(w.n_el, w.p, w.T)
        f = np.zeros(w.shape)
        for ak, ax, ay, at in zip(a, kx, ky, kt):
            gx = bs.restrict_space(bs.load(xs, w.p, lambda x: np.sin(ax * np.pi * x)))
            gy = bs.restrict_space(bs.load(xs, w.p, lambda x: np.sin(ay * np.pi * x)))
            gt = bs.restrict_time(bs.load(xt, w.p, lambda t: np.sin(at * np.pi * t / w.T)))
            f += ak * gt[:, None, None] * gy[None, :, None] * gx[None, None, :]
        return f

    def source_smoothed(self, z):
        """f = z x_1 M_1 ... x_d M_d x_{d+1} M_t (one 1D mass product per direction)."""
        if z.ndim == self.w.d + 2:      # batch
            return np.stack([mass_apply(zz, self.Mt, self.M1d) for zz in z])
        return mass_apply(z, self.Mt, self.M1d)

    def source(self, seed=0):
        w = self.w
        if w.source == "sines":
            return self.source_sines(*wl.sine_terms(seed))
        return self.source_smoothed(wl.source_coefficients(w, seed))
