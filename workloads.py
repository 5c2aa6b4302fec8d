"""Seeded synthetic inputs for the space-time heat-equation workloads.

This module holds the *only* code shared by the CPU oracle (``oracle/``) and
the HIP path (``paper_1909_07309_amd``): workload sizes and the random draws
that define each synthetic input.  It holds none of the method's arithmetic:
no B-spline evaluation, no quadrature, no Kronecker algebra.  Each side turns
these draws into a load vector, a system matrix or a solution with its own code.

Sizes follow the paper's degree-of-freedom count (Section 2.2): an open uniform
knot vector of maximal continuity with ``n_el`` elements and degree ``p`` has
``m = n_el + p`` basis functions; homogeneous Dirichlet conditions remove the
first and last spatial function (``n_s = m - 2``) and the initial condition
removes the first time function (``n_t = m - 1``).  Unknowns are stored as a
C-order array ``[t][x_d]...[x_1]`` (x_1 fastest), which is the colexicographic
``vec`` ordering of Section 2.3.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    d: int                 # spatial dimension
    p: int                 # spline degree, same in space and time (Section 5)
    n_el: int              # elements per parametric direction and in time
    T: float = 1.0         # final time
    gamma: float = 1.0     # heat capacity
    nu: float = 1.0        # thermal conductivity
    rtol: float = 1e-8     # GMRES relative residual target
    restart: int = 30      # GMRES(m) restart length
    maxit: int = 300
    nrhs: int = 1
    geometry: str = "cube"  # "cube" (identity map) or "annulus" (quarter annulus)
    source: str = "smoothed_normal"  # or "sines"
    precisions: tuple = ("fp64",)
    note: str = ""

    @property
    def n_s(self) -> int:
        return self.n_el + self.p - 2

    @property
    def n_t(self) -> int:
        return self.n_el + self.p - 1

    @property
    def N_s(self) -> int:
        return self.n_s ** self.d

    @property
    def N(self) -> int:
        return self.N_s * self.n_t

    @property
    def shape(self) -> tuple:
        return (self.n_t,) + (self.n_s,) * self.d


WORKLOADS = {
    # 2D unit square, p=2, 8 elements, f = 10 random tensor-product sines.
    "square_p2_n8": Workload("square_p2_n8", d=2, p=2, n_el=8, rtol=1e-10,
                             source="sines"),
    # 3D unit cube, p=3, 64 elements: 65^3 x 66 = 18,125,250 unknowns.
    "cube_p3_n64": Workload("cube_p3_n64", d=3, p=3, n_el=64, rtol=1e-8,
                            precisions=("fp64", "fp32", "bf16")),
    # 2D quarter annulus (radii 1, 2), p=4, 128 elements, variable
    # conductivity and heat capacity; full space-time CSR system matrix.
    "annulus_p4_n128": Workload("annulus_p4_n128", d=2, p=4, n_el=128,
                                rtol=1e-8, geometry="annulus",
                                precisions=("fp32",)),
    # 3D quarter annulus (radii 1, 2) extruded along z over [0, 1], p=2, 32
    # elements: variable 3D conductivity and heat capacity, full space-time CSR
    # system matrix, 3D geometry-aware preconditioner.  32^3 x 33 = 1,081,344 unknowns.
    "annulus3d_p2_n32": Workload("annulus3d_p2_n32", d=3, p=2, n_el=32, rtol=1e-8,
                                 geometry="annulus3d", precisions=("fp32",)),
    # 3D unit cube, p=3, 48 elements, a batch of 32 right-hand sides.
    "cube_p3_n48_b32": Workload("cube_p3_n48_b32", d=3, p=3, n_el=48,
                                rtol=1e-13, nrhs=32),
}


def scaled(w: Workload, n_el: int, **kw) -> Workload:
    """The same workload at another resolution (for tests that must finish fast)."""
    from dataclasses import replace
    return replace(w, name=f"{w.name}@n{n_el}", n_el=n_el, **kw)


# ---------------------------------------------------------------- random draws

def sine_terms(seed: int = 0, nterms: int = 10):
    """Amplitudes and integer frequencies of f = sum_k a_k sin(kx pi x) sin(ky pi y) sin(kt pi t).

    Draw order: a ~ N(0,1)^nterms, then (kx, ky, kt) ~ U{1..4}^(3 x nterms).
    """
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(nterms)
    k = rng.integers(1, 5, size=(3, nterms))
    return a, k[0], k[1], k[2]


def source_coefficients(w: Workload, seed: int = 0) -> np.ndarray:
    """N(0,1) spline coefficients z, C-order [rhs][t][x_d]..[x_1] (rhs axis only if nrhs > 1).

    The load vector is f = (M_t (x) M_d (x) ... (x) M_1) z, i.e. one 1D mass-matrix
    product per direction; each side computes that product with its own code.
    """
    rng = np.random.default_rng(seed)
    shape = w.shape if w.nrhs == 1 else (w.nrhs,) + w.shape
    return rng.standard_normal(shape)


def adjoint_target(w: Workload, seed: int = 1) -> np.ndarray:
    """Target u* of the loss 0.5 ||u - u*||^2, N(0,1), same layout as the solution batch."""
    rng = np.random.default_rng(seed)
    shape = w.shape if w.nrhs == 1 else (w.nrhs,) + w.shape
    return rng.standard_normal(shape)


def fd_directions(w: Workload, ndir: int = 8, seed: int = 2):
    """Unit-norm random directions in (f, c0) space for central finite differences.

    Returns a list of (df, dc0) pairs; df has the batch layout of f and dc0 has
    layout [rhs][x_d]..[x_1].  The pair is normalised jointly.
    """
    rng = np.random.default_rng(seed)
    fshape = w.shape if w.nrhs == 1 else (w.nrhs,) + w.shape
    cshape = (w.n_s,) * w.d if w.nrhs == 1 else (w.nrhs,) + (w.n_s,) * w.d
    out = []
    for _ in range(ndir):
        df = rng.standard_normal(fshape)
        dc = rng.standard_normal(cshape)
        s = np.sqrt(np.sum(df * df) + np.sum(dc * dc))
        out.append((df / s, dc / s))
    return out


def random_tensor(shape, seed: int) -> np.ndarray:
    """Generic seeded N(0,1) tensor for parity tests."""
    return np.random.default_rng(seed).standard_normal(shape)


# Coefficients of the quarter-annulus workload (problem data, not method).
def annulus_conductivity(x, y):
    """kappa(x) = 1 + 0.5 sin(2 pi x) sin(2 pi y)."""
    return 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)


def annulus3d_conductivity(x, y, z):
    """kappa(x) = 1 + 0.5 sin(2 pi x) sin(2 pi y) cos(pi z)."""
    return 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.cos(np.pi * z)


def annulus_heat_capacity(t):
    """c(t) = 1 + 0.3 cos(pi t)."""
    return 1.0 + 0.3 * np.cos(np.pi * t)
