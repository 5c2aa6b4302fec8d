"""MI355X (gfx950) hot path of the space-time isogeometric Galerkin heat-equation
solver: the fast-diagonalization preconditioner A-hat^{-1} inside (flexible) GMRES.

The compute lives in libstig.so (HIP kernels behind a C ABI, include/stig.h);
this package only marshals arguments.  Importing it loads the library and fails
if it has not been built.
"""
import torch  # noqa: F401  (torch's HIP runtime first: libstig then binds to the same one)

from ._lib import LIB_PATH, StigError, lib  # noqa: E402,F401

lib()  # fail loudly at import if the HIP library is missing

from .api import Plan, assemble_1d, load_1d, quadrature, sym_eig  # noqa: E402,F401
