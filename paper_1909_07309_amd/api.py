"""Thin Python binding of libstig (argument marshalling only).

Device buffers are PyTorch CUDA (HIP) tensors in float64; every operation
runs in libstig's kernels on torch's current stream.  Names follow the C ABI.
PyTorch allocates all device memory the calls need: before each call the plan's
workspace tensor is grown to stig_workspace_bytes for that call and handed to
the library (stig_set_workspace), which allocates nothing in the call itself.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from ._lib import PREC, StigInfo, check, dptr, lib


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, n: int, name: str) -> C.c_void_p:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return C.c_void_p(t.data_ptr())


class Plan:
    """A libstig plan for d spatial dims with sizes n_s (direction order 1..d), n_t time unknowns."""

    def __init__(self, n_s, n_t, p_s, p_t):
        n_s = [int(v) for v in n_s]
        self.d = len(n_s)
        self.n_s, self.n_t, self.p_s, self.p_t = n_s, int(n_t), int(p_s), int(p_t)
        self.N_s = int(np.prod(n_s))
        self.N = self.N_s * self.n_t
        # tensor shape [t][x_d]..[x_1]
        self.shape = (self.n_t,) + tuple(reversed(n_s))
        h = C.c_void_p()
        arr = (C.c_int * self.d)(*n_s)
        check(lib().stig_plan_create(C.byref(h), self.d, arr, self.n_t, self.p_s, self.p_t,
                                     _stream()))
        self._h = h
        self._keep = {}
        self._ws = None  # caller-owned workspace (uint8 device tensor)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().stig_plan_destroy(h)
            except Exception:  # interpreter shutdown: module globals already cleared
                pass
            self._h = None

    def _sync_stream(self):
        check(lib().stig_set_stream(self._h, _stream()))

    def workspace_bytes(self, nrhs=1, restart=0, prec="fp64", flexible=False):
        """stig_workspace_bytes: device bytes the calls with nrhs right-hand sides need
        (restart > 0: GMRES with that restart length as well)."""
        return int(lib().stig_workspace_bytes(self._h, int(restart), int(bool(flexible)),
                                              PREC[prec], int(nrhs)))

    def _ensure_workspace(self, need, device):
        """Grow the workspace tensor to `need` bytes (torch allocation, outside the library
        calls) and hand it to the plan."""
        if self._ws is not None and self._ws.numel() >= need and self._ws.device == device:
            return
        self._ws = None  # release the old one first
        self._ws = torch.empty(max(int(need), 256), dtype=torch.uint8, device=device)
        check(lib().stig_set_workspace(self._h, C.c_void_p(self._ws.data_ptr()),
                                       self._ws.numel()))

    def set_workspace(self, ws):
        """Use a caller-allocated uint8 device tensor as the workspace (None detaches)."""
        if ws is None:
            self._ws = None
            check(lib().stig_set_workspace(self._h, None, 0))
            return
        assert ws.is_cuda and ws.dtype == torch.uint8 and ws.is_contiguous()
        self._ws = ws
        check(lib().stig_set_workspace(self._h, C.c_void_p(ws.data_ptr()), ws.numel()))

    def _nrhs(self, t):
        n = t.numel()
        if n % self.N:
            raise ValueError(f"tensor size {n} is not a multiple of N = {self.N}")
        return n // self.N

    def setup_1d_pencils(self, K1d, M1d, Wt, Mt, gamma=1.0, nu=1.0):
        mats = [np.ascontiguousarray(m, dtype=np.float64) for m in list(K1d) + list(M1d)]
        self._host = mats
        Ks = (C.POINTER(C.c_double) * self.d)(*[dptr(m) for m in mats[:self.d]])
        Ms = (C.POINTER(C.c_double) * self.d)(*[dptr(m) for m in mats[self.d:]])
        Wt = np.ascontiguousarray(Wt, dtype=np.float64)
        Mt = np.ascontiguousarray(Mt, dtype=np.float64)
        for l in range(self.d):
            if mats[l].shape != (self.n_s[l], self.n_s[l]):
                raise ValueError("spatial factor has the wrong shape")
        if Wt.shape != (self.n_t, self.n_t) or Mt.shape != (self.n_t, self.n_t):
            raise ValueError("time factor has the wrong shape")
        self._sync_stream()
        check(lib().stig_setup_1d_pencils(self._h, Ks, Ms, dptr(Wt), dptr(Mt), float(gamma),
                                          float(nu)))

    def set_diag_scaling(self, D):
        self._sync_stream()
        if D is None:
            check(lib().stig_set_diag_scaling(self._h, None))
        else:
            check(lib().stig_set_diag_scaling(self._h, _dev(D, self.N, "D")))

    def set_A_csr(self, rowptr, col, val):
        self._sync_stream()
        if rowptr is None:
            self._keep.pop("csr", None)
            check(lib().stig_set_A_csr(self._h, None, None, None, 0))
            return
        assert rowptr.dtype == torch.int64 and col.dtype == torch.int32 and val.dtype == torch.float64
        assert rowptr.is_cuda and col.is_cuda and val.is_cuda
        assert rowptr.numel() == self.N + 1 and col.numel() == val.numel()
        self._keep["csr"] = (rowptr, col, val)
        check(lib().stig_set_A_csr(self._h, C.c_void_p(rowptr.data_ptr()),
                                   C.c_void_p(col.data_ptr()), C.c_void_p(val.data_ptr()),
                                   int(val.numel())))

    def set_spatial_factors(self, space_csr):
        """Matvec with sparse spatial factors: A = gamma W_t (x) M_s + nu M_t (x) K_s from a
        host spatial CSR (rowptr, col, valK, valM), as `assemble_2d` / `assemble_3d` return
        it; None removes them."""
        self._sync_stream()
        if space_csr is None:
            check(lib().stig_set_spatial_factors(self._h, None, None, None, None))
            return
        rp, col, vK, vM = space_csr
        rp = np.ascontiguousarray(rp, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        vK = np.ascontiguousarray(vK, dtype=np.float64)
        vM = np.ascontiguousarray(vM, dtype=np.float64)
        assert rp.size == self.N_s + 1 and col.size == vK.size == vM.size == int(rp[-1])
        check(lib().stig_set_spatial_factors(self._h, rp.ctypes.data_as(C.c_void_p),
                                             col.ctypes.data_as(C.c_void_p), dptr(vM), dptr(vK)))
        self._keep.pop("csr", None)

    def apply_Pinv(self, r, s=None, transpose=False, prec="fp64"):
        nrhs = self._nrhs(r)
        if s is None:
            s = torch.empty_like(r)
        self._ensure_workspace(self.workspace_bytes(nrhs, 0, prec), r.device)
        self._sync_stream()
        check(lib().stig_apply_Pinv(self._h, _dev(r, nrhs * self.N, "r"),
                                    _dev(s, nrhs * self.N, "s"), nrhs, int(bool(transpose)),
                                    PREC[prec]))
        return s

    def matvec_A(self, x, y=None, transpose=False):
        nrhs = self._nrhs(x)
        if y is None:
            y = torch.empty_like(x)
        self._ensure_workspace(self.workspace_bytes(nrhs), x.device)
        self._sync_stream()
        check(lib().stig_matvec_A(self._h, _dev(x, nrhs * self.N, "x"),
                                  _dev(y, nrhs * self.N, "y"), nrhs, int(bool(transpose))))
        return y

    def apply_mass(self, z, y=None):
        nrhs = self._nrhs(z)
        if y is None:
            y = torch.empty_like(z)
        self._ensure_workspace(self.workspace_bytes(nrhs), z.device)
        self._sync_stream()
        check(lib().stig_apply_mass(self._h, _dev(z, nrhs * self.N, "z"),
                                    _dev(y, nrhs * self.N, "y"), nrhs))
        return y

    def lift_adjoint(self, a_col, b_col, lam, g=None):
        nrhs = self._nrhs(lam)
        a_col = np.ascontiguousarray(a_col, dtype=np.float64)
        b_col = np.ascontiguousarray(b_col, dtype=np.float64)
        assert a_col.shape == (self.n_t,) and b_col.shape == (self.n_t,)
        if g is None:
            g = torch.empty((nrhs,) + self.shape[1:], dtype=torch.float64, device=lam.device)
        self._ensure_workspace(self.workspace_bytes(nrhs), lam.device)
        self._sync_stream()
        check(lib().stig_lift_adjoint(self._h, dptr(a_col), dptr(b_col),
                                      _dev(lam, nrhs * self.N, "lam"),
                                      _dev(g, nrhs * self.N_s, "g"), nrhs))
        return g

    def lift_apply(self, a_col, b_col, c0, f=None, y=None):
        """Initial-datum lifting, c0 of shape [rhs][x_d]..[x_1]: y = A_{I,0} c0, or
        y = f - A_{I,0} c0 when f is given (the right-hand side of the kept unknowns)."""
        nrhs = c0.numel() // self.N_s
        a_col = np.ascontiguousarray(a_col, dtype=np.float64)
        b_col = np.ascontiguousarray(b_col, dtype=np.float64)
        assert a_col.shape == (self.n_t,) and b_col.shape == (self.n_t,)
        if y is None:
            y = torch.empty((nrhs,) + self.shape, dtype=torch.float64, device=c0.device)
        fp = None if f is None else _dev(f, nrhs * self.N, "f")
        self._ensure_workspace(self.workspace_bytes(nrhs), c0.device)
        self._sync_stream()
        check(lib().stig_lift_apply(self._h, dptr(a_col), dptr(b_col),
                                    _dev(c0, nrhs * self.N_s, "c0"), fp,
                                    _dev(y, nrhs * self.N, "y"), nrhs))
        return y

    def gmres_solve(self, f, u=None, restart=30, rtol=1e-8, maxit=300, flexible=False,
                    transpose=False, prec="fp64", allow_not_converged=False):
        nrhs = self._nrhs(f)
        if u is None:
            u = torch.zeros_like(f)
        info = StigInfo()
        # lockstep first cycle for as many right-hand sides as fit in 60 % of the
        # free device memory (plus the current workspace)
        nb = min(nrhs, 64)
        need = self.workspace_bytes(nb, restart, prec, flexible)
        if nb > 1:
            free_b, _ = torch.cuda.mem_get_info(f.device)
            budget = 0.6 * (free_b + (self._ws.numel() if self._ws is not None else 0))
            while nb > 1 and need > budget:
                nb -= 1
                need = self.workspace_bytes(nb, restart, prec, flexible)
        self._ensure_workspace(need, f.device)
        self._sync_stream()
        code = lib().stig_gmres_solve(self._h, _dev(f, nrhs * self.N, "f"),
                                      _dev(u, nrhs * self.N, "u"), nrhs, int(restart),
                                      float(rtol), int(maxit), int(bool(flexible)),
                                      int(bool(transpose)), PREC[prec], C.byref(info))
        check(code, allow_warning=allow_not_converged)
        return u, {"iters": info.iters, "restarts": info.restarts,
                   "relres_true": info.relres_true, "relres_est": info.relres_est,
                   "t_solve_ms": info.t_solve_ms, "converged": code == 0}

    KERNEL_KINDS = ("mode_gemm", "time_solve", "band_pass", "krylov", "csr", "plane_gemm")

    OPTIONS = {"plane_fusion": 0, "time_kernel": 1, "parity_split": 2}
    TIME_KERNELS = {"right_looking": 0, "left_looking": 1, "generic": 2, "right_looking_stored": 3,
                    "arrowhead": 4}

    def set_option(self, name, value):
        """Kernel choices of apply_Pinv (same results up to rounding order):
        plane_fusion (bool, default True), time_kernel ("right_looking" default,
        "right_looking_stored", "left_looking", "generic", "arrowhead"), parity_split (bool,
        default True)."""
        if name == "time_kernel" and isinstance(value, str):
            value = self.TIME_KERNELS[value]
        check(lib().stig_set_option(self._h, self.OPTIONS[name], int(value)))

    def set_plane_fusion(self, on=True):
        self.set_option("plane_fusion", bool(on))

    def profile_enable(self, on=True):
        self._sync_stream()
        check(lib().stig_profile_enable(self._h, int(bool(on))))

    def profile_reset(self):
        check(lib().stig_profile_reset(self._h))

    def profile(self):
        """{kind: (total_ms, algorithmic_bytes, launches)} for the kernels timed so far."""
        out = {}
        for k, name in enumerate(self.KERNEL_KINDS):
            ms, by, n = C.c_double(), C.c_double(), C.c_longlong()
            check(lib().stig_profile_get(self._h, k, C.byref(ms), C.byref(by), C.byref(n)))
            out[name] = (ms.value, by.value, n.value)
        return out

    def set_diag_scaling_kron(self, dMs, dKs):
        dMs = np.ascontiguousarray(dMs, dtype=np.float64).ravel()
        dKs = np.ascontiguousarray(dKs, dtype=np.float64).ravel()
        assert dMs.size == self.N_s and dKs.size == self.N_s
        self._sync_stream()
        check(lib().stig_set_diag_scaling_kron(self._h, dptr(dMs), dptr(dKs)))

    def kron_csr(self, space_csr, Wt, Mt, device="cuda"):
        """Build W (x) M_s + Mt (x) K_s as a device CSR (int64 rowptr, int32 col, f64 val) from
        a host spatial CSR (rowptr, col, valK, valM) and dense host time factors."""
        rp2, c2, vK, vM = space_csr
        Ns = rp2.size - 1
        rowptr = np.empty(self.n_t * Ns + 1, dtype=np.int64)
        check(lib().stig_kron_csr_rowptr(self.n_t, self.p_t, Ns, rp2.ctypes.data_as(C.c_void_p),
                                         rowptr.ctypes.data_as(C.c_void_p)))
        nnz = int(rowptr[-1])
        d_rowptr = torch.from_numpy(rowptr).to(device)
        d_col = torch.empty(nnz, dtype=torch.int32, device=device)
        d_val = torch.empty(nnz, dtype=torch.float64, device=device)
        t = [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in (rp2, c2, vM, vK)]
        Wt = np.ascontiguousarray(Wt, dtype=np.float64)
        Mt = np.ascontiguousarray(Mt, dtype=np.float64)
        self._sync_stream()
        check(lib().stig_kron_csr_fill(self._h, C.c_void_p(d_rowptr.data_ptr()),
                                       C.c_void_p(d_col.data_ptr()), C.c_void_p(d_val.data_ptr()),
                                       *[C.c_void_p(x.data_ptr()) for x in t], dptr(Wt), dptr(Mt)))
        return d_rowptr, d_col, d_val

    def device_bytes(self):
        return int(lib().stig_plan_device_bytes(self._h))


# ----------------------------------------------------------- 1D assembly (host)

def quadrature(n_el, nq, length=1.0):
    x = np.empty(n_el * nq)
    w = np.empty(n_el * nq)
    check(lib().stig_quadrature(n_el, nq, float(length), dptr(x), dptr(w)))
    return x, w


def assemble_1d(n_el, p, kind, length=1.0, weight=None, nq=0):
    """Full (unrestricted) m x m 1D matrix; kind in {'mass', 'stiffness', 'advection'}."""
    k = {"mass": 0, "stiffness": 1, "advection": 2}[kind]
    m = n_el + p
    out = np.empty((m, m))
    wp = None
    if weight is not None:
        weight = np.ascontiguousarray(weight, dtype=np.float64)
        wp = dptr(weight)
    check(lib().stig_assemble_1d(n_el, p, float(length), k, wp, int(nq), dptr(out)))
    return out


def load_1d(n_el, p, fvals, nq, length=1.0):
    fvals = np.ascontiguousarray(fvals, dtype=np.float64)
    out = np.empty(n_el + p)
    check(lib().stig_load_1d(n_el, p, float(length), dptr(fvals), int(nq), dptr(out)))
    return out


def assemble_2d(n_el, p, nq, c11, c22, c33):
    """Host CSR (rowptr int64, col int32, valK, valM) of the 2D parametric stiffness / mass."""
    c11, c22, c33 = (np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (c11, c22, c33))
    nnz = C.c_int64()
    check(lib().stig_assemble_2d(n_el, p, nq, None, None, None, None, None, None, None,
                                 C.byref(nnz)))
    n = n_el + p - 2
    rowptr = np.empty(n * n + 1, dtype=np.int64)
    col = np.empty(nnz.value, dtype=np.int32)
    valK = np.empty(nnz.value)
    valM = np.empty(nnz.value)
    check(lib().stig_assemble_2d(n_el, p, nq, dptr(c11), dptr(c22), dptr(c33),
                                 rowptr.ctypes.data_as(C.c_void_p), col.ctypes.data_as(C.c_void_p),
                                 dptr(valK), dptr(valM), C.byref(nnz)))
    return rowptr, col, valK, valM


def separate_2d(C11, C22, C33):
    """(phi1, phi2, Phi1, Phi2) from element-midpoint samples shaped [e2][e1]."""
    C11, C22, C33 = (np.ascontiguousarray(a, dtype=np.float64) for a in (C11, C22, C33))
    n2, n1 = C33.shape
    out = [np.empty(n1), np.empty(n2), np.empty(n1), np.empty(n2)]
    check(lib().stig_separate_2d(n1, n2, dptr(C11), dptr(C22), dptr(C33), *[dptr(o) for o in out]))
    return tuple(out)


def assemble_3d(n_el, p, nq, c11, c22, c33, c00):
    """Host CSR (rowptr int64, col int32, valK, valM) of the 3D parametric stiffness / mass."""
    cs = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (c11, c22, c33, c00)]
    nnz = C.c_int64()
    check(lib().stig_assemble_3d(n_el, p, nq, None, None, None, None, None, None, None, None,
                                 C.byref(nnz)))
    n = n_el + p - 2
    rowptr = np.empty(n ** 3 + 1, dtype=np.int64)
    col = np.empty(nnz.value, dtype=np.int32)
    valK = np.empty(nnz.value)
    valM = np.empty(nnz.value)
    check(lib().stig_assemble_3d(n_el, p, nq, *[dptr(c) for c in cs],
                                 rowptr.ctypes.data_as(C.c_void_p), col.ctypes.data_as(C.c_void_p),
                                 dptr(valK), dptr(valM), C.byref(nnz)))
    return rowptr, col, valK, valM


def separate_3d(C11, C22, C33, C00):
    """(phi1, phi2, phi3, Phi1, Phi2, Phi3) from element-midpoint samples shaped [e3][e2][e1]."""
    Cs = [np.ascontiguousarray(a, dtype=np.float64) for a in (C11, C22, C33, C00)]
    n3, n2, n1 = Cs[3].shape
    out = [np.empty(n1), np.empty(n2), np.empty(n3), np.empty(n1), np.empty(n2), np.empty(n3)]
    check(lib().stig_separate_3d(n1, n2, n3, *[dptr(c) for c in Cs], *[dptr(o) for o in out]))
    return tuple(out)


def sym_eig(K, M):
    K = np.ascontiguousarray(K, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    n = K.shape[0]
    U = np.empty((n, n))
    lam = np.empty(n)
    check(lib().stig_sym_eig(n, dptr(K), dptr(M), dptr(U), dptr(lam)))
    return lam, U


def split_eig(K, M):
    """Eigenbasis of a persymmetric pencil, even modes first (see stig_split_eig)."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    n = K.shape[0]
    U = np.empty((n, n))
    lam = np.empty(n)
    check(lib().stig_split_eig(n, dptr(K), dptr(M), dptr(U), dptr(lam)))
    return lam, U


def time_arrowhead(W, M):
    """(U, D, nzero): real block form of the arrowhead factorization (stig_time_arrowhead)."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    n = W.shape[0]
    U = np.empty((n, n))
    D = np.empty((n, n))
    nz = C.c_int()
    check(lib().stig_time_arrowhead(n, dptr(W), dptr(M), dptr(U), dptr(D), C.byref(nz)))
    return U, D, nz.value
