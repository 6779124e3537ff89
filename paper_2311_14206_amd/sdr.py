"""Python binding of libsdr.so (GMRES-SDR on MI355X).

Argument marshalling only: torch supplies device memory and the stream, every
step of the solver runs in the library's HIP kernels.  The library must have
been built (``python -m paper_2311_14206_amd.build``); importing this module
on a machine without it raises instead of falling back to anything else.
"""

from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdr.so")

SDR_F64, SDR_F32, SDR_C128, SDR_C64 = 0, 1, 2, 3
SDR_OK, SDR_NOT_CONVERGED = 0, 1
ERRORS = {-1: "SDR_EINVAL", -2: "SDR_EPATTERN", -3: "SDR_EDEVICE", -4: "SDR_EBREAKDOWN",
          -5: "SDR_ENOMEM"}


class sdr_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("values", C.c_void_p), ("dtype", C.c_int)]


class sdr_stats(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("iters", C.c_int32), ("matvecs", C.c_int32),
                ("inner_products", C.c_int32), ("sketches", C.c_int32),
                ("res_checks", C.c_int32), ("status", C.c_int32), ("k_eff", C.c_int32),
                ("relres", C.c_double), ("sres", C.c_double), ("safety", C.c_double),
                ("seconds", C.c_double), ("host_eig_seconds", C.c_double),
                ("eps", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class sdr_cycle_record(C.Structure):
    _fields_ = [("j_stop", C.c_int32), ("n_checks", C.c_int32), ("ell", C.c_int32),
                ("k_eff", C.c_int32), ("flags", C.c_int32), ("pad", C.c_int32),
                ("sres", C.c_double), ("res", C.c_double)]


EXPORTS = {
    "sdr_create": (C.c_void_p, [C.POINTER(sdr_csr), C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint64]),
    "sdr_set_option": (C.c_int, [C.c_void_p, C.c_char_p, C.c_double]),
    "sdr_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sdr_solve": (C.c_int, [C.c_void_p, C.POINTER(sdr_csr), C.c_void_p, C.c_void_p, C.c_double,
                            C.POINTER(sdr_stats)]),
    "sdr_update_matrix": (C.c_int, [C.c_void_p, C.POINTER(sdr_csr)]),
    "sdr_solve_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                    C.POINTER(sdr_stats)]),
    "sdr_grad_values": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sdr_get_trace": (C.c_int, [C.c_void_p, C.POINTER(sdr_cycle_record), C.c_int]),
    "sdr_get_recycle": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.POINTER(C.c_int)]),
    "sdr_sketch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "sdr_spmv": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sdr_precond_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sdr_sketch_noalloc": (C.c_int, [C.c_int64, C.c_int, C.c_int, C.c_uint64, C.c_int, C.c_void_p,
                                     C.c_int, C.c_void_p, C.c_void_p]),
    "sdr_get_basis": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sdr_reset": (C.c_int, [C.c_void_p]),
    "sdr_get_step_sres": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int]),
    "sdr_kernel_times": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]),
    "sdr_spmv_layout": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.c_int]),
    "sdr_spmv_const_diagonals": (C.c_int, [C.c_void_p]),
    "sdr_destroy": (None, [C.c_void_p]),
    "sdr_last_error": (C.c_char_p, []),
    "sdr_host_harmonic_ritz": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                         C.c_void_p, C.POINTER(C.c_int)]),
}

_lib = None


def lib():
    """Load libsdr.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2311_14206_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class SDRError(RuntimeError):
    pass


def _check(rc, what):
    if rc < 0:
        msg = lib().sdr_last_error().decode()
        raise SDRError(f"{what}: {ERRORS.get(rc, rc)}: {msg}")
    return rc


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _csr(row_ptr, col_idx, values) -> sdr_csr:
    if values.dtype == torch.float64:
        dt = SDR_F64
    elif values.dtype == torch.complex128:
        dt = SDR_C128
    else:
        raise TypeError("matrix values must be float64 or complex128")
    for t in (row_ptr, col_idx, values):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("CSR arrays must be contiguous device tensors")
    if row_ptr.dtype != torch.int32 or col_idx.dtype != torch.int32:
        raise TypeError("row_ptr and col_idx must be int32")
    return sdr_csr(row_ptr.numel() - 1, col_idx.numel(), _ptr(row_ptr), _ptr(col_idx),
                   _ptr(values), dt)


class SDRSolver:
    """GMRES-SDR handle for one sparse matrix (and its sequence updates).

    row_ptr, col_idx: int32 CUDA tensors; values: float64 or complex128 CUDA
    tensor.  m, k, t, s: Algorithm 1's cycle length, recycle dimension,
    truncation window and sketch size.  Options as in ``sdr_set_option``.
    """

    def __init__(self, row_ptr, col_idx, values, *, m, k, t, s, seed=42, **options):
        self.row_ptr, self.col_idx = row_ptr, col_idx
        self.values = values
        self.n = row_ptr.numel() - 1
        self.dtype = values.dtype
        self.device = values.device
        desc = _csr(row_ptr, col_idx, values)
        torch.cuda.synchronize(self.device)
        h = lib().sdr_create(C.byref(desc), m, k, t, s, C.c_uint64(seed & (2 ** 64 - 1)))
        if not h:
            raise SDRError("sdr_create: " + lib().sdr_last_error().decode())
        self.h = C.c_void_p(h)
        self.m, self.k, self.t, self.s = m, k, t, s
        self.generation = 0  # counts update_matrix calls (autograd checks it)
        for key, v in options.items():
            _check(lib().sdr_set_option(self.h, key.encode(), float(v)), f"option {key}")

    def close(self):
        if getattr(self, "h", None):
            lib().sdr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        _check(lib().sdr_set_stream(self.h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)),
               "sdr_set_stream")

    def _vec(self, v):
        if v.dtype != self.dtype or not v.is_cuda or v.numel() != self.n or not v.is_contiguous():
            raise ValueError(f"expected a contiguous {self.dtype} CUDA vector of length {self.n}")
        return v

    def solve(self, b, x=None, tol=1e-8):
        """Solve A x = b; returns (x, stats dict).  x (optional) is the initial guess."""
        self._vec(b)
        x = torch.zeros_like(b) if x is None else self._vec(x).clone()
        self._stream()
        st = sdr_stats()
        rc = _check(lib().sdr_solve(self.h, None, C.c_void_p(_ptr(b)), C.c_void_p(_ptr(x)),
                                    float(tol), C.byref(st)), "sdr_solve")
        d = st.as_dict()
        d["converged"] = rc == SDR_OK
        return x, d

    def update_matrix(self, values):
        if values.shape != self.values.shape or values.dtype != self.dtype:
            raise ValueError("values must keep the pattern's length and dtype")
        values = values.contiguous()
        self._stream()
        _check(lib().sdr_update_matrix(self.h, C.byref(_csr(self.row_ptr, self.col_idx, values))),
               "sdr_update_matrix")
        self.values = values
        self.generation += 1

    def solve_adjoint(self, g, tol=1e-8):
        self._vec(g)
        lam = torch.zeros_like(g)
        self._stream()
        st = sdr_stats()
        rc = _check(lib().sdr_solve_adjoint(self.h, C.c_void_p(_ptr(g)), C.c_void_p(_ptr(lam)),
                                            float(tol), C.byref(st)), "sdr_solve_adjoint")
        d = st.as_dict()
        d["converged"] = rc == SDR_OK
        return lam, d

    def grad_values(self, lam, x):
        self._vec(lam)
        self._vec(x)
        g = torch.empty_like(self.values)
        self._stream()
        _check(lib().sdr_grad_values(self.h, C.c_void_p(_ptr(lam)), C.c_void_p(_ptr(x)),
                                     C.c_void_p(_ptr(g))), "sdr_grad_values")
        return g

    def reset(self):
        """Drop the recycle space."""
        _check(lib().sdr_reset(self.h), "sdr_reset")

    def kernel_times(self):
        """Event timings since the last call (needs the option kernel_timing=n: every
        n-th Arnoldi step's SpMV and update kernels are timed)."""
        ms = (C.c_double * 8)()
        cnt = (C.c_int64 * 8)()
        _check(lib().sdr_kernel_times(self.h, ms, cnt, 8), "sdr_kernel_times")
        return {"spmv_sketch_ms": ms[0], "update_ms": ms[1], "step_ms": ms[2], "dct_sketch_ms": ms[3],
                "launches": cnt[0], "window_hist": [cnt[3 + i] for i in range(5)]}

    def spmv_layout(self):
        """Diagonal offsets of the basis SpMV's storage ([] for CSR)."""
        off = (C.c_int * 16)()
        nd = _check(lib().sdr_spmv_layout(self.h, off, 16), "sdr_spmv_layout")
        return [off[i] for i in range(nd)]

    def const_diagonals(self):
        """Bit mask of the diagonals (spmv_layout's order) found constant at the
        last packing; their values are passed to the step kernel, not read."""
        return _check(lib().sdr_spmv_const_diagonals(self.h), "sdr_spmv_const_diagonals")

    def trace(self):
        n = _check(lib().sdr_get_trace(self.h, None, 0), "sdr_get_trace")
        buf = (sdr_cycle_record * max(n, 1))()
        lib().sdr_get_trace(self.h, buf, n)
        return [{f: getattr(buf[i], f) for f, _ in sdr_cycle_record._fields_ if f != "pad"}
                for i in range(n)]

    def step_sres(self):
        """Sketched residual by Arnoldi step of the last cycle ([0]: over span(U))."""
        n = _check(lib().sdr_get_step_sres(self.h, None, 0), "sdr_get_step_sres")
        buf = (C.c_double * max(n, 1))()
        lib().sdr_get_step_sres(self.h, buf, n)
        return [buf[i] for i in range(n)]

    def recycle(self):
        k = C.c_int(0)
        _check(lib().sdr_get_recycle(self.h, None, None, None, C.byref(k)), "sdr_get_recycle")
        kk = k.value
        U = torch.empty((kk, self.n), dtype=self.dtype, device=self.device)
        SU = torch.empty((kk, self.s), dtype=self.dtype, device=self.device)
        SAU = torch.empty((kk, self.s), dtype=self.dtype, device=self.device)
        if kk:
            self._stream()
            _check(lib().sdr_get_recycle(self.h, C.c_void_p(_ptr(U)), C.c_void_p(_ptr(SU)),
                                         C.c_void_p(_ptr(SAU)), C.byref(k)), "sdr_get_recycle")
        # column-major storage: rows of these tensors are the columns
        return U.T, SU.T, SAU.T

    def sketch(self, X):
        """S X for X of shape (n,) or (n, c) (column c = X[:, c])."""
        one = X.dim() == 1
        Xc = X.reshape(self.n, -1).T.contiguous()  # columns contiguous
        c = Xc.shape[0]
        Y = torch.empty((c, self.s), dtype=self.dtype, device=self.device)
        self._stream()
        _check(lib().sdr_sketch(self.h, C.c_void_p(_ptr(Xc)), c, C.c_void_p(_ptr(Y))), "sdr_sketch")
        return Y[0] if one else Y.T

    def spmv(self, x):
        self._vec(x)
        y = torch.empty_like(x)
        self._stream()
        _check(lib().sdr_spmv(self.h, C.c_void_p(_ptr(x)), C.c_void_p(_ptr(y))), "sdr_spmv")
        return y

    def precond_apply(self, v):
        """z = M^-1 v for the solver's preconditioner (the identity without one)."""
        self._vec(v)
        z = torch.empty_like(v)
        self._stream()
        _check(lib().sdr_precond_apply(self.h, C.c_void_p(_ptr(v)), C.c_void_p(_ptr(z))), "sdr_precond_apply")
        return z

    def basis(self, ncols):
        """Normalised basis V (n x ncols), H ((m+1) x m) and SV (s x ncols) of the last cycle."""
        import numpy as np
        V = torch.empty((ncols, self.n), dtype=self.dtype, device=self.device)
        npdt = np.complex128 if self.dtype == torch.complex128 else np.float64
        H = np.zeros((self.m, self.m + 1), dtype=npdt)
        SV = np.zeros((ncols, self.s), dtype=npdt)
        self._stream()
        _check(lib().sdr_get_basis(self.h, ncols, C.c_void_p(_ptr(V)), C.c_void_p(H.ctypes.data),
                                   C.c_void_p(SV.ctypes.data)), "sdr_get_basis")
        return V.T, H.T, SV.T


def sketch_noalloc(X, s, seed=42, zeta=8):
    """S X through the allocation-free entry point: X of shape (n,) or (n, c)
    (float64 or complex128 CUDA), no handle.  Queued on torch's current stream;
    the library allocates nothing (the output tensor is torch's)."""
    if X.dtype == torch.float64:
        dt = SDR_F64
    elif X.dtype == torch.complex128:
        dt = SDR_C128
    else:
        raise TypeError("X must be float64 or complex128")
    if not X.is_cuda:
        raise ValueError("X must be a CUDA tensor")
    one = X.dim() == 1
    n = X.shape[0]
    Xc = X.reshape(n, -1).T.contiguous()
    c = Xc.shape[0]
    Y = torch.empty((c, s), dtype=X.dtype, device=X.device)
    st = torch.cuda.current_stream(X.device).cuda_stream
    _check(lib().sdr_sketch_noalloc(n, s, zeta, C.c_uint64(seed & (2 ** 64 - 1)), dt, C.c_void_p(_ptr(Xc)),
                                    c, C.c_void_p(_ptr(Y)), C.c_void_p(st)), "sdr_sketch_noalloc")
    return Y[0] if one else Y.T


def host_harmonic_ritz(R, Cm, s, k, is_complex):
    """Host-only harmonic-Ritz step of the library (numpy in, numpy out)."""
    import numpy as np
    l0 = R.shape[0]
    dt = np.complex128 if is_complex else np.float64
    Rf = np.asfortranarray(R, dtype=dt)
    Cf = np.asfortranarray(Cm, dtype=dt)
    G = np.zeros((l0, k + 1), dtype=dt, order="F")
    ell = C.c_int(0)
    keff = _check(lib().sdr_host_harmonic_ritz(l0, C.c_void_p(Rf.ctypes.data), C.c_void_p(Cf.ctypes.data),
                                               s, k, int(is_complex), C.c_void_p(G.ctypes.data),
                                               C.byref(ell)), "sdr_host_harmonic_ritz")
    return G[:, :keff], ell.value, keff
