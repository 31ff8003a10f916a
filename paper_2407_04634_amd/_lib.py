"""ctypes binding of libnullspace.so (include/nullspace.h).

Argument marshalling only: every numerical step runs in the HIP library.
PyTorch provides device memory (tensors' data pointers) and the stream.  The
library is loaded only after ``import torch`` so that the HIP runtime torch
brings is the one the library binds to.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnullspace.so")

NSP_OK, NSP_ERR_ARG, NSP_ERR_HIP, NSP_ERR_NOMEM, NSP_ERR_STATE, NSP_ERR_NOCONV, \
    NSP_ERR_BREAKDOWN, NSP_ERR_NONFINITE = range(8)
STATUS_NAMES = ["NSP_OK", "NSP_ERR_ARG", "NSP_ERR_HIP", "NSP_ERR_NOMEM", "NSP_ERR_STATE",
                "NSP_ERR_NOCONV", "NSP_ERR_BREAKDOWN", "NSP_ERR_NONFINITE"]
PREC_FP64, PREC_MIXED = 0, 1
OP_NORMAL, OP_SYM = 0, 1
PRECOND_NONE, PRECOND_JACOBI, PRECOND_IC = 0, 1, 2


class NspError(RuntimeError):
    def __init__(self, status: int, msg: str):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_double),
        ("d", ctypes.c_int32),
        ("max_dim", ctypes.c_int32),
        ("max_matvec", ctypes.c_int64),
        ("ro_tol", ctypes.c_double),
        ("prec", ctypes.c_int32),
        ("refine", ctypes.c_int32),
        ("tol_rel_resid", ctypes.c_double),
        ("tol_abs_resid", ctypes.c_double),
        ("tol_angle", ctypes.c_double),
        ("max_refine_iter", ctypes.c_int64),
        ("max_cycles", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("reorder", ctypes.c_int32),
        ("op", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("ic_droptol", ctypes.c_double),
        ("ic_diagcomp", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("nullity", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("cycles", ctypes.c_int32),
        ("matvecs", ctypes.c_int64),
        ("reorths", ctypes.c_int64),
        ("refine_iters", ctypes.c_int64),
        ("norm_b", ctypes.c_double),
        ("theta_last", ctypes.c_double),
        ("theta_next", ctypes.c_double),
        ("rel_resid_fro", ctypes.c_double),
        ("orth_err_fro", ctypes.c_double),
        ("t_total_s", ctypes.c_double),
        ("t_lanczos_s", ctypes.c_double),
        ("t_restart_s", ctypes.c_double),
        ("t_refine_s", ctypes.c_double),
        ("t_spmv_a_us", ctypes.c_double),
        ("t_spmv_at_us", ctypes.c_double),
        ("spmv_samples", ctypes.c_int64),
        ("ro_tn_ms", ctypes.c_double),
        ("ro_tn_bytes", ctypes.c_double),
        ("ro_nn_ms", ctypes.c_double),
        ("ro_nn_bytes", ctypes.c_double),
        ("ro_idle_ms", ctypes.c_double),
        ("ro_samples", ctypes.c_int64),
        ("ro_active", ctypes.c_int64),
        ("refine_defl", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


EXPORTS = ["nsp_default_params", "nullspace_init", "apply_op", "lanczos_run", "nullspace_nullity",
           "extract_basis", "nullspace_ritz_values", "nullspace_ritz_eig", "nullspace_ritz_eig_blocks",
           "backward",
           "nullspace_destroy", "nullspace_last_error", "nullspace_locality_order",
           "nullspace_update_values", "nullspace_cycle_times", "nullspace_ritz_residuals",
           "apply_op_noalloc"]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2407_04634_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.nsp_default_params.argtypes = [ctypes.POINTER(Params)]
    lib.nsp_default_params.restype = None
    lib.nullspace_init.argtypes = [ctypes.POINTER(vp), i64, i64, i64, vp, vp, vp, vp, vp,
                                   ctypes.POINTER(Params), vp]
    lib.apply_op.argtypes = [vp, vp, i64, vp, i64, i32]
    lib.apply_op_noalloc.argtypes = [vp, vp, i64, vp, i64, i32]
    lib.lanczos_run.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.nullspace_nullity.argtypes = [vp, ctypes.POINTER(i32)]
    lib.extract_basis.argtypes = [vp, vp, i64]
    lib.nullspace_ritz_values.argtypes = [vp, ctypes.POINTER(dbl), i32, ctypes.POINTER(i32)]
    lib.nullspace_ritz_eig.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp]
    lib.nullspace_ritz_eig_blocks.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]
    lib.backward.argtypes = [vp, vp, i64, vp, dbl, i64, ctypes.POINTER(i64)]
    lib.nullspace_destroy.argtypes = [vp]
    lib.nullspace_destroy.restype = None
    lib.nullspace_last_error.argtypes = []
    lib.nullspace_last_error.restype = ctypes.c_char_p
    lib.nullspace_locality_order.argtypes = [i64, i64, vp, vp, vp, vp]
    lib.nullspace_update_values.argtypes = [vp, vp]
    lib.nullspace_cycle_times.argtypes = [vp, ctypes.POINTER(dbl), i32, ctypes.POINTER(i32)]
    lib.nullspace_ritz_residuals.argtypes = [vp, ctypes.POINTER(dbl), i32, ctypes.POINTER(i32)]
    for name in ("nullspace_init", "apply_op", "apply_op_noalloc", "lanczos_run", "nullspace_nullity", "extract_basis",
                 "nullspace_ritz_values", "nullspace_ritz_eig", "nullspace_ritz_eig_blocks", "backward",
                 "nullspace_locality_order", "nullspace_update_values", "nullspace_cycle_times",
                 "nullspace_ritz_residuals"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int, allow=(NSP_OK,)):
    if status not in allow:
        raise NspError(status, load().nullspace_last_error().decode())
    return status


def default_params(**overrides) -> Params:
    p = Params()
    load().nsp_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def locality_order(rowptr, colind, m: int, n: int):
    """Host-side locality order of a CSR pattern (numpy int64 rowptr, int32 colind).

    Returns (row_order, col_order): the caller's row / column at each position.
    """
    import numpy as np

    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(colind, dtype=np.int32)
    ro = np.empty(m, dtype=np.int32)
    co = np.empty(n, dtype=np.int32)
    _check(load().nullspace_locality_order(int(m), int(n), rp.ctypes.data, ci.ctypes.data if ci.size else None,
                                           ro.ctypes.data, co.ctypes.data))
    return ro, co


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous CUDA tensor of dtype {dtype}")
    return t


class Context:
    """Owns one nsp_ctx.  Keeps references to the tensors the context reads."""

    def __init__(self, rowptr, colind, vals, m: int, n: int, D=None, Omega=None, params=None, **kw):
        lib = load()
        self._keep = (_dev(rowptr, torch.int64, "rowptr"), _dev(colind, torch.int32, "colind"),
                      _dev(vals, torch.float64, "vals"))
        p = params if params is not None else default_params(**kw)
        if D is not None:
            _dev(D, torch.float64, "D")
        om_cm = None
        if Omega is not None:
            if Omega.dtype != torch.float64 or not Omega.is_cuda or Omega.shape[0] != n:
                raise TypeError("Omega must be an n x d CUDA float64 tensor")
            om_cm = Omega.reshape(n, -1).t().contiguous()  # d x n row-major == n x d column-major
        self.m, self.n, self.nnz = int(m), int(n), int(vals.numel())
        self.params = p
        h = ctypes.c_void_p()
        st = lib.nullspace_init(ctypes.byref(h), self.m, self.n, self.nnz, _ptr(rowptr), _ptr(colind),
                                _ptr(vals), _ptr(D), _ptr(om_cm), ctypes.byref(p),
                                _stream_handle())
        _check(st)
        self._h = h

    # -- calls named as in the C ABI -------------------------------------
    def apply_op(self, x: torch.Tensor) -> torch.Tensor:
        """Y = B X for X (n x k) float64 CUDA (any layout; passed column-major)."""
        squeeze = x.dim() == 1
        xc = x.reshape(self.n, -1).t().contiguous()  # k x n row-major == n x k column-major
        k = xc.shape[0]
        y = torch.empty_like(xc)
        _check(load().apply_op(self._h, _ptr(xc), self.n, _ptr(y), self.n, k))
        y = y.t()
        return y.reshape(-1) if squeeze else y

    def apply_op_noalloc(self, x: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """Y = B X into ``out`` through the allocation-free entry point.

        ``x`` and ``out`` are n x k float64 CUDA tensors in column-major layout
        (e.g. ``t.t()`` of a contiguous k x n tensor); the library allocates
        nothing.
        """
        for t, name in ((x, "x"), (out, "out")):
            if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.shape[0] == self.n
                    and t.stride(0) == 1 and t.stride(1) >= self.n):
                raise TypeError(f"{name} must be an n x k column-major float64 CUDA tensor")
        if out.shape[1] != x.shape[1]:
            raise ValueError("x and out must have the same number of columns")
        _check(load().apply_op_noalloc(self._h, _ptr(x), x.stride(1), _ptr(out), out.stride(1),
                                       int(x.shape[1])))
        return out

    def lanczos_run(self, allow_noconv: bool = False) -> dict:
        st = Stats()
        status = load().lanczos_run(self._h, ctypes.byref(st))
        _check(status, (NSP_OK, NSP_ERR_NOCONV) if allow_noconv else (NSP_OK,))
        d = st.as_dict()
        d["status"] = STATUS_NAMES[status]
        return d

    def nullity(self) -> int:
        v = ctypes.c_int32()
        _check(load().nullspace_nullity(self._h, ctypes.byref(v)))
        return int(v.value)

    def extract_basis(self) -> torch.Tensor:
        nul = self.nullity()
        out = torch.empty((nul, self.n), dtype=torch.float64, device="cuda")  # column-major n x N
        _check(load().extract_basis(self._h, _ptr(out), self.n))
        return out.t()

    def ritz_values(self, cap: int = 1 << 14):
        buf = (ctypes.c_double * cap)()
        cnt = ctypes.c_int32()
        _check(load().nullspace_ritz_values(self._h, buf, cap, ctypes.byref(cnt)))
        return [buf[i] for i in range(cnt.value)]

    def ritz_residuals(self, cap: int = 1 << 14):
        """Residual norms ||Gamma_ell V_Z(last d rows, i)|| of the last Ritz pairs."""
        buf = (ctypes.c_double * cap)()
        cnt = ctypes.c_int32()
        _check(load().nullspace_ritz_residuals(self._h, buf, cap, ctypes.byref(cnt)))
        return [buf[i] for i in range(cnt.value)]

    def cycle_times(self, cap: int = 1 << 16):
        """Wall time (s) of each restart cycle of the last lanczos_run."""
        buf = (ctypes.c_double * cap)()
        cnt = ctypes.c_int32()
        _check(load().nullspace_cycle_times(self._h, buf, cap, ctypes.byref(cnt)))
        return [buf[i] for i in range(cnt.value)]

    def ritz_eig(self, theta, f, alpha, beta):
        """Eigenpairs of the restart matrix (d = 1) from device float64 vectors."""
        kk, m = int(theta.numel()), int(alpha.numel())
        k = kk + m
        ev = torch.empty(k, dtype=torch.float64, device="cuda")
        vec = torch.empty((k, k), dtype=torch.float64, device="cuda")  # column-major as k x k^T
        _check(load().nullspace_ritz_eig(self._h, k, kk, _ptr(theta) if kk else None,
                                         _ptr(f) if kk else None, _ptr(alpha), _ptr(beta), _ptr(ev),
                                         _ptr(vec)))
        return ev, vec.t()

    def ritz_eig_blocks(self, d, theta, f, xi, gam):
        """Eigenpairs of the restart matrix for block size d.  theta [kk], f (kk x d
        as the column-major d x kk matrix's transpose), xi and gam as (nblocks, d, d)
        tensors holding each block transposed (column-major), all device float64."""
        kk, nbk = int(theta.numel()), int(xi.shape[0])
        k = kk + nbk * d
        ev = torch.empty(k, dtype=torch.float64, device="cuda")
        vec = torch.empty((k, k), dtype=torch.float64, device="cuda")
        _check(load().nullspace_ritz_eig_blocks(self._h, k, d, kk, _ptr(theta) if kk else None,
                                                _ptr(f) if kk else None, _ptr(xi),
                                                _ptr(gam) if nbk > 1 else None, _ptr(ev), _ptr(vec)))
        return ev, vec.t()

    def update_values(self, vals: torch.Tensor):
        """New values of A (same pattern, caller's CSR order); the basis is dropped."""
        _dev(vals, torch.float64, "vals")
        if vals.numel() != self.nnz:
            raise ValueError("vals must hold nnz values")
        _check(load().nullspace_update_values(self._h, _ptr(vals)))

    def backward(self, dldv: torch.Tensor, tol: float = 1e-12, max_iter: int = 10 ** 6):
        """grad w.r.t. A's stored values for dL/dV (n x N), via the library's CG + SDDMM."""
        g = dldv.t().contiguous()  # column-major n x N
        grad = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        it = ctypes.c_int64()
        _check(load().backward(self._h, _ptr(g), self.n, _ptr(grad), float(tol), int(max_iter),
                               ctypes.byref(it)))
        return grad, int(it.value)

    def close(self):
        if getattr(self, "_h", None):
            load().nullspace_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
