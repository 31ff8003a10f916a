"""The perturbed operator B = A^T A + eps D (Eq. "defB", Sec. 1.2), oracle side.

B is never formed: B x = A^T (A x) + eps (D x), exactly as the paper applies
it.  A is a SciPy CSR matrix; A^T is SciPy's transpose view.  For a symmetric
positive semi-definite A the paper also uses B = A + eps D (the graph
Laplacian experiments of Sec. 5.1), which has the same null space and does not
square the condition number.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def as_scipy(rowptr, colind, vals, m, n) -> sp.csr_matrix:
    return sp.csr_matrix((np.asarray(vals, dtype=np.float64), np.asarray(colind),
                          np.asarray(rowptr)), shape=(m, n))


def apply_b(a: sp.csr_matrix, eps: float, dvec: np.ndarray, x: np.ndarray) -> np.ndarray:
    """B x = A^T (A x) + eps * D x for a vector or an n x k block."""
    x = np.asarray(x, dtype=np.float64)
    y = a @ x
    z = a.T @ y
    if x.ndim == 1:
        return z + eps * dvec * x
    return z + eps * dvec[:, None] * x


def apply_b_sym(a: sp.csr_matrix, eps: float, dvec: np.ndarray, x: np.ndarray) -> np.ndarray:
    """B x = A x + eps * D x (A symmetric positive semi-definite, Sec. 5.1)."""
    x = np.asarray(x, dtype=np.float64)
    z = a @ x
    if x.ndim == 1:
        return z + eps * dvec * x
    return z + eps * dvec[:, None] * x


def operator(op: str):
    """(apply, norm bound of the unperturbed part) for op = 'normal' or 'sym'."""
    if op == "normal":
        return apply_b, norm_upper_bound_ata
    if op == "sym":
        return apply_b_sym, norm_upper_bound_sym
    raise ValueError(op)


def apply_ata(a: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """Unperturbed A^T A x."""
    return a.T @ (a @ x)


def norm_upper_bound_ata(a: sp.csr_matrix) -> float:
    """||A||_1 ||A||_inf, an upper bound on ||A||_2^2 = ||A^T A||_2."""
    absa = abs(a)
    n1 = float(absa.sum(axis=0).max()) if a.nnz else 0.0
    ninf = float(absa.sum(axis=1).max()) if a.nnz else 0.0
    return n1 * ninf


def norm_upper_bound_sym(a: sp.csr_matrix) -> float:
    """||A||_inf, an upper bound on ||A||_2 for a symmetric A (||A||_1 = ||A||_inf)."""
    return float(abs(a).sum(axis=1).max()) if a.nnz else 0.0
