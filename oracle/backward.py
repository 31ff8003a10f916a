"""Gradient of a loss on the null projector with respect to A's nonzeros (oracle).

Test infrastructure only.

Setting.  P(A) = V V^T is the orthogonal projector onto the span of the N
right singular vectors of A belonging to its N smallest singular values (the
null space when A has nullity N; Sec. 2.3 relates such projectors to the
principal angles).  With N held fixed P is smooth wherever sigma_{N+1} > 0,
and first-order perturbation theory of the SVD gives

    dP = -A^+ dA P - P dA^T (A^+)^T .

For a loss L(P) with symmetric gradient G_s = sym(dL/dP),

    dL/dA = -2 (A^+)^T G_s P = -2 (A (A^T A)^+ G_s V) V^T = -2 U V^T,
    U = A W,   W = (A^T A)^+ G_s V = (A^T A)^+ (I - P) G_s V,

so the gradient of the stored value a_p at (i, j) is -2 <U_i, V_j>, a sampled
dense-dense product (SDDMM) on A's sparsity pattern.  If the caller holds
dL/dV instead, dL/dV = 2 G_s V for a loss that depends on V only through P.

Three independent routes:
  dense_grad        -- the closed form with a dense pseudo-inverse (tiny A)
  fd_grad           -- central finite differences of the loss itself
  cg_sddmm_grad     -- CG on A^T A restricted to range(A^T), then SDDMM (large A)
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def fixed_rank_projector(a_dense: np.ndarray, nullity: int) -> np.ndarray:
    """V (n x N): right singular vectors of the N smallest singular values."""
    _, _, vt = np.linalg.svd(a_dense, full_matrices=True)
    return vt[vt.shape[0] - nullity:].T


def loss_pxf(v: np.ndarray, x: np.ndarray) -> float:
    """L = ||P X||_F^2 = ||V^T X||_F^2 (depends on V only through P)."""
    return float(np.sum((v.T @ x) ** 2))


def gs_pxf(x: np.ndarray) -> np.ndarray:
    """dL/dP for L = ||P X||_F^2 = tr(X^T P X): the symmetric matrix X X^T."""
    return x @ x.T


def gsv_pxf(v: np.ndarray, x: np.ndarray) -> np.ndarray:
    """G_s V for L = ||P X||_F^2: dL/dP = X X^T is symmetric, so G_s V = X (X^T V)."""
    return x @ (x.T @ v)


def dense_grad(a_dense: np.ndarray, nullity: int, gs: np.ndarray, rows, cols) -> np.ndarray:
    """Closed form -2 [(A^+)^T G_s P]_{ij} at the given nonzero positions.

    ``gs`` is the symmetric n x n gradient dL/dP; P and the rank-(n-N)
    pseudo-inverse come from one dense SVD of A.
    """
    m, n = a_dense.shape
    u_, s, vt = np.linalg.svd(a_dense, full_matrices=False)
    r = n - nullity
    apinv = (vt[:r].T / s[:r]) @ u_[:, :r].T  # n x m
    v = fixed_rank_projector(a_dense, nullity)
    g = -2.0 * apinv.T @ gs @ (v @ v.T)  # m x n
    return g[np.asarray(rows), np.asarray(cols)]


def fd_grad(a_dense: np.ndarray, nullity: int, x: np.ndarray, rows, cols, rel_h: float = 1e-6):
    """Central differences of L(A) = ||P(A) X||_F^2 with the fixed-N projector."""
    out = np.empty(len(rows))
    for p, (i, j) in enumerate(zip(rows, cols)):
        h = rel_h * max(1.0, abs(a_dense[i, j]))
        ap = a_dense.copy()
        ap[i, j] += h
        am = a_dense.copy()
        am[i, j] -= h
        lp = loss_pxf(fixed_rank_projector(ap, nullity), x)
        lm = loss_pxf(fixed_rank_projector(am, nullity), x)
        out[p] = (lp - lm) / (2 * h)
    return out


def range_cg(a: sp.csr_matrix, v: np.ndarray, rhs: np.ndarray, tol: float = 1e-13,
             max_iter: int = 10 ** 6):
    """W = (A^T A)^+ R with R = (I - V V^T) rhs, by CG started at zero.

    Every CG iterate lies in the Krylov space of A^T A and R; R is projected
    onto range(A^T) = null(A)^perp first, so the iteration stays on the range
    where A^T A is positive definite.  V must span null(A) to working accuracy
    (a closed-form basis): a null-space component of R left by a less
    accurate V is one CG cannot reduce.  Columns stop individually once
    ||r_j|| <= tol * ||R_j||.
    """
    r = rhs - v @ (v.T @ rhs)
    k = r.shape[1]
    w = np.zeros_like(r)
    p = r.copy()
    rr = np.einsum("ij,ij->j", r, r)
    r0 = np.sqrt(rr)
    active = np.sqrt(rr) > tol * r0
    it = 0
    while active.any() and it < max_iter:
        q = a.T @ (a @ p)
        pq = np.einsum("ij,ij->j", p, q)
        alpha = np.where(active & (pq > 0), rr / np.where(pq > 0, pq, 1.0), 0.0)
        w += p * alpha[None, :]
        r -= q * alpha[None, :]
        rnew = np.einsum("ij,ij->j", r, r)
        beta = np.where(active & (rr > 0), rnew / np.where(rr > 0, rr, 1.0), 0.0)
        p = np.where(active[None, :], r + p * beta[None, :], p)
        rr = np.where(active, rnew, rr)
        it += 1
        active = np.sqrt(rr) > tol * r0
    return w, it


def sddmm(rowptr, colind, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """grad_p = -2 <U_i, V_j> for every stored nonzero p = (i, j), in CSR order."""
    rowptr = np.asarray(rowptr)
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    cols = np.asarray(colind)
    return -2.0 * np.einsum("pk,pk->p", u[rows], v[cols])


def cg_sddmm_grad(a: sp.csr_matrix, v: np.ndarray, gsv: np.ndarray, tol: float = 1e-13):
    """Gradient in A's CSR order via range CG and SDDMM (large inputs)."""
    w, it = range_cg(a, v, gsv, tol)
    u = a @ w
    return sddmm(a.indptr, a.indices, u, v), it
