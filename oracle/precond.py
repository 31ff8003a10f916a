"""Outer preconditioning (Sec. 4.4, "Outer preconditioning"), oracle side.

Test infrastructure only: nothing in the library imports this module.

Given an invertible P_R with P_R P_R^T a preconditioner for A^T A, the Lanczos
method runs on B_R = P_R^{-1} A^T A P_R^{-T} + eps D, i.e. on the normal form of
A_R = A P_R^{-T}.  Its output V_R spans (approximately) null(A_R) = P_R^T null(A),
so the null space of A is recovered as P_R^{-T} V_R.  For the symmetric positive
semi-definite form (Sec. 5.1 applies outer preconditioning to the graph
Laplacians) the operator is B_R = P_R^{-1} A P_R^{-T} + eps D, with the same
post-processing.

P_R is either a diagonal (a vector p, P_R = diag(p)) or a dense invertible
lower-triangular matrix, e.g. the incomplete Cholesky factor of ``ichol``
(the preconditioner of the paper's Laplacian experiments, Sec. 5.1).

Readings (where the paper is silent):
  P1  the post-processed basis P_R^{-T} V_R is orthonormalised (thin QR with a
      positive diagonal): the method's output is an orthonormal basis.
  P2  the diagonal ("Jacobi") preconditioner takes P_R = diag(M)^{1/2} with
      M = A^T A (normal form; p_j = ||A e_j||_2) or M = A (symmetric form;
      p_j = sqrt(A_jj)), i.e. the Cholesky factor of M with every off-diagonal
      entry dropped; p_j = 1 where that diagonal entry is not positive.
  P5  incomplete Cholesky (Sec. 5.1 uses a threshold factor with drop
      tolerance 1e-3 and diagonal compensation 0.1): L L^T ~ Mc = M + alpha
      diag(M), computed column by column; the drop rule compares |l_ij| with
      droptol times the 1-norm of Mc(j:n, j); droptol = 0 keeps exactly the
      pattern of M (IC(0)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def jacobi_diagonal(a: sp.csr_matrix, op: str = "normal") -> np.ndarray:
    """Reading P2: p with P_R = diag(p)."""
    a = sp.csr_matrix(a)
    if op == "normal":
        d = np.asarray(a.multiply(a).sum(axis=0)).ravel()
    elif op == "sym":
        d = a.diagonal().astype(np.float64)
    else:
        raise ValueError(op)
    p = np.ones(a.shape[1])
    pos = d > 0
    p[pos] = np.sqrt(d[pos])
    return p


def ichol(m, droptol: float = 0.0, diagcomp: float = 0.0) -> np.ndarray:
    """Incomplete Cholesky factor L (dense lower triangular) of M + diagcomp diag(M) (P5).

    Column by column (j = 0, 1, ...): w = Mc(j:n, j) - L(j:n, :j) L(j, :j)^T,
    l_jj = sqrt(w_j), l_ij = w_i / l_jj, then
      droptol == 0: IC(0) -- l_ij kept only where M has a nonzero (i, j);
      droptol > 0:  threshold -- l_ij dropped when |l_ij| < droptol ||Mc(j:n, j)||_1.
    Raises ValueError on a non-positive pivot.  Dense: small matrices only.
    """
    md = m.toarray() if sp.issparse(m) else np.array(m, dtype=np.float64)
    n = md.shape[0]
    mc = md + diagcomp * np.diag(np.diag(md))
    pattern = md != 0.0
    lo = np.zeros((n, n))
    for j in range(n):
        w = mc[j:, j] - lo[j:, :j] @ lo[j, :j]
        if not np.any(mc[j:, j]) and not np.any(w):
            w[0] = 1.0  # an unknown M does not couple at all keeps l_jj = 1
        if not (w[0] > 0.0):
            raise ValueError(f"incomplete Cholesky: non-positive pivot at column {j}")
        d = np.sqrt(w[0])
        col = w[1:] / d
        if droptol > 0.0:
            keep = np.abs(col) >= droptol * np.sum(np.abs(mc[j:, j]))
        else:
            keep = pattern[j + 1:, j]
        lo[j, j] = d
        lo[j + 1:, j] = np.where(keep, col, 0.0)
    return lo


def _is_diag(pr) -> bool:
    return np.ndim(pr) == 1


def solve_pt(pr, x: np.ndarray) -> np.ndarray:
    """P_R^{-T} x."""
    if _is_diag(pr):
        return x / (pr[:, None] if x.ndim == 2 else pr)
    return sla.solve_triangular(pr, x, trans="T", lower=True)


def solve_p(pr, x: np.ndarray) -> np.ndarray:
    """P_R^{-1} x."""
    if _is_diag(pr):
        return x / (pr[:, None] if x.ndim == 2 else pr)
    return sla.solve_triangular(pr, x, trans="N", lower=True)


def preconditioned_matrix(a: sp.csr_matrix, pr, op: str = "normal") -> sp.csr_matrix:
    """The matrix the Lanczos method sees: A P_R^{-T} (normal form), so that
    B_R = (A P_R^{-T})^T (A P_R^{-T}) + eps D, or P_R^{-1} A P_R^{-T} (symmetric
    form), so that B_R = P_R^{-1} A P_R^{-T} + eps D.  A diagonal P_R keeps the
    sparsity pattern; a triangular one gives a dense matrix (small cases)."""
    a = sp.csr_matrix(a, dtype=np.float64)
    n = a.shape[1]
    if _is_diag(pr):
        s = sp.diags(1.0 / np.asarray(pr, dtype=np.float64))
        ar = a @ s if op == "normal" else s @ a @ s
        return sp.csr_matrix(ar)
    # A P^{-T} = (P^{-1} A^T)^T
    apt = solve_p(pr, a.T.toarray()).T
    if op == "normal":
        return sp.csr_matrix(apt)
    if op == "sym":
        return sp.csr_matrix(solve_p(pr, apt))
    raise ValueError(op)


def apply_b_outer(a: sp.csr_matrix, pr, eps: float, dvec: np.ndarray, x: np.ndarray,
                  op: str = "normal") -> np.ndarray:
    """B_R x with the two triangular solves per application (Sec. 4.4)."""
    x = np.asarray(x, dtype=np.float64)
    y = solve_pt(pr, x)
    if op == "normal":
        z = a.T @ (a @ y)
    elif op == "sym":
        z = a @ y
    else:
        raise ValueError(op)
    dx = eps * (dvec[:, None] * x if x.ndim == 2 else dvec * x)
    return solve_p(pr, z) + dx


def post_process(pr, v_r: np.ndarray) -> np.ndarray:
    """Basis of null(A) from a basis of null(A_R): P_R^{-T} V_R, orthonormalised (P1)."""
    w = solve_pt(pr, np.asarray(v_r, dtype=np.float64))
    if w.shape[1] == 0:
        return w
    q, r = np.linalg.qr(w)
    s = np.sign(np.diag(r)).copy()
    s[s == 0] = 1.0
    return q * s[None, :]
