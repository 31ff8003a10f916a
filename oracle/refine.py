"""FP64 refinement of the Ritz basis (oracle; test infrastructure only).

Step 1 -- Rayleigh-Ritz with the perturbation removed (Remark after
Algorithm 1): eigen-decompose S = (A V)^T (A V) and rotate V by its
eigenvectors, ascending.

Step 2 -- projection onto null(A).  Each column v is replaced by
v - A^+ A v, the component of v in null(A).  x = A^+ A v is the minimum-norm
least-squares solution of A x = A v; it lies in range(A^T) and is computed by
CGLS (conjugate gradients on A^T A started from x = 0, so every iterate stays
in range(A^T)).  The CGLS residual s = A v - A x equals A (v - x), so its norm
is exactly the null-space residual of the refined column.  Iteration stops when
||s_j|| <= tol_j for every column.

Step 3 -- re-orthonormalisation by a thin QR, then ||A V||_F (Sec. 5.3's
residual check, here in FP64).
"""
from __future__ import annotations

import numpy as np


def rayleigh_ritz_unperturbed(a, v: np.ndarray):
    """Rotate V by the eigenvectors of (AV)^T(AV), ascending eigenvalues."""
    av = a @ v
    s = av.T @ av
    s = 0.5 * (s + s.T)
    lam, y = np.linalg.eigh(s)
    return v @ y, lam


def cgls_null_projection(a, v: np.ndarray, tol: np.ndarray, max_iter: int = 10 ** 6):
    """Return (V - A^+ A V, iterations, final residual norms ||A v_j||).

    Column j stops updating once ||s_j|| <= tol[j]; columns are independent
    CGLS runs advanced together.
    """
    v = np.array(v, dtype=np.float64, copy=True)
    k = v.shape[1]
    tol = np.broadcast_to(np.asarray(tol, dtype=np.float64), (k,)).copy()
    x = np.zeros_like(v)
    s = a @ v
    r = a.T @ s
    p = r.copy()
    gamma = np.einsum("ij,ij->j", r, r)
    snorm = np.linalg.norm(s, axis=0)
    active = snorm > tol
    it = 0
    while active.any() and it < max_iter:
        q = a @ p
        qq = np.einsum("ij,ij->j", q, q)
        alpha = np.where(active & (qq > 0), gamma / np.where(qq > 0, qq, 1.0), 0.0)
        x += p * alpha[None, :]
        s -= q * alpha[None, :]
        r = a.T @ s
        gnew = np.einsum("ij,ij->j", r, r)
        beta = np.where(active & (gamma > 0), gnew / np.where(gamma > 0, gamma, 1.0), 0.0)
        p = np.where(active[None, :], r + p * beta[None, :], p)
        gamma = np.where(active, gnew, gamma)
        snorm = np.linalg.norm(s, axis=0)
        active = snorm > tol
        it += 1
    return v - x, it, snorm


def refine(a, v: np.ndarray, tol_abs: float, max_iter: int = 10 ** 6):
    """Steps 1-3.  Returns (V_refined, info)."""
    if v.shape[1] == 0:
        return v, dict(iters=0, rel_resid_fro=0.0)
    v1, lam = rayleigh_ritz_unperturbed(a, v)
    v2, iters, _ = cgls_null_projection(a, v1, np.full(v.shape[1], tol_abs), max_iter)
    q, _ = np.linalg.qr(v2)
    res = float(np.linalg.norm((a @ q)))
    afro = float(np.sqrt(np.sum(a.data ** 2)))
    return q, dict(iters=iters, rr_values=lam, resid_fro=res, rel_resid_fro=res / afro)
