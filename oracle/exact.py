"""Exact null spaces and subspace comparison (oracle; test infrastructure only).

* Closed forms for the structured workloads:
  - graph Laplacian: null(L) is spanned by the indicator vectors of the
    connected components (Sec. 5.1, component counting);
  - coboundary / incidence matrix delta_0 of a graph: same indicator vectors
    (delta_0 x = 0 iff x is constant on every component);
  - planted A = [B, B R] with B of full column rank: null(A) = range([-R; I]).
* Dense SVD null space for tiny inputs (the comparator of Sec. 5.3 is an
  SVD-based dense routine).
* Principal angles (Definition "defPA", Sec. 2.3).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph

U64 = 2.0 ** -52  # unit roundoff as quoted in Sec. 5.3 (u ~ 2.22e-16)


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------
def graph_components(n: int, ei: np.ndarray, ej: np.ndarray) -> np.ndarray:
    """Connected-component label of every vertex of an undirected graph."""
    g = sp.coo_matrix((np.ones(len(ei)), (np.asarray(ei), np.asarray(ej))), shape=(n, n))
    _, lab = csgraph.connected_components(g, directed=False)
    return lab


def laplacian_edges(a: sp.csr_matrix):
    """Edge list (i < j) of the graph whose Laplacian is ``a`` (off-diagonal nonzeros)."""
    c = sp.triu(a, k=1).tocoo()
    keep = c.data != 0
    return c.row[keep], c.col[keep]


def indicator_basis(labels: np.ndarray) -> np.ndarray:
    """Orthonormal basis [1_{C_k}/sqrt(|C_k|)] of the component indicators, labels 0..K-1."""
    labels = np.asarray(labels)
    k = int(labels.max()) + 1
    n = len(labels)
    v = np.zeros((n, k))
    v[np.arange(n), labels] = 1.0
    v /= np.sqrt(v.sum(axis=0))[None, :]
    return v


def planted_basis(r: sp.spmatrix) -> np.ndarray:
    """Orthonormal basis of range([-R; I]) (null space of A = [B, B R])."""
    r = sp.csc_matrix(r)
    k, nn = r.shape
    y = np.vstack([-r.toarray(), np.eye(nn)])
    q, _ = np.linalg.qr(y)
    return q


def column_scaled_basis(v: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Orthonormal basis of null(A S) = S^{-1} null(A), S = diag(s), from one of null(A)."""
    q, _ = np.linalg.qr(np.asarray(v, dtype=np.float64) / np.asarray(s)[:, None])
    return q


# --------------------------------------------------------------------------
# dense SVD (tiny inputs)
# --------------------------------------------------------------------------
def svd_null_space(a_dense: np.ndarray, nullity: int | None = None):
    """Null space from a full SVD.

    Returns (V, sigma) where V holds the right singular vectors belonging to
    the ``nullity`` smallest singular values of the m x n matrix (zero rows
    padded if m < n).  If ``nullity`` is None it is the count of singular
    values <= max(m, n) * u * sigma_max (the usual numerical-rank rule).
    """
    a = np.asarray(a_dense, dtype=np.float64)
    m, n = a.shape
    _, s, vt = np.linalg.svd(a, full_matrices=True)
    sig = np.zeros(n)
    sig[: len(s)] = s
    if nullity is None:
        tol = max(m, n) * U64 * (s[0] if len(s) else 0.0)
        nullity = int(np.sum(sig <= tol))
    order = np.argsort(sig, kind="stable")
    idx = order[:nullity]
    return vt[idx].T.copy(), sig


# --------------------------------------------------------------------------
# principal angles
# --------------------------------------------------------------------------
def orthonormalize(x: np.ndarray) -> np.ndarray:
    q, _ = np.linalg.qr(np.asarray(x, dtype=np.float64))
    return q


def principal_angle_sines(v1: np.ndarray, v0: np.ndarray) -> np.ndarray:
    """Sines of the principal angles between range(v1) and range(v0), descending.

    Both inputs must have orthonormal columns.  Computed from the singular
    values of the residual (I - V0 V0^T) V1 rather than from cos = sigma(V0^T V1):
    for angles near 1e-8 the cosine rounds to one in FP64.  For equal
    dimensions the largest sine equals ||V0 V0^T - V1 V1^T||_2 (Sec. 2.3).
    """
    v1 = np.asarray(v1, dtype=np.float64)
    v0 = np.asarray(v0, dtype=np.float64)
    res = v1 - v0 @ (v0.T @ v1)
    return np.linalg.svd(res, compute_uv=False)


def max_angle_sine(v1: np.ndarray, v0: np.ndarray) -> float:
    """sin of the largest principal angle (0 for empty inputs)."""
    if v1.shape[1] == 0:
        return 0.0
    s = principal_angle_sines(v1, v0)
    return float(s[0]) if len(s) else 0.0


def orth_error_fro(v: np.ndarray) -> float:
    """||V^T V - I||_F (orthonormality check of Sec. 5.3)."""
    k = v.shape[1]
    return float(np.linalg.norm(v.T @ v - np.eye(k)))
