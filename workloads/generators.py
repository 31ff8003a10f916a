"""Seeded generators for the synthetic workloads.

Every matrix is returned as a :class:`CSR` with int64 row offsets, int32
column indices (sorted and unique within each row) and float64 values.
The shapes and structure follow the workloads the paper measures on
(graph Laplacians of collaboration-network subgraphs, Sec. 5.1 Table 2, and
tall cohomology/coboundary matrices, Sec. 5.1 Table 3); those datasets are not
available here, so these seeded instances stand in for them by shape.

Randomness: every generator takes an integer ``seed`` and derives independent
NumPy ``Generator`` streams from ``(seed, tag)`` so that e.g. the matrix and
the start block never share a stream.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph

BASE_SEED = 20240704


@dataclasses.dataclass
class CSR:
    """A sparse matrix in compressed-sparse-row form plus construction metadata."""

    m: int
    n: int
    rowptr: np.ndarray  # int64, m+1
    colind: np.ndarray  # int32, nnz
    vals: np.ndarray  # float64, nnz
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.vals, self.colind, self.rowptr), shape=(self.m, self.n))

    @staticmethod
    def from_scipy(a, meta=None) -> "CSR":
        a = sp.csr_matrix(a)
        a.sum_duplicates()
        a.sort_indices()
        return CSR(
            m=a.shape[0],
            n=a.shape[1],
            rowptr=a.indptr.astype(np.int64),
            colind=a.indices.astype(np.int32),
            vals=a.data.astype(np.float64),
            meta=dict(meta or {}),
        )


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(tag)])


def _laplacian_from_edges(n: int, ei: np.ndarray, ej: np.ndarray, meta: dict) -> CSR:
    """Unit-weight graph Laplacian L = diag(deg) - W from an undirected edge list."""
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    w = sp.coo_matrix((np.ones(len(ei)), (ei, ej)), shape=(n, n)).tocsr()
    w = w + w.T
    w.data[:] = 1.0  # collapse any duplicate edge to weight one
    deg = np.asarray(w.sum(axis=1)).ravel()
    lap = sp.diags(deg) - w
    return CSR.from_scipy(lap, meta)


def _distinct_rows(rng: np.random.Generator, nrows: int, ncols: int, per_col: int) -> np.ndarray:
    """For each of ``ncols`` columns draw ``per_col`` distinct row indices in [0, nrows)."""
    rows = rng.integers(0, nrows, size=(ncols, per_col))
    while True:
        s = np.sort(rows, axis=1)
        bad = np.any(s[:, 1:] == s[:, :-1], axis=1)
        if not bad.any():
            return rows
        rows[bad] = rng.integers(0, nrows, size=(int(bad.sum()), per_col))


def _random_sparse_columns(rng, nrows, ncols, per_col) -> sp.csc_matrix:
    rows = _distinct_rows(rng, nrows, ncols, per_col)
    vals = rng.standard_normal((ncols, per_col))
    cols = np.repeat(np.arange(ncols), per_col)
    return sp.csc_matrix((vals.ravel(), (rows.ravel(), cols)), shape=(nrows, ncols))


# ---------------------------------------------------------------------------
# Workload 1: disjoint Erdos-Renyi components (graph Laplacian, nullity = #components)
# ---------------------------------------------------------------------------
def er_component_laplacian(n_comp: int = 20, comp_size: int = 100, mean_degree: float = 6.0,
                           seed: int = BASE_SEED + 0) -> CSR:
    """Laplacian of ``n_comp`` disjoint G(comp_size, p) graphs, p = mean_degree/(comp_size-1).

    A component is redrawn until it is connected, so the nullity is exactly
    ``n_comp``.  Vertices are relabelled by a seeded global permutation.
    ``meta['labels'][v]`` is the component of vertex ``v``.
    """
    rng = _rng(seed, 1)
    p = mean_degree / (comp_size - 1)
    iu, ju = np.triu_indices(comp_size, 1)
    all_i, all_j = [], []
    for c in range(n_comp):
        while True:
            mask = rng.random(len(iu)) < p
            ei, ej = iu[mask], ju[mask]
            g = sp.coo_matrix((np.ones(len(ei)), (ei, ej)), shape=(comp_size, comp_size))
            ncc, _ = csgraph.connected_components(g, directed=False)
            if ncc == 1:
                break
        all_i.append(ei + c * comp_size)
        all_j.append(ej + c * comp_size)
    n = n_comp * comp_size
    perm = rng.permutation(n)  # old vertex v -> new label perm[v]
    ei = perm[np.concatenate(all_i)]
    ej = perm[np.concatenate(all_j)]
    labels = np.empty(n, dtype=np.int64)
    labels[perm] = np.repeat(np.arange(n_comp), comp_size)
    return _laplacian_from_edges(n, ei, ej, {"kind": "laplacian", "labels": labels,
                                             "n_comp": n_comp, "seed": seed})


# ---------------------------------------------------------------------------
# Workloads 2 and 5: planted nullity A = [B, B R]
# ---------------------------------------------------------------------------
def planted_nullity(m: int = 50000, n: int = 50000, nullity: int = 200, per_col_b: int = 8,
                    per_col_r: int = 4, seed: int = BASE_SEED + 1) -> CSR:
    """A = [B, B R] with B (m x (n-N)) and R ((n-N) x N) sparse Gaussian.

    Each column of B holds ``per_col_b`` N(0,1) values at distinct uniformly
    drawn rows; each column of R holds ``per_col_r`` at distinct rows.
    ``meta['R']`` (CSC) is returned so the exact null space range([-R; I]) can
    be written down by the oracle.
    """
    k = n - nullity
    rng = _rng(seed, 2)
    b = _random_sparse_columns(rng, m, k, per_col_b)
    r = _random_sparse_columns(rng, k, nullity, per_col_r)
    br = (b @ r).tocsc()
    a = sp.hstack([b, br], format="csr")
    return CSR.from_scipy(a, {"kind": "planted", "R": r.tocsc(), "nullity": nullity, "seed": seed})


def column_scaled(c: CSR, decades: float, seed: int) -> CSR:
    """A S with S = diag(10^u_j), u_j iid uniform on [-decades/2, decades/2].

    Columns measured in unrelated units are the usual source of such scaling;
    null(A S) = S^{-1} null(A), so ``meta['col_scale']`` (the diagonal of S) and
    the base matrix's metadata give the exact null space.
    """
    rng = _rng(seed, 9)
    s = 10.0 ** rng.uniform(-decades / 2.0, decades / 2.0, c.n)
    meta = dict(c.meta)
    meta["col_scale"] = s
    return CSR(c.m, c.n, c.rowptr.copy(), c.colind.copy(), c.vals * s[c.colind], meta)


# ---------------------------------------------------------------------------
# Workload 3: coboundary (edge-vertex incidence) of a random geometric graph
# ---------------------------------------------------------------------------
def rgg_coboundary(npoints: int = 1_000_000, mean_degree: float = 8.0,
                   seed: int = BASE_SEED + 2) -> CSR:
    """Incidence matrix delta_0 of a random geometric graph in the unit square.

    Points are uniform in [0,1)^2; the connection radius r solves
    pi r^2 (npoints-1) = mean_degree (no boundary correction).  Row e = (i, j),
    i < j, holds -1 in column i and +1 in column j; rows are sorted by (i, j).
    The nullity equals the number of connected components.
    """
    from scipy.spatial import cKDTree

    rng = _rng(seed, 3)
    pts = rng.random((npoints, 2))
    r = math.sqrt(mean_degree / (math.pi * (npoints - 1)))
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray").astype(np.int64)
    pairs.sort(axis=1)
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    pairs = pairs[order]
    ne = len(pairs)
    rowptr = np.arange(0, 2 * ne + 1, 2, dtype=np.int64)
    colind = pairs.reshape(-1).astype(np.int32)
    vals = np.tile(np.array([-1.0, 1.0]), ne)
    return CSR(ne, npoints, rowptr, colind, vals,
               {"kind": "coboundary", "edges": pairs, "radius": r, "seed": seed})


# ---------------------------------------------------------------------------
# Workload 4: many disjoint components with power-law sizes
# ---------------------------------------------------------------------------
def zipf_component_laplacian(n: int = 4_000_000, n_comp: int = 1000, mean_degree: float = 10.0,
                             seed: int = BASE_SEED + 3) -> CSR:
    """Laplacian of ``n_comp`` disjoint random graphs with Zipf (rank-size) sizes.

    Size of component k (1-based) is round(n / (H_{n_comp} k)), the rank form
    of a power-law size density with exponent 2; the rounding remainder goes
    to the largest component.  Inside a component of size s, Poisson(s *
    mean_degree / 2) random vertex pairs are drawn (self loops and duplicates
    dropped); every connected piece other than the largest is then joined to
    the largest piece by one random edge, so each component is connected and
    the nullity is exactly ``n_comp``.
    """
    rng = _rng(seed, 4)
    h = np.sum(1.0 / np.arange(1, n_comp + 1))
    sizes = np.round(n / (h * np.arange(1, n_comp + 1))).astype(np.int64)
    sizes = np.maximum(sizes, 2)
    sizes[0] += n - sizes.sum()
    offs = np.concatenate([[0], np.cumsum(sizes)])
    all_i, all_j = [], []
    for c in range(n_comp):
        s = int(sizes[c])
        ne = rng.poisson(s * mean_degree / 2.0)
        ei = rng.integers(0, s, ne)
        ej = rng.integers(0, s, ne)
        keep = ei != ej
        ei, ej = np.minimum(ei[keep], ej[keep]), np.maximum(ei[keep], ej[keep])
        key = np.unique(ei * s + ej)
        ei, ej = key // s, key % s
        g = sp.coo_matrix((np.ones(len(ei)), (ei, ej)), shape=(s, s))
        ncc, lab = csgraph.connected_components(g, directed=False)
        if ncc > 1:
            big = np.argmax(np.bincount(lab, minlength=ncc))
            big_vertices = np.flatnonzero(lab == big)
            extra_i, extra_j = [], []
            for piece in range(ncc):
                if piece == big:
                    continue
                members = np.flatnonzero(lab == piece)
                extra_i.append(members[rng.integers(0, len(members))])
                extra_j.append(big_vertices[rng.integers(0, len(big_vertices))])
            ei = np.concatenate([ei, np.array(extra_i)])
            ej = np.concatenate([ej, np.array(extra_j)])
        all_i.append(ei + offs[c])
        all_j.append(ej + offs[c])
    perm = rng.permutation(n)
    ei = perm[np.concatenate(all_i)]
    ej = perm[np.concatenate(all_j)]
    labels = np.empty(n, dtype=np.int64)
    labels[perm] = np.repeat(np.arange(n_comp), sizes)
    return _laplacian_from_edges(n, ei, ej, {"kind": "laplacian", "labels": labels,
                                             "n_comp": n_comp, "sizes": sizes, "seed": seed})


def diagonal_cluster(n_zero: int = 64, n_nonzero: int = 10000) -> CSR:
    """The diagonal matrix of the introduction's example (Sec. 1, Eq. "matrixA").

    diag(0, ..., 0, 1 + 1/n_nonzero, 1 + 2/n_nonzero, ..., 2): ``n_zero`` zero
    entries (the null space is spanned by the first ``n_zero`` unit vectors)
    followed by ``n_nonzero`` equispaced values in (1, 2].  The zeros are
    stored explicitly, so every row holds one entry.  No randomness.
    """
    n = n_zero + n_nonzero
    vals = np.concatenate([np.zeros(n_zero), 1.0 + np.arange(1, n_nonzero + 1) / n_nonzero])
    return CSR(m=n, n=n, rowptr=np.arange(n + 1, dtype=np.int64),
               colind=np.arange(n, dtype=np.int32), vals=vals,
               meta={"kind": "diagonal", "n_zero": n_zero, "n_nonzero": n_nonzero})


def fd_instance(seed: int = BASE_SEED + 4) -> CSR:
    """Small planted instance (m=300, n=280, nullity 8) used for finite differences."""
    return planted_nullity(300, 280, 8, seed=seed)


# ---------------------------------------------------------------------------
# The method's random draws, passed to both sides as inputs
# ---------------------------------------------------------------------------
def perturbation_diagonal(n: int, seed: int) -> np.ndarray:
    """Diagonal of D, entries iid uniform on [0, 1) (Alg. 1 and Alg. 2, first step)."""
    return _rng(seed, 11).random(n)


def gaussian_start_block(n: int, d: int, seed: int) -> np.ndarray:
    """Omega in R^{n x d}, iid N(0,1), returned column-major (Fortran order)."""
    return np.asfortranarray(_rng(seed, 12).standard_normal((n, d)))


def gaussian_matrix(rows: int, cols: int, seed: int, tag: int = 13) -> np.ndarray:
    """A seeded iid N(0,1) dense matrix (column-major), e.g. the loss's X."""
    return np.asfortranarray(_rng(seed, tag).standard_normal((rows, cols)))


# ---------------------------------------------------------------------------
# Named configurations
# ---------------------------------------------------------------------------
def config(name: str, scale: str = "full") -> CSR:
    """Build a named workload.  ``scale='small'`` gives a fast, same-shaped variant."""
    small = scale == "small"
    if name == "er20":
        return er_component_laplacian(20, 100, 6.0)
    if name == "planted50k":
        return planted_nullity(5000, 5000, 20) if small else planted_nullity(50000, 50000, 200)
    if name == "coboundary1m":
        return rgg_coboundary(20000 if small else 1_000_000, 8.0)
    if name == "zipf4m":
        return zipf_component_laplacian(40000 if small else 4_000_000, 10 if small else 1000, 10.0)
    if name == "zipf400k":  # the 4M-vertex Laplacian's construction at a tenth of the size
        return zipf_component_laplacian(4000 if small else 400_000, 10 if small else 100, 10.0,
                                        seed=BASE_SEED + 6)
    if name == "planted200k":
        return (planted_nullity(4000, 4000, 8, seed=BASE_SEED + 5) if small
                else planted_nullity(200000, 200000, 64, seed=BASE_SEED + 5))
    if name == "planted20k_scaled":  # columns spread over two decades
        base = (planted_nullity(2000, 2000, 10, seed=BASE_SEED + 7) if small
                else planted_nullity(20000, 20000, 50, seed=BASE_SEED + 7))
        return column_scaled(base, 2.0, BASE_SEED + 7)
    if name == "fd300":
        return fd_instance()
    if name == "diag10064":  # the introduction's example; small: 16 zeros + 1000 values
        return diagonal_cluster(16, 1000) if small else diagonal_cluster(64, 10000)
    raise KeyError(name)
