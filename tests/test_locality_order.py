"""The host-side locality order of nullspace_init (params.reorder = 1), on the CPU.

The order must be a pair of permutations; a breadth-first search keeps every
connected piece of the row/column graph contiguous, so a block-diagonal matrix
with scrambled labels comes back block-contiguous, and a scrambled band matrix
comes back with a band of comparable width.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2407_04634_amd", "libnullspace.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _order(a):
    from paper_2407_04634_amd import locality_order

    a = sp.csr_matrix(a)
    return locality_order(a.indptr.astype(np.int64), a.indices.astype(np.int32), *a.shape)


def _is_perm(p, k):
    return p.shape == (k,) and np.array_equal(np.sort(p), np.arange(k))


def test_permutations_on_random_rectangular():
    rng = np.random.default_rng(5)
    a = sp.random(700, 300, density=0.01, random_state=rng, format="csr")
    ro, co = _order(a)
    assert _is_perm(ro, 700) and _is_perm(co, 300)
    # rows without entries come last
    empty = np.diff(a.indptr) == 0
    assert np.all(empty[ro[len(ro) - empty.sum():]])
    assert not np.any(empty[ro[:len(ro) - empty.sum()]])


def test_components_come_out_contiguous():
    from workloads import generators as G

    c = G.config("er20")
    ro, co = _order(c.to_scipy())
    lab = c.meta["labels"]
    runs = 1 + np.count_nonzero(np.diff(lab[co]))
    assert runs == 20
    runs_r = 1 + np.count_nonzero(np.diff(lab[ro]))  # Laplacian rows are vertices too
    assert runs_r == 20


def test_scrambled_band_recovers_a_narrow_band():
    n, w = 2000, 3
    rng = np.random.default_rng(9)
    band = sp.diags([np.ones(n - abs(k)) for k in range(-w, w + 1)], list(range(-w, w + 1)), format="csr")
    p = rng.permutation(n)
    q = rng.permutation(n)
    a = band[p][:, q].tocsr()
    ro, co = _order(a)
    b = a[ro][:, co].tocoo()
    assert np.max(np.abs(b.row - b.col)) <= 8 * w
    c = a.tocoo()
    assert np.max(np.abs(c.row - c.col)) > 100 * w  # the scrambled input really was wide


def test_empty_columns_and_matrix_without_entries():
    a = sp.csr_matrix((np.ones(2), ([0, 2], [1, 1])), shape=(4, 3))
    ro, co = _order(a)
    assert _is_perm(ro, 4) and _is_perm(co, 3)
    assert list(co) == [0, 1, 2]  # column 0 is empty: its own piece, visited first
    z = sp.csr_matrix((3, 5))
    ro, co = _order(z)
    assert list(ro) == [0, 1, 2] and list(co) == [0, 1, 2, 3, 4]


def test_invalid_csr_is_rejected():
    from paper_2407_04634_amd import NspError, locality_order

    with pytest.raises(NspError):
        locality_order(np.array([0, 2, 1], dtype=np.int64), np.array([0, 1], dtype=np.int32), 2, 2)
    with pytest.raises(NspError):
        locality_order(np.array([0, 1], dtype=np.int64), np.array([7], dtype=np.int32), 1, 2)
