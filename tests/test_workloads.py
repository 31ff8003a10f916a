"""Generators: shapes, seeds, and structural facts (no method arithmetic)."""
import numpy as np

from workloads import generators as G


def _valid_csr(c):
    assert c.rowptr.dtype == np.int64 and c.colind.dtype == np.int32 and c.vals.dtype == np.float64
    assert c.rowptr[0] == 0 and np.all(np.diff(c.rowptr) >= 0) and c.rowptr[-1] == len(c.colind)
    assert c.colind.min() >= 0 and c.colind.max() < c.n
    for i in range(0, c.m, max(1, c.m // 50)):
        seg = c.colind[c.rowptr[i]:c.rowptr[i + 1]]
        assert np.all(np.diff(seg) > 0)


def test_er_components_shape_and_seed():
    a = G.er_component_laplacian(20, 100, 6.0)
    b = G.er_component_laplacian(20, 100, 6.0)
    _valid_csr(a)
    assert a.m == a.n == 2000
    assert np.array_equal(a.vals, b.vals) and np.array_equal(a.colind, b.colind)
    deg = a.to_scipy().diagonal()
    assert 5.0 < deg.mean() < 7.0
    assert np.bincount(a.meta["labels"]).tolist() == [100] * 20


def test_planted_shape():
    c = G.planted_nullity(600, 500, 10, seed=1)
    _valid_csr(c)
    assert (c.m, c.n) == (600, 500)
    counts = np.bincount(c.colind, minlength=c.n)
    assert np.all(counts[:490] == 8)


def test_rgg_mean_degree():
    c = G.rgg_coboundary(20000, 8.0, seed=2)
    _valid_csr(c)
    assert abs(2 * c.m / c.n - 8.0) < 0.3
    assert np.all(np.diff(c.rowptr) == 2)


def test_zipf_sizes():
    c = G.zipf_component_laplacian(40000, 10, 10.0, seed=4)
    _valid_csr(c)
    sizes = c.meta["sizes"]
    assert sizes.sum() == 40000 and len(sizes) == 10
    assert np.all(np.diff(sizes) <= 0)


def test_random_draws_are_seeded_and_shaped():
    d1 = G.perturbation_diagonal(100, 5)
    assert np.array_equal(d1, G.perturbation_diagonal(100, 5))
    assert d1.min() >= 0 and d1.max() < 1
    om = G.gaussian_start_block(100, 4, 5)
    assert om.shape == (100, 4) and om.flags["F_CONTIGUOUS"]
