"""Pins for oracle/exact.py: closed forms, dense SVD and principal angles."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import exact
from workloads import generators as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_laplacian_indicators_are_exact_null_vectors():
    c = G.er_component_laplacian(5, 30, 6.0, seed=3)
    a = c.to_scipy()
    ei, ej = exact.laplacian_edges(a)
    lab = exact.graph_components(c.n, ei, ej)
    assert lab.max() + 1 == 5  # one component per generated graph
    v = exact.indicator_basis(lab)
    # integer Laplacian times indicator: exact zero in floating point before scaling
    ind = (v > 0).astype(float)
    assert np.all(a @ ind == 0.0)
    assert exact.orth_error_fro(v) < 1e-14
    # BFS labels agree with the generator's construction labels (as partitions)
    gen = c.meta["labels"]
    pairs = set(zip(lab.tolist(), gen.tolist()))
    assert len(pairs) == 5


def test_planted_basis_matches_dense_svd():
    c = G.planted_nullity(120, 100, 6, seed=7)
    a = c.to_scipy().toarray()
    v0 = exact.planted_basis(c.meta["R"])
    assert np.linalg.norm(a @ v0) < 1e-12
    vs, sig = exact.svd_null_space(a)
    assert vs.shape[1] == 6  # numerical rank rule recovers the planted nullity
    assert exact.max_angle_sine(vs, v0) < 1e-10
    assert sig[np.argsort(sig)[6]] > 1e-3  # gap between zero and nonzero singular values


def test_diag_example_nullity_from_svd():
    g = json.load(open(os.path.join(GOLDEN, "diag_example.json")))
    # same structure at reduced size: first z entries zero, then 1 + k*step
    z, tail = 8, 200
    d = np.concatenate([np.zeros(z), 1.0 + g["tail_step"] * np.arange(1, tail + 1)])
    v, sig = exact.svd_null_space(np.diag(d))
    assert v.shape[1] == z
    e = np.eye(len(d))[:, :z]
    assert exact.max_angle_sine(v, e) < 1e-14


def _rot_pair(n, angles, rng):
    """Two bases with prescribed principal angles, embedded by a random rotation."""
    k = len(angles)
    v0 = np.zeros((n, k))
    v1 = np.zeros((n, k))
    for t, th in enumerate(angles):
        v0[t, t] = 1.0
        v1[t, t] = np.cos(th)
        v1[k + t, t] = np.sin(th)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return q @ v0, q @ v1


@pytest.mark.parametrize("angles", [[0.3, 1e-3, 1e-9], [1e-12, 2e-8], [np.pi / 2, 0.1]])
def test_principal_angles_constructed(angles):
    rng = np.random.default_rng(0)
    v0, v1 = _rot_pair(12, angles, rng)
    s = exact.principal_angle_sines(v1, v0)
    want = np.sort(np.sin(angles))[::-1]
    assert np.allclose(s, want, rtol=1e-6, atol=1e-15)
    # largest sine equals the projector distance (Sec. 2.3) for equal dimensions
    pd = np.linalg.norm(v0 @ v0.T - v1 @ v1.T, 2)
    assert abs(exact.max_angle_sine(v1, v0) - pd) < 1e-12


def test_principal_angles_invariant_under_basis_rotation():
    rng = np.random.default_rng(1)
    v0, v1 = _rot_pair(10, [0.2, 1e-6], rng)
    qr, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    assert np.allclose(exact.principal_angle_sines(v1 @ qr, v0), exact.principal_angle_sines(v1, v0))


def test_coboundary_nullity_equals_components():
    c = G.rgg_coboundary(3000, 8.0, seed=11)
    a = c.to_scipy()
    e = c.meta["edges"]
    lab = exact.graph_components(c.n, e[:, 0], e[:, 1])
    v = exact.indicator_basis(lab)
    assert np.abs(a @ v).max() < 1e-14
    # dense SVD agrees on nullity for this small instance
    s = np.linalg.svd(a.toarray(), compute_uv=False)
    sig = np.zeros(c.n)
    sig[: len(s)] = s
    assert int(np.sum(sig <= max(a.shape) * exact.U64 * s[0])) == lab.max() + 1
