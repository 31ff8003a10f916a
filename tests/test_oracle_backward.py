"""Pins for the oracle's gradient of L = ||P X||_F^2 w.r.t. the nonzeros of A."""
import numpy as np

from oracle import backward as bw
from oracle import exact
from workloads import generators as G


def _tiny():
    c = G.planted_nullity(30, 26, 3, per_col_b=5, per_col_r=3, seed=21)
    a = c.to_scipy()
    ad = a.toarray()
    rows = np.repeat(np.arange(c.m), np.diff(c.rowptr))
    return c, a, ad, rows, c.colind.astype(np.int64)


def test_closed_form_matches_central_differences():
    c, a, ad, rows, cols = _tiny()
    x = G.gaussian_matrix(c.n, 2, seed=3)
    v = bw.fixed_rank_projector(ad, 3)
    g = bw.dense_grad(ad, 3, bw.gs_pxf(x), rows, cols)
    fd = bw.fd_grad(ad, 3, x, rows, cols)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)


def test_special_cases_vanish():
    c, a, ad, rows, cols = _tiny()
    v = bw.fixed_rank_projector(ad, 3)
    # X = V: L = ||P V||^2 = N for every A, so the gradient vanishes
    assert np.abs(bw.dense_grad(ad, 3, bw.gs_pxf(v), rows, cols)).max() < 1e-12
    # X orthogonal to null(A): G_s V = X X^T V = 0
    x = G.gaussian_matrix(c.n, 2, seed=4)
    x = x - v @ (v.T @ x)
    assert np.abs(bw.dense_grad(ad, 3, bw.gs_pxf(x), rows, cols)).max() < 1e-12


def test_cg_sddmm_matches_dense_and_rotation_invariant():
    c = G.fd_instance()
    a = c.to_scipy()
    ad = a.toarray()
    rows = np.repeat(np.arange(c.m), np.diff(c.rowptr))
    x = G.gaussian_matrix(c.n, 8, seed=5)
    v = exact.planted_basis(c.meta["R"])
    gd = bw.dense_grad(ad, 8, bw.gs_pxf(x), rows, c.colind)
    gc, it = bw.cg_sddmm_grad(a, v, bw.gsv_pxf(v, x))
    assert np.linalg.norm(gc - gd) <= 1e-9 * np.linalg.norm(gd)
    q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((8, 8)))
    gq, _ = bw.cg_sddmm_grad(a, v @ q, bw.gsv_pxf(v @ q, x))
    assert np.linalg.norm(gq - gc) <= 1e-9 * np.linalg.norm(gc)
