"""Pins for the oracle's symmetric positive semi-definite operator B = A + eps D (Sec. 5.1)."""
import math

import numpy as np

from oracle import exact, lanczos, refine
from oracle import operator as op
from workloads import generators as G


def _small_er(seed=3, comps=5, size=40):
    c = G.er_component_laplacian(comps, size, 6.0, seed=seed)
    a = c.to_scipy()
    lam = np.linalg.eigvalsh(a.toarray())
    return c, a, lam[lam > 1e-9].min(), lam.max()


def test_sym_operator_on_component_indicators():
    """L 1_C = 0, so B 1_C = eps D 1_C exactly; B is symmetric."""
    c, a, _, _ = _small_er()
    dv = np.random.default_rng(1).random(c.n)
    v0 = exact.indicator_basis(c.meta["labels"])
    eps = 0.37
    np.testing.assert_allclose(op.apply_b_sym(a, eps, dv, v0), eps * dv[:, None] * v0, rtol=0, atol=1e-15)
    x = np.random.default_rng(2).standard_normal((c.n, 3))
    y = np.random.default_rng(3).standard_normal((c.n, 3))
    lhs = x.T @ op.apply_b_sym(a, eps, dv, y)
    rhs = op.apply_b_sym(a, eps, dv, x).T @ y
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(lhs))


def test_sym_norm_bound_is_an_upper_bound():
    c, a, _, lmax = _small_er()
    assert op.norm_upper_bound_sym(a) >= lmax * (1 - 1e-12)
    # for a Laplacian the bound is twice the largest degree
    deg = np.asarray(a.diagonal())
    assert op.norm_upper_bound_sym(a) == 2 * deg.max()


def test_sym_first_order_ritz_values():
    """Converged Ritz values ~ eps * mean(D over component) + O(eps^2 / lambda_2)."""
    c, a, lam2, _ = _small_er()
    dv = G.perturbation_diagonal(c.n, 4)
    eps = 1e-2 * lam2
    r = lanczos.algorithm1(a, eps, dv, G.gaussian_start_block(c.n, 1, 4), 120, op="sym")
    assert r["N"] == 5
    lab = c.meta["labels"]
    means = np.sort(np.array([dv[lab == k].mean() for k in range(5)]))
    assert np.all(np.abs(r["theta"][:5] - eps * means) <= eps ** 2 / lam2)
    # the B-eigenvectors sit at an angle O(eps / lambda_2) from the indicators
    assert exact.max_angle_sine(r["V"], exact.indicator_basis(lab)) < 10 * eps / lam2


def test_sym_algorithm2_er20_nullity_refined_subspace():
    c = G.config("er20")
    a = c.to_scipy()
    lam2 = 0.36330958416634257
    eps = 0.1 * lam2
    r = lanczos.algorithm2(a, eps, G.perturbation_diagonal(c.n, 1), G.gaussian_start_block(c.n, 1, 1),
                           64, op="sym", track_orth=True)
    assert r["N"] == 20 and r["converged"]
    tr = np.array(r["orth_trace"])
    assert np.all(tr[:, 2] <= tr[:, 1] * (1 + 1e-9) + 1e-300)  # W stays an upper bound
    v0 = exact.indicator_basis(c.meta["labels"])
    vr, info = refine.refine(a, r["V"], 1e-10)
    assert exact.max_angle_sine(vr, v0) < 1e-8
    assert info["rel_resid_fro"] < 1e-8


def test_sym_needs_fewer_matvecs_than_normal_on_er20():
    """B = L + eps D keeps kappa(L); A^T A + eps D squares it (Sec. 5.1)."""
    c = G.config("er20")
    a = c.to_scipy()
    lam2 = 0.36330958416634257
    dv, om = G.perturbation_diagonal(c.n, 1), G.gaussian_start_block(c.n, 1, 1)
    rs = lanczos.algorithm2(a, 0.1 * lam2, dv, om, 64, op="sym")
    rn = lanczos.algorithm2(a, 0.1 * lam2 ** 2, dv, om, 64)
    assert rs["N"] == rn["N"] == 20
    assert rs["matvecs"] < rn["matvecs"]
    assert math.isfinite(rs["matvecs"])
