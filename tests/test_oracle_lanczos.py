"""Pins for the oracle's operator, Algorithm 1 and Algorithm 2."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import exact, lanczos, operator as op
from workloads import generators as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small_er(seed=3, comps=5, size=40):
    c = G.er_component_laplacian(comps, size, 6.0, seed=seed)
    a = c.to_scipy()
    lam = np.linalg.eigvalsh(a.toarray())
    sig2 = lam[lam > 1e-9].min() ** 2  # sigma_min(A)^2 for symmetric A
    return c, a, sig2


# ------------------------------------------------------------------ operator
def test_operator_symmetric_and_null_action():
    c, a, _ = _small_er()
    rng = np.random.default_rng(0)
    dv = rng.random(c.n)
    x, y = rng.standard_normal(c.n), rng.standard_normal(c.n)
    eps = 0.01
    bx, by = op.apply_b(a, eps, dv, x), op.apply_b(a, eps, dv, y)
    assert abs(bx @ y - x @ by) <= 1e-13 * np.linalg.norm(bx) * np.linalg.norm(y)
    v0 = exact.indicator_basis(c.meta["labels"])
    # on null(A) the operator reduces to the perturbation alone
    assert np.allclose(op.apply_b(a, eps, dv, v0), eps * dv[:, None] * v0, atol=1e-15)


def test_weyl_window_eq_propevB():
    c, a, sig2 = _small_er()
    dv = np.random.default_rng(1).random(c.n)
    eps = 0.1 * sig2
    bmat = op.apply_b(a, eps, dv, np.eye(c.n))
    lam = np.linalg.eigvalsh(0.5 * (bmat + bmat.T))
    n0 = 5
    assert lam[0] >= -1e-12 and lam[n0 - 1] <= eps * dv.max() + 1e-12
    assert lam[n0] >= sig2 - 1e-12
    assert op.norm_upper_bound_ata(a) >= lam[-1] - eps


# ------------------------------------------------------------------ Algorithm 1
@pytest.mark.parametrize("d,ell", [(1, 6), (3, 4)])
def test_algorithm1_spans_block_krylov_space(d, ell):
    c, a, sig2 = _small_er()
    dv = G.perturbation_diagonal(c.n, 2)
    om = G.gaussian_start_block(c.n, d, 2)
    eps = 0.05
    r = lanczos.algorithm1(a, eps, dv, om, ell)
    blocks, x = [], om.copy()
    for _ in range(ell):
        x = x / np.linalg.norm(x, axis=0)
        blocks.append(x)
        x = op.apply_b(a, eps, dv, x)
    kry = exact.orthonormalize(np.hstack(blocks))
    assert exact.max_angle_sine(r["Z"], kry) < 1e-7
    assert exact.orth_error_fro(r["Z"]) < 1e-13


def test_algorithm1_lanczos_relation_and_compression():
    c, a, _ = _small_er()
    d, ell, eps = 2, 12, 0.02
    dv = G.perturbation_diagonal(c.n, 3)
    r = lanczos.algorithm1(a, eps, dv, G.gaussian_start_block(c.n, d, 3), ell)
    z, t = r["Z"], r["T"]
    bz = op.apply_b(a, eps, dv, z)
    e = np.zeros((d, ell * d))
    e[:, -d:] = r["Gamma_last"]
    nb = op.norm_upper_bound_ata(a)
    assert np.linalg.norm(bz - z @ t - r["Q_next"] @ e) < 1e-12 * nb  # Eq. "laniter"
    assert np.linalg.norm(z.T @ bz - t) < 1e-12 * nb  # T = Z^T B Z


def test_algorithm1_ritz_values_first_order_perturbation():
    """Converged Ritz values ~ eps * mean(D over component) + O(eps^2 / sigma^2)."""
    c, a, sig2 = _small_er()
    dv = G.perturbation_diagonal(c.n, 4)
    eps = 1e-2 * sig2
    r = lanczos.algorithm1(a, eps, dv, G.gaussian_start_block(c.n, 1, 4), 190)
    assert r["N"] == 5
    lab = c.meta["labels"]
    means = np.sort(np.array([dv[lab == k].mean() for k in range(5)]))
    assert np.all(np.abs(r["theta"][:5] - eps * means) <= eps ** 2 / sig2)
    # Theorem (null space residual): ||A V_N|| <= eps (sigma^2 - eps)^(-1/2)
    assert np.linalg.norm(a @ r["V"], 2) <= 1.01 * eps / math.sqrt(sig2 - eps)
    assert exact.max_angle_sine(r["V"], exact.indicator_basis(lab)) < 1e-2


# ------------------------------------------------------------------ Algorithm 2
def test_restart_size_and_speed_rule():
    assert lanczos.restart_size(0, 64, 1) == 32
    assert lanczos.restart_size(20, 64, 1) == 42
    assert lanczos.restart_size(20, 64, 4) == 40
    assert lanczos.restart_size(63, 64, 1) == 62  # clamped to dimK - 2d
    hist = [(100, 0), (200, 1), (300, 1), (400, 3), (500, 3), (600, 3)]
    stop, s = lanczos.speed_rule(hist, 1)
    assert s == 2 * 100  # one sample: 200 matvecs for 2 new values -> 100 per value
    assert not stop  # 200 since the last increase, not more than s
    stop, _ = lanczos.speed_rule(hist + [(700, 3)], 1)
    assert stop
    assert lanczos.speed_rule([(100, 1), (900, 1)], 1) == (False, math.inf)  # one increase only
    # d = 2: an interval closes only after >= 2 new values
    hist2 = [(100, 1), (150, 2), (600, 3), (700, 3)]
    stop, s = lanczos.speed_rule(hist2, 2)
    assert s == 2 * (600 - 100) * 2 / 2 and not stop
    assert lanczos.speed_rule([(100, 1), (150, 2), (400, 2)], 2) == (False, math.inf)


def test_algorithm2_first_cycle_matches_algorithm1():
    c, a, sig2 = _small_er()
    dv = G.perturbation_diagonal(c.n, 5)
    om = G.gaussian_start_block(c.n, 1, 5)
    eps = 0.1 * sig2
    r1 = lanczos.algorithm1(a, eps, dv, om, 40)
    r2 = lanczos.algorithm2(a, eps, dv, om, 40, max_cycles=1)
    nb = op.norm_upper_bound_ata(a)
    assert np.max(np.abs(r1["theta"] - r2["theta"])) < 1e-10 * nb


def test_algorithm2_er20_exact_nullity_and_w_bound():
    c = G.config("er20")
    a = c.to_scipy()
    lam2 = 0.36330958416634257  # smallest nonzero Laplacian eigenvalue of this seeded instance
    lam = np.linalg.eigvalsh(a.toarray())
    assert abs(lam[lam > 1e-9].min() - lam2) < 1e-10
    eps = 0.1 * lam2 ** 2
    r = lanczos.algorithm2(a, eps, G.perturbation_diagonal(c.n, 1), G.gaussian_start_block(c.n, 1, 1),
                           64, track_orth=True)
    assert r["N"] == 20 and r["converged"]
    v0 = exact.indicator_basis(c.meta["labels"])
    assert exact.max_angle_sine(r["V"], v0) < 0.05
    tr = np.array(r["orth_trace"])
    assert np.all(tr[:, 2] <= tr[:, 1] * (1 + 1e-9) + 1e-300)  # W is an upper bound
    assert tr[:, 2].max() < 10 * math.sqrt(lanczos.U)  # semi-orthogonality maintained
    assert r["reorths"] > 0


@pytest.mark.parametrize("d", [1, 4])
def test_algorithm2_planted_exact_nullity(d):
    c = G.planted_nullity(600, 600, 6, seed=9)
    a = c.to_scipy()
    s = np.linalg.svd(a.toarray(), compute_uv=False)
    eps = 0.1 * s[-7] ** 2
    r = lanczos.algorithm2(a, eps, G.perturbation_diagonal(c.n, 2), G.gaussian_start_block(c.n, d, 2), 96)
    assert r["N"] == 6 and r["converged"]
    assert exact.max_angle_sine(r["V"], exact.planted_basis(c.meta["R"])) < 0.05


def test_diag_example_recovered_with_d1():
    """Sec. 1, Eq. (matrixA): with the random perturbation d = 1 finds all 64 null vectors."""
    g = json.load(open(os.path.join(GOLDEN, "diag_example.json")))
    n, z = g["n"], g["zeros"]
    diag = np.concatenate([np.zeros(z), 1.0 + g["tail_step"] * np.arange(1, n - z + 1)])
    a = sp.diags(diag).tocsr()
    eps = 0.1 * g["smallest_nonzero_singular_value"] ** 2
    r = lanczos.algorithm2(a, eps, G.perturbation_diagonal(n, 6), G.gaussian_start_block(n, 1, 6), 128)
    assert r["N"] == g["nullity"]
    assert exact.max_angle_sine(r["V"], np.eye(n)[:, :z]) < 0.1


def test_table1_unperturbed_block_lanczos_dimensions():
    """Sec. 1, Table "tabintro": plain block Lanczos (no perturbation: D = 0),
    full reorthogonalisation, 1024 products with A and eigenvalues of T below
    1e-4 counted as zero reports the printed dimensions on the matrix of Eq.
    (matrixA): fewer than 64 for small blocks, always more than d, all 64 from
    d = 32 on.  Algorithm 1 with D = 0 and 3 eps = 1e-4 is that experiment."""
    g = json.load(open(os.path.join(GOLDEN, "diag_example.json")))
    t1 = json.load(open(os.path.join(GOLDEN, "table1_dims.json")))
    n, z = g["n"], g["zeros"]
    diag = np.concatenate([np.zeros(z), 1.0 + g["tail_step"] * np.arange(1, n - z + 1)])
    a = sp.diags(diag).tocsr()
    eps = t1["zero_threshold"] / 3.0
    for d, dim in zip(t1["block_sizes"], t1["dimensions"]):
        r = lanczos.algorithm1(a, eps, np.zeros(n), G.gaussian_start_block(n, d, 1),
                               t1["matvecs"] // d, op="sym")
        assert r["N"] == dim, (d, r["N"], dim)
        # what is counted is (nearly) null: a unit Ritz vector v with Rayleigh
        # quotient below the threshold has ||v outside span(e_1..e_64)||^2 <=
        # threshold / 1.0001, the smallest nonzero entry
        lim = np.sqrt(t1["zero_threshold"] / g["smallest_nonzero_singular_value"])
        assert np.all(np.linalg.norm(r["V"][z:, :], axis=0) <= lim)


def test_table1_matrix_method_finds_whole_null_space():
    """The method on the matrix of Eq. (matrixA) in the symmetric form of Sec.
    5.1 (B = A + eps D, eps below a third of the smallest nonzero entry):
    d = 1 finds all 64 null vectors, in fewer products than the 1024 with which
    plain block Lanczos reports 45 (Table "tabintro")."""
    g = json.load(open(os.path.join(GOLDEN, "diag_example.json")))
    c = G.config("diag10064")
    z = g["zeros"]
    eps = 0.1 * g["smallest_nonzero_singular_value"]
    r = lanczos.algorithm2(c.to_scipy(), eps, G.perturbation_diagonal(c.n, 1),
                           G.gaussian_start_block(c.n, 1, 1), 128, max_matvec=20_000, op="sym")
    assert r["converged"] and r["N"] == g["nullity"] and r["matvecs"] < 1024
    assert exact.max_angle_sine(r["V"], np.eye(c.n)[:, :z]) < 1e-8


def test_full_column_rank_stops_with_nullity_zero():
    """Reading R12: a matrix of full column rank has no Ritz value below 3 eps;
    the run stops once the smallest one has converged above it, well before the
    matvec budget, and that Ritz value is the smallest eigenvalue of B."""
    rng = np.random.default_rng(4)
    b = G._random_sparse_columns(rng, 400, 300, 8)
    a = sp.csr_matrix(b)
    smin2 = np.linalg.svd(a.toarray(), compute_uv=False)[-1] ** 2
    eps = 0.1 * smin2
    dv = G.perturbation_diagonal(300, 1)
    r = lanczos.algorithm2(a, eps, dv, G.gaussian_start_block(300, 1, 1), 64, max_matvec=100_000)
    assert r["N"] == 0 and r["converged"] and r["matvecs"] < 20_000
    lam = np.linalg.eigvalsh(op.apply_b(a, eps, dv, np.eye(300)))
    assert abs(r["theta"][0] - lam[0]) <= r["ritz_res"][0] + 1e-12 * lam[-1]
    assert lanczos.nothing_below(np.array([5 * eps, 1.0]), np.array([0.1 * eps, 1.0]), eps)
    assert not lanczos.nothing_below(np.array([2 * eps, 1.0]), np.array([0.0, 1.0]), eps)
    assert not lanczos.nothing_below(np.array([3.5 * eps, 1.0]), np.array([0.9 * eps, 1.0]), eps)
