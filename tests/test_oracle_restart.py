"""Pins for the oracle's thick restart (Sec. 4.1) and its partial reorthogonalisation (Sec. 4.2).

After two restarts the last cycle's decomposition must still be a Lanczos
decomposition of B (Eq. "laniter"): B Z = Z T + Q_next [0, Gamma_last] with T
the arrowhead-plus-block-tridiagonal matrix of Eq. "defT", and T = Z^T B Z.
Both are checked with B applied directly (not through the oracle's recurrence),
so a wrong coupling block F (rows of V_Z, a dropped Gamma_ell) or a wrong
assembly of T fails them; the planted-mistake test shows that it does.

The bound is the round-off model of Eq. "defmprd": every block step commits an
error of norm at most u_d = d sqrt(n) u ||B||, so the K/d block columns of the
residual have a Frobenius norm of at most sqrt(K/d) u_d.
"""
import math

import numpy as np
import pytest

from oracle import lanczos
from oracle import operator as op
from workloads import generators as G


def _planted600():
    c = G.planted_nullity(600, 600, 6, seed=9)
    a = c.to_scipy()
    s = np.linalg.svd(a.toarray(), compute_uv=False)
    return c, a, 0.1 * s[-7] ** 2, 96


def _er200():
    c = G.er_component_laplacian(5, 40, 6.0, seed=3)
    a = c.to_scipy()
    lam = np.linalg.eigvalsh(a.toarray())
    return c, a, 0.1 * lam[lam > 1e-9].min() ** 2, 40


def _last_cycle(c, a, eps, d, dim_k, full, cycles=3, seed=2):
    dv = G.perturbation_diagonal(c.n, seed)
    om = G.gaussian_start_block(c.n, d, seed)
    r = lanczos.algorithm2(a, eps, dv, om, dim_k, max_cycles=cycles, full_reorth=full)
    z, t = r["Z"], r["T"]
    bz = op.apply_b(a, eps, dv, z)
    e = np.zeros((d, dim_k))
    e[:, -d:] = r["Gamma_last"]
    nb = float(np.max(r["theta"]))  # ||B|| from the last Ritz values (reading R7)
    resid = np.linalg.norm(bz - z @ t - r["Q_next"] @ e)
    compress = np.linalg.norm(z.T @ bz - t)
    bound = math.sqrt(dim_k / d) * d * math.sqrt(c.n) * lanczos.U * nb
    return r, resid, compress, bound


@pytest.mark.parametrize("d", [1, 4])
@pytest.mark.parametrize("full", [False, True], ids=["partial", "full"])
def test_planted_lanczos_relation_after_two_restarts(d, full):
    c, a, eps, dim_k = _planted600()
    r, resid, compress, bound = _last_cycle(c, a, eps, d, dim_k, full)
    assert r["restarts"] == 2 and r["l0"] > 0
    assert full or r["reorths"] > 0
    assert resid <= bound, (resid, bound)
    assert compress <= 2 * bound, (compress, bound)
    # the basis stays semi-orthogonal under partial reorthogonalisation (Sec. 4.2)
    orth = np.linalg.norm(r["Z"].T @ r["Z"] - np.eye(dim_k), 2)
    assert orth <= math.sqrt(lanczos.U)


def test_laplacian_lanczos_relation_after_two_restarts():
    c, a, eps, dim_k = _er200()
    r, resid, compress, bound = _last_cycle(c, a, eps, 1, dim_k, False)
    assert r["restarts"] == 2 and r["reorths"] > 0
    assert resid <= bound and compress <= 2 * bound


def test_kept_ritz_pairs_satisfy_restart_relation():
    """B Z_new = Z_new Theta + Q_{ell_0+1} F right after a restart (Sec. 4.1):
    the first cycle of a 2-cycle run restarts once; the kept block of the
    second cycle's T is diag(Theta) with F below it."""
    c, a, eps, dim_k = _planted600()
    r, _, _, bound = _last_cycle(c, a, eps, 1, dim_k, True, cycles=2)
    kk = r["l0"]
    z, t = r["Z"], r["T"]
    assert np.count_nonzero(t[:kk, :kk] - np.diag(np.diag(t[:kk, :kk]))) == 0
    dv = G.perturbation_diagonal(c.n, 2)
    bzk = op.apply_b(a, eps, dv, z[:, :kk])
    f = t[kk:kk + 1, :kk]
    resid = np.linalg.norm(bzk - z[:, :kk] * np.diag(t)[None, :kk] - z[:, kk:kk + 1] @ f)
    assert resid <= bound


@pytest.mark.parametrize("mistake", ["first rows of V_Z", "Gamma_ell dropped", "Gamma_ell transposed"])
def test_restart_pin_catches_planted_mistakes(monkeypatch, mistake):
    """A wrong coupling block F breaks the relation by many orders of magnitude."""
    wrong = {
        "first rows of V_Z": lambda r, g, vz, k, d, kk: r @ g @ vz[:d, :kk],
        "Gamma_ell dropped": lambda r, g, vz, k, d, kk: r @ vz[k - d:k, :kk],
        "Gamma_ell transposed": lambda r, g, vz, k, d, kk: r @ g.T @ vz[k - d:k, :kk],
    }[mistake]
    monkeypatch.setattr(lanczos, "coupling_block", wrong)
    c, a, eps, dim_k = _planted600()
    _, resid, _, bound = _last_cycle(c, a, eps, 4, dim_k, True)
    assert resid > 1e6 * bound


def test_one_gram_schmidt_pass_at_the_trigger_level():
    """Reading R5: a unit vector whose components along an orthonormal Z are of
    the size that triggers a reorthogonalisation (sqrt(u)) is orthogonal to Z
    to working accuracy after one classical Gram-Schmidt pass, and keeps almost
    all of its norm (the Kahan-Parlett criterion holds)."""
    rng = np.random.default_rng(11)
    n, k = 4000, 300
    z, _ = np.linalg.qr(rng.standard_normal((n, k)))
    w = rng.standard_normal(n)
    w -= z @ (z.T @ w)
    w -= z @ (z.T @ w)
    w /= np.linalg.norm(w)
    q = w + z @ (math.sqrt(lanczos.U) * rng.standard_normal(k))
    q /= np.linalg.norm(q)
    assert np.max(np.abs(z.T @ q)) > 0.5 * math.sqrt(lanczos.U)
    out = lanczos.cgs1_accepted(z, q[:, None])
    assert np.linalg.norm(z.T @ out) <= 10 * math.sqrt(k * n) * lanczos.U
    assert abs(np.linalg.norm(out) - 1.0) <= k * lanczos.U + 1e-15


def test_kahan_parlett_criterion_rejects_cancellation():
    rng = np.random.default_rng(12)
    z, _ = np.linalg.qr(rng.standard_normal((500, 20)))
    q = z @ rng.standard_normal(20) + 0.1 * rng.standard_normal(500)
    q /= np.linalg.norm(q)
    with pytest.raises(RuntimeError, match="W bound failed"):
        lanczos.cgs1_accepted(z, q[:, None])


@pytest.mark.parametrize("d", [1, 4])
def test_ritz_residuals_bound_distance_to_the_spectrum(d):
    """Kahan's bound for a symmetric B: a Ritz pair with residual norm r has an
    eigenvalue of B within r of its Ritz value.  The residual norms the oracle
    returns are ||Gamma_ell V_Z(last d rows, i)||, exact for the pairs of the
    Lanczos decomposition; checked against the dense spectrum of B."""
    c, a, eps, dim_k = _planted600()
    dv = G.perturbation_diagonal(c.n, 2)
    r = lanczos.algorithm2(a, eps, dv, G.gaussian_start_block(c.n, d, 2), dim_k, max_cycles=3)
    lam = np.linalg.eigvalsh(op.apply_b(a, eps, dv, np.eye(c.n)))
    nb = float(lam[-1])
    slack = dim_k * math.sqrt(c.n) * lanczos.U * nb
    dist = np.abs(r["theta"][:, None] - lam[None, :]).min(axis=1)
    assert np.all(dist <= r["ritz_res"] + slack)
    # and they are the true residual norms of the Ritz vectors
    y = r["Z"] @ np.linalg.eigh(r["T"])[1]
    true = np.linalg.norm(op.apply_b(a, eps, dv, y) - y * r["theta"][None, :], axis=0)
    assert np.all(np.abs(true - r["ritz_res"]) <= slack)
