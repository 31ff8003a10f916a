"""Pins for the oracle's outer preconditioning (Sec. 4.4, "Outer preconditioning").

Each check compares against something the oracle does not compute itself: a
closed-form null space, a dense SVD, a textbook bound of the normalised graph
Laplacian, or an exactly known matrix.
"""
import numpy as np
import scipy.sparse as sp

from oracle import exact, lanczos, refine
from oracle import precond as pc
from workloads import generators as G

U = 2.0 ** -52


def _lower_triangular(n, seed):
    rng = np.random.default_rng(seed)
    p = np.tril(0.3 * rng.standard_normal((n, n)) / np.sqrt(n), k=-1)
    p[np.diag_indices(n)] = 1.0 + np.abs(rng.standard_normal(n))
    return p


def test_jacobi_normal_gives_unit_column_norms():
    """P2: p_j = ||A e_j||, so A P^{-T} has unit columns; an empty column keeps p_j = 1."""
    c = G.planted_nullity(80, 70, 5, seed=11)
    a = c.to_scipy().tolil()
    a[:, 7] = 0.0
    a = sp.csr_matrix(a)
    a.eliminate_zeros()
    p = pc.jacobi_diagonal(a, "normal")
    ar = pc.preconditioned_matrix(a, p, "normal").toarray()
    norms = np.linalg.norm(ar, axis=0)
    assert p[7] == 1.0 and norms[7] == 0.0
    keep = np.arange(70) != 7
    assert np.max(np.abs(norms[keep] - 1.0)) <= 8 * U
    # column j of A P^{-T} is column j of A divided by its norm
    ad = a.toarray()
    np.testing.assert_allclose(ar[:, keep], ad[:, keep] / np.linalg.norm(ad[:, keep], axis=0),
                               rtol=4 * U, atol=0)


def test_jacobi_undoes_a_column_scaling_exactly():
    """A0 with unit columns, A = A0 S: the Jacobi-preconditioned matrix is A0 again."""
    c = G.planted_nullity(120, 100, 6, seed=12)
    a0 = c.to_scipy().toarray()
    a0 /= np.linalg.norm(a0, axis=0)[None, :]
    s = 10.0 ** np.random.default_rng(5).uniform(-3, 3, 100)
    a = sp.csr_matrix(a0 * s[None, :])
    ar = pc.preconditioned_matrix(a, pc.jacobi_diagonal(a, "normal"), "normal").toarray()
    assert np.max(np.abs(ar - a0)) <= 8 * U


def test_jacobi_sym_is_the_normalised_laplacian():
    """P^{-1} L P^{-T} with p = sqrt(deg) is D^-1/2 L D^-1/2: unit diagonal,
    symmetric, spectrum in [0, 2]; its null space is D^{1/2} times the component
    indicators, which the post-processing maps back to the indicators."""
    c = G.er_component_laplacian(4, 30, 6.0, seed=7)
    a = c.to_scipy()
    p = pc.jacobi_diagonal(a, "sym")
    np.testing.assert_array_equal(p, np.sqrt(a.diagonal()))
    ar = pc.preconditioned_matrix(a, p, "sym").toarray()
    assert np.max(np.abs(np.diag(ar) - 1.0)) <= 4 * U
    assert np.array_equal(ar, ar.T)
    lam = np.linalg.eigvalsh(ar)
    assert lam.min() >= -1e-13 and lam.max() <= 2.0 + 1e-13
    yr, _ = exact.svd_null_space(ar, 4)
    v = pc.post_process(p, yr)
    assert exact.max_angle_sine(v, exact.indicator_basis(c.meta["labels"])) <= 1e-12


def test_triangular_outer_preconditioning_null_space():
    """With a non-diagonal P_R the operand order matters: null(A P^{-T}) = P^T null(A)
    and P^{-T} maps it back onto the closed-form null space of the planted A."""
    c = G.planted_nullity(48, 40, 4, seed=13)
    a = c.to_scipy()
    pr = _lower_triangular(40, 3)
    ar = pc.preconditioned_matrix(a, pr, "normal").toarray()
    np.testing.assert_allclose(ar @ pr.T, a.toarray(), rtol=0, atol=1e-13)
    yr, sig = exact.svd_null_space(ar, 4)
    assert sig[np.argsort(sig)][3] <= 1e-13 and np.sort(sig)[4] > 1e-6
    v = pc.post_process(pr, yr)
    v0 = exact.planted_basis(c.meta["R"])
    assert exact.max_angle_sine(v, v0) <= 1e-11
    assert exact.orth_error_fro(v) <= 1e-14
    # the wrong map (P^{-1} instead of P^{-T}) misses the null space
    wrong = np.linalg.qr(np.linalg.solve(pr, yr))[0]
    assert exact.max_angle_sine(wrong, v0) > 1e-3


def test_apply_b_outer_matches_the_formed_operator():
    """B_R x by two triangular solves per application equals (A P^{-T})^T (A P^{-T}) x + eps D x."""
    c = G.planted_nullity(48, 40, 4, seed=14)
    a = c.to_scipy()
    pr = _lower_triangular(40, 4)
    dv = np.random.default_rng(2).random(40)
    x = np.random.default_rng(3).standard_normal((40, 3))
    ar = pc.preconditioned_matrix(a, pr, "normal").toarray()
    ref = ar.T @ (ar @ x) + 0.1 * dv[:, None] * x
    y = pc.apply_b_outer(a, pr, 0.1, dv, x, "normal")
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))
    # symmetric form with the exact Cholesky factor of L + I: B_R - eps D is
    # P^{-1} L P^{-T}, and null(L) comes back from its null space
    lc = G.er_component_laplacian(3, 20, 6.0, seed=8)
    la = lc.to_scipy()
    chol = np.linalg.cholesky(la.toarray() + np.eye(60))
    ars = pc.preconditioned_matrix(la, chol, "sym").toarray()
    xs = np.random.default_rng(4).standard_normal((60, 2))
    dvs = np.random.default_rng(5).random(60)
    ys = pc.apply_b_outer(la, chol, 0.2, dvs, xs, "sym")
    assert np.max(np.abs(ys - (ars @ xs + 0.2 * dvs[:, None] * xs))) <= 1e-12
    yr, _ = exact.svd_null_space(ars, 3)
    v = pc.post_process(chol, yr)
    assert exact.max_angle_sine(v, exact.indicator_basis(lc.meta["labels"])) <= 1e-11


def _kappa_eff(a_dense, nullity):
    s = np.sort(np.linalg.svd(a_dense, compute_uv=False))
    nz = s[s.size - (a_dense.shape[1] - nullity):]
    return nz.max() / nz.min()


def test_algorithm2_on_a_column_scaled_planted_matrix():
    """Column scaling over two decades: the Jacobi preconditioner restores the
    conditioning (Sec. 4.4's purpose), Algorithm 2 on B_R finds the exact nullity,
    and refinement plus post-processing give the closed-form null space of A."""
    base = G.planted_nullity(400, 400, 6, seed=15)
    c = G.column_scaled(base, 2.0, 15)
    a = c.to_scipy()
    p = pc.jacobi_diagonal(a, "normal")
    ar = pc.preconditioned_matrix(a, p, "normal")
    k_plain, k_pre = _kappa_eff(a.toarray(), 6), _kappa_eff(ar.toarray(), 6)
    assert k_pre < 0.25 * k_plain
    smin = 1.0 / k_pre * np.linalg.norm(ar.toarray(), 2)
    eps = 0.1 * smin ** 2
    dv = G.perturbation_diagonal(c.n, 1)
    om = G.gaussian_start_block(c.n, 1, 1)
    r = lanczos.algorithm2(ar, eps, dv, om, 96)
    assert r["N"] == 6
    yr, _ = refine.refine(ar, r["V"], 1e-13)
    v = pc.post_process(p, yr)
    v0 = exact.column_scaled_basis(exact.planted_basis(c.meta["R"]), c.meta["col_scale"])
    assert exact.max_angle_sine(v, v0) <= 1e-8
    assert np.linalg.norm(a @ v) <= 1e-10 * np.sqrt(np.sum(a.data ** 2))


# ------------------------------------------------------------ incomplete Cholesky
def test_ichol_without_fill_is_the_cholesky_factor():
    """A tridiagonal matrix has no fill, so IC(0) is its exact Cholesky factor."""
    n = 60
    t = sp.diags([np.full(n - 1, -1.0), np.full(n, 2.5), np.full(n - 1, -1.0)], [-1, 0, 1])
    lo = pc.ichol(t, 0.0, 0.0)
    assert np.abs(lo - np.linalg.cholesky(t.toarray())).max() <= 1e-14


def test_ichol_tiny_drop_tolerance_is_the_compensated_cholesky_factor():
    c = G.er_component_laplacian(5, 40, 6.0, seed=3)
    a = c.to_scipy()
    lo = pc.ichol(a, 1e-16, 0.1)
    ref = np.linalg.cholesky(a.toarray() + 0.1 * np.diag(a.diagonal()))
    assert np.abs(lo - ref).max() <= 1e-13


def test_ic0_matches_the_matrix_on_its_pattern():
    """IC(0): L has the pattern of tril(M) and L L^T = Mc on that pattern."""
    c = G.er_component_laplacian(5, 40, 6.0, seed=3)
    a = c.to_scipy()
    ad = a.toarray()
    lo = pc.ichol(a, 0.0, 0.1)
    assert np.all((lo != 0) <= (np.tril(ad) != 0))
    r = ad + 0.1 * np.diag(np.diag(ad)) - lo @ lo.T
    assert np.abs(r[ad != 0]).max() <= 1e-13


def test_ichol_threshold_preconditions_the_laplacian():
    """The Sec. 5.1 settings (drop tolerance 1e-3, compensation 0.1) shrink the
    effective condition number of the symmetric form and keep its null space:
    null(L^{-1} A L^{-T}) = L^T null(A)."""
    c = G.config("er20")
    a = c.to_scipy()
    lo = pc.ichol(a, 1e-3, 0.1)
    ar = pc.preconditioned_matrix(a, lo, op="sym").toarray()
    lam0 = np.sort(np.linalg.eigvalsh(a.toarray()))
    lam = np.sort(np.linalg.eigvalsh(0.5 * (ar + ar.T)))
    assert lam0[19] < 1e-12 and lam[19] < 1e-12  # nullity 20 kept
    kappa0, kappa = lam0[-1] / lam0[20], lam[-1] / lam[20]
    assert kappa < kappa0 / 5, (kappa0, kappa)
    v0 = exact.indicator_basis(c.meta["labels"])
    assert np.linalg.norm(ar @ exact.orthonormalize(lo.T @ v0)) <= 1e-12
