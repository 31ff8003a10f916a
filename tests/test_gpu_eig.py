"""Structured Ritz eigensolver of the restart matrix (block sizes 1 to 8) vs LAPACK on the dense matrix."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LAM2_ER20 = 0.36330958416634257  # smallest nonzero eigenvalue of the er20 Laplacian


def _dense(theta, f, alpha, beta):
    kk, m = len(theta), len(alpha)
    k = kk + m
    t = np.zeros((k, k))
    t[np.arange(kk), np.arange(kk)] = theta
    t[kk, :kk] = f
    t[:kk, kk] = f
    t[np.arange(kk, k), np.arange(kk, k)] = alpha
    t[np.arange(kk, k - 1), np.arange(kk + 1, k)] = beta
    t[np.arange(kk + 1, k), np.arange(kk, k - 1)] = beta
    return t


def _case(k, kk, kind, seed):
    rng = np.random.default_rng(seed)
    theta = np.sort(rng.random(kk) * 10)
    f = rng.standard_normal(kk)
    if kind == "cluster":  # a tight cluster near zero, like the perturbed null space
        nc = kk // 2
        theta[:nc] = np.sort(1e-6 * rng.random(nc))
        f[:nc] *= 1e-9
    if kind == "deflate":  # exact zeros, tiny couplings and repeated poles
        f[::3] = 0.0
        f[1::5] = 1e-17
        theta[2::4] = theta[1::4][: len(theta[2::4])]
        theta = np.sort(theta)
    alpha = rng.random(k - kk) * 10
    beta = np.abs(rng.standard_normal(k - kk - 1)) + 0.1
    if kind == "weak":  # nearly decoupled tail
        beta[0] = 1e-14
    return theta, f, alpha, beta


@pytest.mark.parametrize("k,kk,kind", [
    (2, 0, "plain"), (3, 1, "plain"), (10, 0, "plain"), (10, 8, "plain"), (64, 32, "plain"),
    (257, 160, "plain"), (512, 356, "cluster"), (300, 150, "deflate"), (128, 64, "weak"),
    (512, 256, "plain"),
])
def test_ritz_eig_matches_lapack(k, kk, kind):
    import torch
    from tests.gpu_util import context
    from workloads import generators as G

    print(f"[eig] K={k} kk={kk} {kind}", flush=True)
    c = G.config("er20")
    ctx, _, _ = context(c, 0.01, d=1, max_dim=64)
    theta, f, alpha, beta = _case(k, kk, kind, seed=k + kk)
    t = _dense(theta, f, alpha, beta)
    ref = np.linalg.eigvalsh(t)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    ev, vec = ctx.ritz_eig(dev(theta), dev(f), dev(alpha), dev(beta))
    ev, vec = ev.cpu().numpy(), vec.cpu().numpy()
    nt = np.abs(t).sum(axis=1).max()
    orth = np.linalg.norm(vec.T @ vec - np.eye(k))
    resid = np.linalg.norm(t @ vec - vec * ev[None, :]) / nt
    print(f"[eig] max |lambda - lapack| / ||T|| {np.max(np.abs(ev - ref)) / nt:.2e}; orthogonality {orth:.2e}; "
          f"residual {resid:.2e}", flush=True)
    assert np.all(np.diff(ev) >= 0)
    assert np.max(np.abs(ev - ref)) <= 1e-13 * nt
    assert resid <= 1e-12 * np.sqrt(k)
    assert orth <= 1e-12 * k
    ctx.close()


def _block_case(d, kk, nbk, kind, seed):
    """theta, F (d x kk), Xi blocks (nbk, d, d), Gamma blocks (nbk-1, d, d) and the dense T."""
    rng = np.random.default_rng(seed)
    theta = np.sort(rng.random(kk) * 10)
    f = rng.standard_normal((d, kk))
    xi = rng.standard_normal((nbk, d, d))
    xi = xi + xi.transpose(0, 2, 1) + 5.0
    gam = np.triu(rng.standard_normal((max(nbk - 1, 0), d, d))) + 0.3 * np.eye(d)
    if kind == "cluster":  # a tight cluster near zero with tiny couplings (the perturbed null space)
        nc = kk // 2
        theta[:nc] = np.sort(1e-6 * rng.random(nc))
        f[:, :nc] *= 1e-9
    if kind == "deflate":  # zero couplings, repeated poles, a rank-deficient coupling block
        f[:, ::3] = 0.0
        theta[2::4] = theta[1::4][: len(theta[2::4])]
        theta = np.sort(theta)
        if nbk > 2:
            gam[1][:, 0] = 0.0
            gam[1][0, :] = 0.0
    if kind == "weak" and nbk > 1:  # nearly decoupled tail
        gam[0] *= 1e-14
    if kind == "graded":  # steep diagonal, unit couplings: localised eigenvectors, so the
        # merges see weights down to the rounding level next to their outermost poles
        xi = 0.01 * xi + (np.arange(nbk)[:, None, None] * (200.0 / nbk)) * np.eye(d)
        gam = 0.01 * gam + np.eye(d)
    k = kk + nbk * d
    t = np.zeros((k, k))
    t[np.arange(kk), np.arange(kk)] = theta
    t[kk:kk + d, :kk] = f
    t[:kk, kk:kk + d] = f.T
    for j in range(nbk):
        r = kk + j * d
        t[r:r + d, r:r + d] = xi[j]
        if j + 1 < nbk:
            t[r + d:r + 2 * d, r:r + d] = gam[j]
            t[r:r + d, r + d:r + 2 * d] = gam[j].T
    return theta, f, xi, gam, t


@pytest.mark.parametrize("d,kk,nbk,kind", [
    (2, 0, 1, "plain"), (2, 0, 7, "plain"), (2, 6, 5, "plain"), (4, 0, 13, "plain"), (4, 16, 2, "plain"),
    (4, 40, 30, "plain"), (4, 512, 128, "cluster"), (4, 300, 75, "deflate"), (8, 64, 40, "plain"),
    (8, 128, 17, "weak"), (2, 200, 157, "cluster"), (1, 300, 211, "deflate"), (4, 612, 103, "plain"),
    (1, 0, 1024, "graded"), (4, 64, 256, "graded"), (1, 300, 700, "graded"),
])
def test_block_ritz_eig_matches_lapack(d, kk, nbk, kind):
    import torch
    from tests.gpu_util import context
    from workloads import generators as G

    k = kk + nbk * d
    print(f"[eig] blocks d={d} K={k} kk={kk} {kind}", flush=True)
    c = G.config("er20")
    ctx, _, _ = context(c, 0.01, d=1, max_dim=64)
    theta, f, xi, gam, t = _block_case(d, kk, nbk, kind, seed=17 * d + k + kk)
    ref = np.linalg.eigvalsh(t)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa: E731
    # column-major blocks: pass each block transposed
    ev, vec = ctx.ritz_eig_blocks(d, dev(theta), dev(f.T), dev(xi.transpose(0, 2, 1)),
                                  dev(gam.transpose(0, 2, 1)) if nbk > 1 else dev(np.zeros(1)))
    ev, vec = ev.cpu().numpy(), vec.cpu().numpy()
    nt = np.abs(t).sum(axis=1).max()
    orth = np.linalg.norm(vec.T @ vec - np.eye(k))
    resid = np.linalg.norm(t @ vec - vec * ev[None, :]) / nt
    print(f"[eig] max |lambda - lapack| / ||T|| {np.max(np.abs(ev - ref)) / nt:.2e}; orthogonality {orth:.2e}; "
          f"residual {resid:.2e}", flush=True)
    assert np.all(np.diff(ev) >= 0)
    assert np.max(np.abs(ev - ref)) <= 1e-13 * nt
    assert resid <= 1e-12 * np.sqrt(k)
    assert orth <= 1e-12 * k
    ctx.close()


@pytest.mark.parametrize("d,cycles", [(4, 3), (4, 6), (2, 4), (1, 4)])
def test_block_ritz_eig_on_restarted_lanczos_matrix(d, cycles):
    """T from the oracle's Algorithm 2 after several thick restarts (er20 in the
    symmetric form, nullity 20): kept Ritz values with part of the null cluster,
    their coupling F and the block tail, split into the solver's inputs.
    Orthogonality and residual of the structured solution next to LAPACK's on
    the same matrix."""
    import torch
    from oracle import lanczos as lz
    from tests.gpu_util import context
    from workloads import generators as G

    c = G.config("er20")
    a = c.to_scipy()
    res = lz.algorithm2(a, 0.1 * LAM2_ER20, G.perturbation_diagonal(c.n, 1), G.gaussian_start_block(c.n, d, 1),
                        96, max_cycles=cycles, op="sym")
    t, l0 = res["T"], res["l0"]
    k, kk = t.shape[0], l0 * d
    nbk = (k - kk) // d
    theta = np.diag(t)[:kk].copy()
    f = t[kk:kk + d, :kk].copy()
    xi = np.stack([t[kk + j * d:kk + (j + 1) * d, kk + j * d:kk + (j + 1) * d] for j in range(nbk)])
    gam = np.stack([t[kk + (j + 1) * d:kk + (j + 2) * d, kk + j * d:kk + (j + 1) * d] for j in range(nbk - 1)])
    print(f"[eig] oracle T after {cycles} cycles: d={d} K={k} kk={kk} N={res['N']}", flush=True)
    ctx, _, _ = context(c, 0.01, d=1, max_dim=64)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()  # noqa: E731
    ev, vec = ctx.ritz_eig_blocks(d, dev(theta), dev(f.T), dev(xi.transpose(0, 2, 1)),
                                  dev(gam.transpose(0, 2, 1)))
    ev, vec = ev.cpu().numpy(), vec.cpu().numpy()
    lam, u = np.linalg.eigh(t)
    nt = np.abs(t).sum(axis=1).max()
    orth, orth_ref = np.linalg.norm(vec.T @ vec - np.eye(k)), np.linalg.norm(u.T @ u - np.eye(k))
    resid = np.linalg.norm(t @ vec - vec * ev[None, :]) / nt
    resid_ref = np.linalg.norm(t @ u - u * lam[None, :]) / nt
    print(f"[eig] max |lambda - lapack| / ||T|| {np.abs(ev - lam).max() / nt:.2e}; orthogonality {orth:.2e} "
          f"(lapack {orth_ref:.2e}); residual {resid:.2e} (lapack {resid_ref:.2e})", flush=True)
    assert np.abs(ev - lam).max() <= 1e-13 * nt
    assert orth <= 100 * max(orth_ref, 1e-15 * k)
    assert resid <= 100 * max(resid_ref, 1e-15 * k)
    ctx.close()
