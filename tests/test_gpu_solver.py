"""Algorithm 2 on the GPU (through the C ABI) vs the oracle and the closed forms."""
import math

import numpy as np
import pytest

from oracle import exact, lanczos, refine
from workloads import generators as G

pytestmark = pytest.mark.gpu

LAM2_ER20 = 0.36330958416634257  # smallest nonzero Laplacian eigenvalue of the seeded er20 instance
EPS_ER20 = 0.1 * LAM2_ER20 ** 2


def _basis(ctx):
    return ctx.extract_basis().cpu().numpy()


@pytest.mark.parametrize("d", [1, 4, 8])
def test_first_cycle_ritz_values_match_oracle(d):
    """Ritz values of the first cycle, element by element.  At d = 8 the step's
    Gram sums and the 16-column projection run on the matrix cores.  (The
    oracle's own values move by below 2e-16 ||B|| when its start block is
    perturbed by 1e-14.)"""
    from tests.gpu_util import context

    c = G.config("er20")
    print(f"[solver] er20 first cycle d={d}", flush=True)
    ctx, dv, om = context(c, EPS_ER20, d=d, max_dim=64, refine=0, max_cycles=1)
    ctx.lanczos_run(allow_noconv=True)
    th = np.array(ctx.ritz_values())
    r = lanczos.algorithm2(c.to_scipy(), EPS_ER20, dv, om, 64, max_cycles=1)
    nb = 4 * 16.67 ** 2  # ||B|| scale of this instance
    assert th.shape == r["theta"].shape
    assert np.max(np.abs(th - r["theta"])) < 1e-9 * nb


@pytest.mark.parametrize("prec", [0, 1])
def test_er20_nullity_and_subspace(prec):
    from tests.gpu_util import context

    c = G.config("er20")
    print(f"[solver] er20 d=1 prec={prec}", flush=True)
    ctx, dv, om = context(c, EPS_ER20, d=1, max_dim=64, prec=prec)
    st = ctx.lanczos_run()
    v0 = exact.indicator_basis(c.meta["labels"])
    a = c.to_scipy()
    r = lanczos.algorithm2(a, EPS_ER20, dv, om, 64)
    assert st["nullity"] == r["N"] == 20
    v = _basis(ctx)
    assert v.shape == (c.n, 20)
    assert exact.max_angle_sine(v, v0) <= 1e-8
    afro = np.sqrt(np.sum(c.vals ** 2))
    assert np.linalg.norm(a @ v) <= 1e-8 * afro
    assert st["rel_resid_fro"] <= 1e-8
    assert exact.orth_error_fro(v) <= c.n * 20 * exact.U64
    vr, _ = refine.refine(a, r["V"], 1e-10)
    assert exact.max_angle_sine(v, vr) <= 1e-8


@pytest.mark.parametrize("d", [2, 4, 8])
def test_er20_mixed_precision_block_sizes(d):
    """FP32 storage with block sizes > 1 (the reorthogonalisation pair then has
    2d = 4, 8, 16 columns: FP32 variants of both update kernels)."""
    from tests.gpu_util import context

    c = G.config("er20")
    print(f"[solver] er20 mixed d={d}", flush=True)
    ctx, dv, om = context(c, EPS_ER20, d=d, max_dim=128, prec=1)
    st = ctx.lanczos_run()
    assert st["nullity"] == 20
    v = _basis(ctx)
    assert exact.max_angle_sine(v, exact.indicator_basis(c.meta["labels"])) <= 1e-8
    assert st["rel_resid_fro"] <= 1e-8


@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_planted_small_block_sizes(d):
    from tests.gpu_util import context

    c = G.planted_nullity(1000, 1000, 10, seed=5)
    a = c.to_scipy()
    s = np.linalg.svd(a.toarray(), compute_uv=False)
    smin = s[-11]
    eps = 0.1 * smin ** 2
    print(f"[solver] planted 1000 N=10 d={d}", flush=True)
    ctx, dv, om = context(c, eps, d=d, max_dim=128, tol_abs_resid=1e-10 * smin, tol_rel_resid=0.0)
    st = ctx.lanczos_run()
    assert st["nullity"] == 10
    v = _basis(ctx)
    v0 = exact.planted_basis(c.meta["R"])
    assert exact.max_angle_sine(v, v0) <= 1e-8
    assert st["rel_resid_fro"] <= 1e-8


def test_restart_state_planted_vs_oracle_nullity():
    """Same D and Omega: the oracle's Algorithm 2 and the GPU agree on the nullity."""
    from tests.gpu_util import context

    c = G.planted_nullity(600, 600, 6, seed=9)
    a = c.to_scipy()
    s = np.linalg.svd(a.toarray(), compute_uv=False)
    eps = 0.1 * s[-7] ** 2
    print("[solver] planted 600 vs oracle", flush=True)
    for d in (1, 4):
        ctx, dv, om = context(c, eps, d=d, max_dim=96, seed=2)
        st = ctx.lanczos_run()
        r = lanczos.algorithm2(a, eps, dv, om, 96)
        assert st["nullity"] == r["N"] == 6


@pytest.mark.parametrize("kind", ["rank2", "fullrank"])
def test_fd_instance_backward_other_right_hand_sides(kind):
    """Range reduction of G_s V: a rank-2 loss and a full-rank symmetric G_s."""
    import torch
    from oracle import backward as bw
    from tests.gpu_util import context

    c = G.fd_instance()
    a = c.to_scipy()
    ad = a.toarray()
    s = np.linalg.svd(ad, compute_uv=False)
    smin = s[-9]
    print(f"[solver] fd300 backward {kind}", flush=True)
    ctx, dv, om = context(c, 0.1 * smin ** 2, d=1, max_dim=64, tol_abs_resid=1e-12 * smin,
                          tol_rel_resid=0.0)
    assert ctx.lanczos_run()["nullity"] == 8
    v = _basis(ctx)
    if kind == "rank2":
        gs = bw.gs_pxf(G.gaussian_matrix(c.n, 2, seed=6))
    else:
        h = G.gaussian_matrix(c.n, c.n, seed=7)
        gs = h + h.T
    dldv = 2.0 * (gs @ v)  # dL/dV = 2 G_s V for a loss on P
    grad, it = ctx.backward(torch.from_numpy(np.ascontiguousarray(dldv)).cuda(), tol=1e-13)
    grad = grad.cpu().numpy()
    rows = np.repeat(np.arange(c.m), np.diff(c.rowptr))
    ref = bw.dense_grad(ad, 8, gs, rows, c.colind)
    assert np.linalg.norm(grad - ref) <= 1e-6 * np.linalg.norm(ref)


def test_fd_instance_backward_matches_dense_gradient():
    import torch
    from oracle import backward as bw
    from tests.gpu_util import context

    c = G.fd_instance()
    a = c.to_scipy()
    ad = a.toarray()
    s = np.linalg.svd(ad, compute_uv=False)
    smin = s[-9]
    print("[solver] fd300 backward", flush=True)
    ctx, dv, om = context(c, 0.1 * smin ** 2, d=1, max_dim=64, tol_abs_resid=1e-12 * smin,
                          tol_rel_resid=0.0)
    st = ctx.lanczos_run()
    assert st["nullity"] == 8
    v = _basis(ctx)
    x = G.gaussian_matrix(c.n, 8, seed=5)
    dldv = 2.0 * bw.gsv_pxf(v, x)  # L = ||P X||_F^2: dL/dV = 2 G_s V
    grad, it = ctx.backward(torch.from_numpy(dldv).cuda(), tol=1e-13)
    grad = grad.cpu().numpy()
    rows = np.repeat(np.arange(c.m), np.diff(c.rowptr))
    ref = bw.dense_grad(ad, 8, bw.gs_pxf(x), rows, c.colind)
    assert np.linalg.norm(grad - ref) <= 1e-6 * np.linalg.norm(ref)


def test_backward_matches_oracle_cg_sddmm_planted5000():
    """The backward pass at the largest planted size the oracle's range CG
    finishes within a test (5000 x 5000, nullity 20, 15k CG iterations):
    L = ||P X||_F^2 with X seeded n x 8, against oracle.backward.cg_sddmm_grad
    on the closed-form null basis (the GPU's own basis agrees with it to sin
    angle <= 1e-8, and the gradient depends on V only through P)."""
    import time

    import torch
    from oracle import backward as bw
    from tests.gpu_util import context

    c = G.config("planted50k", "small")
    a = c.to_scipy()
    v0 = exact.planted_basis(c.meta["R"])
    print("[solver] planted5000 backward vs oracle CG + SDDMM", flush=True)
    t0 = time.time()
    ctx, dv, om = context(c, 2e-6, d=1, max_dim=200, tol_angle=1e-10)  # eps ~ 0.1 sigma^2
    st = ctx.lanczos_run()
    print(f"[solver] solve {time.time() - t0:.1f} s: nullity {st['nullity']}, {st['matvecs']} matvecs, "
          f"{st['refine_iters']} refinement iterations", flush=True)
    assert st["nullity"] == 20
    v = _basis(ctx)
    assert exact.max_angle_sine(v, v0) <= 1e-8
    x = G.gaussian_matrix(c.n, 8, seed=5)
    dldv = 2.0 * bw.gsv_pxf(v, x)  # L = ||P X||_F^2: dL/dV = 2 G_s V
    t0 = time.time()
    grad, it = ctx.backward(torch.from_numpy(np.ascontiguousarray(dldv)).cuda(), tol=1e-12)
    grad = grad.cpu().numpy()
    print(f"[solver] GPU backward {time.time() - t0:.1f} s, {it} CG iterations", flush=True)
    t0 = time.time()
    ref, it_o = bw.cg_sddmm_grad(a, v0, bw.gsv_pxf(v0, x), tol=1e-12)
    print(f"[solver] oracle backward {time.time() - t0:.1f} s", flush=True)
    err = np.linalg.norm(grad - ref) / np.linalg.norm(ref)
    print(f"[solver] backward rel. error {err:.2e} (GPU {it} CG iterations, oracle {it_o})", flush=True)
    assert err <= 1e-6
