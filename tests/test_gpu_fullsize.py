"""Parity at the measured sizes, in the launch configurations bench.py times.

* planted50k (50 000 x 50 000, 405k nonzeros; lanes-per-row SpMV pair):
  apply_op on every output, and the first restart cycle at d = 1, K = 1024,
  eps = 2e-6 (the bench solve's configuration) against the oracle's Algorithm 2.
* 4M-vertex Laplacian (44M nonzeros; streaming SpMV, symmetric form) and the
  1M-point coboundary (8M nonzeros; streaming SpMV pair, normal form): apply_op
  on every output.
The full solves at these sizes are checked against the closed-form null spaces
by bench.py itself (its ``valid`` field).
"""
import numpy as np
import pytest

from oracle import lanczos
from oracle import operator as op
from workloads import generators as G

pytestmark = pytest.mark.gpu

U = 2.0 ** -52


def _apply_check(c, eps, form, ncols=1):
    import torch
    from paper_2407_04634_amd import OP_NORMAL, OP_SYM
    from tests.gpu_util import context

    ctx, dv, _ = context(c, eps, max_dim=64, op=OP_SYM if form == "sym" else OP_NORMAL)
    a = c.to_scipy()
    x = np.random.default_rng(3).standard_normal((c.n, ncols))
    y = ctx.apply_op(torch.from_numpy(x).cuda()).cpu().numpy()
    aa = abs(a)
    rl = int(np.diff(a.indptr).max())
    if form == "sym":
        ref = op.apply_b_sym(a, eps, dv, x)
        mag = aa @ np.abs(x) + eps * dv[:, None] * np.abs(x)
        k = 4 + rl
    else:
        ref = op.apply_b(a, eps, dv, x)
        mag = aa.T @ (aa @ np.abs(x)) + eps * dv[:, None] * np.abs(x)
        k = 4 + rl + int(np.diff(a.tocsc().indptr).max())
    err = np.abs(y - ref)
    assert np.all(err <= k * U * mag + 1e-300), float((err / (k * U * mag + 1e-300)).max())
    ctx.close()


def test_apply_op_planted50k_full():
    print("[full] apply_op planted50k", flush=True)
    _apply_check(G.config("planted50k"), 2e-6, "normal")


def test_first_cycle_planted50k_bench_configuration():
    from tests.gpu_util import context

    c = G.config("planted50k")
    print("[full] planted50k first cycle, d=1, K=1024", flush=True)
    ctx, dv, om = context(c, 2e-6, d=1, max_dim=1024, refine=0, max_cycles=1)
    ctx.lanczos_run(allow_noconv=True)
    th = np.array(ctx.ritz_values())
    a = c.to_scipy()
    r = lanczos.algorithm2(a, 2e-6, dv, om, 1024, max_cycles=1)
    assert th.shape == r["theta"].shape == (1024,)
    assert np.max(np.abs(th - r["theta"])) < 1e-9 * op.norm_upper_bound_ata(a)


def test_apply_op_zipf4m_full():
    print("[full] apply_op 4M-vertex Laplacian (symmetric form)", flush=True)
    _apply_check(G.config("zipf4m"), 1e-2, "sym")


def test_apply_op_coboundary1m_full():
    print("[full] apply_op 1M-point coboundary", flush=True)
    _apply_check(G.config("coboundary1m"), 1e-5, "normal")
