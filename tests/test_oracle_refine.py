"""Pins for the oracle's FP64 refinement."""
import numpy as np

from oracle import exact, lanczos, refine
from workloads import generators as G


def test_cgls_projection_recovers_null_component():
    c = G.planted_nullity(200, 180, 5, seed=4)
    a = c.to_scipy()
    v0 = exact.planted_basis(c.meta["R"])
    rng = np.random.default_rng(0)
    coeff = rng.standard_normal((5, 3))
    rng_part = a.T @ rng.standard_normal((200, 3))  # lies in range(A^T) = null(A)^perp
    v = v0 @ coeff + 0.1 * rng_part / np.linalg.norm(rng_part, axis=0)
    out, it, res = refine.cgls_null_projection(a, v, 1e-14)
    assert np.linalg.norm(out - v0 @ coeff) < 1e-11
    assert np.all(res <= 1e-14)


def test_refine_reaches_targets_er20():
    c = G.config("er20")
    a = c.to_scipy()
    eps = 0.1 * 0.36330958416634257 ** 2
    r = lanczos.algorithm2(a, eps, G.perturbation_diagonal(c.n, 1), G.gaussian_start_block(c.n, 1, 1), 64)
    v0 = exact.indicator_basis(c.meta["labels"])
    vr, info = refine.refine(a, r["V"], 1e-10)
    assert exact.max_angle_sine(vr, v0) < 1e-8
    assert info["rel_resid_fro"] < 1e-8
    assert exact.orth_error_fro(vr) < c.n * 20 * exact.U64  # ||V^T V - I||_F <= n N u (Sec. 5.3)
