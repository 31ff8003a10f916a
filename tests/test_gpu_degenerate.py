"""Degenerate inputs: no null space, empty columns, a wide matrix, a matrix without entries."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import exact, lanczos
from workloads import generators as G

pytestmark = pytest.mark.gpu


def _smin(a_dense, nullity):
    return np.sort(np.linalg.svd(a_dense, compute_uv=False))[nullity]


def test_full_column_rank_has_nullity_zero():
    """No Ritz value ever drops below 3 eps, so the speed rule has no sample;
    the run stops once the smallest Ritz value has converged above 3 eps
    (reading R12, Sec. 4.3), with nullity 0 and an empty basis, as the
    oracle does; the backward pass of an empty basis is zero."""
    import torch
    from paper_2407_04634_amd import _lib
    from tests.gpu_util import context

    rng = np.random.default_rng(4)
    b = G._random_sparse_columns(rng, 400, 300, 8)
    c = G.CSR.from_scipy(b)
    eps = 0.1 * _smin(c.to_scipy().toarray(), 0) ** 2
    print("[degenerate] full column rank", flush=True)
    ctx, dv, om = context(c, eps, max_dim=64, max_matvec=100_000)
    st = ctx.lanczos_run()
    assert st["nullity"] == 0 and st["converged"] == 1 and st["matvecs"] < 20_000
    assert st["status"] == _lib.STATUS_NAMES[_lib.NSP_OK]
    assert ctx.extract_basis().shape == (300, 0)
    grad, it = ctx.backward(torch.zeros((300, 0), dtype=torch.float64, device="cuda"))
    assert it == 0 and float(grad.abs().max()) == 0.0
    r = lanczos.algorithm2(c.to_scipy(), eps, dv, om, 64, max_matvec=100_000)
    assert r["N"] == 0 and r["converged"]


def test_empty_columns_are_null_vectors():
    """Three empty columns appended to the planted 300 x 280 instance: nullity
    8 + 3, spanned by the planted basis and the unit vectors of the empty columns."""
    from tests.gpu_util import context

    f = G.fd_instance()
    a = sp.hstack([f.to_scipy(), sp.csr_matrix((f.m, 3))], format="csr")
    c = G.CSR.from_scipy(a)
    v0 = np.zeros((283, 11))
    v0[:280, :8] = exact.planted_basis(f.meta["R"])
    v0[280:, 8:] = np.eye(3)
    eps = 0.1 * _smin(a.toarray(), 11) ** 2
    print("[degenerate] empty columns", flush=True)
    ctx, dv, om = context(c, eps, max_dim=64)
    st = ctx.lanczos_run()
    assert st["nullity"] == 11
    v = ctx.extract_basis().cpu().numpy()
    assert exact.max_angle_sine(v, v0) <= 1e-8
    assert st["rel_resid_fro"] <= 1e-8
    assert lanczos.algorithm2(a, eps, dv, om, 64)["N"] == 11


def test_wide_matrix_against_dense_svd():
    """m < n: a 200 x 260 sparse Gaussian matrix has nullity 60 (full row rank)."""
    from tests.gpu_util import context

    rng = np.random.default_rng(6)
    a = sp.csr_matrix(G._random_sparse_columns(rng, 200, 260, 6))
    c = G.CSR.from_scipy(a)
    ad = a.toarray()
    v0, sig = exact.svd_null_space(ad, 60)
    assert np.sort(sig)[60] > 1e-3  # full row rank
    eps = 0.1 * np.sort(sig)[60] ** 2
    print("[degenerate] wide 200 x 260", flush=True)
    ctx, dv, om = context(c, eps, max_dim=192)
    st = ctx.lanczos_run()
    assert st["nullity"] == 60
    v = ctx.extract_basis().cpu().numpy()
    assert exact.max_angle_sine(v, v0) <= 1e-8
    assert st["rel_resid_fro"] <= 1e-8


def test_matrix_without_entries_is_rejected_cleanly():
    """A = 0: every Ritz value of B = eps D lies below 3 eps, more than dim K can
    hold; the run stops with NSP_ERR_ARG instead of returning a partial basis."""
    from paper_2407_04634_amd import NspError, _lib
    from tests.gpu_util import context

    c = G.CSR(40, 50, np.zeros(41, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0), {})
    print("[degenerate] no entries", flush=True)
    ctx, _, _ = context(c, 1e-3, max_dim=24)
    with pytest.raises(NspError) as e:
        ctx.lanczos_run()
    assert e.value.status == _lib.NSP_ERR_ARG
    assert "max_dim too small" in str(e.value)
