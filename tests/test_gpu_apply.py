"""apply_op (y = A^T A x + eps D x through the HIP SpMV pair) vs the oracle, element by element."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import operator as op
from workloads import generators as G

pytestmark = pytest.mark.gpu

U = 2.0 ** -52


def _bound(a, eps, dv, x):
    """Rounding-error scale of B x: k u (|A|^T (|A| |x|) + eps D |x|), k from the row lengths."""
    aa = abs(a)
    k = 4 + int(np.diff(a.indptr).max(initial=0)) + int(np.diff(a.tocsc().indptr).max(initial=0))
    return k * U * (aa.T @ (aa @ np.abs(x)) + eps * dv[:, None] * np.abs(x))


def _check(c, eps, ncols, seed=0):
    import torch
    from tests.gpu_util import context

    print(f"[apply_op] m={c.m} n={c.n} nnz={c.nnz} ncols={ncols}", flush=True)
    ctx, dv, _ = context(c, eps, d=1, max_dim=min(64, c.n - 1) // 1)
    a = c.to_scipy()
    x = np.random.default_rng(seed).standard_normal((c.n, ncols))
    y = ctx.apply_op(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = op.apply_b(a, eps, dv, x)
    err = np.abs(y - ref)
    bnd = _bound(a, eps, dv, x)
    assert np.all(err <= bnd + 1e-300), float((err / (bnd + 1e-300)).max())
    ctx.close()


@pytest.mark.parametrize("ncols", [1, 3, 8, 11])
def test_apply_er20(ncols):
    _check(G.config("er20"), 0.0132, ncols)


@pytest.mark.parametrize("ncols", [1, 4])
def test_apply_planted(ncols):
    _check(G.planted_nullity(5000, 5000, 20, seed=5), 1e-6, ncols)


def test_apply_coboundary_tall():
    _check(G.rgg_coboundary(20000, 8.0, seed=2), 1e-5, 2)


def test_apply_fd_instance_rectangular():
    _check(G.fd_instance(), 1e-2, 5)


def test_apply_empty_rows_and_columns():
    # rows 1 and 4 of A are empty, column 2 never appears (an empty row of A^T)
    rows = [0, 0, 2, 3, 3, 5, 5, 5]
    cols = [0, 3, 1, 0, 4, 1, 3, 4]
    vals = [1.0, -2.0, 0.5, 3.0, -1.0, 2.0, 1.5, -0.25]
    a = sp.csr_matrix((vals, (rows, cols)), shape=(6, 5))
    c = G.CSR.from_scipy(a)
    _check(c, 0.1, 2)
