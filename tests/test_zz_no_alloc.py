"""apply_op_noalloc (the allocation-free entry point) against apply_op.

Both run the same kernels on the same chunks of columns, so the outputs must
agree bit for bit.  Two calls in a row on one device, the second with a
smaller input (the array keeps the first call's contents), then a matrix too
large for the array, which must be rejected.
"""
import numpy as np
import pytest

from workloads import generators as G

pytestmark = pytest.mark.gpu


def _run(c, eps, ncols, seed, **kw):
    import torch
    from tests.gpu_util import context

    ctx, _, _ = context(c, eps, max_dim=64, **kw)
    x = torch.from_numpy(np.random.default_rng(seed).standard_normal((ncols, c.n))).cuda()
    xcm = x.t()  # n x ncols column-major view
    ref = ctx.apply_op(xcm)
    out = torch.full((ncols, c.n), float("nan"), dtype=torch.float64, device="cuda").t()
    ctx.apply_op_noalloc(xcm, out)
    torch.cuda.synchronize()
    ctx.close()
    return ref, out


def test_noalloc_matches_apply_op_two_calls():
    import torch

    print("[noalloc] planted50k, 11 columns", flush=True)
    ref1, out1 = _run(G.config("planted50k"), 2e-6, 11, 1)
    assert torch.equal(out1, ref1)
    print("[noalloc] er20, 3 columns (smaller, after the first call)", flush=True)
    ref2, out2 = _run(G.config("er20"), 0.01, 3, 2)
    assert torch.equal(out2, ref2)


def test_noalloc_symmetric_form_streaming():
    import torch
    from paper_2407_04634_amd import OP_SYM

    c = G.zipf_component_laplacian(200_000, 50, 10.0, seed=G.BASE_SEED + 8)
    print("[noalloc] 200k-vertex Laplacian, symmetric form, 1 column", flush=True)
    ref, out = _run(c, 1e-3, 1, 3, op=OP_SYM)
    assert torch.equal(out, ref)


def test_noalloc_rejects_matrices_beyond_the_array():
    import scipy.sparse as sp
    import torch
    from paper_2407_04634_amd import NspError
    from paper_2407_04634_amd._lib import NSP_ERR_ARG
    from tests.gpu_util import context

    n = 2_100_000  # 3 n + m doubles = 67.2 MB > 64 MiB
    c = G.CSR.from_scipy(sp.identity(n, format="csr"), {"kind": "test"})
    print("[noalloc] rejection, n = 2.1M", flush=True)
    ctx, _, _ = context(c, 0.1, max_dim=64)
    x = torch.ones((1, n), dtype=torch.float64, device="cuda").t()
    out = torch.empty((1, n), dtype=torch.float64, device="cuda").t()
    with pytest.raises(NspError) as e:
        ctx.apply_op_noalloc(x, out)
    assert e.value.status == NSP_ERR_ARG and "scratch" in str(e.value)
    ctx.close()
