"""torch.autograd wrapper of the solver: gradient of L = ||P X||_F^2 w.r.t. A's nonzeros."""
import numpy as np
import pytest

from oracle import backward as bw
from oracle import precond as pc
from workloads import generators as G

pytestmark = pytest.mark.gpu


def _setup(c, precond):
    import torch
    from paper_2407_04634_amd import Context

    a = c.to_scipy()
    mat = pc.preconditioned_matrix(a, pc.jacobi_diagonal(a)).toarray() if precond else a.toarray()
    smin = np.sort(np.linalg.svd(mat, compute_uv=False))[8]
    dv = torch.from_numpy(G.perturbation_diagonal(c.n, 1)).cuda()
    om = torch.from_numpy(np.ascontiguousarray(G.gaussian_start_block(c.n, 1, 1))).cuda()
    vals = torch.from_numpy(c.vals).cuda()
    ctx = Context(torch.from_numpy(c.rowptr).cuda(), torch.from_numpy(c.colind).cuda(), vals, c.m, c.n,
                  D=dv, Omega=om, eps=0.1 * smin ** 2, d=1, max_dim=64, tol_abs_resid=1e-12 * smin,
                  tol_rel_resid=0.0, precond=precond)
    return ctx, vals.clone().requires_grad_(True)


@pytest.mark.parametrize("scaled,precond", [(False, 0), (True, 1)])
def test_autograd_gradient_matches_dense_closed_form(scaled, precond):
    import torch
    from paper_2407_04634_amd import null_space

    c = G.fd_instance()
    if scaled:
        c = G.column_scaled(c, 2.0, 21)
    print(f"[autograd] fd300 scaled={scaled} precond={precond}", flush=True)
    ctx, vals = _setup(c, precond)
    x_np = G.gaussian_matrix(c.n, 8, seed=5)
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    v = null_space(vals, ctx, tol=1e-13)
    assert v.shape == (c.n, 8)
    loss = ((v.T @ x) ** 2).sum()
    loss.backward()
    ad = c.to_scipy().toarray()
    rows = np.repeat(np.arange(c.m), np.diff(c.rowptr))
    ref = bw.dense_grad(ad, 8, bw.gs_pxf(x_np), rows, c.colind)
    g = vals.grad.cpu().numpy()
    assert np.linalg.norm(g - ref) <= 1e-6 * np.linalg.norm(ref)
    # the loss itself against the dense SVD null basis
    _, s, vt = np.linalg.svd(ad, full_matrices=True)
    v0 = vt[np.argsort(np.concatenate([s, np.zeros(c.n - len(s))]))[:8]].T
    assert abs(float(loss) - np.sum((v0.T @ x_np) ** 2)) <= 1e-9 * float(loss)


def test_autograd_rejects_a_stale_backward():
    import torch
    from paper_2407_04634_amd import null_space

    c = G.fd_instance()
    print("[autograd] stale backward", flush=True)
    ctx, vals = _setup(c, 0)
    x = torch.from_numpy(np.ascontiguousarray(G.gaussian_matrix(c.n, 8, seed=5))).cuda()
    v1 = null_space(vals, ctx)
    null_space(vals.detach(), ctx)  # a second forward pass on the same Context
    with pytest.raises(RuntimeError):
        ((v1.T @ x) ** 2).sum().backward()
