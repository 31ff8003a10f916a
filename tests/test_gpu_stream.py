"""The streaming CSR kernels (matrices with >= 2M nonzeros) vs the oracle."""
import numpy as np
import pytest

from oracle import lanczos
from oracle import operator as op
from workloads import generators as G

pytestmark = pytest.mark.gpu

U = 2.0 ** -52


def _lap():
    # 200 000 vertices, 20 components, mean degree 10: about 2.2M nonzeros
    c = G.zipf_component_laplacian(200_000, 20, 10.0, seed=G.BASE_SEED + 7)
    assert c.nnz >= 1 << 21
    return c


@pytest.mark.parametrize("d", [1, 4])
def test_apply_op_streaming(d):
    import torch
    from tests.gpu_util import context

    c = _lap()
    a = c.to_scipy()
    print(f"[stream] apply_op nnz={c.nnz} d={d}", flush=True)
    ctx, dv, _ = context(c, 1e-2, d=d, max_dim=64)
    x = np.random.default_rng(1).standard_normal((c.n, d))
    y = ctx.apply_op(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = op.apply_b(a, 1e-2, dv, x)
    aa = abs(a)
    k = 4 + 2 * int(np.diff(a.indptr).max())
    bnd = k * U * (aa.T @ (aa @ np.abs(x)) + 1e-2 * dv[:, None] * np.abs(x))
    assert np.all(np.abs(y - ref) <= bnd)
    ctx.close()


@pytest.mark.parametrize("opname", ["normal", "sym"])
def test_first_cycle_streaming_matches_oracle(opname):
    from paper_2407_04634_amd import OP_NORMAL, OP_SYM
    from tests.gpu_util import context

    c = _lap()
    a = c.to_scipy()
    print(f"[stream] first cycle op={opname}", flush=True)
    ctx, dv, om = context(c, 1e-2, max_dim=64, refine=0, max_cycles=1,
                          op=OP_SYM if opname == "sym" else OP_NORMAL)
    ctx.lanczos_run(allow_noconv=True)
    th = np.array(ctx.ritz_values())
    r = lanczos.algorithm2(a, 1e-2, dv, om, 64, max_cycles=1, op=opname)
    nb = op.norm_upper_bound_sym(a) if opname == "sym" else op.norm_upper_bound_ata(a)
    assert np.max(np.abs(th - r["theta"])) < 1e-9 * nb
    ctx.close()
