"""The introduction's diagonal example (Sec. 1, Eq. "matrixA", Table "tabintro") through the library.

Plain block Lanczos is the library's run with D = 0 (B = A in the symmetric
form), reorthogonalisation at every step (a threshold far below any bound of
the W-recurrence), a budget of 1024 products and 3 eps = 1e-4 as the zero
threshold: the setting of the table.  The method itself (D uniform, eps below
a third of the smallest nonzero entry, Krylov dimension 128) must find the
whole null space span(e_1..e_64) within fewer products.
"""
import json
import os

import numpy as np
import pytest

from oracle import exact
from workloads import generators as G

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ctx(c, d, D, eps, **kw):
    import torch
    from paper_2407_04634_amd import Context, OP_SYM
    from tests.gpu_util import to_dev

    om = torch.from_numpy(np.ascontiguousarray(G.gaussian_start_block(c.n, d, 1))).cuda()
    return Context(*to_dev(c), c.m, c.n, D=D, Omega=om, eps=eps, d=d, op=OP_SYM, **kw)


@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_table1_unperturbed_dimensions(d):
    import torch

    t1 = json.load(open(os.path.join(GOLDEN, "table1_dims.json")))
    g = json.load(open(os.path.join(GOLDEN, "diag_example.json")))
    c = G.config("diag10064")
    z = c.meta["n_zero"]
    print(f"[table1] unperturbed d={d}", flush=True)
    ctx = _ctx(c, d, torch.zeros(c.n, dtype=torch.float64, device="cuda"), t1["zero_threshold"] / 3.0,
               max_dim=t1["matvecs"], max_matvec=t1["matvecs"], ro_tol=1e-300, refine=0)
    st = ctx.lanczos_run(allow_noconv=True)
    dim = t1["dimensions"][t1["block_sizes"].index(d)]
    print(f"[table1] d={d}: dimension {st['nullity']} (printed: {dim}), {st['matvecs']} products", flush=True)
    assert st["matvecs"] == t1["matvecs"]
    assert st["nullity"] == dim
    # a unit Ritz vector with Rayleigh quotient below the threshold has at most
    # threshold / 1.0001 of its squared norm outside span(e_1..e_64)
    v = ctx.extract_basis().cpu().numpy()
    lim = np.sqrt(t1["zero_threshold"] / g["smallest_nonzero_singular_value"])
    assert np.all(np.linalg.norm(v[z:, :], axis=0) <= lim * (1 + 1e-6))
    ctx.close()


@pytest.mark.parametrize("d", [1, 4])
def test_table1_matrix_method_finds_whole_null_space(d):
    import torch

    g = json.load(open(os.path.join(GOLDEN, "diag_example.json")))
    c = G.config("diag10064")
    z = c.meta["n_zero"]
    print(f"[table1] method d={d}", flush=True)
    ctx = _ctx(c, d, torch.from_numpy(G.perturbation_diagonal(c.n, 1)).cuda(),
               0.1 * g["smallest_nonzero_singular_value"], max_dim=128, max_matvec=20_000)
    st = ctx.lanczos_run()
    print(f"[table1] method d={d}: nullity {st['nullity']}, {st['matvecs']} products", flush=True)
    assert st["nullity"] == g["nullity"]
    assert st["matvecs"] < 1024  # fewer products than the table's plain runs, which miss null vectors
    v = ctx.extract_basis().cpu().numpy()
    assert exact.max_angle_sine(v, np.eye(c.n)[:, :z]) <= 1e-8
    ctx.close()
