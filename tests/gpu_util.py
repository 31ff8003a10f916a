"""Helpers for GPU tests: move a workload to the device and build a context."""
import numpy as np
import torch

from workloads import generators as G


def to_dev(c):
    return (torch.from_numpy(c.rowptr).cuda(), torch.from_numpy(c.colind).cuda(),
            torch.from_numpy(c.vals).cuda())


def context(c, eps, d=1, max_dim=64, seed=1, max_matvec=300000, **kw):
    from paper_2407_04634_amd import Context

    rp, ci, va = to_dev(c)
    dv = G.perturbation_diagonal(c.n, seed)
    om = G.gaussian_start_block(c.n, d, seed)
    ctx = Context(rp, ci, va, c.m, c.n, D=torch.from_numpy(dv).cuda(),
                  Omega=torch.from_numpy(np.ascontiguousarray(om)).cuda(), eps=eps, d=d,
                  max_dim=max_dim, max_matvec=max_matvec, **kw)
    return ctx, dv, om
