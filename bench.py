"""Benchmark: null vectors per second of the randomized small-block Lanczos solver.

Default workload: the 4M-vertex graph Laplacian (1000 disjoint components with
power-law sizes, mean degree 10, 43 950 418 stored entries), solved in the
symmetric form B = L + eps D that the paper uses for graph Laplacians
(Sec. 5.1), d = 1, dim K = 2048, once in mixed precision and once in plain
FP64, each refined in FP64 to the same targets.  A solve counts only if the
nullity is exact (1000), ||L V||_F <= 1e-8 ||L||_F and the sine of the largest
principal angle to the closed-form null space (component indicators) is at
most 1e-8; ``valid`` says whether both did.

A "step" is one restart cycle of Algorithm 2 (the Lanczos steps of the cycle
with their SpMV, three-term recurrence, W-recurrence and partial
reorthogonalisation, then the Rayleigh-Ritz step and the thick restart) of the
mixed-precision solve: the solve's first ``--warmup`` cycles are the warmup,
the next ``--steps`` cycles are timed (each interval runs between two
synchronisations of the library's stream), and ``ms_per_step`` is their mean.
``value`` is whole-solve throughput: nullity / wall time of the complete mixed
solve (Lanczos cycles plus FP64 refinement, inputs resident in HBM).

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload zipf4m]
                    [--precs mixed,fp64] [--no-cpu-baseline] [--legs LIST]

Prints one JSON line on stdout; progress goes to stderr.  Only one GPU is
supported.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of a kernel, from two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch) scaled by the same counters on the plain
# copy of --copy-calibration (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0), as a ratio to
# the algorithmic bytes.  Keyed by (workload, d, precision, kernel); an entry is
# dropped whenever that kernel changes.  The summaries with their commands are
# in profiles/.
TRAFFIC = {
    # profiles/k_ts_pair_zipf4m_traffic.md: 1511 reorthogonalising launches
    ("zipf4m", 1, "mixed", "k_ts_tn"): {"ratio": 0.94},
    ("zipf4m", 1, "mixed", "k_ts_nn_v"): {"ratio": 0.88},
}

# eps = c * sigma^2 with c = 0.1 (the Remark after Thm. "thmmain" asks for
# c < 1/3), sigma^2 the smallest nonzero eigenvalue of A^T A (normal form) or
# the smallest nonzero eigenvalue of A (symmetric form)
WORKLOADS = {
    "er20": dict(gen=("er20",), eps=0.1 * 0.36330958416634257 ** 2, max_dim=64, op="normal",
                 desc="Laplacian of 20 disjoint G(100, 6/99) components, n=2000, nullity 20"),
    "planted50k": dict(gen=("planted50k",), eps=2e-6, max_dim=1024, op="normal",
                       desc="planted A=[B, BR], m=n=50000, B 8 N(0,1)/col, R 4 N(0,1)/col, nullity 200"),
    "zipf400k": dict(gen=("zipf400k",), eps=0.035, max_dim=256, op="sym",
                     desc="Laplacian of 100 components, Zipf sizes, mean degree 10, n=400000, nullity 100"),
    "zipf4m": dict(gen=("zipf4m",), eps=0.074, max_dim=2048, op="sym",
                   desc="Laplacian of 1000 components, Zipf sizes (exponent 2), mean degree 10, "
                        "n=4000000, nnz=43950418, nullity 1000"),
}


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- validity
def closed_form_check(c, v):
    """Largest principal-angle sine between V (n x N, CUDA) and the exact null space.

    Laplacians: null(L) is spanned by the component indicators, so the part of
    V outside it is V minus its per-component row means (segment sums on the
    GPU, no dense n x N_exact matrix).  Planted matrices: qr([-R; I]).
    """
    import torch

    kind = c.meta["kind"]
    if kind == "laplacian":
        lab = torch.from_numpy(c.meta["labels"].astype(np.int64)).to(v.device)
        ncomp = int(c.meta["labels"].max()) + 1
        if v.shape[1] != ncomp:
            return None
        cnt = torch.bincount(lab, minlength=ncomp).double()
        means = torch.zeros((ncomp, v.shape[1]), dtype=torch.float64, device=v.device)
        means.index_add_(0, lab, v)
        means /= cnt[:, None]
        res = v - means[lab]
    elif kind == "planted":
        r = c.meta["R"].toarray()
        q, _ = np.linalg.qr(np.vstack([-r, np.eye(r.shape[1])]))
        v0 = torch.from_numpy(q).to(v.device)
        if v.shape[1] != v0.shape[1]:
            return None
        res = v - v0 @ (v0.T @ v)
    else:
        raise ValueError(kind)
    g = res.T @ res
    del res
    return float(torch.sqrt(torch.clamp(torch.linalg.eigvalsh(g)[-1], min=0.0)))


def exact_nullity(c):
    kind = c.meta["kind"]
    if kind == "laplacian":
        return int(c.meta["labels"].max()) + 1
    if kind == "planted":
        return int(c.meta["R"].shape[1])
    raise ValueError(kind)


# ---------------------------------------------------------------- rooflines
def spmv_bytes(m, n, nnz, d, esize, sym):
    """Algorithmic HBM bytes of one Lanczos step's operator application.

    Normal form: y = A x reads A's CSR once (int32 row offsets and column
    indices, values of ``esize`` bytes), x once and writes y; the fused second
    product reads the stored transpose, y, x, the previous block and D (FP64)
    and writes P.  Symmetric form: one fused product with A reading x (gathers
    counted once), the previous block and D and writing P.
    Returns (bytes of the first product, bytes of the fused product).
    """
    if sym:
        return 0, 4 * (n + 1) + nnz * (4 + esize) + esize * d * 3 * n + 8 * n
    a = 4 * (m + 1) + nnz * (4 + esize) + esize * d * (n + m)
    at = 4 * (n + 1) + nnz * (4 + esize) + esize * d * (m + n + n + n) + 8 * n
    return a, at


def kernel_rows(st, m, n, nnz, d, esize, sym, stream):
    """Per-kernel achieved GB/s from the solver's HIP-event samples (profile mode)."""
    a_b, at_b = spmv_bytes(m, n, nnz, d, esize, sym)
    k1 = "k_csr_stream" if stream else "k_spmm"
    k2 = "k_csr_stream" if stream else "k_spmmT_step"
    out = []
    if st.get("spmv_samples", 0) > 0:
        if sym:
            out.append((f"{k2} (P = A x + eps D x - Xp Gamma^T)", st["t_spmv_at_us"], at_b))
        else:
            out.append((f"{k1} (y = A x)", st["t_spmv_a_us"], a_b))
            out.append((f"{k2} (P = A^T y + eps D x - Xp Gamma^T)", st["t_spmv_at_us"], at_b))
    na = st.get("ro_active", 0)
    if na > 0:
        # launches at steps whose W-recurrence flag was clear return at once; the
        # figures below are per launch that reorthogonalised
        out.append(("k_ts_tn (H = Z^T [q_l, q_l+1], per-chunk partials)", st["ro_tn_ms"] / na * 1e3,
                    st["ro_tn_bytes"] / na))
        out.append(("k_ts_nn_v ([q_l, q_l+1] -= Z H, fused Gram)", st["ro_nn_ms"] / na * 1e3,
                    st["ro_nn_bytes"] / na))
    rows = []
    for name, us, b in out:
        gbs = b / (us * 1e-6) / 1e9 if us > 0 else 0.0
        rows.append({"kernel": name, "avg_us": us, "bytes_per_launch": b, "achieved_gbs": gbs,
                     "frac_hbm": gbs / HBM_PEAK_GBS})
    return rows


def dominant(rows, st, d):
    """The kernel with the largest total time: the SpMV every step, the
    reorthogonalisation pair at the flagged steps (fraction from the samples)."""
    steps = st["matvecs"] / d
    frac = st["ro_active"] / max(1, st["ro_samples"])
    weight = [steps * frac if r["kernel"].startswith("k_ts_") else steps for r in rows]
    return max(zip(rows, weight), key=lambda t: t[0]["avg_us"] * t[1])[0], frac


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain copy of known size for scaling rocprofv3's FETCH_SIZE / WRITE_SIZE:
    ``reps`` launches of dst = src * 1.0 (FP64) reading and writing ``nbytes``."""
    import torch

    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": nbytes, "bytes_written": nbytes,
                                           "launches": reps, "kernel": "torch.mul(src, 1.0, out=dst)"}}))


# ---------------------------------------------------------------- one solve
def solve(c, dev, wl, prec, d, max_dim, eps, args, label):
    """One full solve through the C ABI; returns (record, context stats, cycle times)."""
    import torch
    from paper_2407_04634_amd import Context, OP_NORMAL, OP_SYM, PREC_FP64, PREC_MIXED

    rp, ci, va, dv, om = dev
    t0 = time.perf_counter()
    ctx = Context(rp, ci, va, c.m, c.n, D=dv, Omega=om, eps=eps, d=d, max_dim=max_dim,
                  prec=PREC_MIXED if prec == "mixed" else PREC_FP64, tol_angle=1e-9,
                  tol_rel_resid=1e-10, max_matvec=args.max_matvec, max_cycles=args.max_cycles,
                  refine=0 if args.no_refine else 1, profile=1,
                  op=OP_SYM if wl["op"] == "sym" else OP_NORMAL)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"{label}: context ready in {t1 - t0:.1f} s, solving ({prec}, d={d}, K={max_dim}, eps={eps:g})")
    partial = args.max_cycles > 0 or args.no_refine
    st = ctx.lanczos_run(allow_noconv=partial)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    cyc = ctx.cycle_times()
    v = ctx.extract_basis().contiguous()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    sine = closed_form_check(c, v)
    del v
    torch.cuda.empty_cache()
    n_exact = exact_nullity(c)
    valid = bool(not partial and st["nullity"] == n_exact and sine is not None and sine <= 1e-8
                 and 0 <= st["rel_resid_fro"] <= 1e-8)
    rec = {"prec": prec, "d": d, "solve_s": t2 - t1, "init_s": t1 - t0,
           "null_vectors_per_s": st["nullity"] / (t2 - t1), "valid": valid,
           "nullity": st["nullity"], "nullity_exact": n_exact,
           "rel_resid_fro": st["rel_resid_fro"], "max_sin_angle": sine,
           "orth_err_fro": st["orth_err_fro"],
           **{k: st[k] for k in ("matvecs", "restarts", "reorths", "refine_iters", "t_lanczos_s",
                                 "t_restart_s", "t_refine_s", "theta_next", "norm_b")}}
    log(f"{label}: {json.dumps(rec)}")
    return rec, st, cyc


# ---------------------------------------------------------------- CPU baseline
def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(c, wl, eps, d, max_dim, rec, reorth_k_avg):
    """The oracle (FP64 NumPy/SciPy) timed on a bounded sample of the same
    workload, extrapolated to the mixed GPU run's operation counts.

    Sample (about 10-30 s): the oracle's operator application (Sec. 1.2 /
    Sec. 5.1 form) on the full matrix, one classical Gram-Schmidt pass of its
    partial reorthogonalisation against a 32-column basis of full height, the
    restart's basis update Z V_Z on a row slice of full width dim K, and one
    iteration of its refinement (CGLS) on 4 columns (two runs of 1 and 2
    iterations, differenced).  Each is scaled linearly
    (basis width, rows, columns) to the GPU run's counts: matvecs, reorth
    events at the measured mean basis width, restarts, refinement iterations
    on N columns.  The oracle's refinement is CGLS and needs more iterations
    than the library's CG for the symmetric form, so that term is a lower
    bound.  A full oracle solve at this size would hold a 65 GB basis.
    """
    from oracle import lanczos, refine
    from oracle import operator as op
    from workloads import generators as G

    a = c.to_scipy()
    n = c.n
    apply_b, _ = op.operator("sym" if wl["op"] == "sym" else "normal")
    dv = G.perturbation_diagonal(n, 1)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(n)

    def timed(fn, reps=1):
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        return (time.perf_counter() - t0) / reps

    t_apply = timed(lambda: apply_b(a, eps, dv, x), 2)
    # the cost of a Gram-Schmidt pass depends on the shapes only
    kz = 32
    z = rng.standard_normal((n, kz))
    pair = rng.standard_normal((n, 2 * d))
    t_ro = timed(lambda: lanczos.cgs1(z, pair), 2) * (reorth_k_avg / kz)
    del z
    rows = min(n, 50_000)
    zs = rng.standard_normal((rows, max_dim))
    kk = lanczos.restart_size(rec["nullity"], max_dim, d)
    vz = rng.standard_normal((max_dim, kk))
    t_rs = timed(lambda: zs @ vz) * (n / rows)
    del zs, vz
    cols = 4
    vs = rng.standard_normal((n, cols))
    t1 = timed(lambda: refine.cgls_null_projection(a, vs, 0.0, max_iter=1))
    t2 = timed(lambda: refine.cgls_null_projection(a, vs, 0.0, max_iter=2))
    t_cg = max(t2 - t1, 1e-3) * max(1, rec["nullity"]) / cols
    t_est = (rec["matvecs"] * t_apply + rec["reorths"] * t_ro + rec["restarts"] * t_rs
             + rec["refine_iters"] * t_cg)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {
        "value": rec["nullity"] / t_est,
        "unit": "null vectors/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "extrapolated": True,
        "est_solve_s": t_est,
        "sample": (f"oracle per-operation times on the full {n}-unknown matrix: operator application "
                   f"{t_apply * 1e3:.1f} ms, one CGS reorthogonalisation pass {t_ro * 1e3:.1f} ms at "
                   f"{reorth_k_avg:.0f} basis vectors (timed at {kz}, scaled), restart update "
                   f"{t_rs:.2f} s (timed on {rows} rows, scaled), CGLS refinement iteration "
                   f"{t_cg:.2f} s on {rec['nullity']} columns (timed on {cols}, scaled); times the mixed "
                   f"GPU run's {rec['matvecs']} matvecs, {rec['reorths']} reorthogonalisations, "
                   f"{rec['restarts']} restarts and {rec['refine_iters']} refinement iterations"),
    }


# ---------------------------------------------------------------- optional legs
def leg_spmv(name, prec, d=1, max_dim=64):
    """SpMV pair inside real Lanczos steps (one restart cycle, normal form) on a
    large matrix; the library times every 4th step's pair with HIP events."""
    import torch
    from paper_2407_04634_amd import Context, PREC_FP64, PREC_MIXED
    from workloads import generators as G

    c = G.config(name)
    ctx = Context(torch.from_numpy(c.rowptr).cuda(), torch.from_numpy(c.colind).cuda(),
                  torch.from_numpy(c.vals).cuda(), c.m, c.n,
                  D=torch.from_numpy(G.perturbation_diagonal(c.n, 1)).cuda(),
                  Omega=torch.from_numpy(np.ascontiguousarray(G.gaussian_start_block(c.n, d, 1))).cuda(),
                  eps=1e-3, d=d, max_dim=max_dim, prec=PREC_MIXED if prec == "mixed" else PREC_FP64,
                  max_cycles=1, refine=0, profile=1)
    st = ctx.lanczos_run(allow_noconv=True)
    ctx.close()
    esize = 4 if prec == "mixed" else 8
    a_b, at_b = spmv_bytes(c.m, c.n, c.nnz, d, esize, False)
    t = st["t_spmv_a_us"] + st["t_spmv_at_us"]
    gbs = (a_b + at_b) / (t * 1e-6) / 1e9
    return {"workload": name, "form": "B = A^T A + eps D", "m": c.m, "n": c.n, "nnz": c.nnz, "d": d,
            "prec": prec, "samples": st["spmv_samples"], "us_A": st["t_spmv_a_us"],
            "us_AT": st["t_spmv_at_us"], "bytes_pair": a_b + at_b, "achieved_gbs": gbs,
            "frac_hbm": gbs / HBM_PEAK_GBS}


def leg_gather(name="zipf4m", reps=20):
    """Reference rates for the streaming SpMV's two access streams on the
    pattern its kernel sees (the library's locality order): a pure gather
    x[colind] (torch index_select, FP32 and FP64 x, int32 indices) and a plain
    copy of the CSR stream's bytes (torch copy_).  The SpMV needs both; the
    faster of the two references is a floor for its time."""
    import torch
    from paper_2407_04634_amd import locality_order
    from workloads import generators as G

    c = G.config(name)
    ro, co = locality_order(c.rowptr, c.colind, c.m, c.n)
    inv = np.empty(c.n, dtype=np.int32)
    inv[co] = np.arange(c.n, dtype=np.int32)
    lens = np.diff(c.rowptr)[ro]
    starts = c.rowptr[:-1][ro]
    take = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) + np.arange(c.nnz)
    ci = torch.from_numpy(inv[c.colind[take]]).cuda()
    del take

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    out = {"workload": name, "nnz": c.nnz, "n": c.n, "order": "library locality order"}
    for tag, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        x = torch.randn(c.n, dtype=dt, device="cuda")
        y = torch.empty(c.nnz, dtype=dt, device="cuda")
        us = timed(lambda: torch.index_select(x, 0, ci, out=y))
        out[f"gather_{tag}_us"] = us
        out[f"gather_{tag}_gnnz_per_s"] = c.nnz / (us * 1e-6) / 1e9
        nbytes = c.nnz * (4 + x.element_size())
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        us_c = timed(lambda: dst.copy_(src))
        out[f"stream_copy_{tag}_us"] = us_c
        out[f"stream_copy_{tag}_bytes"] = nbytes
        del x, y, src, dst
    return out


def leg_stream(gib=8, reps=10):
    """Reference rates of plain streaming on this GPU for the HBM-bound kernels'
    rooflines: a read-only pass (torch.sum over a resident buffer, FP32 and
    FP64) and a copy (read + write), each over ``gib`` GiB, best of ``reps``."""
    import torch

    n = (gib << 30) // 4
    out = {"bytes": gib << 30}
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for tag, fn, nbytes in (("read_fp32", lambda: src.sum(), gib << 30),
                            ("read_fp64", lambda: src.view(torch.float64).sum(), gib << 30),
                            ("copy", lambda: dst.copy_(src), 2 * (gib << 30))):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        out[f"{tag}_gbs"] = nbytes / best / 1e9
    del src, dst
    return out


def leg_table1():
    """The introduction's diagonal example (Sec. 1, Eq. "matrixA", Table "tabintro").

    Plain block Lanczos on A (D = 0, so B = A; reorthogonalisation at every
    step; 1024 products; Ritz values below 3 eps = 1e-4 counted) for each
    block size the library supports, next to the paper's printed dimensions;
    then the method itself (D uniform, eps = 0.1 * 1.0001, Krylov dimension
    128, d = 1 and 4) with the sine of the largest principal angle to
    span(e_1..e_64)."""
    import torch
    from paper_2407_04634_amd import Context, OP_SYM
    from workloads import generators as G

    c = G.config("diag10064")
    z = c.meta["n_zero"]
    dev = (torch.from_numpy(c.rowptr).cuda(), torch.from_numpy(c.colind).cuda(),
           torch.from_numpy(c.vals).cuda())
    paper = dict(zip((1, 2, 4, 8, 16, 32, 64), (45, 46, 48, 48, 48, 64, 64)))
    out = {"workload": "diag10064", "unperturbed": [], "method": []}
    for d in (1, 2, 4, 8):
        om = torch.from_numpy(np.ascontiguousarray(G.gaussian_start_block(c.n, d, 1))).cuda()
        ctx = Context(*dev, c.m, c.n, D=torch.zeros(c.n, dtype=torch.float64, device="cuda"), Omega=om,
                      eps=1e-4 / 3, d=d, max_dim=1024, max_matvec=1024, ro_tol=1e-300, refine=0, op=OP_SYM)
        st = ctx.lanczos_run(allow_noconv=True)
        ctx.close()
        out["unperturbed"].append({"d": d, "dimension": st["nullity"], "paper": paper[d],
                                   "matvecs": st["matvecs"]})
    for d in (1, 4):
        om = torch.from_numpy(np.ascontiguousarray(G.gaussian_start_block(c.n, d, 1))).cuda()
        ctx = Context(*dev, c.m, c.n, D=torch.from_numpy(G.perturbation_diagonal(c.n, 1)).cuda(), Omega=om,
                      eps=0.1 * 1.0001, d=d, max_dim=128, max_matvec=20_000, op=OP_SYM)
        t0 = time.perf_counter()
        st = ctx.lanczos_run()
        t1 = time.perf_counter()
        v = np.linalg.qr(ctx.extract_basis().cpu().numpy())[0]
        ctx.close()
        # with orthonormal V the sine of the largest principal angle to
        # span(e_1..e_64) is the 2-norm of V's rows outside the first 64
        out["method"].append({"d": d, "nullity": st["nullity"], "matvecs": st["matvecs"], "s": t1 - t0,
                              "sin_angle": float(np.linalg.norm(v[z:, :], 2)) if v.shape[1] else None})
    return out


def leg_backward(ctx_args):
    """Backward pass at the planted50k size: L = ||P X||_F^2, X seeded n x 8."""
    import torch
    from paper_2407_04634_amd import Context
    from workloads import generators as G

    c = G.config("planted50k")
    ctx = Context(torch.from_numpy(c.rowptr).cuda(), torch.from_numpy(c.colind).cuda(),
                  torch.from_numpy(c.vals).cuda(), c.m, c.n,
                  D=torch.from_numpy(G.perturbation_diagonal(c.n, 1)).cuda(),
                  Omega=torch.from_numpy(np.ascontiguousarray(G.gaussian_start_block(c.n, 1, 1))).cuda(),
                  eps=2e-6, d=1, max_dim=1024, tol_angle=1e-9, tol_rel_resid=1e-10, **ctx_args)
    st = ctx.lanczos_run()
    v = ctx.extract_basis().contiguous()
    x = torch.from_numpy(np.ascontiguousarray(G.gaussian_matrix(c.n, 8, seed=5))).cuda()
    dldv = 2.0 * (x @ (x.T @ v))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grad, iters = ctx.backward(dldv, tol=1e-10)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # new values for the same pattern (an optimisation loop's next step): the
    # same values again, so the cost is the refresh alone (the basis is dropped)
    va = torch.from_numpy(c.vals).cuda()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.update_values(va)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ctx.close()
    return {"workload": "planted50k", "loss": "||P X||_F^2, X seeded N(0,1) n x 8", "nullity": st["nullity"],
            "cg_iters": iters, "s": t1 - t0, "finite": bool(torch.isfinite(grad).all()),
            "update_values_ms": (t3 - t2) * 1e3}


def leg_precond(name="planted20k_scaled", eps_pre=3.4e-8, eps_plain=2.2e-8, budget_factor=5):
    """Outer preconditioning with the diagonal P_R (Sec. 4.4) against none.

    A planted matrix whose columns are scaled over two decades (A S, S
    diagonal): the Jacobi P_R undoes the scaling.  eps is 0.1 sigma_min^2 of
    the matrix each run iterates with (A P_R^{-T}: sigma^2 ~ 3.4e-7; A S:
    sigma^2 ~ 2.2e-7).  The preconditioned solve is refined and checked
    against the closed-form null space S^{-1} range([-R; I]); the plain one
    gets budget_factor times the preconditioned run's matvecs (no refinement)
    and reports how much of the null space it found."""
    import torch
    from paper_2407_04634_amd import Context, PRECOND_JACOBI, PRECOND_NONE
    from workloads import generators as G

    c = G.config(name)
    r = c.meta["R"].toarray()
    v0 = np.vstack([-r, np.eye(r.shape[1])]) / c.meta["col_scale"][:, None]  # null(A S) = S^-1 null(A)
    v0 = torch.from_numpy(np.linalg.qr(v0)[0]).cuda()
    dev = (torch.from_numpy(c.rowptr).cuda(), torch.from_numpy(c.colind).cuda(), torch.from_numpy(c.vals).cuda())
    dv = torch.from_numpy(G.perturbation_diagonal(c.n, 1)).cuda()
    om = torch.from_numpy(np.ascontiguousarray(G.gaussian_start_block(c.n, 1, 1))).cuda()
    runs = []
    budget = 20_000_000
    for pre in ("jacobi", "none"):
        jac = pre == "jacobi"
        kw = dict(eps=eps_pre, max_dim=512, refine=1, max_matvec=budget) if jac else \
            dict(eps=eps_plain, max_dim=1024, refine=0, max_matvec=budget)
        ctx = Context(*dev, c.m, c.n, D=dv, Omega=om, d=1, tol_angle=1e-9, tol_rel_resid=1e-10,
                      precond=PRECOND_JACOBI if jac else PRECOND_NONE, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.lanczos_run(allow_noconv=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        v = ctx.extract_basis().contiguous()
        sine = None
        if v.shape[1] == v0.shape[1]:
            q = torch.linalg.qr(v)[0]
            sine = float(torch.linalg.matrix_norm(q - v0 @ (v0.T @ q), ord=2))
        runs.append({"precond": pre, "s": t1 - t0, "status": st["status"], "nullity": st["nullity"],
                     "matvecs": st["matvecs"], "eps": kw["eps"], "max_dim": kw["max_dim"],
                     "theta_next": st["theta_next"], "refine_iters": st["refine_iters"], "max_sin_angle": sine,
                     "rel_resid_fro": st["rel_resid_fro"] if jac else None,
                     "valid": bool(jac and st["nullity"] == v0.shape[1] and sine is not None
                                   and sine <= 1e-8 and st["rel_resid_fro"] <= 1e-8)})
        log(f"precond {json.dumps(runs[-1])}")
        ctx.close()
        if jac:
            budget = budget_factor * st["matvecs"]
    return {"workload": name, "n": c.n, "nnz": c.nnz, "nullity": int(v0.shape[1]),
            "desc": "planted A=[B, BR] (n=20000, nullity 50) times a diagonal S with log10 S ~ U[-1, 1]",
            "runs": runs}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed restart cycles of the mixed solve")
    ap.add_argument("--warmup", type=int, default=5, help="restart cycles before the timed ones")
    ap.add_argument("--workload", default="zipf4m", choices=sorted(WORKLOADS))
    ap.add_argument("--precs", default="mixed,fp64",
                    help="precisions to solve in, the first one carries the headline")
    ap.add_argument("--d", type=int, default=1)
    ap.add_argument("--max-dim", type=int, default=0)
    ap.add_argument("--eps", type=float, default=0.0)
    ap.add_argument("--max-matvec", type=int, default=2_000_000)
    ap.add_argument("--max-cycles", type=int, default=0,
                    help="stop after this many restart cycles (profiling runs; not valid)")
    ap.add_argument("--no-refine", action="store_true", help="skip the FP64 refinement (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="",
                    help="comma-separated extra measurements: spmv (streaming SpMV pair on the 4M-vertex "
                         "Laplacian and the 1M-point coboundary, normal form), gather (pure gather and streaming-copy "
                         "references on the workload's pattern), backward (planted50k), table1 (the introduction's "
                         "diagonal example: plain block Lanczos vs the method), precond (Jacobi P_R vs none on the "
                         "column-scaled 20k planted matrix), stream (plain read and copy "
                         "rates over 8 GiB; also run when no leg is named)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain copy that scales the rocprofv3 byte counters")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described, not implemented)", file=sys.stderr)
        sys.exit(2)
    os.environ.setdefault("NSP_VERBOSE", "1")  # the library's per-cycle progress lines

    import torch
    from workloads import generators as G

    wl = WORKLOADS[args.workload]
    max_dim = args.max_dim or wl["max_dim"]
    eps = args.eps or wl["eps"]
    precs = args.precs.split(",")
    t0 = time.perf_counter()
    c = G.config(*wl["gen"])
    log(f"workload {args.workload}: m={c.m} n={c.n} nnz={c.nnz} generated in "
        f"{time.perf_counter() - t0:.1f} s")
    dev = (torch.from_numpy(c.rowptr).cuda(), torch.from_numpy(c.colind).cuda(),
           torch.from_numpy(c.vals).cuda(), torch.from_numpy(G.perturbation_diagonal(c.n, 1)).cuda(),
           torch.from_numpy(np.ascontiguousarray(G.gaussian_start_block(c.n, args.d, 1))).cuda())
    runs, stats, cycles = {}, {}, {}
    for prec in precs:
        runs[prec], stats[prec], cycles[prec] = solve(c, dev, wl, prec, args.d, max_dim, eps, args, prec)
    head = precs[0]
    rec, st, cyc = runs[head], stats[head], cycles[head]
    w = min(args.warmup, max(0, len(cyc) - 1))
    timed = cyc[w:w + args.steps]
    ms = 1e3 * sum(timed) / max(1, len(timed))

    esize = 4 if head == "mixed" else 8
    sym = wl["op"] == "sym"
    stream = c.nnz >= 1 << 21
    kr = {p: kernel_rows(stats[p], c.m, c.n, c.nnz, args.d, 4 if p == "mixed" else 8, sym, stream)
          for p in precs}
    line = {
        "metric": "null vectors/s at ||AV||_F<=1e-8||A||_F (exact nullity, sin angle<=1e-8), "
                  + " vs ".join(precs),
        "value": rec["null_vectors_per_s"],
        "unit": "null vectors/s",
        "n_gpus": 1,
        "steps": len(timed),
        "warmup": w,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic, seeded",
        "config": {"workload": wl["desc"], "name": args.workload,
                   "operator": "B = L + eps D (symmetric form, Sec. 5.1)" if sym else "B = A^T A + eps D",
                   "d": args.d, "max_dim": max_dim, "eps": eps, "precision": head,
                   "step": "one restart cycle of the mixed solve (Lanczos steps + Rayleigh-Ritz + restart)"},
        "valid": all(runs[p]["valid"] for p in precs),
        "solves": runs,
        "speedup_vs_fp64": (runs["fp64"]["solve_s"] / runs["mixed"]["solve_s"]
                            if "fp64" in runs and "mixed" in runs else None),
        "cycles": {"count": len(cyc), "timed_s": timed},
    }
    if kr[head]:
        dom, frac = dominant(kr[head], st, args.d)
        tr = TRAFFIC.get((args.workload, args.d, head, dom["kernel"].split()[0]))
        line["roofline"] = {"kernel": dom["kernel"], "bound": "hbm", "achieved": dom["achieved_gbs"],
                            "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": dom["achieved_gbs"] / HBM_PEAK_GBS,
                            "traffic": tr["ratio"] * dom["bytes_per_launch"] if tr else None,
                            "avg_us": dom["avg_us"], "bytes_per_launch": dom["bytes_per_launch"],
                            "launches": ("per launch that reorthogonalised" if "ts_" in dom["kernel"]
                                         else "per launch")}
        line["reorth_active_frac"] = frac
        # sampled steps whose W flag was clear: the projection and update
        # launches there return at once; their summed time per such step
        idle = st["ro_samples"] - st["ro_active"]
        line["reorth_idle_launch_us"] = st["ro_idle_ms"] * 1e3 / idle if idle > 0 else None
        line["kernels"] = kr
        line["spmv_hbm"] = [dict(r, prec=p, workload=args.workload) for p in precs for r in kr[p]
                            if r["kernel"].startswith("k_csr") or r["kernel"].startswith("k_spmm")]
    legs = [x for x in args.legs.split(",") if x]
    if "spmv" in legs:
        line["spmv_normal_form"] = [leg_spmv(w_, p) for w_ in ("zipf4m", "coboundary1m")
                                    for p in ("fp64", "mixed")]
        for r in line["spmv_normal_form"]:
            log(f"spmv {json.dumps(r)}")
    if "gather" in legs:
        line["gather_reference"] = leg_gather(args.workload)
        log(f"gather {json.dumps(line['gather_reference'])}")
    if "stream" in legs or not legs:  # cheap (a few seconds): part of the default run
        line["stream_reference"] = leg_stream()
        log(f"stream {json.dumps(line['stream_reference'])}")
    if "precond" in legs:
        line["precond_vs_plain"] = leg_precond()
    if "table1" in legs:
        line["table1"] = leg_table1()
        log(f"table1 {json.dumps(line['table1'])}")
    if "backward" in legs:
        line["backward"] = leg_backward({})
        log(f"backward {json.dumps(line['backward'])}")
    if not args.no_cpu_baseline:
        na = st.get("ro_active", 0)
        k_avg = (st["ro_tn_bytes"] / na / esize - 2 * args.d * c.n) / c.n if na else max_dim
        log("cpu baseline (oracle on the host, bounded sample)")
        line["cpu_baseline"] = cpu_baseline(c, wl, eps, args.d, max_dim, rec, k_avg)
    log(f"done in {time.perf_counter() - t0:.1f} s")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
