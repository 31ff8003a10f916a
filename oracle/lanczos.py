"""Randomized small-block Lanczos on B = A^T A + eps D (oracle; test infrastructure only).

Two routines, written from the paper in its notation (blocks Q_j of width d,
diagonal blocks Xi_j, subdiagonal blocks Gamma_j, kept Ritz values Theta and
coupling block F):

* :func:`algorithm1` -- Algorithm 1 (Sec. 1.2): ell block-Lanczos steps with
  full reorthogonalisation (classical Gram-Schmidt, twice, against every
  previous block), Rayleigh-Ritz on T_ell, nullity N = #{theta < 3 eps}
  (Remark "cormain").
* :func:`algorithm2` -- Algorithm 2 (Sec. 4.3): thick restart (Sec. 4.1),
  partial reorthogonalisation driven by the W-recurrence (Sec. 4.2),
  adaptive nullity and the convergence-speed stopping rule (Sec. 4.3).

Readings taken where the paper is silent, garbled or inconsistent (each is
listed with its justification in the design notes):

  R1  restart size: k_keep = d * floor((N_ell + dimK) / (2 d)) vectors,
      clamped to [d, dimK - 2d]; ell_0 = k_keep / d blocks.
  R2  the three-term recurrence subtracts Q_{ell-1} Gamma_{ell-1}^T (the
      transpose printed in Eq. "laniterfp"; identical for d = 1).
  R3  for kept blocks k <= ell_0 the coupling is B Q_k = Q_k Theta_k +
      Q_{ell_0+1} F_k, so the first W case reads
      w_{k,l+1} = |G_l^-1| (w_{k,l}(|Theta_k|+|Xi_l|) + w_{l0+1,l}|F_k|
                             + w_{k,l-1}|G_{l-1}| + 2 u_d).
  R4  W next to the diagonal: w_{l,l+1} = u_d (local orthogonality from the
      explicit subtraction of Q_l Xi_l); for k = l-1 the pair
      w_{k+1,l}|G_k| + w_{k,l-1}|G_{l-1}| cancels exactly in the derivation
      (the Q_{l-1} coupling is subtracted explicitly) and is dropped.
  R5  "reorthogonalize" in the partial reorthogonalisation events = one
      pass of classical Gram-Schmidt against Z_{ell-1}, accepted by the
      Kahan-Parlett criterion ("twice is enough", Parlett, The Symmetric
      Eigenvalue Problem, Sec. 6.9; the paper cites Parlett for the
      round-off model of Sec. 4.2): a projected vector that keeps at least
      1/sqrt(2) of its norm is orthogonal to the basis to working accuracy
      after one pass, and a second pass is needed only when the projection
      cancelled more.  At a flagged step the W bound sits just above
      u_RO = sqrt(u), so a unit Lanczos vector loses a fraction of order
      k u_RO^2 of its squared norm and the criterion holds with a wide
      margin; it is checked anyway, and a violation (the W bound failed)
      stops the run.  The first step of a cycle and the restart (components
      of order ||B|| or 1) use classical Gram-Schmidt twice (CGS2).
  R6  QR = orthonormal factor with positive-diagonal triangular factor (the
      unique thin QR of a full-rank block); d = 1 is normalisation.
  R7  ||B|| in u_d: ||A||_1 ||A||_inf + eps in the first cycle, then the
      largest Ritz value.
  R8  u = 2^-52 (the value quoted in Sec. 5.3); u_RO = sqrt(u).
  R9  block norms in the W-recurrence are Frobenius norms (upper bounds of
      the spectral norms, so W stays an upper bound); |G_l^-1| is the
      Frobenius norm of the inverse triangular factor.
  R10 stopping rule (s = matvecs needed for d newly converged Ritz values):
      at each restart record (matvecs, N_ell).  Starting at the first
      increase of N_ell, an interval closes at the first later restart where
      N_ell has grown by at least d; it gives the sample
      (matvecs spent) * d / (growth).  s = 2 * max sample; stop once a sample
      exists and more than s matvecs passed since the last increase.  The
      stretch before the first increase is not a sample: the first Ritz
      value only has to separate the perturbed-zero cluster from the rest of
      the spectrum, the later ones must also resolve the cluster, so it
      under-estimates s.  Without a sample the run goes to the matvec budget,
      unless R12 applies.
  R11 the restart's coupling block is F = R Gamma_ell V_Z(last d rows, 1:k_keep),
      where R (~ I) is the triangular factor of re-orthonormalising Q_{ell+1}
      against the new Z_{ell_0}; the printed "[O, Gamma_{ell_0}] V_Z" drops
      Gamma_ell (Sec. 4.1 derives F = E_{ell+1} V_Z with E_{ell+1} = [0, Gamma_ell]).
  R12 with N_ell = 0, stop once the smallest Ritz value has converged above
      3 eps (see nothing_below).
"""
from __future__ import annotations

import math

import numpy as np

from .operator import operator

U = 2.0 ** -52


def block_qr(p: np.ndarray):
    """Thin QR with positive diagonal R (reading R6)."""
    q, r = np.linalg.qr(p)
    s = np.sign(np.diag(r)).copy()
    s[s == 0] = 1.0
    return q * s[None, :], r * s[:, None]


def cgs1(z: np.ndarray, p: np.ndarray) -> np.ndarray:
    """(I - Z Z^T) P by one pass of classical Gram-Schmidt (reading R5)."""
    if z.shape[1] == 0:
        return p
    return p - z @ (z.T @ p)


KAHAN_PARLETT = 1.0 / math.sqrt(2.0)


def cgs1_accepted(z: np.ndarray, p: np.ndarray) -> np.ndarray:
    """One classical Gram-Schmidt pass of the unit columns of P, checked by the
    Kahan-Parlett criterion (reading R5): every projected column must keep at
    least 1/sqrt(2) of its norm, else one pass is not enough."""
    out = cgs1(z, p)
    kept = np.linalg.norm(out, axis=0) / np.linalg.norm(p, axis=0)
    if np.any(kept < KAHAN_PARLETT):
        raise RuntimeError("partial reorthogonalisation: one Gram-Schmidt pass removed more than "
                           "1 - 1/sqrt(2) of a vector's norm (the W bound failed)")
    return out


def cgs2(z: np.ndarray, p: np.ndarray) -> np.ndarray:
    """(I - Z Z^T) P by classical Gram-Schmidt applied twice (reading R5)."""
    if z.shape[1] == 0:
        return p
    p = p - z @ (z.T @ p)
    p = p - z @ (z.T @ p)
    return p


def _fro(x) -> float:
    return float(np.linalg.norm(np.atleast_2d(x)))


def _inv_fro(g: np.ndarray) -> float:
    return _fro(np.linalg.inv(np.atleast_2d(g)))


# ---------------------------------------------------------------------------
# Algorithm 1
# ---------------------------------------------------------------------------
def algorithm1(a, eps: float, dvec: np.ndarray, omega: np.ndarray, ell: int, op: str = "normal"):
    """Algorithm 1 with full reorthogonalisation.

    Returns dict(V, theta, N, Z, T, Q_next, Gamma_last) with V = Z_ell V_Z(:, 1:N)
    and N = #{theta < 3 eps}.  ``op`` selects B = A^T A + eps D ('normal') or
    B = A + eps D ('sym', A symmetric positive semi-definite).
    """
    apply_b, _ = operator(op)
    n, d = omega.shape
    q1, _ = block_qr(omega)
    blocks = [q1]
    xis, gams = [], []
    for j in range(ell):
        qj = blocks[-1]
        p = apply_b(a, eps, dvec, qj)
        if j > 0:
            p = p - blocks[-2] @ gams[-1].T
        xi = qj.T @ p
        p = p - qj @ xi
        p = cgs2(np.hstack(blocks), p)
        qn, g = block_qr(p)
        xis.append(0.5 * (xi + xi.T))
        gams.append(g)
        blocks.append(qn)
    t = np.zeros((ell * d, ell * d))
    for j in range(ell):
        t[j * d:(j + 1) * d, j * d:(j + 1) * d] = xis[j]
        if j + 1 < ell:
            t[(j + 1) * d:(j + 2) * d, j * d:(j + 1) * d] = gams[j]
            t[j * d:(j + 1) * d, (j + 1) * d:(j + 2) * d] = gams[j].T
    z = np.hstack(blocks[:ell])
    theta, vz = np.linalg.eigh(t)
    nul = int(np.sum(theta < 3.0 * eps))
    return dict(V=z @ vz[:, :nul], theta=theta, N=nul, Z=z, T=t, Q_next=blocks[ell],
                Gamma_last=gams[-1])


# ---------------------------------------------------------------------------
# Algorithm 2
# ---------------------------------------------------------------------------
class _WRecurrence:
    """Upper bounds w_{k,j} >= ||Q_k^T Q_j|| (Sec. 4.2), blocks numbered from 1."""

    def __init__(self, nblocks: int):
        self.w = np.zeros((nblocks + 2, nblocks + 2))

    def reset_column(self, j: int, u_d: float):
        self.w[1:j, j] = u_d

    def next_column(self, ell, l0, u_d, n_theta, n_f, n_xi, n_gam, gi):
        """Column ell+1 from columns ell and ell-1 (readings R3, R4)."""
        w = self.w
        col = np.zeros(ell + 1)
        sum_f = sum(w[i, ell] * n_f[i] for i in range(1, l0 + 1))
        for k in range(1, ell + 1):
            if k == ell:
                col[k] = u_d
            elif k <= l0:
                col[k] = gi * (w[k, ell] * (n_theta[k] + n_xi[ell]) + w[l0 + 1, ell] * n_f[k]
                               + w[k, ell - 1] * n_gam[ell - 1] + 2 * u_d)
            elif k == l0 + 1:
                acc = w[k, ell] * (n_xi[k] + n_xi[ell]) + sum_f + 2 * u_d
                if k < ell - 1:
                    acc += w[k + 1, ell] * n_gam[k] + w[k, ell - 1] * n_gam[ell - 1]
                col[k] = gi * acc
            else:
                acc = w[k, ell] * (n_xi[k] + n_xi[ell]) + w[k - 1, ell] * n_gam[k - 1] + 2 * u_d
                if k < ell - 1:
                    acc += w[k + 1, ell] * n_gam[k] + w[k, ell - 1] * n_gam[ell - 1]
                col[k] = gi * acc
        w[1:ell + 1, ell + 1] = col[1:]
        return float(col[1:ell].max()) if ell > 1 else 0.0


def _assemble_t(theta_kept, f, xis, gams, l0, nblocks, d):
    """Block tridiagonal T with the arrowhead [Theta, F^T; F, Xi_{l0+1}] (Eq. "defT")."""
    kk = l0 * d
    t = np.zeros((nblocks * d, nblocks * d))
    if kk:
        t[np.arange(kk), np.arange(kk)] = theta_kept
        t[kk:kk + d, :kk] = f
        t[:kk, kk:kk + d] = f.T
    for j in range(l0 + 1, nblocks + 1):
        r = (j - 1) * d
        t[r:r + d, r:r + d] = xis[j]
        if j < nblocks:
            t[r + d:r + 2 * d, r:r + d] = gams[j]
            t[r:r + d, r + d:r + 2 * d] = gams[j].T
    return t


def coupling_block(r: np.ndarray, gamma_last: np.ndarray, vz: np.ndarray, dim_k: int, d: int,
                   k_keep: int) -> np.ndarray:
    """F = R Gamma_ell V_Z(last d rows, 1:k_keep) (Sec. 4.1, reading R11).

    Multiplying B Z_ell = Z_ell T_ell + Q_{ell+1} [0, Gamma_ell] by the kept Ritz
    vectors V_Z(:, 1:k_keep) leaves Q_{ell+1} Gamma_ell V_Z(last d rows, :) as
    the residual; Q_{ell+1} = Q_{ell_0+1} R + Z_{ell_0} (...) turns it into
    Q_{ell_0+1} F.
    """
    return r @ gamma_last @ vz[dim_k - d:dim_k, :k_keep]


def restart_size(n_ell: int, dim_k: int, d: int) -> int:
    """Reading R1."""
    k_keep = d * ((n_ell + dim_k) // (2 * d))
    return int(min(max(k_keep, d), dim_k - 2 * d))


def speed_rule(history, d: int):
    """Reading R10: returns (stop, s) from the restart history [(matvecs, N_ell), ...]."""
    events = []
    best = 0
    for mv, nl in history:
        if nl > best:
            events.append((mv, nl))
            best = nl
    samples = []
    if events:
        start = events[0]
        for mv, nl in events[1:]:
            if nl - start[1] >= d:
                samples.append((mv - start[0]) * d / (nl - start[1]))
                start = (mv, nl)
    if not samples:
        return False, math.inf
    s = 2.0 * max(samples)
    return (history[-1][0] - events[-1][0]) > s, s


def nothing_below(theta, ritz_res, eps: float) -> bool:
    """Reading R12: no Ritz value below 3 eps and the smallest one converged above it.

    With N_ell = 0 the speed rule never gets a sample.  Sec. 4.3 names the
    simpler idea of stopping once an unwanted Ritz value above 3 eps has
    converged; here only for that case: theta_1 has residual r_1 <= eps and
    theta_1 - r_1 >= 3 eps, so an eigenvalue of B lies in
    [theta_1 - r_1, theta_1 + r_1], above the nullity threshold.
    """
    if len(theta) == 0 or theta[0] < 3.0 * eps:
        return False
    return bool(ritz_res[0] <= eps and theta[0] - ritz_res[0] >= 3.0 * eps)


def algorithm2(a, eps: float, dvec: np.ndarray, omega: np.ndarray, dim_k: int,
               max_matvec: int = 10 ** 7, ro_tol: float | None = None, full_reorth: bool = False,
               track_orth: bool = False, max_cycles: int | None = None, op: str = "normal"):
    """Algorithm 2: restarted randomized small-block Lanczos with partial reorthogonalisation.

    Returns dict(V, N, theta, matvecs, restarts, reorths, history, converged,
    orth_trace) where V = Z_ell V_Z(:, 1:N_ell) from the final cycle.  ``op`` as
    in algorithm1.
    ``track_orth`` records max_k ||Q_k^T Q_{ell+1}|| (true value) next to the W
    bound at every step, for testing that the bound holds.
    """
    n, d = omega.shape
    if dim_k % d or dim_k < 3 * d:
        raise ValueError("dim_k must be a multiple of d and at least 3d")
    nb = dim_k // d
    u_ro = math.sqrt(U) if ro_tol is None else ro_tol
    apply_b, norm_bound = operator(op)
    norm_b = norm_bound(a) + eps * float(np.max(dvec))
    u_d = d * math.sqrt(n) * U * norm_b

    zb = np.zeros((n, dim_k + d))
    zb[:, :d], _ = block_qr(omega)
    l0 = 0
    theta_kept = np.zeros(0)
    f = np.zeros((d, 0))
    matvecs = restarts = reorths = 0
    history = []
    orth_trace = []
    bop = lambda x: apply_b(a, eps, dvec, x)  # noqa: E731

    while True:
        xis, gams = {}, {}
        wrec = _WRecurrence(nb + 1)
        kk = l0 * d
        # ---- first step of the cycle: Q' = B Q_{l0+1}, Xi, QR of the projected Q'
        qa = zb[:, kk:kk + d]
        p = bop(qa)
        matvecs += d
        xis[l0 + 1] = qa.T @ p
        xis[l0 + 1] = 0.5 * (xis[l0 + 1] + xis[l0 + 1].T)
        p = cgs2(zb[:, :kk + d], p)
        qn, g = block_qr(p)
        gams[l0 + 1] = g
        zb[:, kk + d:kk + 2 * d] = qn
        wrec.reset_column(l0 + 1, u_d)
        wrec.reset_column(l0 + 2, u_d)
        # block norms used by the W-recurrence (reading R9)
        n_theta = {k: float(np.max(np.abs(theta_kept[(k - 1) * d:k * d]))) for k in range(1, l0 + 1)}
        n_f = {k: _fro(f[:, (k - 1) * d:k * d]) for k in range(1, l0 + 1)}
        n_xi = {l0 + 1: _fro(xis[l0 + 1])}
        n_gam = {l0 + 1: _fro(gams[l0 + 1])}
        # ---- Lanczos steps ell = l0+2 .. nb
        for ell in range(l0 + 2, nb + 1):
            c = (ell - 1) * d
            ql = zb[:, c:c + d]
            p = bop(ql) - zb[:, c - d:c] @ gams[ell - 1].T
            matvecs += d
            xi = ql.T @ p
            qn, g = block_qr(p - ql @ xi)
            if full_reorth:
                qn, g2 = block_qr(cgs2(zb[:, :c + d], qn))
                g = g2 @ g
            zb[:, c + d:c + 2 * d] = qn
            xis[ell] = 0.5 * (xi + xi.T)
            gams[ell] = g
            n_xi[ell] = _fro(xis[ell])
            n_gam[ell] = _fro(g)
            wmax = wrec.next_column(ell, l0, u_d, n_theta, n_f, n_xi, n_gam, _inv_fro(g))
            if track_orth:
                true = float(np.max(np.abs(zb[:, :c + d].T @ zb[:, c + d:c + 2 * d])))
                orth_trace.append((ell, wmax, true))
            if not full_reorth and wmax > u_ro:
                # reorthogonalise Q_ell and Q_{ell+1} against Z_{ell-1} (Sec. 4.2)
                blk = cgs1_accepted(zb[:, :c], zb[:, c:c + 2 * d])
                qlr, _ = block_qr(blk[:, :d])
                qnr, _ = block_qr(cgs1(qlr, blk[:, d:]))
                zb[:, c:c + d] = qlr
                zb[:, c + d:c + 2 * d] = qnr
                wrec.reset_column(ell, u_d)
                wrec.reset_column(ell + 1, u_d)
                reorths += 1
        # ---- Rayleigh-Ritz on T_ell (Alg. 2, after the inner loop)
        t = _assemble_t(theta_kept, f, xis, gams, l0, nb, d)
        theta, vz = np.linalg.eigh(t)
        n_ell = int(np.sum(theta < 3.0 * eps))
        history.append((matvecs, n_ell))
        # residual norm of each Ritz pair: ||Gamma_last V_Z(last d rows, i)||
        ritz_res = np.linalg.norm(gams[nb] @ vz[dim_k - d:dim_k, :], axis=0)
        stop, _ = speed_rule(history, d)
        stop = stop or nothing_below(theta, ritz_res, eps)
        out_of_budget = matvecs >= max_matvec or (max_cycles is not None and restarts + 1 >= max_cycles)
        if stop or out_of_budget:
            v = zb[:, :dim_k] @ vz[:, :n_ell]
            # the last cycle's Lanczos decomposition B Z = Z T + Q_next [0, Gamma_last]
            # (Eq. "laniter"), returned for the invariant checks of the tests
            return dict(V=v, N=n_ell, theta=theta, matvecs=matvecs, restarts=restarts,
                        reorths=reorths, history=history, converged=bool(stop),
                        orth_trace=orth_trace, u_d=u_d, Z=zb[:, :dim_k].copy(), T=t,
                        Q_next=zb[:, dim_k:dim_k + d].copy(), Gamma_last=gams[nb], l0=l0,
                        ritz_res=ritz_res)
        # ---- thick restart (Sec. 4.1)
        k_keep = restart_size(n_ell, dim_k, d)
        if n_ell > k_keep:
            raise RuntimeError("dim_k too small for the detected nullity")
        z_new = zb[:, :dim_k] @ vz[:, :k_keep]
        q_last = zb[:, dim_k:dim_k + d]
        qn, r = block_qr(cgs2(z_new, q_last))
        f = coupling_block(r, gams[nb], vz, dim_k, d, k_keep)
        theta_kept = theta[:k_keep].copy()
        zb[:, :k_keep] = z_new
        zb[:, k_keep:k_keep + d] = qn
        l0 = k_keep // d
        restarts += 1
        norm_b = float(np.max(theta))  # reading R7
        u_d = d * math.sqrt(n) * U * norm_b
