"""Oracle: block flexible Arnoldi / block FGMRES-Sh for several right-hand sides.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

The paper solves each right-hand side with its own basis and notes that block
methods for multiple right-hand sides extend the approach (section 5, closing
remark on multiple right-hand sides; section 7).  This module states that
extension plainly, as the block analogue of Algorithms 3 and 4:

* start: B = V_1 beta, a QR factorisation of the n x s right-hand-side block
  (beta s x s upper triangular; the diagonal of every triangular factor here is
  made real and non-negative, which fixes the factorisation of a full-rank
  block uniquely);
* step k: Z_k ~ (K + tau_k M)^{-1} V_k column by column (the inner solves of
  section 4), W = M Z_k, block modified Gram-Schmidt H_ik = V_i^H W,
  W -= V_i H_ik (i = 1..k), then W = V_{k+1} H_{k+1,k} (QR).  This gives the
  block form of eq. arnoldimod, M Z_m = V_{m+1} Hbar_m, with Hbar_m block upper
  Hessenberg ((m+1)s x ms), and of eq. zmvmrelation, K Z_k + tau_k M Z_k =
  V_k - P_k (P_k the inner residuals), hence for every shift
      (K + sigma M) Z_m = V_{m+1} Hbar(sigma;T) - P_m,
      Hbar(sigma;T) = [I;0] + Hbar_m (sigma I - T),  T = diag(tau_k I_s)
  (eq. shiftedarnoldimod with identity blocks);
* per shift and right-hand side r: y = argmin ||E_1 beta e_r - Hbar(sigma;T) y||
  (the GMRES projected problem of Algorithm 4, one column of the block least
  squares), x = Z_m y;
* stopping (eq. resdiff, eq. trueresidual with one inner residual per basis
  column): the pair is accepted when rho + sum_{k,c} |y_{k,c}| ||p_{k,c}|| <=
  tol ||b_r||, rho the projected residual; INNER_LIMITED when rho <= 0.1 x the
  inexact term, as in the one-vector oracle;
* breakdown: a new block that vanishes (||W|| <= 1e-14 ||M Z_k||) means the
  current space holds every solution (the block analogue of section 3); the
  square projected systems are then solved.  A block that is only rank
  deficient keeps its Householder Q (orthonormal; the small diagonal of
  H_{k+1,k} carries the deficiency).

There is no restart: unconverged pairs after m block steps keep their last
least-squares iterate and go to refinement (oracle.fgmres_sh.refine applied to
each right-hand side with this solver as the correction solve).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .fgmres_sh import (make_inner, ShiftInfo, CONVERGED, NOT_CONVERGED, INNER_LIMITED,
                        BREAKDOWN_EXACT, NAN_STATUS, BREAKDOWN_REL, INNER_LIMIT_RATIO)


def qr_pos(W: np.ndarray):
    """Householder QR (reduced) with the diagonal of R made real, >= 0."""
    Q, R = np.linalg.qr(W)
    d = np.diag(R)
    ph = np.where(np.abs(d) > 0, d / np.where(np.abs(d) > 0, np.abs(d), 1.0), 1.0)
    return Q * ph[None, :], R * ph.conj()[:, None]


def block_mgs_step(Vblocks, W):
    """Block modified Gram-Schmidt of W (n x s) against the blocks V_1..V_k
    (each n x s, orthonormal columns), then QR of the remainder.  Returns
    (H column blocks [H_1k .. H_kk], H_{k+1,k}, V_{k+1})."""
    W = np.array(W, dtype=np.complex128)
    Hs = []
    for Vi in Vblocks:
        Hik = Vi.conj().T @ W
        W = W - Vi @ Hik
        Hs.append(Hik)
    Q, R = qr_pos(W)
    return Hs, R, Q


def shifted_block_hessenberg(H: np.ndarray, taus: np.ndarray, s: int, sigma: complex) -> np.ndarray:
    """Hbar(sigma;T) = [I;0] + Hbar (sigma I - T) for a ((k+1)s) x (ks) Hbar,
    T = diag(tau_k I_s)."""
    ks = H.shape[1]
    E = np.zeros_like(H)
    E[:ks, :ks] = np.eye(ks)
    d = np.repeat(sigma - np.asarray(taus), s)
    return E + H * d[None, :]


@dataclass
class BlockResult:
    x: np.ndarray                      # (n, n_f, s)
    info: List[List[ShiftInfo]]        # info[r][j]
    inner_its: int = 0
    outer_steps: int = 0
    V: Optional[np.ndarray] = None
    Z: Optional[np.ndarray] = None
    H: Optional[np.ndarray] = None
    beta: Optional[np.ndarray] = None
    taus: Optional[np.ndarray] = None
    pnorms: Optional[np.ndarray] = None
    P: Optional[np.ndarray] = None
    quasi_hist: list = field(default_factory=list)


def block_fgmres_sh(problem, B, sigmas, tau_seq, *, m=50, tol=1e-8, inner="cocg", eps=1e-10,
                    inner_maxit=None, keep_basis=False, mg_nu=1, mg_omega=0.8) -> BlockResult:
    """Block FGMRES-Sh for (K + sigma_j M) X_j = B, B (n, s).  ``tau_seq`` is
    used cyclically over the block steps; ``inner`` as in oracle.fgmres_sh.
    Returns x[:, j, r] and info[r][j]."""
    B = np.asarray(B, dtype=np.complex128)
    if B.ndim == 1:
        B = B[:, None]
    sigmas = np.asarray(sigmas, dtype=np.complex128)
    tau_seq = np.asarray(tau_seq, dtype=np.complex128)
    n, s = B.shape
    nf = len(sigmas)
    x = np.zeros((n, nf, s), dtype=np.complex128)
    info = [[ShiftInfo() for _ in range(nf)] for _ in range(s)]
    res = BlockResult(x=x, info=info)
    bn = np.linalg.norm(B, axis=0)
    if not np.all(np.isfinite(B)) or not np.all(np.isfinite(sigmas)):
        for row in info:
            for q in row:
                q.status = NAN_STATUS
        x[:] = np.nan
        return res
    active = np.ones((nf, s), dtype=bool)
    for r in range(s):
        if bn[r] == 0.0:
            active[:, r] = False
            for q in info[r]:
                q.status, q.quasi_relres, q.bound_relres, q.true_relres = CONVERGED, 0.0, 0.0, 0.0
    if not active.any():
        return res
    solve_inner = make_inner(problem, inner, eps, inner_maxit, mg_nu, mg_omega)
    M = problem.Mdiag
    V1, beta = qr_pos(B)
    Vb = [V1]
    Zb, Pb = [], []
    H = np.zeros(((m + 1) * s, m * s), dtype=np.complex128)
    taus = np.zeros(m, dtype=np.complex128)
    pn = np.zeros((m, s))
    ylast = {}
    kend = 0
    for k in range(m):
        tau = tau_seq[k % len(tau_seq)]
        taus[k] = tau
        res.outer_steps += 1
        Zk = np.zeros((n, s), dtype=np.complex128)
        Pk = np.zeros((n, s), dtype=np.complex128)
        for c in range(s):
            v = Vb[k][:, c]
            if np.linalg.norm(v) == 0.0:
                continue
            z, its = solve_inner(v, tau)
            res.inner_its += its
            Zk[:, c] = z
            Pk[:, c] = v - problem.apply(tau, z)
            pn[k, c] = np.linalg.norm(Pk[:, c])
        Zb.append(Zk)
        Pb.append(Pk)
        W = M[:, None] * Zk
        nmz = np.linalg.norm(W)
        Hs, Rn, Vn = block_mgs_step(Vb, W)
        for i, Hik in enumerate(Hs):
            H[i * s:(i + 1) * s, k * s:(k + 1) * s] = Hik
        H[(k + 1) * s:(k + 2) * s, k * s:(k + 1) * s] = Rn
        broke = np.linalg.norm(Rn) <= BREAKDOWN_REL * nmz
        Vb.append(Vn if not broke else np.zeros_like(Vn))
        kend = k + 1
        Hk = H[:(k + 2) * s, :(k + 1) * s]
        Zall = np.concatenate(Zb, axis=1)
        pflat = pn[:k + 1].ravel()
        hist = np.full((nf, s), np.nan)
        for j in range(nf):
            if not active[j].any():
                continue
            Hs_ = shifted_block_hessenberg(Hk, taus[:k + 1], s, sigmas[j])
            for r in np.nonzero(active[j])[0]:
                rhs = np.zeros((k + 2) * s, dtype=np.complex128)
                rhs[:s] = beta[:, r]
                if broke:
                    y = np.linalg.solve(Hs_[:(k + 1) * s], rhs[:(k + 1) * s])
                    rho = 0.0
                else:
                    y = np.linalg.lstsq(Hs_, rhs, rcond=None)[0]
                    rho = float(np.linalg.norm(rhs - Hs_ @ y))
                gap = float(np.sum(np.abs(y) * pflat))
                bound = rho + gap
                ylast[(j, r)] = y
                q = info[r][j]
                q.outer_its, q.quasi_relres, q.bound_relres = res.outer_steps, rho / bn[r], bound / bn[r]
                hist[j, r] = rho / bn[r]
                done = None
                if broke:
                    done = BREAKDOWN_EXACT if bound <= tol * bn[r] else INNER_LIMITED
                elif bound <= tol * bn[r]:
                    done = CONVERGED
                elif rho <= INNER_LIMIT_RATIO * gap:
                    done = INNER_LIMITED
                if done is not None:
                    q.status = done
                    x[:, j, r] = Zall @ y
                    active[j, r] = False
        res.quasi_hist.append(hist)
        if broke or not active.any():
            break
    if active.any():
        Zall = np.concatenate(Zb, axis=1)
        for j, r in zip(*np.nonzero(active)):
            x[:, j, r] = Zall @ ylast[(j, r)]
            info[r][j].status = NOT_CONVERGED
    if keep_basis:
        res.V = np.concatenate(Vb[:kend + 1], axis=1)
        res.Z = np.concatenate(Zb, axis=1)
        res.H = H[:(kend + 1) * s, :kend * s]
        res.beta, res.taus, res.pnorms = beta, taus[:kend], pn[:kend]
        res.P = np.concatenate(Pb, axis=1)
    for r in range(s):
        for j in range(nf):
            rr = B[:, r] - problem.apply(sigmas[j], x[:, j, r])
            info[r][j].true_relres = np.linalg.norm(rr) / bn[r] if bn[r] > 0 else 0.0
    return res
