"""Oracle: flexible FOM/GMRES for shifted systems (FGMRES-Sh / FFOM-Sh).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Plain, slow, complex128 statement of the paper's method:

* flexible Arnoldi with modified Gram-Schmidt (Algorithm 3; Algorithm 1 is the
  single-tau case): z_k solves (K + tau_k M) z_k = v_k (eq. zmmod), w = M z_k,
  then w is orthogonalised against v_1..v_k, h_{k+1,k} = ||w||, v_{k+1} = w / h.
  Reading of the printed loop: the coefficient is h_{ik} = v_i^H w and the update
  subtracts h_{ik} v_i (the printed index k and the order of the conjugated
  factor do not give an orthogonal basis for complex data).
* the relations M Z = V_{m+1} Hbar (eq. arnoldimod), K Z + M Z T = V_m
  (eq. zmvmrelation) give, for every shift, (K + sigma M) Z = V_{m+1} Hbar(sigma;T)
  with Hbar(sigma;T) = [I;0] + Hbar (sigma I - T) (eq. shiftedarnoldimod).
* per shift (Algorithm 4): GMRES y = argmin ||beta e_1 - Hbar(sigma;T) y|| (here
  with a library least-squares solve), FOM y = H(sigma;T)^{-1} beta e_1, and
  x = Z y.
* inexact preconditioning (section 4): with inner residuals p_k the true
  residual differs from the quasi-residual by P y, bounded by sum |y_k| ||p_k||
  (eq. resdiff); a shift is accepted when ||beta e_1 - Hbar y|| + sum |y_k| ||p_k||
  <= tol ||b|| (eq. trueresidual, with the measured ||p_k|| in place of eps).
* restart (section 2.2.2 defers to Gu et al. / Frommer-Glassner; reading): GMRES
  keeps the residuals of all shifts collinear with the residual of a seed shift
  (the unconverged shift of largest quasi-residual, ties to the lowest index):
  the others solve [Hbar(sigma_j;T), z_s] [y_j; gamma_j] = beta_j e_1, the new
  start vector is V_{m+1} z_s / ||z_s|| and beta_j <- gamma_j ||z_s||.  FOM
  residuals are collinear with v_{m+1} already.  The tau schedule continues
  cyclically across restarts (the "recycle" of section 6.1).
* breakdown h_{k+1,k} = 0 means the current iterate is exact for every shift
  (section 3); the threshold read here is h_{k+1,k} <= 1e-14 ||M z_k||.

Status codes (shared meaning with the GPU library's per-(shift, rhs) status):
CONVERGED 0, NOT_CONVERGED 1, INNER_LIMITED 2, BREAKDOWN_EXACT 3, NAN 4.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .cocg import cocg
from .exact import banded_solve, dense_solve, superlu_solve
from .mg import Hierarchy, mg_cocg

CONVERGED, NOT_CONVERGED, INNER_LIMITED, BREAKDOWN_EXACT, NAN_STATUS = 0, 1, 2, 3, 4
BREAKDOWN_REL = 1e-14
INNER_LIMIT_RATIO = 0.1


@dataclass
class ShiftInfo:
    status: int = NOT_CONVERGED
    outer_its: int = 0
    restarts: int = 0
    quasi_relres: float = np.inf
    bound_relres: float = np.inf
    true_relres: float = np.inf
    refine_sweeps: int = 0


@dataclass
class Result:
    x: np.ndarray
    info: List[ShiftInfo]
    inner_its: int = 0
    outer_steps: int = 0
    # last cycle's basis (for the relations of Algorithm 3)
    V: Optional[np.ndarray] = None
    Z: Optional[np.ndarray] = None
    H: Optional[np.ndarray] = None
    taus: Optional[np.ndarray] = None
    pnorms: Optional[np.ndarray] = None
    P: Optional[np.ndarray] = None
    y_last: dict = field(default_factory=dict)
    quasi_hist: Optional[np.ndarray] = None


def mgs_step(V: np.ndarray, w: np.ndarray):
    """One modified Gram-Schmidt orthogonalisation of w against the columns of
    V (Algorithm 3, inner loop, as read above).  Returns (h, hnext, v_next)."""
    w = np.array(w, dtype=np.complex128)
    k = V.shape[1]
    h = np.zeros(k, dtype=np.complex128)
    for i in range(k):
        h[i] = np.vdot(V[:, i], w)
        w = w - h[i] * V[:, i]
    hn = np.linalg.norm(w)
    return h, hn, (w / hn if hn > 0 else w)


def shifted_hessenberg(H: np.ndarray, taus: np.ndarray, sigma: complex) -> np.ndarray:
    """Hbar(sigma;T) = [I;0] + Hbar (sigma I - T) for a (k+1) x k Hbar."""
    k = H.shape[1]
    E = np.zeros((k + 1, k), dtype=np.complex128)
    E[:k, :k] = np.eye(k)
    return E + H * (sigma - np.asarray(taus))[None, :]


def small_solve(Hs: np.ndarray, beta: complex, variant: str):
    """Projected problem of Algorithm 4 for one shift: returns (y, quasi-residual
    vector beta e_1 - Hs y)."""
    kp1, k = Hs.shape
    rhs = np.zeros(kp1, dtype=np.complex128)
    rhs[0] = beta
    if variant == "fom":
        y = np.linalg.solve(Hs[:k, :k], rhs[:k])
    else:
        y = np.linalg.lstsq(Hs, rhs, rcond=None)[0]
    return y, rhs - Hs @ y


def make_inner(problem, inner: str, eps: float, inner_maxit: Optional[int], mg_nu: int = 1,
               mg_omega: float = 0.8):
    """Returns f(v, tau) -> (z, its)."""
    cache = {}
    if inner_maxit is None:
        dims = problem.shape if problem.shape is not None else (problem.n,)
        inner_maxit = 20 * max(dims)

    if inner == "cocg":
        def f(v, tau, eps_k=eps):
            diag = problem.diag(tau)
            z, its, _ok, _h = cocg(lambda x: problem.apply(tau, x), diag, v, eps_k, inner_maxit)
            return z, its
        return f
    if inner == "mg":
        H = Hierarchy.of(problem)

        def f(v, tau, eps_k=eps):
            z, its, _ok, _h = mg_cocg(problem, tau, v, eps_k, inner_maxit, H, mg_nu, mg_omega)
            return z, its
        return f

    def f(v, tau, eps_k=eps):
        A = problem.shifted(tau)
        if inner == "dense":
            return dense_solve(A, v), 0
        if inner == "banded":
            dims = tuple(reversed(problem.shape))
            blk = dims[0] if len(dims) == 2 else dims[0] * dims[1]
            return banded_solve(A, v, blk), 0
        key = complex(tau)
        if key not in cache:
            import scipy.sparse as sp
            import scipy.sparse.linalg as spla
            cache[key] = spla.splu(sp.csc_matrix(A))
        return cache[key].solve(np.asarray(v, dtype=np.complex128)), 0
    return f


def fgmres_sh(problem, b, sigmas, tau_seq, *, m_restart=50, max_restarts=20, tol=1e-8,
              inner="cocg", eps=1e-10, inner_maxit=None, variant="gmres",
              max_steps=None, keep_basis=False, record_quasi=False,
              stop_after_restart=None, mg_nu=1, mg_omega=0.8, relax=0.0, eps_max=1e-2) -> Result:
    """Solve (K + sigma_j M) x_j = b for all shifts with one flexible basis.

    ``tau_seq`` is used cyclically over the global step counter.  ``inner`` is
    "cocg" (Jacobi-COCG to ``eps``), "mg" (COCG preconditioned by the multigrid
    V-cycle of oracle.mg with ``mg_nu`` damped-Jacobi sweeps of weight
    ``mg_omega``), or an exact solve ("superlu", "banded", "dense").  ``max_steps`` caps the total number of outer steps (for timing
    samples); ``stop_after_restart`` returns right after the restart update of
    that cycle (0-based), to inspect the restarted residuals.  ``relax`` > 0
    relaxes the inner tolerance as the outer residual falls (the Simoncini-Szyld
    idea the paper cites in section 4 without pursuing it): after each outer
    step the next inner solve asks for
        eps_k = min(eps_max, max(eps, relax * tol / q)),
    q the largest relative quasi-residual rho_j / ||b|| over the shifts still
    running; the stopping bound of eq. trueresidual uses the measured ||p_k||,
    so it stays a bound whatever eps_k is.  Returns x as an (n, n_f) array plus
    per-shift information."""
    sigmas = np.asarray(sigmas, dtype=np.complex128)
    tau_seq = np.asarray(tau_seq, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    n, nf = problem.n, len(sigmas)
    x = np.zeros((n, nf), dtype=np.complex128)
    info = [ShiftInfo() for _ in range(nf)]
    beta0 = np.linalg.norm(b)
    res = Result(x=x, info=info)
    if not np.all(np.isfinite(b)) or not np.all(np.isfinite(sigmas)):
        for s in info:
            s.status = NAN_STATUS
        x[:] = np.nan
        return res
    if beta0 == 0.0:
        for s in info:
            s.status, s.quasi_relres, s.bound_relres, s.true_relres = CONVERGED, 0.0, 0.0, 0.0
        return res
    solve_inner = make_inner(problem, inner, eps, inner_maxit, mg_nu, mg_omega)
    eps_k = eps
    M = problem.Mdiag
    beta = np.full(nf, beta0, dtype=np.complex128)
    gap_prev = np.zeros(nf)
    active = np.ones(nf, dtype=bool)
    v1 = b / beta0
    kk = 0
    quasi_hist = []
    m = m_restart
    for cycle in range(max_restarts + 1):
        V = np.zeros((n, m + 1), dtype=np.complex128)
        Z = np.zeros((n, m), dtype=np.complex128)
        P = np.zeros((n, m), dtype=np.complex128) if keep_basis else None
        H = np.zeros((m + 1, m), dtype=np.complex128)
        taus = np.zeros(m, dtype=np.complex128)
        pn = np.zeros(m)
        V[:, 0] = v1
        ylast = {}
        kend = 0
        broke = False
        for k in range(m):
            if max_steps is not None and res.outer_steps >= max_steps:
                break
            tau = tau_seq[kk % len(tau_seq)]
            kk += 1
            res.outer_steps += 1
            taus[k] = tau
            z, its = solve_inner(V[:, k], tau, eps_k)
            res.inner_its += its
            p = V[:, k] - problem.apply(tau, z)
            pn[k] = np.linalg.norm(p)
            if P is not None:
                P[:, k] = p
            Z[:, k] = z
            w = M * z
            nmz = np.linalg.norm(w)
            h, hn, vn = mgs_step(V[:, :k + 1], w)
            H[:k + 1, k] = h
            H[k + 1, k] = hn
            broke = hn <= BREAKDOWN_REL * nmz
            if not broke:
                V[:, k + 1] = vn
            kend = k + 1
            step_q = np.full(nf, np.nan)
            for j in np.nonzero(active)[0]:
                Hs = shifted_hessenberg(H[:k + 2, :k + 1], taus[:k + 1], sigmas[j])
                if broke:
                    y, qv = small_solve(Hs, beta[j], "fom")
                    qv[:] = 0.0
                else:
                    y, qv = small_solve(Hs, beta[j], variant)
                rho = np.linalg.norm(qv)
                gap = float(np.sum(np.abs(y) * pn[:k + 1]))
                bound = rho + gap_prev[j] + gap
                ylast[j] = (y, qv)
                s = info[j]
                s.outer_its = res.outer_steps
                s.restarts = cycle
                s.quasi_relres = rho / beta0
                s.bound_relres = bound / beta0
                step_q[j] = rho / beta0
                done = None
                if broke:
                    done = BREAKDOWN_EXACT if bound <= tol * beta0 else INNER_LIMITED
                elif bound <= tol * beta0:
                    done = CONVERGED
                elif rho <= INNER_LIMIT_RATIO * (gap_prev[j] + gap):
                    done = INNER_LIMITED
                if done is not None:
                    s.status = done
                    x[:, j] += Z[:, :k + 1] @ y
                    active[j] = False
            if record_quasi:
                quasi_hist.append(step_q)
            if relax > 0.0 and np.any(np.isfinite(step_q)):
                q = float(np.nanmax(step_q))
                if q > 0.0:
                    eps_k = min(eps_max, max(eps, relax * tol / q))
            if broke or not active.any():
                break
        if keep_basis:
            res.V, res.Z, res.H = V[:, :kend + 1], Z[:, :kend], H[:kend + 1, :kend]
            res.taus, res.pnorms, res.P = taus[:kend], pn[:kend], (P[:, :kend] if P is not None else None)
            res.y_last = ylast
        if not active.any() or broke:
            break
        if max_steps is not None and res.outer_steps >= max_steps:
            for j in np.nonzero(active)[0]:
                y, _ = ylast[j]
                x[:, j] += Z[:, :kend] @ y
            break
        if cycle == max_restarts:
            for j in np.nonzero(active)[0]:
                y, _ = ylast[j]
                x[:, j] += Z[:, :kend] @ y
                info[j].status = NOT_CONVERGED
            break
        # ---- restart (all active shifts have a full cycle of m steps) ----
        act = np.nonzero(active)[0]
        if variant == "fom":
            for j in act:
                y, qv = ylast[j]
                x[:, j] += Z @ y
                gap_prev[j] += float(np.sum(np.abs(y) * pn))
                beta[j] = qv[m]            # residual = qv[m] v_{m+1}
            v1 = V[:, m].copy()
            continue
        rhos = np.array([np.linalg.norm(ylast[j][1]) for j in act])
        s_idx = act[int(np.argmax(rhos))]
        ys, zs = ylast[s_idx]
        nzs = np.linalg.norm(zs)
        for j in act:
            if j == s_idx:
                y, gam = ys, 1.0
            else:
                Hs = shifted_hessenberg(H, taus, sigmas[j])
                A = np.concatenate([Hs, zs[:, None]], axis=1)
                rhs = np.zeros(m + 1, dtype=np.complex128)
                rhs[0] = beta[j]
                sol = np.linalg.solve(A, rhs)
                y, gam = sol[:m], sol[m]
            x[:, j] += Z @ y
            gap_prev[j] += float(np.sum(np.abs(y) * pn))
            beta[j] = gam * nzs
        v1 = V @ zs / nzs
        if stop_after_restart is not None and cycle == stop_after_restart:
            res.y_last = {"beta": beta.copy(), "seed": int(s_idx)}
            return res
    if record_quasi:
        res.quasi_hist = np.array(quasi_hist)
    true_residuals(problem, b, sigmas, x, info)
    return res


def true_residuals(problem, b, sigmas, x, info=None):
    """FP64 true relative residual ||b - (K + sigma_j M) x_j|| / ||b|| per shift
    (the paper's ||r_m|| / ||r_0|| with x_0 = 0)."""
    nb = np.linalg.norm(b)
    out = np.empty(len(sigmas))
    for j, s in enumerate(sigmas):
        r = b - problem.apply(s, x[:, j])
        out[j] = np.linalg.norm(r) / nb if nb > 0 else 0.0
        if info is not None:
            info[j].true_relres = out[j]
    return out


def refine(problem, b, sigmas, x, solve, tol, max_refine, info=None):
    """Collinear refinement (reading; the paper gives none): with true residuals
    r_j, take the seed s = argmax ||r_j|| (ties to the lowest index), solve the
    shifted family with right-hand side r_s (``solve(rhs) -> (n, n_f)``), and
    update every shift still above ``tol``: x_j += gamma_j d_j with
    gamma_j = r_s^H r_j / r_s^H r_s.  Repeats up to ``max_refine`` times.
    Returns the number of sweeps made."""
    sigmas = np.asarray(sigmas)
    nb = np.linalg.norm(b)
    sweeps = 0
    for _ in range(max_refine):
        R = np.stack([b - problem.apply(s, x[:, j]) for j, s in enumerate(sigmas)], axis=1)
        nr = np.linalg.norm(R, axis=0)
        bad = nr > tol * nb
        if not bad.any():
            break
        s = int(np.argmax(nr))
        rs = R[:, s]
        gam = (rs.conj() @ R) / (rs.conj() @ rs)
        d = solve(rs)
        for j in np.nonzero(bad)[0]:
            x[:, j] += gam[j] * d[:, j]
        sweeps += 1
    rel = true_residuals(problem, b, sigmas, x)
    if info is not None:
        for j, s in enumerate(info):
            s.true_relres = rel[j]
            s.refine_sweeps = sweeps
            if rel[j] <= tol:
                s.status = CONVERGED
            elif s.status == CONVERGED:
                s.status = NOT_CONVERGED
    return sweeps
