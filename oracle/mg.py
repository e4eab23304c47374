"""Oracle: geometric multigrid preconditioner for the inner solves.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Section 4 (eq. zmmoditer) lets the preconditioner systems (K + tau_k M) z = v be
solved by any inner iteration stopped at ||v - (K + tau_k M) z|| <= eps ||v||;
the paper itself preconditions its inner Krylov solver with algebraic
multigrid (section 6, smoothed aggregation).  The reading here, for the
structured finite-volume grids of the workloads, is a geometric aggregation
multigrid V-cycle used as the preconditioner B of COCG:

* levels: cells are grouped 2 x 2 (x 2 in 3-D) into the cells of the next level
  (a trailing odd cell forms a group of its own along that axis) until one
  cell is left; P is the piecewise-constant prolongation of that grouping;
* coarse operators: K_{l+1} = (1/2) P^T K_l P and M_{l+1} = P^T M_l.  For a
  homogeneous field this is exactly the finite-volume operator of the coarse
  grid with spacing 2h in 2-D and 3-D (the stiffness of the plain Galerkin
  product P^T K P is twice that), which keeps the coarse correction from
  being too small for the smooth error it has to remove;
* smoothing: nu damped Jacobi sweeps x += omega D^-1 (b - A x) from x = 0
  before the coarse correction and nu after it, D = diag(A_l);
* restriction P^T, prolongation P, exact solve on the one-cell level.

With symmetric smoothing and R = P^T the V-cycle B is a complex symmetric
linear operator (B^T = B), as COCG requires of its preconditioner.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def aggregation(shape):
    """Piecewise-constant prolongation P (n_fine x n_coarse) of the 2^d grouping
    and the coarse shape.  ``shape`` is numpy order (.., ny, nx)."""
    cshape = tuple((s + 1) // 2 for s in shape)
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    fine = np.ravel_multi_index([g.ravel() for g in grids], shape)
    coarse = np.ravel_multi_index([(g // 2).ravel() for g in grids], cshape)
    n, nc = int(np.prod(shape)), int(np.prod(cshape))
    P = sp.csr_matrix((np.ones(n), (fine, coarse)), shape=(n, nc))
    return P, cshape


class Hierarchy:
    """The tau-independent part: K_l, M_l, P_l for every level down to one cell."""

    def __init__(self, K, Mdiag, shape, kscale: float = 0.5):
        self.K = [sp.csr_matrix(K, dtype=np.float64)]
        self.M = [np.asarray(Mdiag, dtype=np.float64)]
        self.shape = [tuple(shape)]
        self.P = []
        while int(np.prod(self.shape[-1])) > 1:
            P, cshape = aggregation(self.shape[-1])
            self.P.append(P)
            self.K.append(sp.csr_matrix(kscale * (P.T @ self.K[-1] @ P)))
            self.M.append(P.T @ self.M[-1])
            self.shape.append(cshape)

    @classmethod
    def of(cls, problem, kscale: float = 0.5):
        return cls(problem.K, problem.Mdiag, problem.shape, kscale)

    @property
    def levels(self):
        return len(self.K)

    def operator(self, level, tau):
        return (self.K[level].astype(np.complex128) + sp.diags(tau * self.M[level])).tocsr()


def vcycle(H: Hierarchy, tau, b, nu: int = 1, omega: float = 0.8, level: int = 0, ops=None):
    """z = B b for one V-cycle started at ``level`` (x = 0 on every level)."""
    if ops is None:
        ops = [H.operator(l, tau) for l in range(H.levels)]
    A = ops[level]
    D = A.diagonal()
    b = np.asarray(b, dtype=np.complex128)
    if level == H.levels - 1:
        return b / D                           # one cell: exact
    x = np.zeros_like(b)
    for _ in range(nu):
        x = x + omega * (b - A @ x) / D
    r = b - A @ x
    P = H.P[level]
    x = x + P @ vcycle(H, tau, P.T @ r, nu, omega, level + 1, ops)
    for _ in range(nu):
        x = x + omega * (b - A @ x) / D
    return x


def pcocg(apply_A, apply_B, v, eps, maxit, fixed_iters=None):
    """Preconditioned COCG (van der Vorst & Melissen) with a complex symmetric
    preconditioner B; x_0 = 0.  Same recurrences as the Jacobi form with
    u = B r in place of D^-1 r.  Returns (x, iterations, converged, history)."""
    v = np.asarray(v, dtype=np.complex128)
    nv = np.linalg.norm(v)
    x = np.zeros_like(v)
    if nv == 0.0:
        return x, 0, True, [0.0]
    r = v.copy()
    u = apply_B(r)
    p = u.copy()
    rho = np.sum(r * u)
    hist = [nv]
    its = 0
    limit = fixed_iters if fixed_iters is not None else maxit
    while its < limit:
        q = apply_A(p)
        mu = np.sum(p * q)
        if mu == 0:
            return x, its, False, hist
        alpha = rho / mu
        x = x + alpha * p
        r = r - alpha * q
        its += 1
        nr = np.linalg.norm(r)
        hist.append(nr)
        if fixed_iters is None and nr <= eps * nv:
            return x, its, True, hist
        u = apply_B(r)
        rho_new = np.sum(r * u)
        if rho == 0:
            return x, its, False, hist
        p = u + (rho_new / rho) * p
        rho = rho_new
    return x, its, fixed_iters is not None, hist


def mg_cocg(problem, tau, v, eps, maxit, H: Hierarchy = None, nu: int = 1, omega: float = 0.8,
            fixed_iters=None):
    """Multigrid-preconditioned COCG for (K + tau M) z = v."""
    if H is None:
        H = Hierarchy.of(problem)
    ops = [H.operator(l, tau) for l in range(H.levels)]
    return pcocg(lambda x: problem.apply(tau, x), lambda r: vcycle(H, tau, r, nu, omega, 0, ops), v, eps, maxit,
                 fixed_iters)
