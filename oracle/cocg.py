"""Oracle: Jacobi-preconditioned COCG, the inner solver for z_k ~ (K + tau_k M)^{-1} v_k.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Section 4 (eq. zmmoditer) allows the preconditioner systems to be solved by an
inner iteration stopped once the inner residual p_k = v_k - (K + tau_k M) z_k
satisfies ||p_k|| <= eps ||v_k||.  The paper's own inner solver (PyAMG
smoothed-aggregation BiCGSTAB, section 6) is not available; the reading here is
the conjugate orthogonal conjugate gradient method of van der Vorst and
Melissen (1990) for complex symmetric matrices (A^T = A, bilinear form x^T y
without conjugation) with the diagonal (Jacobi) preconditioner
D = diag(K) + tau diag(M), which keeps the complex symmetry.

Textbook recurrences, x_0 = 0:
    r_0 = v, u_0 = D^{-1} r_0, p_0 = u_0, rho_0 = r_0^T u_0
    repeat:  q = A p;  alpha = rho / (p^T q);  x += alpha p;  r -= alpha q
             stop if ||r||_2 <= eps ||v||_2
             u = D^{-1} r;  rho' = r^T u;  beta = rho' / rho;  p = u + beta p
The iteration count is the number of products q = A p.
"""
from __future__ import annotations

import numpy as np


def bilinear(a, b):
    return np.sum(a * b)


def cocg(apply_A, diag, v, eps, maxit, x0=None, fixed_iters=None):
    """Returns (x, iterations, converged, residual_history).  With
    ``fixed_iters`` set the loop runs exactly that many products and ignores
    ``eps`` (used to compare iterates step by step)."""
    v = np.asarray(v, dtype=np.complex128)
    nv = np.linalg.norm(v)
    x = np.zeros_like(v) if x0 is None else np.array(x0, dtype=np.complex128)
    if nv == 0.0:
        return x, 0, True, [0.0]
    r = v - apply_A(x) if x0 is not None else v.copy()
    u = r / diag
    p = u.copy()
    rho = bilinear(r, u)
    hist = [np.linalg.norm(r)]
    its = 0
    limit = fixed_iters if fixed_iters is not None else maxit
    while its < limit:
        q = apply_A(p)
        mu = bilinear(p, q)
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
        u = r / diag
        rho_new = bilinear(r, u)
        if rho == 0:
            return x, its, False, hist
        beta = rho_new / rho
        rho = rho_new
        p = u + beta * p
    return x, its, fixed_iters is not None, hist
