"""Oracle: exact solutions x_j = (K + sigma_j M)^{-1} b of eq. multipleshifted.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Four independent routes to the same quantity:

* ``banded_solve``: Gaussian elimination of the banded matrix organised in
  blocks of grid rows (block size nx in 2-D, nx*ny in 3-D; no pivoting across
  blocks).  K + sigma M is complex symmetric and (weakly, strictly at Dirichlet
  rows) diagonally dominant, so elimination without cross-block pivoting is
  stable.  Feasible up to about 256x256.
* ``superlu_solve``: SciPy's SuperLU, the direct solver the paper itself uses
  for its "Direct" runs and exact preconditioners (section 6).
* ``dense_solve``: brute force on tiny grids.
* closed forms for homogeneous K (``dst_closed_form``) and the 1-D discrete
  Green's function (``green_1d``).
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def dense_solve(A, b):
    A = A.toarray() if sp.issparse(A) else np.asarray(A)
    return np.linalg.solve(A.astype(np.complex128), np.asarray(b, dtype=np.complex128))


def superlu_solve(A, b):
    lu = spla.splu(sp.csc_matrix(A, dtype=np.complex128))
    return lu.solve(np.asarray(b, dtype=np.complex128))


def banded_solve(A, b, block: int):
    """Solve A x = b for a matrix whose nonzeros lie within ``block`` of the
    diagonal (block tridiagonal in blocks of size ``block``)."""
    A = sp.csr_matrix(A, dtype=np.complex128)
    n = A.shape[0]
    assert n % block == 0
    nb = n // block
    b = np.asarray(b, dtype=np.complex128)
    vec = b.ndim == 1
    B = b.reshape(n, -1)

    def blk(i, j):
        return A[i * block:(i + 1) * block, j * block:(j + 1) * block].toarray()

    S_inv = [None] * nb      # inverse Schur complements
    Y = [None] * nb
    S = blk(0, 0)
    S_inv[0] = np.linalg.inv(S)
    Y[0] = B[0:block]
    for j in range(1, nb):
        L = blk(j, j - 1)
        U = blk(j - 1, j)
        S = blk(j, j) - L @ (S_inv[j - 1] @ U)
        S_inv[j] = np.linalg.inv(S)
        Y[j] = B[j * block:(j + 1) * block] - L @ (S_inv[j - 1] @ Y[j - 1])
    X = [None] * nb
    X[nb - 1] = S_inv[nb - 1] @ Y[nb - 1]
    for j in range(nb - 2, -1, -1):
        U = blk(j, j + 1)
        X[j] = S_inv[j] @ (Y[j] - U @ X[j + 1])
    x = np.concatenate(X, axis=0)
    return x[:, 0] if vec else x


def laplacian_eigenvalues(dims):
    """Eigenvalues of the (2d+1)-point Dirichlet Laplacian on a grid with
    ``dims`` = (nx, ny[, nz]) interior points: sum over axes of
    4 sin^2(p pi / (2 (n+1))), p = 1..n.  Returned in (.., ny, nx) layout."""
    lam = 0.0
    d = len(dims)
    for ax_x, nax in enumerate(dims):
        p = np.arange(1, nax + 1)
        l1 = 4.0 * np.sin(p * np.pi / (2.0 * (nax + 1))) ** 2
        shape = [1] * d
        shape[d - 1 - ax_x] = nax
        lam = lam + l1.reshape(shape)
    return lam


def dst_closed_form(K0: float, Ss: float, h: float, dims, sigma: complex, b: np.ndarray):
    """Exact solution for homogeneous conductivity K0: K = K0 h^(d-2) L with L
    the Dirichlet Laplacian, diagonalised by the type-I sine transform, and
    M = Ss h^d I.  x = S (K0 h^(d-2) Lambda + sigma Ss h^d)^{-1} S b."""
    d = len(dims)
    shape = tuple(reversed(dims))
    mu = K0 * h ** (d - 2) * laplacian_eigenvalues(dims) + sigma * Ss * h ** d
    bb = np.asarray(b, dtype=np.complex128).reshape(shape)
    c = scipy.fft.dstn(bb, type=1)
    x = scipy.fft.idstn(c / mu, type=1)
    return x.ravel()


def dst_mode(dims, modes):
    """Eigenvector of the Dirichlet Laplacian with 1-based mode numbers
    ``modes`` = (p, q[, r]), as a flat vector (x fastest)."""
    v = 1.0
    d = len(dims)
    for ax_x, (nax, p) in enumerate(zip(dims, modes)):
        xs = np.arange(nax)
        s = np.sin(p * (xs + 1) * np.pi / (nax + 1))
        shape = [1] * d
        shape[d - 1 - ax_x] = nax
        v = v * s.reshape(shape)
    return np.asarray(v, dtype=np.float64).ravel()


def green_1d(N: int, K0: float, Ss: float, h: float, sigma: complex) -> np.ndarray:
    """Closed-form inverse of the 1-D operator (K0/h) tridiag(-1, 2, -1) +
    sigma Ss h I (N cells, Dirichlet ghosts at distance h): with
    cosh(theta) = 1 + sigma Ss h^2 / (2 K0),
    G_ij = sinh(i_< theta) sinh((N+1-i_>) theta) / (sinh(theta) sinh((N+1) theta))
    (1-based indices) and A^{-1} = (h/K0) G."""
    theta = np.arccosh(np.complex128(1.0 + sigma * Ss * h * h / (2.0 * K0)))
    i = np.arange(1, N + 1)
    lo = np.minimum.outer(i, i)
    hi = np.maximum.outer(i, i)
    G = np.sinh(lo * theta) * np.sinh((N + 1 - hi) * theta) / (np.sinh(theta) * np.sinh((N + 1) * theta))
    return (h / K0) * G


def exact_family(problem, sigmas, b, method="auto"):
    """x_j for every shift: returns an (n, n_f) complex array (b a vector)."""
    n = problem.n
    out = np.empty((n, len(sigmas)), dtype=np.complex128)
    for j, s in enumerate(sigmas):
        A = problem.shifted(s)
        if method == "dense" or (method == "auto" and n <= 600):
            out[:, j] = dense_solve(A, b)
        elif method == "banded":
            dims = tuple(reversed(problem.shape))
            blk = dims[0] if len(dims) == 2 else dims[0] * dims[1]
            out[:, j] = banded_solve(A, b, blk)
        else:
            out[:, j] = superlu_solve(A, b)
    return out
