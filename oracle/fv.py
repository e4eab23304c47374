"""Oracle: finite-volume discretisation of the phasor groundwater equation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

The phasor equation  -div(K grad Phi) + i*omega*S_s*Phi = Q0 delta(x - x_s)
with Phi = 0 on the Dirichlet boundary (section 5.1, eq. phasor1) discretised on
a cell-centred grid of spacing h gives the shifted family (K + sigma M) x = b of
eq. genshifted with sigma = i*omega.  Readings used here (the paper discretises
with linear finite elements instead; the synthetic workloads fix a finite-volume
operator):

* face transmissivity between cells a, b: T = 2 K_a K_b / (K_a + K_b) * h^(d-2)
  (harmonic mean of the two cell conductivities, flux area h^(d-1) over centre
  distance h);
* a boundary face couples its cell to a Dirichlet ghost value 0 placed at
  distance h, with T = K_cell * h^(d-2); for homogeneous K this makes K exactly
  K0 h^(d-2) times the standard (2d+1)-point Dirichlet Laplacian;
* lumped mass M = S_s h^d on the diagonal (section 2: M diagonal by lumping).

Cell index: x fastest, c = x + nx*(y + ny*z).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def harmonic(a, b):
    return 2.0 * a * b / (a + b)


def face_transmissivities(cell_K: np.ndarray, h: float = 1.0):
    """Return a list (one entry per axis, x first) of arrays of face T including
    the two boundary faces on that axis: along axis x the array has nx+1 faces.
    Arrays keep the (.., ny, nx) layout of ``cell_K`` with the face axis grown by 1."""
    Kc = np.asarray(cell_K, dtype=np.float64)
    d = Kc.ndim
    scale = h ** (d - 2)
    faces = []
    # numpy axis of x is the last one
    for ax_x in range(d):           # ax_x = 0 -> x, 1 -> y, 2 -> z
        ax = d - 1 - ax_x
        n = Kc.shape[ax]
        shp = list(Kc.shape)
        shp[ax] = n + 1
        T = np.empty(shp)
        lo = [slice(None)] * d
        hi = [slice(None)] * d
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        inner = [slice(None)] * d
        inner[ax] = slice(1, n)
        T[tuple(inner)] = harmonic(Kc[tuple(lo)], Kc[tuple(hi)]) * scale
        first = [slice(None)] * d
        first[ax] = slice(0, 1)
        last = [slice(None)] * d
        last[ax] = slice(n, n + 1)
        src_first = [slice(None)] * d
        src_first[ax] = slice(0, 1)
        src_last = [slice(None)] * d
        src_last[ax] = slice(n - 1, n)
        T[tuple(first)] = Kc[tuple(src_first)] * scale     # Dirichlet ghost face
        T[tuple(last)] = Kc[tuple(src_last)] * scale
        faces.append(T)
    return faces


def assemble_stiffness(cell_K: np.ndarray, h: float = 1.0) -> sp.csr_matrix:
    """Stiffness matrix K (real, symmetric, positive definite): for every face,
    the flux T (phi_a - phi_b) enters row a with +T on the diagonal and -T on
    column b; a boundary face contributes only its diagonal +T."""
    Kc = np.asarray(cell_K, dtype=np.float64)
    d = Kc.ndim
    n = Kc.size
    idx = np.arange(n).reshape(Kc.shape)
    faces = face_transmissivities(Kc, h)
    diag = np.zeros(Kc.shape)
    rows, cols, vals = [], [], []
    for ax_x in range(d):
        ax = d - 1 - ax_x
        T = faces[ax_x]
        nax = Kc.shape[ax]

        def sl(a, b):
            s = [slice(None)] * d
            s[ax] = slice(a, b)
            return tuple(s)
        # every cell gets the T of its low and high face on this axis
        diag += T[sl(0, nax)] + T[sl(1, nax + 1)]
        # interior faces couple neighbours a = i-1, b = i
        Ti = T[sl(1, nax)]
        a = idx[sl(0, nax - 1)]
        b = idx[sl(1, nax)]
        rows += [a.ravel(), b.ravel()]
        cols += [b.ravel(), a.ravel()]
        vals += [-Ti.ravel(), -Ti.ravel()]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    K.sum_duplicates()
    return K


def mass_diagonal(shape, Ss: float = 1e-5, h: float = 1.0) -> np.ndarray:
    """Lumped mass: S_s * h^d for every cell."""
    d = len(shape)
    return np.full(int(np.prod(shape)), Ss * h ** d, dtype=np.float64)


def shifted_matrix(K: sp.spmatrix, Mdiag: np.ndarray, sigma: complex) -> sp.csr_matrix:
    """K + sigma M (eq. multipleshifted) as a complex sparse matrix."""
    return (K.astype(np.complex128) + sp.diags(sigma * Mdiag.astype(np.complex128))).tocsr()


def apply_shifted(K: sp.spmatrix, Mdiag: np.ndarray, sigma: complex, x: np.ndarray) -> np.ndarray:
    """y = (K + sigma M) x for a vector or a block of columns."""
    x = np.asarray(x)
    if x.ndim == 1:
        return K @ x + sigma * Mdiag * x
    return K @ x + sigma * Mdiag[:, None] * x


class Problem:
    """Oracle problem: real K (sparse), diagonal M, cell shape."""

    def __init__(self, K: sp.spmatrix, Mdiag: np.ndarray, shape=None):
        self.K = sp.csr_matrix(K, dtype=np.float64)
        self.Mdiag = np.asarray(Mdiag, dtype=np.float64)
        self.n = self.K.shape[0]
        self.shape = shape

    @classmethod
    def fv(cls, cell_K, Ss=1e-5, h=1.0):
        cell_K = np.asarray(cell_K, dtype=np.float64)
        return cls(assemble_stiffness(cell_K, h), mass_diagonal(cell_K.shape, Ss, h), cell_K.shape)

    def apply(self, sigma, x):
        return apply_shifted(self.K, self.Mdiag, sigma, x)

    def shifted(self, sigma):
        return shifted_matrix(self.K, self.Mdiag, sigma)

    def diag(self, sigma):
        return self.K.diagonal().astype(np.complex128) + sigma * self.Mdiag
