"""Oracle: sensitivity of point measurements to the log-conductivity field
(section 5, eq. sensitivity and Algorithm 6) for the finite-volume operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

With s = ln K per cell, a measurement is the phasor h = e_m^T Phi of a forward
solve A Phi = b, A = K(s) + sigma M.  Differentiating A Phi = b with respect
to s_c (M does not depend on s here):

    dh/ds_c = - Psi^T (dK/ds_c) Phi,    Psi = A^{-T} e_m = A^{-1} e_m,

A being complex symmetric.  Psi is the adjoint solution of eq. adjoint; the
paper's adjoint carries the source -delta, i.e. it is -Psi, which turns the
sign of the bilinear term into the + of eq. sensitivity.  The stiffness is a
sum over faces, K = sum_f T_f g_f g_f^T (g_f = e_a - e_b for the face between
cells a and b, g_f = e_a for a boundary face of cell a), so

    dh/ds_c = - sum_{faces f of c} (dT_f/ds_c) (g_f^T Psi)(g_f^T Phi),

with, for the harmonic-mean face T = 2 K_a K_b / (K_a + K_b) h^(d-2),
dT/ds_a = K_a dT/dK_a = T K_b / (K_a + K_b), and dT/ds_a = T for a boundary
face (T = K_a h^(d-2)).  The real and imaginary parts of dh/ds_c are the
paper's two measurements per location and frequency.  Computed face by face
in plain loops (small grids only).
"""
from __future__ import annotations

import numpy as np

from .fv import harmonic


def faces(cell_K: np.ndarray, h: float = 1.0):
    """Every face as (a, b, T, dT/ds_a, dT/ds_b); b = -1 for a boundary face
    (its dT/ds_b is 0).  Cell index x fastest."""
    Kc = np.asarray(cell_K, dtype=np.float64)
    d = Kc.ndim
    shape = Kc.shape                      # (.., ny, nx)
    scale = h ** (d - 2)
    flat = Kc.ravel()
    idx = np.arange(Kc.size).reshape(shape)
    out = []
    for ax in range(d):                   # numpy axis
        n = shape[ax]
        for pos in np.ndindex(*shape):
            a = idx[pos]
            k = pos[ax]
            if k == 0:                    # the face below the first cell: boundary
                T = flat[a] * scale
                out.append((a, -1, T, T, 0.0))
            if k == n - 1:                # the face above the last cell: boundary
                T = flat[a] * scale
                out.append((a, -1, T, T, 0.0))
            else:                         # interior face between a and its upper neighbour
                nb = list(pos)
                nb[ax] += 1
                b = idx[tuple(nb)]
                Ka, Kb = flat[a], flat[b]
                T = harmonic(Ka, Kb) * scale
                out.append((a, b, T, T * Kb / (Ka + Kb), T * Ka / (Ka + Kb)))
    return out


def sensitivity(cell_K, phi, psi, h: float = 1.0) -> np.ndarray:
    """dh/ds_c for every cell c, one forward solution phi and one adjoint psi."""
    phi = np.asarray(phi, dtype=np.complex128)
    psi = np.asarray(psi, dtype=np.complex128)
    J = np.zeros(phi.shape[0], dtype=np.complex128)
    for a, b, _T, da, db in faces(cell_K, h):
        gphi = phi[a] - (phi[b] if b >= 0 else 0.0)
        gpsi = psi[a] - (psi[b] if b >= 0 else 0.0)
        prod = gpsi * gphi
        J[a] -= da * prod
        if b >= 0:
            J[b] -= db * prod
    return J


def sensitivity_block(cell_K, Phi, Psi, h: float = 1.0) -> np.ndarray:
    """Phi: (n, n_shifts, n_src), Psi: (n, n_shifts, n_rec) (the solver's output
    layout read as arrays); returns J of shape (n_shifts, n_src, n_rec, n)."""
    n, nf, ns = Phi.shape
    nr = Psi.shape[2]
    J = np.zeros((nf, ns, nr, n), dtype=np.complex128)
    for j in range(nf):
        for s in range(ns):
            for r in range(nr):
                J[j, s, r] = sensitivity(cell_K, Phi[:, j, s], Psi[:, j, r], h)
    return J
