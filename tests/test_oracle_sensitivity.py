"""Pins of the oracle's sensitivity (section 5, eq. sensitivity): central finite
differences of the measured phasor with respect to ln K, the scaling identity
and the face count."""
import numpy as np
import pytest

import synth
from oracle import Problem, assemble_stiffness, dense_solve
from oracle.sensitivity import faces, sensitivity, sensitivity_block


def _K(shape, seed):
    return synth.cell_conductivity(shape, -11.5, 1.0, 3, cfg=92, idx=seed)


def _measure(K, sigma, b, m, h=1.0):
    op = Problem.fv(K, 1e-5, h)
    return dense_solve(op.shifted(sigma), b)[m]


@pytest.mark.parametrize("shape,h", [((5, 4), 1.0), ((3, 4, 3), 2.0)])
def test_matches_central_differences(shape, h):
    """dh/ds_c against (h(s + d e_c) - h(s - d e_c)) / 2d with dense solves."""
    K = _K(shape, len(shape))
    n = K.size
    op = Problem.fv(K, 1e-5, h)
    sigma = 2j * np.pi / 40.0
    src, m = 1, n - 2
    b = np.zeros(n, dtype=np.complex128)
    b[src] = 1.0
    em = np.zeros(n, dtype=np.complex128)
    em[m] = 1.0
    A = op.shifted(sigma)
    phi = dense_solve(A, b)
    psi = dense_solve(A, em)
    J = sensitivity(K, phi, psi, h)
    d = 1e-5
    for c in range(n):
        Kp = K.ravel().copy()
        Km = K.ravel().copy()
        Kp[c] *= np.exp(d)
        Km[c] *= np.exp(-d)
        fd = (_measure(Kp.reshape(K.shape), sigma, b, m, h) - _measure(Km.reshape(K.shape), sigma, b, m, h)) / (2 * d)
        assert abs(fd - J[c]) <= 1e-6 * np.abs(J).max(), c


def test_sum_over_cells_is_the_stiffness_form():
    """Scaling every K by e^a scales every face by e^a, so sum_c dh/ds_c = -Psi^T K Phi."""
    K = _K((6, 7), 5)
    rng = np.random.default_rng(2)
    phi = rng.normal(size=K.size) + 1j * rng.normal(size=K.size)
    psi = rng.normal(size=K.size) + 1j * rng.normal(size=K.size)
    J = sensitivity(K, phi, psi, 1.0)
    Ks = assemble_stiffness(K, 1.0)
    assert np.isclose(J.sum(), -(psi @ (Ks @ phi)), rtol=1e-12)


def test_face_count_and_block_layout():
    K = _K((3, 4, 2), 1)          # nz = 3, ny = 4, nx = 2
    f = faces(K)
    nx, ny, nz = 2, 4, 3
    assert len(f) == (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    rng = np.random.default_rng(4)
    n = K.size
    Phi = rng.normal(size=(n, 2, 3)) + 1j * rng.normal(size=(n, 2, 3))
    Psi = rng.normal(size=(n, 2, 2)) + 1j * rng.normal(size=(n, 2, 2))
    J = sensitivity_block(K, Phi, Psi)
    assert J.shape == (2, 3, 2, n)
    assert np.array_equal(J[1, 2, 0], sensitivity(K, Phi[:, 1, 2], Psi[:, 1, 0]))
