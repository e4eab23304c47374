"""Pins of the oracle's exact solvers: brute force, SuperLU, closed forms."""
import numpy as np
import pytest

from oracle import (Problem, banded_solve, dense_solve, superlu_solve, dst_closed_form,
                    dst_mode, green_1d, laplacian_eigenvalues)


def _rand_field(shape, seed):
    return np.exp(np.random.default_rng(seed).normal(-11.5, 1.0, shape))


@pytest.mark.parametrize("shape", [(6, 8), (5, 4, 3)])
def test_banded_equals_dense_and_superlu(shape):
    pb = Problem.fv(_rand_field(shape, 11))
    rng = np.random.default_rng(2)
    b = rng.normal(size=pb.n) + 1j * rng.normal(size=pb.n)
    for sigma in (2j * np.pi / 10, 2j * np.pi / 1000):
        A = pb.shifted(sigma)
        xd = dense_solve(A, b)
        blk = shape[-1] if len(shape) == 2 else shape[-1] * shape[-2]
        xb = banded_solve(A, b, blk)
        xs = superlu_solve(A, b)
        assert np.allclose(xb, xd, rtol=1e-10, atol=0)
        assert np.allclose(xs, xd, rtol=1e-10, atol=0)


@pytest.mark.parametrize("dims", [(7, 5), (4, 3, 5)])
def test_dst_closed_form_equals_dense(dims):
    K0, Ss, h = 1.3e-5, 1e-5, 1.0
    shape = tuple(reversed(dims))
    pb = Problem.fv(np.full(shape, K0), Ss, h)
    rng = np.random.default_rng(5)
    b = rng.normal(size=pb.n) + 0j
    for sigma in (0.5j, 2j * np.pi / 3000):
        x = dst_closed_form(K0, Ss, h, dims, sigma, b)
        assert np.allclose(x, dense_solve(pb.shifted(sigma), b), rtol=1e-10)


def test_dst_mode_is_eigenvector():
    dims = (6, 5)
    K0 = 2e-5
    pb = Problem.fv(np.full((5, 6), K0))
    v = dst_mode(dims, (2, 3))
    lam = laplacian_eigenvalues(dims)[3 - 1, 2 - 1] * K0
    assert np.allclose(pb.K @ v, lam * v, rtol=1e-12, atol=1e-20)


def test_green_1d_closed_form():
    N, K0, Ss, h = 40, 1e-5, 1e-5, 1.0
    pb = Problem.fv(np.full((N,), K0), Ss, h)
    for sigma in (2j * np.pi / 50, 2j * np.pi / 5000):
        G = green_1d(N, K0, Ss, h, sigma)
        Ainv = np.linalg.inv(pb.shifted(sigma).toarray())
        assert np.allclose(G, Ainv, rtol=1e-9, atol=0)
