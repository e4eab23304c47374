"""Pins of the oracle's inner solver (Jacobi-COCG)."""
import numpy as np
import pytest

from oracle import Problem, cocg


def _problem(shape=(5, 6), seed=4):
    return Problem.fv(np.exp(np.random.default_rng(seed).normal(-11.5, 1.0, shape)))


def test_converges_and_true_residual_small():
    pb = _problem((12, 10))
    tau = 2j * np.pi / 77.0
    v = np.zeros(pb.n, complex)
    v[55] = 1.0
    z, its, ok, hist = cocg(lambda x: pb.apply(tau, x), pb.diag(tau), v, 1e-10, 2000)
    assert ok
    assert np.linalg.norm(v - pb.apply(tau, z)) <= 2e-10
    assert hist[-1] <= 1e-10


def test_galerkin_property_of_iterates():
    # COCG's k-th iterate satisfies the bilinear Galerkin condition on the
    # preconditioned Krylov space W = span{u0, D^-1 A u0, ...}: W^T (v - A x_k) = 0,
    # so x_k = W (W^T A W)^{-1} W^T v.  Compared against that explicit solve.
    pb = _problem((4, 5), 9)
    tau = 0.03j
    A = pb.shifted(tau).toarray()
    D = pb.diag(tau)
    rng = np.random.default_rng(1)
    v = rng.normal(size=pb.n) + 1j * rng.normal(size=pb.n)
    for k in (1, 3, 6):
        xk, its, _, _ = cocg(lambda x: A @ x, D, v, 0.0, 100, fixed_iters=k)
        assert its == k
        W = np.zeros((pb.n, k), complex)
        w = v / D
        for i in range(k):
            W[:, i] = w
            w = (A @ w) / D
        Q, _ = np.linalg.qr(W)   # same span, better conditioned
        xg = Q @ np.linalg.solve(Q.T @ A @ Q, Q.T @ v)
        assert np.allclose(xk, xg, rtol=1e-8, atol=1e-8 * np.linalg.norm(xg))


def test_terminates_within_dimension():
    pb = _problem((4, 4), 2)
    tau = 0.2j
    v = np.random.default_rng(0).normal(size=16) + 0j
    z, its, ok, _ = cocg(lambda x: pb.apply(tau, x), pb.diag(tau), v, 1e-12, 200)
    assert ok and its <= pb.n + 2


def test_zero_rhs():
    pb = _problem((3, 3))
    z, its, ok, _ = cocg(lambda x: pb.apply(1j, x), pb.diag(1j), np.zeros(9, complex), 1e-8, 10)
    assert ok and its == 0 and not z.any()
