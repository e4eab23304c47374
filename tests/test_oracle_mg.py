"""Pins of the oracle's multigrid preconditioner (geometric aggregation V-cycle
preconditioning COCG for the inner solves of section 4)."""
import numpy as np
import pytest

import synth
from oracle import Problem, assemble_stiffness, mass_diagonal, cocg, dense_solve
from oracle.mg import Hierarchy, aggregation, vcycle, pcocg, mg_cocg


def test_aggregation_groups_cells_and_keeps_odd_edges():
    P, cshape = aggregation((3, 5))                 # ny = 3, nx = 5
    assert cshape == (2, 3)
    P = P.toarray()
    assert np.all(P.sum(axis=1) == 1)              # every fine cell in one group
    counts = P.sum(axis=0).reshape(cshape)
    assert counts.tolist() == [[4, 4, 2], [2, 2, 1]]
    # fine (y=2, x=4) -> coarse (1, 2); fine (y=1, x=3) -> coarse (0, 1)
    assert P[2 * 5 + 4, 1 * 3 + 2] == 1 and P[1 * 5 + 3, 0 * 3 + 1] == 1


@pytest.mark.parametrize("shape", [(8, 8), (4, 4, 4), (6, 10)])
def test_coarse_operator_is_the_2h_discretisation_for_homogeneous_K(shape):
    K0, Ss = 2.5e-5, 1e-5
    fine = np.full(shape, K0)
    H = Hierarchy.of(Problem.fv(fine, Ss, 1.0))
    cshape = tuple(s // 2 for s in shape)
    Kc = assemble_stiffness(np.full(cshape, K0), h=2.0)
    assert np.allclose(H.K[1].toarray(), Kc.toarray(), rtol=1e-14, atol=0)
    assert np.allclose(H.M[1], mass_diagonal(cshape, Ss, 2.0), rtol=1e-14)
    assert H.shape[-1] == tuple(1 for _ in shape)


def _field(shape, seed):
    return synth.cell_conductivity(shape, -11.5, 1.0, 3, cfg=90, idx=seed)


@pytest.mark.parametrize("shape,nu", [((13, 10), 1), ((9, 7, 6), 2)])
def test_vcycle_is_linear_and_complex_symmetric(shape, nu):
    op = Problem.fv(_field(shape, len(shape)))
    H = Hierarchy.of(op)
    tau = 2j * np.pi / 200.0
    rng = np.random.default_rng(3)
    x = rng.normal(size=op.n) + 1j * rng.normal(size=op.n)
    y = rng.normal(size=op.n) + 1j * rng.normal(size=op.n)
    Bx, By = vcycle(H, tau, x, nu), vcycle(H, tau, y, nu)
    a = 0.3 - 1.7j
    assert np.allclose(vcycle(H, tau, a * x + y, nu), a * Bx + By, rtol=1e-12, atol=1e-12 * np.abs(Bx).max())
    lhs, rhs = y @ Bx, x @ By                        # bilinear, no conjugation
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(y) @ np.abs(Bx))


def test_vcycle_is_exact_on_one_cell():
    op = Problem.fv(np.full((1, 1), 3e-5))
    H = Hierarchy.of(op)
    tau = 0.7j
    b = np.array([2.0 - 1.0j])
    assert H.levels == 1
    assert np.allclose(vcycle(H, tau, b), dense_solve(op.shifted(tau), b), rtol=1e-15)


def test_pcocg_with_jacobi_reproduces_cocg():
    op = Problem.fv(_field((12, 11), 5))
    tau = 2j * np.pi / 50.0
    v = synth.unit_vector(op.n, 40)
    d = op.diag(tau)
    for k in (1, 4, 9):
        xa, _, _, _ = cocg(lambda x: op.apply(tau, x), d, v, 0.0, 100, fixed_iters=k)
        xb, _, _, _ = pcocg(lambda x: op.apply(tau, x), lambda r: r / d, v, 0.0, 100, fixed_iters=k)
        assert np.allclose(xa, xb, rtol=1e-13, atol=1e-13 * np.abs(xa).max())


@pytest.mark.parametrize("shape,T", [((24, 20), 5000.0), ((24, 20), 20.0), ((6, 7, 5), 1000.0)])
def test_mg_cocg_solves_and_beats_jacobi(shape, T):
    op = Problem.fv(_field(shape, 7))
    tau = 2j * np.pi / T
    v = synth.unit_vector(op.n, op.n // 2 + 3)
    x, its, ok, _ = mg_cocg(op, tau, v, 1e-10, 500)
    assert ok
    assert np.linalg.norm(v - op.apply(tau, x)) <= 1e-10 * np.linalg.norm(v) * (1 + 1e-9)
    xe = dense_solve(op.shifted(tau), v)
    # ||x - x*|| <= ||r|| / (omega Ss) for K positive semidefinite (sigma M = i omega Ss h^d)
    assert np.linalg.norm(x - xe) <= 1e-10 / (abs(tau) * 1e-5) * (1 + 1e-6)
    _, jits, jok, _ = cocg(lambda y: op.apply(tau, y), op.diag(tau), v, 1e-10, 5000)
    assert jok and its < jits


def test_fgmres_sh_with_multigrid_inner_matches_direct():
    """Algorithm 4 with the multigrid-preconditioned inner solve: every shift to
    the requested true residual, and the solutions agree with the direct
    per-shift solve within the residual bound."""
    from oracle import fgmres_sh, exact_family
    op = Problem.fv(_field((20, 18), 11))
    sig = synth.shifts_from_periods(synth.periods(6, 10.0, 1000.0))
    b = synth.unit_vector(op.n, 190)
    res = fgmres_sh(op, b, sig, sig[[1, 4]], m_restart=30, tol=1e-9, inner="mg", eps=1e-11)
    xe = exact_family(op, sig, b, "dense")
    for j, s in enumerate(sig):
        r = np.linalg.norm(b - op.apply(s, res.x[:, j]))
        assert r <= 1e-9 * np.linalg.norm(b) * (1 + 1e-6)
        assert np.linalg.norm(res.x[:, j] - xe[:, j]) <= r / (abs(s) * 1e-5) * (1 + 1e-6)
    assert res.inner_its < 40 * res.outer_steps
