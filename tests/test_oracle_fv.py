"""Pins of the oracle's operator assembly (section 5.1, eq. phasor1/genshifted)
against values fixed by hand derivation and by closed forms."""
import json
import os

import numpy as np
import pytest

from oracle import Problem, assemble_stiffness, mass_diagonal, laplacian_eigenvalues

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_derived_3x2():
    g = json.load(open(os.path.join(GOLD, "fv_3x2_hand.json")))
    K = assemble_stiffness(np.array(g["cell_K"]), 1.0).toarray()
    ref = np.array(g["K_num"], dtype=float) / g["K_den"]
    assert np.allclose(K, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dims", [(5, 4), (3, 7), (4, 3, 5)])
def test_homogeneous_spectrum_is_dirichlet_laplacian(dims):
    # Homogeneous K0: the operator must be K0 h^(d-2) times the Dirichlet
    # Laplacian, whose eigenvalues are sums of 4 sin^2(p pi / (2(n+1))).
    K0, h = 2.5e-5, 0.7
    shape = tuple(reversed(dims))
    K = assemble_stiffness(np.full(shape, K0), h).toarray()
    ev = np.sort(np.linalg.eigvalsh(K))
    lam = np.sort(laplacian_eigenvalues(dims).ravel()) * K0 * h ** (len(dims) - 2)
    assert np.allclose(ev, lam, rtol=1e-12, atol=1e-20)


def test_structure_invariants():
    rng = np.random.default_rng(7)
    Kc = np.exp(rng.normal(-11.5, 1.0, (6, 9)))
    K = assemble_stiffness(Kc, 1.0)
    Kd = K.toarray()
    assert np.allclose(Kd, Kd.T)
    assert np.all(np.linalg.eigvalsh(Kd) > 0)
    # interior rows conserve flux: row sums vanish away from the boundary
    rs = Kd.sum(axis=1).reshape(Kc.shape)
    assert np.allclose(rs[1:-1, 1:-1], 0.0, atol=1e-18)
    # a boundary (non-corner) cell on the west edge loses exactly its own K
    assert np.isclose(rs[3, 0], Kc[3, 0])
    # corner: two boundary faces
    assert np.isclose(rs[0, 0], 2 * Kc[0, 0])
    # off-diagonals are non-positive, 5-point pattern
    off = Kd - np.diag(np.diag(Kd))
    assert np.all(off <= 0)
    assert np.all((off != 0).sum(axis=1) <= 4)


def test_h_scaling_and_mass():
    rng = np.random.default_rng(3)
    Kc2 = np.exp(rng.normal(-11, 0.5, (4, 5)))
    Kc3 = np.exp(rng.normal(-11, 0.5, (3, 4, 5)))
    for Kc, d in ((Kc2, 2), (Kc3, 3)):
        a = assemble_stiffness(Kc, 1.0).toarray()
        b = assemble_stiffness(Kc, 2.0).toarray()
        assert np.allclose(b, a * 2.0 ** (d - 2))
        assert np.allclose(mass_diagonal(Kc.shape, 1e-5, 2.0), 1e-5 * 2.0 ** d)


def test_problem_apply_matches_matrix():
    rng = np.random.default_rng(1)
    Kc = np.exp(rng.normal(-11.5, 1, (5, 6)))
    pb = Problem.fv(Kc)
    x = rng.normal(size=30) + 1j * rng.normal(size=30)
    s = 0.37j
    assert np.allclose(pb.apply(s, x), pb.shifted(s).toarray() @ x)
