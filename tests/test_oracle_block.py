"""Pins of the oracle's block FGMRES-Sh (the block extension of Algorithms 3
and 4 for several right-hand sides sharing K and M) against exact solutions,
the block Arnoldi relations, the one-vector oracle and properties of the block
Krylov space."""
import numpy as np

import synth
from oracle import Problem, fgmres_sh, exact_family, dst_mode, CONVERGED, BREAKDOWN_EXACT
from oracle.block import block_fgmres_sh, block_mgs_step, qr_pos, shifted_block_hessenberg


def _setup(shape=(14, 12), n_f=6, s=3, seed=4):
    K = synth.cell_conductivity(shape, -11.5, 1.0, 5, cfg=93, idx=seed)
    pb = Problem.fv(K)
    sig = synth.shifts_from_periods(synth.periods(n_f, 10.0, 1000.0))
    cells = synth.distinct_interior_cells(shape, s, 93 + seed, synth.P_WELLS)
    B = np.zeros((pb.n, s), complex)
    for r, c in enumerate(cells):
        B[c, r] = 1.0
    return pb, sig, B


def test_qr_pos_and_block_mgs_step():
    rng = np.random.default_rng(1)
    W = rng.normal(size=(40, 4)) + 1j * rng.normal(size=(40, 4))
    Q, R = qr_pos(W)
    assert np.allclose(Q @ R, W, atol=1e-13)
    assert np.allclose(Q.conj().T @ Q, np.eye(4), atol=1e-13)
    assert np.all(np.abs(np.diag(R).imag) < 1e-14) and np.all(np.diag(R).real > 0)
    assert np.allclose(np.tril(R, -1), 0)
    V1, _ = qr_pos(rng.normal(size=(40, 4)) + 1j * rng.normal(size=(40, 4)))
    V2, _ = qr_pos(rng.normal(size=(40, 4)) - 1j * (V1 @ rng.normal(size=(4, 4))))
    V2 = V2 - V1 @ (V1.conj().T @ V2)
    V2, _ = qr_pos(V2)
    Hs, Rn, Vn = block_mgs_step([V1, V2], W)
    # W = V1 H1 + V2 H2 + Vn Rn, with Vn orthogonal to both blocks
    assert np.allclose(V1 @ Hs[0] + V2 @ Hs[1] + Vn @ Rn, W, atol=1e-12)
    assert np.allclose(V1.conj().T @ Vn, 0, atol=1e-12) and np.allclose(V2.conj().T @ Vn, 0, atol=1e-12)


def test_block_arnoldi_relations_exact_and_inexact():
    pb, sig, B = _setup()
    s = B.shape[1]
    for inner, eps in (("dense", 0.0), ("cocg", 1e-6)):
        r = block_fgmres_sh(pb, B, sig, sig[[1, 4]], m=8, tol=1e-14, inner=inner, eps=eps, keep_basis=True)
        V, Z, H, T = r.V, r.Z, r.H, np.repeat(r.taus, s)
        kz = Z.shape[1]
        # block eq. arnoldimod: M Z = V Hbar
        assert np.linalg.norm(pb.Mdiag[:, None] * Z - V @ H) <= 1e-12 * np.linalg.norm(pb.Mdiag[:, None] * Z)
        assert np.allclose(V.conj().T @ V, np.eye(V.shape[1]), atol=1e-12)
        # block eq. zmvmrelation with the inner residuals: K Z + M Z T = V_m - P
        lhs = pb.K @ Z + pb.Mdiag[:, None] * Z * T[None, :]
        assert np.linalg.norm(lhs - (V[:, :kz] - r.P)) <= 1e-12 * np.linalg.norm(V[:, :kz])
        if inner == "cocg":
            assert np.all(r.pnorms <= eps * 1.0 + 1e-15)
        # shifted relation: (K + sigma M) Z = V Hbar(sigma;T) - P
        for j in (0, 5):
            Hs = shifted_block_hessenberg(H, r.taus, s, sig[j])
            A = pb.K @ Z + sig[j] * pb.Mdiag[:, None] * Z
            assert np.linalg.norm(A - (V @ Hs - r.P)) <= 1e-11 * np.linalg.norm(A)


def test_exact_inner_gives_direct_solutions():
    pb, sig, B = _setup(s=4)
    r = block_fgmres_sh(pb, B, sig, sig[[1, 4]], m=40, tol=1e-10, inner="dense")
    for c in range(B.shape[1]):
        xe = exact_family(pb, sig, B[:, c], "dense")
        for j in range(len(sig)):
            q = r.info[c][j]
            assert q.status == CONVERGED and q.true_relres <= 1e-10 * 1.01
            assert np.linalg.norm(r.x[:, j, c] - xe[:, j]) <= 1e-6 * np.linalg.norm(xe[:, j])


def test_one_column_block_is_the_one_vector_method():
    pb, sig, B = _setup(s=1)
    taus = sig[[1, 3, 5]]
    rb = block_fgmres_sh(pb, B, sig, taus, m=50, tol=1e-8, inner="cocg", eps=1e-10)
    r1 = fgmres_sh(pb, B[:, 0], sig, taus, m_restart=50, tol=1e-8, inner="cocg", eps=1e-10)
    assert rb.outer_steps == r1.outer_steps
    for j in range(len(sig)):
        assert rb.info[0][j].outer_its == r1.info[j].outer_its
        assert rb.info[0][j].status == r1.info[j].status
        assert np.linalg.norm(rb.x[:, j, 0] - r1.x[:, j]) <= 1e-10 * np.linalg.norm(r1.x[:, j])


def test_block_space_contains_each_vector_space():
    """With exact inner solves and the same tau sequence the block space after
    k steps contains each right-hand side's own flexible Krylov space, so the
    block least-squares residual of every pair is at most the one-vector
    method's at every step."""
    pb, sig, B = _setup(s=3)
    taus = sig[[1, 4]]
    m = 6
    rb = block_fgmres_sh(pb, B, sig, taus, m=m, tol=1e-30, inner="dense")
    for c in range(B.shape[1]):
        r1 = fgmres_sh(pb, B[:, c], sig, taus, m_restart=m, tol=1e-30, inner="dense", record_quasi=True,
                       max_restarts=0)
        q1 = r1.quasi_hist
        for k in range(m):
            qb, qs = rb.quasi_hist[k][:, c], q1[k]
            live = np.isfinite(qb) & np.isfinite(qs)     # a pair stops once it has converged
            assert np.all(qb[live] <= qs[live] * (1 + 1e-8) + 1e-13), (c, k)
        # and strictly smaller somewhere: the other columns help
        qb, qs = rb.quasi_hist[m - 1][:, c], q1[m - 1]
        live = np.isfinite(qb) & np.isfinite(qs) & (qs > 1e-12)
        assert np.any(qb[live] < 0.9 * qs[live])


def test_permuting_right_hand_sides_permutes_solutions():
    pb, sig, B = _setup(s=4)
    perm = [2, 0, 3, 1]
    r0 = block_fgmres_sh(pb, B, sig, sig[[2]], m=40, tol=1e-11, inner="dense")
    r1 = block_fgmres_sh(pb, B[:, perm], sig, sig[[2]], m=40, tol=1e-11, inner="dense")
    for c, pc in enumerate(perm):
        for j in range(len(sig)):
            a, b = r1.x[:, j, c], r0.x[:, j, pc]
            assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b)


def test_rank_deficient_block_and_zero_column():
    pb, sig, B = _setup(s=2)
    B3 = np.concatenate([B, B[:, :1] * 2.0, np.zeros((pb.n, 1))], axis=1)   # dependent column and a zero one
    r = block_fgmres_sh(pb, B3, sig, sig[[1, 4]], m=40, tol=1e-10, inner="dense")
    xe0 = exact_family(pb, sig, B[:, 0], "dense")
    for j in range(len(sig)):
        assert r.info[0][j].true_relres <= 1e-10 * 1.01 and r.info[2][j].true_relres <= 1e-10 * 1.01
        assert np.linalg.norm(r.x[:, j, 2] - 2.0 * xe0[:, j]) <= 1e-6 * np.linalg.norm(xe0[:, j])
        assert r.info[3][j].status == CONVERGED and np.all(r.x[:, j, 3] == 0)


def test_eigenmode_block_breaks_down_with_exact_answers():
    """A block of generalized eigenvectors (DST modes of a homogeneous field):
    M Z_1 lies in span V_1, so the first new block vanishes and the square
    projected systems give the exact solutions x = b / (Ss (lambda + sigma))
    (section 3, breakdown means an exact solution)."""
    dims, K0 = (9, 7), 1e-5
    pb = Problem.fv(np.full((7, 9), K0))
    sig = synth.shifts_from_periods(synth.periods(4, 10.0, 1000.0))
    modes = [(1, 1), (2, 3)]
    B = np.stack([dst_mode(dims, md) for md in modes], axis=1).astype(complex)
    r = block_fgmres_sh(pb, B, sig, sig[[1]], m=10, tol=1e-10, inner="dense")
    assert r.outer_steps == 1
    for c, md in enumerate(modes):
        b = B[:, c]
        idx = np.argmax(np.abs(b))
        lam_c = (pb.K @ b)[idx] / b[idx]
        for j in range(len(sig)):
            assert r.info[c][j].status == BREAKDOWN_EXACT
            xe = b / (lam_c + sig[j] * 1e-5)
            assert np.linalg.norm(r.x[:, j, c] - xe) <= 1e-10 * np.linalg.norm(xe)
