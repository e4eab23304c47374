"""Pins of the oracle's FGMRES-Sh (Algorithms 3 and 4, sections 2-4) against
exact solutions, closed forms and the paper's identities and bounds."""
import numpy as np
import pytest

import synth
from oracle import (Problem, fgmres_sh, refine, true_residuals, dense_solve, dst_mode,
                    laplacian_eigenvalues, shifted_hessenberg, exact_family,
                    CONVERGED, INNER_LIMITED, BREAKDOWN_EXACT, NAN_STATUS)


def _field(shape, seed=3, var=1.0):
    return synth.cell_conductivity(shape, -11.5, var, 5 if min(shape) > 6 else 1, cfg=90, idx=seed)


def _setup(shape=(14, 12), n_f=6, seed=3):
    pb = Problem.fv(_field(shape, seed))
    T = synth.periods(n_f, 10.0, 1000.0)
    sig = synth.shifts_from_periods(T)
    b = synth.unit_vector(pb.n, pb.n // 2 + shape[1] // 2)
    return pb, sig, b


def test_exact_inner_matches_dense_solution():
    pb, sig, b = _setup()
    tau = sig[[1, 4]]
    r = fgmres_sh(pb, b, sig, tau, m_restart=60, tol=1e-10, inner="dense")
    xe = exact_family(pb, sig, b, "dense")
    for j in range(len(sig)):
        assert r.info[j].status == CONVERGED
        assert r.info[j].true_relres <= 1e-10 * 1.01
        # error is bounded by the residual times the conditioning; this mild
        # operator keeps it within a few orders of the residual
        assert np.linalg.norm(r.x[:, j] - xe[:, j]) <= 1e-6 * np.linalg.norm(xe[:, j])


def test_arnoldi_relations_exact_and_inexact():
    # eq. arnoldimod M Z = V Hbar, eq. zmvmrelation K Z + M Z T = V_m (exact),
    # eq. flexshiftedarnoldimod (K + sigma M) Z + P = V Hbar(sigma;T) (inexact)
    pb, sig, b = _setup((10, 9))
    for inner, eps in (("dense", 0.0), ("cocg", 1e-6)):
        r = fgmres_sh(pb, b, sig, sig[[0, 3, 5]], m_restart=12, max_restarts=0, tol=1e-30,
                      inner=inner, eps=eps, keep_basis=True)
        V, Z, H, T, P = r.V, r.Z, r.H, r.taus, r.P
        k = Z.shape[1]
        M = pb.Mdiag[:, None]
        scale = np.linalg.norm(M * Z)
        assert np.linalg.norm(M * Z - V @ H) <= 1e-13 * scale
        assert np.linalg.norm(V.conj().T @ V - np.eye(k + 1)) <= 1e-12
        lhs = pb.K @ Z + (M * Z) * T[None, :]
        assert np.linalg.norm(lhs - (V[:, :k] - P)) <= 1e-12 * np.linalg.norm(lhs)
        for s in sig:
            Hs = shifted_hessenberg(H, T, s)
            A = pb.apply(s, Z) + P
            assert np.linalg.norm(A - V @ Hs) <= 1e-12 * np.linalg.norm(A)
        if inner == "cocg":
            assert np.all(r.pnorms <= eps * 1.0001)
            assert np.allclose(np.linalg.norm(P, axis=0), r.pnorms)


def test_sigma_equal_tau_converges_in_one_step():
    # Hbar(tau;tau) = [I;0] so the projected problem is solved exactly at k=1
    pb, sig, b = _setup()
    tau = sig[2]
    r = fgmres_sh(pb, b, sig, [tau], m_restart=40, tol=1e-9, inner="dense")
    assert r.info[2].outer_its == 1
    xe = dense_solve(pb.shifted(tau), b)
    assert np.allclose(r.x[:, 2], xe, rtol=1e-12, atol=1e-12 * np.abs(xe).max())


def test_eigenmode_rhs_breaks_down_with_exact_answer():
    # b a generalised eigenvector (K b = K0 lam M b / Ss): the Krylov space is
    # one-dimensional, h_21 = 0, and x_j = b / (K0 lam + sigma_j Ss)
    dims, K0, Ss = (9, 7), 1.2e-5, 1e-5
    pb = Problem.fv(np.full((7, 9), K0), Ss)
    b = dst_mode(dims, (2, 3)).astype(complex)
    lam = laplacian_eigenvalues(dims)[2, 1] * K0
    sig = synth.shifts_from_periods(synth.periods(5, 10, 1000))
    r = fgmres_sh(pb, b, sig, [0.01j], m_restart=10, tol=1e-10, inner="dense")
    assert r.outer_steps == 1
    for j, s in enumerate(sig):
        assert r.info[j].status == BREAKDOWN_EXACT
        assert np.allclose(r.x[:, j], b / (lam + s * Ss), rtol=1e-11)


def test_true_residual_gap_bound():
    # eq. resdiff: ||r - r~|| <= sum |y_k| ||p_k|| <= eps ||y||_1; eq. trueresidual
    pb, sig, b = _setup((16, 16), 8)
    eps = 1e-6
    r = fgmres_sh(pb, b, sig, sig[[1, 4, 6]], m_restart=40, tol=1e-12, max_restarts=0,
                  inner="cocg", eps=eps, keep_basis=True)
    for j, (y, qv) in r.y_last.items():
        k = len(y)
        true = b - pb.apply(sig[j], r.Z[:, :k] @ y)
        inexact = r.V[:, :k + 1] @ qv
        gap = np.linalg.norm(true - inexact)
        assert gap <= np.sum(np.abs(y) * r.pnorms[:k]) * (1 + 1e-9) + 1e-14
        assert np.sum(np.abs(y) * r.pnorms[:k]) <= eps * np.sum(np.abs(y)) * 1.0001
        assert np.linalg.norm(true) <= (np.linalg.norm(qv) + eps * np.sum(np.abs(y))) * 1.0001


def test_fom_residual_closed_form_and_prop3_bound():
    # FOM residual = -(sigma - tau_m) h_{m+1,m} (e_m^T y) v_{m+1} (proof of
    # Prop. 2) and ||r_fom - r_gmres|| <= alpha (1+alpha)/(1+alpha^2) ||r_fom||
    # (Prop. 3), alpha = ||eta H_m(sigma;T)^{-H} e_m||, eta = h_{m+1,m}(sigma - tau_m).
    pb, sig, b = _setup((10, 10), 5)
    r = fgmres_sh(pb, b, sig, sig[[0, 4]], m_restart=6, max_restarts=0, tol=1e-30,
                  inner="dense", keep_basis=True)
    V, Z, H, T = r.V, r.Z, r.H, r.taus
    m = Z.shape[1]
    for s in sig:
        Hs = shifted_hessenberg(H, T, s)
        rhs = np.zeros(m + 1, complex)
        rhs[0] = np.linalg.norm(b)
        y_f = np.linalg.solve(Hs[:m, :m], rhs[:m])
        y_g = np.linalg.lstsq(Hs, rhs, rcond=None)[0]
        r_f = b - pb.apply(s, Z @ y_f)
        r_g = b - pb.apply(s, Z @ y_g)
        eta = H[m, m - 1] * (s - T[m - 1])
        closed = -eta * y_f[m - 1] * V[:, m]
        assert np.linalg.norm(r_f - closed) <= 1e-10 * np.linalg.norm(r_f) + 1e-13 * np.linalg.norm(b)
        em = np.zeros(m, complex)
        em[-1] = 1
        alpha = np.linalg.norm(eta * np.linalg.solve(Hs[:m, :m].conj().T, em))
        assert np.linalg.norm(r_f - r_g) <= (alpha * (1 + alpha) / (1 + alpha ** 2) * np.linalg.norm(r_f) * (1 + 1e-9)
                                             + 1e-13 * np.linalg.norm(b))


def test_reciprocity_and_conjugate_symmetry():
    # K + sigma M is complex symmetric: e_r^T x(e_s) = e_s^T x(e_r); for real b
    # x(conj sigma) = conj x(sigma)
    pb, sig, _ = _setup((12, 12), 4)
    s_cell, r_cell = 30, 101
    kw = dict(m_restart=60, tol=1e-11, inner="dense")
    xs = fgmres_sh(pb, synth.unit_vector(pb.n, s_cell), sig, sig[[0, 3]], **kw).x
    xr = fgmres_sh(pb, synth.unit_vector(pb.n, r_cell), sig, sig[[0, 3]], **kw).x
    assert np.allclose(xs[r_cell], xr[s_cell], rtol=1e-8)
    xc = fgmres_sh(pb, synth.unit_vector(pb.n, s_cell), sig.conj(), sig[[0, 3]].conj(), **kw).x
    assert np.allclose(xc, xs.conj(), rtol=1e-8, atol=1e-8 * np.abs(xs).max())


def test_identity_mass_reduces_to_shifted_a_plus_sigma():
    # M = I (Gu et al.'s setting (A + sigma I) x = b): same method, exact answers
    rng = np.random.default_rng(0)
    n = 30
    B = rng.normal(size=(n, n))
    A = B @ B.T + n * np.eye(n)
    pb = Problem(A, np.ones(n))
    b = rng.normal(size=n) + 0j
    sig = np.array([0.5j, 3.0j, 10.0 + 1j])
    r = fgmres_sh(pb, b, sig, [1j, 5j], m_restart=40, tol=1e-11, inner="dense")
    for j, s in enumerate(sig):
        assert np.allclose(r.x[:, j], np.linalg.solve(A + s * np.eye(n), b), rtol=1e-9)


def test_restart_keeps_residuals_collinear_and_converges():
    pb, sig, b = _setup((14, 14), 6)
    tau = 2j * np.pi / np.array([20.0, 700.0])   # no shift equals a tau: all stay active
    r = fgmres_sh(pb, b, sig, tau, m_restart=5, tol=1e-30, inner="dense", stop_after_restart=0)
    R = np.stack([b - pb.apply(s, r.x[:, j]) for j, s in enumerate(sig)], axis=1)
    sv = np.linalg.svd(R, compute_uv=False)
    assert sv[1] <= 1e-8 * sv[0]
    # residual of shift j equals beta_j times the new start vector direction
    beta = r.y_last["beta"]
    seed = r.y_last["seed"]
    v1 = R[:, seed] / np.linalg.norm(R[:, seed])
    for j in range(len(sig)):
        assert np.allclose(R[:, j], beta[j] * v1, atol=1e-9 * np.linalg.norm(R[:, j]) + 1e-300)
    full = fgmres_sh(pb, b, sig, tau, m_restart=5, max_restarts=60, tol=1e-9, inner="dense")
    xe = exact_family(pb, sig, b, "dense")
    for j in range(len(sig)):
        assert full.info[j].status == CONVERGED and full.info[j].restarts >= 1 or full.info[j].outer_its <= 5
        assert np.linalg.norm(full.x[:, j] - xe[:, j]) <= 1e-6 * np.linalg.norm(xe[:, j])


def test_fom_variant_and_fom_restart():
    pb, sig, b = _setup((12, 10), 5)
    r = fgmres_sh(pb, b, sig, sig[[0, 2, 4]], m_restart=8, max_restarts=40, tol=1e-9,
                  inner="dense", variant="fom")
    xe = exact_family(pb, sig, b, "dense")
    for j in range(len(sig)):
        assert r.info[j].true_relres <= 1.5e-9
        assert np.linalg.norm(r.x[:, j] - xe[:, j]) <= 1e-6 * np.linalg.norm(xe[:, j])


def test_inexact_inner_floor_and_refinement():
    # an inner tolerance above the target limits the attainable residual
    # (section 4, eq. trueresidual): every shift stops INNER_LIMITED near eps;
    # one collinear refinement sweep with FP64 true residuals meets the target
    pb, sig, b = _setup((24, 24), 10)
    eps, tol = 3e-6, 1e-6
    r = fgmres_sh(pb, b, sig, sig[[1, 5, 8]], m_restart=50, tol=tol, inner="cocg", eps=eps)
    rel0 = true_residuals(pb, b, sig, r.x)
    assert all(s.status == INNER_LIMITED for s in r.info)
    assert np.all(rel0 > tol) and np.all(rel0 < 2 * eps)
    x = r.x.copy()

    def solve(rhs):
        return fgmres_sh(pb, rhs, sig, sig[[1, 5, 8]], m_restart=50, tol=1e-2, inner="cocg", eps=1e-3).x
    sweeps = refine(pb, b, sig, x, solve, tol, 6, r.info)
    assert sweeps == 1
    rel1 = true_residuals(pb, b, sig, x)
    assert np.all(rel1 <= tol) and rel1.max() <= 0.5 * rel0.min()
    assert all(s.status == CONVERGED and s.refine_sweeps == 1 for s in r.info)


def test_paper_style_blocked_log_tau():
    # section 6.1: n_p preconditioners log-spaced over the frequency range,
    # blocks of m/n_p steps, cycled; all shifts converge
    pb = Problem.fv(_field((20, 20), 8))
    T = synth.periods(20, 3.0, 600.0)
    sig = synth.shifts_from_periods(T)
    taus = synth.blocked_tau(synth.log_spaced_tau(2 * np.pi / 600, 2 * np.pi / 3, 5), 40)
    b = synth.unit_vector(pb.n, 210)
    r = fgmres_sh(pb, b, sig, taus, m_restart=40, tol=1e-10, inner="superlu")
    assert all(s.status == CONVERGED for s in r.info)
    assert max(s.true_relres for s in r.info) <= 1.1e-10


def test_single_tau_favours_nearby_shifts():
    # section 2.1 / 6.1: a single preconditioner K + tau M works best for
    # shifts near tau
    pb = Problem.fv(_field((20, 20), 5))
    sig = synth.shifts_from_periods(synth.periods(9, 3.0, 3000.0))
    b = synth.unit_vector(pb.n, 210)
    r = fgmres_sh(pb, b, sig, [sig[4]], m_restart=200, max_restarts=0, tol=1e-10, inner="superlu")
    its = np.array([s.outer_its for s in r.info])
    assert its[4] == its.min() == 1
    assert its[0] > its[3] and its[8] > its[5]


def test_degenerate_inputs():
    pb, sig, b = _setup((6, 6), 3)
    r = fgmres_sh(pb, np.zeros(pb.n, complex), sig, sig[:1], inner="dense")
    assert all(s.status == CONVERGED for s in r.info) and not r.x.any()
    bn = b.copy()
    bn[3] = np.nan
    r = fgmres_sh(pb, bn, sig, sig[:1], inner="dense")
    assert all(s.status == NAN_STATUS for s in r.info)


def test_three_dimensional_and_general_matrix():
    pb = Problem.fv(_field((5, 6, 7), 2))
    sig = synth.shifts_from_periods(synth.periods(4, 10, 1000))
    b = synth.unit_vector(pb.n, 100)
    r = fgmres_sh(pb, b, sig, sig[[0, 3]], m_restart=60, tol=1e-10, inner="cocg", eps=1e-12)
    xe = exact_family(pb, sig, b, "superlu")
    for j in range(len(sig)):
        assert r.info[j].true_relres <= 1.2e-10
        assert np.linalg.norm(r.x[:, j] - xe[:, j]) <= 1e-6 * np.linalg.norm(xe[:, j])
