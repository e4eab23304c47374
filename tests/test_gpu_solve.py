"""GPU parity of whole FGMRES-Sh solves against the oracle and exact solutions.

Several results are correct at once here (iterative solutions within a
tolerance), so the tests compare what is unique: the exact solution of each
shifted system (oracle banded elimination / SuperLU / closed form), the FP64
true residual against the target, and the per-shift outer step counts (equal
to the oracle's within one step at the stopping threshold).  Error bound used:
||x - x*|| / ||x*|| <= kappa_j * relres with kappa_j = ||A_j|| ||A_j^-1||
estimated from the extreme eigenvalues; the tests use a fixed factor 2e3 that
exceeds the condition numbers of these operators (max ~1e3 for the lowest
frequency on 64x64).
"""
import numpy as np
import pytest

import synth
from oracle import Problem as OProblem, exact_family, fgmres_sh, dst_closed_form, dst_mode, \
    laplacian_eigenvalues, superlu_solve
from tests.gpu_util import require_gpu, to_dev, announce

pytestmark = pytest.mark.gpu


def _params(P, w, **kw):
    a = dict(m_restart=w.m_restart, max_restarts=20, max_refine=2, tol=w.tol, eps_inner=w.eps_inner)
    a.update(kw)
    return P.make_params(w.tau_seq, **a)


def test_config1_fp64_all_shifts_and_oracle_agreement():
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce("c1 fp64")
    w = synth.config1()
    op = OProblem.fv(w.cell_K, w.Ss, w.h)
    gp = P.Problem.fv2d(w.cell_K, w.Ss, w.h)
    prm, keep = _params(P, w)
    x, st = P.fgmres_sh_solve(gp, prm, w.sigma, w.b)          # host pointers
    xe = exact_family(op, w.sigma, w.b[:, 0], "banded")
    ro = fgmres_sh(op, w.b[:, 0], w.sigma, w.tau_seq, m_restart=50, tol=w.tol, inner="cocg", eps=w.eps_inner)
    for j in range(len(w.sigma)):
        s = st[0, j]
        assert s["status"] == P.SHK_CONVERGED, (j, s)
        assert s["true_relres"] <= 1e-8
        err = np.linalg.norm(x[:, j, 0] - xe[:, j]) / np.linalg.norm(xe[:, j])
        assert err <= 2e3 * 1e-8, (j, err)
        assert abs(int(s["outer_its"]) - ro.info[j].outer_its) <= 1
    # device pointers give the same numbers
    bd = to_dev(w.b[:, 0])[None, :].contiguous()
    xd, st2 = P.fgmres_sh_solve(gp, prm, w.sigma, bd)
    assert np.array_equal(xd[0].cpu().numpy().T, x[:, :, 0])


def test_determinism_bitwise():
    require_gpu()
    import paper_1212_3660_amd as P
    announce("determinism")
    w = synth.config1()
    gp = P.Problem.fv2d(w.cell_K, w.Ss, w.h)
    prm, keep = _params(P, w)
    x1, s1 = P.fgmres_sh_solve(gp, prm, w.sigma, w.b)
    x2, s2 = P.fgmres_sh_solve(gp, prm, w.sigma, w.b)
    assert np.array_equal(x1, x2) and np.array_equal(s1, s2)


def test_homogeneous_closed_form_ragged_grid():
    require_gpu()
    import paper_1212_3660_amd as P
    announce("closed form 61x47")
    dims, K0 = (61, 47), 1.1e-5
    Kc = np.full((47, 61), K0)
    gp = P.Problem.fv2d(Kc)
    sig = synth.shifts_from_periods(synth.periods(8, 10, 1000))
    b = synth.unit_vector(61 * 47, synth.cell_index((47, 61), (30, 20)))
    prm, keep = P.make_params(sig[[1, 5]], tol=1e-9, eps_inner=1e-11, m_restart=60)
    x, st = P.fgmres_sh_solve(gp, prm, sig, b)
    for j, s in enumerate(sig):
        xe = dst_closed_form(K0, 1e-5, 1.0, dims, s, b)
        assert st[0, j]["true_relres"] <= 1e-9
        assert np.linalg.norm(x[:, j, 0] - xe) <= 2e3 * 1e-9 * np.linalg.norm(xe)


def test_eigenmode_breakdown_exact():
    require_gpu()
    import paper_1212_3660_amd as P
    announce("breakdown")
    dims, K0, Ss = (20, 16), 1.3e-5, 1e-5
    gp = P.Problem.fv2d(np.full((16, 20), K0), Ss)
    b = dst_mode(dims, (3, 2)).astype(complex)
    lam = laplacian_eigenvalues(dims)[1, 2] * K0
    sig = synth.shifts_from_periods(synth.periods(5, 10, 1000))
    prm, keep = P.make_params([0.01j], tol=1e-10, eps_inner=1e-13, m_restart=10)
    x, st = P.fgmres_sh_solve(gp, prm, sig, b)
    for j, s in enumerate(sig):
        assert st[0, j]["status"] == P.SHK_BREAKDOWN_EXACT
        assert st[0, j]["outer_its"] == 1
        assert np.allclose(x[:, j, 0], b / (lam + s * Ss), rtol=1e-9, atol=1e-9 * np.abs(b / (lam + s * Ss)).max())


def test_restart_path_converges():
    require_gpu()
    import paper_1212_3660_amd as P
    announce("restart m=6")
    K = synth.cell_conductivity((32, 32), -11.5, 1.0, 5, cfg=71)
    op = OProblem.fv(K)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(6, 10, 1000))
    b = synth.unit_vector(op.n, 528)
    taus = 2j * np.pi / np.array([20.0, 700.0])
    prm, keep = P.make_params(taus, tol=1e-9, eps_inner=1e-12, m_restart=6, max_restarts=80, max_refine=0)
    x, st = P.fgmres_sh_solve(gp, prm, sig, b)
    ro = fgmres_sh(op, b, sig, taus, m_restart=6, max_restarts=80, tol=1e-9, inner="cocg", eps=1e-12)
    xe = exact_family(op, sig, b, "banded")
    for j in range(len(sig)):
        assert st[0, j]["status"] == P.SHK_CONVERGED
        assert st[0, j]["restarts"] >= 1
        assert abs(int(st[0, j]["outer_its"]) - ro.info[j].outer_its) <= 2
        assert np.linalg.norm(x[:, j, 0] - xe[:, j]) <= 2e3 * 1e-9 * np.linalg.norm(xe[:, j])


def test_multi_rhs_lockstep_matches_single_and_reciprocity():
    require_gpu()
    import paper_1212_3660_amd as P
    announce("multi rhs")
    K = synth.cell_conductivity((48, 48), -11.5, 1.0, 5, cfg=72)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(5, 10, 1000))
    cells = [300, 1200, 1777]
    B = np.zeros((48 * 48, 3), complex)
    for r, c in enumerate(cells):
        B[c, r] = 1.0
    prm, keep = P.make_params(sig[[1, 3]], tol=1e-10, eps_inner=1e-12, m_restart=50)
    X, st = P.fgmres_sh_solve(gp, prm, sig, B)
    assert np.all(st["true_relres"] <= 1e-10)
    for r in range(3):
        xr, _ = P.fgmres_sh_solve(gp, prm, sig, B[:, r])
        assert np.allclose(X[:, :, r], xr[:, :, 0], rtol=1e-7, atol=1e-7 * np.abs(xr).max())
    # reciprocity of the complex-symmetric operator: x_a[cell_b] = x_b[cell_a].
    # Each entry carries an error <= ||A_j^-1|| ||r|| <= tol ||b|| / (omega_j Ss)
    # (K is positive semidefinite and sigma M = i omega Ss I, so
    # |z^H A_j z| >= omega_j Ss ||z||^2); two solves enter each comparison.
    bound = 2 * 1e-10 / (np.abs(sig.imag) * 1e-5)
    for a in range(3):
        for bb in range(3):
            assert np.all(np.abs(X[cells[bb], :, a] - X[cells[a], :, bb]) <= bound)


def test_mixed_precision_with_refinement():
    require_gpu()
    import paper_1212_3660_amd as P
    announce("mixed 128x128")
    K = synth.cell_conductivity((128, 128), -11.5, 1.0, 5, cfg=73)
    op = OProblem.fv(K)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(40, 5, 5000))
    b = synth.unit_vector(op.n, synth.cell_index((128, 128), (64, 64)))
    prm, keep = P.make_params(sig[[4, 20, 36]], tol=1e-6, eps_inner=1e-6, m_restart=50, precision=P.SHK_MIXED,
                              max_refine=4)
    x, st = P.fgmres_sh_solve(gp, prm, sig, b)
    assert np.all(st["true_relres"] <= 1e-6), st["true_relres"]
    assert np.all(st["status"] == P.SHK_CONVERGED)
    for j in (0, 17, 39):
        xe = superlu_solve(op.shifted(sig[j]), b)
        assert np.linalg.norm(x[:, j, 0] - xe) <= 5e3 * 1e-6 * np.linalg.norm(xe)


def test_degenerate_inputs():
    require_gpu()
    import paper_1212_3660_amd as P
    announce("degenerate")
    K = synth.cell_conductivity((16, 16), -11.5, 1.0, 5, cfg=74)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(3, 10, 1000))
    prm, keep = P.make_params(sig[:1], tol=1e-8, eps_inner=1e-10)
    x, st = P.fgmres_sh_solve(gp, prm, sig, np.zeros(256, complex))
    assert not x.any() and np.all(st["status"] == P.SHK_CONVERGED)
    B = np.zeros((256, 2), complex)
    B[10, 1] = 1.0
    x, st = P.fgmres_sh_solve(gp, prm, sig, B)
    assert not x[:, :, 0].any() and np.all(st[1]["true_relres"] <= 1e-8)
    with pytest.raises(P.ShkError):
        P.Problem.fv2d(np.zeros((4, 4)))
    bad, keep2 = P.make_params(sig[:1], m_restart=0)
    with pytest.raises(P.ShkError):
        P.fgmres_sh_solve(gp, bad, sig, np.ones(256, complex))


def test_mgs_orthogonalisation_solve_matches_oracle():
    # the paper's modified Gram-Schmidt (Algorithm 3) on the device: the same
    # outer step counts as the oracle, which uses it too, and the exact
    # solutions; a bad ortho value is a call error
    require_gpu()
    import paper_1212_3660_amd as P
    announce("c1 fp64 mgs")
    w = synth.config1()
    op = OProblem.fv(w.cell_K, w.Ss, w.h)
    gp = P.Problem.fv2d(w.cell_K, w.Ss, w.h)
    prm, keep = _params(P, w, ortho=P.SHK_MGS)
    x, st = P.fgmres_sh_solve(gp, prm, w.sigma, w.b)
    xe = exact_family(op, w.sigma, w.b[:, 0], "banded")
    ro = fgmres_sh(op, w.b[:, 0], w.sigma, w.tau_seq, m_restart=50, tol=w.tol, inner="cocg", eps=w.eps_inner)
    for j in range(len(w.sigma)):
        s = st[0, j]
        assert s["status"] == P.SHK_CONVERGED and s["true_relres"] <= 1e-8, (j, s)
        assert np.linalg.norm(x[:, j, 0] - xe[:, j]) <= 2e3 * 1e-8 * np.linalg.norm(xe[:, j]), j
        assert abs(int(s["outer_its"]) - ro.info[j].outer_its) <= 1
    bad, keep2 = _params(P, w, ortho=5)
    with pytest.raises(P.ShkError):
        P.fgmres_sh_solve(gp, bad, w.sigma, w.b)


@pytest.mark.parametrize("variant", ["gmres", "fom"])
def test_long_bases_on_both_least_squares_kernels(variant):
    # restart length 64 (a wave per (shift, rhs) lane) and 65 (a thread per
    # lane): both reach the direct solutions and agree with each other
    require_gpu()
    import paper_1212_3660_amd as P
    announce(f"m=64/65 {variant}")
    K = synth.cell_conductivity((40, 36), -11.5, 1.0, 5, cfg=73)
    op = OProblem.fv(K)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(9, 5, 3000))
    b = synth.unit_vector(op.n, 700)
    v = P.SHK_FOM if variant == "fom" else P.SHK_GMRES
    xe = exact_family(op, sig, b, "banded")
    xs = []
    for m in (64, 65):
        prm, keep = P.make_params(sig[[1, 4, 7]], tol=1e-9, eps_inner=1e-12, m_restart=m, max_restarts=10,
                                  max_refine=2, variant=v)
        x, st = P.fgmres_sh_solve(gp, prm, sig, b)
        assert np.all(st["status"] == P.SHK_CONVERGED) and np.all(st["true_relres"] <= 1e-9), m
        for j in range(len(sig)):
            assert np.linalg.norm(x[:, j, 0] - xe[:, j]) <= 2e3 * 1e-9 * np.linalg.norm(xe[:, j]), (m, j)
        xs.append(x)
    assert np.allclose(xs[0], xs[1], rtol=0, atol=1e-6 * np.abs(xs[0]).max())


def test_paper_style_blocked_log_tau_schedule():
    # section 2.2.1 / 6.1: n_p = 5 preconditioners log-spaced over the frequency
    # range, each used for a block of m / n_p steps, cycled; every shift
    # converges to the direct solution
    require_gpu()
    import paper_1212_3660_amd as P
    announce("blocked log tau")
    K = synth.cell_conductivity((20, 20), -11.5, 1.0, 5, cfg=75)
    op = OProblem.fv(K)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(20, 3.0, 600.0))
    taus = synth.blocked_tau(synth.log_spaced_tau(2 * np.pi / 600, 2 * np.pi / 3, 5), 40)
    b = synth.unit_vector(op.n, 210)
    prm, keep = P.make_params(taus, tol=1e-10, eps_inner=1e-13, m_restart=40, max_restarts=20, max_refine=2)
    x, st = P.fgmres_sh_solve(gp, prm, sig, b)
    xe = exact_family(op, sig, b, "banded")
    for j in range(len(sig)):
        assert st[0, j]["status"] == P.SHK_CONVERGED and st[0, j]["true_relres"] <= 1e-10, (j, st[0, j])
        assert np.linalg.norm(x[:, j, 0] - xe[:, j]) <= 2e3 * 1e-10 * np.linalg.norm(xe[:, j]), j


def test_single_tau_equal_to_a_shift_converges_in_one_step():
    # Hbar(tau;T) = [I;0] when sigma = tau (eq. shiftedarnoldimod): that shift
    # is exact after one outer step, and shifts far from tau need the most
    require_gpu()
    import paper_1212_3660_amd as P
    announce("sigma = tau")
    K = synth.cell_conductivity((20, 20), -11.5, 1.0, 5, cfg=76)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(9, 3.0, 3000.0))
    b = synth.unit_vector(K.size, 210)
    prm, keep = P.make_params(sig[[4]], tol=1e-9, eps_inner=1e-13, m_restart=150, max_restarts=2, max_refine=2)
    x, st = P.fgmres_sh_solve(gp, prm, sig, b)
    its = np.array([int(st[0, j]["outer_its"]) for j in range(len(sig))])
    assert its[4] == its.min() == 1, its
    assert its[0] > its[3] and its[8] > its[5], its
    assert np.all(st["true_relres"] <= 1e-9)


def test_csr_problem_matches_the_1d_greens_function():
    # a general (CSR) problem: the 1-D homogeneous operator, whose inverse is
    # the closed-form discrete Green's function (K0/h) G
    require_gpu()
    import paper_1212_3660_amd as P
    from oracle import green_1d
    announce("csr 1-D green")
    N, K0, Ss = 300, 1e-5, 1e-5
    op = OProblem.fv(np.full((N,), K0), Ss)
    A = op.K.tocsr()
    gp = P.Problem.csr(A.indptr, A.indices, A.data, op.Mdiag)
    sig = synth.shifts_from_periods(synth.periods(6, 10, 1000))
    b = synth.unit_vector(N, 123)
    prm, keep = P.make_params(sig[[1, 4]], tol=1e-10, eps_inner=1e-13, m_restart=60, max_restarts=20, max_refine=2)
    x, st = P.fgmres_sh_solve(gp, prm, sig, b)
    for j, s_ in enumerate(sig):
        xe = green_1d(N, K0, Ss, 1.0, s_) @ b
        assert st[0, j]["status"] == P.SHK_CONVERGED and st[0, j]["true_relres"] <= 1e-10, (j, st[0, j])
        assert np.linalg.norm(x[:, j, 0] - xe) <= 1e-10 / (abs(s_) * Ss) * np.linalg.norm(b) * 1.01, j


def test_csr_problem_with_identity_mass():
    # M = I turns the family into (K + sigma_j I) x_j = b, the shifted systems
    # the flexible method generalises; against a dense solve of each
    require_gpu()
    import paper_1212_3660_amd as P
    announce("csr identity mass")
    K = synth.cell_conductivity((18, 15), -11.5, 1.0, 5, cfg=77)
    op = OProblem.fv(K)
    A = (op.K * 1e5).tocsr()                  # scale so that the shifts below sit inside its spectrum
    n = A.shape[0]
    gp = P.Problem.csr(A.indptr, A.indices, A.data, np.ones(n))
    sig = 1j * np.array([0.05, 0.2, 1.0, 4.0])
    b = synth.unit_vector(n, 140)
    prm, keep = P.make_params(sig[[0, 2]], tol=1e-10, eps_inner=1e-13, m_restart=80, max_restarts=20, max_refine=2)
    x, st = P.fgmres_sh_solve(gp, prm, sig, b)
    Ad = A.toarray().astype(complex)
    for j, s_ in enumerate(sig):
        xe = np.linalg.solve(Ad + s_ * np.eye(n), b)
        assert st[0, j]["status"] == P.SHK_CONVERGED and st[0, j]["true_relres"] <= 1e-10, (j, st[0, j])
        assert np.linalg.norm(x[:, j, 0] - xe) <= 1e-10 / abs(s_) * np.linalg.norm(b) * 1.01, j


def test_maximum_restart_length():
    # m_restart = 400, the largest accepted: the basis, the packed factors and
    # the thread-per-lane least squares at full length; 401 is a call error
    require_gpu()
    import paper_1212_3660_amd as P
    announce("m = 400")
    K = synth.cell_conductivity((30, 28), -11.5, 1.0, 5, cfg=78)
    op = OProblem.fv(K)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(8, 5, 3000))
    b = synth.unit_vector(op.n, 333)
    prm, keep = P.make_params(sig[[3]], tol=1e-10, eps_inner=1e-13, m_restart=400, max_restarts=2, max_refine=2)
    x, st = P.fgmres_sh_solve(gp, prm, sig, b)
    xe = exact_family(op, sig, b, "banded")
    for j in range(len(sig)):
        assert st[0, j]["status"] == P.SHK_CONVERGED and st[0, j]["true_relres"] <= 1e-10, (j, st[0, j])
        assert np.linalg.norm(x[:, j, 0] - xe[:, j]) <= 2e3 * 1e-10 * np.linalg.norm(xe[:, j]), j
    bad, keep2 = P.make_params(sig[[3]], tol=1e-10, m_restart=401)
    with pytest.raises(P.ShkError):
        P.fgmres_sh_solve(gp, bad, sig, b)


def test_two_thousand_shifts():
    # a large shift family (2000 periods from 2 s to 20000 s) from one basis
    require_gpu()
    import paper_1212_3660_amd as P
    announce("2000 shifts")
    K = synth.cell_conductivity((24, 22), -11.5, 1.0, 5, cfg=79)
    op = OProblem.fv(K)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(2000, 2.0, 20000.0))
    b = synth.unit_vector(op.n, 250)
    prm, keep = P.make_params(sig[[200, 1000, 1800]], tol=1e-9, eps_inner=1e-12, m_restart=30, max_restarts=40,
                              max_refine=2)
    x, st = P.fgmres_sh_solve(gp, prm, sig, b)
    assert np.all(st["status"] == P.SHK_CONVERGED) and np.all(st["true_relres"] <= 1e-9)
    for j in (0, 777, 1999):
        xe = exact_family(op, sig[[j]], b, "banded")[:, 0]
        assert np.linalg.norm(x[:, j, 0] - xe) <= 2e3 * 1e-9 * np.linalg.norm(xe), j


def test_more_right_hand_sides_than_one_group():
    # 66 right-hand sides: a group of 64 lanes, then a group of 2 in the same
    # workspace; every (shift, rhs) converged, the second group's solutions the
    # direct ones
    require_gpu()
    import paper_1212_3660_amd as P
    announce("66 rhs")
    K = synth.cell_conductivity((16, 14), -11.5, 1.0, 5, cfg=80)
    op = OProblem.fv(K)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(5, 10, 1000))
    B = np.zeros((op.n, 66), complex)
    for r in range(66):
        B[(37 * r + 11) % op.n, r] = 1.0
    prm, keep = P.make_params(sig[[1, 3]], tol=1e-9, eps_inner=1e-12, m_restart=60, max_restarts=10, max_refine=2)
    x, st = P.fgmres_sh_solve(gp, prm, sig, B)
    assert x.shape == (op.n, len(sig), 66) and st.shape == (66, len(sig))
    assert np.all(st["status"] == P.SHK_CONVERGED) and np.all(st["true_relres"] <= 1e-9)
    for r in (0, 63, 64, 65):
        xe = exact_family(op, sig, B[:, r], "banded")
        for j in range(len(sig)):
            assert np.linalg.norm(x[:, j, r] - xe[:, j]) <= 2e3 * 1e-9 * np.linalg.norm(xe[:, j]), (r, j)
