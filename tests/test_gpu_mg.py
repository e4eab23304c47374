"""GPU parity of the multigrid-preconditioned inner solve and of FGMRES-Sh with
it, against the oracle (oracle.mg)."""
import numpy as np
import pytest

import synth
from oracle import Problem as OProblem, superlu_solve, exact_family
from oracle.mg import Hierarchy, mg_cocg
from tests.gpu_util import require_gpu, to_dev, announce

pytestmark = pytest.mark.gpu


def _field(shape, seed):
    return synth.cell_conductivity(shape, -11.5, 1.0, 5, cfg=91, idx=seed)


def _gpu_problem(P, K):
    return P.Problem.fv2d(K) if K.ndim == 2 else P.Problem.fv3d(K)


@pytest.mark.parametrize("shape,S", [((37, 29), 1), ((24, 40), 4), ((11, 9, 7), 2)])
def test_mg_cocg_iterates_match_oracle(shape, S):
    """Fixed iteration counts: the single-reduction GPU arrangement gives the
    textbook preconditioned-COCG iterates, with the same V-cycle."""
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce(f"mg iterates {shape} S={S}")
    K = _field(shape, len(shape))
    op = OProblem.fv(K)
    gp = _gpu_problem(P, K)
    H = Hierarchy.of(op)
    tau = 2j * np.pi / 700.0
    rng = np.random.default_rng(5)
    V = rng.normal(size=(op.n, S)) + 1j * rng.normal(size=(op.n, S))
    for k in (1, 3, 8):
        z = torch.zeros(op.n * S, dtype=torch.complex128, device="cuda")
        P.shk_inner_solve(gp, tau, to_dev(V.ravel()), z, fixed_iters=k, n_rhs=S, precond=P.SHK_PRECOND_MULTIGRID)
        Z = z.cpu().numpy().reshape(op.n, S)
        for r in range(S):
            xo, _, _, _ = mg_cocg(op, tau, V[:, r], 0.0, 100, H, fixed_iters=k)
            assert np.allclose(Z[:, r], xo, rtol=0, atol=1e-9 * np.abs(xo).max()), (k, r)


@pytest.mark.parametrize("shape", [(64, 64), (33, 50), (12, 10, 9)])
def test_mg_cocg_converges_like_oracle(shape):
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce(f"mg converged {shape}")
    K = _field(shape, 9)
    op = OProblem.fv(K)
    gp = _gpu_problem(P, K)
    H = Hierarchy.of(op)
    v = synth.unit_vector(op.n, op.n // 2 + 1)
    for T in (10.0, 300.0, 5000.0):
        tau = 2j * np.pi / T
        for eps in (1e-6, 1e-10):
            z = torch.zeros(op.n, dtype=torch.complex128, device="cuda")
            its, pn = P.shk_inner_solve(gp, tau, to_dev(v), z, eps=eps, precond=P.SHK_PRECOND_MULTIGRID)
            _, oits, ok, _ = mg_cocg(op, tau, v, eps, 1000, H)
            assert ok and abs(int(its[0]) - oits) <= 1
            true = np.linalg.norm(v - op.apply(tau, z.cpu().numpy()))
            assert true <= 1.5 * eps and np.isclose(pn[0], true, rtol=1e-6)
        # complex64 path: refinement rounds meet eps in the FP64 residual
        z = torch.zeros(op.n, dtype=torch.complex128, device="cuda")
        its, pn = P.shk_inner_solve(gp, tau, to_dev(v, "c64"), z, eps=1e-6, precond=P.SHK_PRECOND_MULTIGRID)
        true = np.linalg.norm(v - op.apply(tau, z.cpu().numpy()))
        assert true <= 1e-6 * 1.01


@pytest.mark.parametrize("shape,S", [((6, 5), 1), ((4, 3, 2), 1), ((7, 9), 2)])
def test_mg_whole_hierarchy_in_one_workgroup(shape, S):
    """Grids small enough for every level to sit in the one-workgroup tail
    (no grid-wide restriction or prolongation at all): iterates as the oracle's,
    complex128 and complex64 inputs."""
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce(f"mg tail only {shape} S={S}")
    K = _field(shape, 3)
    op = OProblem.fv(K)
    gp = _gpu_problem(P, K)
    H = Hierarchy.of(op)
    tau = 2j * np.pi / 90.0
    rng = np.random.default_rng(11)
    V = rng.normal(size=(op.n, S)) + 1j * rng.normal(size=(op.n, S))
    for k in (1, 4):
        z = torch.zeros(op.n * S, dtype=torch.complex128, device="cuda")
        P.shk_inner_solve(gp, tau, to_dev(V.ravel()), z, fixed_iters=k, n_rhs=S, precond=P.SHK_PRECOND_MULTIGRID)
        Z = z.cpu().numpy().reshape(op.n, S)
        for r in range(S):
            xo, _, _, _ = mg_cocg(op, tau, V[:, r], 0.0, 100, H, fixed_iters=k)
            assert np.allclose(Z[:, r], xo, rtol=0, atol=1e-10 * np.abs(xo).max()), (k, r)
    V32 = V.astype(np.complex64).astype(np.complex128)      # the right-hand side the complex64 path sees
    z = torch.zeros(op.n * S, dtype=torch.complex128, device="cuda")
    its, pn = P.shk_inner_solve(gp, tau, to_dev(V32.ravel(), "c64"), z, eps=1e-6, n_rhs=S,
                                precond=P.SHK_PRECOND_MULTIGRID)
    Z = z.cpu().numpy().reshape(op.n, S)
    for r in range(S):
        true = np.linalg.norm(V32[:, r] - op.apply(tau, Z[:, r]))
        assert true <= 1e-6 * np.linalg.norm(V32[:, r]) * 1.01


@pytest.mark.parametrize("shape,S", [((64, 64), 2), ((96, 80), 1), ((24, 20, 18), 1)])
def test_mg_tail_two_levels_down(shape, S):
    """Grids whose one-workgroup tail starts two or more levels down (grid
    restriction and prolongation legs on the levels above it): iterates as the
    oracle's (complex128), and the complex64 path meets its FP64 residual
    target."""
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce(f"mg tail two levels down {shape} S={S}")
    K = _field(shape, 4)
    op = OProblem.fv(K)
    gp = _gpu_problem(P, K)
    H = Hierarchy.of(op)
    tau = 2j * np.pi / 250.0
    rng = np.random.default_rng(13)
    V = rng.normal(size=(op.n, S)) + 1j * rng.normal(size=(op.n, S))
    for k in (1, 3, 8):
        z = torch.zeros(op.n * S, dtype=torch.complex128, device="cuda")
        P.shk_inner_solve(gp, tau, to_dev(V.ravel()), z, fixed_iters=k, n_rhs=S, precond=P.SHK_PRECOND_MULTIGRID)
        Z = z.cpu().numpy().reshape(op.n, S)
        for r in range(S):
            xo, _, _, _ = mg_cocg(op, tau, V[:, r], 0.0, 100, H, fixed_iters=k)
            assert np.allclose(Z[:, r], xo, rtol=0, atol=1e-9 * np.abs(xo).max()), (k, r)
    V32 = V.astype(np.complex64).astype(np.complex128)
    z = torch.zeros(op.n * S, dtype=torch.complex128, device="cuda")
    its, pn = P.shk_inner_solve(gp, tau, to_dev(V32.ravel(), "c64"), z, eps=1e-6, n_rhs=S,
                                precond=P.SHK_PRECOND_MULTIGRID)
    Z = z.cpu().numpy().reshape(op.n, S)
    for r in range(S):
        true = np.linalg.norm(V32[:, r] - op.apply(tau, Z[:, r]))
        assert true <= 1e-6 * np.linalg.norm(V32[:, r]) * 1.01


@pytest.mark.parametrize("shape,S", [((40, 36), 8), ((24, 20), 16), ((12, 10, 9), 4), ((24, 20, 18), 8)])
def test_mg_complex64_lanes_iterates(shape, S):
    """Complex64 path with several lanes (grid legs and product working chunks
    of lanes per thread): fixed iteration counts against the oracle's FP64
    iterates, to complex64 accuracy; a lane or chunk mixed up would be off by
    O(1).  One iteration (the V-cycle's output scaled) agrees to ~1e-6 of the
    largest entry; after a few, COCG can amplify single-precision rounding
    for some vectors (3e-4 seen for one of these on the single-lane path
    too), hence the looser bound there."""
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce(f"mg c64 lanes {shape} S={S}")
    K = _field(shape, 5)
    op = OProblem.fv(K)
    gp = _gpu_problem(P, K)
    H = Hierarchy.of(op)
    tau = 2j * np.pi / 400.0
    rng = np.random.default_rng(17)
    V = (rng.normal(size=(op.n, S)) + 1j * rng.normal(size=(op.n, S))).astype(np.complex64).astype(np.complex128)
    def run(Vs, k):
        s_ = Vs.shape[1]
        z = torch.zeros(op.n * s_, dtype=torch.complex128, device="cuda")
        P.shk_inner_solve(gp, tau, to_dev(np.ascontiguousarray(Vs).ravel(), "c64"), z, fixed_iters=k, n_rhs=s_,
                          precond=P.SHK_PRECOND_MULTIGRID)
        return z.cpu().numpy().reshape(op.n, s_)

    for k, tol in ((1, 2e-5), (3, 1e-3)):
        Z = run(V, k)
        for r in range(S):
            xo, _, _, _ = mg_cocg(op, tau, V[:, r], 0.0, 100, H, fixed_iters=k)
            assert np.allclose(Z[:, r], xo, rtol=0, atol=tol * np.abs(xo).max()), (k, r)


def test_mg_rejected_for_csr():
    torch = require_gpu()
    import paper_1212_3660_amd as P
    K = _field((8, 8), 1)
    op = OProblem.fv(K)
    A = op.K.tocsr()
    gp = P.Problem.csr(A.indptr, A.indices, A.data, op.Mdiag)
    z = torch.zeros(op.n, dtype=torch.complex128, device="cuda")
    with pytest.raises(P.ShkError):
        P.shk_inner_solve(gp, 0.1j, to_dev(synth.unit_vector(op.n, 3)), z, precond=P.SHK_PRECOND_MULTIGRID)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_with_multigrid_inner(precision):
    """FGMRES-Sh with the multigrid inner solve on a ragged 2-D grid: every shift
    meets the tolerance and agrees with the exact family within the bound."""
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce(f"mg solve {precision}")
    K = _field((45, 38), 12)
    op = OProblem.fv(K)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(8, 10.0, 2000.0))
    b = synth.unit_vector(op.n, 800)
    prec = P.SHK_FP64 if precision == "fp64" else P.SHK_MIXED
    tol, eps = (1e-9, 1e-11) if precision == "fp64" else (1e-6, 1e-6)
    prm, keep = P.make_params(sig[[1, 4, 6]], tol=tol, eps_inner=eps, m_restart=40, precision=prec, max_refine=4,
                              inner_precond=P.SHK_PRECOND_MULTIGRID)
    x, st = P.fgmres_sh_solve(gp, prm, sig, b)
    assert np.all(st["true_relres"] <= tol)
    xe = exact_family(op, sig, b, "superlu")
    for j in range(len(sig)):
        assert np.linalg.norm(x[:, j, 0] - xe[:, j]) <= st[0, j]["true_relres"] / (abs(sig[j]) * 1e-5) * (1 + 1e-6)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_relaxed_inner_tolerance(precision):
    """Relaxed inner tolerance (eps_k = min(eps_max, max(eps, relax tol / q))):
    every shift still meets the tolerance, within the bound of the exact family,
    with fewer inner iterations than the fixed tolerance."""
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce(f"relaxed inner {precision}")
    K = _field((45, 38), 13)
    op = OProblem.fv(K)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(10, 5.0, 2000.0))
    b = synth.unit_vector(op.n, 900)
    prec = P.SHK_FP64 if precision == "fp64" else P.SHK_MIXED
    tol, eps = (1e-8, 1e-10) if precision == "fp64" else (1e-6, 1e-6)
    runs = {}
    for relax in (0.0, 0.1):
        prm, keep = P.make_params(sig[[2, 5, 8]], tol=tol, eps_inner=eps, m_restart=50, precision=prec, max_refine=4,
                                  inner_precond=P.SHK_PRECOND_MULTIGRID, inner_relax=relax, inner_eps_max=1e-2)
        x, st = P.fgmres_sh_solve(gp, prm, sig, b)
        assert np.all(st["true_relres"] <= tol)
        runs[relax] = (x, int(st["inner_its"].max()), st)
    x, its, st = runs[0.1]
    assert its < runs[0.0][1], (its, runs[0.0][1])
    xe = exact_family(op, sig, b, "superlu")
    for j in range(len(sig)):
        assert np.linalg.norm(x[:, j, 0] - xe[:, j]) <= tol / (abs(sig[j]) * 1e-5) * (1 + 1e-6)
    if precision == "fp64":
        # the oracle's relaxed run (same rule for eps_k, multigrid inner solve):
        # the same outer step counts within two
        from oracle import fgmres_sh
        ro = fgmres_sh(op, b, sig, sig[[2, 5, 8]], m_restart=50, tol=tol, inner="mg", eps=eps, relax=0.1,
                       eps_max=1e-2)
        for j in range(len(sig)):
            assert abs(int(st[0, j]["outer_its"]) - ro.info[j].outer_its) <= 2, (j, int(st[0, j]["outer_its"]),
                                                                               ro.info[j].outer_its)


def test_relaxed_tolerance_rejects_bad_parameters():
    torch = require_gpu()
    import paper_1212_3660_amd as P
    K = _field((10, 8), 2)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(3, 10.0, 100.0))
    b = synth.unit_vector(K.size, 20)
    for relax, emax in ((-1.0, 1e-2), (0.1, 2.0), (0.1, 1e-12)):
        prm, keep = P.make_params(sig, tol=1e-6, eps_inner=1e-8, inner_relax=relax, inner_eps_max=emax)
        with pytest.raises(P.ShkError):
            P.fgmres_sh_solve(gp, prm, sig, b)
