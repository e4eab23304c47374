"""GPU parity of the FOM variant of Algorithm 4 (flexible FOM for shifted
systems, with the FOM restart) against the oracle.

Step level: the device's per-shift square solves H_k(sigma;T) y = beta e_1 and
their residual norms |hbar_{k+1,k}(sigma)| |y_k| against a library solve of the
same square system, the bound of Prop. 3 between the FOM and GMRES residuals
evaluated on the device's own y's, and an exactly singular square system.
Whole solves: every shift converged to the requested true residual, the error
against the direct solution of each shifted system, and outer step counts
within two of the oracle's FOM run (same tau schedule, inner tolerance and
restart length).
"""
import numpy as np
import pytest

import synth
from oracle import Problem as OProblem, exact_family, fgmres_sh, shifted_hessenberg, small_solve
from tests.gpu_util import require_gpu, announce

pytestmark = pytest.mark.gpu


def _field(shape, seed):
    return synth.cell_conductivity(shape, -11.5, 1.0, 5, cfg=70, idx=seed)


def _arnoldi(shape, seed, k):
    K = _field(shape, seed)
    op = OProblem.fv(K)
    sig = synth.shifts_from_periods(synth.periods(12, 5, 5000))
    b = synth.unit_vector(op.n, op.n // 2 + 3)
    r = fgmres_sh(op, b, sig, sig[[2, 6, 10]], m_restart=k, max_restarts=0, tol=1e-30, inner="dense",
                  keep_basis=True)
    return r.H, r.taus, sig, float(np.linalg.norm(b))


@pytest.mark.parametrize("m", [14, 64, 70])
def test_fom_projected_solves_match_oracle(m):
    require_gpu()
    import paper_1212_3660_amd as P
    announce(f"shifted fom m={m}")
    H, taus, sig, beta = _arnoldi((20, 20), 9, m)
    k = H.shape[1]
    y, rho = P.shk_shifted_lsq(H, taus, sig, beta, P.SHK_FOM)
    for j, s in enumerate(sig):
        for kk in range(1, k + 1):
            Hs = shifted_hessenberg(H[:kk + 1, :kk], taus[:kk], s)
            yo, qv = small_solve(Hs, beta, "fom")
            assert np.isclose(rho[kk - 1, j], np.linalg.norm(qv), rtol=1e-8, atol=1e-13 * beta), (j, kk)
        Hs = shifted_hessenberg(H, taus, s)
        yo, _ = small_solve(Hs, beta, "fom")
        assert np.allclose(y[j], yo, rtol=1e-8, atol=1e-9 * np.abs(yo).max()), j


def test_prop3_bound_on_device_solutions():
    # Prop. 3: ||r_fom - r_gmres|| <= alpha (1 + alpha) / (1 + alpha^2) ||r_fom||,
    # alpha = ||eta H_k(sigma;T)^{-H} e_k||, eta = hbar_{k+1,k}(sigma).  With an
    # exact Arnoldi relation both residuals are V_{k+1} times the projected
    # residual beta e_1 - Hbar(sigma;T) y, so the bound holds for those; and the
    # least-squares residual is never the larger one.
    require_gpu()
    import paper_1212_3660_amd as P
    announce("prop3")
    H, taus, sig, beta = _arnoldi((16, 18), 4, 10)
    yf, rf = P.shk_shifted_lsq(H, taus, sig, beta, P.SHK_FOM)
    yg, rg = P.shk_shifted_lsq(H, taus, sig, beta, P.SHK_GMRES)
    k = H.shape[1]
    e1 = np.zeros(k + 1, complex)
    e1[0] = beta
    ek = np.zeros(k, complex)
    ek[-1] = 1.0
    for j, s in enumerate(sig):
        Hs = shifted_hessenberg(H, taus, s)
        qf = e1 - Hs @ yf[j]
        qg = e1 - Hs @ yg[j]
        eta = Hs[k, k - 1]
        alpha = np.linalg.norm(eta * np.linalg.solve(Hs[:k, :k].conj().T, ek))
        bound = alpha * (1 + alpha) / (1 + alpha ** 2) * np.linalg.norm(qf)
        assert np.linalg.norm(qf - qg) <= bound * (1 + 1e-8) + 1e-12 * beta, j
        assert np.all(rg[:, j] <= rf[:, j] * (1 + 1e-10) + 1e-14 * beta), j
        # the FOM residual has no component in the first k directions
        assert np.abs(qf[:k]).max() <= 1e-9 * beta
        assert np.isclose(np.abs(qf[k]), rf[k - 1, j], rtol=1e-8)


def test_fom_singular_square_system():
    # 1 + h_11 (sigma - tau_1) = 0 exactly (sigma - tau_1 = 2i, h_11 = i/2): the
    # one-column FOM system of that shift is singular, the step reports an
    # infinite residual, and later steps solve their (regular) systems
    require_gpu()
    import paper_1212_3660_amd as P
    announce("fom singular")
    rng = np.random.default_rng(5)
    k = 4
    H = np.zeros((k + 1, k), complex)
    for c in range(k):
        H[:c + 1, c] = rng.standard_normal(c + 1) + 1j * rng.standard_normal(c + 1)
        H[c + 1, c] = 0.5 + rng.random()
    H[0, 0] = 0.5j
    taus = np.array([1j, 2j, 0.5j, 3j])
    sig = np.array([3j, 5j, 0.7j])
    beta = 2.0
    y, rho = P.shk_shifted_lsq(H, taus, sig, beta, P.SHK_FOM)
    assert np.isinf(rho[0, 0]) and np.all(np.isfinite(rho[0, 1:]))
    assert np.all(np.isfinite(rho[1:])) and np.all(np.isfinite(y))
    for j, s in enumerate(sig):
        for kk in range(2, k + 1):
            Hs = shifted_hessenberg(H[:kk + 1, :kk], taus[:kk], s)
            yo, qv = small_solve(Hs, beta, "fom")
            assert np.isclose(rho[kk - 1, j], np.linalg.norm(qv), rtol=1e-9, atol=1e-13), (j, kk)
        yo, _ = small_solve(shifted_hessenberg(H, taus, s), beta, "fom")
        assert np.allclose(y[j], yo, rtol=1e-9, atol=1e-12), j
    with pytest.raises(P.ShkError):
        P.shk_shifted_lsq(H, taus, sig, beta, 7)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fom_solve_with_restarts_matches_oracle(precision):
    require_gpu()
    import paper_1212_3660_amd as P
    announce(f"fom solve m=6 {precision}")
    K = synth.cell_conductivity((32, 32), -11.5, 1.0, 5, cfg=71)
    op = OProblem.fv(K)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(6, 10, 1000))
    b = synth.unit_vector(op.n, 528)
    taus = 2j * np.pi / np.array([20.0, 700.0])
    prec = P.SHK_FP64 if precision == "fp64" else P.SHK_MIXED
    tol = 1e-9 if precision == "fp64" else 1e-6
    prm, keep = P.make_params(taus, tol=tol, eps_inner=1e-12 if precision == "fp64" else 1e-8, m_restart=6,
                              max_restarts=80, max_refine=2, variant=P.SHK_FOM, precision=prec)
    x, st = P.fgmres_sh_solve(gp, prm, sig, b)
    xe = exact_family(op, sig, b, "banded")
    assert st["restarts"].max() >= 1          # the FOM restart ran
    ro = None
    if precision == "fp64":
        ro = fgmres_sh(op, b, sig, taus, m_restart=6, max_restarts=80, tol=tol, inner="cocg", eps=1e-12,
                       variant="fom")
    for j in range(len(sig)):
        s = st[0, j]
        assert s["status"] == P.SHK_CONVERGED, (j, s)
        assert s["true_relres"] <= tol
        assert np.linalg.norm(x[:, j, 0] - xe[:, j]) <= 2e3 * tol * np.linalg.norm(xe[:, j]), j
        if ro is not None:
            assert ro.info[j].status == 0
            assert abs(int(s["outer_its"]) - ro.info[j].outer_its) <= 2, (j, int(s["outer_its"]),
                                                                         ro.info[j].outer_its)


def test_fom_and_gmres_agree_with_multigrid_inner():
    # both variants reach the same solutions (the direct ones) on a multigrid
    # inner solve, several right-hand sides in lockstep
    require_gpu()
    import paper_1212_3660_amd as P
    announce("fom mg 3 rhs")
    K = _field((45, 38), 13)
    op = OProblem.fv(K)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(10, 5.0, 2000.0))
    B = np.stack([synth.unit_vector(op.n, c) for c in (900, 17, 1501)], axis=1)
    taus = sig[[1, 5, 8]]
    out = {}
    for v in (P.SHK_FOM, P.SHK_GMRES):
        prm, keep = P.make_params(taus, tol=1e-8, eps_inner=1e-10, m_restart=40, max_restarts=10, max_refine=2,
                                  variant=v, inner_precond=P.SHK_PRECOND_MULTIGRID)
        out[v] = P.fgmres_sh_solve(gp, prm, sig, B)
    for r in range(B.shape[1]):
        xe = exact_family(op, sig, B[:, r], "banded")
        for v, (x, st) in out.items():
            for j in range(len(sig)):
                assert st[r, j]["status"] == P.SHK_CONVERGED and st[r, j]["true_relres"] <= 1e-8, (v, r, j)
                assert np.linalg.norm(x[:, j, r] - xe[:, j]) <= 2e3 * 1e-8 * np.linalg.norm(xe[:, j])
        # the oracle's FOM run with the multigrid inner solve: outer steps within two
        ro = fgmres_sh(op, B[:, r], sig, taus, m_restart=40, max_restarts=10, tol=1e-8, inner="mg", eps=1e-10,
                       variant="fom")
        st = out[P.SHK_FOM][1]
        for j in range(len(sig)):
            assert abs(int(st[r, j]["outer_its"]) - ro.info[j].outer_its) <= 2, (r, j)


def test_fom_restarts_with_several_rhs():
    # three right-hand sides in lockstep, restart length 6: each lane restarts
    # from its own v_{m+1} with its own residual coefficient
    require_gpu()
    import paper_1212_3660_amd as P
    announce("fom restarts 3 rhs")
    K = synth.cell_conductivity((30, 26), -11.5, 1.0, 5, cfg=74)
    op = OProblem.fv(K)
    gp = P.Problem.fv2d(K)
    sig = synth.shifts_from_periods(synth.periods(7, 10, 1000))
    B = np.stack([synth.unit_vector(op.n, c) for c in (100, 390, 611)], axis=1)
    taus = 2j * np.pi / np.array([20.0, 500.0])
    prm, keep = P.make_params(taus, tol=1e-9, eps_inner=1e-12, m_restart=6, max_restarts=80, max_refine=2,
                              variant=P.SHK_FOM)
    x, st = P.fgmres_sh_solve(gp, prm, sig, B)
    assert st["restarts"].max() >= 1
    for r in range(B.shape[1]):
        xe = exact_family(op, sig, B[:, r], "banded")
        for j in range(len(sig)):
            assert st[r, j]["status"] == P.SHK_CONVERGED and st[r, j]["true_relres"] <= 1e-9, (r, j)
            assert np.linalg.norm(x[:, j, r] - xe[:, j]) <= 2e3 * 1e-9 * np.linalg.norm(xe[:, j]), (r, j)
