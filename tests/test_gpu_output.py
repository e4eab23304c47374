"""Output modes of the solve (SHK_OUT_FULL / ROWS / FACTORED) and the solve
server's caller-supplied device arena, through the C ABI.

ROWS gathers the same device-formed solution FULL returns, so the two agree
bitwise.  FACTORED returns the basis vectors of every cycle and refinement
pass with their coefficients, so Z Y reproduces the FULL solution up to the
order of the sums (checked at 1e-12 relative, with restarts and a
refinement sweep in the run).  The server with an arena that the caller
allocates returns the same outputs as the standalone solves, and the rows
agree with SuperLU within the residual bound.
"""
import numpy as np
import pytest

import synth
from oracle import Problem as OProblem, superlu_solve
from tests.gpu_util import require_gpu, announce

pytestmark = pytest.mark.gpu


def _bound(sig, rho, nb, Ss=1e-5):
    return rho * nb / (np.abs(sig.imag) * Ss)


def _case(shape=(30, 26), nf=7, nr=3, cfg=98):
    K = synth.cell_conductivity(shape, -11.5, 1.0, 5, cfg=cfg)
    sig = synth.shifts_from_periods(synth.periods(nf, 10.0, 1000.0))
    cells = synth.distinct_interior_cells(shape, nr, cfg, synth.P_WELLS)
    B = np.zeros((K.size, nr), complex)
    for r, c in enumerate(cells):
        B[c, r] = 1.0
    return K, sig, B, cells


@pytest.mark.parametrize("rhs_mode", ["lockstep", "block"])
def test_rows_output_matches_full(rhs_mode):
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce(f"rows output {rhs_mode}")
    K, sig, B, cells = _case()
    gp = P.Problem.fv2d(K)
    rows = np.array(cells + [0, K.size - 1, 123, 123], dtype=np.int64)
    mode = P.SHK_RHS_BLOCK if rhs_mode == "block" else P.SHK_RHS_LOCKSTEP
    common = dict(m_restart=40, tol=1e-6, eps_inner=1e-6, precision=P.SHK_MIXED, max_refine=4, rhs_mode=mode,
                  inner_precond=P.SHK_PRECOND_MULTIGRID)
    pf, kf = P.make_params(sig[[1, 4]], **common)
    pr, kr = P.make_params(sig[[1, 4]], output=P.SHK_OUT_ROWS, out_rows=rows, **common)
    xf, sf = P.fgmres_sh_solve(gp, pf, sig, B)
    xr, sr = P.fgmres_sh_solve(gp, pr, sig, B)                     # host pointers
    assert xr.shape == (len(rows), len(sig), B.shape[1])
    assert np.array_equal(xr, xf[rows])
    assert np.array_equal(sf["true_relres"], sr["true_relres"])
    bd = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    xd, sd = P.fgmres_sh_solve(gp, pr, sig, bd)                    # device pointers
    assert np.array_equal(xd.cpu().numpy(), np.transpose(xr, (2, 1, 0)))
    elems, kcap = P.shk_output_elems(gp, pr, len(sig), B.shape[1])
    assert elems == len(rows) * len(sig) * B.shape[1] and kcap == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_factored_output_reconstructs_full(precision):
    """Restart length 6 forces several cycles and the mixed run a refinement
    sweep: Z Y over every returned column equals the FULL solution."""
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce(f"factored output {precision}")
    K, sig, B, cells = _case(nf=6, nr=2)
    gp = P.Problem.fv2d(K)
    prec = P.SHK_FP64 if precision == "fp64" else P.SHK_MIXED
    tol, eps = (1e-9, 1e-11) if precision == "fp64" else (1e-6, 3e-6)
    common = dict(m_restart=6, max_restarts=30, max_refine=3, tol=tol, eps_inner=eps, precision=prec,
                  refine_tol=1e-2, refine_eps_inner=1e-3)
    pf, kf = P.make_params(sig[[1, 4]], **common)
    pz, kz = P.make_params(sig[[1, 4]], output=P.SHK_OUT_FACTORED, **common)
    xf, sf = P.fgmres_sh_solve(gp, pf, sig, B)
    (Z, Y), sz = P.fgmres_sh_solve(gp, pz, sig, B)
    elems, kcap = P.shk_output_elems(gp, pz, len(sig), B.shape[1])
    assert kcap == 6 * 31 * 4 and Z.shape == (K.size, kcap, 2) and Y.shape == (kcap, len(sig), 2)
    used = int(sz["basis_cols"][0, 0])
    assert used > 6 and np.all(sz["basis_cols"] == used)
    assert np.all(Z[:, used:] == 0) and np.all(Y[used:] == 0)
    if precision == "mixed":
        assert np.all(sz["refine_sweeps"] >= 1)
    for r in range(2):
        X = Z[:, :, r] @ Y[:, :, r]
        assert np.allclose(X, xf[:, :, r], rtol=0, atol=1e-12 * np.abs(xf[:, :, r]).max())
    # device pointers: the same numbers
    bd = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    (Zd, Yd), _ = P.fgmres_sh_solve(gp, pz, sig, bd)
    assert np.array_equal(Zd.cpu().numpy(), np.transpose(Z, (2, 1, 0)))
    assert np.array_equal(Yd.cpu().numpy(), np.transpose(Y, (2, 1, 0)))


def test_output_mode_errors():
    require_gpu()
    import paper_1212_3660_amd as P
    announce("output mode errors")
    K, sig, B, cells = _case(nf=3, nr=1)
    gp = P.Problem.fv2d(K)
    for kw, code in ((dict(output=P.SHK_OUT_ROWS, out_rows=[0, K.size]), -1),
                     (dict(output=P.SHK_OUT_ROWS), -1),
                     (dict(output=P.SHK_OUT_FACTORED, rhs_mode=P.SHK_RHS_BLOCK), -5),
                     (dict(output=9), -1)):
        prm, keep = P.make_params(sig[[1]], **kw)
        with pytest.raises(P.ShkError) as e:
            P.fgmres_sh_solve(gp, prm, sig, B)
        assert e.value.code == code, kw


def test_server_caller_arena_rows_output():
    """A server whose device memory is a tensor the caller allocated: requests
    with ROWS output at their source cells return the rows of the standalone
    FULL solve (same library kernels on another stream), and the rows agree
    with SuperLU within the residual bound."""
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce("server caller arena rows")
    # the 256 x 256 request needs a multigrid workspace well beyond any slack
    # in the region estimate, so a mis-sized region would show as an error
    reqs = [synth.Request(i, 0.0, g, 2000 + i, nf, nr)
            for i, (g, nf, nr) in enumerate([(48, 7, 2), (64, 12, 3), (256, 5, 3), (40, 6, 1), (56, 9, 4)])]
    works = [synth.request_workload(r) for r in reqs]
    budget = 1 << 30
    arena = torch.empty(budget, dtype=torch.uint8, device="cuda")
    srv = P.Server(budget, max_slots=3, arena=arena)
    jobs = []
    for w in works:
        rows = np.array([int(np.argmax(np.abs(w.b[:, r]))) for r in range(w.b.shape[1])], dtype=np.int64)
        prm, keep = P.make_params(w.tau_seq, m_restart=40, tol=1e-6, eps_inner=1e-6, precision=P.SHK_MIXED,
                                  max_refine=4, inner_precond=P.SHK_PRECOND_MULTIGRID, output=P.SHK_OUT_ROWS,
                                  out_rows=rows)
        t = srv.submit(w.cell_K, w.sigma, w.b, prm, keep_solution=True)
        jobs.append((t, w, rows, keep))
    srv.drain()
    for t, w, rows, keep in jobs:
        res, xr, st = srv.poll(t, want_solution=True)
        assert res["error"] == 0 and res["done"] == 1
        assert np.all(st["true_relres"] <= 1e-6)
        assert xr.shape == (len(rows), len(w.sigma), w.b.shape[1])
        gp = P.Problem.fv2d(w.cell_K, w.Ss, w.h)
        pf, kf = P.make_params(w.tau_seq, m_restart=40, tol=1e-6, eps_inner=1e-6, precision=P.SHK_MIXED,
                               max_refine=4, inner_precond=P.SHK_PRECOND_MULTIGRID)
        xf, sf = P.fgmres_sh_solve(gp, pf, w.sigma, w.b)
        assert np.allclose(xr, xf[rows], rtol=1e-12, atol=1e-12 * np.abs(xf).max())
        op = OProblem.fv(w.cell_K, w.Ss, w.h)
        for j in (0, len(w.sigma) - 1):
            A = op.shifted(w.sigma[j])
            for r in range(w.b.shape[1]):
                xe = superlu_solve(A, w.b[:, r])
                assert np.max(np.abs(xr[:, j, r] - xe[rows])) <= _bound(w.sigma[j], st[r, j]["true_relres"], 1.0)
        gp.close()
    srv.close()
    del arena
