"""The autotuner end to end on a small workload: the coordinate search keeps
only converged settings, its picks land in the class's table entry, the cache
round-trips through a file, and a solve under the picks agrees with the solve
under the default settings within the residual bound."""
import numpy as np
import pytest

import synth
from tests.gpu_util import require_gpu, announce

pytestmark = pytest.mark.gpu


def test_autotune_small_workload(tmp_path):
    torch = require_gpu()
    import paper_1212_3660_amd as P
    from paper_1212_3660_amd import autotune as T
    announce("autotune 48x40, 2 rhs, mixed multigrid")
    K = synth.cell_conductivity((48, 40), -11.5, 1.0, 5, cfg=41)
    sig = synth.shifts_from_periods(synth.periods(8, 10.0, 1000.0))
    cells = synth.distinct_interior_cells((48, 40), 2, 41, synth.P_WELLS)
    B = np.zeros((K.size, 2), complex)
    for r, c in enumerate(cells):
        B[c, r] = 1.0
    gp = P.Problem.fv2d(K)
    kw = dict(taus=sig[[1, 5]], m_restart=40, max_refine=4, tol=1e-6, eps_inner=1e-6, precision=P.SHK_MIXED,
              inner_precond=P.SHK_PRECOND_MULTIGRID)
    b = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    P.shk_tune_reset()
    try:
        with torch.cuda.stream(torch.cuda.Stream()):
            e = T.tune(gp, sig, b, kw, reps=1, workload="48x40 test")
            key = T._key_of(e["class"])
            assert key == (0, K.size, 2, P.SHK_MIXED, P.SHK_PRECOND_MULTIGRID)
            assert set(e["knobs"]) == set(T.knobs_for(key)) and e["trials"] > 10
            assert e["ms"] <= e["ms_start"]
            for k, v in e["knobs"].items():
                assert P.shk_tune_get(key, k) == float(v)
            path = str(tmp_path / "cache.json")
            T.save([e], path, device="test")
            prm, keep = P.make_params(kw["taus"], **{k: v for k, v in kw.items() if k != "taus"})
            xt, st_t = P.fgmres_sh_solve(gp, prm, sig, B)
            P.shk_tune_reset()
            assert P.shk_tune_get(key, "tail_lds") == 63 * 1024
            xd, st_d = P.fgmres_sh_solve(gp, prm, sig, B)
            got = T.load(path)
            assert len(got) == 1 and all(P.shk_tune_get(key, k) == float(v) for k, v in e["knobs"].items())
            assert T.restart_for(key, 7, got) == 40
            xt2, _ = P.fgmres_sh_solve(gp, prm, sig, B)
            assert np.array_equal(xt, xt2)
        for st in (st_t, st_d):
            assert np.all(st["status"] == P.SHK_CONVERGED) and np.all(st["true_relres"] <= 1e-6)
        # two converged solutions of the same systems: each within its residual
        # bound of the exact one (the smallest shift sets the scale)
        scale = np.abs(xd).max()
        assert np.max(np.abs(xt - xd)) <= 1e-3 * scale
    finally:
        P.shk_tune_reset()
        T.load()
        gp.close()
