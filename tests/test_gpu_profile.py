"""The library's phase timer: HIP events at the phase boundaries of a solve
account for the solve's device time, phase by phase."""
import numpy as np
import pytest

import synth
from tests.gpu_util import require_gpu, announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rhs_mode", ["lockstep", "block"])
def test_phase_timer_accounts_for_the_solve(rhs_mode):
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce(f"phase timer {rhs_mode}")
    K = synth.cell_conductivity((64, 60), -11.5, 1.0, 5, cfg=77)
    sig = synth.shifts_from_periods(synth.periods(12, 10.0, 1000.0))
    cells = synth.distinct_interior_cells((64, 60), 3, 77, synth.P_WELLS)
    B = np.zeros((K.size, 3), complex)
    for r, c in enumerate(cells):
        B[c, r] = 1.0
    gp = P.Problem.fv2d(K)
    mode = P.SHK_RHS_BLOCK if rhs_mode == "block" else P.SHK_RHS_LOCKSTEP
    prm, keep = P.make_params(sig[[1, 6]], m_restart=40, max_refine=4, tol=1e-6, eps_inner=1e-6,
                              precision=P.SHK_MIXED, inner_precond=P.SHK_PRECOND_MULTIGRID, rhs_mode=mode)
    b = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    with torch.cuda.stream(torch.cuda.Stream()):
        P.fgmres_sh_solve(gp, prm, sig, b)
        torch.cuda.synchronize()
        P.shk_profile_enable(False, phases=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        x, st = P.fgmres_sh_solve(gp, prm, sig, b)
        e1.record()
        e1.synchronize()
        ph = P.shk_profile_read_phases()
        P.shk_profile_enable(False)
    assert np.all(st["status"] == P.SHK_CONVERGED)
    total = e0.elapsed_time(e1)
    s = sum(ph.values())
    assert set(ph) == set(P.PHASES) and all(v >= 0 for v in ph.values())
    assert 0.5 * total <= s <= 1.02 * total, (s, total, ph)
    assert ph["true residuals"] > 0
    if rhs_mode == "block":
        assert ph["block passes"] > 0 and ph["inner solves"] == 0
    else:
        for k in ("inner solves", "Gram-Schmidt", "least squares and step test", "assembly and restarts"):
            assert ph[k] > 0, k
        assert ph["block passes"] == 0
        assert ph["inner solves"] > ph["Gram-Schmidt"]
    # disabled: nothing accumulates
    P.shk_profile_enable(False)
    P.fgmres_sh_solve(gp, prm, sig, B)
    assert sum(P.shk_profile_read_phases().values()) == 0
    gp.close()
