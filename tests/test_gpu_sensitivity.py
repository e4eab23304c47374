"""GPU parity of the sensitivity kernel (section 5, eq. sensitivity; Algorithm 6
step 3) against the oracle (oracle.sensitivity), and the workflow from the
solver's forward and adjoint solutions."""
import numpy as np
import pytest

import synth
from oracle import Problem as OProblem, dense_solve
from oracle.sensitivity import sensitivity_block
from tests.gpu_util import require_gpu, announce

pytestmark = pytest.mark.gpu


def _K(shape, seed):
    return synth.cell_conductivity(shape, -11.5, 1.0, 3, cfg=93, idx=seed)


def _flat(A):
    """(n, nf, cols) -> the solver's column-major layout c + n (j + nf col)."""
    return np.ascontiguousarray(np.transpose(A, (2, 1, 0))).ravel()


@pytest.mark.parametrize("shape,ns,nr", [((23, 17), 5, 3), ((7, 6, 5), 3, 2), ((1, 9), 1, 1)])
def test_matches_oracle(shape, ns, nr):
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce(f"sensitivity {shape} ns={ns} nr={nr}")
    K = _K(shape, len(shape))
    n, nf = K.size, 3
    gp = P.Problem.fv2d(K) if K.ndim == 2 else P.Problem.fv3d(K)
    rng = np.random.default_rng(7)
    Phi = rng.normal(size=(n, nf, ns)) + 1j * rng.normal(size=(n, nf, ns))
    Psi = rng.normal(size=(n, nf, nr)) + 1j * rng.normal(size=(n, nf, nr))
    ref = sensitivity_block(K, Phi, Psi)                       # (nf, ns, nr, n)
    phi = torch.from_numpy(_flat(Phi)).cuda()
    psi = torch.from_numpy(_flat(Psi)).cuda()
    for dt, tol in ((torch.complex128, 1e-12), (torch.complex64, 2e-6)):
        J = torch.zeros(nf * ns * nr * n, dtype=dt, device="cuda")
        P.shk_sensitivity(gp, phi, psi, J, nf, ns, nr)
        got = J.cpu().numpy().astype(np.complex128).reshape(nf, ns, nr, n)
        assert np.allclose(got, ref, rtol=tol, atol=tol * np.abs(ref).max()), dt


def test_from_solver_outputs():
    """Forward and adjoint solves by fgmres_sh_solve, then the kernel: agrees
    with the oracle's sensitivity of the exact solutions within the solves'
    accuracy."""
    torch = require_gpu()
    import paper_1212_3660_amd as P
    announce("sensitivity from solves")
    K = _K((20, 16), 4)
    op = OProblem.fv(K)
    n = op.n
    sig = synth.shifts_from_periods(synth.periods(3, 20.0, 500.0))
    src, rec = [37, 250], [101, 170, 300]
    B = np.zeros((n, 2), dtype=np.complex128)
    B[src, [0, 1]] = 1.0
    E = np.zeros((n, 3), dtype=np.complex128)
    E[rec, [0, 1, 2]] = 1.0
    gp = P.Problem.fv2d(K)
    prm, keep = P.make_params(sig, tol=1e-11, eps_inner=1e-12, m_restart=60, precision=P.SHK_FP64, max_refine=4)

    def solve(Bm):
        # device path: x is (cols, nf, n), i.e. already the layout c + n (j + nf col)
        x, st = P.fgmres_sh_solve(gp, prm, sig, torch.from_numpy(np.ascontiguousarray(Bm.T)).cuda())
        assert np.all(st["true_relres"] <= 1e-11)
        return x.contiguous()

    phi, psi = solve(B), solve(E)
    J = torch.zeros(len(sig) * 2 * 3 * n, dtype=torch.complex128, device="cuda")
    P.shk_sensitivity(gp, phi, psi, J, len(sig), 2, 3)
    got = J.cpu().numpy().reshape(len(sig), 2, 3, n)
    Pe = np.stack([np.stack([dense_solve(op.shifted(s), B[:, k]) for s in sig], 1) for k in range(2)], 2)
    Qe = np.stack([np.stack([dense_solve(op.shifted(s), E[:, k]) for s in sig], 1) for k in range(3)], 2)
    ref = sensitivity_block(K, Pe, Qe)
    assert np.allclose(got, ref, rtol=1e-7, atol=1e-7 * np.abs(ref).max())


def test_rejects_csr_problem():
    torch = require_gpu()
    import paper_1212_3660_amd as P
    op = OProblem.fv(_K((6, 5), 1))
    A = op.K.tocsr()
    gp = P.Problem.csr(A.indptr, A.indices, A.data, op.Mdiag)
    z = torch.zeros(op.n, dtype=torch.complex128, device="cuda")
    with pytest.raises(P.ShkError):
        P.shk_sensitivity(gp, z, z, z, 1, 1, 1)
