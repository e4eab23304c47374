"""Independent CPU oracle for the flexible shifted-system solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import anything in this package; the GPU library and
its Python binding never do, and this package never imports them.  It shares no
code with the GPU path: only the seeded input generators in ``synth`` serve
both.

Contents (complex128 throughout):
  fv         finite-volume operator K, M (section 5.1, eq. phasor1 / genshifted)
  exact      exact x_j = (K + sigma_j M)^{-1} b: banded elimination, SuperLU,
             dense, DST-I closed form, 1-D discrete Green's function
  cocg       Jacobi-COCG inner solve (section 4, eq. zmmoditer)
  mg         geometric aggregation multigrid V-cycle, multigrid-preconditioned
             COCG (the inner solve with a multigrid preconditioner, section 6)
  fgmres_sh  Algorithms 3 and 4 with inexact inner solves, restart, refinement
  block      block FGMRES-Sh: one shared block basis for several right-hand
             sides (the multiple right-hand-side extension of sections 5 and 7)
  sensitivity  adjoint-state sensitivity of point measurements to ln K per
             cell (section 5, eq. sensitivity, Algorithm 6)
"""
from .fv import Problem, assemble_stiffness, face_transmissivities, mass_diagonal  # noqa: F401
from .exact import (banded_solve, dense_solve, superlu_solve, dst_closed_form,  # noqa: F401
                    dst_mode, green_1d, laplacian_eigenvalues, exact_family)
from .cocg import cocg  # noqa: F401
from .mg import Hierarchy, vcycle, pcocg, mg_cocg  # noqa: F401
from .fgmres_sh import (fgmres_sh, refine, true_residuals, mgs_step,  # noqa: F401
                        shifted_hessenberg, small_solve, CONVERGED, NOT_CONVERGED,
                        INNER_LIMITED, BREAKDOWN_EXACT, NAN_STATUS)
from .sensitivity import sensitivity, sensitivity_block  # noqa: F401
