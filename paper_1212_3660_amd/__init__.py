"""MI355X flexible Krylov solver for shifted systems (K + sigma_j M) x_j = b.

The compute path is the HIP library ``libshk.so`` (sources in ``csrc/``, C ABI
in ``include/shk.h``); ``binding`` marshals arguments to it.  Build with
``python -m paper_1212_3660_amd.build``.
"""
from .binding import (Problem, Server, fgmres_sh_solve, make_params, shk_apply_shifted,  # noqa: F401
                      shk_assemble, shk_block_orthogonalize, shk_block_shifted_lsq, shk_inner_solve, shk_orthogonalize, shk_shifted_lsq,
                      shk_true_residual, shk_true_residual_noalloc, shk_sensitivity, shk_workspace_bytes, shk_profile_enable, shk_profile_read, shk_profile_read_block, lib, STATUS_DTYPE, SHK_FP64, SHK_MIXED,
                      SHK_GMRES, SHK_FOM, SHK_CGS2, SHK_MGS, SHK_CONVERGED, SHK_NOT_CONVERGED, SHK_INNER_LIMITED,
                      SHK_BREAKDOWN_EXACT, SHK_NAN, SHK_PRECOND_JACOBI, SHK_PRECOND_MULTIGRID, SHK_RHS_LOCKSTEP, SHK_RHS_BLOCK,
                      SHK_OUT_FULL, SHK_OUT_ROWS, SHK_OUT_FACTORED, shk_output_elems, TUNE_ALL, shk_tune_set,
                      shk_tune_get, shk_tune_reset, shk_tune_class, shk_profile_read_phases, PHASES,
                      ShkError)
from . import autotune  # noqa: F401,E402
