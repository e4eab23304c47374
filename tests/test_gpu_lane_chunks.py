"""Lane-chunk settings of the multigrid kernels.

With several right-hand sides a thread of the grid legs and of the product
w = A u works a chunk of lanes; the chunk sizes are launch parameters read
from SHK_MG_POST_LT, SHK_MG_DOWN_LT, SHK_MG_UP_LT (complex64) and SHK_MG_LT64
(complex128) when the library loads, and every choice runs the same per-lane
arithmetic.  The defaults are covered by the rest of the suite; here each
non-default setting reruns, in a child process with that environment, the
multi-lane multigrid tests: fixed inner iterations against the oracle's
iterates (complex64: 8, 16 and 4 lanes; complex128: 4 and 2 lanes), and the
256x256 / 64-rhs solves with the multigrid inner solve (the kernels these
settings select) on both paths against SuperLU and reciprocity.
"""
import os
import subprocess
import sys

import pytest

from tests.gpu_util import require_gpu, announce

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("post,down,up,lt64", [(0, 8, 8, 0), (4, 2, 2, 4), (8, 8, 4, 0)])
def test_lane_chunk_settings(post, down, up, lt64):
    require_gpu()
    announce(f"lane chunks post={post} down={down} up={up} lt64={lt64}")
    env = dict(os.environ, SHK_MG_POST_LT=str(post), SHK_MG_DOWN_LT=str(down), SHK_MG_UP_LT=str(up),
               SHK_MG_LT64=str(lt64))
    cmd = [sys.executable, "-u", "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "--timeout", "240",
           "--timeout-method", "thread",
           "tests/test_gpu_mg.py::test_mg_complex64_lanes_iterates",
           "tests/test_gpu_mg.py::test_mg_cocg_iterates_match_oracle",
           "tests/test_gpu_workloads.py::test_256x256_64_rhs_forward_adjoint[fp64-multigrid]",
           "tests/test_gpu_workloads.py::test_256x256_64_rhs_forward_adjoint[mixed-multigrid]"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-2000:]
    assert "8 passed" in r.stdout, r.stdout[-2000:]
