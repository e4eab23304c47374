"""Tuning-table settings of the multigrid inner solve.

The launch settings of a workload class (lanes per thread of the grid legs
and of the product w = A u, the LDS budget of the V-cycle's one-workgroup
tail, the fused first restriction, the iteration block size, graph-captured
iterations) change launch shapes only: every choice runs the same per-lane
arithmetic.  The defaults are covered by the rest of the suite; here each
non-default setting reruns, in a child process whose shared settings are set
through shk_tune_set, the multi-lane multigrid tests: fixed inner iterations
against the oracle's iterates (complex64: 8, 16 and 4 lanes; complex128: 1, 4
and 2 lanes), the tail started two levels down, and the 256x256 / 64-rhs and
3-D 8-rhs solves with the multigrid inner solve on both paths against SuperLU
(and reciprocity).  Every pick in the packaged tuning cache runs the same
way, applied to all classes.
"""
import json
import os
import subprocess
import sys

import pytest

from tests.gpu_util import require_gpu, announce

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SETTINGS = [
    "post_lt=0,down_lt=8,up_lt=8,lt64=0",
    "post_lt=4,down_lt=2,up_lt=2,lt64=4",
    "post_lt=8,down_lt=8,up_lt=4,lt64=0",
    "graph=1",
    "tail_lds=162816",
    "tail_lds=16384,mg_fuse=0,cg_block=512",
    "tile3=1,tail_lds=16384",
    "tile3=1,tile3_zb=2,tile3_lt=8,tile3_post=1,post3_lt=4,tail_lds=4096",
    "tile3=1,tile3_post=1",
    "mg_chain=1",
    "mg_chain=1,tail_lds=4096",
    "asm_mfma=0",
    "tail_lanes=0",
    "tail_lanes=2,tail_lds=162816",
    "tail_lanes=4,tail_lds=16384",
    "rows=1,rows64=1,rows_yb=2,down_lt=2,up_lt=2",
    "rows=1,rows64=0,rows_yb=8,down_lt=8,up_lt=8",
]

def _cached_picks():
    """knob=value strings of the packaged tuning cache's entries."""
    path = os.path.join(ROOT, "paper_1212_3660_amd", "tune_cache.json")
    if not os.path.exists(path):
        return []
    out = []
    for e in json.load(open(path))["entries"]:
        t = ",".join(f"{k}={v}" for k, v in sorted(e["knobs"].items()))
        if t and t not in out:
            out.append(t)
    return out


SETTINGS += [t for t in _cached_picks() if t not in SETTINGS]
TESTS = ["tests/test_gpu_mg.py::test_mg_complex64_lanes_iterates",
         "tests/test_gpu_mg.py::test_mg_cocg_iterates_match_oracle",
         "tests/test_gpu_mg.py::test_mg_tail_two_levels_down",
         "tests/test_gpu_workloads.py::test_256x256_64_rhs_forward_adjoint[fp64-multigrid]",
         "tests/test_gpu_workloads.py::test_256x256_64_rhs_forward_adjoint[mixed-multigrid]",
         "tests/test_gpu_workloads.py::test_3d_multigrid_8_rhs_against_superlu"]


@pytest.mark.parametrize("tune", SETTINGS)
def test_tuning_settings(tune):
    require_gpu()
    announce(f"tuning settings {tune}")
    cmd = [sys.executable, "-u", "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "--timeout", "240",
           "--timeout-method", "thread", "--shk-tune", tune] + TESTS
    r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-2000:]
    assert "14 passed" in r.stdout, r.stdout[-2000:]
