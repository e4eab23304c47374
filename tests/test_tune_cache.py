"""The packaged tuning cache (written by the autotuner on MI355X): every entry
names a valid class and only knobs that apply to it, with values the library
accepts (shk_tune_set checks names and ranges on the host; no GPU needed)."""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_packaged_cache_is_valid():
    import paper_1212_3660_amd as P
    from paper_1212_3660_amd import autotune as T
    if not os.path.exists(T.CACHE):
        pytest.skip("no packaged tuning cache")
    doc = json.load(open(T.CACHE))
    assert doc["version"] == 1 and doc["entries"]
    keys = set()
    for e in doc["entries"]:
        key = T._key_of(e["class"])
        assert key not in keys
        keys.add(key)
        assert key[0] in T.KINDS and key[1] > 0 and key[2] in (1, 2, 4, 8, 16, 32, 64)
        assert set(e["knobs"]) <= set(T.knobs_for(key))
        assert e["ms"] <= e["ms_start"] and e["workload"]
    P.shk_tune_reset()
    try:
        T.load()
        for e in doc["entries"]:
            for k, v in e["knobs"].items():
                assert P.shk_tune_get(T._key_of(e["class"]), k) == pytest.approx(float(v))
    finally:
        P.shk_tune_reset()
        T.load()


def test_tune_table_rejects_bad_settings():
    import paper_1212_3660_amd as P
    key = (0, 1000, 1, P.SHK_MIXED, P.SHK_PRECOND_MULTIGRID)
    for k, v in (("cg_block", 128), ("tail_lds", 200 * 1024), ("round_tol", 1.5), ("no_such_knob", 1),
                 ("tail_lanes", 3), ("tail_lanes", 128), ("rows", -1), ("rows64", -5), ("rows_yb", 3),
                 ("rows_yb", 0), ("tile3_lt", 16), ("post3_lt", 8), ("mg_chain", 2)):
        with pytest.raises(P.ShkError):
            P.shk_tune_set(key, k, v)
    from paper_1212_3660_amd import autotune as T
    P.shk_tune_reset()
    try:
        P.shk_tune_set(key, "post_lt", 4)
        assert P.shk_tune_get(key, "post_lt") == 4
        assert P.shk_tune_get(P.TUNE_ALL, "post_lt") == 2
        P.shk_tune_set(P.TUNE_ALL, "down_lt", 8)          # shared: classes without an entry
        assert P.shk_tune_get((1, 5, 1, 0, 0), "down_lt") == 8
        P.shk_tune_reset()
        assert P.shk_tune_get(key, "post_lt") == 2 and P.shk_tune_get(P.TUNE_ALL, "down_lt") == 4
        # the defaults of the lane-split tail and the row-marching legs
        assert P.shk_tune_get(P.TUNE_ALL, "tail_lanes") == 1
        assert P.shk_tune_get(P.TUNE_ALL, "rows") == 0 and P.shk_tune_get(P.TUNE_ALL, "rows64") == 16384
        assert P.shk_tune_get(P.TUNE_ALL, "rows_yb") == 4
        for k, v in (("tail_lanes", 0), ("tail_lanes", 64), ("rows", 65536), ("rows_yb", 16)):
            P.shk_tune_set(key, k, v)
            assert P.shk_tune_get(key, k) == v
    finally:
        P.shk_tune_reset()
        T.load()


def test_tuner_knobs_follow_the_class():
    """The autotuner searches a knob only where it changes something: the
    tail's lanes per workgroup with several lanes, the row-marching legs on
    2-D several-lane classes (rows for complex64, rows64 for complex128), the
    plane-marching ones in 3-D, the chained legs with one 2-D lane."""
    import paper_1212_3660_amd as P
    from paper_1212_3660_amd import autotune as T
    mg, jac = P.SHK_PRECOND_MULTIGRID, P.SHK_PRECOND_JACOBI
    k2m = T.knobs_for((0, 65536, 64, P.SHK_MIXED, mg))
    k2d = T.knobs_for((0, 65536, 64, P.SHK_FP64, mg))
    k1 = T.knobs_for((0, 262144, 1, P.SHK_MIXED, mg))
    k3 = T.knobs_for((1, 2097152, 8, P.SHK_MIXED, mg))
    kj = T.knobs_for((0, 262144, 4, P.SHK_MIXED, jac))
    assert {"tail_lanes", "rows", "rows_yb"} <= set(k2m) and "rows64" not in k2m
    assert {"tail_lanes", "rows64", "rows_yb", "lt64"} <= set(k2d) and "rows" not in k2d
    assert "tail_lanes" not in k1 and "rows" not in k1 and {"mg_chain", "mg_fuse"} <= set(k1)
    assert "rows" not in k3 and {"tile3", "tile3_zb", "tile3_lt", "tail_lanes"} <= set(k3)
    assert not {"tail_lds", "tail_lanes", "rows", "tile3"} & set(kj) and "round_tol" in kj
    for k in k2m + k2d + k1 + k3 + kj:
        assert k in T.SPACE
