"""Autotuner of the solver's launch settings, per workload class.

A workload class is the key of the library's tuning table (shk_tune_class):
operator kind, unknowns, lane count, precision and inner preconditioner.  For
one representative solve of a class the tuner runs a coordinate search over
the knobs that apply to it (lanes per thread of the multigrid legs, the LDS
budget of the V-cycle's coarse tail and its lanes per workgroup, the fused
first restriction, the iteration block size, the complex64 round tolerance, graph-captured
iterations) and, when asked, over the restart length: each candidate is timed
as whole solves on the device (median of several, after an untimed one), and
a candidate counts only when every (shift, rhs) pair converges to the
requested tolerance by its true residual.  A change is kept when it is faster
than the best so far by more than the noise margin.

The picks go to a JSON cache (``tune_cache.json`` beside this file by
default) that ``load`` applies through shk_tune_set; ``lib()`` loads the
packaged cache when the library is first loaded.  Settings only change launch
shapes and the inner solve's rounds, never what the method computes, and the
GPU tests rerun the parity cases under every cached pick.
"""
import json
import os
import time

import numpy as np

from . import binding as B

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
KINDS = {0: "2-D finite volume", 1: "3-D finite volume", 2: "CSR"}

# knob -> candidate values, searched in this order
SPACE = {
    "tail_lds": [16384, 32768, 64512, 98304, 162816],
    "tail_lanes": [0, 1, 2, 4, 8],
    "mg_fuse": [0, 1],
    "post_lt": [0, 2, 4, 8],
    "down_lt": [2, 4, 8],
    "up_lt": [2, 4, 8],
    "lt64": [0, 2, 4],
    "cg_block": [256, 512],
    "round_tol_mg": [1e-3, 3e-3, 1e-2],
    "round_tol": [3e-3, 1e-2, 3e-2],
    "nt_store32": [0, 1],
    "nt_store64": [0, 1],
    "graph": [0, 1],
    "rows": [0, 65536, 16384],
    "rows64": [0, 65536, 16384],
    "rows_yb": [2, 4, 8],
    "tile3": [0, 32768, 262144],
    "tile3_zb": [4, 8, 16],
    "tile3_lt": [4, 8],
    "mg_chain": [0, 1],
    "tile3_post": [0, 1],
    "asm_mfma": [0, 1],
}


def knobs_for(key, n_lanes_real=None):
    """The knobs that change anything for a class (kind, n, lanes, precision,
    precond)."""
    kind, n, lanes, prec, pc = key
    mixed = prec == B.SHK_MIXED
    ks = ["cg_block", "graph", "asm_mfma"]
    if pc == B.SHK_PRECOND_MULTIGRID and kind in (0, 1):
        ks += ["tail_lds"] + (["tail_lanes"] if lanes > 1 else [])
        if kind == 1:
            ks += ["tile3", "tile3_zb"] + (["tile3_lt"] if mixed else []) + (["tile3_post"] if lanes > 1 else [])
        if lanes == 1:
            ks += ["mg_fuse"] + (["mg_chain"] if kind == 0 else [])
        elif mixed:
            ks += ["post_lt", "down_lt", "up_lt"] + (["rows", "rows_yb"] if kind == 0 else [])
        else:
            ks += ["lt64"] + (["rows64", "rows_yb"] if kind == 0 else [])
        if mixed:
            ks += ["round_tol_mg"]
    else:
        ks += ["nt_store32" if mixed else "nt_store64"]
        if mixed:
            ks += ["round_tol"]
    return [k for k in SPACE if k in ks]


def _class_dict(key):
    kind, n, lanes, prec, pc = key
    return {"kind": kind, "n": n, "lanes": lanes, "precision": prec, "precond": pc}


def _key_of(d):
    return (int(d["kind"]), int(d["n"]), int(d["lanes"]), int(d["precision"]), int(d["precond"]))


class _Runner:
    """Times whole solves of one workload on the current stream."""

    def __init__(self, problem, sigma, b_dev, params_kw, reps):
        import torch
        self.torch = torch
        self.problem, self.sigma, self.b = problem, np.asarray(sigma), b_dev
        self.kw = {k: v for k, v in params_kw.items() if k != "taus"}
        self.taus = params_kw["taus"]
        self.reps = reps
        self.tol = self.kw.get("tol", 1e-8)

    def params(self, m=None):
        kw = dict(self.kw)
        if m is not None:
            kw["m_restart"] = m
        return B.make_params(self.taus, **kw)

    def time(self, m=None):
        torch = self.torch
        prm, keep = self.params(m)
        nr = self.b.shape[0]
        ws = torch.empty(B.shk_workspace_bytes(self.problem, prm, len(self.sigma), nr), dtype=torch.uint8,
                         device=self.b.device)
        x = torch.empty(B.shk_output_elems(self.problem, prm, len(self.sigma), nr)[0], dtype=torch.complex128,
                        device=self.b.device)
        ok = True
        per = []
        for i in range(self.reps + 1):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            _, st = B.fgmres_sh_solve(self.problem, prm, self.sigma, self.b, x=x, workspace=ws)
            e1.record()
            e1.synchronize()
            ok &= bool((st["status"] == B.SHK_CONVERGED).all()) and float(st["true_relres"].max()) <= self.tol
            if i > 0:
                per.append(e0.elapsed_time(e1))
        return float(np.median(per)), ok


def tune(problem, sigma, b_dev, params_kw, reps=3, restarts=None, margin=0.01, passes=1, log=None,
         workload=""):
    """Coordinate search for one workload; returns the cache entry.

    problem: a Problem; sigma: the shifts; b_dev: torch CUDA complex128 tensor
    (n_rhs, n); params_kw: keyword arguments of make_params including
    ``taus`` (the preconditioner shifts).  restarts: restart lengths to try
    after the knobs (None: keep params_kw's).  The class's table entry is left
    at the picks; the settings in force before are restored for the knobs
    that are not picked."""
    run = _Runner(problem, sigma, b_dev, params_kw, reps)
    prm, _ = run.params()
    key = B.shk_tune_class(problem, prm, b_dev.shape[0])
    knobs = knobs_for(key)
    cur = {k: B.shk_tune_get(key, k) for k in knobs}
    t0 = time.perf_counter()
    base_ms, ok = run.time()
    if not ok:
        raise RuntimeError("the workload does not converge at the current settings")
    best = base_ms
    trials = [{"knobs": dict(cur), "ms": base_ms, "ok": ok}]
    for _ in range(passes):
        changed = False
        for k in knobs:
            for v in SPACE[k]:
                if float(v) == float(cur[k]):
                    continue
                B.shk_tune_set(key, k, v)
                ms, ok = run.time()
                trials.append({"knob": k, "value": v, "ms": ms, "ok": ok})
                if log:
                    log(f"[tune] {k}={v}: {ms:.3f} ms{'' if ok else ' (not converged)'}")
                if ok and ms < best * (1.0 - margin):
                    best, cur[k], changed = ms, v, True
            B.shk_tune_set(key, k, cur[k])
        if not changed:
            break
    m_pick = params_kw.get("m_restart")
    if restarts:
        for m in restarts:
            if m == m_pick:
                continue
            ms, ok = run.time(m)
            trials.append({"m_restart": m, "ms": ms, "ok": ok})
            if log:
                log(f"[tune] m_restart={m}: {ms:.3f} ms{'' if ok else ' (not converged)'}")
            if ok and ms < best * (1.0 - margin):
                best, m_pick = ms, m
    return {"class": _class_dict(key), "workload": workload, "knobs": {k: cur[k] for k in knobs},
            "m_restart": m_pick, "ms": round(best, 4), "ms_start": round(base_ms, 4),
            "search_s": round(time.perf_counter() - t0, 1), "trials": len(trials)}


def save(entries, path=CACHE, device=None):
    """Writes entries (replacing those of the same class in an existing
    cache)."""
    old = []
    if os.path.exists(path):
        old = json.load(open(path)).get("entries", [])
    keys = {_key_of(e["class"]) for e in entries}
    merged = [e for e in old if _key_of(e["class"]) not in keys] + list(entries)
    doc = {"version": 1, "device": device, "entries": merged}
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")


def load(path=CACHE, apply=True):
    """Reads a cache; with apply sets every entry's knobs in the library's
    table.  Returns the entries (empty when the file does not exist)."""
    if not os.path.exists(path):
        return []
    doc = json.load(open(path))
    if doc.get("version") != 1:
        raise ValueError(f"{path}: unknown tuning cache version {doc.get('version')}")
    entries = doc.get("entries", [])
    if apply:
        for e in entries:
            key = _key_of(e["class"])
            for k, v in e["knobs"].items():
                B.shk_tune_set(key, k, v)
    return entries


def restart_for(key, default, entries=None):
    """The cached restart length of a class, else default."""
    for e in (load(apply=False) if entries is None else entries):
        if _key_of(e["class"]) == tuple(key) and e.get("m_restart"):
            return int(e["m_restart"])
    return default


def tune_string(entry):
    """knob=value,... of an entry (the form tests pass to --shk-tune)."""
    return ",".join(f"{k}={v}" for k, v in entry["knobs"].items())
