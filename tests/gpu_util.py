"""Helpers shared by the GPU tests: device checks and host<->device transfer of
interleaved vectors.  No solver arithmetic lives here."""
import numpy as np
import pytest


def require_gpu():
    import torch
    import paper_1212_3660_amd as P
    P.lib()   # raises if the HIP library is not built
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def to_dev(a, dtype="c128"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    t = t.to(torch.complex128 if dtype == "c128" else torch.complex64)
    return t.cuda()


def interleave(cols):
    """(n, S) -> flat interleaved c*S + r."""
    return np.ascontiguousarray(np.asarray(cols)).ravel()


def deinterleave(flat, S):
    return np.asarray(flat).reshape(-1, S)


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
