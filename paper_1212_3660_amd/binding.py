"""ctypes binding of ``libshk.so`` (the C ABI in include/shk.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device buffers and streams come from PyTorch (complex128 / complex64 CUDA
tensors, ``torch.cuda.current_stream()``); host buffers are NumPy arrays.  If
the library has not been built this module raises on first use: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshk.so")

SHK_OK, SHK_ERR_NOT_READY = 0, -4
SHK_CONVERGED, SHK_NOT_CONVERGED, SHK_INNER_LIMITED, SHK_BREAKDOWN_EXACT, SHK_NAN = 0, 1, 2, 3, 4
SHK_GMRES, SHK_FOM = 0, 1
SHK_CGS2, SHK_MGS = 0, 1
SHK_FP64, SHK_MIXED = 0, 1
SHK_PTR_HOST, SHK_PTR_DEVICE = 0, 1
SHK_PRECOND_JACOBI, SHK_PRECOND_MULTIGRID = 0, 1
SHK_RHS_LOCKSTEP, SHK_RHS_BLOCK = 0, 1
SHK_OUT_FULL, SHK_OUT_ROWS, SHK_OUT_FACTORED = 0, 1, 2


class shk_c128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class shk_params(C.Structure):
    _fields_ = [("m_restart", C.c_int), ("max_restarts", C.c_int), ("max_refine", C.c_int),
                ("inner_maxit", C.c_int), ("tol", C.c_double), ("eps_inner", C.c_double),
                ("n_tau", C.c_int), ("tau_seq", C.POINTER(shk_c128)), ("variant", C.c_int),
                ("precision", C.c_int), ("refine_tol", C.c_double), ("refine_eps_inner", C.c_double),
                ("inner_precond", C.c_int), ("mg_sweeps", C.c_int), ("mg_omega", C.c_double),
                ("inner_relax", C.c_double), ("inner_eps_max", C.c_double), ("ortho", C.c_int),
                ("rhs_mode", C.c_int), ("output", C.c_int), ("n_out_rows", C.c_int),
                ("out_rows", C.POINTER(C.c_longlong))]


class shk_status(C.Structure):
    _fields_ = [("status", C.c_int), ("outer_its", C.c_int), ("restarts", C.c_int),
                ("refine_sweeps", C.c_int), ("basis_cols", C.c_int), ("reserved", C.c_int),
                ("inner_its", C.c_longlong), ("quasi_relres", C.c_double),
                ("bound_relres", C.c_double), ("true_relres", C.c_double)]


STATUS_DTYPE = np.dtype([("status", np.int32), ("outer_its", np.int32), ("restarts", np.int32),
                         ("refine_sweeps", np.int32), ("basis_cols", np.int32), ("reserved", np.int32),
                         ("inner_its", np.int64), ("quasi_relres", np.float64),
                         ("bound_relres", np.float64), ("true_relres", np.float64)])
assert STATUS_DTYPE.itemsize == C.sizeof(shk_status)


class shk_request(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("cell_K", C.POINTER(C.c_double)), ("Ss", C.c_double),
                ("h", C.c_double), ("n_shifts", C.c_int), ("sigma", C.POINTER(shk_c128)), ("n_rhs", C.c_int),
                ("b", C.POINTER(shk_c128)), ("params", shk_params), ("keep_solution", C.c_int)]


class shk_result(C.Structure):
    _fields_ = [("done", C.c_int), ("error", C.c_int), ("t_arrival", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double), ("n_converged", C.c_int), ("max_true_relres", C.c_double)]


# exported symbols and their signatures
_SIGS = {
    "shk_params_default": (None, [C.POINTER(shk_params)]),
    "shk_problem_create_fv2d": (C.c_int, [C.c_int, C.c_int, C.c_void_p, C.c_double, C.c_double, C.POINTER(C.c_void_p)]),
    "shk_problem_create_fv3d": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_double, C.c_double,
                                          C.POINTER(C.c_void_p)]),
    "shk_problem_create_csr": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.POINTER(C.c_void_p)]),
    "shk_problem_destroy": (None, [C.c_void_p]),
    "shk_problem_size": (C.c_longlong, [C.c_void_p]),
    "shk_output_elems": (C.c_int, [C.c_void_p, C.POINTER(shk_params), C.c_int, C.c_int, C.POINTER(C.c_size_t),
                                   C.POINTER(C.c_int)]),
    "shk_workspace_bytes": (C.c_int, [C.c_void_p, C.POINTER(shk_params), C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
    "fgmres_sh_solve": (C.c_int, [C.c_void_p, C.POINTER(shk_params), C.c_int, C.c_void_p, C.c_int, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_int]),
    "shk_apply_shifted": (C.c_int, [C.c_void_p, shk_c128, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "shk_inner_solve": (C.c_int, [C.c_void_p, shk_c128, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                  C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "shk_orthogonalize": (C.c_int, [C.c_longlong, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                    C.c_int, C.c_void_p]),
    "shk_shifted_lsq": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_void_p,
                                  C.c_void_p, C.c_int]),
    "shk_block_orthogonalize": (C.c_int, [C.c_longlong, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_int, C.c_void_p]),
    "shk_block_shifted_lsq": (C.c_int, [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]),
    "shk_assemble": (C.c_int, [C.c_longlong, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                               C.c_int, C.c_void_p]),
    "shk_true_residual": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "shk_true_residual_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p]),
    "shk_sensitivity": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                  C.c_int, C.c_void_p]),
    "shk_profile_enable": (C.c_int, [C.c_int]),
    "shk_profile_read": (C.c_int, [C.POINTER(C.c_longlong), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "shk_profile_read_block": (C.c_int, [C.POINTER(C.c_longlong), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "shk_profile_read_phases": (C.c_int, [C.POINTER(C.c_double), C.c_int]),
    "shk_tune_set": (C.c_int, [C.c_int, C.c_longlong, C.c_int, C.c_int, C.c_int, C.c_char_p, C.c_double]),
    "shk_tune_get": (C.c_int, [C.c_int, C.c_longlong, C.c_int, C.c_int, C.c_int, C.c_char_p,
                               C.POINTER(C.c_double)]),
    "shk_tune_reset": (C.c_int, []),
    "shk_tune_class": (C.c_int, [C.c_void_p, C.POINTER(shk_params), C.c_int, C.POINTER(C.c_int),
                                 C.POINTER(C.c_longlong), C.POINTER(C.c_int)]),
    "shk_status_string": (C.c_char_p, [C.c_int]),
    "shk_last_error": (C.c_char_p, []),
    "shk_server_create": (C.c_int, [C.c_size_t, C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "shk_server_submit": (C.c_int, [C.c_void_p, C.POINTER(shk_request), C.POINTER(C.c_longlong)]),
    "shk_server_poll": (C.c_int, [C.c_void_p, C.c_longlong, C.POINTER(shk_result), C.c_void_p, C.c_void_p]),
    "shk_server_drain": (C.c_int, [C.c_void_p]),
    "shk_server_clock": (C.c_double, [C.c_void_p]),
    "shk_server_destroy": (C.c_int, [C.c_void_p]),
}

_lib = None


def lib():
    """Load libshk.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1212_3660_amd.build`")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded instead of bringing up a second one in the process
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        # the packaged autotuner picks, when there are any
        from . import autotune
        autotune.load()
    return _lib


class ShkError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().shk_last_error().decode()
        super().__init__(f"{where}: {lib().shk_status_string(code).decode()} ({code}): {msg}")
        self.code = code


def _check(rc, where):
    if rc != SHK_OK:
        raise ShkError(rc, where)


def _c128_array(values) -> "C.Array":
    v = np.asarray(values, dtype=np.complex128).ravel()
    arr = (shk_c128 * len(v))()
    for i, z in enumerate(v):
        arr[i].re, arr[i].im = float(z.real), float(z.imag)
    return arr


def make_params(tau_seq, *, m_restart=50, max_restarts=20, max_refine=2, inner_maxit=0, tol=1e-8,
                eps_inner=1e-10, precision=SHK_FP64, variant=SHK_GMRES, refine_tol=0.05,
                refine_eps_inner=5e-3, inner_precond=None, mg_omega=0.8, inner_relax=0.0, inner_eps_max=1e-2,
                ortho=SHK_CGS2, rhs_mode=SHK_RHS_LOCKSTEP, output=SHK_OUT_FULL, out_rows=None):
    """Returns (shk_params, keepalive) with tau_seq (and out_rows) marshalled to C."""
    taus = _c128_array(tau_seq)
    p = shk_params()
    lib().shk_params_default(C.byref(p))
    p.m_restart, p.max_restarts, p.max_refine, p.inner_maxit = m_restart, max_restarts, max_refine, inner_maxit
    p.tol, p.eps_inner = tol, eps_inner
    p.n_tau = len(taus)
    p.tau_seq = C.cast(taus, C.POINTER(shk_c128))
    p.variant, p.precision = variant, precision
    p.refine_tol, p.refine_eps_inner = refine_tol, refine_eps_inner
    if inner_precond is not None:
        p.inner_precond = inner_precond
    p.mg_omega = mg_omega
    p.inner_relax, p.inner_eps_max = inner_relax, inner_eps_max
    p.ortho = ortho
    p.rhs_mode = rhs_mode
    p.output = output
    rows = None
    if out_rows is not None:
        rows = np.ascontiguousarray(out_rows, dtype=np.int64)
        p.n_out_rows = len(rows)
        p.out_rows = rows.ctypes.data_as(C.POINTER(C.c_longlong))
    return p, (taus, rows)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream)


class Problem:
    """Owns a shk_problem handle (operator coefficients on the device)."""

    def __init__(self, handle: C.c_void_p, shape):
        self._h = handle
        self.shape = shape

    @property
    def handle(self):
        return self._h

    @property
    def n(self) -> int:
        return int(lib().shk_problem_size(self._h))

    @classmethod
    def fv2d(cls, cell_K: np.ndarray, Ss: float = 1e-5, h: float = 1.0) -> "Problem":
        K = np.ascontiguousarray(cell_K, dtype=np.float64)
        ny, nx = K.shape
        out = C.c_void_p()
        _check(lib().shk_problem_create_fv2d(nx, ny, K.ctypes.data, Ss, h, C.byref(out)), "shk_problem_create_fv2d")
        return cls(out, K.shape)

    @classmethod
    def fv3d(cls, cell_K: np.ndarray, Ss: float = 1e-5, h: float = 1.0) -> "Problem":
        K = np.ascontiguousarray(cell_K, dtype=np.float64)
        nz, ny, nx = K.shape
        out = C.c_void_p()
        _check(lib().shk_problem_create_fv3d(nx, ny, nz, K.ctypes.data, Ss, h, C.byref(out)),
               "shk_problem_create_fv3d")
        return cls(out, K.shape)

    @classmethod
    def csr(cls, rowptr, col, val, mdiag) -> "Problem":
        rp = np.ascontiguousarray(rowptr, dtype=np.int32)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        vl = np.ascontiguousarray(val, dtype=np.float64)
        md = np.ascontiguousarray(mdiag, dtype=np.float64)
        out = C.c_void_p()
        _check(lib().shk_problem_create_csr(len(rp) - 1, rp.ctypes.data, cl.ctypes.data, vl.ctypes.data,
                                            md.ctypes.data, C.byref(out)), "shk_problem_create_csr")
        return cls(out, (len(rp) - 1,))

    def close(self):
        if self._h:
            lib().shk_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shk_workspace_bytes(problem: Problem, params: shk_params, n_shifts: int, n_rhs: int) -> int:
    out = C.c_size_t()
    _check(lib().shk_workspace_bytes(problem.handle, C.byref(params), n_shifts, n_rhs, C.byref(out)),
           "shk_workspace_bytes")
    return int(out.value)


def shk_output_elems(problem: Problem, params: shk_params, n_shifts: int, n_rhs: int):
    """(complex elements of x, k_cap) for params.output."""
    e, k = C.c_size_t(), C.c_int()
    _check(lib().shk_output_elems(problem.handle, C.byref(params), n_shifts, n_rhs, C.byref(e), C.byref(k)),
           "shk_output_elems")
    return int(e.value), int(k.value)


def _split_output(flat, params, n, nf, nr, kcap, host):
    """Views of a flat output buffer per mode: FULL (n, nf, nr) / ROWS
    (n_rows, nf, nr) Fortran-ordered on the host, (nr, nf, n) / (nr, nf,
    n_rows) on the device; FACTORED a pair (Z, Y)."""
    if params.output == SHK_OUT_FACTORED:
        nz = n * kcap * nr
        if host:
            return (flat[:nz].reshape((n, kcap, nr), order="F"), flat[nz:].reshape((kcap, nf, nr), order="F"))
        return flat[:nz].view(nr, kcap, n), flat[nz:].view(nr, nf, kcap)
    rows = params.n_out_rows if params.output == SHK_OUT_ROWS else n
    if host:
        return flat.reshape((rows, nf, nr), order="F")
    return flat.view(nr, nf, rows)


def fgmres_sh_solve(problem: Problem, params: shk_params, sigma, b, x=None, workspace=None, stream=None):
    """Solve all shifts for all right-hand sides.

    ``b``: NumPy (n,) / (n, n_rhs) complex128 -> host path, x returned as NumPy
    (n, n_shifts, n_rhs) in Fortran order; or a torch CUDA complex128 tensor of
    shape (n_rhs, n) (each row one rhs, i.e. n x n_rhs column-major) -> device
    path, x a torch tensor (n_rhs, n_shifts, n).  With params.output ROWS the
    cell axis has n_out_rows entries; FACTORED returns x as a pair (Z, Y) with
    x_{j,r} = Z[:, :, r] @ Y[:, j, r] (host) / Z[r].T @ Y[r, j] (device).
    Returns (x, statuses) with statuses a structured array of shape
    (n_rhs, n_shifts)."""
    sig = _c128_array(sigma)
    nf = len(sig)
    st = np.zeros(nf * 1, dtype=STATUS_DTYPE)
    if isinstance(b, np.ndarray):
        bb = np.asarray(b, dtype=np.complex128)
        if bb.ndim == 1:
            bb = bb[:, None]
        n, nr = bb.shape
        bf = np.asfortranarray(bb)
        elems, kcap = shk_output_elems(problem, params, nf, nr)
        xflat = np.zeros(elems, dtype=np.complex128)
        st = np.zeros((nr, nf), dtype=STATUS_DTYPE)
        ws_ptr = workspace.data_ptr() if workspace is not None else None
        ws_len = workspace.numel() * workspace.element_size() if workspace is not None else 0
        rc = lib().fgmres_sh_solve(problem.handle, C.byref(params), nf, sig, nr, bf.ctypes.data, xflat.ctypes.data,
                                   st.ctypes.data, ws_ptr, ws_len, None if stream is None else C.c_void_p(stream),
                                   SHK_PTR_HOST)
        _check(rc, "fgmres_sh_solve")
        return _split_output(xflat, params, n, nf, nr, kcap, True), st
    import torch
    assert b.is_cuda and b.dtype == torch.complex128 and b.is_contiguous()
    nr, n = b.shape
    elems, kcap = shk_output_elems(problem, params, nf, nr)
    if x is None:
        x = torch.empty(elems, dtype=torch.complex128, device=b.device)
    assert x.is_cuda and x.dtype == torch.complex128 and x.is_contiguous() and x.numel() == elems
    st = np.zeros((nr, nf), dtype=STATUS_DTYPE)
    if workspace is None:
        need = shk_workspace_bytes(problem, params, nf, nr)
        workspace = torch.empty(need, dtype=torch.uint8, device=b.device)
    rc = lib().fgmres_sh_solve(problem.handle, C.byref(params), nf, sig, nr, C.c_void_p(b.data_ptr()),
                               C.c_void_p(x.data_ptr()), st.ctypes.data, C.c_void_p(workspace.data_ptr()),
                               workspace.numel(), _stream_ptr(stream), SHK_PTR_DEVICE)
    _check(rc, "fgmres_sh_solve")
    return _split_output(x.view(-1), params, n, nf, nr, kcap, False), st


def _prec(t):
    import torch
    if t.dtype == torch.complex128:
        return SHK_FP64
    if t.dtype == torch.complex64:
        return SHK_MIXED
    raise TypeError("complex128 or complex64 tensor expected")


def shk_apply_shifted(problem: Problem, sigma: complex, x, y, n_rhs: int = 1, stream=None):
    """y = (K + sigma M) x on interleaved device vectors (torch tensors)."""
    s = shk_c128(float(np.real(sigma)), float(np.imag(sigma)))
    _check(lib().shk_apply_shifted(problem.handle, s, n_rhs, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                   _prec(x), _stream_ptr(stream)), "shk_apply_shifted")


def shk_inner_solve(problem: Problem, tau: complex, v, z, w=None, eps=1e-10, maxit=0, fixed_iters=0, n_rhs=1,
                    precond=SHK_PRECOND_JACOBI, stream=None):
    """COCG z ~ (K + tau M)^{-1} v (Jacobi or multigrid preconditioner); returns
    (iterations, true residual norms)."""
    t = shk_c128(float(np.real(tau)), float(np.imag(tau)))
    its = np.zeros(n_rhs, dtype=np.int32)
    pn = np.zeros(n_rhs, dtype=np.float64)
    _check(lib().shk_inner_solve(problem.handle, t, n_rhs, C.c_void_p(v.data_ptr()), C.c_void_p(z.data_ptr()),
                                 C.c_void_p(w.data_ptr()) if w is not None else None, eps, maxit, fixed_iters,
                                 _prec(v), precond, its.ctypes.data, pn.ctypes.data, _stream_ptr(stream)),
           "shk_inner_solve")
    return its, pn


def shk_orthogonalize(n: int, k: int, V, w, n_rhs: int = 1, stream=None, ortho: int = SHK_CGS2):
    """Gram-Schmidt (CGS2 or MGS) of w against k columns of V (device, column
    stride n*n_rhs); writes V column k; returns h as (n_rhs, k+1) complex128."""
    h = np.zeros((n_rhs, k + 1), dtype=np.complex128)
    _check(lib().shk_orthogonalize(n, n_rhs, k, C.c_void_p(V.data_ptr()), C.c_void_p(w.data_ptr()), h.ctypes.data,
                                   _prec(w), ortho, _stream_ptr(stream)), "shk_orthogonalize")
    return h


def shk_shifted_lsq(Hbar: np.ndarray, taus, sigma, beta: float, variant: int = SHK_GMRES):
    """Device Givens solution of the per-shift projected problems (least
    squares, or the square FOM system) for a (k+1) x k Hessenberg; returns
    (y (n_shifts, k), rho (k, n_shifts))."""
    H = np.asfortranarray(Hbar, dtype=np.complex128)
    k = H.shape[1]
    tt = np.ascontiguousarray(taus, dtype=np.complex128)
    sg = np.ascontiguousarray(sigma, dtype=np.complex128)
    nf = len(sg)
    y = np.zeros((nf, k), dtype=np.complex128)
    rho = np.zeros((k, nf), dtype=np.float64)
    _check(lib().shk_shifted_lsq(k, H.ctypes.data, tt.ctypes.data, nf, sg.ctypes.data, beta, y.ctypes.data,
                                 rho.ctypes.data, variant), "shk_shifted_lsq")
    return y, rho


def shk_block_orthogonalize(n: int, k: int, V, W, n_rhs: int, stream=None):
    """Block CGS2 of W (device, n x n_rhs interleaved) against k blocks of V and
    CholQR2 into V block k; returns h as ((k+1) n_rhs, n_rhs) complex128."""
    h = np.zeros(((k + 1) * n_rhs, n_rhs), dtype=np.complex128, order="F")
    _check(lib().shk_block_orthogonalize(n, n_rhs, k, C.c_void_p(V.data_ptr()), C.c_void_p(W.data_ptr()),
                                         h.ctypes.data, _prec(W), _stream_ptr(stream)), "shk_block_orthogonalize")
    return h


def shk_block_shifted_lsq(Hbar: np.ndarray, taus, sigma, beta: np.ndarray, n_rhs: int):
    """Device block least squares of every shift for a ((k+1)s x ks) block
    Hessenberg; returns (y (n_shifts, s, k s), rho (k, n_shifts, s))."""
    H = np.asfortranarray(Hbar, dtype=np.complex128)
    k = H.shape[1] // n_rhs
    tt = np.ascontiguousarray(taus, dtype=np.complex128)
    sg = np.ascontiguousarray(sigma, dtype=np.complex128)
    bb = np.asfortranarray(beta, dtype=np.complex128)
    nf = len(sg)
    y = np.zeros((nf, n_rhs, k * n_rhs), dtype=np.complex128)
    rho = np.zeros((k, nf, n_rhs), dtype=np.float64)
    _check(lib().shk_block_shifted_lsq(k, n_rhs, H.ctypes.data, tt.ctypes.data, nf, sg.ctypes.data, bb.ctypes.data,
                                       y.ctypes.data, rho.ctypes.data), "shk_block_shifted_lsq")
    return y, rho


def shk_assemble(n: int, k: int, n_shifts: int, Z, Y, X, accumulate=False, stream=None):
    _check(lib().shk_assemble(n, k, n_shifts, C.c_void_p(Z.data_ptr()), C.c_void_p(Y.data_ptr()),
                              C.c_void_p(X.data_ptr()), 1 if accumulate else 0, _prec(Z), _stream_ptr(stream)),
           "shk_assemble")


def shk_true_residual(problem: Problem, sigma, b, x, stream=None) -> np.ndarray:
    sg = np.ascontiguousarray(sigma, dtype=np.complex128)
    out = np.zeros(len(sg), dtype=np.float64)
    _check(lib().shk_true_residual(problem.handle, len(sg), sg.ctypes.data, C.c_void_p(b.data_ptr()),
                                   C.c_void_p(x.data_ptr()), out.ctypes.data, _stream_ptr(stream)),
           "shk_true_residual")
    return out


def shk_true_residual_noalloc(problem: Problem, sigma, b, x, stream=None) -> np.ndarray:
    """shk_true_residual with the library's fixed device scratch (no device
    allocation)."""
    sg = np.ascontiguousarray(sigma, dtype=np.complex128)
    out = np.zeros(len(sg), dtype=np.float64)
    _check(lib().shk_true_residual_noalloc(problem.handle, len(sg), sg.ctypes.data, C.c_void_p(b.data_ptr()),
                                           C.c_void_p(x.data_ptr()), out.ctypes.data, _stream_ptr(stream)),
           "shk_true_residual_noalloc")
    return out


def shk_sensitivity(problem: Problem, phi, psi, J, n_shifts: int, n_src: int, n_rec: int, stream=None):
    """Sensitivities dh/d(ln K_c) (device tensors; phi: n*n_shifts*n_src and psi:
    n*n_shifts*n_rec complex128 in the solver's layout; J complex128 or
    complex64 with n*n_rec*n_src*n_shifts entries, cell fastest)."""
    import torch
    prec = SHK_FP64 if J.dtype == torch.complex128 else SHK_MIXED
    _check(lib().shk_sensitivity(problem.handle, n_shifts, n_src, C.c_void_p(phi.data_ptr()), n_rec,
                                 C.c_void_p(psi.data_ptr()), C.c_void_p(J.data_ptr()), prec, _stream_ptr(stream)),
           "shk_sensitivity")


def shk_profile_enable(on: bool = True, phases: bool = False):
    """on: the inner-iteration instrumentation; phases: the phase timer."""
    _check(lib().shk_profile_enable((1 if on else 0) | (2 if phases else 0)), "shk_profile_enable")


def shk_profile_read():
    """(launches, total_ms, total_bytes) of the timed inner-iteration kernel launches."""
    n, ms, by = C.c_longlong(), C.c_double(), C.c_double()
    _check(lib().shk_profile_read(C.byref(n), C.byref(ms), C.byref(by)), "shk_profile_read")
    return int(n.value), float(ms.value), float(by.value)


def shk_profile_read_block():
    """(calls, total_ms, total_flops) of the timed block Gram-Schmidt steps."""
    n, ms, fl = C.c_longlong(), C.c_double(), C.c_double()
    _check(lib().shk_profile_read_block(C.byref(n), C.byref(ms), C.byref(fl)), "shk_profile_read_block")
    return int(n.value), float(ms.value), float(fl.value)


# Workload class key of the tuning table: (kind, n, lanes, precision, precond);
# kind -1 addresses the settings shared by every class without an entry.
TUNE_ALL = (-1, 0, 0, 0, 0)


def shk_tune_set(key, knob: str, value: float):
    """Sets one knob of a class (shk_tune_set)."""
    k, n, lanes, prec, pc = key
    _check(lib().shk_tune_set(int(k), int(n), int(lanes), int(prec), int(pc), knob.encode(), float(value)),
           "shk_tune_set")


def shk_tune_get(key, knob: str) -> float:
    k, n, lanes, prec, pc = key
    v = C.c_double()
    _check(lib().shk_tune_get(int(k), int(n), int(lanes), int(prec), int(pc), knob.encode(), C.byref(v)),
           "shk_tune_get")
    return float(v.value)


def shk_tune_reset():
    _check(lib().shk_tune_reset(), "shk_tune_reset")


def shk_tune_class(problem: Problem, params: shk_params, n_rhs: int):
    """The class key (kind, n, lanes, precision, precond) of a solve."""
    k, n, lanes = C.c_int(), C.c_longlong(), C.c_int()
    _check(lib().shk_tune_class(problem.handle, C.byref(params), int(n_rhs), C.byref(k), C.byref(n),
                                C.byref(lanes)), "shk_tune_class")
    return (int(k.value), int(n.value), int(lanes.value), int(params.precision), int(params.inner_precond))


PHASES = ("pass start", "inner solves", "Gram-Schmidt", "least squares and step test", "host turnaround",
          "assembly and restarts", "true residuals", "block passes")


def shk_profile_read_phases():
    """Phase totals (ms) since shk_profile_enable with bit 1 set, keyed by
    PHASES."""
    ms = (C.c_double * len(PHASES))()
    n = lib().shk_profile_read_phases(ms, len(PHASES))
    if n < 0:
        _check(n, "shk_profile_read_phases")
    return {PHASES[i]: float(ms[i]) for i in range(min(n, len(PHASES)))}


class Server:
    """Continuous-admission solve server (shk_server_*)."""

    def __init__(self, mem_budget_bytes: int, max_slots: int = 4, arena=None):
        """arena: a CUDA tensor of at least mem_budget_bytes (kept alive by this
        object), or None to let the server allocate its arena once."""
        self._h = C.c_void_p()
        self._arena = arena
        ptr = None
        if arena is not None:
            assert arena.is_cuda and arena.numel() * arena.element_size() >= mem_budget_bytes
            ptr = C.c_void_p(arena.data_ptr())
        _check(lib().shk_server_create(mem_budget_bytes, max_slots, ptr, C.byref(self._h)), "shk_server_create")
        self._keep = {}

    def submit(self, cell_K, sigma, b, params: shk_params, Ss=1e-5, h=1.0, keep_solution=False) -> int:
        K = np.ascontiguousarray(cell_K, dtype=np.float64)
        ny, nx = K.shape
        sg = np.ascontiguousarray(sigma, dtype=np.complex128)
        bb = np.asarray(b, dtype=np.complex128)
        if bb.ndim == 1:
            bb = bb[:, None]
        bf = np.asfortranarray(bb)
        req = shk_request()
        req.nx, req.ny = nx, ny
        req.cell_K = K.ctypes.data_as(C.POINTER(C.c_double))
        req.Ss, req.h = Ss, h
        req.n_shifts = len(sg)
        req.sigma = sg.ctypes.data_as(C.POINTER(shk_c128))
        req.n_rhs = bf.shape[1]
        req.b = bf.ctypes.data_as(C.POINTER(shk_c128))
        req.params = params
        req.keep_solution = 1 if keep_solution else 0
        t = C.c_longlong()
        _check(lib().shk_server_submit(self._h, C.byref(req), C.byref(t)), "shk_server_submit")
        out = shk_params()
        C.pointer(out)[0] = params
        kcap = params.m_restart * (params.max_restarts + 1) * (params.max_refine + 1)
        self._keep[t.value] = (K.shape, len(sg), bf.shape[1], out, kcap)
        return t.value

    def poll(self, ticket: int, want_solution=False):
        """None while running; else (result dict, output or None, statuses);
        the output is shaped per the request's output mode as in
        fgmres_sh_solve's host path."""
        shape, nf, nr, prm, kcap = self._keep[ticket]
        n = int(np.prod(shape))
        res = shk_result()
        if prm.output == SHK_OUT_ROWS:
            elems = prm.n_out_rows * nf * nr
        elif prm.output == SHK_OUT_FACTORED:
            elems = kcap * (n + nf) * nr
        else:
            elems = n * nf * nr
        flat = np.zeros(elems, dtype=np.complex128) if want_solution else None
        st = np.zeros((nr, nf), dtype=STATUS_DTYPE)
        rc = lib().shk_server_poll(self._h, ticket, C.byref(res), flat.ctypes.data if flat is not None else None,
                                   st.ctypes.data)
        if rc == SHK_ERR_NOT_READY:
            return None
        _check(rc, "shk_server_poll")
        d = {f: getattr(res, f) for f, _ in shk_result._fields_}
        x = _split_output(flat, prm, n, nf, nr, kcap, True) if flat is not None else None
        return d, x, st

    def drain(self):
        _check(lib().shk_server_drain(self._h), "shk_server_drain")

    def clock(self) -> float:
        return float(lib().shk_server_clock(self._h))

    def close(self):
        if self._h:
            lib().shk_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exported_symbols() -> Sequence[str]:
    return list(_SIGS.keys())
