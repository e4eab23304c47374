"""Seeded synthetic inputs for the shifted-system solver.

This module produces *inputs only*: conductivity fields, frequency lists,
preconditioner-shift schedules, right-hand sides and request traces.  It holds
none of the solver's arithmetic (no operator assembly, no Krylov step), so
both the independent CPU oracle and the GPU library may consume what it
returns.

Regime (paper section 6.1, Table 1): conductivities around 1e-5 m/s, specific
storage around 1e-5 1/m, up to 200 frequencies.  The paper's own random field
is not available; these recipes stand in for it.

Random numbers: NumPy PCG64 streams keyed by ``SeedSequence([cfg, purpose,
idx])`` so that each (configuration, purpose, index) triple is reproducible
and independent of the others.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# purpose codes for the seed sequence
P_FIELD, P_WELLS, P_RECEIVERS, P_TRACE, P_RHS = 0, 1, 2, 3, 4


def rng(cfg: int, purpose: int, idx: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(cfg), int(purpose), int(idx)]))


def periods(n: int, t_min: float, t_max: float) -> np.ndarray:
    """n periods log-spaced from t_min to t_max (ascending), 1-based index j:
    T_j = t_min (t_max/t_min)^((j-1)/(n-1))."""
    if n == 1:
        return np.array([float(t_min)])
    j = np.arange(n, dtype=np.float64)
    return t_min * (t_max / t_min) ** (j / (n - 1))


def shifts_from_periods(T: np.ndarray) -> np.ndarray:
    """Phasor shifts sigma = i*omega with omega = 2*pi/T (section 5.1)."""
    return 1j * (2.0 * math.pi / np.asarray(T, dtype=np.float64))


def box_mean(a: np.ndarray, half: int) -> np.ndarray:
    """Truncated-window box mean: each cell becomes the mean of the cells of the
    (2*half+1)^d window that lie inside the grid."""
    out = np.asarray(a, dtype=np.float64)
    for ax in range(out.ndim):
        n = out.shape[ax]
        c = np.cumsum(out, axis=ax)
        zero_shape = list(out.shape)
        zero_shape[ax] = 1
        c = np.concatenate([np.zeros(zero_shape), c], axis=ax)
        idx = np.arange(n)
        hi = np.minimum(idx + half + 1, n)
        lo = np.maximum(idx - half, 0)
        s = np.take(c, hi, axis=ax) - np.take(c, lo, axis=ax)
        cnt = (hi - lo).astype(np.float64)
        shape = [1] * out.ndim
        shape[ax] = n
        out = s / cnt.reshape(shape)
    return out


def lnk_field(shape: Tuple[int, ...], mean: float, var: float, box: int,
              cfg: int, idx: int = 0) -> np.ndarray:
    """ln K ~ N(mean, var) iid per cell, then a box filter of width ``box``.
    Returned with shape (nz, ny, nx) or (ny, nx): x varies fastest in memory."""
    g = rng(cfg, P_FIELD, idx)
    raw = mean + math.sqrt(var) * g.standard_normal(shape)
    if box > 1:
        raw = box_mean(raw, box // 2)
    return raw


def cell_conductivity(shape, mean=-11.5, var=1.0, box=5, cfg=1, idx=0) -> np.ndarray:
    """Cell conductivity K = exp(ln K) as a C-ordered float64 array."""
    return np.ascontiguousarray(np.exp(lnk_field(shape, mean, var, box, cfg, idx)))


def cell_index(shape: Sequence[int], coords: Sequence[int]) -> int:
    """Row-major cell index with x fastest: coords are (x, y[, z])."""
    if len(shape) == 2:
        ny, nx = shape
        x, y = coords
        return int(x + nx * y)
    nz, ny, nx = shape
    x, y, z = coords
    return int(x + nx * (y + ny * z))


def unit_vector(n: int, i: int) -> np.ndarray:
    b = np.zeros(n, dtype=np.complex128)
    b[i] = 1.0
    return b


def distinct_interior_cells(shape, count, cfg, purpose, margin=2, exclude=()) -> List[int]:
    """``count`` distinct cells at least ``margin`` cells from the boundary,
    avoiding ``exclude``; seeded."""
    g = rng(cfg, purpose)
    dims = list(reversed(shape))  # (nx, ny[, nz])
    chosen: List[int] = []
    excl = set(int(e) for e in exclude)
    while len(chosen) < count:
        coords = [int(g.integers(margin, d - margin)) for d in dims]
        c = cell_index(shape, coords)
        if c in excl or c in chosen:
            continue
        chosen.append(c)
    return chosen


def cyclic_tau(omegas: np.ndarray, idx1: Sequence[int]) -> np.ndarray:
    """tau values i*omega_k for the given 1-based frequency indices; the solver
    uses them cyclically."""
    return np.array([1j * omegas[k - 1] for k in idx1], dtype=np.complex128)


def blocked_tau(tau_bar: Sequence[complex], m: int) -> np.ndarray:
    """Blocked schedule of section 2.2.1: the first m/n_p steps use tau_bar[0],
    the next m/n_p tau_bar[1], and so on (m_k = m/n_p)."""
    n_p = len(tau_bar)
    mk = m // n_p
    seq = []
    for t in tau_bar:
        seq += [complex(t)] * mk
    while len(seq) < m:
        seq.append(complex(tau_bar[-1]))
    return np.array(seq, dtype=np.complex128)


def log_spaced_tau(omega_min: float, omega_max: float, n_p: int) -> np.ndarray:
    """n_p preconditioner frequencies evenly spaced on a log scale over the
    frequency range (section 6.1)."""
    w = np.exp(np.linspace(math.log(omega_min), math.log(omega_max), n_p))
    return 1j * w


@dataclass
class Workload:
    """One synthetic problem: field, shifts, schedule, right-hand sides."""
    name: str
    shape: Tuple[int, ...]          # (ny, nx) or (nz, ny, nx)
    cell_K: np.ndarray              # float64, same shape
    Ss: float
    h: float
    periods: np.ndarray
    sigma: np.ndarray               # complex128 (n_f,)
    tau_seq: np.ndarray             # complex128, used cyclically
    b: np.ndarray                   # complex128 (n, n_rhs), column-major semantics
    eps_inner: float
    tol: float
    m_restart: int
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))

    @property
    def dims(self) -> Tuple[int, ...]:
        return tuple(reversed(self.shape))  # (nx, ny[, nz])


def config1(n_grid: int = 64) -> Workload:
    """64x64 2-D, 10 periods 10..1000 s, point source at the centre, single
    tau = i*omega_5, inner 1e-10, restart 50, complex128."""
    shape = (n_grid, n_grid)
    K = cell_conductivity(shape, -11.5, 1.0, 5, cfg=1)
    T = periods(10, 10.0, 1000.0)
    om = 2 * math.pi / T
    n = n_grid * n_grid
    b = unit_vector(n, cell_index(shape, (n_grid // 2, n_grid // 2)))[:, None]
    return Workload("c1_2d_64x64_10shifts", shape, K, 1e-5, 1.0, T, 1j * om,
                    cyclic_tau(om, [5]), b, 1e-10, 1e-8, 50)


def config2(n_grid: int = 512, n_f: int = 200) -> Workload:
    """512x512 2-D, 200 periods 5..5000 s, one point source at the centre,
    tau cyclic over {i w_20, i w_100, i w_180}, inner COCG 1e-6, target 1e-6."""
    shape = (n_grid, n_grid)
    K = cell_conductivity(shape, -11.5, 1.0, 5, cfg=2)
    T = periods(n_f, 5.0, 5000.0)
    om = 2 * math.pi / T
    n = n_grid * n_grid
    b = unit_vector(n, cell_index(shape, (n_grid // 2, n_grid // 2)))[:, None]
    idx = [20, 100, 180] if n_f >= 180 else [max(1, n_f // 10), max(1, n_f // 2), max(1, (9 * n_f) // 10)]
    return Workload("c2_2d_512x512_200shifts", shape, K, 1e-5, 1.0, T, 1j * om,
                    cyclic_tau(om, idx), b, 1e-6, 1e-6, 50)


def config3(n_grid: int = 256, n_f: int = 50, n_src: int = 32, n_rec: int = 32) -> Workload:
    """256x256 2-D, 50 periods 10..2000 s, 32 unit sources at well cells and 32
    adjoint unit vectors at receiver cells; tau cyclic {i w_5, i w_25, i w_45}."""
    shape = (n_grid, n_grid)
    K = cell_conductivity(shape, -11.5, 1.0, 5, cfg=3)
    T = periods(n_f, 10.0, 2000.0)
    om = 2 * math.pi / T
    n = n_grid * n_grid
    wells = distinct_interior_cells(shape, n_src, 3, P_WELLS)
    recv = distinct_interior_cells(shape, n_rec, 3, P_RECEIVERS, exclude=wells)
    b = np.zeros((n, n_src + n_rec), dtype=np.complex128)
    for r, c in enumerate(wells + recv):
        b[c, r] = 1.0
    idx = [5, 25, 45] if n_f >= 45 else [1, max(1, n_f // 2), n_f]
    return Workload("c3_2d_256x256_50shifts_64rhs", shape, K, 1e-5, 1.0, T, 1j * om,
                    cyclic_tau(om, idx), b, 1e-6, 1e-6, 50,
                    extra={"wells": wells, "receivers": recv})


def config4(n_grid: int = 128, n_f: int = 100, n_rhs: int = 8) -> Workload:
    """128^3 3-D 7-point, ln K ~ N(-11.5, var 1.5) with a 5^3 box, 100 periods
    10..1000 s, 8 point sources, tau cyclic {i w_25, i w_75}."""
    shape = (n_grid, n_grid, n_grid)
    K = cell_conductivity(shape, -11.5, 1.5, 5, cfg=4)
    T = periods(n_f, 10.0, 1000.0)
    om = 2 * math.pi / T
    n = n_grid ** 3
    src = distinct_interior_cells(shape, n_rhs, 4, P_WELLS)
    b = np.zeros((n, n_rhs), dtype=np.complex128)
    for r, c in enumerate(src):
        b[c, r] = 1.0
    idx = [25, 75] if n_f >= 75 else [max(1, n_f // 4), max(1, (3 * n_f) // 4)]
    return Workload("c4_3d_128cubed_100shifts_8rhs", shape, K, 1e-5, 1.0, T, 1j * om,
                    cyclic_tau(om, idx), b, 1e-6, 1e-6, 50, extra={"sources": src})


@dataclass
class Request:
    rid: int
    arrival: float        # seconds from trace start
    n_grid: int
    field_seed: int
    n_f: int
    n_rhs: int


def server_trace(rate: float = 20.0, duration: float = 600.0,
                 grids=(128, 256, 512), nf_range=(5, 200), rhs_range=(1, 16),
                 cfg: int = 5, max_requests: Optional[int] = None) -> List[Request]:
    """Poisson arrivals at ``rate``/s for ``duration`` s.  Each request: a 2-D
    grid drawn uniformly from ``grids`` with its own field seed, n_f uniform in
    ``nf_range`` (inclusive), n_rhs uniform in ``rhs_range`` (inclusive)."""
    g = rng(cfg, P_TRACE)
    t = 0.0
    out: List[Request] = []
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            break
        out.append(Request(len(out), t, int(g.choice(grids)), int(g.integers(0, 2**31 - 1)),
                           int(g.integers(nf_range[0], nf_range[1] + 1)),
                           int(g.integers(rhs_range[0], rhs_range[1] + 1))))
        if max_requests is not None and len(out) >= max_requests:
            break
    return out


def request_workload(req: Request, t_min=10.0, t_max=1000.0) -> Workload:
    """Materialise one serving request: its own field (seed from the trace),
    shifts, tau at the 10/50/90 % positions of its shift list, and n_rhs point
    sources at seeded interior cells."""
    shape = (req.n_grid, req.n_grid)
    K = cell_conductivity(shape, -11.5, 1.0, 5, cfg=5, idx=1000 + req.field_seed % 1000003)
    T = periods(req.n_f, t_min, t_max)
    om = 2 * math.pi / T
    n = req.n_grid ** 2
    src = distinct_interior_cells(shape, req.n_rhs, 5, P_RHS * 1000 + req.rid % 997)
    b = np.zeros((n, req.n_rhs), dtype=np.complex128)
    for r, c in enumerate(src):
        b[c, r] = 1.0
    nf = req.n_f
    idx = sorted(set([max(1, round(0.1 * nf)), max(1, round(0.5 * nf)), max(1, round(0.9 * nf))]))
    return Workload(f"req{req.rid}", shape, K, 1e-5, 1.0, T, 1j * om,
                    cyclic_tau(om, idx), b, 1e-6, 1e-6, 50)
