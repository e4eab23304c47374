// HIP kernels of the flexible shifted-Krylov solver (gfx950, wave64).
//
// Layout: S right-hand-side lanes interleaved, element (cell c, lane r) at
// c*S + r, S a power of two <= 64.  Item kernels use 256-thread blocks with a
// grid-stride loop whose stride is a multiple of S, so each thread keeps one
// lane r for its whole life and per-lane sums need no atomics.
//
// Reductions are deterministic: per-thread sums, a fixed wave tree, a fixed
// cross-wave sum per block written as a block partial; the kernel that needs
// the total (the next one in stream order, so the kernel boundary makes the
// partials visible without device-scope fences) adds the partials in block
// order, redundantly in every block that needs them.  Repeated runs give
// bitwise identical results.
#pragma once
#include "common.hpp"
#include "ops.hpp"
#include "../../include/shk.h"

namespace shk {

constexpr int BS = 256;
constexpr int NWAVE = BS / WAVE;

// XCD-aware block order: gfx950 dispatches consecutive workgroups round-robin
// over its 8 XCDs, each with its own L2.  Mapping block b to tile
// (b % 8) * (G / 8) + b / 8 gives every XCD a contiguous band of tiles, so the
// stencil's halo rows are mostly read from the XCD's own L2.  Identity when G
// is not a multiple of 8.
__device__ __forceinline__ int xcd_tile(int b, int G) {
  if (G & 7) return b;
  return (b & 7) * (G >> 3) + (b >> 3);
}

// Grid-stride walk over the items (cell, lane chunk) of a stencil kernel,
// chunks fastest (lC = log2 of the chunks per cell).  On a grid operator with
// the launch grid and ny
// multiples of 8, XCD x takes the cells of the rows [x ny/8, (x+1) ny/8) of
// every plane, in order (x, then y in the slab, then z), and its blocks stride
// through them together, so the rows and planes next to the ones in work are
// its own, in its L2.  Otherwise the items go in order, dealt to the XCDs in
// bands per stride (xcd_tile).
struct SlabWalk {
  long start, step, end;
  int slab, nx, ny, ry, lC;
  template <typename Op>
  __device__ SlabWalk(const Op& op, long items, int lC_, int cgb) : lC(lC_) {
    const int G = gridDim.x;
    nx = ny = 1;
    int nz = 1;
    if constexpr (Op::NB > 0) {
      nx = op.nx;
      ny = op.ny;
    }
    if constexpr (Op::NB == 6) nz = op.nz;
    if (Op::NB > 0 && (G & 7) == 0 && (ny & 7) == 0) {
      slab = (int)(blockIdx.x & 7);
      ry = ny >> 3;
      start = (long)(blockIdx.x >> 3) * cgb + threadIdx.x;
      step = (long)(G >> 3) * cgb;
      end = ((long)nx * ry * nz) << lC;
    } else {
      slab = -1;
      ry = 0;
      start = (long)xcd_tile(blockIdx.x, G) * cgb + threadIdx.x;
      step = (long)G * cgb;
      end = items;
    }
  }
  __device__ long first() const { return start; }
  __device__ int cell(long t) const {
    const long c = t >> lC;
    if (slab < 0) return (int)c;
    const long r = c / nx;
    const int i = (int)(c - r * nx);
    const long z = r / ry;
    const int y = slab * ry + (int)(r - z * ry);
    return i + nx * (y + ny * (int)z);
  }
};

// ------------------------------------------------------------ reductions ---
// Workgroup barrier that orders LDS only: outstanding global loads stay in
// flight across it (a full __syncthreads would wait for them).
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block partial per lane: wave tree over lanes of equal r, then the waves in
// order.  Writes out[q*S + r] for r < S.
template <int NV, int BSZ = BS>
__device__ __forceinline__ void block_partials(c128 (&v)[NV], int S, c128* __restrict__ out) {
  constexpr int NW = BSZ / WAVE;
  __shared__ c128 sh[NW][NV][WAVE];
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum_strided(v[q], S);
  if (lane < S) {
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[wv][q][lane] = v[q];
  }
  lds_sync();
  if ((int)threadIdx.x < S) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      c128 a = sh[0][q][threadIdx.x];
      for (int w = 1; w < NW; ++w) a = a + sh[w][q][threadIdx.x];
      out[q * S + threadIdx.x] = a;
    }
  }
  lds_sync();
}

// Sum partials laid out [block][NV][S] over G blocks in a fixed order (strided
// per-thread sums, a wave tree, then the waves in order).  Every thread gets
// the totals of its lane r = threadIdx.x % S.
//
// Split in two so a kernel can issue the partial loads, then its own loads,
// and only then wait: PartLoad holds up to KMAX blocks' partials per thread
// (predicated, fully unrolled: all loads in flight at once); blocks beyond
// KMAX * (BSZ / S) are summed by a plain loop in part_sum.
template <int NV, int KMAX> struct PartLoad {
  c128 v[KMAX][NV];
};
template <int NV, int KMAX, int BSZ>
__device__ __forceinline__ void part_load(const c128* __restrict__ part, int G, int S, PartLoad<NV, KMAX>& L) {
  const int r = threadIdx.x & (S - 1), c0 = threadIdx.x / S, C = BSZ / S;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int b = c0 + k * C;
#pragma unroll
    for (int q = 0; q < NV; ++q) L.v[k][q] = b < G ? part[((size_t)b * NV + q) * S + r] : c128{0.0, 0.0};
  }
}
template <int NV, int KMAX, int BSZ>
__device__ __forceinline__ void part_sum(const c128* __restrict__ part, int G, int S, const PartLoad<NV, KMAX>& L,
                                         c128 (&res)[NV]) {
  constexpr int NW = BSZ / WAVE;
  __shared__ c128 sh[NW][NV][WAVE];
  const int r = threadIdx.x & (S - 1), c0 = threadIdx.x / S, C = BSZ / S;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  c128 acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    acc[q] = L.v[0][q];
#pragma unroll
    for (int k = 1; k < KMAX; ++k) acc[q] = acc[q] + L.v[k][q];
  }
  for (int b = c0 + KMAX * C; b < G; b += C) {
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = acc[q] + part[((size_t)b * NV + q) * S + r];
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = wave_sum_strided(acc[q], S);
  if (lane < S) {
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[wv][q][lane] = acc[q];
  }
  lds_sync();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    c128 a = sh[0][q][r];
    for (int w = 1; w < NW; ++w) a = a + sh[w][q][r];
    res[q] = a;
  }
  lds_sync();
}
template <int NV, int BSZ = BS>
__device__ __forceinline__ void final_sum(const c128* __restrict__ part, int G, int S, c128 (&res)[NV]) {
  PartLoad<NV, 4> L;
  part_load<NV, 4, BSZ>(part, G, S, L);
  part_sum<NV, 4, BSZ>(part, G, S, L, res);
}

// Block-wide sum of one complex value (all threads one lane), fixed order.
__device__ __forceinline__ c128 block_sum_all(c128 v) {
  __shared__ c128 sh[NWAVE];
  v = wave_sum_strided(v, 1);
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = v;
  lds_sync();
  c128 a = sh[0];
  for (int w = 1; w < NWAVE; ++w) a = a + sh[w];
  lds_sync();
  return a;
}

// ------------------------------------------------------------- setup -------
// Face transmissivities from cell conductivities (section 5.1 discretisation):
// interior faces get the harmonic mean times h^(d-2), boundary faces the cell
// value times h^(d-2) (Dirichlet ghost at distance h).
__global__ void __launch_bounds__(BS) k_faces(const double* __restrict__ K, int nx, int ny, int nz,
                                              int axis, double scale, double* __restrict__ T,
                                              float* __restrict__ T32) {
  const int ex = nx + (axis == 0), ey = ny + (axis == 1), ez = nz + (axis == 2);
  const long total = (long)ex * ey * ez;
  for (long f = blockIdx.x * (long)BS + threadIdx.x; f < total; f += (long)gridDim.x * BS) {
    const int i = (int)(f % ex);
    const long rest = f / ex;
    const int j = (int)(rest % ey);
    const int k = (int)(rest / ey);
    const int a = axis == 0 ? i : (axis == 1 ? j : k);
    const int na = axis == 0 ? nx : (axis == 1 ? ny : nz);
    auto cell = [&](int ii, int jj, int kk) { return K[ii + (long)nx * (jj + (long)ny * kk)]; };
    double t;
    if (a == 0) {
      t = cell(i, j, k);
    } else if (a == na) {
      t = axis == 0 ? cell(i - 1, j, k) : (axis == 1 ? cell(i, j - 1, k) : cell(i, j, k - 1));
    } else {
      const double kb = cell(i, j, k);
      const double ka = axis == 0 ? cell(i - 1, j, k) : (axis == 1 ? cell(i, j - 1, k) : cell(i, j, k - 1));
      t = 2.0 * ka * kb / (ka + kb);
    }
    T[f] = t * scale;
    T32[f] = (float)(t * scale);
  }
}

// ----------------------------------------------------------- vectors -------
// ABI layout (n x s_real column-major) -> interleaved c128 with S lanes.
__global__ void __launch_bounds__(BS) k_interleave(const c128* __restrict__ b, long n, int s_real, int S,
                                                   c128* __restrict__ out) {
  const long N = n * S;
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < N; t += (long)gridDim.x * BS) {
    const long c = t / S;
    const int r = (int)(t - c * S);
    out[t] = r < s_real ? b[c + n * r] : c128{0.0, 0.0};
  }
}

// Per-lane partial sums of |x|^2 (block partials [G][1][S]); k_final_sqrt
// turns them into norms.
template <typename R>
__global__ void __launch_bounds__(BS) k_norm2(const cx<R>* __restrict__ x, long N, int S,
                                              c128* __restrict__ part) {
  c128 acc[1] = {{0.0, 0.0}};
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < N; t += (long)gridDim.x * BS)
    acc[0].re += (double)abs2(x[t]);
  block_partials<1>(acc, S, part + (size_t)blockIdx.x * S);
}

// One block: out_q[r] = sqrt(sum of partial q) for q < NV; optionally also
// written as a complex Hessenberg entry (the subdiagonal h_{k+1,k}).
template <int NV>
__global__ void __launch_bounds__(BS) k_final_sqrt(const c128* __restrict__ part, int G, int S,
                                                   double* __restrict__ out0, double* __restrict__ out1,
                                                   c128* __restrict__ hcol) {
  c128 tot[NV];
  final_sum<NV>(part, G, S, tot);
  if ((int)threadIdx.x < S) {
    const double a = sqrt(tot[0].re);
    if (out0) out0[threadIdx.x] = a;
    if (hcol) hcol[threadIdx.x] = c128{a, 0.0};
    if (NV > 1 && out1) out1[threadIdx.x] = sqrt(tot[NV - 1].re);
  }
}

// The same with one block per lane (launch: S blocks), for many lanes: block
// r sums lane r's G partials in a fixed order.
template <int NV>
__global__ void __launch_bounds__(BS) k_final_sqrt_lanes(const c128* __restrict__ part, int G, int S,
                                                         double* __restrict__ out0, double* __restrict__ out1,
                                                         c128* __restrict__ hcol) {
  const int r = blockIdx.x;
  c128 acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = c128{0.0, 0.0};
  for (int b = threadIdx.x; b < G; b += BS) {
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = acc[q] + part[((size_t)b * NV + q) * S + r];
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = block_sum_all(acc[q]);
  if (threadIdx.x == 0) {
    const double a = sqrt(acc[0].re);
    if (out0) out0[r] = a;
    if (hcol) hcol[r] = c128{a, 0.0};
    if (NV > 1 && out1) out1[r] = sqrt(acc[NV - 1].re);
  }
}

// out = in / beta[r] converted to R (zero lanes stay zero).
template <typename R>
__global__ void __launch_bounds__(BS) k_scale_conv(const c128* __restrict__ in, long N, int S,
                                                   const double* __restrict__ beta, cx<R>* __restrict__ out) {
  const int r = threadIdx.x & (S - 1);
  const double b = beta[r];
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < N; t += (long)gridDim.x * BS)
    out[t] = cvt<R>(inv * in[t]);
}

template <typename R>
__global__ void __launch_bounds__(BS) k_copy(const cx<R>* __restrict__ in, long N, cx<R>* __restrict__ out) {
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < N; t += (long)gridDim.x * BS) out[t] = in[t];
}

template <typename Op, typename R>
__global__ void __launch_bounds__(BS) k_apply(Op op, c128 sigma, long n, int S, const cx<R>* __restrict__ x,
                                              cx<R>* __restrict__ y) {
  const long N = n * S;
  const int r = threadIdx.x & (S - 1);
  const cx<R> sg = cvt<R>(sigma);
  auto g = [&](long cc) { return x[cc * S + r]; };
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < N; t += (long)gridDim.x * BS) {
    const long c = t / S;
    y[t] = op.template apply<R>(c, sg, g);
  }
}

// -------------------------------------------------------- inner COCG --------
// Jacobi-preconditioned COCG (conjugate orthogonal CG for the complex
// symmetric K + tau M, bilinear products x^T y) for z ~ (K + tau M)^{-1} v,
// section 4 eq. zmmoditer, in the single-reduction arrangement of Chronopoulos
// and Gear: with u = D^{-1} r, w = A u and s = A p carried by recurrence, the
// two inner products gamma = r^T u and delta = w^T u of one step fix both
//   beta_{i+1} = gamma_{i+1} / gamma_i,
//   alpha_{i+1} = gamma_{i+1} / (delta_{i+1} - beta_{i+1} gamma_{i+1} / alpha_i),
// which equal the textbook COCG coefficients in exact arithmetic.  One kernel
// per iteration: its prologue sums the previous step's block partials (every
// block the same, fixed order) and applies the stop test ||r|| <= eps ||v||;
// then, per cell,
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r' = r - alpha s,
//   w' = A D^{-1} r'  (r' at the stencil neighbours formed on the fly),
// and partials of r'^T u', w'^T u', ||r'||^2.  r, w, s are read at neighbours
// and so live in two buffers each, selected by the parity of the lane's
// iteration count; p and x (own cell only) are updated in place.  x is FP64 on
// both paths.  On the complex64 path the recurrence residual drifts from the
// true one; once every lane has converged, r = v - A x is recomputed in FP64
// (and w with it) and the iteration resumes where needed (residual
// replacement, van der Vorst and Ye), so the inner tolerance holds for the
// true residual.
// What a lane does in a launch of the iteration kernel.
enum CgMode : int {
  CG_ITER = 0,   // one COCG iteration
  CG_RR = 1,     // FP64 residual r = v - (K + tau M) x of the FP64 iterate
  CG_KX = 2,     // damped Jacobi step x += D^-1 r / 2
  CG_RW = 3,     // round start: w = A D^-1 r and the round's first bilinear forms
  CG_FRESH = 4   // state left by k_cg_init (its r, w and forms are a round start)
};

// Settings of one inner solve, the same for every lane.
struct CgCfg {
  double eps;        // stop at ||r|| <= eps ||v|| (negative: a fixed count)
  double round_tol;  // reduction per round (complex64 path), 0 on the FP64 path
  int maxit;
  int trust;         // 1: the recurrence residual is final (FP64 path, no rounds)
  int stall_min, stall_mult;  // a round without progress for max(stall_min,
                              // stall_mult x its productive length) ends (0: never)
  int fused_start;   // 1: the launch after a residual replacement already has the
                     // new round's forms (multigrid path), 0: it forms them (RW)
};

// The settings of the running inner solve live in device memory, so that a
// captured sequence of iterations serves every inner solve with the same tau.
__global__ void k_set_cfg(CgCfg* __restrict__ d, CgCfg c) {
  if (threadIdx.x == 0) *d = c;
}

// Per-lane state of the inner solve (kept small: a single-lane launch holds it
// in scalar registers; the flags fill one whole dword, as the scalar loads
// that fetch the state need).
struct CgScal {
  c128 gamma, alpha, beta;
  c128 apend;        // multigrid path: coefficient of a deferred x += apend p
  double vnorm, rnorm, rstop;
  double rn0;        // residual norm at the start of the current round
  double rbest;      // best residual of the round, halving by halving
  int its;
  int its0;          // iteration count at the start of the current round
  int its_best;      // iteration at which rbest was reached
  int rounds;        // rounds started
  int pend;          // 1: x lacks apend p (p as stored now)
  signed char done, conv;
  signed char mode;  // CgMode of the launch that produced this state
  signed char kick;  // 1: a Jacobi step was taken for the current round
};


__device__ __forceinline__ bool is_zero(c128 a) { return a.re == 0.0 && a.im == 0.0; }

// A round starts from the forms gamma = r^T D^-1 r (tg), delta = w^T D^-1 r
// (td) and ||r||^2 of the residual r it starts from; this launch iterates.
__device__ __forceinline__ void cg_round_start(CgScal& s, const CgCfg& cfg, c128 tg, c128 td, double trr) {
  const double eps = cfg.eps;
  const double rn = sqrt(trr);
  s.rnorm = rn;
  if (rn <= eps * s.vnorm || s.vnorm == 0.0) {
    s.done = 1; s.conv = 1;
    return;
  }
  if (s.its >= cfg.maxit || is_zero(td) || !(rn == rn)) {
    s.done = 1; s.conv = 0;
    return;
  }
  s.rn0 = rn;
  s.its0 = s.its;
  s.rbest = rn;
  s.its_best = s.its;
  s.rounds += 1;
  s.gamma = tg;
  s.beta = c128{0.0, 0.0};
  s.alpha = cdiv(tg, td);
  s.rstop = fmax(eps * s.vnorm, cfg.round_tol * rn);
  s.mode = CG_ITER;
}

// Lane state transition from the previous launch's totals (three forms whose
// meaning follows the mode of that launch) to what this launch does.
//
// On the complex64 path the solve runs in rounds, entirely on the device: a
// round iterates until its recurrence residual has dropped by round_tol (or
// reached eps ||v||), or until it stalls (no halving of its best residual for
// a number of iterations set by stall_min and stall_mult); the lane then
// spends one launch forming the FP64 residual of its FP64 iterate (RR).  If
// that meets eps ||v|| the lane is done; if the round failed to halve it,
// COCG has met a near-breakdown of its bilinear form at that residual
// (r^T D^-1 r small against ||r||^2 / |D|) and restarting from it would meet
// it again, so one damped Jacobi step on the iterate (KX) and a new FP64
// residual come first; otherwise the next launch (RW) forms w = A D^-1 r and
// the new round's forms, and the round starts.  Lanes go through rounds
// independently.  On the FP64 path the recurrence residual is final.
__device__ __forceinline__ void cg_advance(CgScal& s, const CgCfg& cfg, c128 tg, c128 td, double trr) {
  const double eps = cfg.eps;
  if (s.done) return;
  switch (s.mode) {
    case CG_FRESH:
      s.vnorm = sqrt(trr);
      s.its = 0;
      cg_round_start(s, cfg, tg, td, trr);
      return;
    case CG_RW:
      cg_round_start(s, cfg, tg, td, trr);
      return;
    case CG_KX:
      s.mode = CG_RR;
      return;
    case CG_RR: {
      const double rn = sqrt(trr);
      s.rnorm = rn;
      if (rn <= eps * s.vnorm) {
        s.done = 1; s.conv = 1;
      } else if (s.its >= cfg.maxit || !(rn == rn)) {
        s.done = 1; s.conv = 0;
      } else if (s.kick == 0 && rn > 0.5 * s.rn0) {
        s.kick = 1;
        s.mode = CG_KX;
      } else {
        s.kick = 0;
        if (cfg.fused_start) cg_round_start(s, cfg, tg, td, trr);
        else s.mode = CG_RW;
      }
      return;
    }
    default:
      break;
  }
  s.its += 1;
  s.rnorm = sqrt(trr);
  if (s.rnorm <= s.rstop) {
    if (cfg.trust) {
      s.done = 1; s.conv = 1;
    } else {
      s.mode = CG_RR;
    }
    return;
  }
  if (s.rnorm < 0.5 * s.rbest) {
    s.rbest = s.rnorm;
    s.its_best = s.its;
  } else if (!cfg.trust && cfg.stall_min > 0 &&
             s.its - s.its_best > max(cfg.stall_min, cfg.stall_mult * (s.its_best - s.its0))) {
    s.mode = CG_RR;
    return;
  }
  c128 den{0.0, 0.0};
  c128 beta{0.0, 0.0};
  if (!is_zero(s.gamma) && !is_zero(s.alpha)) {
    beta = cdiv(tg, s.gamma);
    den = td - cdiv(beta * tg, s.alpha);
  }
  if (s.its >= cfg.maxit || !(s.rnorm == s.rnorm) || is_zero(den)) {
    if (cfg.trust || !(s.rnorm == s.rnorm)) {
      s.done = 1; s.conv = 0;
    } else {
      s.mode = CG_RR;   // judge the iterate in FP64
    }
    return;
  }
  s.beta = beta;
  s.alpha = cdiv(tg, den);
  s.gamma = tg;
}

// Inverse Jacobi diagonal 1/(diag(K) + tau diag(M)) for one inner solve, so
// the iteration multiplies instead of dividing at every stencil point.
template <typename Op, typename R>
__global__ void __launch_bounds__(BS) k_dinv(Op op, const double* __restrict__ dK, c128 tau, int n,
                                             cx<R>* __restrict__ dinv) {
  for (int c = blockIdx.x * BS + threadIdx.x; c < n; c += gridDim.x * BS) {
    const double m = op.mass(c);
    dinv[c] = cvt<R>(cdiv(c128{1.0, 0.0}, c128{dK[c] + tau.re * m, tau.im * m}));
  }
}

// Vector set of the iteration: r, w, s in two parity buffers.
template <typename R> struct CgVecs {
  cx<R>* r[2];
  cx<R>* w[2];
  cx<R>* s[2];
  cx<R>* p;
  c128* x;
};

// x = 0, p = 0, s = 0, r = v, w = A D^{-1} v; partials v^T u, w^T u, ||v||^2.
template <typename Op, typename R>
__global__ void __launch_bounds__(BS) k_cg_init(Op op, const cx<R>* __restrict__ dinv, c128 tau, int n, int lS,
                                                const cx<R>* __restrict__ v,
                                                CgVecs<R> vec,
                                                c128* __restrict__ part, CgScal* __restrict__ sc0,
                                                int* __restrict__ all_done) {
  const int S = 1 << lS;
  const int N = n << lS;
  const int rl = threadIdx.x & (S - 1);
  const cx<R> tr = cvt<R>(tau);
  auto gu = [&](int cc) { return v[(cc << lS) + rl] * dinv[cc]; };
  c128 ag{0, 0}, ad{0, 0};
  double arr = 0;
  for (int t = blockIdx.x * BS + threadIdx.x; t < N; t += gridDim.x * BS) {
    const int c = t >> lS;
    const cx<R> vv = v[t];
    const cx<R> uu = vv * dinv[c];
    const cx<R> ww = op.template apply<R>(c, tr, gu);
    vec.x[t] = c128{0.0, 0.0};
    vec.p[t] = cx<R>{0, 0};
    vec.s[0][t] = cx<R>{0, 0};
    vec.r[0][t] = vv;
    vec.w[0][t] = ww;
    ag = ag + cvt<double>(vv) * cvt<double>(uu);
    ad = ad + cvt<double>(ww) * cvt<double>(uu);
    arr += abs2(cvt<double>(vv));
  }
  c128 acc[3] = {ag, ad, {arr, 0.0}};
  block_partials<3>(acc, S, part + (size_t)blockIdx.x * 3 * S);
  if (blockIdx.x == 0) {
    if ((int)threadIdx.x < S) {
      CgScal s{};
      s.mode = CG_FRESH;
      sc0[threadIdx.x] = s;
    }
    if (threadIdx.x == 0) {
      all_done[0] = 0;
      all_done[1] = 0;
    }
  }
}

// all_done[0]: every lane of the inner solve has stopped; all_done[1]: the
// iteration launches that did work since the solve started (what the host's
// timer divides by).  Called by a launch that goes on past its prologue.
__device__ __forceinline__ void count_live(int* all_done, bool lead) {
  if (lead && threadIdx.x == 0) atomicAdd(all_done + 1, 1);
}

// Loads of one cell for the stencil iteration (issued before any arithmetic,
// with clamped neighbour indices instead of branches).
template <typename Op, typename R> struct CgCell {
  int idx[Op::NB > 0 ? Op::NB : 1];
  R fo[Op::NB > 0 ? Op::NB : 1];
  R fsum, m;
  cx<R> rq[Op::NB > 0 ? Op::NB : 1], wq[Op::NB > 0 ? Op::NB : 1], sq[Op::NB > 0 ? Op::NB : 1],
      dq[Op::NB > 0 ? Op::NB : 1];
  cx<R> di, rc, wc, sc, pc;
  c128 xc;
};

template <typename Op, typename R>
__device__ __forceinline__ void cg_load(const Op& op, const cx<R>* __restrict__ dinv, int lS, int rl, int t,
                                        const cx<R>* __restrict__ r0, const cx<R>* __restrict__ w0,
                                        const cx<R>* __restrict__ s0, const CgVecs<R>& vec, CgCell<Op, R>& L) {
  constexpr int NB = Op::NB;
  const int c = t >> lS;
  op.template stencil<R>(c, L.idx, L.fo, L.fsum);
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int k = (L.idx[q] << lS) + rl;
    L.rq[q] = r0[k];
    L.wq[q] = w0[k];
    L.sq[q] = s0[k];
    L.dq[q] = dinv[L.idx[q]];
  }
  L.di = dinv[c];
  L.rc = r0[t];
  L.wc = w0[t];
  L.sc = s0[t];
  L.pc = vec.p[t];
  L.xc = vec.x[t];
  L.m = (R)op.mass(c);
}

template <typename Op, typename R, bool NT>
__device__ __forceinline__ void cg_compute(const CgCell<Op, R>& L, int t, cx<R> al, cx<R> be, c128 al64, cx<R> tr,
                                           const CgVecs<R>& vec, cx<R>* __restrict__ r1, cx<R>* __restrict__ w1,
                                           cx<R>* __restrict__ s1, c128& ag, c128& ad, double& arr) {
  constexpr int NB = Op::NB;
  const cx<R> sn = L.wc + be * L.sc;
  const cx<R> rn = L.rc - al * sn;
  const cx<R> pn = L.rc * L.di + be * L.pc;
  const cx<R> un = rn * L.di;
  cx<R> wn = L.fsum * un + L.m * (tr * un);
#pragma unroll
  for (int q = 0; q < NB; ++q) wn = wn - L.fo[q] * ((L.rq[q] - al * (L.wq[q] + be * L.sq[q])) * L.dq[q]);
  st<NT>(vec.p + t, pn);
  st<NT>(vec.x + t, L.xc + al64 * cvt<double>(pn));
  st<NT>(r1 + t, rn);
  st<NT>(w1 + t, wn);
  st<NT>(s1 + t, sn);
  // products of the stored (rounded) values formed exactly in FP64: the
  // bilinear forms can cancel strongly, and FP32 products would then
  // dominate their error
  const c128 rd = cvt<double>(rn), ud = cvt<double>(un);
  ag = ag + rd * ud;
  ad = ad + cvt<double>(wn) * ud;
  arr += abs2(rd);
}

// One launch of the inner solve for every lane: an iteration, or a step of a
// round change on the complex64 path (see cg_advance).  Vectors alternate
// between two buffers by launch parity (par, from the host): a lane that has
// stopped leaves its vectors where they are, and a lane that starts a round
// writes r and w for it into the next buffers (its s enters multiplied by
// beta = 0 and every buffer holds finite values).  The all-done flag, the
// previous launch's partials and the lane state are loaded together and the
// flag is judged only after the sums (one memory round trip instead of two;
// when the flag is set the sums are discarded).  ONE = the launch has a single
// lane (S = 1): the lane state is then uniform and lives in scalar registers.
// MULTI = the grid is smaller than the items and threads loop over several
// cells (large problems); otherwise each thread owns one cell.  Blocks take
// tiles in XCD-aware order.
template <typename Op, typename OpD, typename R, int CGB, bool NT, bool ONE, bool MULTI>
__global__ void __launch_bounds__(CGB) k_cg_step(Op op, OpD opd, const cx<R>* __restrict__ dinv, c128 tau, int n,
                                                 int lS_, const CgCfg* __restrict__ cfgp,
                                                 const cx<R>* __restrict__ v,
                                                 const c128* __restrict__ partIn, int Gin,
                                                 const CgScal* __restrict__ scIn, CgScal* __restrict__ scOut,
                                                 CgVecs<R> vec, int par, c128* __restrict__ partOut,
                                                 int* __restrict__ all_done) {
  const CgCfg cfg = *cfgp;
  const int lS = ONE ? 0 : lS_;
  const int S = 1 << lS;
  const int rl = ONE ? 0 : (int)threadIdx.x & (S - 1);
  const int flag = *all_done;
  constexpr int KMAX = 4;
  PartLoad<3, KMAX> PL;
  part_load<3, KMAX, CGB>(partIn, Gin, S, PL);
  CgScal s = scIn[rl];
  const int N = n << lS;
  const cx<R>* __restrict__ r0 = vec.r[par];
  const cx<R>* __restrict__ w0 = vec.w[par];
  const cx<R>* __restrict__ s0 = vec.s[par];
  cx<R>* __restrict__ r1 = vec.r[par ^ 1];
  cx<R>* __restrict__ w1 = vec.w[par ^ 1];
  cx<R>* __restrict__ s1 = vec.s[par ^ 1];
  const int t0 = xcd_tile(blockIdx.x, gridDim.x) * CGB + threadIdx.x;
  // the thread's cells: one, or a grid-stride loop when the grid is capped
  auto for_cells = [&](auto&& f) {
    if constexpr (MULTI) {
      const SlabWalk sw(op, N, lS, CGB);
      for (long q = sw.first(); q < sw.end; q += sw.step) f((sw.cell(q) << lS) + rl);
    } else {
      if (t0 < N) f(t0);
    }
  };
  c128 tot[3];
  part_sum<3, KMAX, CGB>(partIn, Gin, S, PL, tot);
  if (flag) {
    if (blockIdx.x == 0 && (int)threadIdx.x < S) scOut[threadIdx.x] = s;
    return;
  }
  cg_advance(s, cfg, tot[0], tot[1], tot[2].re);
  const bool any_open = __any(!s.done);
  if (blockIdx.x == 0 && (int)threadIdx.x < S) scOut[threadIdx.x] = s;
  if (!any_open) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *all_done = 1;
    return;
  }
  count_live(all_done, blockIdx.x == 0);
  c128 ag{0, 0}, ad{0, 0};
  double arr = 0;
  if (!s.done) {
    const cx<R> tr = cvt<R>(tau);
    if (s.mode == CG_ITER) {
      const cx<R> al = cvt<R>(s.alpha), be = cvt<R>(s.beta);
      const c128 al64 = s.alpha;
      if constexpr (Op::NB > 0) {
        for_cells([&](int t) {
          CgCell<Op, R> L;
          cg_load<Op, R>(op, dinv, lS, rl, t, r0, w0, s0, vec, L);
          cg_compute<Op, R, NT>(L, t, al, be, al64, tr, vec, r1, w1, s1, ag, ad, arr);
        });
      } else {
        // general sparse K: u' formed on the fly at every column of the row
        auto gu = [&](int cc) {
          const int k = (cc << lS) + rl;
          return (r0[k] - al * (w0[k] + be * s0[k])) * dinv[cc];
        };
        for_cells([&](int t) {
          const int c = t >> lS;
          const cx<R> di = dinv[c];
          const cx<R> rc = r0[t];
          const cx<R> sn = w0[t] + be * s0[t];
          const cx<R> rn = rc - al * sn;
          const cx<R> pn = rc * di + be * vec.p[t];
          vec.p[t] = pn;
          vec.x[t] = vec.x[t] + al64 * cvt<double>(pn);
          const cx<R> un = rn * di;
          const cx<R> wn = op.template apply<R>(c, tr, gu);
          r1[t] = rn;
          w1[t] = wn;
          s1[t] = sn;
          const c128 rd = cvt<double>(rn), ud = cvt<double>(un);
          ag = ag + rd * ud;
          ad = ad + cvt<double>(wn) * ud;
          arr += abs2(rd);
        });
      }
    } else if (s.mode == CG_RR) {
      // FP64 residual of the FP64 iterate, stored rounded; its FP64 norm
      const c128* __restrict__ x = vec.x;
      auto gx = [&](int cc) { return x[(cc << lS) + rl]; };
      for_cells([&](int t) {
        const int c = t >> lS;
        const c128 res = cvt<double>(v[t]) - opd.template apply<double>(c, tau, gx);
        r1[t] = cvt<R>(res);
        arr += abs2(res);
      });
    } else if (s.mode == CG_KX) {
      // damped Jacobi step on the iterate from the residual just formed; the
      // diagonal dominance of K + tau M keeps it from growing the residual
      for_cells([&](int t) {
        const int c = t >> lS;
        vec.x[t] = vec.x[t] + 0.5 * (cvt<double>(dinv[c]) * cvt<double>(r0[t]));
      });
    } else {
      // CG_RW: w = A D^-1 r of the residual just formed, carried into the
      // next buffers with r (s cleared), and the round's first forms
      auto gu = [&](int cc) { return r0[(cc << lS) + rl] * dinv[cc]; };
      for_cells([&](int t) {
        const int c = t >> lS;
        const cx<R> rc = r0[t];
        const cx<R> uu = rc * dinv[c];
        const cx<R> ww = op.template apply<R>(c, tr, gu);
        r1[t] = rc;
        w1[t] = ww;
        s1[t] = cx<R>{0, 0};
        const c128 rd = cvt<double>(rc), ud = cvt<double>(uu);
        ag = ag + rd * ud;
        ad = ad + cvt<double>(ww) * ud;
        arr += abs2(rd);
      });
    }
  }
  c128 acc[3] = {ag, ad, {arr, 0.0}};
  block_partials<3, CGB>(acc, S, partOut + (size_t)blockIdx.x * 3 * S);
}


// After the inner solve: true inner residual p = v - (K + tau M) z in FP64
// (its norm enters the bound of eq. resdiff) and the mass product w = M z
// (Algorithm 3).  Partials [G][2][S]: ||p||^2, ||M z||^2.
template <typename OpD, typename R>
__global__ void __launch_bounds__(BS) k_cocg_finish(OpD opd, c128 tau, long n, int S,
                                                    const cx<R>* __restrict__ v, const c128* __restrict__ z,
                                                    cx<R>* __restrict__ w, c128* __restrict__ part) {
  const long N = n * S;
  const int rl = threadIdx.x & (S - 1);
  auto g = [&](long cc) { return z[cc * S + rl]; };
  double a0 = 0.0, a1 = 0.0;
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < N; t += (long)gridDim.x * BS) {
    const long c = t / S;
    const c128 pv = cvt<double>(v[t]) - opd.template apply<double>(c, tau, g);
    const c128 ww = opd.mass(c) * z[t];
    if (w) w[t] = cvt<R>(ww);
    a0 += abs2(pv);
    a1 += abs2(ww);
  }
  c128 acc[2] = {{a0, 0.0}, {a1, 0.0}};
  block_partials<2>(acc, S, part + (size_t)blockIdx.x * 2 * S);
}

// Real diagonal of K from the operator (diagonal of the Jacobi preconditioner
// D = diag(K) + tau diag(M)), in FP64 and FP32.
template <typename OpD>
__global__ void __launch_bounds__(BS) k_diag(OpD opd, long n, double* __restrict__ d64, float* __restrict__ d32) {
  for (long c = blockIdx.x * (long)BS + threadIdx.x; c < n; c += (long)gridDim.x * BS) {
    const double d = opd.diagK(c);
    d64[c] = d;
    d32[c] = (float)d;
  }
}

// -------------------------------------------------- Gram-Schmidt (CGS2) ----
// Partial products v_i^H w over a block of items for columns i < kc.  Wave w
// of the block handles columns w, w+NWAVE, ...; each lane runs over the items
// at stride 64 (its rhs lane stays fixed), then a wave tree per lane group.
template <typename R>
__global__ void __launch_bounds__(BS) k_gs_dot(long N, int S, int kc, const cx<R>* __restrict__ V,
                                               size_t cstride, const cx<R>* __restrict__ w,
                                               c128* __restrict__ part, long ipb) {
  const long start = blockIdx.x * ipb;
  const long end = start + ipb < N ? start + ipb : N;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  for (int i = wv; i < kc; i += NWAVE) {
    const cx<R>* Vi = V + (size_t)i * cstride;
    // exact products of the stored values, FP64 sums (the projections in the
    // second pass are small differences of large terms)
    c128 a{0, 0};
#pragma unroll 8
    for (long t = start + lane; t < end; t += WAVE) a = a + cdot(cvt<double>(Vi[t]), cvt<double>(w[t]));
    c128 s = wave_sum_strided(a, S);
    if (lane < S) part[((size_t)blockIdx.x * kc + i) * S + lane] = s;
  }
}

// One block per (column i, lane r): sum the partials over G blocks.
__global__ void __launch_bounds__(BS) k_gs_reduce(const c128* __restrict__ part, int G, int kc, int S,
                                                  c128* __restrict__ main_out, c128* __restrict__ aux_out,
                                                  int accumulate) {
  const int i = blockIdx.x / S, r = blockIdx.x % S;
  c128 a{0.0, 0.0};
  for (int b = threadIdx.x; b < G; b += BS) a = a + part[((size_t)b * kc + i) * S + r];
  a = block_sum_all(a);
  if (threadIdx.x == 0) {
    aux_out[i * S + r] = a;
    main_out[i * S + r] = accumulate ? main_out[i * S + r] + a : a;
  }
}

// w -= sum_i h_i v_i for each item; optionally partials of the FP64 norm
// ||w||^2 per lane (k_final_sqrt turns them into h_{k+1,k}).
constexpr int GSQ = 4;
template <typename R>
__global__ void __launch_bounds__(BS) k_gs_update(long N, int S, int kc, const cx<R>* __restrict__ V,
                                                  size_t cstride, const c128* __restrict__ h,
                                                  cx<R>* __restrict__ w, int with_norm,
                                                  c128* __restrict__ part) {
  const int r = threadIdx.x & (S - 1);
  const long base = (long)blockIdx.x * BS * GSQ + threadIdx.x;
  // the update runs in FP64 and w is rounded to its storage precision once:
  // after the projection w is a small difference of large terms
  c128 wq[GSQ];
#pragma unroll
  for (int qq = 0; qq < GSQ; ++qq) {
    const long t = base + (long)qq * BS;
    wq[qq] = t < N ? cvt<double>(w[t]) : c128{0, 0};
  }
  for (int i = 0; i < kc; ++i) {
    const c128 hi = h[i * S + r];
    const cx<R>* Vi = V + (size_t)i * cstride;
#pragma unroll
    for (int qq = 0; qq < GSQ; ++qq) {
      const long t = base + (long)qq * BS;
      if (t < N) wq[qq] = wq[qq] - hi * cvt<double>(Vi[t]);
    }
  }
  double a = 0.0;
#pragma unroll
  for (int qq = 0; qq < GSQ; ++qq) {
    const long t = base + (long)qq * BS;
    if (t < N) {
      const cx<R> ws = cvt<R>(wq[qq]);
      w[t] = ws;
      a += abs2(cvt<double>(ws));
    }
  }
  if (!with_norm) return;
  c128 acc[1] = {{a, 0.0}};
  block_partials<1>(acc, S, part + (size_t)blockIdx.x * S);
}

// v_{k+1} = w / h_{k+1,k}; lanes that broke down (h <= 1e-14 ||M z||, section
// 3) or carry no rhs get a zero column.
template <typename R>
__global__ void __launch_bounds__(BS) k_scale_col(long N, int S, const cx<R>* __restrict__ w,
                                                  const double* __restrict__ hn, const double* __restrict__ mz,
                                                  cx<R>* __restrict__ vout) {
  const int r = threadIdx.x & (S - 1);
  const double h = hn[r];
  const bool ok = h > 1e-14 * mz[r] && h > 0.0;
  const R inv = ok ? (R)(1.0 / h) : (R)0;
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < N; t += (long)gridDim.x * BS) vout[t] = inv * w[t];
}

// out = sum_i coef[i][r] V_i (restart start vector V_{m+1} z_s / ||z_s||).
template <typename R>
__global__ void __launch_bounds__(BS) k_basis_combine(long N, int S, int kc, const cx<R>* __restrict__ V,
                                                      size_t cstride, const c128* __restrict__ coef,
                                                      cx<R>* __restrict__ out) {
  const int r = threadIdx.x & (S - 1);
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < N; t += (long)gridDim.x * BS) {
    c128 a{0.0, 0.0};
    for (int i = 0; i < kc; ++i) a = a + coef[i * S + r] * cvt<double>(V[(size_t)i * cstride + t]);
    out[t] = cvt<R>(a);
  }
}

// -------------------------------------------- per-shift least squares ------
// One thread per (shift j, rhs r) lane, FP64 throughout.  Column k of
// Hbar(sigma_j;T) = [I;0] + Hbar (sigma_j I - T) (eq. shiftedarnoldimod) is
// rotated by the stored Givens rotations, a new rotation zeroes its
// subdiagonal, |g_{k+1}| is the quasi-residual ||beta e_1 - Hbar(sigma;T) y||,
// y comes from the triangular factor, and eq. trueresidual's bound
// rho + sum |y_i| ||p_i|| decides whether the lane freezes.
//
// FOM variant (Algorithm 4, FOM): y solves the square system H_k(sigma;T) y =
// beta e_1.  The rotations that zero the earlier subdiagonals turn it into the
// triangular factor with the last diagonal and right-hand side taken before
// the new rotation, so the same stored factor serves both variants.  The FOM
// residual is -hbar_{k+1,k}(sigma) y_k v_{k+1} (the closed form in the proof of
// Prop. 2); its coefficient is kept for the restart.  An exactly singular
// H_k(sigma;T) has no FOM iterate: the step reports an infinite quasi-residual
// and keeps the least-squares y.
struct LaneState {
  c128 beta;        // current start coefficient beta_j of this cycle
  c128 fres;        // FOM: residual coefficient along the next basis vector
  double gap_prev;  // inexact-inner term accumulated over earlier cycles
  double rho;       // quasi-residual at the last step
  double bound;     // bound of eq. trueresidual at the last step
  int status;       // SHK_* per-shift status
  int active;       // 1 while the lane still takes outer steps
  int kfz;          // columns of the cycle used by y
  int cycle_fz;     // cycle in which the lane froze (-1 while active)
  int outer_its;
  int restarts;
  int pad0, pad1;
};

struct GivensArgs {
  int L, S, m, k, cycle, kglob;
  int fom;               // 1: FOM projected problem, 0: least squares (GMRES)
  double tol, inexact_ratio, breakdown_rel;
  const c128* Hk;        // column k: Hk[i*S + r], i <= k+1 (k+1 = subdiagonal)
  const double* hn;      // h_{k+1,k} per lane r
  const double* mz;      // ||M z_k|| per lane r
  const double* pn;      // ||p_i|| at pn[i*S + r], i <= k
  const double* beta0;   // ||b_r||
  const c128* sigma;     // shifts
  const c128* taus;      // tau of every column of this cycle
  LaneState* ls;
  double* rc; c128* rs; c128* g; c128* Rp; c128* Yb;
};

__device__ __forceinline__ void givens_make(c128 a, c128 b, double& c, c128& s, c128& rr) {
  // [c s; -conj(s) c] [a; b] = [rr; 0], c real >= 0
  const double na = hypot(a.re, a.im), nb = hypot(b.re, b.im);
  if (nb == 0.0) { c = 1.0; s = c128{0.0, 0.0}; rr = a; return; }
  if (na == 0.0) { c = 0.0; s = c128{b.re / nb, -b.im / nb}; rr = c128{nb, 0.0}; return; }
  const double nu = hypot(na, nb);
  c = na / nu;
  const c128 ph{a.re / na, a.im / na};     // a / |a|
  s = (1.0 / nu) * (ph * conj(b));
  rr = nu * ph;
}

__device__ __forceinline__ size_t tri(int i, int k) { return (size_t)k * (k + 1) / 2 + i; }

// y = R^{-1} g over the first kc columns into y[i * ys]; returns the inexact
// term sum |y_i| ||p_i||.  The R loads do not depend on the running sum, so
// several are in flight at once.  With `last`, the last row uses the diagonal
// last[0] and right-hand side last[1] instead of the stored ones.
__device__ inline double backsolve(const GivensArgs& a, int lane, int r, int kc, const c128* gv, size_t gstride,
                                  c128* y, int ys, const c128* last = nullptr) {
  const int L = a.L;
  double gap = 0.0;
  int i0 = kc - 1;
  if (last) {
    const c128 yi = cdiv(last[1], last[0]);
    y[i0 * ys] = yi;
    gap += hypot(yi.re, yi.im) * a.pn[i0 * a.S + r];
    --i0;
  }
  for (int i = i0; i >= 0; --i) {
    c128 acc = gv[(size_t)i * gstride];
#pragma unroll 4
    for (int l = i + 1; l < kc; ++l) acc = acc - a.Rp[tri(i, l) * L + lane] * y[l * ys];
    const c128 yi = cdiv(acc, a.Rp[tri(i, i) * L + lane]);
    y[i * ys] = yi;
    gap += hypot(yi.re, yi.im) * a.pn[i * a.S + r];
  }
  return gap;
}

// Thread per lane (bases longer than GIVW_MAXM; shorter ones use
// k_givens_wave below).  y goes straight to the lane's row of Yb.
__global__ void __launch_bounds__(BS) k_givens(GivensArgs a) {
  const int lane = blockIdx.x * blockDim.x + threadIdx.x;
  if (lane >= a.L) return;
  LaneState st = a.ls[lane];
  if (!st.active) return;
  const int S = a.S, r = lane % S, j = lane / S, k = a.k, L = a.L;
  const c128 d = a.sigma[j] - a.taus[k];
  const double hn = a.hn[r];
  const bool broke = !(hn > a.breakdown_rel * a.mz[r]);
  // rotate the new column
  c128 carry = d * a.Hk[0 * S + r];
  if (k == 0) carry.re += 1.0;
#pragma unroll 4
  for (int i = 0; i < k; ++i) {
    c128 nxt = d * a.Hk[(i + 1) * S + r];
    if (i + 1 == k) nxt.re += 1.0;
    const double c = a.rc[(size_t)i * L + lane];
    const c128 s = a.rs[(size_t)i * L + lane];
    a.Rp[tri(i, k) * L + lane] = c * carry + s * nxt;
    carry = (-1.0) * (conj(s) * carry) + c * nxt;
  }
  const c128 sub = broke ? c128{0.0, 0.0} : hn * d;
  double c;
  c128 s, rr;
  givens_make(carry, sub, c, s, rr);
  a.Rp[tri(k, k) * L + lane] = rr;
  a.rc[(size_t)k * L + lane] = c;
  a.rs[(size_t)k * L + lane] = s;
  const c128 gk = a.g[(size_t)k * L + lane];
  a.g[(size_t)k * L + lane] = c * gk;
  const c128 gk1 = (-1.0) * (conj(s) * gk);
  a.g[(size_t)(k + 1) * L + lane] = gk1;
  double rho = broke ? 0.0 : hypot(gk1.re, gk1.im);
  c128* yrow = a.Yb + (size_t)lane * a.m;
  c128* y = yrow;
  const int ys = 1;
  // FOM: the square system's factor ends in the unrotated pivot; after a
  // breakdown (zero subdiagonal) the two variants coincide
  const bool fom = a.fom && !broke;
  const bool singular = fom && carry.re == 0.0 && carry.im == 0.0;
  const c128 last[2] = {carry, gk};
  const double gap = backsolve(a, lane, r, k + 1, a.g + lane, (size_t)L, y, ys, fom && !singular ? last : nullptr);
  st.fres = c128{0.0, 0.0};
  if (fom) {
    if (singular) {
      rho = __builtin_inf();
    } else {
      st.fres = (-1.0) * (sub * y[k * ys]);
      rho = hypot(st.fres.re, st.fres.im);
    }
  }
  for (int i = k + 1; i < a.m; ++i) yrow[i] = c128{0.0, 0.0};
  const double bound = rho + st.gap_prev + gap;
  const double b0 = a.beta0[r];
  st.rho = rho;
  st.bound = bound;
  st.kfz = k + 1;
  st.outer_its = a.kglob + 1;
  st.restarts = a.cycle;
  int done = -1;
  if (broke) done = bound <= a.tol * b0 ? SHK_BREAKDOWN_EXACT : SHK_INNER_LIMITED;
  else if (bound <= a.tol * b0) done = SHK_CONVERGED;
  else if (rho <= a.inexact_ratio * (st.gap_prev + gap)) done = SHK_INNER_LIMITED;
  if (done >= 0) {
    st.status = done;
    st.active = 0;
    st.cycle_fz = a.cycle;
  }
  a.ls[lane] = st;
}

// Wave per (shift, rhs) lane, bases up to GIVW_MAXM columns (launch: one
// 64-thread block per lane, givens_wave_lds(m) bytes of LDS).  The lane's
// triangular factor, rotations and the new Hessenberg column are staged in LDS
// with independent loads; thread 0 rotates the new column (a serial chain of
// k rotations read from LDS); the back substitution then runs by columns with
// thread t owning row t: y_i = acc_i / R_ii on thread i, broadcast by readlane,
// and every row above subtracts R_ti y_i.  The inexact term sum |y_i| ||p_i||
// is a wave sum.  Same arithmetic as k_givens up to the order of the
// subtractions and of the sum.
constexpr int GIVW_MAXM = 64;

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__global__ void __launch_bounds__(64) k_givens_wave(GivensArgs a) {
  extern __shared__ __align__(16) char gw_lds[];
  __shared__ c128 last_rhs;
  const int m = a.m, k = a.k, S = a.S, L = a.L;
  c128* R = reinterpret_cast<c128*>(gw_lds);   // tri(i, l), l <= k
  c128* rs = R + (size_t)m * (m + 1) / 2;       // rotations 0..k-1
  c128* hk = rs + m;                            // column k of Hbar, k + 2 entries
  double* rc = reinterpret_cast<double*>(hk + m + 2);
  const int lane = blockIdx.x;
  const int t = threadIdx.x;
  LaneState st = a.ls[lane];
  if (!st.active) return;                       // uniform over the block
  const int r = lane % S, j = lane / S;
  const int nold = k * (k + 1) / 2;
  for (int e = t; e < nold; e += 64) R[e] = a.Rp[(size_t)e * L + lane];
  for (int e = t; e < k; e += 64) {
    rc[e] = a.rc[(size_t)e * L + lane];
    rs[e] = a.rs[(size_t)e * L + lane];
  }
  for (int e = t; e <= k + 1; e += 64) hk[e] = a.Hk[e * S + r];
  const c128 g_own = t < k ? a.g[(size_t)t * L + lane] : c128{0.0, 0.0};
  const c128 d = a.sigma[j] - a.taus[k];
  const double hn = a.hn[r];
  const bool broke = !(hn > a.breakdown_rel * a.mz[r]);
  const c128 sub = broke ? c128{0.0, 0.0} : hn * d;
  const bool fom = a.fom && !broke;
  __syncthreads();
  // thread 0: rotate the new column by the stored rotations, make the new one
  double c = 1.0;
  c128 s{0.0, 0.0}, carry{0.0, 0.0}, gk1{0.0, 0.0};
  if (t == 0) {
    carry = d * hk[0];
    if (k == 0) carry.re += 1.0;
    for (int i = 0; i < k; ++i) {
      c128 nxt = d * hk[i + 1];
      if (i + 1 == k) nxt.re += 1.0;
      const double ci = rc[i];
      const c128 si = rs[i];
      const c128 v = ci * carry + si * nxt;
      R[tri(i, k)] = v;
      a.Rp[tri(i, k) * L + lane] = v;
      carry = (-1.0) * (conj(si) * carry) + ci * nxt;
    }
    c128 rr;
    givens_make(carry, sub, c, s, rr);
    a.Rp[tri(k, k) * L + lane] = rr;
    a.rc[(size_t)k * L + lane] = c;
    a.rs[(size_t)k * L + lane] = s;
    const c128 gk = a.g[(size_t)k * L + lane];
    a.g[(size_t)k * L + lane] = c * gk;
    gk1 = (-1.0) * (conj(s) * gk);
    a.g[(size_t)(k + 1) * L + lane] = gk1;
    // FOM: the square system's factor ends in the unrotated pivot and
    // right-hand side (an exactly singular one keeps the least-squares y)
    const bool use_fom = fom && !(carry.re == 0.0 && carry.im == 0.0);
    R[tri(k, k)] = use_fom ? carry : rr;
    last_rhs = use_fom ? gk : c * gk;
  }
  __syncthreads();
  c128 acc = t < k ? g_own : (t == k ? last_rhs : c128{0.0, 0.0});
  c128 yown{0.0, 0.0};
  for (int i = k; i >= 0; --i) {
    if (t == i) yown = cdiv(acc, R[tri(i, i)]);
    const c128 yi{readlane_f64(yown.re, i), readlane_f64(yown.im, i)};
    if (t < i) acc = acc - R[tri(t, i)] * yi;
  }
  const bool owned = t <= k;
  double gp = owned ? hypot(yown.re, yown.im) * a.pn[t * S + r] : 0.0;
  const double gap = wave_sum_strided(gp, 1);
  if (t < m) a.Yb[(size_t)lane * m + t] = owned ? yown : c128{0.0, 0.0};
  const c128 yk{readlane_f64(yown.re, k), readlane_f64(yown.im, k)};
  if (t != 0) return;
  double rho = broke ? 0.0 : hypot(gk1.re, gk1.im);
  st.fres = c128{0.0, 0.0};
  if (fom) {
    if (carry.re == 0.0 && carry.im == 0.0) {
      rho = __builtin_inf();
    } else {
      st.fres = (-1.0) * (sub * yk);
      rho = hypot(st.fres.re, st.fres.im);
    }
  }
  const double bound = rho + st.gap_prev + gap;
  const double b0 = a.beta0[r];
  st.rho = rho;
  st.bound = bound;
  st.kfz = k + 1;
  st.outer_its = a.kglob + 1;
  st.restarts = a.cycle;
  int done = -1;
  if (broke) done = bound <= a.tol * b0 ? SHK_BREAKDOWN_EXACT : SHK_INNER_LIMITED;
  else if (bound <= a.tol * b0) done = SHK_CONVERGED;
  else if (rho <= a.inexact_ratio * (st.gap_prev + gap)) done = SHK_INNER_LIMITED;
  if (done >= 0) {
    st.status = done;
    st.active = 0;
    st.cycle_fz = a.cycle;
  }
  a.ls[lane] = st;
}

// Lane initialisation for a solve: beta_j = ||b_r||, g = beta e_1.
__global__ void __launch_bounds__(BS) k_lanes_init(int L, int S, int s_real, const double* __restrict__ beta0,
                                                   LaneState* __restrict__ ls, c128* __restrict__ g) {
  const int lane = blockIdx.x * BS + threadIdx.x;
  if (lane >= L) return;
  const int r = lane % S;
  LaneState st{};
  const double b = beta0[r];
  st.beta = c128{b, 0.0};
  st.gap_prev = 0.0;
  st.rho = b;
  st.bound = b;
  st.cycle_fz = -1;
  st.kfz = 0;
  st.outer_its = 0;
  st.restarts = 0;
  if (r >= s_real || !(b > 0.0)) {
    st.active = 0;
    st.status = (r < s_real && !(b == b)) ? SHK_NAN : SHK_CONVERGED;
    st.cycle_fz = 0;
    st.rho = 0.0;
    st.bound = 0.0;
  } else {
    st.active = 1;
    st.status = SHK_NOT_CONVERGED;
  }
  ls[lane] = st;
  g[lane] = st.beta;
}

// Restart, seed selection (one thread per rhs lane): the active shift with the
// largest quasi-residual (ties to the lowest index); its residual in the
// (m+1)-space is z_s = Q_s [0..0, g_m]^T, built by undoing the rotations.
__global__ void k_restart_seed(int S, int nf, int m, const LaneState* __restrict__ ls,
                               const double* __restrict__ rc, const c128* __restrict__ rs,
                               const c128* __restrict__ g, int* __restrict__ seed,
                               c128* __restrict__ zs, double* __restrict__ nzs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= S) return;
  const int L = nf * S;
  int best = -1;
  double bv = -1.0;
  for (int j = 0; j < nf; ++j) {
    const LaneState& st = ls[j * S + r];
    if (st.active && st.rho > bv) { bv = st.rho; best = j; }
  }
  seed[r] = best;
  if (best < 0) { nzs[r] = 0.0; return; }
  const int lane = best * S + r;
  // z = G_0^H ... G_{m-1}^H (g_m e_m)
  for (int i = 0; i <= m; ++i) zs[i * S + r] = c128{0.0, 0.0};
  c128 b = g[(size_t)m * L + lane];
  for (int i = m - 1; i >= 0; --i) {
    const double c = rc[(size_t)i * L + lane];
    const c128 s = rs[(size_t)i * L + lane];
    // (a, b) <- (c a - s b, conj(s) a + c b) with a = 0 on entry
    zs[(i + 1) * S + r] = c * b;
    b = (-1.0) * (s * b);
  }
  zs[0 * S + r] = b;
  double nn = 0.0;
  for (int i = 0; i <= m; ++i) nn += abs2(zs[i * S + r]);
  nn = sqrt(nn);
  nzs[r] = nn;
  const double inv = nn > 0.0 ? 1.0 / nn : 0.0;
  for (int i = 0; i <= m; ++i) zs[i * S + r] = inv * zs[i * S + r];
}

// Restart, every active lane: keep its residual collinear with the seed's by
// solving [Hbar(sigma_j;T), z][y; gamma] = beta_j e_1 through its QR factors,
// with z = z_s / ||z_s|| (stored normalised); the residual is then gamma V z,
// so the next cycle starts from v_1 = V z with beta_j <- gamma (the seed keeps
// its own y and gets beta = ||z_s||); g = beta_j e_1, and the inexact term
// grows by sum |y_i| ||p_i||.
__global__ void __launch_bounds__(BS) k_restart_lanes(GivensArgs a, const int* __restrict__ seed,
                                                      const c128* __restrict__ zs, const double* __restrict__ nzs) {
  const int lane = blockIdx.x * BS + threadIdx.x;
  if (lane >= a.L) return;
  LaneState st = a.ls[lane];
  if (!st.active) return;
  const int S = a.S, r = lane % S, j = lane / S, m = a.m, L = a.L;
  c128 gamma{1.0, 0.0};
  double gap;
  if (j == seed[r]) {
    gap = 0.0;
    const c128* y = a.Yb + (size_t)lane * m;
    for (int i = 0; i < m; ++i) gap += hypot(y[i].re, y[i].im) * a.pn[i * S + r];
  } else {
    // zhat = Q_j^H z_s, streamed; first pass for its last entry
    c128 carry = zs[0 * S + r];
    for (int i = 0; i < m; ++i) {
      const double c = a.rc[(size_t)i * L + lane];
      const c128 s = a.rs[(size_t)i * L + lane];
      const c128 nx = zs[(i + 1) * S + r];
      carry = (-1.0) * (conj(s) * carry) + c * nx;
    }
    gamma = cdiv(a.g[(size_t)m * L + lane], carry);
    carry = zs[0 * S + r];
    for (int i = 0; i < m; ++i) {
      const double c = a.rc[(size_t)i * L + lane];
      const c128 s = a.rs[(size_t)i * L + lane];
      const c128 nx = zs[(i + 1) * S + r];
      const c128 zi = c * carry + s * nx;
      carry = (-1.0) * (conj(s) * carry) + c * nx;
      a.g[(size_t)i * L + lane] = a.g[(size_t)i * L + lane] - gamma * zi;
    }
    gap = backsolve(a, lane, r, m, a.g + lane, (size_t)L, a.Yb + (size_t)lane * m, 1);
  }
  st.gap_prev += gap;
  st.beta = (j == seed[r]) ? c128{nzs[r], 0.0} : gamma;
  st.cycle_fz = -1;
  a.ls[lane] = st;
  a.g[lane] = st.beta;
}

// FOM restart, every active lane: the residual beta e_1 - Hbar(sigma;T) y of
// the cycle is fres v_{m+1} already (no seed needed), so the next cycle starts
// from v_1 = v_{m+1} with beta_j <- fres, the lane's y (the last step's FOM
// solution in Yb) is assembled, and the inexact term grows by sum |y_i|
// ||p_i||.  A lane whose last projected system was singular has no collinear
// residual: it freezes NOT_CONVERGED with its least-squares y.
__global__ void __launch_bounds__(BS) k_restart_fom(GivensArgs a) {
  const int lane = blockIdx.x * BS + threadIdx.x;
  if (lane >= a.L) return;
  LaneState st = a.ls[lane];
  if (!st.active) return;
  const int r = lane % a.S;
  if (!(st.rho < __builtin_inf())) {
    st.status = SHK_NOT_CONVERGED;
    st.active = 0;
    st.cycle_fz = a.cycle;
    a.ls[lane] = st;
    return;
  }
  const c128* y = a.Yb + (size_t)lane * a.m;
  double gap = 0.0;
  for (int i = 0; i < a.m; ++i) gap += hypot(y[i].re, y[i].im) * a.pn[i * a.S + r];
  st.gap_prev += gap;
  st.beta = st.fres;
  st.cycle_fz = -1;
  a.ls[lane] = st;
  a.g[lane] = st.beta;
}

// Lanes still active when the restart budget is spent: NOT_CONVERGED, frozen.
__global__ void __launch_bounds__(BS) k_finalize_active(int L, LaneState* __restrict__ ls) {
  const int lane = blockIdx.x * BS + threadIdx.x;
  if (lane >= L) return;
  if (ls[lane].active) {
    ls[lane].active = 0;
    ls[lane].status = SHK_NOT_CONVERGED;
  }
}

// Active lanes per rhs lane r (one block; LDS integer counts).
// Running lanes per rhs, and per rhs the largest quasi-residual rho / ||b||
// among them (0 when none runs; the relaxed inner tolerance reads it).
__global__ void __launch_bounds__(BS) k_count_active(int S, int nf, const LaneState* __restrict__ ls,
                                                     const double* __restrict__ beta0, int* __restrict__ out,
                                                     double* __restrict__ qmax) {
  __shared__ int cnt[64];
  __shared__ unsigned long long qm[64];   // bit patterns of non-negative doubles order as integers
  if ((int)threadIdx.x < 64) {
    cnt[threadIdx.x] = 0;
    qm[threadIdx.x] = 0ull;
  }
  __syncthreads();
  const int L = nf * S;
  for (int lane = threadIdx.x; lane < L; lane += BS) {
    const LaneState st = ls[lane];
    if (!st.active) continue;
    const int r = lane % S;
    atomicAdd(&cnt[r], 1);
    const double q = beta0[r] > 0.0 ? st.rho / beta0[r] : 0.0;
    if (q > 0.0 && q < 1e300) atomicMax(&qm[r], (unsigned long long)__double_as_longlong(q));
  }
  __syncthreads();
  if ((int)threadIdx.x < S) {
    out[threadIdx.x] = cnt[threadIdx.x];
    qmax[threadIdx.x] = __longlong_as_double((long long)qm[threadIdx.x]);
  }
}

// Per-lane multiplier of the assembly: lanes still active at the end of the
// cycle or frozen during it contribute Z y scaled by extra[lane] (1 or the
// refinement coefficient gamma_j), the others nothing.
__global__ void __launch_bounds__(BS) k_asm_scale(int L, int cycle, const LaneState* __restrict__ ls,
                                                  const c128* __restrict__ extra, c128* __restrict__ out) {
  const int lane = blockIdx.x * BS + threadIdx.x;
  if (lane >= L) return;
  const LaneState st = ls[lane];
  const bool use = st.active || st.cycle_fz == cycle;
  out[lane] = use ? (extra ? extra[lane] : c128{1.0, 0.0}) : c128{0.0, 0.0};
}

// ---------------------------------------------------------- output modes ---
// Factored output of one assembly (x = Z y, Algorithm 4): the kc basis vectors
// of the cycle (FP64 basis Z, lane-interleaved) appended as columns koff..
// of fz (n x kcap per rhs) and the coefficients, scaled per (shift, rhs) as
// the assembly scales them, into rows koff.. of fy (kcap x nf per rhs).
__global__ void __launch_bounds__(BS) k_factored_out(long n, int S, int s_real, int nf, int kc, int m,
                                                     const c128* __restrict__ Z, size_t cstride,
                                                     const c128* __restrict__ Yb, const c128* __restrict__ ascale,
                                                     c128* __restrict__ fz, c128* __restrict__ fy, int kcap,
                                                     int koff) {
  const long tz = n * kc * s_real, ty = (long)kc * nf * s_real;
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < tz + ty; t += (long)gridDim.x * BS) {
    if (t < tz) {
      const long c = t % n, rest = t / n;
      const int i = (int)(rest % kc), r = (int)(rest / kc);
      fz[c + n * ((long)koff + i + (long)kcap * r)] = Z[(size_t)i * cstride + c * S + r];
    } else {
      const long u = t - tz;
      const int i = (int)(u % kc);
      const long rest = u / kc;
      const int j = (int)(rest % nf), r = (int)(rest / nf);
      fy[(koff + i) + (long)kcap * (j + (long)nf * r)] =
          ascale[(size_t)j * S + r] * Yb[((size_t)j * S + r) * m + i];
    }
  }
}

// Solution rows at selected cells: out[q + nr (j + nf r)] = X[rows[q] + n (j + nf r)].
__global__ void __launch_bounds__(BS) k_gather_rows(const c128* __restrict__ X, long n, long cols,
                                                    const long long* __restrict__ rows, int nr,
                                                    c128* __restrict__ out) {
  const long total = (long)nr * cols;
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < total; t += (long)gridDim.x * BS) {
    const long q = t % nr, col = t / nr;
    out[t] = X[rows[q] + n * col];
  }
}

// ------------------------------------------------------------ assembly -----
// X[:, j, r] (+)= scale_j * Z_r y_{j,r} (Algorithm 4, x = Z y), FP64
// accumulation.  Thread per item (cell, lane), JT shifts per block row.
constexpr int JT = 16;
template <typename R>
__global__ void __launch_bounds__(BS) k_assemble(long n, int S, int s_real, int nf, int kc, int m,
                                                 const cx<R>* __restrict__ Z, size_t cstride,
                                                 const c128* __restrict__ Yb, const c128* __restrict__ ascale,
                                                 c128* __restrict__ X, int accumulate) {
  const long N = n * S;
  const int j0 = blockIdx.y * JT;
  const int r = threadIdx.x & (S - 1);
  if (r >= s_real) return;
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < N; t += (long)gridDim.x * BS) {
    const long c = t / S;
    c128 acc[JT];
#pragma unroll
    for (int q = 0; q < JT; ++q) acc[q] = c128{0.0, 0.0};
    for (int i = 0; i < kc; ++i) {
      const c128 z = cvt<double>(Z[(size_t)i * cstride + t]);
#pragma unroll
      for (int q = 0; q < JT; ++q) {
        const int j = j0 + q < nf ? j0 + q : nf - 1;
        acc[q] = acc[q] + z * Yb[((size_t)j * S + r) * m + i];
      }
    }
#pragma unroll
    for (int q = 0; q < JT; ++q) {
      const int j = j0 + q;
      if (j < nf) {
        const c128 v = ascale[(size_t)j * S + r] * acc[q];
        c128* dst = X + c + n * ((long)j + (long)nf * r);
        *dst = accumulate ? *dst + v : v;
      }
    }
  }
}

// Y transposed for the product when it is read straight from memory with
// several lanes: Yt[(j m + i) S + r] = Yb[(j S + r) m + i] for i < kc, so the
// lanes of one (shift, column) are contiguous.
__global__ void __launch_bounds__(BS) k_y_transpose(int S, int nf, int kc, int m, const c128* __restrict__ Yb,
                                                    c128* __restrict__ Yt) {
  const long total = (long)nf * kc * S;
  for (long e = blockIdx.x * (long)BS + threadIdx.x; e < total; e += (long)gridDim.x * BS) {
    const int r = (int)(e % S);
    const long ji = e / S;
    const int i = (int)(ji % kc), j = (int)(ji / kc);
    Yt[((long)j * m + i) * S + r] = Yb[((long)j * S + r) * m + i];
  }
}

// The product with Y in that layout (several lanes, Y too large for LDS),
// register-blocked: a thread takes CT consecutive cells of one lane and JQ
// shifts, so each Y entry it loads serves CT cells and its X stores are CT
// contiguous entries.  Launch grid (items, ceil(nf / JQ)); lS = log2 S.
template <typename R, int CT, int JQ>
__global__ void __launch_bounds__(BS) k_assemble_rb(long n, int S, int lS, int s_real, int nf, int kc, int m,
                                                    const cx<R>* __restrict__ Z, size_t cstride,
                                                    const c128* __restrict__ Yt, const c128* __restrict__ ascale,
                                                    c128* __restrict__ X, int accumulate) {
  const long groups = (n + CT - 1) / CT;
  const long T = groups << lS;
  const int j0 = blockIdx.y * JQ;
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < T; t += (long)gridDim.x * BS) {
    const int r = (int)(t & (S - 1));
    if (r >= s_real) continue;
    const long c0 = (t >> lS) * CT;
    c128 acc[CT][JQ];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int q = 0; q < JQ; ++q) acc[ct][q] = c128{0.0, 0.0};
    for (int i = 0; i < kc; ++i) {
      c128 z[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        z[ct] = c0 + ct < n ? cvt<double>(Z[(size_t)i * cstride + (size_t)(c0 + ct) * S + r]) : c128{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < JQ; ++q) {
        const int j = j0 + q < nf ? j0 + q : nf - 1;
        const c128 y = Yt[((size_t)j * m + i) * S + r];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ct][q] = acc[ct][q] + z[ct] * y;
      }
    }
#pragma unroll
    for (int q = 0; q < JQ; ++q) {
      const int j = j0 + q;
      if (j >= nf) break;
      const c128 sc = ascale[(size_t)j * S + r];
      c128* col = X + n * ((long)j + (long)nf * r);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        if (c0 + ct < n) {
          const c128 v = sc * acc[ct][q];
          col[c0 + ct] = accumulate ? col[c0 + ct] + v : v;
        }
      }
    }
  }
}

// The same product with the block's JT columns of Y (every rhs lane, kc rows)
// staged once in LDS at ys[(i JT + q) S + lane] instead of being reloaded for
// every item; each thread accumulates two items, t and t + BS, per LDS read.
// Needs kc * JT * S * 16 bytes of LDS (the launcher keeps it within 64 KB).
// Same FP64 accumulation order as k_assemble.
template <typename R>
__global__ void __launch_bounds__(BS) k_assemble_lds(long n, int S, int s_real, int nf, int kc, int m,
                                                     const cx<R>* __restrict__ Z, size_t cstride,
                                                     const c128* __restrict__ Yb, const c128* __restrict__ ascale,
                                                     c128* __restrict__ X, int accumulate) {
  extern __shared__ __align__(16) char asm_lds[];
  c128* ys = reinterpret_cast<c128*>(asm_lds);
  const long N = n * S;
  const int j0 = blockIdx.y * JT;
  const int tot = kc * JT * S;
  for (int e = threadIdx.x; e < tot; e += BS) {
    const int rr = e % S, q = (e / S) % JT, i = e / (S * JT);
    const int j = j0 + q < nf ? j0 + q : nf - 1;
    ys[e] = Yb[((size_t)j * S + rr) * m + i];
  }
  __syncthreads();
  const int r = threadIdx.x & (S - 1);
  if (r >= s_real) return;
  for (long base = (long)blockIdx.x * 2 * BS; base < N; base += (long)gridDim.x * 2 * BS) {
    const long t0 = base + threadIdx.x, t1 = t0 + BS;
    const bool h0 = t0 < N, h1 = t1 < N;
    c128 a0[JT], a1[JT];
#pragma unroll
    for (int q = 0; q < JT; ++q) a0[q] = a1[q] = c128{0.0, 0.0};
    for (int i = 0; i < kc; ++i) {
      const c128 z0 = h0 ? cvt<double>(Z[(size_t)i * cstride + t0]) : c128{0.0, 0.0};
      const c128 z1 = h1 ? cvt<double>(Z[(size_t)i * cstride + t1]) : c128{0.0, 0.0};
      const c128* yr = ys + (size_t)i * JT * S + r;
#pragma unroll
      for (int q = 0; q < JT; ++q) {
        const c128 y = yr[q * S];
        a0[q] = a0[q] + z0 * y;
        a1[q] = a1[q] + z1 * y;
      }
    }
    const long c0 = t0 / S, c1 = t1 / S;
#pragma unroll
    for (int q = 0; q < JT; ++q) {
      const int j = j0 + q;
      if (j >= nf) break;
      const c128 sc = ascale[(size_t)j * S + r];
      const long off = n * ((long)j + (long)nf * r);
      if (h0) {
        c128* d = X + c0 + off;
        const c128 v = sc * a0[q];
        *d = accumulate ? *d + v : v;
      }
      if (h1) {
        c128* d = X + c1 + off;
        const c128 v = sc * a1[q];
        *d = accumulate ? *d + v : v;
      }
    }
  }
}

// ------------------------------------------------------ true residuals -----
// Partial ||b_r - (K + sigma_j M) x_{j,r}||^2 (mode 0) or conj(rs_r)^T
// (b_r - (K + sigma_j M) x_{j,r}) (mode 1) per block; blockIdx.y = shift,
// blockIdx.z = rhs; cells over blockIdx.x in y-slabs per XCD (SlabWalk), so
// the neighbours' x comes from the XCD's own L2.
template <typename Op>
__global__ void __launch_bounds__(BS) k_resid(Op op, long n, int S, int nf, const c128* __restrict__ sigma,
                                              const c128* __restrict__ bint, const c128* __restrict__ X,
                                              const c128* __restrict__ rs, int mode, c128* __restrict__ part) {
  const int j = blockIdx.y, r = blockIdx.z;
  const c128* xj = X + n * ((long)j + (long)nf * r);
  const c128 sg = sigma[j];
  auto g = [&](long cc) { return xj[cc]; };
  c128 a{0.0, 0.0};
  const SlabWalk sw(op, n, 0, BS);
  for (long q = sw.first(); q < sw.end; q += sw.step) {
    const long c = sw.cell(q);
    const c128 res = bint[c * S + r] - op.template apply<double>(c, sg, g);
    if (mode == 0) a.re += abs2(res);
    else a = a + cdot(rs[c * S + r], res);
  }
  a = block_sum_all(a);
  if (threadIdx.x == 0) part[((size_t)r * nf + j) * gridDim.x + blockIdx.x] = a;
}

// The same for JR shifts per block (blockIdx.y = block of JR shifts): with
// several lanes b and rs are strided by S (one cache line per lane and cell),
// so each cell's b, rs, faces and mass are loaded once for JR shifts.
template <typename Op, int JR>
__global__ void __launch_bounds__(BS) k_resid_jr(Op op, long n, int S, int nf, const c128* __restrict__ sigma,
                                                 const c128* __restrict__ bint, const c128* __restrict__ X,
                                                 const c128* __restrict__ rs, int mode, c128* __restrict__ part) {
  const int j0 = blockIdx.y * JR, r = blockIdx.z;
  const int nj = nf - j0 < JR ? nf - j0 : JR;
  c128 a[JR];
#pragma unroll
  for (int q = 0; q < JR; ++q) a[q] = c128{0.0, 0.0};
  const SlabWalk sw(op, n, 0, BS);
  for (long q = sw.first(); q < sw.end; q += sw.step) {
    const long c = sw.cell(q);
    const c128 bc = bint[c * S + r];
    const c128 rc = mode == 0 ? c128{0.0, 0.0} : rs[c * S + r];
#pragma unroll
    for (int q = 0; q < JR; ++q) {
      if (q < nj) {
        const c128* xj = X + n * ((long)(j0 + q) + (long)nf * r);
        auto g = [&](long cc) { return xj[cc]; };
        const c128 res = bc - op.template apply<double>(c, sigma[j0 + q], g);
        if (mode == 0) a[q].re += abs2(res);
        else a[q] = a[q] + cdot(rc, res);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < JR; ++q) {
    const c128 t = block_sum_all(a[q]);
    if (q < nj && threadIdx.x == 0) part[((size_t)r * nf + j0 + q) * gridDim.x + blockIdx.x] = t;
  }
}

// rows partial sums -> out[row] (fixed order), one block per row.
__global__ void __launch_bounds__(BS) k_rows_reduce(const c128* __restrict__ part, int G, c128* __restrict__ out) {
  const size_t row = blockIdx.x;
  c128 a{0.0, 0.0};
  for (int b = threadIdx.x; b < G; b += BS) a = a + part[row * G + b];
  a = block_sum_all(a);
  if (threadIdx.x == 0) out[row] = a;
}

// rs[:, r] = b_r - (K + sigma_{seed_r} M) x_{seed_r, r} (refinement seed residual).
template <typename Op>
__global__ void __launch_bounds__(BS) k_resid_vec(Op op, long n, int S, int s_real, int nf,
                                                  const c128* __restrict__ sigma, const int* __restrict__ seed,
                                                  const c128* __restrict__ bint, const c128* __restrict__ X,
                                                  c128* __restrict__ rs) {
  const long N = n * S;
  const int r = threadIdx.x & (S - 1);
  const int j = r < s_real ? seed[r] : -1;
  const c128* xj = j >= 0 ? X + n * ((long)j + (long)nf * r) : nullptr;
  const c128 sg = j >= 0 ? sigma[j] : c128{0.0, 0.0};
  auto g = [&](long cc) { return xj[cc]; };
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < N; t += (long)gridDim.x * BS) {
    const long c = t / S;
    rs[t] = j >= 0 ? bint[t] - op.template apply<double>(c, sg, g) : c128{0.0, 0.0};
  }
}

}  // namespace shk
