// Geometric multigrid preconditioner for the inner COCG solves (section 4 lets
// the systems (K + tau M) z = v be solved by any inner iteration stopped at
// ||v - (K + tau M) z|| <= eps ||v||; the paper preconditions its inner solver
// with algebraic multigrid, section 6).
//
// Structured finite-volume grids only.  Level l+1 groups the cells of level l
// 2 x 2 (x 2): coarse cell (I, J[, L]) holds fine cells (2I + a, 2J + b[, 2L + c])
// that exist, down to a single cell.  Coarse operators are finite-volume
// operators of the same form: a coarse face carries half the sum of the fine
// faces it covers (this is (1/2) P^T K P for the piecewise-constant
// prolongation P, the 2h discretisation for a homogeneous field), a coarse
// cell the sum of its fine cells' mass (P^T M).  One V-cycle: one damped Jacobi
// sweep x = omega D^-1 b from x = 0, restriction of b - A x by summation (P^T),
// the coarse correction, prolongation by injection (P), one more sweep; the
// one-cell level is solved exactly.  Symmetric smoothing and R = P^T make the
// V-cycle a complex symmetric operator, as COCG needs.
//
// Kernels are launched per level down to the first level small enough for
// one workgroup's LDS; that level and all coarser ones run in a single
// workgroup.  Vectors carry S interleaved lanes like the rest of the library.
#pragma once
#include "kernels.hpp"

namespace shk {

// Grid shape of one level (cells along x, y, z; z = 1 in 2-D).
struct LevelDims {
  int nx, ny, nz;
  __host__ __device__ int n() const { return nx * ny * nz; }
  __host__ __device__ LevelDims coarse() const { return {(nx + 1) / 2, (ny + 1) / 2, nz > 1 ? (nz + 1) / 2 : 1}; }
};

// ------------------------------------------------------------------ setup --
// Coarse faces along axis a from the fine ones: face (c0, c1, c2) of the coarse
// grid (c_a in [0, nc_a], the others inside the coarse grid) covers the fine
// faces at index min(2 c_a, nf_a) along a and 2 c_b, 2 c_b + 1 (where they
// exist) along each other axis b; its value is half their sum.
__global__ void __launch_bounds__(BS) k_mg_faces(LevelDims f, LevelDims c, int axis, const double* __restrict__ Tf,
                                                 double* __restrict__ Tc, float* __restrict__ Tc32) {
  const int ex = c.nx + (axis == 0), ey = c.ny + (axis == 1), ez = c.nz + (axis == 2);
  const long total = (long)ex * ey * ez;
  const int fex = f.nx + (axis == 0), fey = f.ny + (axis == 1);
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < total; t += (long)gridDim.x * BS) {
    const int i = (int)(t % ex);
    const int j = (int)((t / ex) % ey);
    const int k = (int)(t / ((long)ex * ey));
    int lo[3] = {2 * i, 2 * j, 2 * k}, cnt[3] = {2, 2, 2};
    const int nf[3] = {f.nx, f.ny, f.nz};
    for (int b = 0; b < 3; ++b) {
      if (b == axis) {
        lo[b] = lo[b] < nf[b] ? lo[b] : nf[b];
        cnt[b] = 1;
      } else {
        cnt[b] = lo[b] + 1 < nf[b] ? 2 : 1;
      }
    }
    double s = 0.0;
    for (int dk = 0; dk < cnt[2]; ++dk)
      for (int dj = 0; dj < cnt[1]; ++dj)
        for (int di = 0; di < cnt[0]; ++di)
          s += Tf[(lo[0] + di) + (long)fex * ((lo[1] + dj) + (long)fey * (lo[2] + dk))];
    Tc[t] = 0.5 * s;
    Tc32[t] = (float)(0.5 * s);
  }
}

// Coarse mass: the sum of the fine cells' mass (mf null: uniform m0).
__global__ void __launch_bounds__(BS) k_mg_mass(LevelDims f, LevelDims c, const double* __restrict__ mf, double m0,
                                                double* __restrict__ mc) {
  for (int t = blockIdx.x * BS + threadIdx.x; t < c.n(); t += gridDim.x * BS) {
    const int I = t % c.nx, J = (t / c.nx) % c.ny, L = t / (c.nx * c.ny);
    double s = 0.0;
    for (int dk = 0; dk < 2; ++dk)
      for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
          const int x = 2 * I + di, y = 2 * J + dj, z = 2 * L + dk;
          if (x < f.nx && y < f.ny && z < f.nz) s += mf ? mf[x + f.nx * (y + f.ny * z)] : m0;
        }
    mc[t] = s;
  }
}

// Inverse diagonal of one level for the solve's tau: 1 / (diag K_l + tau M_l).
template <typename OpD, typename R>
__global__ void __launch_bounds__(BS) k_mg_dinv(OpD opd, c128 tau, int n, cx<R>* __restrict__ dinv) {
  for (int c = blockIdx.x * BS + threadIdx.x; c < n; c += gridDim.x * BS) {
    const double m = opd.mass(c);
    dinv[c] = cvt<R>(cdiv(c128{1.0, 0.0}, c128{opd.diagK(c) + tau.re * m, tau.im * m}));
  }
}

// ---------------------------------------------------------------- V-cycle --
// Downward leg, one coarse cell (cx_, cy, cz) and lane: the sum over its fine
// cells of the residual b - A x1 after the first sweep x1 = omega D^-1 b
// (x1 at the stencil neighbours formed on the fly).  gb(i), gd(i): b and
// D^-1 at fine cell i for the lane.
template <typename Op, typename R, typename GB, typename GD>
__device__ __forceinline__ cx<R> mg_down_cell(const Op& op, const LevelDims& f, int cx_, int cy, int cz, cx<R> tr,
                                              R om, GB gb, GD gd) {
  constexpr int NB = Op::NB;
  cx<R> acc{0, 0};
  for (int dk = 0; dk < (f.nz > 1 ? 2 : 1); ++dk)
    for (int dj = 0; dj < 2; ++dj)
      for (int di = 0; di < 2; ++di) {
        const int x = 2 * cx_ + di, y = 2 * cy + dj, z = 2 * cz + dk;
        if (x >= f.nx || y >= f.ny || z >= f.nz) continue;
        const int i = x + f.nx * (y + f.ny * z);
        int idx[NB];
        R fo[NB];
        R fsum;
        op.template stencil<R>(i, idx, fo, fsum);
        const cx<R> bi = gb(i);
        const cx<R> x1 = om * (gd(i) * bi);
        cx<R> ax = fsum * x1 + (R)op.mass(i) * (tr * x1);
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          const int j = idx[q];
          ax = ax - fo[q] * (om * (gd(j) * gb(j)));
        }
        acc = acc + (bi - ax);
      }
  return acc;
}

// Upward leg, one fine cell i and lane: x2 = x1 + P x_c (x1 = omega D^-1 b),
// then one sweep x = x2 + omega D^-1 (b - A x2), with x2 at the stencil
// neighbours formed on the fly; gxc(I): coarse solution at coarse cell I.
template <typename Op, typename R, typename GB, typename GD, typename GX>
__device__ __forceinline__ cx<R> mg_up_cell(const Op& op, const LevelDims& f, const LevelDims& c, int i, cx<R> tr,
                                            R om, GB gb, GD gd, GX gxc) {
  constexpr int NB = Op::NB;
  auto parent = [&](int k) {
    const int x = k % f.nx, y = (k / f.nx) % f.ny, z = k / (f.nx * f.ny);
    return (x >> 1) + c.nx * ((y >> 1) + c.ny * (z >> 1));
  };
  auto x2 = [&](int k) { return om * (gd(k) * gb(k)) + gxc(parent(k)); };
  int idx[NB];
  R fo[NB];
  R fsum;
  op.template stencil<R>(i, idx, fo, fsum);
  const cx<R> xi = x2(i);
  cx<R> ax = fsum * xi + (R)op.mass(i) * (tr * xi);
#pragma unroll
  for (int q = 0; q < NB; ++q) ax = ax - fo[q] * x2(idx[q]);
  return xi + om * (gd(i) * (gb(i) - ax));
}

// Downward leg of one level over the grid: coarse right-hand side b_c.
template <typename Op, typename R>
__global__ void __launch_bounds__(BS) k_mg_down(Op op, LevelDims f, LevelDims c, c128 tau, double omega, int lS,
                                                const cx<R>* __restrict__ b, const cx<R>* __restrict__ dinv,
                                                cx<R>* __restrict__ out, const int* __restrict__ all_done) {
  if (*all_done) return;
  const int S = 1 << lS;
  const int rl = threadIdx.x & (S - 1);
  const int Nc = c.n() << lS;
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  auto gb = [&](int i) { return b[(i << lS) + rl]; };
  auto gd = [&](int i) { return dinv[i]; };
  for (int t = blockIdx.x * BS + threadIdx.x; t < Nc; t += gridDim.x * BS) {
    const int I = t >> lS;
    out[t] = mg_down_cell<Op, R>(op, f, I % c.nx, (I / c.nx) % c.ny, I / (c.nx * c.ny), tr, om, gb, gd);
  }
}

// Upward leg of one level over the grid.
template <typename Op, typename R>
__global__ void __launch_bounds__(BS) k_mg_up(Op op, LevelDims f, LevelDims c, c128 tau, double omega, int lS,
                                              const cx<R>* __restrict__ b, const cx<R>* __restrict__ dinv,
                                              const cx<R>* __restrict__ xc, cx<R>* __restrict__ xout,
                                              const int* __restrict__ all_done) {
  if (*all_done) return;
  const int S = 1 << lS;
  const int rl = threadIdx.x & (S - 1);
  const int N = f.n() << lS;
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  auto gb = [&](int i) { return b[(i << lS) + rl]; };
  auto gd = [&](int i) { return dinv[i]; };
  auto gx = [&](int I) { return xc[(I << lS) + rl]; };
  for (int t = blockIdx.x * BS + threadIdx.x; t < N; t += gridDim.x * BS)
    xout[t] = mg_up_cell<Op, R>(op, f, c, t >> lS, tr, om, gb, gd, gx);
}

// The coarse end of the V-cycle in one workgroup: levels t..L-1 (right-hand
// side of level t from global memory, solution of level t back to it), every
// level's b and x in LDS, a barrier between legs.  Saves two launches per
// coarse level, which are all latency.
constexpr int MG_MAXL = 14;
constexpr int MG_TAIL_THREADS = 1024;
constexpr int MG_TAIL_LDS = 64 * 1024;
template <typename Op, typename R> struct MgTail {
  int T;                        // levels in the tail
  Op op[MG_MAXL];
  LevelDims dims[MG_MAXL];
  const cx<R>* dinv[MG_MAXL];
  int off[MG_MAXL];             // LDS offset of b_k; x_k follows it (n_k S each)
};
template <typename Op, typename R>
__global__ void __launch_bounds__(MG_TAIL_THREADS) k_mg_tail(MgTail<Op, R> a, c128 tau, double omega, int lS,
                                                             const cx<R>* __restrict__ btop, cx<R>* __restrict__ xtop,
                                                             const int* __restrict__ all_done) {
  if (*all_done) return;
  extern __shared__ __align__(16) char lds_raw[];
  cx<R>* sh = reinterpret_cast<cx<R>*>(lds_raw);
  const int S = 1 << lS;
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  const int nth = blockDim.x;
  const int T = a.T;
  {
    const int n0 = a.dims[0].n() << lS;
    for (int j = threadIdx.x; j < n0; j += nth) sh[a.off[0] + j] = btop[j];
  }
  __syncthreads();
  for (int k = 0; k + 1 < T; ++k) {
    const LevelDims f = a.dims[k], c = a.dims[k + 1];
    const cx<R>* bk = sh + a.off[k];
    cx<R>* bc = sh + a.off[k + 1];
    const cx<R>* dk = a.dinv[k];
    const int Nc = c.n() << lS;
    for (int j = threadIdx.x; j < Nc; j += nth) {
      const int rl = j & (S - 1), I = j >> lS;
      auto gb = [&](int i) { return bk[(i << lS) + rl]; };
      auto gd = [&](int i) { return dk[i]; };
      bc[j] = mg_down_cell<Op, R>(a.op[k], f, I % c.nx, (I / c.nx) % c.ny, I / (c.nx * c.ny), tr, om, gb, gd);
    }
    __syncthreads();
  }
  {
    const int k = T - 1;
    const int nk = a.dims[k].n() << lS;
    for (int j = threadIdx.x; j < nk; j += nth)
      sh[a.off[k] + nk + j] = a.dinv[k][j >> lS] * sh[a.off[k] + j];
  }
  __syncthreads();
  for (int k = T - 2; k >= 0; --k) {
    const LevelDims f = a.dims[k], c = a.dims[k + 1];
    const int nk = f.n() << lS, nc = c.n() << lS;
    const cx<R>* bk = sh + a.off[k];
    cx<R>* xk = sh + a.off[k] + nk;
    const cx<R>* xc = sh + a.off[k + 1] + nc;
    const cx<R>* dk = a.dinv[k];
    for (int j = threadIdx.x; j < nk; j += nth) {
      const int rl = j & (S - 1);
      auto gb = [&](int i) { return bk[(i << lS) + rl]; };
      auto gd = [&](int i) { return dk[i]; };
      auto gx = [&](int I) { return xc[(I << lS) + rl]; };
      xk[j] = mg_up_cell<Op, R>(a.op[k], f, c, j >> lS, tr, om, gb, gd, gx);
    }
    __syncthreads();
  }
  {
    const int n0 = a.dims[0].n() << lS;
    for (int j = threadIdx.x; j < n0; j += nth) xtop[j] = sh[a.off[0] + n0 + j];
  }
}

// The coarsest level solved on the grid (only when even its lanes exceed the
// tail's LDS): x = D^-1 b.
template <typename R>
__global__ void __launch_bounds__(BS) k_mg_scale_grid(long N, int lS, const cx<R>* __restrict__ dinv,
                                                      const cx<R>* __restrict__ b, cx<R>* __restrict__ x,
                                                      const int* __restrict__ all_done) {
  if (*all_done) return;
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < N; t += (long)gridDim.x * BS) x[t] = dinv[t >> lS] * b[t];
}

// ------------------------------------------------------- COCG with the V-cycle
// Lane prologue shared with the Jacobi kernel: the flag, the previous
// partials and the state in one round trip, the sums, then the advance.
// Returns false when the launch has nothing to do.
template <int CGB, bool ONE>
__device__ __forceinline__ bool cg_prologue(int lS, const CgCfg& cfg, const c128* __restrict__ partIn, int Gin,
                                            const CgScal* __restrict__ scIn, CgScal* __restrict__ scOut,
                                            int* __restrict__ all_done, CgScal& s) {
  const int S = 1 << lS;
  const int rl = ONE ? 0 : (int)threadIdx.x & (S - 1);
  const int flag = *all_done;
  constexpr int KMAX = 4;
  PartLoad<3, KMAX> PL;
  part_load<3, KMAX, CGB>(partIn, Gin, S, PL);
  s = scIn[rl];
  c128 tot[3];
  part_sum<3, KMAX, CGB>(partIn, Gin, S, PL, tot);
  if (flag) {
    if (blockIdx.x == 0 && (int)threadIdx.x < S) scOut[threadIdx.x] = s;
    return false;
  }
  cg_advance(s, cfg, tot[0], tot[1], tot[2].re);
  const bool any_open = __any(!s.done);
  if (blockIdx.x == 0 && (int)threadIdx.x < S) scOut[threadIdx.x] = s;
  if (!any_open) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *all_done = 1;
    return false;
  }
  return true;
}

// Vector part of one multigrid-COCG iteration (the V-cycle and the operator
// product follow in their own launches):
//   ITER: s' = w + beta s, r' = r - alpha s', p' = u + beta p, x += alpha p'
//         (u = B r from the previous V-cycle);
//   RR:   r' = v - (K + tau M) x in FP64, stored rounded (a round change of the
//         complex64 path; the V-cycle and the product then give the new round's
//         forms directly);
//   KX:   x += u, one preconditioned Richardson step on the iterate (u = B r of
//         the residual just formed), before a new residual.
template <typename Op, typename OpD, typename R, int CGB, bool ONE, bool MULTI>
__global__ void __launch_bounds__(CGB) k_cgmg_step(OpD opd, c128 tau, int n, int lS_, CgCfg cfg,
                                                   const cx<R>* __restrict__ v, const cx<R>* __restrict__ u,
                                                   const c128* __restrict__ partIn, int Gin,
                                                   const CgScal* __restrict__ scIn, CgScal* __restrict__ scOut,
                                                   CgVecs<R> vec, int par, int* __restrict__ all_done) {
  const int lS = ONE ? 0 : lS_;
  const int rl = ONE ? 0 : (int)threadIdx.x & ((1 << lS) - 1);
  CgScal s;
  if (!cg_prologue<CGB, ONE>(lS, cfg, partIn, Gin, scIn, scOut, all_done, s)) return;
  if (s.done) return;
  const int N = n << lS;
  const cx<R>* __restrict__ r0 = vec.r[par];
  const cx<R>* __restrict__ w0 = vec.w[par];
  const cx<R>* __restrict__ s0 = vec.s[par];
  cx<R>* __restrict__ r1 = vec.r[par ^ 1];
  cx<R>* __restrict__ s1 = vec.s[par ^ 1];
  const int t0 = xcd_tile(blockIdx.x, gridDim.x) * CGB + threadIdx.x;
  auto for_cells = [&](auto&& f) {
    if constexpr (MULTI) {
      for (int t = t0; t < N; t += gridDim.x * CGB) f(t);
    } else {
      if (t0 < N) f(t0);
    }
  };
  if (s.mode == CG_ITER) {
    const cx<R> al = cvt<R>(s.alpha), be = cvt<R>(s.beta);
    const c128 al64 = s.alpha;
    for_cells([&](int t) {
      const cx<R> sn = w0[t] + be * s0[t];
      const cx<R> pn = u[t] + be * vec.p[t];
      r1[t] = r0[t] - al * sn;
      s1[t] = sn;
      vec.p[t] = pn;
      vec.x[t] = vec.x[t] + al64 * cvt<double>(pn);
    });
  } else if (s.mode == CG_RR) {
    const c128* __restrict__ x = vec.x;
    auto gx = [&](int cc) { return x[(cc << lS) + rl]; };
    for_cells([&](int t) {
      const int c = t >> lS;
      r1[t] = cvt<R>(cvt<double>(v[t]) - opd.template apply<double>(c, tau, gx));
      s1[t] = cx<R>{0, 0};
    });
  } else if (s.mode == CG_KX) {
    for_cells([&](int t) { vec.x[t] = vec.x[t] + cvt<double>(u[t]); });
  }
}

// Operator product and forms of one multigrid-COCG iteration: w' = A u' for
// u' = B r' (the V-cycle's output), and the block partials of r'^T u',
// w'^T u', ||r'||^2 (exact FP64 products of the stored values).  Lanes that
// are done contribute zeros.
template <typename Op, typename R, int CGB, bool ONE, bool MULTI>
__global__ void __launch_bounds__(CGB) k_cgmg_post(Op op, c128 tau, int n, int lS_, const CgScal* __restrict__ sc,
                                                   const cx<R>* __restrict__ r, const cx<R>* __restrict__ u,
                                                   cx<R>* __restrict__ w, c128* __restrict__ partOut,
                                                   const int* __restrict__ all_done) {
  if (*all_done) return;
  const int lS = ONE ? 0 : lS_;
  const int S = 1 << lS;
  const int rl = ONE ? 0 : (int)threadIdx.x & (S - 1);
  const int N = n << lS;
  const bool live = !sc[rl].done;
  const cx<R> tr = cvt<R>(tau);
  auto gu = [&](int cc) { return u[(cc << lS) + rl]; };
  const int t0 = xcd_tile(blockIdx.x, gridDim.x) * CGB + threadIdx.x;
  c128 ag{0, 0}, ad{0, 0};
  double arr = 0.0;
  auto cell = [&](int t) {
    const int c = t >> lS;
    const cx<R> ww = op.template apply<R>(c, tr, gu);
    w[t] = ww;
    const c128 rd = cvt<double>(r[t]), ud = cvt<double>(u[t]);
    ag = ag + rd * ud;
    ad = ad + cvt<double>(ww) * ud;
    arr += abs2(rd);
  };
  if (live) {
    if constexpr (MULTI) {
      for (int t = t0; t < N; t += gridDim.x * CGB) cell(t);
    } else {
      if (t0 < N) cell(t0);
    }
  }
  c128 acc[3] = {ag, ad, {arr, 0.0}};
  block_partials<3, CGB>(acc, S, partOut + (size_t)blockIdx.x * 3 * S);
}

}  // namespace shk
