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
#include <type_traits>
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

// Inverse diagonals for the solve's tau, 1 / (diag K_l + tau M_l), of up to
// MG_DINV_TAB levels in one launch: level q holds cells [start[q],
// start[q + 1]) of the launch's index range.
constexpr int MG_DINV_TAB = 16;
template <typename OpD, typename R> struct MgDinvTab {
  int nl;
  long start[MG_DINV_TAB + 1];
  OpD op[MG_DINV_TAB];
  cx<R>* out[MG_DINV_TAB];
};
template <typename OpD, typename R>
__global__ void __launch_bounds__(BS) k_mg_dinv_levels(MgDinvTab<OpD, R> tab, c128 tau) {
  const long total = tab.start[tab.nl];
  for (long g = blockIdx.x * (long)BS + threadIdx.x; g < total; g += (long)gridDim.x * BS) {
    int l = 0;
    while (l + 1 < tab.nl && g >= tab.start[l + 1]) ++l;
    const int c = (int)(g - tab.start[l]);
    const OpD& o = tab.op[l];
    const double m = o.mass(c);
    tab.out[l][c] = cvt<R>(cdiv(c128{1.0, 0.0}, c128{o.diagK(c) + tau.re * m, tau.im * m}));
  }
}

// ---------------------------------------------------------------- V-cycle --
// The grid kernels below load the done flag together with their operands and
// judge it only before their stores, so a launch costs one round trip to
// memory rather than two.  hold(v, flag) marks the point where both are
// needed: the loads behind v are issued before it and the flag is neither
// tested nor waited for ahead of it (else the compiler tends to test a
// loop-invariant flag first, or to move the loads into the branch that
// stores).
template <typename R> __device__ __forceinline__ void hold(cx<R>& v, int& flag) {
  asm volatile("" : "+v"(v.re), "+v"(v.im), "+s"(flag));
}
// Sum of v over the Q = 2^d adjacent lanes of an aligned group (d = 2, 3), in
// the same order in every lane: quad permutes (DPP) for lane distances 1 and
// 2, a cross-lane read for 4.
template <int CTRL> __device__ __forceinline__ float dpp_quad(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_quad(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int Q, typename R> __device__ __forceinline__ cx<R> group_sum(cx<R> v) {
  constexpr int X1 = 0xB1, X2 = 0x4E;   // quad_perm [1,0,3,2] and [2,3,0,1]
  v.re += dpp_quad<X1>(v.re);
  v.im += dpp_quad<X1>(v.im);
  v.re += dpp_quad<X2>(v.re);
  v.im += dpp_quad<X2>(v.im);
  if constexpr (Q == 8) {
    v.re += __shfl_xor(v.re, 4);
    v.im += __shfl_xor(v.im, 4);
  }
  return v;
}

// A pointer the compiler cannot see through: a load from it stays where it is
// written instead of being merged with an earlier one.
template <typename T> __device__ __forceinline__ T* opaque(T* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// Downward leg, one fine cell c = (i, j, k) and lane: the residual
// b_c - (A x1)_c after the first sweep x1 = omega D^-1 b (x1 at the stencil
// neighbours formed on the fly).  gb(c), gd(c): b and D^-1 at fine cell c
// for the lane.  Callers pass coordinates so that no index is divided.
template <typename Op, typename R, typename GB, typename GD>
__device__ __forceinline__ cx<R> mg_down_fine(const Op& op, int i, int j, int k, int c, cx<R> tr, R om, GB gb,
                                              GD gd) {
  constexpr int NB = Op::NB;
  int idx[NB];
  R fo[NB];
  R fsum;
  op.template stencil_at<R>(i, j, k, c, idx, fo, fsum);
  const cx<R> bi = gb(c);
  const cx<R> x1 = om * (gd(c) * bi);
  cx<R> ax = fsum * x1 + (R)op.mass(c) * (tr * x1);
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int n = idx[q];
    ax = ax - fo[q] * (om * (gd(n) * gb(n)));
  }
  return bi - ax;
}

// Upward leg, one fine cell c = (i, j, k) and lane: x2 = x1 + P x_c
// (x1 = omega D^-1 b), then one sweep x = x2 + omega D^-1 (b - A x2), with x2
// at the stencil neighbours formed on the fly; gxc(C): coarse solution at
// coarse cell C of the grid cd.  A neighbour's parent differs from the
// cell's own only along the neighbour's axis.
template <typename Op, typename R, typename GB, typename GD, typename GX>
__device__ __forceinline__ cx<R> mg_up_cell(const Op& op, const LevelDims& f, const LevelDims& cd, int i, int j,
                                            int k, int c, cx<R> tr, R om, GB gb, GD gd, GX gxc) {
  constexpr int NB = Op::NB;
  int idx[NB];
  R fo[NB];
  R fsum;
  op.template stencil_at<R>(i, j, k, c, idx, fo, fsum);
  const int pi = i >> 1, pj = j >> 1, pk = k >> 1;
  auto par = [&](int a, int b, int e) { return a + cd.nx * (b + cd.ny * e); };
  int pq[NB];
  pq[0] = par((i > 0 ? i - 1 : i) >> 1, pj, pk);
  pq[1] = par((i < f.nx - 1 ? i + 1 : i) >> 1, pj, pk);
  pq[2] = par(pi, (j > 0 ? j - 1 : j) >> 1, pk);
  pq[3] = par(pi, (j < f.ny - 1 ? j + 1 : j) >> 1, pk);
  if constexpr (NB == 6) {
    pq[4] = par(pi, pj, (k > 0 ? k - 1 : k) >> 1);
    pq[5] = par(pi, pj, (k < f.nz - 1 ? k + 1 : k) >> 1);
  }
  const cx<R> xi = om * (gd(c) * gb(c)) + gxc(par(pi, pj, pk));
  cx<R> ax = fsum * xi + (R)op.mass(c) * (tr * xi);
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int n = idx[q];
    ax = ax - fo[q] * (om * (gd(n) * gb(n)) + gxc(pq[q]));
  }
  return xi + om * (gd(c) * (gb(c) - ax));
}

// Block coordinates of a (gx, gy, gz) launch, the linear block index taken
// through xcd_tile: each XCD walks a contiguous band of rows (and planes), so
// the stencil's neighbour rows are mostly in its own L2.
// In 3-D with gy a multiple of 8, XCD x (workgroups are dealt out to the XCDs
// round-robin, linear id mod 8) takes instead the y-slab of rows
// [x gy/8, (x+1) gy/8) of every plane, walked plane after plane: the blocks an
// XCD runs at once then span a few planes of its slab, whose planes before and
// after are still in its L2 (a band of whole planes is too large for it).
__device__ __forceinline__ void xcd_block3(int& bx, int& by, int& bz) {
  const int gx = gridDim.x, gy = gridDim.y;
  const int w = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  if (gridDim.z > 1 && (gy & 7) == 0) {
    const int ry = gy >> 3, u = w >> 3;
    bx = u % gx;
    const int r = u / gx;
    by = (w & 7) * ry + r % ry;
    bz = r / ry;
    return;
  }
  const int T = xcd_tile(w, gx * gy * gridDim.z);
  const int r = T / gx;
  bx = T - r * gx;
  by = r % gy;
  bz = r / gy;
}

// Downward leg of one level over the grid: coarse right-hand side b_c.
// Launch grid (ceil(c.nx S 2^d / BS), c.ny, c.nz): along a coarse row,
// thread t holds child t mod 2^d of lane (t >> d) mod S of coarse cell
// t >> (d + log2 S), so the 2^d children of a coarse cell sit in adjacent
// lanes of one wavefront and are summed by cross-lane exchange.
template <typename Op, typename R>
__global__ void __launch_bounds__(BS) k_mg_down(Op op, LevelDims f, LevelDims c, c128 tau, double omega, int lS,
                                                const cx<R>* __restrict__ b, const cx<R>* __restrict__ dinv,
                                                cx<R>* __restrict__ out, const int* __restrict__ all_done) {
  constexpr int D = Op::NB / 2;
  constexpr int Q = 1 << D;
  int flag = *all_done;
  int bx, J, L;
  xcd_block3(bx, J, L);
  const int t = bx * BS + threadIdx.x;
  if (t >= (c.nx << (lS + D))) return;   // whole groups of 2^d lanes leave together
  const int S = 1 << lS;
  const int q = t & (Q - 1), rl = (t >> D) & (S - 1), I = t >> (D + lS);
  const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = 2 * L + (q >> 2);
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  cx<R> v{0, 0};
  if (i < f.nx && j < f.ny && k < f.nz) {
    auto gb = [&](int n) { return b[((long)n << lS) + rl]; };
    auto gd = [&](int n) { return dinv[n]; };
    v = mg_down_fine<Op, R>(op, i, j, k, i + f.nx * (j + f.ny * k), tr, om, gb, gd);
  }
  v = group_sum<Q>(v);
  hold(v, flag);
  if (!flag && q == 0) out[((long)(I + c.nx * (J + c.ny * L)) << lS) + rl] = v;
}

// Upward leg of one level over the grid.  Launch grid (ceil(f.nx S / BS),
// f.ny, f.nz): along a fine row thread t holds lane t mod S of cell t >> log2 S.
template <typename Op, typename R>
__global__ void __launch_bounds__(BS) k_mg_up(Op op, LevelDims f, LevelDims c, c128 tau, double omega, int lS,
                                              const cx<R>* __restrict__ b, const cx<R>* __restrict__ dinv,
                                              const cx<R>* __restrict__ xc, cx<R>* __restrict__ xout,
                                              const int* __restrict__ all_done) {
  int flag = *all_done;
  int bx, j, k;
  xcd_block3(bx, j, k);
  const int t = bx * BS + threadIdx.x;
  if (t >= (f.nx << lS)) return;
  const int S = 1 << lS;
  const int rl = t & (S - 1), i = t >> lS;
  const int cell = i + f.nx * (j + f.ny * k);
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  auto gb = [&](int n) { return b[((long)n << lS) + rl]; };
  auto gd = [&](int n) { return dinv[n]; };
  auto gx = [&](int n) { return xc[((long)n << lS) + rl]; };
  cx<R> v = mg_up_cell<Op, R>(op, f, c, i, j, k, cell, tr, om, gb, gd, gx);
  hold(v, flag);
  if (!flag) xout[((long)cell << lS) + rl] = v;
}

// True when some lane of the chunk l0 .. l0 + LT - 1 still runs (its state as
// the step of this iteration left it): the V-cycle and the product skip the
// chunks whose lanes have all stopped, whose results nothing reads.
template <int LT> __device__ __forceinline__ bool chunk_live(const CgScal* __restrict__ sc, int l0) {
  bool live = false;
#pragma unroll
  for (int l = 0; l < LT; ++l) live = live || !sc[l0 + l].done;
  return live;
}

// The two legs for several right-hand sides: a thread works LT lanes of one
// cell (down: of one child of a coarse cell) and loads the cell's stencil,
// mass and D^-1 once for them instead of once per lane; per lane the
// expressions of mg_down_fine and mg_up_cell.  Lane chunk lc holds lanes
// lc LT .. lc LT + LT - 1; lNC = log2(S / LT).
// Down: grid (ceil(c.nx 2^(lNC + d) / BS), c.ny, c.nz); the 2^d children of a
// coarse cell and its chunks share a run of 2^(d + lNC) threads.
template <typename Op, typename R, int LT>
__global__ void __launch_bounds__(BS) k_mg_down_lanes(Op op, LevelDims f, LevelDims c, c128 tau, double omega,
                                                      int lS, int lNC, const cx<R>* __restrict__ b,
                                                      const cx<R>* __restrict__ dinv, cx<R>* __restrict__ out,
                                                      const CgScal* __restrict__ sc, const int* __restrict__ all_done) {
  constexpr int D = Op::NB / 2;
  constexpr int Q = 1 << D;
  constexpr int NB = Op::NB;
  int flag = *all_done;
  int bx, J, L;
  xcd_block3(bx, J, L);
  const int t = bx * BS + threadIdx.x;
  if (t >= (c.nx << (lNC + D))) return;   // whole groups of 2^d lanes leave together
  // Chunks fastest when a coarse cell's children and chunks fit in a wave
  // (2^(d + lNC) <= 64): consecutive threads read consecutive pieces of one
  // cell's lanes (coalesced) and the 2^d children of a coarse cell sit 2^lNC
  // lanes apart; otherwise children fastest (summed by quad permutes)
  const bool cf = D + lNC <= 6;
  const int q = cf ? (t >> lNC) & (Q - 1) : t & (Q - 1);
  const int lc = cf ? t & ((1 << lNC) - 1) : (t >> D) & ((1 << lNC) - 1);
  const int I = t >> (D + lNC);
  const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = 2 * L + (q >> 2);
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  const bool live = chunk_live<LT>(sc, lc * LT);
  cx<R> v[LT];
#pragma unroll
  for (int l = 0; l < LT; ++l) v[l] = cx<R>{0, 0};
  if (live && i < f.nx && j < f.ny && k < f.nz) {
    const int cell = i + f.nx * (j + f.ny * k);
    int idx[NB];
    R fo[NB];
    R fsum;
    op.template stencil_at<R>(i, j, k, cell, idx, fo, fsum);
    const R m = (R)op.mass(cell);
    const cx<R> dc = dinv[cell];
    cx<R> dn[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) dn[e] = dinv[idx[e]];
#pragma unroll
    for (int l = 0; l < LT; ++l) {
      const int rl = lc * LT + l;
      auto gb = [&](int n) { return b[((long)n << lS) + rl]; };
      const cx<R> bi = gb(cell);
      const cx<R> x1 = om * (dc * bi);
      cx<R> ax = fsum * x1 + m * (tr * x1);
#pragma unroll
      for (int e = 0; e < NB; ++e) ax = ax - fo[e] * (om * (dn[e] * gb(idx[e])));
      v[l] = bi - ax;
    }
  }
  if (cf) {
    // the children, 2^lNC lanes apart: a butterfly in the same order in
    // every lane of the group
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const int dl = 1 << (lNC + e);
#pragma unroll
      for (int l = 0; l < LT; ++l) {
        v[l].re += __shfl_xor(v[l].re, dl);
        v[l].im += __shfl_xor(v[l].im, dl);
      }
    }
  } else {
#pragma unroll
    for (int l = 0; l < LT; ++l) v[l] = group_sum<Q>(v[l]);
  }
  hold(v[0], flag);
  if (!flag && q == 0 && live) {
    cx<R>* o = out + ((long)(I + c.nx * (J + c.ny * L)) << lS) + lc * LT;
#pragma unroll
    for (int l = 0; l < LT; ++l) o[l] = v[l];
  }
}

// Up: grid (ceil(f.nx 2^lNC / BS), f.ny, f.nz), thread t holds chunk
// t mod 2^lNC of cell t >> lNC along a fine row.
template <typename Op, typename R, int LT>
__global__ void __launch_bounds__(BS) k_mg_up_lanes(Op op, LevelDims f, LevelDims cd, c128 tau, double omega, int lS,
                                                    int lNC, const cx<R>* __restrict__ b,
                                                    const cx<R>* __restrict__ dinv, const cx<R>* __restrict__ xc,
                                                    cx<R>* __restrict__ xout, const CgScal* __restrict__ sc,
                                                    const int* __restrict__ all_done) {
  constexpr int NB = Op::NB;
  int flag = *all_done;
  int bx, j, k;
  xcd_block3(bx, j, k);
  const int t = bx * BS + threadIdx.x;
  if (t >= (f.nx << lNC)) return;
  const int lc = t & ((1 << lNC) - 1), i = t >> lNC;
  if (!chunk_live<LT>(sc, lc * LT)) return;
  const int cell = i + f.nx * (j + f.ny * k);
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  int idx[NB];
  R fo[NB];
  R fsum;
  op.template stencil_at<R>(i, j, k, cell, idx, fo, fsum);
  const int pi = i >> 1, pj = j >> 1, pk = k >> 1;
  auto par = [&](int a, int bb, int e) { return a + cd.nx * (bb + cd.ny * e); };
  int pq[NB];
  pq[0] = par((i > 0 ? i - 1 : i) >> 1, pj, pk);
  pq[1] = par((i < f.nx - 1 ? i + 1 : i) >> 1, pj, pk);
  pq[2] = par(pi, (j > 0 ? j - 1 : j) >> 1, pk);
  pq[3] = par(pi, (j < f.ny - 1 ? j + 1 : j) >> 1, pk);
  if constexpr (NB == 6) {
    pq[4] = par(pi, pj, (k > 0 ? k - 1 : k) >> 1);
    pq[5] = par(pi, pj, (k < f.nz - 1 ? k + 1 : k) >> 1);
  }
  const int pc = par(pi, pj, pk);
  const R m = (R)op.mass(cell);
  const cx<R> dc = dinv[cell];
  cx<R> dn[NB];
#pragma unroll
  for (int e = 0; e < NB; ++e) dn[e] = dinv[idx[e]];
  cx<R> v[LT];
#pragma unroll
  for (int l = 0; l < LT; ++l) {
    const int rl = lc * LT + l;
    auto gb = [&](int n) { return b[((long)n << lS) + rl]; };
    auto gx = [&](int n) { return xc[((long)n << lS) + rl]; };
    const cx<R> bc = gb(cell);
    const cx<R> xi = om * (dc * bc) + gx(pc);
    cx<R> ax = fsum * xi + m * (tr * xi);
#pragma unroll
    for (int e = 0; e < NB; ++e) ax = ax - fo[e] * (om * (dn[e] * gb(idx[e])) + gx(pq[e]));
    v[l] = xi + om * (dc * (bc - ax));
  }
  hold(v[0], flag);
  if (!flag) {
    cx<R>* o = xout + ((long)cell << lS) + lc * LT;
#pragma unroll
    for (int l = 0; l < LT; ++l) o[l] = v[l];
  }
}

// One cell's inputs of the smoothed value: b, D^-1 and (on the way up) x_c of
// its parent.
template <typename R, int LT, bool UP> struct Tile3Raw {
  cx<R> b[LT];
  cx<R> x[UP ? LT : 1];
  cx<R> d;
};

// ------------------------------------------ 2-D legs, marching the rows ----
// The two legs of a 2-D level for several lanes with every input read once:
// a block owns a segment of SW = BS / 2^lNC cells of a row (a thread per cell
// and chunk of LT lanes, chunks fastest, so a row segment's lanes are one
// contiguous run) and marches through YB rows.  On each row the block forms
// the smoothed value x1 (omega D^-1 b, plus the prolongated coarse solution
// on the way up) of its cells and of the segment's two end neighbours once,
// in LDS; the x neighbours of the stencil come from there, the y neighbours
// from the thread's registers (its cell's x1 on the rows below and above).
// The one-cell kernels read every lane chunk once per stencil point.  Same
// arithmetic per lane as k_mg_down_lanes / k_mg_up_lanes, and the same
// children order on the way down (the x pair of each row, then the rows).
// Needs 2^lNC <= 32 and even YB; launched on G = ceil(nx / SW) ceil(ny / YB)
// blocks, block b taking tile xcd_tile(b, G) (segment fastest).
template <typename Op, typename R, int LT, bool UP>
__global__ void __launch_bounds__(BS) k_mg_leg_rows(Op op, LevelDims f, LevelDims cd, c128 tau, double omega,
                                                    int lS, int lNC, int YB, const cx<R>* __restrict__ b,
                                                    const cx<R>* __restrict__ dinv, const cx<R>* __restrict__ xc,
                                                    cx<R>* __restrict__ out, const CgScal* __restrict__ sc,
                                                    const int* __restrict__ all_done) {
  static_assert(Op::NB == 4, "2-D operator");
  __shared__ cx<R> xs[2][BS * LT + 2 * 64];   // x1 of a row: (SW + 2) cells x S lanes, double-buffered
  const int flag = *all_done;
  const int NC = 1 << lNC, S = 1 << lS, SW = BS >> lNC;
  const int nseg = (f.nx + SW - 1) / SW;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int seg = tile % nseg, rb = tile / nseg;
  const int lc = (int)threadIdx.x & (NC - 1), ci = (int)threadIdx.x >> lNC;
  const int i = seg * SW + ci;
  const bool live = chunk_live<LT>(sc, lc * LT);   // a stopped chunk loads and stores nothing
  const bool own = i < f.nx && live;
  // the segment's end neighbours: threads 0 .. 2 NC - 1, left then right
  const int hs = (int)threadIdx.x >> lNC;
  const bool hal = (int)threadIdx.x < 2 * NC;
  const int hi = hs == 0 ? seg * SW - 1 : seg * SW + SW;
  const bool hin = hal && hi >= 0 && hi < f.nx && live;
  const int j0 = rb * YB, j1 = min(j0 + YB, f.ny);
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  const int l0 = lc * LT;
  using Raw = Tile3Raw<R, LT, UP>;
  auto load = [&](int ci_, int cj, Raw& r) {
    const int c = ci_ + f.nx * cj;
    r.d = dinv[c];
    const long bb = ((long)c << lS) + l0;
#pragma unroll
    for (int l = 0; l < LT; ++l) r.b[l] = b[bb + l];
    if constexpr (UP) {
      const long pb = ((long)((ci_ >> 1) + cd.nx * (cj >> 1)) << lS) + l0;
#pragma unroll
      for (int l = 0; l < LT; ++l) r.x[l] = xc[pb + l];
    }
  };
  auto smooth = [&](const Raw& r, cx<R> (&o)[LT]) {
#pragma unroll
    for (int l = 0; l < LT; ++l) {
      if constexpr (UP) o[l] = om * (r.d * r.b[l]) + r.x[l];
      else o[l] = om * (r.d * r.b[l]);
    }
  };
  auto zero = [](cx<R> (&o)[LT]) {
#pragma unroll
    for (int l = 0; l < LT; ++l) o[l] = cx<R>{0, 0};
  };
  cx<R> xp[LT], xcur[LT], xn[LT], bcur[LT], hv[LT], acc[LT];
  cx<R> dcur{0, 0};
  Raw rn, hr;
  zero(xp);
  zero(xcur);
  zero(bcur);
  zero(acc);
  if (hin && j0 < j1) load(hi, j0, hr);
  if (own && j0 < j1) {
    if (j0 > 0) {
      load(i, j0 - 1, rn);
      smooth(rn, xp);
    }
    load(i, j0, rn);
    smooth(rn, xcur);
#pragma unroll
    for (int l = 0; l < LT; ++l) bcur[l] = rn.b[l];
    dcur = rn.d;
  }
  const int own_slot = (ci + 1) * S + l0;
  const int hal_slot = (hs == 0 ? 0 : (SW + 1) * S) + l0;
  int buf = 0;
  for (int j = j0; j < j1; ++j) {
    // this row's end neighbours (inputs loaded on the previous step), then
    // the loads this step and the next need, issued together
    zero(hv);
    if (hin) smooth(hr, hv);
    if (hin && j + 1 < j1) load(hi, j + 1, hr);
    const bool up_in = own && j + 1 < f.ny;
    if (up_in) load(i, j + 1, rn);
    const int c = i + f.nx * j;
    int idx[4];
    R fo[4];
    R fsum = 0;
    R m = 0;
    if (own) {
      op.template stencil_at<R>(i, j, 0, c, idx, fo, fsum);
      m = (R)op.mass(c);
    }
    cx<R>* row = xs[buf];
#pragma unroll
    for (int l = 0; l < LT; ++l) row[own_slot + l] = xcur[l];   // zeros past the grid's end
    if (hal) {
#pragma unroll
      for (int l = 0; l < LT; ++l) row[hal_slot + l] = hv[l];
    }
    __syncthreads();   // one barrier a row: the buffers alternate
    zero(xn);
    if (up_in) smooth(rn, xn);
    cx<R> v[LT];
    zero(v);
    if (own) {
#pragma unroll
      for (int l = 0; l < LT; ++l) {
        const cx<R> xi = xcur[l];
        cx<R> ax = fsum * xi + m * (tr * xi);
        ax = ax - fo[0] * row[own_slot - S + l];
        ax = ax - fo[1] * row[own_slot + S + l];
        ax = ax - fo[2] * xp[l];
        ax = ax - fo[3] * xn[l];
        if constexpr (UP) v[l] = xi + om * (dcur * (bcur[l] - ax));
        else v[l] = bcur[l] - ax;
      }
    }
    if constexpr (UP) {
      int fl = flag;
      hold(v[0], fl);
      if (own && !fl) {
        cx<R>* o = out + ((long)c << lS) + l0;
#pragma unroll
        for (int l = 0; l < LT; ++l) o[l] = v[l];
      }
    } else {
      // the x pair of children on this row (2^lNC lanes apart), then the rows
#pragma unroll
      for (int l = 0; l < LT; ++l) {
        v[l].re += __shfl_xor(v[l].re, NC);
        v[l].im += __shfl_xor(v[l].im, NC);
        acc[l] = (j & 1) ? acc[l] + v[l] : v[l];
      }
      if ((j & 1) || j + 1 == f.ny) {
        const int I = i >> 1, J = j >> 1;
        int fl = flag;
        hold(acc[0], fl);
        if (!(ci & 1) && I < cd.nx && live && !fl) {
          cx<R>* o = out + ((long)(I + cd.nx * J) << lS) + l0;
#pragma unroll
          for (int l = 0; l < LT; ++l) o[l] = acc[l];
        }
      }
    }
#pragma unroll
    for (int l = 0; l < LT; ++l) {
      xp[l] = xcur[l];
      xcur[l] = xn[l];
      if (up_in) bcur[l] = rn.b[l];
    }
    if (up_in) dcur = rn.d;
    buf ^= 1;
  }
}

// ------------------------------------------------ 2-D chains of legs ------
// Several consecutive grid legs of a single-lane 2-D V-cycle in one launch,
// for the middle levels whose one-leg launches are latency-bound: each block
// owns a tile of the chain's last level and recomputes the cells of the
// earlier levels that its tile depends on (a ring of one cell per level and
// the children of that).  Every input of every level (right-hand side, D^-1,
// faces, masses) is loaded into LDS at the start, all loads in flight at
// once; the legs then run from LDS with a barrier between levels, so the
// chain costs one memory round trip instead of one or two per leg.  Only the
// chain's outputs go to memory.  Same per-cell expressions and children order
// as k_mg_down / k_mg_up.
constexpr int MGC_F = 3;   // legs per chain at most
template <typename Op, typename R> struct MgChain {
  int nl;                        // legs in the chain (1..MGC_F)
  LevelDims d[MGC_F + 1];        // level dims, d[0] the chain's finest level
  Op op[MGC_F];                  // operators of levels 0..nl-1
  const cx<R>* dinv[MGC_F + 1];  // inverse diagonals of levels 0..nl
  const cx<R>* b[MGC_F];         // down: b[0] the input; up: right-hand sides of levels 0..nl-1
  cx<R>* out[MGC_F + 1];         // down: out[k] the right-hand side of level k (1..nl); up: out[0]
  const cx<R>* xc;               // up: solution of level nl
};

// One cell's stencil data staged in LDS: its four face coefficients (west,
// east, south, north; boundary faces included) and its mass.
template <typename R> struct MgcCell {
  R f[4];
  R m;
};
template <typename Op, typename R>
__device__ __forceinline__ MgcCell<R> mgc_load_cell(const Op& o, int i, int j) {
  const int fx = i + (o.nx + 1) * j, fy = i + o.nx * j;
  MgcCell<R> a;
  a.f[0] = (R)o.tx[fx];
  a.f[1] = (R)o.tx[fx + 1];
  a.f[2] = (R)o.ty[fy];
  a.f[3] = (R)o.ty[fy + o.nx];
  a.m = (R)o.mass(i + o.nx * j);
  return a;
}
// A x at cell (i, j) of an nx x ny level from its staged stencil data, x at
// the cell and at its four neighbours (the face coefficient of a neighbour
// outside the grid is zero, as in the stencil's own form).
template <typename R>
__device__ __forceinline__ cx<R> mgc_apply(const MgcCell<R>& a, int i, int j, int nx, int ny, cx<R> tr, cx<R> xi,
                                           cx<R> xw, cx<R> xe, cx<R> xs, cx<R> xn) {
  const R fsum = a.f[0] + a.f[1] + a.f[2] + a.f[3];
  const R fo0 = i > 0 ? a.f[0] : (R)0, fo1 = i < nx - 1 ? a.f[1] : (R)0;
  const R fo2 = j > 0 ? a.f[2] : (R)0, fo3 = j < ny - 1 ? a.f[3] : (R)0;
  cx<R> ax = fsum * xi + a.m * (tr * xi);
  ax = ax - fo0 * xw;
  ax = ax - fo1 * xe;
  ax = ax - fo2 * xs;
  ax = ax - fo3 * xn;
  return ax;
}

// Restriction chain: right-hand sides of levels 1..nl from that of level 0.
// Block tile T x T of level nl; level k's region is the children of level
// k+1's region and one ring more (the stencil).
template <int T> __host__ __device__ constexpr int mgc_down_side(int up) {   // up = nl - k
  return up == 0 ? T : 2 * mgc_down_side<T>(up - 1) + 2;
}
template <int T> constexpr int mgc_down_cells() {
  return mgc_down_side<T>(1) * mgc_down_side<T>(1) + mgc_down_side<T>(2) * mgc_down_side<T>(2) +
         mgc_down_side<T>(3) * mgc_down_side<T>(3);
}
template <typename Op, typename R, int T>
__global__ void __launch_bounds__(BS) k_mg_down_chain2d(MgChain<Op, R> ch, c128 tau, double omega,
                                                        const int* __restrict__ all_done) {
  constexpr int NC = mgc_down_cells<T>();
  __shared__ cx<R> sb[NC], sx[NC], sd[NC];   // b, x1 and D^-1 of levels 0..nl-1 (level 0 first)
  __shared__ MgcCell<R> sc[NC];              // stencil data of the same cells
  const int flag = *all_done;
  const int nl = ch.nl;
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  int lox[MGC_F + 1], loy[MGC_F + 1], side[MGC_F + 1], off[MGC_F + 1];
  // level k's region, k = nl .. 0 (entries past nl unused)
#pragma unroll
  for (int k = MGC_F; k >= 0; --k) {
    if (k >= nl) {
      lox[k] = (int)blockIdx.x * T;
      loy[k] = (int)blockIdx.y * T;
      side[k] = T;
    } else {
      lox[k] = 2 * lox[k + 1] - 1;
      loy[k] = 2 * loy[k + 1] - 1;
      side[k] = 2 * side[k + 1] + 2;
    }
  }
  off[0] = 0;
#pragma unroll
  for (int k = 1; k <= MGC_F; ++k) off[k] = off[k - 1] + (k <= nl ? side[k - 1] * side[k - 1] : 0);
  // every level's inputs over its region, all loads issued together; x1 of
  // level 0 (the later levels' x1 follow their right-hand sides)
#pragma unroll
  for (int k = 0; k < MGC_F; ++k) {
    if (k >= nl) break;
    const int W = side[k];
    const LevelDims d = ch.d[k];
    for (int le = threadIdx.x; le < W * W; le += BS) {
      const int e = off[k] + le;
      const int gi = lox[k] + le % W, gj = loy[k] + le / W;
      cx<R> bv{0, 0}, dv{0, 0};
      MgcCell<R> cl{};
      if (gi >= 0 && gi < d.nx && gj >= 0 && gj < d.ny) {
        const int c = gi + d.nx * gj;
        dv = ch.dinv[k][c];
        if (k == 0) bv = ch.b[0][c];
        cl = mgc_load_cell<Op, R>(ch.op[k], gi, gj);
      }
      sd[e] = dv;
      sc[e] = cl;
      if (k == 0) {
        sb[e] = bv;
        sx[e] = om * (dv * bv);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < MGC_F; ++k) {
    if (k >= nl) break;
    const LevelDims f = ch.d[k], c = ch.d[k + 1];
    const int Wf = side[k], W = side[k + 1];
    const cx<R>* bf = sb + off[k];
    const cx<R>* xf = sx + off[k];
    const MgcCell<R>* cf = sc + off[k];
    // this block's own cells of level k + 1 (the rest of its region is ring)
    const int sh = nl - (k + 1);
    const int ox0 = (int)blockIdx.x * T << sh, oy0 = (int)blockIdx.y * T << sh;
    const int ow = T << sh;
    for (int e = threadIdx.x; e < W * W; e += BS) {
      const int pi = e % W, pj = e / W;
      const int PI = lox[k + 1] + pi, PJ = loy[k + 1] + pj;
      cx<R> v{0, 0};
      const bool in = PI >= 0 && PI < c.nx && PJ >= 0 && PJ < c.ny;
      if (in) {
        cx<R> r[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 2 * PI + (q & 1), j = 2 * PJ + (q >> 1);
          r[q] = cx<R>{0, 0};
          if (i < f.nx && j < f.ny) {
            const int lc = (i - lox[k]) + Wf * (j - loy[k]);
            const cx<R> ax = mgc_apply(cf[lc], i, j, f.nx, f.ny, tr, xf[lc], xf[lc - 1], xf[lc + 1], xf[lc - Wf],
                                       xf[lc + Wf]);
            r[q] = bf[lc] - ax;
          }
        }
        v = (r[0] + r[1]) + (r[2] + r[3]);
      }
      if (k + 1 < nl) {
        sb[off[k + 1] + e] = v;
        sx[off[k + 1] + e] = om * (sd[off[k + 1] + e] * v);
      }
      int fl = flag;
      hold(v, fl);
      if (in && !fl && PI >= ox0 && PI < ox0 + ow && PJ >= oy0 && PJ < oy0 + ow) ch.out[k + 1][PI + c.nx * PJ] = v;
    }
    __syncthreads();
  }
}

// Prolongation chain: x of level 0 from x of level nl.  Block tile T0 x T0 of
// level 0; level k needs x2 = om D^-1 b + P x_{k+1} on its region and a ring,
// and x_{k+1} on the parents of those cells.
template <int T0> __host__ __device__ constexpr int mgc_up_reg(int k) {   // side of level k's region, at most
  return k == 0 ? T0 : (mgc_up_reg<T0>(k - 1) + 2) / 2 + 1;
}
template <int T0> constexpr int mgc_up_ext_cells() {
  int n = 0;
  for (int k = 0; k < MGC_F; ++k) n += (mgc_up_reg<T0>(k) + 2) * (mgc_up_reg<T0>(k) + 2);
  return n;
}
template <int T0> constexpr int mgc_up_reg_cells() {
  int n = 0;
  for (int k = 0; k <= MGC_F; ++k) n += mgc_up_reg<T0>(k) * mgc_up_reg<T0>(k);
  return n;
}
template <typename Op, typename R, int T0>
__global__ void __launch_bounds__(BS) k_mg_up_chain2d(MgChain<Op, R> ch, c128 tau, double omega,
                                                      const int* __restrict__ all_done) {
  constexpr int NE = mgc_up_ext_cells<T0>(), NR = mgc_up_reg_cells<T0>();
  __shared__ cx<R> sbe[NE], sde[NE], sx2[NE];   // b, D^-1, x2 over each level's region and ring
  __shared__ cx<R> sxr[NR];                     // x over each level's region (levels 1..nl)
  __shared__ MgcCell<R> scr[NR];                // stencil data over each level's region (levels 0..nl-1)
  const int flag = *all_done;
  const int nl = ch.nl;
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  // regions: reg[k] = [lo, lo + side); ext[k] = reg[k] and one ring
  int lox[MGC_F + 1], loy[MGC_F + 1], sw[MGC_F + 1], shh[MGC_F + 1], oe[MGC_F + 1], orr[MGC_F + 2];
  lox[0] = (int)blockIdx.x * T0;
  loy[0] = (int)blockIdx.y * T0;
  sw[0] = shh[0] = T0;
#pragma unroll
  for (int k = 0; k < MGC_F; ++k) {
    lox[k + 1] = (lox[k] - 1) >> 1;
    loy[k + 1] = (loy[k] - 1) >> 1;
    sw[k + 1] = ((lox[k] + sw[k]) >> 1) - lox[k + 1] + 1;
    shh[k + 1] = ((loy[k] + shh[k]) >> 1) - loy[k + 1] + 1;
  }
  oe[0] = 0;
#pragma unroll
  for (int k = 0; k < MGC_F; ++k) oe[k + 1] = oe[k] + (k < nl ? (sw[k] + 2) * (shh[k] + 2) : 0);
  orr[0] = 0;
#pragma unroll
  for (int k = 0; k <= MGC_F; ++k) orr[k + 1] = orr[k] + (k <= nl ? sw[k] * shh[k] : 0);
  // every input, all loads issued together: b and D^-1 over each level's
  // region and ring, the stencil data over each region, x of level nl
#pragma unroll
  for (int k = 0; k <= MGC_F; ++k) {
    if (k > nl) break;
    const LevelDims d = ch.d[k];
    if (k < nl) {
      const int W2 = sw[k] + 2, H2 = shh[k] + 2;
      for (int le = threadIdx.x; le < W2 * H2; le += BS) {
        const int gi = lox[k] - 1 + le % W2, gj = loy[k] - 1 + le / W2;
        cx<R> bv{0, 0}, dv{0, 0};
        if (gi >= 0 && gi < d.nx && gj >= 0 && gj < d.ny) {
          const int c = gi + d.nx * gj;
          bv = ch.b[k][c];
          dv = ch.dinv[k][c];
        }
        sbe[oe[k] + le] = bv;
        sde[oe[k] + le] = dv;
      }
    }
    const int W = sw[k], H = shh[k];
    for (int le = threadIdx.x; le < W * H; le += BS) {
      const int gi = lox[k] + le % W, gj = loy[k] + le / W;
      const bool in = gi >= 0 && gi < d.nx && gj >= 0 && gj < d.ny;
      if (k == nl) {
        sxr[orr[k] + le] = in ? ch.xc[gi + d.nx * gj] : cx<R>{0, 0};
      } else {
        MgcCell<R> cl{};
        if (in) cl = mgc_load_cell<Op, R>(ch.op[k], gi, gj);
        scr[orr[k] + le] = cl;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = MGC_F - 1; k >= 0; --k) {
    if (k >= nl) continue;
    const LevelDims f = ch.d[k];
    const int W2 = sw[k] + 2, H2 = shh[k] + 2;
    const int Wc = sw[k + 1];
    // x2 over the region and its ring
    for (int e = threadIdx.x; e < W2 * H2; e += BS) {
      const int gi = lox[k] - 1 + e % W2, gj = loy[k] - 1 + e / W2;
      cx<R> v{0, 0};
      if (gi >= 0 && gi < f.nx && gj >= 0 && gj < f.ny) {
        const int pl = ((gi >> 1) - lox[k + 1]) + Wc * ((gj >> 1) - loy[k + 1]);
        v = om * (sde[oe[k] + e] * sbe[oe[k] + e]) + sxr[orr[k + 1] + pl];
      }
      sx2[oe[k] + e] = v;
    }
    __syncthreads();
    // x = x2 + om D^-1 (b - A x2) over the region
    const int W = sw[k], H = shh[k];
    for (int e = threadIdx.x; e < W * H; e += BS) {
      const int li = e % W, lj = e / W;
      const int gi = lox[k] + li, gj = loy[k] + lj;
      cx<R> v{0, 0};
      const bool in = gi >= 0 && gi < f.nx && gj >= 0 && gj < f.ny;
      if (in) {
        const int lc = oe[k] + (li + 1) + W2 * (lj + 1);
        const cx<R> xi = sx2[lc];
        const cx<R> ax = mgc_apply(scr[orr[k] + e], gi, gj, f.nx, f.ny, tr, xi, sx2[lc - 1], sx2[lc + 1],
                                   sx2[lc - W2], sx2[lc + W2]);
        v = xi + om * (sde[lc] * (sbe[lc] - ax));
      }
      if (k > 0) {
        sxr[orr[k] + e] = v;
      } else {
        int fl = flag;
        hold(v, fl);
        if (in && !fl) ch.out[0][gi + f.nx * gj] = v;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------- 3-D legs, marching the planes --
// The grid legs of a 3-D level with the x-y neighbours taken from LDS: a block
// owns a T3X x T3Y tile of cells (a thread per cell) and one chunk of LT lanes
// (blockIdx.x = tile column * C + chunk), and marches through ZB planes.  On
// each plane the block forms the smoothed value (x1 = omega D^-1 b, plus the
// prolongated coarse solution on the way up) of its cells and of the tile's
// ring of 2 T3X + 2 T3Y neighbours once, in LDS; the x-y neighbours of the
// stencil come from there, the z neighbours from the thread's registers (its
// cell's values on the planes below and above).  Each input is read about once
// (plus the ring and the two planes past the block's ends) where the one-cell
// kernels read it once per stencil point, which made them bound by the
// requests their vector caches serve rather than by HBM.  Same arithmetic per
// lane as k_mg_down_lanes / k_mg_up_lanes: slots of neighbours outside the
// grid hold zeros and their face coefficients are zero.
constexpr int T3X = 64, T3Y = 8, T3T = T3X * T3Y, T3H = 2 * (T3X + T3Y);

// This thread's ring cell (tile coordinates, -1 .. T3X / T3Y), or hx = -2.
__device__ __forceinline__ void tile3_ring(int t, int& hx, int& hy) {
  hx = hy = -2;
  if (t >= T3H) return;
  if (t < T3X) { hx = t; hy = -1; }
  else if (t < 2 * T3X) { hx = t - T3X; hy = T3Y; }
  else if (t < 2 * T3X + T3Y) { hx = -1; hy = t - 2 * T3X; }
  else { hx = T3X; hy = t - 2 * T3X - T3Y; }
}

template <typename Op, typename R, int LT, bool UP>
__global__ void __launch_bounds__(T3T) k_mg_leg_tile3(Op op, LevelDims f, LevelDims cd, c128 tau, double omega,
                                                      int lS, int C, int ZB, const cx<R>* __restrict__ b,
                                                      const cx<R>* __restrict__ dinv,
                                                      const cx<R>* __restrict__ xc, cx<R>* __restrict__ out,
                                                      const CgScal* __restrict__ sc,
                                                      const int* __restrict__ all_done) {
  __shared__ cx<R> sh[T3Y + 2][T3X + 2][LT];
  __shared__ cx<R> stg[UP ? 1 : T3Y][UP ? 1 : T3X][LT];   // restriction: the children's sums
  const int flag = *all_done;
  int bxc, by, bz;
  xcd_block3(bxc, by, bz);
  const int ch = bxc % C, bx = bxc / C;
  if (!chunk_live<LT>(sc, ch * LT)) return;   // the block's chunk has stopped (uniform)
  const int tx = (int)threadIdx.x % T3X, ty = (int)threadIdx.x / T3X;
  const int i = bx * T3X + tx, j = by * T3Y + ty;
  const bool own = i < f.nx && j < f.ny;
  const int z0 = bz * ZB, z1 = min(z0 + ZB, f.nz);
  int hx, hy;
  tile3_ring((int)threadIdx.x, hx, hy);
  const int hi = bx * T3X + hx, hj = by * T3Y + hy;
  const bool ring = hx > -2 && hi >= 0 && hi < f.nx && hj >= 0 && hj < f.ny;
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  const int l0 = ch * LT;
  using Raw = Tile3Raw<R, LT, UP>;
  auto load = [&](int ci, int cj, int k, Raw& r) {
    const int c = ci + f.nx * (cj + f.ny * k);
    r.d = dinv[c];
    const long bb = ((long)c << lS) + l0;
#pragma unroll
    for (int l = 0; l < LT; ++l) r.b[l] = b[bb + l];
    if constexpr (UP) {
      const int pc = (ci >> 1) + cd.nx * ((cj >> 1) + cd.ny * (k >> 1));
      const long pb = ((long)pc << lS) + l0;
#pragma unroll
      for (int l = 0; l < LT; ++l) r.x[l] = xc[pb + l];
    }
  };
  // smoothed value: x1 = om D^-1 b, plus x_c of the parent on the way up
  auto smooth = [&](const Raw& r, cx<R> (&o)[LT]) {
#pragma unroll
    for (int l = 0; l < LT; ++l) {
      if constexpr (UP) o[l] = om * (r.d * r.b[l]) + r.x[l];
      else o[l] = om * (r.d * r.b[l]);
    }
  };
  auto zero = [](cx<R> (&o)[LT]) {
#pragma unroll
    for (int l = 0; l < LT; ++l) o[l] = cx<R>{0, 0};
  };
  cx<R> xp[LT], xcur[LT], xn[LT], bcur[LT], hv[LT], acc[LT];
  cx<R> dcur{0, 0};
  Raw rn, hr;
  zero(xp);
  zero(xcur);
  zero(bcur);
  zero(acc);
  if (ring) load(hi, hj, z0, hr);
  if (own) {
    if (z0 > 0) {
      load(i, j, z0 - 1, rn);
      smooth(rn, xp);
    }
    load(i, j, z0, rn);
    smooth(rn, xcur);
#pragma unroll
    for (int l = 0; l < LT; ++l) bcur[l] = rn.b[l];
    dcur = rn.d;
  }
  for (int k = z0; k < z1; ++k) {
    // the ring's values on this plane (inputs loaded on the previous step),
    // then every load this step and the next need, issued together: the
    // ring's inputs on the next plane, this cell's on the next plane and
    // this cell's faces and mass
    zero(hv);
    if (ring) smooth(hr, hv);
    if (ring && k + 1 < z1) load(hi, hj, k + 1, hr);
    const bool up_in = own && k + 1 < f.nz;
    if (up_in) load(i, j, k + 1, rn);
    const int c = i + f.nx * (j + f.ny * k);
    int idx[Op::NB];
    R fo[Op::NB];
    R fsum = 0;
    R m = 0;
    if (own) {
      op.template stencil_at<R>(i, j, k, c, idx, fo, fsum);
      m = (R)op.mass(c);
    }
    __syncthreads();   // the previous plane's reads of sh are done
#pragma unroll
    for (int l = 0; l < LT; ++l) sh[ty + 1][tx + 1][l] = xcur[l];
    if (hx > -2) {
#pragma unroll
      for (int l = 0; l < LT; ++l) sh[hy + 1][hx + 1][l] = hv[l];
    }
    __syncthreads();
    zero(xn);
    if (up_in) smooth(rn, xn);
    cx<R> v[LT];
    zero(v);
    if (own) {
#pragma unroll
      for (int l = 0; l < LT; ++l) {
        const cx<R> xi = xcur[l];
        cx<R> ax = fsum * xi + m * (tr * xi);
        ax = ax - fo[0] * sh[ty + 1][tx][l];
        ax = ax - fo[1] * sh[ty + 1][tx + 2][l];
        ax = ax - fo[2] * sh[ty][tx + 1][l];
        ax = ax - fo[3] * sh[ty + 2][tx + 1][l];
        ax = ax - fo[4] * xp[l];
        ax = ax - fo[5] * xn[l];
        if constexpr (UP) v[l] = xi + om * (dcur * (bcur[l] - ax));
        else v[l] = bcur[l] - ax;
      }
    }
    if constexpr (UP) {
      int fl = flag;
      hold(v[0], fl);
      if (own && !fl) {
        cx<R>* o = out + ((long)c << lS) + l0;
#pragma unroll
        for (int l = 0; l < LT; ++l) o[l] = v[l];
      }
    } else {
#pragma unroll
      for (int l = 0; l < LT; ++l) acc[l] = acc[l] + v[l];
      if ((k & 1) || k + 1 == z1) {
        // both child planes of coarse plane k / 2 are in: sum the 2 x 2
        // children in the plane and store the coarse cell
#pragma unroll
        for (int l = 0; l < LT; ++l) stg[ty][tx][l] = acc[l];
        __syncthreads();
        const int I = i >> 1, J = j >> 1;
        if (!(tx & 1) && !(ty & 1) && I < cd.nx && J < cd.ny) {
          cx<R> s2[LT];
#pragma unroll
          for (int l = 0; l < LT; ++l)
            s2[l] = (stg[ty][tx][l] + stg[ty][tx + 1][l]) + (stg[ty + 1][tx][l] + stg[ty + 1][tx + 1][l]);
          int fl = flag;
          hold(s2[0], fl);
          if (!fl) {
            cx<R>* o = out + ((long)(I + cd.nx * (J + cd.ny * (k >> 1))) << lS) + l0;
#pragma unroll
            for (int l = 0; l < LT; ++l) o[l] = s2[l];
          }
        }
        zero(acc);
      }
    }
#pragma unroll
    for (int l = 0; l < LT; ++l) {
      xp[l] = xcur[l];
      xcur[l] = xn[l];
      if (up_in) bcur[l] = rn.b[l];
    }
    if (up_in) dcur = rn.d;
  }
}

// The product w = A u and the next iteration's forms (k_cgmg_post_lanes) on the
// same plane-marching tiles: u of the tile and its ring in LDS per plane, u of
// the planes below and above in registers.  Block partials of the forms go to
// row (tile index) of partOut, lanes l0 .. l0 + LT - 1 of it written by the
// block of that chunk, so the rows number the tiles (fewer than the one-cell
// kernel's blocks; the fold of the partials is told how many).
template <typename Op, typename R, int LT>
__global__ void __launch_bounds__(T3T) k_cgmg_post_tile3(Op op, LevelDims f, c128 tau, int lS, int C, int ZB,
                                                         const CgScal* __restrict__ sc,
                                                         const cx<R>* __restrict__ r, const cx<R>* __restrict__ u,
                                                         cx<R>* __restrict__ w, c128* __restrict__ partOut,
                                                         const int* __restrict__ all_done) {
  __shared__ cx<R> sh[T3Y + 2][T3X + 2][LT];
  __shared__ c128 red[T3T / WAVE][3 * LT];
  const int flag = *all_done;
  int bxc, by, bz;
  xcd_block3(bxc, by, bz);
  const int ch = bxc % C, bx = bxc / C;
  const int tx = (int)threadIdx.x % T3X, ty = (int)threadIdx.x / T3X;
  const int i = bx * T3X + tx, j = by * T3Y + ty;
  const bool own = i < f.nx && j < f.ny;
  const int z0 = bz * ZB, z1 = min(z0 + ZB, f.nz);
  int hx, hy;
  tile3_ring((int)threadIdx.x, hx, hy);
  const int hi = bx * T3X + hx, hj = by * T3Y + hy;
  const bool ring = hx > -2 && hi >= 0 && hi < f.nx && hj >= 0 && hj < f.ny;
  const cx<R> tr = cvt<R>(tau);
  const int l0 = ch * LT;
  const int plane = f.nx * f.ny;
  bool live[LT];
#pragma unroll
  for (int l = 0; l < LT; ++l) live[l] = !sc[l0 + l].done;
  auto load = [&](int c, cx<R> (&o)[LT]) {
    const long bb = ((long)c << lS) + l0;
#pragma unroll
    for (int l = 0; l < LT; ++l) o[l] = u[bb + l];
  };
  auto zero = [](cx<R> (&o)[LT]) {
#pragma unroll
    for (int l = 0; l < LT; ++l) o[l] = cx<R>{0, 0};
  };
  c128 acc[3][LT];
#pragma unroll
  for (int l = 0; l < LT; ++l) acc[0][l] = acc[1][l] = acc[2][l] = c128{0.0, 0.0};
  cx<R> up_[LT], uc[LT], un[LT], hu[LT], hv[LT];
  zero(up_);
  zero(uc);
  zero(hu);
  const int c0 = i + f.nx * j;
  if (ring) load(hi + f.nx * (hj + f.ny * z0), hu);
  if (own) {
    if (z0 > 0) load(c0 + plane * (z0 - 1), up_);
    load(c0 + plane * z0, uc);
  }
  for (int k = z0; k < z1; ++k) {
#pragma unroll
    for (int l = 0; l < LT; ++l) hv[l] = hu[l];
    if (ring && k + 1 < z1) load(hi + f.nx * (hj + f.ny * (k + 1)), hu);
    const bool up_in = own && k + 1 < f.nz;
    zero(un);
    if (up_in) load(c0 + plane * (k + 1), un);
    const int c = c0 + plane * k;
    int idx[Op::NB];
    R fo[Op::NB];
    R fsum = 0, m = 0;
    cx<R> rr[LT];
    zero(rr);
    if (own) {
      op.template stencil_at<R>(i, j, k, c, idx, fo, fsum);
      m = (R)op.mass(c);
      const long bb = ((long)c << lS) + l0;
#pragma unroll
      for (int l = 0; l < LT; ++l) rr[l] = r[bb + l];
    }
    __syncthreads();   // the previous plane's reads of sh are done
#pragma unroll
    for (int l = 0; l < LT; ++l) sh[ty + 1][tx + 1][l] = uc[l];
    if (hx > -2) {
#pragma unroll
      for (int l = 0; l < LT; ++l) sh[hy + 1][hx + 1][l] = hv[l];
    }
    __syncthreads();
    if (own && !flag) {
      cx<R> ww[LT];
#pragma unroll
      for (int l = 0; l < LT; ++l) {
        ww[l] = fsum * uc[l] + m * (tr * uc[l]);
        ww[l] = ww[l] - fo[0] * sh[ty + 1][tx][l];
        ww[l] = ww[l] - fo[1] * sh[ty + 1][tx + 2][l];
        ww[l] = ww[l] - fo[2] * sh[ty][tx + 1][l];
        ww[l] = ww[l] - fo[3] * sh[ty + 2][tx + 1][l];
        ww[l] = ww[l] - fo[4] * up_[l];
        ww[l] = ww[l] - fo[5] * un[l];
      }
      const long bb = ((long)c << lS) + l0;
#pragma unroll
      for (int l = 0; l < LT; ++l) {
        if (!live[l]) continue;
        w[bb + l] = ww[l];
        const c128 rd = cvt<double>(rr[l]), ud = cvt<double>(uc[l]);
        acc[0][l] = acc[0][l] + rd * ud;
        acc[1][l] = acc[1][l] + cvt<double>(ww[l]) * ud;
        acc[2][l].re += abs2(rd);
      }
    }
#pragma unroll
    for (int l = 0; l < LT; ++l) {
      up_[l] = uc[l];
      uc[l] = un[l];
    }
  }
  if (flag) return;
  // block partials: a wave sum per (form, lane), then the waves in order
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int l = 0; l < LT; ++l) {
      const c128 v = wave_sum_strided(acc[q][l], 1);
      if (lane == 0) red[wv][q * LT + l] = v;
    }
  __syncthreads();
  if ((int)threadIdx.x < 3 * LT) {
    const int e = threadIdx.x, q = e / LT, l = e - q * LT;
    c128 a = red[0][e];
    for (int v = 1; v < T3T / WAVE; ++v) a = a + red[v][e];
    const int gxt = (int)gridDim.x / C;
    const long tile = bx + (long)gxt * (by + (long)gridDim.y * bz);
    partOut[(tile * 3 + q) * (1 << lS) + l0 + l] = a;
  }
}

// The coarse end of the V-cycle in one workgroup: levels t..L-1 (right-hand
// side of level t from global memory, solution of level t back to it), every
// level's b and x in LDS, a barrier between legs.  Saves two launches per
// coarse level, which are all latency.  The levels' coefficients (D^-1, cell
// masses, faces) come packed in one block that the workgroup copies into LDS
// at its start, all loads in flight at once, so that no leg after that waits
// on global memory.
constexpr int MG_MAXL = 14;
constexpr int MG_TAIL_THREADS = 1024;
// Dynamic LDS of the tail: the default budget, and the largest one (gfx950
// gives a workgroup 160 KB; the level table takes static LDS beside it).
// Each size has its own instantiation, whose staging registers scale with it.
constexpr int MG_TAIL_LDS = 63 * 1024;
constexpr int MG_TAIL_LDS_MAX = 159 * 1024;
constexpr int MG_MAXSEG = 5 * MG_MAXL;
struct MgTailLevel {
  int nx, ny, nz;
  int lpx, lpy;  // log2 of the power-of-two row and column pitches the phases walk (no index division)
  int off;       // LDS offset (elements) of b; x follows it (n S each)
  int doff;      // LDS byte offset of D^-1
  int moff;      // LDS byte offset of the cell masses (doubles)
  int foff[3];   // LDS byte offsets of the face arrays along x, y, z
};
struct MgTail {
  int T;                        // levels in the tail
  int pack_lds;                 // LDS byte offset of the packed block
  int pack_words;               // its length in 4-byte words
  MgTailLevel lv[MG_MAXL];
};

// One segment of the packed block: `words` 4-byte words copied from src, or
// (src null) words / 2 doubles equal to `fill`, at byte offset dst.
struct MgSeg {
  const void* src;
  int dst, words;
  double fill;
};
struct MgPack {
  int nseg;
  MgSeg seg[MG_MAXSEG];
};
// One block per segment.
__global__ void __launch_bounds__(BS) k_mg_pack(MgPack p, unsigned* __restrict__ dst) {
  const MgSeg s = p.seg[blockIdx.x];
  unsigned* d = dst + s.dst / 4;
  if (s.src) {
    const unsigned* src = static_cast<const unsigned*>(s.src);
    for (int j = threadIdx.x; j < s.words; j += BS) d[j] = src[j];
  } else {
    double* dd = reinterpret_cast<double*>(d);
    for (int j = threadIdx.x; j < s.words / 2; j += BS) dd[j] = s.fill;
  }
}

// Lanes are independent systems: the launch may split them over 2^(lSg - lS)
// workgroups, workgroup g taking lanes g 2^lS .. (g + 1) 2^lS - 1 of the 2^lSg
// that btop and xtop interleave (lS: lanes per workgroup, the layout in LDS).
template <typename Op, typename R, int CAP>
__global__ void __launch_bounds__(MG_TAIL_THREADS) k_mg_tail(MgTail a, c128 tau, double omega, int lS, int lSg,
                                                             const unsigned* __restrict__ pack,
                                                             const cx<R>* __restrict__ btop, cx<R>* __restrict__ xtop,
                                                             const CgScal* __restrict__ sc,
                                                             const int* __restrict__ all_done) {
  using F = typename std::remove_const<typename std::remove_pointer<decltype(Op::tx)>::type>::type;
  constexpr int NW = CAP / 4 / MG_TAIL_THREADS + 1;                        // packed words per thread
  constexpr int NB0 = CAP / (2 * (int)sizeof(cx<R>)) / MG_TAIL_THREADS + 1; // top rhs elements per thread
  constexpr int NP = (int)(sizeof(MgTailLevel) * MG_MAXL / 4);                    // level table words
  static_assert(NP <= MG_TAIL_THREADS, "level table");
  extern __shared__ __align__(16) char lds_raw[];
  __shared__ MgTailLevel lv[MG_MAXL];
  cx<R>* sh = reinterpret_cast<cx<R>*>(lds_raw);
  const int flag = *all_done;
  const int tid = threadIdx.x;
  // several lanes: the workgroup's lanes still running (loaded with everything
  // else; one lane stops with the all-done flag)
  const int run = lSg > 0 && tid < (1 << lS) && !sc[((int)blockIdx.x << lS) + tid].done;
  const int T = a.T;
  const int n0 = (a.lv[0].nx * a.lv[0].ny * a.lv[0].nz) << lS;
  // element j of the workgroup's top level in the interleaved global arrays
  const int g0 = (int)blockIdx.x << lS, lmask = (1 << lS) - 1;
  auto gidx = [&](int j) { return ((j >> lS) << lSg) + g0 + (j & lmask); };
  {
    // every global load of the kernel is issued here, at once: the level
    // table, the packed coefficients and the top right-hand side
    const int pw0 = tid < NP ? reinterpret_cast<const int*>(a.lv)[tid] : 0;
    unsigned wv[NW];
    cx<R> bv[NB0];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int j = tid + k * MG_TAIL_THREADS;
      wv[k] = j < a.pack_words ? pack[j] : 0u;
    }
#pragma unroll
    for (int k = 0; k < NB0; ++k) {
      const int j = tid + k * MG_TAIL_THREADS;
      bv[k] = j < n0 ? btop[gidx(j)] : cx<R>{0, 0};
    }
    if (tid < NP) reinterpret_cast<int*>(lv)[tid] = pw0;
    unsigned* pw = reinterpret_cast<unsigned*>(lds_raw + a.pack_lds);
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int j = tid + k * MG_TAIL_THREADS;
      if (j < a.pack_words) pw[j] = wv[k];
    }
#pragma unroll
    for (int k = 0; k < NB0; ++k) {
      const int j = tid + k * MG_TAIL_THREADS;
      if (j < n0) sh[j] = bv[k];
    }
  }
  if (flag) return;   // uniform: the whole workgroup leaves
  __syncthreads();
  if (lSg > 0 && !__syncthreads_or(run)) return;   // every lane of the workgroup has stopped
  const int S = 1 << lS;
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  constexpr int nth = MG_TAIL_THREADS;
  auto dims = [&](int k) { return LevelDims{lv[k].nx, lv[k].ny, lv[k].nz}; };
  auto lop = [&](int k) {
    Op o{};
    o.nx = lv[k].nx;
    o.ny = lv[k].ny;
    o.tx = reinterpret_cast<const F*>(lds_raw + lv[k].foff[0]);
    o.ty = reinterpret_cast<const F*>(lds_raw + lv[k].foff[1]);
    if constexpr (Op::NB == 6) {
      o.nz = lv[k].nz;
      o.tz = reinterpret_cast<const F*>(lds_raw + lv[k].foff[2]);
    }
    o.mdiag = reinterpret_cast<const double*>(lds_raw + lv[k].moff);
    return o;
  };
  auto ldinv = [&](int k) { return reinterpret_cast<const cx<R>*>(lds_raw + lv[k].doff); };
  // downward legs: as on the grid, one thread per (coarse cell, lane, fine
  // child) and a cross-lane sum over the children
  constexpr int D = Op::NB / 2;
  constexpr int Q = 1 << D;
  for (int k = 0; k + 1 < T; ++k) {
    const LevelDims f = dims(k), c = dims(k + 1);
    const Op o = lop(k);
    const cx<R>* bk = sh + lv[k].off;
    cx<R>* bc = sh + lv[k + 1].off;
    const cx<R>* dk = ldinv(k);
    // threads walk the coarse grid with power-of-two pitches: coordinates by
    // shifts and masks, padding threads idle
    const int lpx = lv[k + 1].lpx, lpy = lv[k + 1].lpy;
    const int total = (c.nz << (lpx + lpy)) << (lS + D);
    for (int j = tid; j < total; j += nth) {   // whole groups of 2^d lanes in or out
      const int q = j & (Q - 1), rl = (j >> D) & (S - 1), r2 = j >> (D + lS);
      const int Ix = r2 & ((1 << lpx) - 1), r3 = r2 >> lpx;
      const int Jy = r3 & ((1 << lpy) - 1), Lz = r3 >> lpy;
      if (Ix >= c.nx || Jy >= c.ny) continue;
      const int x = 2 * Ix + (q & 1), y = 2 * Jy + ((q >> 1) & 1), z = 2 * Lz + (q >> 2);
      auto gb = [&](int n) { return bk[(n << lS) + rl]; };
      auto gd = [&](int n) { return dk[n]; };
      cx<R> v{0, 0};
      if (x < f.nx && y < f.ny && z < f.nz) v = mg_down_fine<Op, R>(o, x, y, z, x + f.nx * (y + f.ny * z), tr, om, gb, gd);
      v = group_sum<Q>(v);
      if (q == 0) bc[((Ix + c.nx * (Jy + c.ny * Lz)) << lS) + rl] = v;
    }
    __syncthreads();
  }
  {
    const int k = T - 1;
    const int nk = dims(k).n() << lS;
    const cx<R>* dk = ldinv(k);
    for (int j = tid; j < nk; j += nth) sh[lv[k].off + nk + j] = dk[j >> lS] * sh[lv[k].off + j];
  }
  __syncthreads();
  for (int k = T - 2; k >= 0; --k) {
    const LevelDims f = dims(k), c = dims(k + 1);
    const Op o = lop(k);
    const int nk = f.n() << lS, nc = c.n() << lS;
    const cx<R>* bk = sh + lv[k].off;
    cx<R>* xk = sh + lv[k].off + nk;
    const cx<R>* xc = sh + lv[k + 1].off + nc;
    const cx<R>* dk = ldinv(k);
    const int lpx = lv[k].lpx, lpy = lv[k].lpy;
    const int total = (f.nz << (lpx + lpy)) << lS;
    for (int j = tid; j < total; j += nth) {
      const int rl = j & (S - 1), r2 = j >> lS;
      const int i = r2 & ((1 << lpx) - 1), r3 = r2 >> lpx;
      const int jy = r3 & ((1 << lpy) - 1), kz = r3 >> lpy;
      if (i >= f.nx || jy >= f.ny) continue;
      const int cell = i + f.nx * (jy + f.ny * kz);
      auto gb = [&](int n) { return bk[(n << lS) + rl]; };
      auto gd = [&](int n) { return dk[n]; };
      auto gx = [&](int n) { return xc[(n << lS) + rl]; };
      xk[(cell << lS) + rl] = mg_up_cell<Op, R>(o, f, c, i, jy, kz, cell, tr, om, gb, gd, gx);
    }
    __syncthreads();
  }
  for (int j = tid; j < n0; j += nth) xtop[gidx(j)] = sh[n0 + j];
}

// The coarsest level solved on the grid (only when even its lanes exceed the
// tail's LDS): x = D^-1 b.
template <typename R>
__global__ void __launch_bounds__(BS) k_mg_scale_grid(long N, int lS, const cx<R>* __restrict__ dinv,
                                                      const cx<R>* __restrict__ b, cx<R>* __restrict__ x,
                                                      const int* __restrict__ all_done) {
  if (*all_done) return;   // rare path (coarsest level beyond the tail): not worth the overlap
  for (long t = blockIdx.x * (long)BS + threadIdx.x; t < N; t += (long)gridDim.x * BS) x[t] = dinv[t >> lS] * b[t];
}

// ------------------------------------------------------- COCG with the V-cycle
// What a launch of the multigrid step does with a lane's FP64 iterate.  The
// update x += alpha p of an iteration may wait for the next launch: p is
// updated in place, so that launch still reads the same p, and it adds both
// terms in the order the immediate updates would, (x + a0 p) + alpha p' (the
// same values up to FP64 rounding).  x is then read and written every other
// iteration.  A lane
// defers at even launch parity only, so the lanes of a cache line of x skip
// together.  A residual replacement reads x + a0 p at the neighbours (the
// term stays deferred), a Jacobi step adds it, and the launch in which the
// lane stops adds it alone.
struct XPlan {
  c128 a0;      // coefficient of the deferred term
  bool fold;    // a deferred term a0 p is pending from the previous launch
  bool write;   // ITER: x is read and written in this launch
  bool stop;    // the lane stopped in this launch with a term to add
};
__device__ __forceinline__ XPlan x_plan(CgScal& s, bool was_done, int par) {
  XPlan xp;
  xp.fold = s.pend != 0;
  xp.a0 = s.apend;
  xp.write = true;
  xp.stop = false;
  if (s.done) {
    xp.stop = !was_done && xp.fold;
    s.pend = 0;
  } else if (s.mode == CG_ITER) {
    xp.write = xp.fold || par != 0;
    s.pend = xp.write ? 0 : 1;
    s.apend = xp.write ? c128{0.0, 0.0} : s.alpha;
  } else if (s.mode == CG_KX) {
    s.pend = 0;
  }
  return xp;
}

// Lane prologue of the step kernels: the flag, the previous partials and the
// state in one round trip, the sums, then the advance and the iterate's plan.
// Returns false when the launch has nothing to do (when every lane has
// stopped, true only while a stopping lane still has a term to add to x).
template <int CGB, bool ONE>
__device__ __forceinline__ bool cg_prologue(int lS, const CgCfg& cfg, const c128* __restrict__ partIn, int Gin,
                                            const CgScal* __restrict__ scIn, CgScal* __restrict__ scOut,
                                            int* __restrict__ all_done, CgScal& s, XPlan& xp, int par, bool lead) {
  const int S = 1 << lS;
  const int rl = ONE ? 0 : (int)threadIdx.x & (S - 1);
  const int flag = *all_done;
  constexpr int KMAX = 4;
  PartLoad<3, KMAX> PL;
  part_load<3, KMAX, CGB>(partIn, Gin, S, PL);
  s = scIn[rl];
  c128 tot[3];
  part_sum<3, KMAX, CGB>(partIn, Gin, S, PL, tot);
  // The flag is set by the lead block of the launch in which the last lanes
  // stop, while other blocks of that launch may still be starting: a block
  // that sees it while a lane was still running before this launch carries
  // on as the lead block does (its stopping lanes' deferred terms go into x).
  if (flag && __all(s.done != 0)) {
    if (lead && (int)threadIdx.x < S) scOut[threadIdx.x] = s;
    return false;
  }
  const bool was_done = s.done != 0;
  cg_advance(s, cfg, tot[0], tot[1], tot[2].re);
  xp = x_plan(s, was_done, par);
  const bool any_open = __any(!s.done);
  if (lead && (int)threadIdx.x < S) scOut[threadIdx.x] = s;
  if (!any_open) {
    if (lead && threadIdx.x == 0) *all_done = 1;
    return __any(xp.stop);
  }
  count_live(all_done, lead);
  return true;
}

// Vector part of one multigrid-COCG iteration (the V-cycle and the operator
// product follow in their own launches):
//   ITER: s' = w + beta s, r' = r - alpha s', p' = u + beta p, x += alpha p'
//         (u = B r from the previous V-cycle; the x update as XPlan says);
//   RR:   r' = v - (K + tau M) x in FP64, stored rounded (a round change of the
//         complex64 path; the V-cycle and the product then give the new round's
//         forms directly);
//   KX:   x += u, one preconditioned Richardson step on the iterate (u = B r of
//         the residual just formed), before a new residual.
template <typename Op, typename OpD, typename R, int CGB, bool ONE, bool MULTI>
__global__ void __launch_bounds__(CGB) k_cgmg_step(OpD opd, c128 tau, int n, int lS_,
                                                   const CgCfg* __restrict__ cfgp,
                                                   const cx<R>* __restrict__ v, const cx<R>* __restrict__ u,
                                                   const c128* __restrict__ partIn, int Gin,
                                                   const CgScal* __restrict__ scIn, CgScal* __restrict__ scOut,
                                                   CgVecs<R> vec, int par, int* __restrict__ all_done) {
  const CgCfg cfg = *cfgp;
  const int lS = ONE ? 0 : lS_;
  const int N = n << lS;
  const cx<R>* __restrict__ r0 = vec.r[par];
  const cx<R>* __restrict__ w0 = vec.w[par];
  const cx<R>* __restrict__ s0 = vec.s[par];
  cx<R>* __restrict__ r1 = vec.r[par ^ 1];
  cx<R>* __restrict__ s1 = vec.s[par ^ 1];
  const int t0 = xcd_tile(blockIdx.x, gridDim.x) * CGB + threadIdx.x;
  CgScal s;
  XPlan xp;
  if (!cg_prologue<CGB, ONE>(lS, cfg, partIn, Gin, scIn, scOut, all_done, s, xp, par, blockIdx.x == 0)) return;
  auto for_cells = [&](auto&& f) {
    if constexpr (MULTI) {
      for (int t = t0; t < N; t += gridDim.x * CGB) f(t);
    } else {
      if (t0 < N) f(t0);
    }
  };
  // x with the deferred term (the value the immediate updates give)
  auto xeff = [&](int t) {
    const c128 xv = vec.x[t];
    return xp.fold ? xv + xp.a0 * cvt<double>(vec.p[t]) : xv;
  };
  if (s.done) {
    if (xp.stop) for_cells([&](int t) { vec.x[t] = xeff(t); });
  } else if (s.mode == CG_ITER) {
    const cx<R> al = cvt<R>(s.alpha), be = cvt<R>(s.beta);
    const c128 al64 = s.alpha;
    for_cells([&](int t) {
      const cx<R> po = vec.p[t];
      const cx<R> sn = w0[t] + be * s0[t];
      const cx<R> pn = u[t] + be * po;
      r1[t] = r0[t] - al * sn;
      s1[t] = sn;
      vec.p[t] = pn;
      if (xp.write) {
        const c128 xv = vec.x[t];
        vec.x[t] = (xp.fold ? xv + xp.a0 * cvt<double>(po) : xv) + al64 * cvt<double>(pn);
      }
    });
  } else if (s.mode == CG_RR) {
    if constexpr (ONE) {
      auto gx = [&](int cc) { return xeff(cc); };
      for_cells([&](int t) {
        r1[t] = cvt<R>(cvt<double>(v[t]) - opd.template apply<double>(t, tau, gx));
        s1[t] = cx<R>{0, 0};
      });
    }
  } else if (s.mode == CG_KX) {
    for_cells([&](int t) { vec.x[t] = xeff(t) + cvt<double>(u[t]); });
  }
  if constexpr (!ONE) {
    // Residual replacements of several lanes: the block's (cell, lane) items
    // of the lanes in mode RR, compacted over all its threads (lanes fastest),
    // instead of each thread forming its own lane's: a launch in which a few
    // lanes replace theirs then pays their FP64 stencil once per block rather
    // than once per wave and cell.  Every wave holds every lane, so the
    // ballot gives the block's lane set.
    const int S = 1 << lS;
    const unsigned long long bal = __ballot(!s.done && s.mode == CG_RR);
    const unsigned long long lanes = S == 64 ? bal : bal & ((1ull << S) - 1);
    if (lanes == 0) return;   // uniform over the block
    __shared__ c128 rr_a0[64];
    __shared__ int rr_fold[64];
    if ((int)threadIdx.x < S) {
      rr_a0[threadIdx.x] = xp.a0;
      rr_fold[threadIdx.x] = xp.fold ? 1 : 0;
    }
    __syncthreads();
    const int nrr = __popcll(lanes);
    const int cpb = CGB >> lS;                              // cells per block and step
    const long base = (long)xcd_tile(blockIdx.x, gridDim.x) * CGB;
    const long stride = MULTI ? (long)gridDim.x * CGB : (long)N;
    const long steps = base < N ? (N - base + stride - 1) / stride : 0;
    const long items = steps * cpb * nrr;
    for (long it = threadIdx.x; it < items; it += CGB) {
      const int q = (int)(it % nrr);
      const long rest = it / nrr;
      const int j = (int)(rest % cpb);
      const long k = rest / cpb;
      const long c = ((base + k * stride) >> lS) + j;
      if (c >= n) continue;
      int lane;
      if (nrr == S) {
        lane = q;
      } else {
        unsigned long long mm = lanes;
        for (int z = 0; z < q; ++z) mm &= mm - 1;
        lane = __builtin_ctzll(mm);
      }
      const bool fo = rr_fold[lane] != 0;
      const c128 a0 = rr_a0[lane];
      auto gx = [&](int cc) {
        const long e = ((long)cc << lS) + lane;
        const c128 xv = vec.x[e];
        return fo ? xv + a0 * cvt<double>(vec.p[e]) : xv;
      };
      const long e = (c << lS) + lane;
      r1[e] = cvt<R>(cvt<double>(v[e]) - opd.template apply<double>((int)c, tau, gx));
      s1[e] = cx<R>{0, 0};
    }
  }
}

// The step fused with the V-cycle's first restriction, for one lane (S = 1):
// launched on the restriction's grid (one thread per fine cell, children of a
// coarse cell in adjacent lanes), every block runs the step's prologue, each
// thread updates its own cell as k_cgmg_step does and restricts the new
// residual, whose values at the stencil neighbours it forms from their old
// r, w, s (ITER) or their FP64 residual (RR) with the step's own expressions,
// so they are the values the step stores.  In any other mode the stored r'
// is restricted, as the separate kernels do.  Saves the step's launch and its
// second read of r'.
template <typename Op, typename OpD, typename R>
__global__ void __launch_bounds__(BS) k_cgmg_step_down(Op op, OpD opd, LevelDims f, LevelDims c, c128 tau,
                                                       double omega, const CgCfg* __restrict__ cfgp,
                                                       const cx<R>* __restrict__ v,
                                                       const cx<R>* __restrict__ u,
                                                       const c128* __restrict__ partIn, int Gin,
                                                       const CgScal* __restrict__ scIn, CgScal* __restrict__ scOut,
                                                       CgVecs<R> vec, int par, const cx<R>* __restrict__ dinv,
                                                       cx<R>* __restrict__ out, int* __restrict__ all_done) {
  const CgCfg cfg = *cfgp;
  constexpr int D = Op::NB / 2;
  constexpr int Q = 1 << D;
  int bx, J, L;
  xcd_block3(bx, J, L);
  const bool lead = (blockIdx.x | blockIdx.y | blockIdx.z) == 0;
  CgScal s;
  XPlan xp;
  if (!cg_prologue<BS, true>(0, cfg, partIn, Gin, scIn, scOut, all_done, s, xp, par, lead)) return;
  const int t = bx * BS + threadIdx.x;
  if (t >= (c.nx << D)) return;   // after the prologue's barriers; whole groups of 2^d lanes
  const int q = t & (Q - 1), I = t >> D;
  const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = 2 * L + (q >> 2);
  const bool in = i < f.nx && j < f.ny && k < f.nz;
  const int cell = i + f.nx * (j + f.ny * k);
  // x with the deferred term (the value the immediate updates give)
  auto xeff = [&](int e) {
    const c128 xv = vec.x[e];
    return xp.fold ? xv + xp.a0 * cvt<double>(vec.p[e]) : xv;
  };
  if (s.done) {   // only a lane that stops here with a deferred term
    if (in) vec.x[cell] = xeff(cell);
    return;
  }
  const cx<R>* __restrict__ r0 = vec.r[par];
  const cx<R>* __restrict__ w0 = vec.w[par];
  const cx<R>* __restrict__ s0 = vec.s[par];
  cx<R>* __restrict__ r1 = vec.r[par ^ 1];
  cx<R>* __restrict__ s1 = vec.s[par ^ 1];
  const cx<R> tr = cvt<R>(tau);
  const R om = (R)omega;
  auto gd = [&](int n) { return dinv[n]; };
  cx<R> res{0, 0};
  if (s.mode == CG_ITER) {
    const cx<R> al = cvt<R>(s.alpha), be = cvt<R>(s.beta);
    const c128 al64 = s.alpha;
    auto gb = [&](int n) { return r0[n] - al * (w0[n] + be * s0[n]); };
    if (in) {
      res = mg_down_fine<Op, R>(op, i, j, k, cell, tr, om, gb, gd);
      const cx<R> po = vec.p[cell];
      const cx<R> sn = w0[cell] + be * s0[cell];
      const cx<R> pn = u[cell] + be * po;
      r1[cell] = gb(cell);
      s1[cell] = sn;
      vec.p[cell] = pn;
      if (xp.write) {
        const c128 xv = vec.x[cell];
        vec.x[cell] = (xp.fold ? xv + xp.a0 * cvt<double>(po) : xv) + al64 * cvt<double>(pn);
      }
    }
  } else if (s.mode == CG_RR) {
    auto gx = [&](int cc) { return xeff(cc); };
    auto gb = [&](int n) { return cvt<R>(cvt<double>(v[n]) - opd.template apply<double>(n, tau, gx)); };
    if (in) {
      res = mg_down_fine<Op, R>(op, i, j, k, cell, tr, om, gb, gd);
      r1[cell] = gb(cell);
      s1[cell] = cx<R>{0, 0};
    }
  } else {
    auto gb = [&](int n) { return r1[n]; };
    if (in) {
      res = mg_down_fine<Op, R>(op, i, j, k, cell, tr, om, gb, gd);
      if (s.mode == CG_KX) vec.x[cell] = xeff(cell) + cvt<double>(u[cell]);
    }
  }
  res = group_sum<Q>(res);
  if (q == 0) out[I + c.nx * (J + c.ny * L)] = res;
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
  // The operands are loaded whatever the flags say (done lanes' sums are
  // masked out) and the done flag is read after their loads are issued, so
  // its round trip overlaps theirs.
  auto cell = [&](int c, int t) {
    constexpr int NB = Op::NB;
    int idx[NB];
    R fo[NB];
    R fsum;
    op.template stencil<R>(c, idx, fo, fsum);
    const cx<R> uc = gu(c);
    cx<R> ww = fsum * uc + (R)op.mass(c) * (tr * uc);
#pragma unroll
    for (int q = 0; q < NB; ++q) ww = ww - fo[q] * gu(idx[q]);
    cx<R> rr = r[t];
    int flag = *opaque(all_done);
    asm volatile("" : "+v"(ww.re), "+v"(ww.im), "+v"(rr.re), "+v"(rr.im), "+v"(flag));
    if (flag) return;
    const c128 rd = cvt<double>(rr), ud = cvt<double>(uc);
    if (live) {
      w[t] = ww;
      ag = ag + rd * ud;
      ad = ad + cvt<double>(ww) * ud;
      arr += abs2(rd);
    }
  };
  if constexpr (MULTI) {
    const SlabWalk sw(op, N, lS, CGB);
    for (long q = sw.first(); q < sw.end; q += sw.step) {
      const int c = sw.cell(q);
      cell(c, (c << lS) + rl);
    }
  } else {
    if (t0 < N) cell(t0 >> lS, t0);
  }
  if (*opaque(all_done)) return;
  c128 acc[3] = {ag, ad, {arr, 0.0}};
  block_partials<3, CGB>(acc, S, partOut + (size_t)blockIdx.x * 3 * S);
}

// k_cgmg_post with a thread per (cell, chunk of LT lanes): the stencil, the
// cell mass and the done flags are loaded once for LT lanes.  Same grid and
// partial layout [block][3][S]; item t is chunk t mod 2^lC (lC = lS - log2 LT)
// of cell t >> lC, and since the grid stride is a multiple of 2^lC a thread
// keeps its chunk.  Block partials: a strided wave sum per (form, lane) over
// the threads of one chunk, then the waves in order.
template <typename Op, typename R, int CGB, int LT>
__global__ void __launch_bounds__(CGB) k_cgmg_post_lanes(Op op, c128 tau, int n, int lS,
                                                         const CgScal* __restrict__ sc, const cx<R>* __restrict__ r,
                                                         const cx<R>* __restrict__ u, cx<R>* __restrict__ w,
                                                         c128* __restrict__ partOut, const int* __restrict__ all_done) {
  constexpr int NB = Op::NB;
  constexpr int NW = CGB / WAVE;
  constexpr int LLT = LT == 2 ? 1 : LT == 4 ? 2 : 3;
  const int S = 1 << lS, lC = lS - LLT, C = 1 << lC;
  const int ch = (int)threadIdx.x & (C - 1);
  const long items = (long)n << lC;
  bool live[LT];
  bool any = false;
#pragma unroll
  for (int j = 0; j < LT; ++j) {
    live[j] = !sc[ch * LT + j].done;
    any = any || live[j];
  }
  const cx<R> tr = cvt<R>(tau);
  c128 acc[3][LT];
#pragma unroll
  for (int j = 0; j < LT; ++j) acc[0][j] = acc[1][j] = acc[2][j] = c128{0.0, 0.0};
  const SlabWalk sw(op, items, lC, CGB);
  for (long t = any ? sw.first() : sw.end; t < sw.end; t += sw.step) {   // a stopped chunk loads nothing
    const int c = sw.cell(t);
    int idx[NB];
    R fo[NB];
    R fsum;
    op.template stencil<R>(c, idx, fo, fsum);
    const R m = (R)op.mass(c);
    const long base = ((long)c << lS) + ch * LT;
    cx<R> uc[LT], ww[LT], rr[LT];
#pragma unroll
    for (int j = 0; j < LT; ++j) {
      uc[j] = u[base + j];
      rr[j] = r[base + j];
      ww[j] = fsum * uc[j] + m * (tr * uc[j]);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const cx<R>* un = u + ((long)idx[q] << lS) + ch * LT;
#pragma unroll
      for (int j = 0; j < LT; ++j) ww[j] = ww[j] - fo[q] * un[j];
    }
    int flag = *opaque(all_done);
    asm volatile("" : "+v"(ww[0].re), "+v"(rr[0].re), "+v"(flag));
    if (flag) break;
#pragma unroll
    for (int j = 0; j < LT; ++j) {
      if (!live[j]) continue;
      w[base + j] = ww[j];
      const c128 rd = cvt<double>(rr[j]), ud = cvt<double>(uc[j]);
      acc[0][j] = acc[0][j] + rd * ud;
      acc[1][j] = acc[1][j] + cvt<double>(ww[j]) * ud;
      acc[2][j].re += abs2(rd);
    }
  }
  if (*opaque(all_done)) return;
  __shared__ c128 sh[NW][3][WAVE];
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
#pragma unroll
    for (int j = 0; j < LT; ++j) {
      const c128 v = wave_sum_strided(acc[q][j], C);
      if (lane < C) sh[wv][q][lane * LT + j] = v;
    }
  }
  lds_sync();
  if ((int)threadIdx.x < S) {
    c128* out = partOut + (size_t)blockIdx.x * 3 * S;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      c128 a = sh[0][q][threadIdx.x];
      for (int v = 1; v < NW; ++v) a = a + sh[v][q][threadIdx.x];
      out[q * S + threadIdx.x] = a;
    }
  }
}

}  // namespace shk
