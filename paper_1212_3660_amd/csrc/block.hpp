// Block FGMRES-Sh kernels: one shared block basis for S right-hand sides that
// share K and M (the block extension of Algorithms 3 and 4 for several
// right-hand sides, sections 5 and 7).
//
// Layout as everywhere: a block of S vectors is n x S, element (cell c,
// column r) at c*S + r.  The block Gram-Schmidt products V^H W and the updates
// W -= V C are dense complex contractions over the n cells; they run on the
// matrix cores (16x16x4 MFMA, FP32 on the complex64 path, FP64 on the
// complex128 path), with complex arithmetic split into real products:
//   Re(A^H B) = Ar^T Br + Ai^T Bi,  Im(A^H B) = Ar^T Bi - Ai^T Br,
//   Re(A C)   = Ar Cr - Ai Ci,      Im(A C)   = Ar Ci + Ai Cr.
// MFMA 16x16x4 lane layout (checked on gfx950): lane l = 16 g + m feeds
// A[m][g] and B[g][m]; it receives D[4 g + v][m], v = 0..3, from the FP32
// instruction and D[g + 4 v][m] from the FP64 one.
//
// The per-shift block least squares (FP64): each shift keeps the QR factors
// of its block Hessenberg Hbar(sigma;T) = [I;0] + Hbar (sigma I - T),
// updated one block column per outer step with Householder reflectors.
#pragma once
#include <type_traits>
#include "kernels.hpp"

namespace shk {

typedef float f4m __attribute__((ext_vector_type(4)));
typedef double d4m __attribute__((ext_vector_type(4)));
template <typename T> struct Acc4;
template <> struct Acc4<float> { using type = f4m; };
template <> struct Acc4<double> { using type = d4m; };

__device__ __forceinline__ f4m mfma16(float a, float b, f4m c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4m mfma16(double a, double b, d4m c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Row of D held in accumulator slot v by lane group g.
template <typename T> __device__ __forceinline__ int mfma_row(int g, int v) {
  return std::is_same<T, double>::value ? g + 4 * v : 4 * g + v;
}

// ------------------------------------------------- block projections ------
// Partial products C_i = A_i^H B over one chunk of cells, for block i of A
// (blocks astride elements apart) and one group of TN n-tiles: one wave per
// (chunk, block, n-tile group).  K runs over 4 cells per step: one MFMA on the
// real parts of A, one on the imaginary parts.  Output: part[((i * nch +
// chunk) * S + r) * S + r'] (TAcc complex), summed over chunks by
// k_blk_reduce in a fixed order.
template <typename TIn, typename TAcc, int TM, int TN>
__global__ void __launch_bounds__(64) k_blk_gram(const cx<TIn>* __restrict__ A, size_t astride,
                                                 const cx<TIn>* __restrict__ B, long n, int ch,
                                                 cx<TAcc>* __restrict__ part) {
  constexpr int S = 16 * TM;
  using V4 = typename Acc4<TAcc>::type;
  const int lane = threadIdx.x, g = lane >> 4, m = lane & 15;
  const int chunk = blockIdx.x, i = blockIdx.y, nb0 = blockIdx.z * TN;
  const int nch = gridDim.x;
  const cx<TIn>* Ai = A + (size_t)i * astride;
  const long c0 = (long)chunk * ch, c1 = c0 + ch < n ? c0 + ch : n;
  V4 re[TM][TN], im[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      re[a][b] = V4{0, 0, 0, 0};
      im[a][b] = V4{0, 0, 0, 0};
    }
  cx<TIn> av[TM], bv[TN];
  auto load = [&](long c) {
    const long cell = c + g;
    const bool ok = cell < c1;
#pragma unroll
    for (int a = 0; a < TM; ++a) av[a] = ok ? Ai[cell * S + 16 * a + m] : cx<TIn>{0, 0};
#pragma unroll
    for (int b = 0; b < TN; ++b) bv[b] = ok ? B[cell * S + 16 * (nb0 + b) + m] : cx<TIn>{0, 0};
  };
  for (long c = c0; c < c1; c += 4) {
    load(c);
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const TAcc ar = (TAcc)av[a].re, ai = (TAcc)av[a].im;
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const TAcc br = (TAcc)bv[b].re, bi = (TAcc)bv[b].im;
        re[a][b] = mfma16(ar, br, re[a][b]);
        re[a][b] = mfma16(ai, bi, re[a][b]);
        im[a][b] = mfma16(ar, bi, im[a][b]);
        im[a][b] = mfma16(ai, -br, im[a][b]);
      }
    }
  }
  cx<TAcc>* out = part + ((size_t)i * nch + chunk) * S * S;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * a + mfma_row<TAcc>(g, v), rp = 16 * (nb0 + b) + m;
        out[(size_t)r * S + rp] = cx<TAcc>{re[a][b][v], im[a][b][v]};
      }
}

// Sum of the chunk partials of nb blocks in chunk order (FP64), one thread per
// entry: block i's S x S result goes to H + i*S + ldh*col ((row, col) of the
// block, column-major with leading dimension ldh; add != 0 accumulates), and
// rounded to R into Cc[i] (row-major [r][r'], the update kernel's operand).
template <typename TAcc, typename R>
__global__ void __launch_bounds__(BS) k_blk_reduce(const cx<TAcc>* __restrict__ part, int nch, int S,
                                                   c128* __restrict__ H, int ldh, int add,
                                                   cx<R>* __restrict__ Cc) {
  const int e = blockIdx.x * BS + threadIdx.x;
  if (e >= S * S) return;
  const int i = blockIdx.y;
  const cx<TAcc>* p = part + (size_t)i * nch * S * S + e;
  c128 a0{0, 0}, a1{0, 0}, a2{0, 0}, a3{0, 0};
  int q = 0;
  for (; q + 4 <= nch; q += 4) {
    a0 = a0 + cvt<double>(p[(size_t)q * S * S]);
    a1 = a1 + cvt<double>(p[(size_t)(q + 1) * S * S]);
    a2 = a2 + cvt<double>(p[(size_t)(q + 2) * S * S]);
    a3 = a3 + cvt<double>(p[(size_t)(q + 3) * S * S]);
  }
  for (; q < nch; ++q) a0 = a0 + cvt<double>(p[(size_t)q * S * S]);
  const c128 s = (a0 + a1) + (a2 + a3);
  const int r = e / S, rp = e - r * S;
  if (H) {
    c128* h = H + (size_t)i * S + r + (size_t)ldh * rp;
    *h = add ? *h + s : s;
  }
  if (Cc) Cc[(size_t)i * S * S + e] = cvt<R>(s);
}

// Out = beta In + sgn sum_i A_i C_i over nb blocks (A_i n x S, C_i S x S
// row-major in Cc[i]), on the matrix cores.  A block of 4 waves shares C_i in
// LDS; each wave owns 16 TMC cells and all S columns.  The K dimension (the
// S rows r of C_i) is taken 16 at a time: lane group g holds r = r0 + 4g + t
// for t = 0..3 (a contiguous run of its cell's row), B[g][n] = C_i[r][n].
// In may alias Out (each wave reads only its own cells' rows of A and In).
template <typename TIn, typename TC, typename TOut, int TM, int TMC>
__global__ void __launch_bounds__(256) k_blk_update(const cx<TIn>* A, size_t astride, int nb,
                                                    const cx<TC>* __restrict__ Cc, const cx<TOut>* In,
                                                    cx<TOut>* Out, long n, TC beta, TC sgn) {
  constexpr int S = 16 * TM, LD = S + 1;
  using V4 = typename Acc4<TC>::type;
  extern __shared__ unsigned char blk_lds[];
  cx<TC>* sc = reinterpret_cast<cx<TC>*>(blk_lds);   // [S][LD]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, m = lane & 15;
  const long cw = ((long)blockIdx.x * 4 + wv) * (16 * TMC);   // first cell of this wave
  V4 re[TMC][TM], im[TMC][TM];
#pragma unroll
  for (int a = 0; a < TMC; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      re[a][b] = V4{0, 0, 0, 0};
      im[a][b] = V4{0, 0, 0, 0};
    }
  for (int i = 0; i < nb; ++i) {
    __syncthreads();
    const cx<TC>* ci = Cc + (size_t)i * S * S;
    for (int e = threadIdx.x; e < S * S; e += 256) sc[(e / S) * LD + (e % S)] = ci[e];
    __syncthreads();
    const cx<TIn>* Ai = A + (size_t)i * astride;
    for (int r0 = 0; r0 < S; r0 += 16) {
      cx<TIn> av[TMC][4];
#pragma unroll
      for (int a = 0; a < TMC; ++a) {
        const long cell = cw + 16 * a + m;
#pragma unroll
        for (int t = 0; t < 4; ++t) av[a][t] = cell < n ? Ai[cell * S + r0 + 4 * g + t] : cx<TIn>{0, 0};
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = r0 + 4 * g + t;
#pragma unroll
        for (int b = 0; b < TM; ++b) {
          const cx<TC> cv = sc[r * LD + 16 * b + m];
#pragma unroll
          for (int a = 0; a < TMC; ++a) {
            const TC ar = (TC)av[a][t].re, ai = (TC)av[a][t].im;
            re[a][b] = mfma16(ar, cv.re, re[a][b]);
            re[a][b] = mfma16(ai, -cv.im, re[a][b]);
            im[a][b] = mfma16(ar, cv.im, im[a][b]);
            im[a][b] = mfma16(ai, cv.re, im[a][b]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < TMC; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long cell = cw + 16 * a + mfma_row<TC>(g, v);
        if (cell >= n) continue;
        const size_t at = (size_t)cell * S + 16 * b + m;
        cx<TC> o{sgn * re[a][b][v], sgn * im[a][b][v]};
        if (In && beta != (TC)0) {
          const cx<TC> x = cvt<TC>(In[at]);
          o = cx<TC>{o.re + beta * x.re, o.im + beta * x.im};
        }
        Out[at] = cvt<TOut>(o);
      }
}

// ------------------------------------------------ block QR (CholQR) -------
// Cholesky of the Hermitian S x S Gram matrix G = W^H W (FP64) in one block:
// G = R^H R, R upper triangular with a real positive diagonal; a pivot below
// 1e-26 x the largest diagonal entry of G marks a dependent column, whose row
// of R and column of R^{-1} are set to zero (the column of the new basis block
// is then zero).  Writes Rinv = R^{-1} (row-major, rounded to R) for the
// update kernel, and Rout = R Rprev (column-major into H with leading
// dimension ldh; Rprev row-major, or none).  Also ||Rout||_F^2 into *fro.
template <typename R>
__global__ void __launch_bounds__(256) k_blk_chol(const c128* __restrict__ G, int S, const c128* __restrict__ Rprev,
                                                  c128* __restrict__ Rout, int ldh, c128* __restrict__ Rrow,
                                                  cx<R>* __restrict__ Rinv, double* __restrict__ fro) {
  extern __shared__ unsigned char blk_lds[];
  c128* A = reinterpret_cast<c128*>(blk_lds);        // [S][S] row-major working copy, then R
  c128* X = A + S * S;                                // [S][S] R^{-1}
  __shared__ double dmax;
  __shared__ int dead[64];
  const int t = threadIdx.x;
  for (int e = t; e < S * S; e += 256) A[e] = G[(e % S) * S + e / S];   // G column-major -> row-major
  if (t < 64) dead[t] = 0;
  __syncthreads();
  if (t == 0) {
    double mx = 0.0;
    for (int q = 0; q < S; ++q) mx = fmax(mx, A[q * S + q].re);
    dmax = mx;
  }
  __syncthreads();
  for (int q = 0; q < S; ++q) {
    const double d = A[q * S + q].re;
    const bool gone = !(d > 1e-26 * dmax);
    __syncthreads();
    if (gone) {
      for (int j = q + t; j < S; j += 256) A[q * S + j] = c128{0.0, 0.0};
      if (t == 0) dead[q] = 1;
    } else {
      const double rq = sqrt(d);
      for (int j = q + 1 + t; j < S; j += 256) A[q * S + j] = (1.0 / rq) * A[q * S + j];
      __syncthreads();
      if (t == 0) A[q * S + q] = c128{rq, 0.0};
    }
    __syncthreads();
    // trailing update of the upper triangle: A[i][j] -= conj(R[q][i]) R[q][j]
    const int nt = S - q - 1;
    for (int e = t; e < nt * nt; e += 256) {
      const int i = q + 1 + e / nt, j = q + 1 + e % nt;
      if (j >= i) A[i * S + j] = A[i * S + j] - conj(A[q * S + i]) * A[q * S + j];
    }
    __syncthreads();
  }
  // R^{-1}, one column per thread, rows from the diagonal up
  for (int j = t; j < S; j += 256) {
    for (int i = 0; i < S; ++i) X[i * S + j] = c128{0.0, 0.0};
    if (!dead[j]) {
      X[j * S + j] = cdiv(c128{1.0, 0.0}, A[j * S + j]);
      for (int i = j - 1; i >= 0; --i) {
        if (dead[i]) continue;
        c128 s{0.0, 0.0};
        for (int p = i + 1; p <= j; ++p) s = s + A[i * S + p] * X[p * S + j];
        X[i * S + j] = cdiv(-s, A[i * S + i]);
      }
    }
  }
  __syncthreads();
  for (int e = t; e < S * S; e += 256) {
    const int i = e / S, j = e % S;
    Rinv[e] = cvt<R>(j >= i ? X[e] : c128{0.0, 0.0});
  }
  // Rout = R Rprev (both upper triangular)
  __shared__ double fsum[256];
  double f = 0.0;
  for (int e = t; e < S * S; e += 256) {
    const int i = e / S, j = e % S;
    c128 s{0.0, 0.0};
    if (j >= i) {
      if (Rprev) {
        for (int p = i; p <= j; ++p) s = s + A[i * S + p] * Rprev[p * S + j];
      } else {
        s = A[i * S + j];
      }
    }
    if (Rout) Rout[i + (size_t)ldh * j] = s;
    if (Rrow) Rrow[e] = s;
    f += abs2(s);
  }
  fsum[t] = f;
  __syncthreads();
  if (t == 0) {
    double a = 0.0;
    for (int q = 0; q < 256; ++q) a += fsum[q];
    if (fro) *fro = a;
  }
}

// Breakdown of the block step (section 3, the block analogue): the new block
// vanishes, ||H_{k+1,k}||_F <= 1e-14 ||M Z_k||_F.
__global__ void k_blk_breakdown(const double* __restrict__ fro, const double* __restrict__ mz, int S,
                                int* __restrict__ broke) {
  if (threadIdx.x != 0) return;
  double z2 = 0.0;
  for (int r = 0; r < S; ++r) z2 += mz[r] * mz[r];
  broke[0] = fro[0] <= 1e-28 * z2 ? 1 : 0;
}

// ----------------------------------------- per-shift block least squares --
// Packed upper triangle, column by column: entry (row <= col) of an upper
// triangular matrix at col (col + 1) / 2 + row.
__host__ __device__ __forceinline__ size_t rpk(int row, int col) { return (size_t)col * (col + 1) / 2 + row; }

// Householder reflector P = I - tau v v^H (tau real, P Hermitian and unitary)
// mapping a vector x onto beta e_1, beta = -e^{i arg x_0} ||x||: v = x - beta
// e_1, tau = 2 / ||v||^2 = 1 / (||x|| (||x|| + |x_0|)).
struct BlkLsqArgs {
  int S, m, k, nf;
  int ldh;                      // leading dimension of Hbar ((m + 1) S)
  const c128* H;                // Hbar, column-major, ldh x m S
  const c128* sigma;            // shifts
  c128 tau;                     // preconditioner shift of block column k
  c128* Rf;                     // per shift: m S x m S upper triangle, packed (rpk)
  c128* Vr;                     // per shift: reflectors [block][q][t = 0..S] (S + 1 entries)
  double* Tr;                   // per shift: tau of each reflector [block][q]
  c128* Gq;                     // per shift: rotated right-hand sides, ((m + 1) S) x S column-major
  double* rho;                  // per (shift, rhs): ||residual block|| at this step
  const LaneState* ls;          // frozen pairs need no new quasi-residual
};

// Applies reflector (v, tau) acting on window rows q..q+S to a column held
// two entries per lane (lane t: window rows t and S + t).
__device__ __forceinline__ void blk_reflect(c128& top, c128& bot, int q, int S, const c128* v, double tau) {
  const int t = threadIdx.x & 63;
  c128 s{0.0, 0.0};
  const bool ut = t >= q && t < S, ub = t <= q && t < S;
  c128 vt{0, 0}, vb{0, 0};
  if (ut) { vt = v[t - q]; s = s + cdot(vt, top); }
  if (ub) { vb = v[S + t - q]; s = s + cdot(vb, bot); }
  s = wave_sum_strided(s, 1);
  const c128 ts = tau * s;
  if (ut) top = top - vt * ts;
  if (ub) bot = bot - vb * ts;
}

// One outer step k of every shift's block least squares: grid = nf blocks of
// 1024 threads (16 waves).  Wave w owns block columns c = w, w + 16, ... of
// the new block column of Hbar(sigma_j;T) and the same columns of G.
//  1. each owned Hbar column is built (e_{kS+c} + (sigma_j - tau_k) Hbar
//     column) and the reflectors of blocks 0..k-1 are applied window by
//     window (rows iS..iS+2S), finished rows going to R;
//  2. the new block's S reflectors are formed one column at a time (the
//     owner of column q forms reflector q; one barrier per q) and applied to
//     the later columns and to G's rows kS..kS+2S;
//  3. R's diagonal block, the reflectors and G are stored; rho_{j,r} is the
//     norm of G's rows (k+1)S..(k+2)S in column r.
constexpr int BLK_LSQ_THREADS = 1024;
__global__ void __launch_bounds__(BLK_LSQ_THREADS) k_blk_lsq(BlkLsqArgs a) {
  extern __shared__ unsigned char blk_lds[];
  const int S = a.S, k = a.k, j = blockIdx.x, mS = a.m * S;
  c128* refl = reinterpret_cast<c128*>(blk_lds);               // [S][S+1] reflectors of one block
  double* rtau = reinterpret_cast<double*>(refl + S * (S + 1)); // [S]
  c128* nv = reinterpret_cast<c128*>(rtau + S);                // [2][S+1] new reflector (double buffer)
  double* ntau = reinterpret_cast<double*>(nv + 2 * (S + 1));  // [2]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = BLK_LSQ_THREADS / 64;
  const int per = (S + NW - 1) / NW;   // columns per wave (1..4)
  const c128 ds = a.sigma[j] - a.tau;
  c128* Rj = a.Rf + (size_t)j * rpk(0, mS);
  c128* Vj = a.Vr + (size_t)j * a.m * S * (S + 1);
  double* Tj = a.Tr + (size_t)j * a.m * S;
  c128* Gj = a.Gq + (size_t)j * a.ldh * S;
  const int col0 = k * S;
  // owned columns: entries at window rows lane and S + lane
  c128 top[4], bot[4];
  auto hval = [&](int row, int c) -> c128 {   // entry of column kS + c of Hbar(sigma;T)
    const c128 h = a.H[row + (size_t)a.ldh * (col0 + c)];
    c128 v = ds * h;
    if (row == col0 + c) v.re += 1.0;
    return v;
  };
  for (int u = 0; u < per; ++u) {
    const int c = w + NW * u;
    top[u] = (c < S && lane < S) ? hval(lane, c) : c128{0, 0};
    bot[u] = (c < S && lane < S) ? hval(S + lane, c) : c128{0, 0};
  }
  // 1. reflectors of the earlier blocks
  for (int i = 0; i < k; ++i) {
    __syncthreads();
    for (int e = threadIdx.x; e < S * (S + 1); e += BLK_LSQ_THREADS) refl[e] = Vj[(size_t)i * S * (S + 1) + e];
    for (int e = threadIdx.x; e < S; e += BLK_LSQ_THREADS) rtau[e] = Tj[(size_t)i * S + e];
    __syncthreads();
    for (int u = 0; u < per; ++u) {
      const int c = w + NW * u;
      if (c >= S) continue;
      for (int q = 0; q < S; ++q) blk_reflect(top[u], bot[u], q, S, refl + q * (S + 1), rtau[q]);
      // rows iS..iS+S are final: R entries of this column
      if (lane < S) Rj[rpk(i * S + lane, col0 + c)] = top[u];
      // slide the window: next window rows (i+1)S .. (i+3)S
      top[u] = bot[u];
      bot[u] = lane < S ? hval((i + 2) * S + lane, c) : c128{0, 0};
    }
  }
  // G's window rows kS .. kS+2S for the owned right-hand-side columns
  c128 gt[4], gb[4];
  for (int u = 0; u < per; ++u) {
    const int r = w + NW * u;
    gt[u] = (r < S && lane < S) ? Gj[(size_t)(col0 + lane) + (size_t)a.ldh * r] : c128{0, 0};
    gb[u] = c128{0, 0};
  }
  // 2. the new block's reflectors, one column at a time
  auto form = [&](int q, int u, int slot) {
    // reflector from window rows q..q+S of owned column u (lane t: rows t, S+t)
    c128* v = nv + slot * (S + 1);
    const int t = lane;
    const bool ut = t >= q && t < S, ub = t <= q && t < S;
    double s2 = 0.0;
    if (ut) s2 += abs2(top[u]);
    if (ub) s2 += abs2(bot[u]);
    s2 = wave_sum_strided(s2, 1);
    const double nx = sqrt(s2);
    const c128 x0{__shfl(top[u].re, q, 64), __shfl(top[u].im, q, 64)};
    const double a0 = hypot(x0.re, x0.im);
    const c128 ph = a0 > 0.0 ? c128{x0.re / a0, x0.im / a0} : c128{1.0, 0.0};
    const c128 beta = -nx * ph;
    const double tau = nx > 0.0 ? 1.0 / (nx * (nx + a0)) : 0.0;
    if (ut) v[t - q] = (t == q) ? top[u] - beta : top[u];
    if (ub) v[S + t - q] = bot[u];
    if (t == 0) ntau[slot] = tau;
    // the column itself becomes beta e_q
    if (ut) top[u] = (t == q) ? beta : c128{0.0, 0.0};
    if (ub) bot[u] = c128{0.0, 0.0};
  };
  // reflector 0's owner forms it before the loop
  if (w == 0) form(0, 0, 0);
  for (int q = 0; q < S; ++q) {
    __syncthreads();
    const int slot = q & 1;
    const c128* v = nv + slot * (S + 1);
    const double tq = ntau[slot];
    for (int u = 0; u < per; ++u) {
      const int c = w + NW * u;
      if (c < S && c > q) blk_reflect(top[u], bot[u], q, S, v, tq);
      const int r = w + NW * u;
      if (r < S) blk_reflect(gt[u], gb[u], q, S, v, tq);
    }
    // store reflector q for later steps
    for (int e = threadIdx.x; e < S + 1; e += BLK_LSQ_THREADS) Vj[((size_t)k * S + q) * (S + 1) + e] = v[e];
    if (threadIdx.x == 0) Tj[(size_t)k * S + q] = tq;
    // the owner of column q + 1 forms its reflector into the other slot
    if (q + 1 < S && w == (q + 1) % NW) form(q + 1, (q + 1) / NW, slot ^ 1);
  }
  __syncthreads();
  // 3. R's rows kS..kS+S of the new columns; G's rows kS..kS+2S; residuals
  for (int u = 0; u < per; ++u) {
    const int c = w + NW * u;
    if (c < S && lane <= c) Rj[rpk(col0 + lane, col0 + c)] = top[u];
    const int r = w + NW * u;
    if (r < S) {
      if (lane < S) {
        Gj[(size_t)(col0 + lane) + (size_t)a.ldh * r] = gt[u];
        Gj[(size_t)(col0 + S + lane) + (size_t)a.ldh * r] = gb[u];
      }
      double s2 = lane < S ? abs2(gb[u]) : 0.0;
      s2 = wave_sum_strided(s2, 1);
      if (lane == 0) a.rho[(size_t)j * S + r] = sqrt(s2);
    }
  }
}

// G's start: rows 0..S of every shift's rotated right-hand side hold beta
// (the R factor of the first block, row-major in beta), the rest zero.
__global__ void __launch_bounds__(BS) k_blk_g_init(int S, int ldh, int nf, const c128* __restrict__ beta,
                                                   c128* __restrict__ Gq) {
  const size_t per = (size_t)ldh * S;
  for (size_t e = blockIdx.x * (size_t)BS + threadIdx.x; e < per * nf; e += (size_t)gridDim.x * BS) {
    const size_t q = e % per;
    const int row = (int)(q % ldh), r = (int)(q / ldh);
    Gq[e] = row < S ? beta[row * S + r] : c128{0.0, 0.0};
  }
}

// ------------------------------------------------ back substitution -------
// y = R^{-1} G[0:kS, r] for the right-hand sides r of shift j marked in
// want[j*S + r] (grid: nf blocks of 256 threads; R's diagonal blocks are
// solved one row at a time with the later blocks' contributions subtracted
// first).  Y[(j*S + r)*mS + row] receives y (rows kS.. untouched).  Then, per
// marked pair, the inexact term gap = sum |y_i| ||p_i|| (section 4, eq.
// resdiff, one inner residual per basis column) and the freeze decision of
// the one-vector method: CONVERGED when rho + gap <= tol ||b_r||, INNER_LIMITED
// when rho <= ratio * gap; final != 0 freezes every marked pair that is still
// active with NOT_CONVERGED.
struct BlkSolveArgs {
  int S, m, kc, nf, ldh, step, final_;
  const c128* Rf;
  const c128* Gq;
  const int* want;
  c128* Y;
  const double* pn;        // [i*S + c] inner residual norms of basis column (i, c)
  const double* rho;
  const double* beta0;     // ||b_r||
  double tol, ratio;
  const int* broke;        // the step ended in breakdown (device flag)
  LaneState* ls;
};
__global__ void __launch_bounds__(BS) k_blk_backsolve(BlkSolveArgs a) {
  const int j = blockIdx.x, S = a.S, K = a.kc * S, mS = a.m * S;
  const c128* Rj = a.Rf + (size_t)j * rpk(0, mS);
  const c128* Gj = a.Gq + (size_t)j * a.ldh * S;
  __shared__ int wanted[64];
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if ((int)threadIdx.x < S) {
    wanted[threadIdx.x] = a.want[(size_t)j * S + threadIdx.x];
    if (wanted[threadIdx.x]) atomicOr(&any, 1);
  }
  __syncthreads();
  if (!any) return;
  // work vector: G[0:K, r] for wanted r, reduced in place into y (in Y)
  for (int e = threadIdx.x; e < K * S; e += BS) {
    const int row = e % K, r = e / K;
    if (wanted[r]) a.Y[((size_t)j * S + r) * mS + row] = Gj[(size_t)row + (size_t)a.ldh * r];
  }
  __syncthreads();
  for (int col = K - 1; col >= 0; --col) {
    const c128 d = Rj[rpk(col, col)];
    // y_col = g_col / R_col,col for every wanted r (thread r)
    if ((int)threadIdx.x < S && wanted[threadIdx.x]) {
      c128* y = a.Y + ((size_t)j * S + threadIdx.x) * mS;
      y[col] = (d.re == 0.0 && d.im == 0.0) ? c128{0.0, 0.0} : cdiv(y[col], d);
    }
    __syncthreads();
    // g[0:col] -= R[0:col, col] y_col
    for (int e = threadIdx.x; e < col * S; e += BS) {
      const int row = e % col, r = e / col;
      if (!wanted[r]) continue;
      c128* y = a.Y + ((size_t)j * S + r) * mS;
      y[row] = y[row] - Rj[rpk(row, col)] * y[col];
    }
    __syncthreads();
  }
  // freeze decisions
  if ((int)threadIdx.x < S && wanted[threadIdx.x]) {
    const int r = threadIdx.x;
    const c128* y = a.Y + ((size_t)j * S + r) * mS;
    double gap = 0.0;
    for (int i = 0; i < K; ++i) gap += hypot(y[i].re, y[i].im) * a.pn[i];
    LaneState st = a.ls[(size_t)j * S + r];
    if (st.active) {
      const int brk = *a.broke;
      const double rho = brk ? 0.0 : a.rho[(size_t)j * S + r];
      const double bnd = rho + gap;
      st.rho = rho;
      st.bound = bnd;
      st.outer_its = a.step;
      st.kfz = a.kc;
      int done = -1;
      if (brk) done = bnd <= a.tol * a.beta0[r] ? SHK_BREAKDOWN_EXACT : SHK_INNER_LIMITED;
      else if (bnd <= a.tol * a.beta0[r]) done = SHK_CONVERGED;
      else if (rho <= a.ratio * gap) done = SHK_INNER_LIMITED;
      else if (a.final_) done = SHK_NOT_CONVERGED;
      if (done >= 0) {
        st.status = done;
        st.active = 0;
      }
      a.ls[(size_t)j * S + r] = st;
    }
  }
}

// Pairs whose least-squares solution is needed this step: active pairs with
// rho within lim x ||b_r|| (where the stopping rule can trigger), or every
// active pair (all != 0, or a breakdown step).  Also records rho and the step
// in the lane state of every active pair.
__global__ void __launch_bounds__(BS) k_blk_mark(int L, int S, const double* __restrict__ rho,
                                                 const double* __restrict__ beta0, double lim, int all,
                                                 const int* __restrict__ broke, int step,
                                                 LaneState* __restrict__ ls, int* __restrict__ want) {
  const int p = blockIdx.x * BS + threadIdx.x;
  if (p >= L) return;
  LaneState st = ls[p];
  int wnt = 0;
  if (st.active) {
    const int r = p % S;
    st.rho = rho[p];
    st.outer_its = step;
    ls[p] = st;
    wnt = all || *broke || rho[p] <= lim * beta0[r];
  }
  want[p] = wnt;
}

// X[:, j, r] (+)= scale_{j,r} Z y_{j,r} for the block basis: Z (n x kc S,
// FP64 blocks astride apart), y of every pair in Y[(j*S + r)*mS + (i*S + c)].
// The same matrix-core contraction as k_blk_update, with C_i the S x S slice
// of shift j's coefficients (scaled per column) and the result written to the
// solver's output layout x[c + n (j + nf r)] for r < s_real.
template <int TM, int TMC>
__global__ void __launch_bounds__(256) k_blk_assemble(const c128* __restrict__ Z, size_t astride, int kc, int mS,
                                                      const c128* __restrict__ Y, const c128* __restrict__ scale,
                                                      long n, int nf, int s_real, c128* __restrict__ X, int acc) {
  constexpr int S = 16 * TM, LD = S + 1;
  extern __shared__ unsigned char blk_lds[];
  c128* sc = reinterpret_cast<c128*>(blk_lds);   // [S][LD]: rows c (basis column), columns r
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, m = lane & 15;
  const int j = blockIdx.y;
  const long cw = ((long)blockIdx.x * 4 + wv) * (16 * TMC);
  d4m re[TMC][TM], im[TMC][TM];
#pragma unroll
  for (int a = 0; a < TMC; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      re[a][b] = d4m{0, 0, 0, 0};
      im[a][b] = d4m{0, 0, 0, 0};
    }
  for (int i = 0; i < kc; ++i) {
    __syncthreads();
    for (int e = threadIdx.x; e < S * S; e += 256) {
      const int c = e % S, r = e / S;
      const c128 sr = scale ? scale[(size_t)j * S + r] : c128{1.0, 0.0};
      sc[c * LD + r] = sr * Y[((size_t)j * S + r) * mS + (size_t)i * S + c];
    }
    __syncthreads();
    const c128* Zi = Z + (size_t)i * astride;
    for (int r0 = 0; r0 < S; r0 += 16) {
      c128 av[TMC][4];
#pragma unroll
      for (int a = 0; a < TMC; ++a) {
        const long cell = cw + 16 * a + m;
#pragma unroll
        for (int t = 0; t < 4; ++t) av[a][t] = cell < n ? Zi[cell * S + r0 + 4 * g + t] : c128{0, 0};
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = r0 + 4 * g + t;
#pragma unroll
        for (int b = 0; b < TM; ++b) {
          const c128 cv = sc[r * LD + 16 * b + m];
#pragma unroll
          for (int a = 0; a < TMC; ++a) {
            re[a][b] = mfma16(av[a][t].re, cv.re, re[a][b]);
            re[a][b] = mfma16(av[a][t].im, -cv.im, re[a][b]);
            im[a][b] = mfma16(av[a][t].re, cv.im, im[a][b]);
            im[a][b] = mfma16(av[a][t].im, cv.re, im[a][b]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < TMC; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      const int r = 16 * b + m;
      if (r >= s_real) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long cell = cw + 16 * a + mfma_row<double>(g, v);
        if (cell >= n) continue;
        c128* xp = X + (size_t)cell + (size_t)n * ((size_t)j + (size_t)nf * r);
        const c128 o{re[a][b][v], im[a][b][v]};
        *xp = acc ? *xp + o : o;
      }
    }
}

}  // namespace shk
