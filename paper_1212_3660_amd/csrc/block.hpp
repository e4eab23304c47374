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

// ---------------------------------------------- lockstep-basis assembly ----
// X[:, j, r] (+)= scale_{j,r} Z_r y_{j,r} for independent bases (one basis
// per right-hand-side lane r; Algorithm 4, x = Z y) on the FP64 matrix cores:
// per lane a product of the n x kc block Z_r of its basis columns and the
// kc x nf block of its coefficients.  A wave computes 16 cells x 16 TN shifts
// of one lane (TN output tiles, complex as four real products per step of 4
// basis columns); a block's 4 waves take 4 adjacent lanes of one tile of 16
// cells, and the blocks of the other lanes of that tile sit 8 block indices
// apart, on the same XCD (workgroups go to the XCDs round-robin), so the
// basis rows of a tile come into one L2 only.  Z is read once per 16 TN
// shifts and X written once.  FP64 accumulation (the order over the basis
// columns is the matrix core's).
template <typename R, int TN>
__global__ void __launch_bounds__(256) k_assemble_mfma(long n, int S, int s_real, int nf, int kc, int m,
                                                       const cx<R>* __restrict__ Z, size_t cstride,
                                                       const c128* __restrict__ Yb,
                                                       const c128* __restrict__ ascale, c128* __restrict__ X,
                                                       int acc) {
  const int lane = threadIdx.x & 63, g = lane >> 4, mm = lane & 15;
  // block -> (tile of 16 cells, group of 4 lanes): groups of 8 tiles x LG lane
  // groups, the tile's XCD slot fastest (fewer than 4 lanes: 4 / S tiles per
  // block)
  long tile;
  int r;
  if (S >= 4) {
    const int LG = S >> 2;
    const long b = blockIdx.x, per = 8L * LG;
    const long grp = b / per;
    const int rem = (int)(b - grp * per);
    tile = grp * 8 + (rem & 7);
    r = (rem >> 3) * 4 + (int)(threadIdx.x >> 6);
  } else {
    const long qq = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    tile = qq / S;
    r = (int)(qq % S);
  }
  const long cell0 = tile * 16;
  if (cell0 >= n || r >= s_real) return;   // whole waves
  const int j0 = (int)blockIdx.y * 16 * TN;
  d4m re[TN], im[TN];
#pragma unroll
  for (int t = 0; t < TN; ++t) {
    re[t] = d4m{0, 0, 0, 0};
    im[t] = d4m{0, 0, 0, 0};
  }
  const bool zin = cell0 + mm < n;
  const size_t zc = (size_t)(cell0 + mm) * S + r;
  for (int i0 = 0; i0 < kc; i0 += 4) {
    const int i = i0 + g;
    const bool iin = i < kc;
    const c128 a = zin && iin ? cvt<double>(Z[(size_t)i * cstride + zc]) : c128{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      const int j = j0 + 16 * t + mm;
      const c128 y = iin && j < nf ? Yb[((size_t)j * S + r) * m + i] : c128{0.0, 0.0};
      re[t] = mfma16(a.re, y.re, re[t]);
      re[t] = mfma16(a.im, -y.im, re[t]);
      im[t] = mfma16(a.re, y.im, im[t]);
      im[t] = mfma16(a.im, y.re, im[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < TN; ++t) {
    const int j = j0 + 16 * t + mm;
    if (j >= nf) continue;
    const c128 sc = ascale[(size_t)j * S + r];
    c128* col = X + n * ((long)j + (long)nf * r);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long cell = cell0 + mfma_row<double>(g, v);
      if (cell >= n) continue;
      const c128 val = sc * c128{re[t][v], im[t][v]};
      col[cell] = acc ? col[cell] + val : val;
    }
  }
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
  c128* X = A + S * S;                                // [S][S] R^{-1}, then Rprev
  __shared__ double dmax;
  __shared__ int dead[64];
  __shared__ c128 rdi[64];                            // 1 / R_qq (0 for a dependent column)
  const int t = threadIdx.x;
  // thread t: column jc = t % 64, row group rg = t / 64 (rows rg, rg + 4, ...)
  const int jc = t & 63, rg = t >> 6;
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
    const double rq = gone ? 0.0 : sqrt(d);
    const double iq = gone ? 0.0 : 1.0 / rq;
    __syncthreads();
    // row q of R: R_qq = sqrt(d), R_qj = A_qj / R_qq (zero for a dependent column)
    if (rg == 0 && jc >= q && jc < S) A[q * S + jc] = jc == q ? c128{rq, 0.0} : iq * A[q * S + jc];
    if (t == 0) {
      dead[q] = gone ? 1 : 0;
      rdi[q] = c128{iq, 0.0};
    }
    __syncthreads();
    // trailing update of the upper triangle: A_ij -= conj(R_qi) R_qj, q < i <= j
    if (jc > q && jc < S) {
      const c128 rj = A[q * S + jc];
      for (int i = q + 1 + rg; i <= jc; i += 4) A[i * S + jc] = A[i * S + jc] - conj(A[q * S + i]) * rj;
    }
    __syncthreads();
  }
  // R^{-1}: column jc by the thread group of rg == 0 (rows upwards, four
  // independent partial sums per row)
  if (rg == 0 && jc < S) {
    for (int i = 0; i < S; ++i) X[i * S + jc] = c128{0.0, 0.0};
    if (!dead[jc]) {
      X[jc * S + jc] = rdi[jc];
      for (int i = jc - 1; i >= 0; --i) {
        if (dead[i]) continue;
        c128 s0{0, 0}, s1{0, 0}, s2{0, 0}, s3{0, 0};
        int p = i + 1;
        for (; p + 3 <= jc; p += 4) {
          s0 = s0 + A[i * S + p] * X[p * S + jc];
          s1 = s1 + A[i * S + p + 1] * X[(p + 1) * S + jc];
          s2 = s2 + A[i * S + p + 2] * X[(p + 2) * S + jc];
          s3 = s3 + A[i * S + p + 3] * X[(p + 3) * S + jc];
        }
        for (; p <= jc; ++p) s0 = s0 + A[i * S + p] * X[p * S + jc];
        const c128 sum = (s0 + s1) + (s2 + s3);
        X[i * S + jc] = -(rdi[i].re * sum);      // R_ii real positive
      }
    }
  }
  __syncthreads();
  for (int e = t; e < S * S; e += 256) {
    const int i = e / S, j = e % S;
    Rinv[e] = cvt<R>(j >= i ? X[e] : c128{0.0, 0.0});
  }
  // Rout = R Rprev (both upper triangular), Rprev staged in X's space
  __syncthreads();
  if (Rprev)
    for (int e = t; e < S * S; e += 256) X[e] = Rprev[e];
  __syncthreads();
  __shared__ double fsum[256];
  double f = 0.0;
  if (jc < S) {
    for (int i = rg; i <= jc; i += 4) {
      c128 sv{0.0, 0.0};
      if (Rprev) {
        c128 s0{0, 0}, s1{0, 0};
        int p = i;
        for (; p + 1 <= jc; p += 2) {
          s0 = s0 + A[i * S + p] * X[p * S + jc];
          s1 = s1 + A[i * S + p + 1] * X[(p + 1) * S + jc];
        }
        for (; p <= jc; ++p) s0 = s0 + A[i * S + p] * X[p * S + jc];
        sv = s0 + s1;
      } else {
        sv = A[i * S + jc];
      }
      if (Rout) Rout[i + (size_t)ldh * jc] = sv;
      if (Rrow) Rrow[i * S + jc] = sv;
      f += abs2(sv);
    }
    // entries below the diagonal are zero
    for (int i = jc + 1 + ((rg - (jc + 1) % 4 + 4) % 4); i < S; i += 4) {
      if (Rout) Rout[i + (size_t)ldh * jc] = c128{0.0, 0.0};
      if (Rrow) Rrow[i * S + jc] = c128{0.0, 0.0};
    }
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
  c128* Vr;                     // per shift: this step's reflectors [q][t = 0..S] (S + 1 entries)
  double* Tr;                   // per shift: their tau [q]
  c128* Qb;                     // per shift: per block, the 2S x 2S product of its reflectors (column-major)
  c128* Rdinv;                  // per shift: per block, the inverse of R's diagonal block (S x S column-major)
  c128* Tile;                   // per shift: the new block column's window rows kS..kS+2S (2S x S column-major)
  c128* Gq;                     // per shift: rotated right-hand sides, ((m + 1) S) x S column-major
  double* rho;                  // per (shift, rhs): ||residual block|| at this step
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

// Entry (row, col) of Hbar(sigma;T) = [I;0] + Hbar (sigma - tau_col) for a
// column of block column k (ds = sigma - tau_k).
__device__ __forceinline__ c128 blk_hval(const BlkLsqArgs& a, c128 ds, int row, int col) {
  c128 v = ds * a.H[row + (size_t)a.ldh * col];
  if (row == col) v.re += 1.0;
  return v;
}

// Step 1 of the per-shift update: the new block column k of Hbar(sigma_j;T)
// times the earlier blocks' reflectors, block by block.  Block i's S
// reflectors act on rows iS..iS+2S only; their product Q_i (2S x 2S, formed
// when block i was factored) is applied as one matrix-core contraction to the
// 2S-row window of 16 columns held in LDS; rows iS..iS+S are then final
// entries of R.  Grid (nf, S/16), 256 threads; the window that is left
// (rows kS..kS+2S) goes to Tile for step 2.
template <int S>
__global__ void __launch_bounds__(256) k_blk_lsq_prev(BlkLsqArgs a) {
  extern __shared__ unsigned char blk_lds[];
  constexpr int S2 = 2 * S;
  const int k = a.k, j = blockIdx.x, q0 = 16 * blockIdx.y, mS = a.m * S;
  c128* win = reinterpret_cast<c128*>(blk_lds);   // [2S][16]
  c128* nxt = win + S2 * 16;                       // [2S][16]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, m = lane & 15;
  const c128 ds = a.sigma[j] - a.tau;
  const int col0 = k * S;
  c128* Rj = a.Rf + (size_t)j * rpk(0, mS);
  for (int e = threadIdx.x; e < S2 * 16; e += 256) {
    const int row = e >> 4, n = e & 15;
    win[e] = blk_hval(a, ds, row, col0 + q0 + n);
  }
  constexpr int tiles = S2 / 16;
  for (int i = 0; i < k; ++i) {
    __syncthreads();
    const c128* Q = a.Qb + ((size_t)j * a.m + i) * S2 * S2;
    for (int tl = wv; tl < tiles; tl += 4) {
      d4m re{0, 0, 0, 0}, im{0, 0, 0, 0};
#pragma unroll 4
      for (int k0 = 0; k0 < S2; k0 += 4) {
        const c128 q = Q[(size_t)(k0 + g) * S2 + 16 * tl + m];
        const c128 w = win[(k0 + g) * 16 + m];
        re = mfma16(q.re, w.re, re);
        re = mfma16(q.im, -w.im, re);
        im = mfma16(q.re, w.im, im);
        im = mfma16(q.im, w.re, im);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) nxt[(16 * tl + mfma_row<double>(g, v)) * 16 + m] = c128{re[v], im[v]};
    }
    __syncthreads();
    // rows iS..iS+S final; slide the window down one block
    for (int e = threadIdx.x; e < S * 16; e += 256) {
      const int row = e >> 4, n = e & 15;
      Rj[rpk(i * S + row, col0 + q0 + n)] = nxt[e];
      win[e] = nxt[S * 16 + e];
      win[S * 16 + e] = blk_hval(a, ds, (i + 2) * S + row, col0 + q0 + n);
    }
  }
  __syncthreads();
  c128* Tj = a.Tile + (size_t)j * S2 * S;
  for (int e = threadIdx.x; e < S2 * 16; e += 256) {
    const int row = e >> 4, n = e & 15;
    Tj[(size_t)(q0 + n) * S2 + row] = win[e];
  }
}

// Step 2: Householder QR of the 2S x S window left by step 1 (rows kS..kS+2S
// of the new block column; its lower half is the upper triangular (sigma -
// tau_k) H_{k+1,k}), one reflector per column.  Grid nf, NT threads (NW = NT/64 waves); wave w owns columns w,
// w + NW, ... (PER of them); the owner of column q forms reflector q, one
// barrier per q.  Stores
// R's diagonal block and its inverse and the reflectors (for step 3).
template <int PER, int NT>
__global__ void __launch_bounds__(NT) k_blk_lsq_new(BlkLsqArgs a) {
  extern __shared__ unsigned char blk_lds[];
  const int S = a.S, S2 = 2 * S, k = a.k, j = blockIdx.x, mS = a.m * S;
  c128* nv = reinterpret_cast<c128*>(blk_lds);        // [2][S+1] reflector double buffer
  double* ntau = reinterpret_cast<double*>(nv + 2 * (S + 1));
  c128* Rd = reinterpret_cast<c128*>(ntau + 2);       // [S][S] R's diagonal block, row-major
  c128* Xi = Rd + S * S;                              // [S][S] its inverse, row-major
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  c128* Rj = a.Rf + (size_t)j * rpk(0, mS);
  c128* Vj = a.Vr + (size_t)j * S * (S + 1);
  double* Tj = a.Tr + (size_t)j * S;
  const c128* Tl = a.Tile + (size_t)j * S2 * S;
  const int col0 = k * S;
  // owned columns c = w + 16 u, u < PER (S = 16 PER): register arrays with
  // compile-time indices only
  c128 top[PER], bot[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int c = w + NW * u;
    top[u] = lane < S ? Tl[(size_t)c * S2 + lane] : c128{0, 0};
    bot[u] = lane < S ? Tl[(size_t)c * S2 + S + lane] : c128{0, 0};
  }
  auto form = [&](int q, c128& tp, c128& bt, int slot) {
    c128* v = nv + slot * (S + 1);
    const int t = lane;
    const bool ut = t >= q && t < S, ub = t <= q && t < S;
    double s2 = 0.0;
    if (ut) s2 += abs2(tp);
    if (ub) s2 += abs2(bt);
    s2 = wave_sum_strided(s2, 1);
    const double nx = sqrt(s2);
    const c128 x0{__shfl(tp.re, q, 64), __shfl(tp.im, q, 64)};
    const double a0 = hypot(x0.re, x0.im);
    const c128 ph = a0 > 0.0 ? c128{x0.re / a0, x0.im / a0} : c128{1.0, 0.0};
    const c128 beta = -nx * ph;
    const double tau = nx > 0.0 ? 1.0 / (nx * (nx + a0)) : 0.0;
    if (ut) v[t - q] = (t == q) ? tp - beta : tp;
    if (ub) v[S + t - q] = bt;
    if (t == 0) ntau[slot] = tau;
    if (ut) tp = (t == q) ? beta : c128{0.0, 0.0};
    if (ub) bt = c128{0.0, 0.0};
  };
  if (w == 0) form(0, top[0], bot[0], 0);
  for (int q = 0; q < S; ++q) {
    __syncthreads();
    const int slot = q & 1;
    const c128* v = nv + slot * (S + 1);
    const double tq = ntau[slot];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int c = w + NW * u;
      if (c > q) blk_reflect(top[u], bot[u], q, S, v, tq);
    }
    for (int e = threadIdx.x; e < S + 1; e += NT) Vj[(size_t)q * (S + 1) + e] = v[e];
    if (threadIdx.x == 0) Tj[q] = tq;
    if (q + 1 < S && w == (q + 1) % NW) {
#pragma unroll
      for (int u = 0; u < PER; ++u)
        if (u == (q + 1) / NW) form(q + 1, top[u], bot[u], slot ^ 1);
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int c = w + NW * u;
    if (lane < S) {
      if (lane <= c) Rj[rpk(col0 + lane, col0 + c)] = top[u];
      Rd[lane * S + c] = lane <= c ? top[u] : c128{0.0, 0.0};
    }
  }
  __syncthreads();
  // inverse of the diagonal block, one column per thread, rows upwards
  for (int c = threadIdx.x; c < S; c += NT) {
    for (int i = 0; i < S; ++i) Xi[i * S + c] = c128{0.0, 0.0};
    const c128 d = Rd[c * S + c];
    Xi[c * S + c] = (d.re == 0.0 && d.im == 0.0) ? c128{0.0, 0.0} : cdiv(c128{1.0, 0.0}, d);
    for (int i = c - 1; i >= 0; --i) {
      c128 s{0.0, 0.0};
      for (int p = i + 1; p <= c; ++p) s = s + Rd[i * S + p] * Xi[p * S + c];
      const c128 di = Rd[i * S + i];
      Xi[i * S + c] = (di.re == 0.0 && di.im == 0.0) ? c128{0.0, 0.0} : cdiv(-s, di);
    }
  }
  __syncthreads();
  c128* Di = a.Rdinv + ((size_t)j * a.m + k) * S * S;
  for (int e = threadIdx.x; e < S * S; e += NT) {
    const int row = e % S, col = e / S;
    Di[e] = Xi[row * S + col];      // column-major
  }
}

// Step 3: this step's reflectors applied column by column (grid (nf, 3S/16),
// 256 threads, each wave owns 4 columns): columns 0..2S are the identity's,
// giving Q_k = P_{S-1} ... P_0 on the 2S-row window (stored column-major for
// step 1 of later steps); columns 2S..3S are G's rows kS..kS+2S, after which
// rho_{j,r} = the norm of G's rows (k+1)S..(k+2)S in column r.
__global__ void __launch_bounds__(256) k_blk_lsq_q(BlkLsqArgs a) {
  extern __shared__ unsigned char blk_lds[];
  const int S = a.S, S2 = 2 * S, j = blockIdx.x;
  c128* refl = reinterpret_cast<c128*>(blk_lds);      // [S][S+1]
  double* rt = reinterpret_cast<double*>(refl + S * (S + 1));
  const c128* Vj = a.Vr + (size_t)j * S * (S + 1);
  for (int e = threadIdx.x; e < S * (S + 1); e += 256) refl[e] = Vj[e];
  for (int e = threadIdx.x; e < S; e += 256) rt[e] = a.Tr[(size_t)j * S + e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  c128* Q = a.Qb + ((size_t)j * a.m + a.k) * S2 * S2;
  c128* Gj = a.Gq + (size_t)j * a.ldh * S;
  const int col0 = a.k * S;
  for (int u = 0; u < 4; ++u) {
    const int c = 16 * blockIdx.y + 4 * wv + u;
    if (c >= 3 * S) continue;
    const bool gcol = c >= S2;
    const int r = c - S2;
    c128 top, bot;
    if (gcol) {
      top = lane < S ? Gj[(size_t)(col0 + lane) + (size_t)a.ldh * r] : c128{0.0, 0.0};
      bot = lane < S ? Gj[(size_t)(col0 + S + lane) + (size_t)a.ldh * r] : c128{0.0, 0.0};
    } else {
      top = (lane < S && lane == c) ? c128{1.0, 0.0} : c128{0.0, 0.0};
      bot = (lane < S && S + lane == c) ? c128{1.0, 0.0} : c128{0.0, 0.0};
    }
    for (int q = 0; q < S; ++q) blk_reflect(top, bot, q, S, refl + q * (S + 1), rt[q]);
    if (gcol) {
      if (lane < S) {
        Gj[(size_t)(col0 + lane) + (size_t)a.ldh * r] = top;
        Gj[(size_t)(col0 + S + lane) + (size_t)a.ldh * r] = bot;
      }
      double s2 = lane < S ? abs2(bot) : 0.0;
      s2 = wave_sum_strided(s2, 1);
      if (lane == 0) a.rho[(size_t)j * S + r] = sqrt(s2);
    } else if (lane < S) {
      Q[(size_t)c * S2 + lane] = top;
      Q[(size_t)c * S2 + S + lane] = bot;
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
// want[j*S + r]: grid (nf, S/16), 256 threads, 16 columns per block.  Block
// rows are solved from the bottom: Y_b = (R_bb)^{-1} G_b with the stored
// inverse of the diagonal block, then G_0..G_{b-1} -= R_{0:b, b} Y_b, both as
// matrix-core contractions; G's working copy lives in Gw.  Y[(j*S + r)*mS +
// row] receives y for the marked columns.  Then, per marked pair, the inexact
// term gap = sum |y_i| ||p_i|| (section 4, eq. resdiff, one inner residual per
// basis column) and the freeze decision of the one-vector method: CONVERGED
// when rho + gap <= tol ||b_r||, INNER_LIMITED when rho <= ratio * gap;
// final != 0 freezes every marked pair still active with NOT_CONVERGED.
struct BlkSolveArgs {
  int S, m, kc, nf, ldh, step, final_;
  const c128* Rf;
  const c128* Rdinv;
  const c128* Gq;
  const int* want;
  c128* Y;
  c128* Gw;                // working copy of G: per (shift, 16-column group) mS x 16 row-major
  const double* pn;        // [i*S + c] inner residual norms of basis column (i, c)
  const double* rho;
  const double* beta0;     // ||b_r||
  double tol, ratio;
  const int* broke;        // the step ended in breakdown (device flag)
  LaneState* ls;
};
template <int S>
__global__ void __launch_bounds__(256) k_blk_backsolve(BlkSolveArgs a) {
  const int j = blockIdx.x, grp = blockIdx.y, c0 = 16 * grp, K = a.kc * S, mS = a.m * S;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, m = lane & 15;
  __shared__ int wanted[16];
  __shared__ int any;
  __shared__ c128 Yb[64 * 16];
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if ((int)threadIdx.x < 16) {
    wanted[threadIdx.x] = a.want[(size_t)j * S + c0 + threadIdx.x];
    if (wanted[threadIdx.x]) atomicOr(&any, 1);
  }
  __syncthreads();
  if (!any) return;
  const c128* Rj = a.Rf + (size_t)j * rpk(0, mS);
  const c128* Gj = a.Gq + (size_t)j * a.ldh * S;
  c128* Gw = a.Gw + ((size_t)j * (S / 16) + grp) * mS * 16;
  for (int e = threadIdx.x; e < K * 16; e += 256) {
    const int row = e >> 4, n = e & 15;
    Gw[e] = Gj[(size_t)row + (size_t)a.ldh * (c0 + n)];
  }
  __syncthreads();
  constexpr int st = S / 16;
  for (int b = a.kc - 1; b >= 0; --b) {
    // Y_b = inv(R_bb) G_b
    const c128* Di = a.Rdinv + ((size_t)j * a.m + b) * S * S;
    for (int tl = wv; tl < st; tl += 4) {
      d4m re{0, 0, 0, 0}, im{0, 0, 0, 0};
#pragma unroll 4
      for (int k0 = 0; k0 < S; k0 += 4) {
        const c128 d = Di[(size_t)(k0 + g) * S + 16 * tl + m];
        const c128 x = Gw[(size_t)(b * S + k0 + g) * 16 + m];
        re = mfma16(d.re, x.re, re);
        re = mfma16(d.im, -x.im, re);
        im = mfma16(d.re, x.im, im);
        im = mfma16(d.im, x.re, im);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * tl + mfma_row<double>(g, v);
        const c128 y{re[v], im[v]};
        Yb[row * 16 + m] = y;
        if (wanted[m]) a.Y[((size_t)j * S + c0 + m) * mS + (size_t)b * S + row] = y;
      }
    }
    __syncthreads();
    // G_0..G_{b-1} -= R[0:bS, bS:bS+S] Y_b
    const int rt = b * st;
    for (int tl = wv; tl < rt; tl += 4) {
      d4m re{0, 0, 0, 0}, im{0, 0, 0, 0};
#pragma unroll 4
      for (int k0 = 0; k0 < S; k0 += 4) {
        const c128 r = Rj[rpk(16 * tl + m, b * S + k0 + g)];
        const c128 y = Yb[(k0 + g) * 16 + m];
        re = mfma16(r.re, y.re, re);
        re = mfma16(r.im, -y.im, re);
        im = mfma16(r.re, y.im, im);
        im = mfma16(r.im, y.re, im);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const size_t at = (size_t)(16 * tl + mfma_row<double>(g, v)) * 16 + m;
        Gw[at] = Gw[at] - c128{re[v], im[v]};
      }
    }
    __syncthreads();
  }
  // freeze decisions
  if ((int)threadIdx.x < 16 && wanted[threadIdx.x]) {
    const int r = c0 + threadIdx.x;
    const c128* y = a.Y + ((size_t)j * S + r) * mS;
    double gap = 0.0;
    for (int i = 0; i < K; ++i) gap += hypot(y[i].re, y[i].im) * a.pn[i];
    LaneState stt = a.ls[(size_t)j * S + r];
    if (stt.active) {
      const int brk = *a.broke;
      const double rho = brk ? 0.0 : a.rho[(size_t)j * S + r];
      const double bnd = rho + gap;
      stt.rho = rho;
      stt.bound = bnd;
      stt.outer_its = a.step;
      stt.kfz = a.kc;
      int done = -1;
      if (brk) done = bnd <= a.tol * a.beta0[r] ? SHK_BREAKDOWN_EXACT : SHK_INNER_LIMITED;
      else if (bnd <= a.tol * a.beta0[r]) done = SHK_CONVERGED;
      else if (rho <= a.ratio * gap) done = SHK_INNER_LIMITED;
      else if (a.final_) done = SHK_NOT_CONVERGED;
      if (done >= 0) {
        stt.status = done;
        stt.active = 0;
      }
      a.ls[(size_t)j * S + r] = stt;
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
