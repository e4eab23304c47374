// Device-side operators y = (K + sigma M) x for the shifted family
// (K + sigma_j M) x_j = b (section 2, eq. multipleshifted; section 5.1,
// eq. genshifted).
//
// Vectors hold S right-hand sides interleaved: element (cell c, rhs r) lives at
// index c*S + r.  The operators take a getter g(cell) returning the vector value
// of the calling lane's rhs at any cell, so callers can form the operand on the
// fly (e.g. p = u + beta p_old in the inner solver) without a separate pass.
//
// Finite-volume stencils store one transmissivity per face, boundary faces
// included: along x there are nx+1 faces per row, face i sits between cells i-1
// and i, faces 0 and nx couple to the Dirichlet ghost (value 0).  The diagonal
// of K is the sum of a cell's faces; off-diagonals are -T on interior faces.
// Every face a cell needs for its off-diagonals is also needed for its diagonal,
// so no separate diagonal array is read.
#pragma once
#include "common.hpp"

namespace shk {

template <typename F> struct Op2D {
  int nx, ny;
  const F* tx;        // (nx+1) * ny, index i + (nx+1) j
  const F* ty;        // nx * (ny+1), index i + nx j
  const double* mdiag;  // per-cell mass, or nullptr for the uniform value m0
  double m0;

  __device__ __forceinline__ double mass(long c) const { return mdiag ? mdiag[c] : m0; }

  __device__ __forceinline__ double diagK(long c) const {
    const int i = (int)(c % nx), j = (int)(c / nx);
    const long fx = i + (long)(nx + 1) * j;
    const long fy = i + (long)nx * j;
    return (double)tx[fx] + (double)tx[fx + 1] + (double)ty[fy] + (double)ty[fy + nx];
  }

  template <typename R, typename G>
  __device__ __forceinline__ cx<R> apply(long c, cx<R> sig, G g) const {
    const int i = (int)(c % nx), j = (int)(c / nx);
    const long fx = i + (long)(nx + 1) * j;
    const long fy = i + (long)nx * j;
    const R fw = (R)tx[fx], fe = (R)tx[fx + 1], fs = (R)ty[fy], fn = (R)ty[fy + nx];
    const cx<R> xc = g(c);
    const R m = (R)mass(c);
    cx<R> acc = (fw + fe + fs + fn) * xc + m * (sig * xc);
    if (i > 0) acc = acc - fw * g(c - 1);
    if (i < nx - 1) acc = acc - fe * g(c + 1);
    if (j > 0) acc = acc - fs * g(c - nx);
    if (j < ny - 1) acc = acc - fn * g(c + nx);
    return acc;
  }
};

template <typename F> struct Op3D {
  int nx, ny, nz;
  const F* tx;        // (nx+1) * ny * nz
  const F* ty;        // nx * (ny+1) * nz
  const F* tz;        // nx * ny * (nz+1)
  const double* mdiag;
  double m0;

  __device__ __forceinline__ double mass(long c) const { return mdiag ? mdiag[c] : m0; }

  __device__ __forceinline__ void coords(long c, int& i, int& j, int& k) const {
    const long pl = (long)nx * ny;
    k = (int)(c / pl);
    const long rem = c - (long)k * pl;
    j = (int)(rem / nx);
    i = (int)(rem - (long)j * nx);
  }

  __device__ __forceinline__ double diagK(long c) const {
    int i, j, k;
    coords(c, i, j, k);
    const long fx = i + (long)(nx + 1) * (j + (long)ny * k);
    const long fy = i + (long)nx * (j + (long)(ny + 1) * k);
    const long fz = c;
    return (double)tx[fx] + (double)tx[fx + 1] + (double)ty[fy] + (double)ty[fy + nx] +
           (double)tz[fz] + (double)tz[fz + (long)nx * ny];
  }

  template <typename R, typename G>
  __device__ __forceinline__ cx<R> apply(long c, cx<R> sig, G g) const {
    int i, j, k;
    coords(c, i, j, k);
    const long pl = (long)nx * ny;
    const long fx = i + (long)(nx + 1) * (j + (long)ny * k);
    const long fy = i + (long)nx * (j + (long)(ny + 1) * k);
    const R fw = (R)tx[fx], fe = (R)tx[fx + 1];
    const R fs = (R)ty[fy], fn = (R)ty[fy + nx];
    const R fd = (R)tz[c], fu = (R)tz[c + pl];
    const cx<R> xc = g(c);
    const R m = (R)mass(c);
    cx<R> acc = (fw + fe + fs + fn + fd + fu) * xc + m * (sig * xc);
    if (i > 0) acc = acc - fw * g(c - 1);
    if (i < nx - 1) acc = acc - fe * g(c + 1);
    if (j > 0) acc = acc - fs * g(c - nx);
    if (j < ny - 1) acc = acc - fn * g(c + nx);
    if (k > 0) acc = acc - fd * g(c - pl);
    if (k < nz - 1) acc = acc - fu * g(c + pl);
    return acc;
  }
};

// General sparse K (CSR, real values; the inner solver needs K symmetric).
template <typename F> struct OpCSR {
  long n;
  const int* rowptr;
  const int* col;
  const F* val;
  const double* diag;   // diagonal of K (FP64)
  const double* mdiag;  // per-row mass, or nullptr for m0
  double m0;

  __device__ __forceinline__ double mass(long c) const { return mdiag ? mdiag[c] : m0; }
  __device__ __forceinline__ double diagK(long c) const { return diag[c]; }

  template <typename R, typename G>
  __device__ __forceinline__ cx<R> apply(long c, cx<R> sig, G g) const {
    const R m = (R)mass(c);
    cx<R> acc = m * (sig * g(c));
    for (int e = rowptr[c]; e < rowptr[c + 1]; ++e) acc = acc + (R)val[e] * g(col[e]);
    return acc;
  }
};

}  // namespace shk
