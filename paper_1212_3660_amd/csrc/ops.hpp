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
  static constexpr int NB = 4;   // stencil neighbours
  int nx, ny;
  const F* tx;        // (nx+1) * ny, index i + (nx+1) j
  const F* ty;        // nx * (ny+1), index i + nx j
  const double* mdiag;  // per-cell mass, or nullptr for the uniform value m0
  double m0;

  __device__ __forceinline__ double mass(int c) const { return mdiag ? mdiag[c] : m0; }

  __device__ __forceinline__ double diagK(int c) const {
    const int j = c / nx, i = c - j * nx;
    const int fx = i + (nx + 1) * j;
    const int fy = c;
    return (double)tx[fx] + (double)tx[fx + 1] + (double)ty[fy] + (double)ty[fy + nx];
  }

  template <typename R, typename G>
  __device__ __forceinline__ cx<R> apply(int c, cx<R> sig, G g) const {
    const int j = c / nx, i = c - j * nx;
    const int fx = c + j;          // i + (nx + 1) j
    const int fy = c;              // i + nx j
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

  // Branch-free stencil: neighbour indices (clamped to c where the neighbour
  // is the Dirichlet ghost), off-diagonal multipliers (zero there) and the
  // diagonal sum of all faces, so callers can issue every load at once.
  template <typename R>
  __device__ __forceinline__ void stencil(int c, int (&idx)[NB], R (&fo)[NB], R& fsum) const {
    const int j = c / nx, i = c - j * nx;
    stencil_at<R>(i, j, 0, c, idx, fo, fsum);
  }
  // The same for cell c = i + nx j whose coordinates the caller already has.
  template <typename R>
  __device__ __forceinline__ void stencil_at(int i, int j, int, int c, int (&idx)[NB], R (&fo)[NB], R& fsum) const {
    const int fx = c + j;
    const R fw = (R)tx[fx], fe = (R)tx[fx + 1], fs = (R)ty[c], fn = (R)ty[c + nx];
    fsum = fw + fe + fs + fn;
    const bool w = i > 0, e = i < nx - 1, so = j > 0, no = j < ny - 1;
    idx[0] = w ? c - 1 : c;
    idx[1] = e ? c + 1 : c;
    idx[2] = so ? c - nx : c;
    idx[3] = no ? c + nx : c;
    fo[0] = w ? fw : (R)0;
    fo[1] = e ? fe : (R)0;
    fo[2] = so ? fs : (R)0;
    fo[3] = no ? fn : (R)0;
  }
};

template <typename F> struct Op3D {
  static constexpr int NB = 6;
  int nx, ny, nz;
  const F* tx;        // (nx+1) * ny * nz
  const F* ty;        // nx * (ny+1) * nz
  const F* tz;        // nx * ny * (nz+1)
  const double* mdiag;
  double m0;

  __device__ __forceinline__ double mass(int c) const { return mdiag ? mdiag[c] : m0; }

  __device__ __forceinline__ void coords(int c, int& i, int& j, int& k) const {
    const int pl = nx * ny;
    k = c / pl;
    const int rem = c - k * pl;
    j = rem / nx;
    i = rem - j * nx;
  }

  __device__ __forceinline__ double diagK(int c) const {
    int i, j, k;
    coords(c, i, j, k);
    const int fx = i + (nx + 1) * (j + ny * k);
    const int fy = i + nx * (j + (ny + 1) * k);
    const int fz = c;
    return (double)tx[fx] + (double)tx[fx + 1] + (double)ty[fy] + (double)ty[fy + nx] +
           (double)tz[fz] + (double)tz[fz + (long)nx * ny];
  }

  template <typename R, typename G>
  __device__ __forceinline__ cx<R> apply(int c, cx<R> sig, G g) const {
    int i, j, k;
    coords(c, i, j, k);
    const int pl = nx * ny;
    const int fx = i + (nx + 1) * (j + ny * k);
    const int fy = i + nx * (j + (ny + 1) * k);
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

  template <typename R>
  __device__ __forceinline__ void stencil(int c, int (&idx)[NB], R (&fo)[NB], R& fsum) const {
    int i, j, k;
    coords(c, i, j, k);
    stencil_at<R>(i, j, k, c, idx, fo, fsum);
  }
  // The same for cell c = i + nx (j + ny k) whose coordinates the caller has.
  template <typename R>
  __device__ __forceinline__ void stencil_at(int i, int j, int k, int c, int (&idx)[NB], R (&fo)[NB],
                                             R& fsum) const {
    const int pl = nx * ny;
    const int fx = i + (nx + 1) * (j + ny * k);
    const int fy = i + nx * (j + (ny + 1) * k);
    const R f[6] = {(R)tx[fx], (R)tx[fx + 1], (R)ty[fy], (R)ty[fy + nx], (R)tz[c], (R)tz[c + pl]};
    fsum = f[0] + f[1] + f[2] + f[3] + f[4] + f[5];
    const bool in[6] = {i > 0, i < nx - 1, j > 0, j < ny - 1, k > 0, k < nz - 1};
    const int d[6] = {-1, 1, -nx, nx, -pl, pl};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      idx[q] = in[q] ? c + d[q] : c;
      fo[q] = in[q] ? f[q] : (R)0;
    }
  }
};

// General sparse K (CSR, real values; the inner solver needs K symmetric).
template <typename F> struct OpCSR {
  static constexpr int NB = 0;   // no fixed stencil: the generic path is used
  int n;
  const int* rowptr;
  const int* col;
  const F* val;
  const double* diag;   // diagonal of K (FP64)
  const double* mdiag;  // per-row mass, or nullptr for m0
  double m0;

  __device__ __forceinline__ double mass(int c) const { return mdiag ? mdiag[c] : m0; }
  __device__ __forceinline__ double diagK(int c) const { return diag[c]; }

  template <typename R, typename G>
  __device__ __forceinline__ cx<R> apply(int c, cx<R> sig, G g) const {
    const R m = (R)mass(c);
    cx<R> acc = m * (sig * g(c));
    for (int e = rowptr[c]; e < rowptr[c + 1]; ++e) acc = acc + (R)val[e] * g(col[e]);
    return acc;
  }
};

}  // namespace shk
