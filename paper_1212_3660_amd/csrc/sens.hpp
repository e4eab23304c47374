// Sensitivity of point measurements to the log-conductivity field (section 5,
// eq. sensitivity; step 3 of Algorithm 6) for the finite-volume operator.
//
// For a forward solution Phi (A Phi = b) and an adjoint solution Psi
// (A Psi = e_m, A = K + sigma M complex symmetric), the measurement
// h = e_m^T Phi has dh/d(ln K_c) = -Psi^T (dK/d ln K_c) Phi.  K is a sum over
// faces T_f g_f g_f^T (g_f = e_a - e_b between cells a and b, g_f = e_a at a
// Dirichlet boundary face), so the derivative gathers the faces of cell c:
//
//   J_c = - sum_{faces f of c} (dT_f / d ln K_c) (g_f^T Psi)(g_f^T Phi),
//
// dT/d ln K_c = T K_other / (K_c + K_other) for a harmonic-mean interior face,
// = T for a boundary face (T = K_c h^(d-2)).  The paper's adjoint carries the
// source -delta, which flips the sign of its bilinear term.
//
// One thread per cell, shift and tile of TS forward solutions (held in
// registers as face differences); the thread
// walks the adjoint solutions and writes TS entries of J for each (c fastest,
// so every store is coalesced; streaming stores, J is not read back here).
// Face differences and products in FP64, J rounded once to its storage type.
// The launch is bound by the writes of J.
#pragma once
#include "kernels.hpp"

namespace shk {

struct SensArgs {
  int nx, ny, nz;
  const double* tx;      // faces along x, (nx+1) ny nz
  const double* ty;      // along y, nx (ny+1) nz
  const double* tz;      // along z, nx ny (nz+1) (3-D)
  const double* K;       // cell conductivity
  const c128* phi;       // phi[c + n (j + nf s)]
  const c128* psi;       // psi[c + n (j + nf r)]
  int nf, ns, nr;
};

// Launch grid (ceil(n / BS) * ceil(ns / TS), nf): the source tiles of one
// block of cells are adjacent blocks, and the linear block index goes through
// xcd_tile, so one XCD's L2 serves the neighbour rows and the adjoint
// solutions to every tile of a band of cells.
template <typename RO, int TS, int NF>
__global__ void __launch_bounds__(BS) k_sensitivity(SensArgs a, cx<RO>* __restrict__ J) {
  const long n = (long)a.nx * a.ny * a.nz;
  const int ntile = (a.ns + TS - 1) / TS;
  const int T = xcd_tile(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int j = T / gridDim.x, bx = T - j * gridDim.x;
  const long c = (long)(bx / ntile) * BS + threadIdx.x;
  if (c >= n) return;
  const int s0 = (bx % ntile) * TS;
  const int pl = a.nx * a.ny;
  const int k = (int)(c / pl), rem = (int)(c - (long)k * pl);
  const int y = rem / a.nx, x = rem - y * a.nx;
  // the cell's faces: neighbour and dT / d ln K_c; at a boundary face the
  // neighbour index is the cell itself (every load stays in range) and the
  // face uses the cell's own value alone
  int nb[NF];
  bool in[NF];
  double dT[NF];
  const double Kc = a.K[c];
  auto face = [&](int q, double T, bool inside, long other) {
    in[q] = inside;
    nb[q] = inside ? (int)other : (int)c;
    const double Ko = a.K[nb[q]];
    dT[q] = inside ? T * Ko / (Kc + Ko) : T;
  };
  const long fx = x + (long)(a.nx + 1) * (y + (long)a.ny * k);
  const long fy = x + (long)a.nx * (y + (long)(a.ny + 1) * k);
  face(0, a.tx[fx], x > 0, c - 1);
  face(1, a.tx[fx + 1], x < a.nx - 1, c + 1);
  face(2, a.ty[fy], y > 0, c - a.nx);
  face(3, a.ty[fy + a.nx], y < a.ny - 1, c + a.nx);
  if constexpr (NF == 6) {
    face(4, a.tz[c], k > 0, c - pl);
    face(5, a.tz[c + pl], k < a.nz - 1, c + pl);
  }
  // face differences of the tile's forward solutions
  c128 gphi[TS][NF];
#pragma unroll
  for (int t = 0; t < TS; ++t) {
    const int s = s0 + t < a.ns ? s0 + t : a.ns - 1;
    const c128* ph = a.phi + n * ((long)j + (long)a.nf * s);
    const c128 pc = ph[c];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      const c128 po = ph[nb[q]];
      gphi[t][q] = in[q] ? pc - po : pc;
    }
  }
  for (int r = 0; r < a.nr; ++r) {
    const c128* ps = a.psi + n * ((long)j + (long)a.nf * r);
    const c128 qc = ps[c];
    c128 gpsi[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      const c128 qo = ps[nb[q]];
      gpsi[q] = in[q] ? qc - qo : qc;
    }
#pragma unroll
    for (int t = 0; t < TS; ++t) {
      if (s0 + t >= a.ns) break;
      c128 acc{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < NF; ++q) acc = acc + dT[q] * (gpsi[q] * gphi[t][q]);
      st<true>(J + c + n * ((long)r + (long)a.nr * ((long)(s0 + t) + (long)a.ns * j)), cvt<RO>(c128{-acc.re, -acc.im}));
    }
  }
}

}  // namespace shk
