// Host driver of the flexible shifted-Krylov solver: problem setup, the outer
// loop of Algorithm 4 around the flexible Arnoldi step of Algorithm 3, restarts,
// FP64 true residuals and refinement, and the step-level entry points.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "mg.hpp"
#include "sens.hpp"
#include "block.hpp"

namespace shk {

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}
const char* last_error_text() { return g_err.c_str(); }

static int ceil_log2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}
static int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

static int grid_items(long items, int cap) {
  long b = (items + BS - 1) / BS;
  if (b < 1) b = 1;
  return (int)std::min<long>(b, cap);
}

// Blocks of the item kernels whose last block sums [G][2][S] partials: keep
// G*S bounded so that final sum stays short.


static size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Pinned staging for small device-to-host reads (one per host thread).
struct Pinned {
  void* p = nullptr;
  size_t cap = 0;
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
  void* get(size_t bytes) {
    if (bytes > cap) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      cap = 0;
      if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
      cap = bytes;
    }
    return p;
  }
};
static thread_local Pinned g_pinned;

// Inner-iteration kernel timing (shk_profile_*).
struct KernelTimer {
  bool on = false;
  long long launches = 0;
  double total_ms = 0.0, total_bytes = 0.0;
  std::vector<hipEvent_t> ev;
  void ensure(size_t pairs) {
    while (ev.size() < 2 * pairs) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      ev.push_back(e);
    }
  }
};
static KernelTimer g_timer;

// Block Gram-Schmidt timing (shk_profile_read_block): HIP events around each
// block CGS2 of the shared-basis path (its two projections V^H W and two
// updates W -= V C), with the flops of those four contractions.
struct BlockTimer {
  long long calls = 0;
  double ms = 0.0, flops = 0.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
};
static BlockTimer g_btimer;

// Phase timing (shk_profile_read_phases): HIP events recorded on the solve
// stream at the boundaries of the solve's phases.  The GPU time between two
// marks is charged to the phase the later mark closes, so time in which the
// GPU waits for the host falls into the phase whose launches follow the wait
// (the turnaround between outer steps is a phase of its own).  For one solve
// at a time; the events are read when the solve's stream has drained.
enum { PH_START, PH_INNER, PH_GS, PH_LSQ, PH_TURN, PH_ASM, PH_RESID, PH_BLOCK, PH_N };
struct PhaseTimer {
  bool on = false;
  double ms[PH_N] = {};
  std::vector<hipEvent_t> pool;
  std::vector<int> ph;      // phase closed by each recorded mark
  void mark(hipStream_t st, int phase) {
    if (!on) return;
    if (ph.size() == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      pool.push_back(e);
    }
    if (hipEventRecord(pool[ph.size()], st) == hipSuccess) ph.push_back(phase);
  }
  // after the stream has drained: charge the intervals and start over
  void flush() {
    if (!on) return;
    for (size_t i = 1; i < ph.size(); ++i) {
      float t = 0.f;
      if (ph[i] >= 0 && hipEventElapsedTime(&t, pool[i - 1], pool[i]) == hipSuccess) ms[ph[i]] += t;
    }
    ph.clear();
  }
};
static PhaseTimer g_phase;

int profile_read_phases(double* ms, int n) {
  if (!ms || n < 0) return fail(SHK_ERR_INVALID_ARG, "phase output");
  for (int i = 0; i < n && i < PH_N; ++i) ms[i] = g_phase.ms[i];
  return PH_N;
}

int profile_enable(int on) {
  g_phase.on = (on & 2) != 0;
  g_phase.ph.clear();
  for (double& v : g_phase.ms) v = 0.0;
  on &= 1;
  g_timer.on = on != 0;
  g_timer.launches = 0;
  g_timer.total_ms = 0.0;
  g_timer.total_bytes = 0.0;
  g_btimer.calls = 0;
  g_btimer.ms = 0.0;
  g_btimer.flops = 0.0;
  return SHK_OK;
}
int profile_read_block(long long* calls, double* ms, double* flops) {
  if (calls) *calls = g_btimer.calls;
  if (ms) *ms = g_btimer.ms;
  if (flops) *flops = g_btimer.flops;
  return SHK_OK;
}
int profile_read(long long* launches, double* ms, double* bytes) {
  if (launches) *launches = g_timer.launches;
  if (ms) *ms = g_timer.total_ms;
  if (bytes) *bytes = g_timer.total_bytes;
  return SHK_OK;
}

// --------------------------------------------------------------- problem ---
// Device arrays of a problem: from its bump region when it has one, else from
// the stream-ordered HIP allocator.
static hipError_t dev_alloc(shk_problem* p, void** ptr, size_t bytes, hipStream_t st) {
  if (p->bump) {
    *ptr = p->bump->take(bytes);
    return *ptr ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMallocAsync(ptr, bytes, st);
}

void problem_free(shk_problem* p, hipStream_t st) {
  if (p->bump) {   // the region's owner releases it as a whole
    p->mg.clear();
    return;
  }
  void* ptrs[] = {p->tx, p->ty, p->tz, p->tx32, p->ty32, p->tz32, p->rowptr, p->col, p->val, p->val32, p->diag, p->mdiag,
                  p->dK, p->dK32, p->cellK};
  for (void* q : ptrs)
    if (q) (void)hipFreeAsync(q, st);
  for (MgLevel& l : p->mg) {
    for (int a = 0; a < 3; ++a) {
      if (l.t[a]) (void)hipFreeAsync(l.t[a], st);
      if (l.t32[a]) (void)hipFreeAsync(l.t32[a], st);
    }
    if (l.mass) (void)hipFreeAsync(l.mass, st);
  }
  p->mg.clear();
  (void)hipStreamSynchronize(st);
}

// Coarse levels of the multigrid hierarchy, down to one cell: faces (half the
// sum of the fine faces each covers) and mass (the sum over the group).
// The V-cycle's grid kernels put rows and planes on the launch grid's y and z.
static bool mg_grid_ok(const shk_problem* p) { return p->ny <= 65535 && p->nz <= 65535; }

static int mg_setup(shk_problem* p, hipStream_t st) {
  const int d = p->kind == Kind::FV3D ? 3 : 2;
  LevelDims f{p->nx, p->ny, p->nz};
  const double* ft[3] = {p->tx, p->ty, p->tz};
  const double* fm = nullptr;
  while (f.n() > 1) {
    const LevelDims c = f.coarse();
    MgLevel l;
    l.nx = c.nx; l.ny = c.ny; l.nz = c.nz; l.n = c.n();
    p->mg.push_back(l);
    MgLevel& L = p->mg.back();
    for (int a = 0; a < d; ++a) {
      const long cnt = (long)(c.nx + (a == 0)) * (c.ny + (a == 1)) * (c.nz + (a == 2));
      if (dev_alloc(p, (void**)&L.t[a], cnt * sizeof(double), st) != hipSuccess ||
          dev_alloc(p, (void**)&L.t32[a], cnt * sizeof(float), st) != hipSuccess)
        return fail(SHK_ERR_OOM, "multigrid faces");
      k_mg_faces<<<grid_items(cnt, 4096), BS, 0, st>>>(f, c, a, ft[a], L.t[a], L.t32[a]);
      SHK_HIP(hipGetLastError());
    }
    if (dev_alloc(p, (void**)&L.mass, (size_t)c.n() * sizeof(double), st) != hipSuccess)
      return fail(SHK_ERR_OOM, "multigrid mass");
    k_mg_mass<<<grid_items(c.n(), 4096), BS, 0, st>>>(f, c, fm, p->m0, L.mass);
    SHK_HIP(hipGetLastError());
    for (int a = 0; a < 3; ++a) ft[a] = L.t[a];
    fm = L.mass;
    f = c;
  }
  return SHK_OK;
}

// The multigrid levels' dimensions without device arrays (for sizing a
// workspace before the problem is set up).
void problem_plan_levels(shk_problem* p) {
  p->mg.clear();
  LevelDims f{p->nx, p->ny, p->nz};
  while (f.n() > 1) {
    const LevelDims c = f.coarse();
    MgLevel l;
    l.nx = c.nx; l.ny = c.ny; l.nz = c.nz; l.n = c.n();
    p->mg.push_back(l);
    f = c;
  }
}

// Device bytes of a problem's arrays (an upper bound: every array rounded up
// to the 256-byte alignment of a bump region).
size_t problem_bytes(const shk_problem* p) {
  if (p->kind == Kind::CSR) return (size_t)p->nnz * 16 + (size_t)p->n * 24 + 16 * 256;
  const size_t faces = (size_t)(p->nx + 1) * p->ny * p->nz + (size_t)p->nx * (p->ny + 1) * p->nz +
                       (p->kind == Kind::FV3D ? (size_t)p->nx * p->ny * (p->nz + 1) : 0);
  // the multigrid hierarchy from the grid dimensions (set up or not yet)
  size_t coarse = 0, levels = 0;
  LevelDims f{p->nx, p->ny, p->nz};
  while (f.n() > 1) {
    const LevelDims l = f.coarse();
    coarse += (size_t)l.n() * 8 + ((size_t)(l.nx + 1) * l.ny * l.nz + (size_t)l.nx * (l.ny + 1) * l.nz +
                                   (p->kind == Kind::FV3D ? (size_t)l.nx * l.ny * (l.nz + 1) : 0)) * 12;
    ++levels;
    f = l;
  }
  const size_t arrays = 16 + 8 * levels;
  return faces * 12 + (size_t)p->n * 20 + coarse + arrays * 256;
}

int problem_setup_fv(shk_problem* p, const double* K, double Ss, double h, hipStream_t st) {
  const long n = (long)p->nx * p->ny * p->nz;
  for (long i = 0; i < n; ++i)
    if (!(K[i] > 0.0) || !std::isfinite(K[i])) return fail(SHK_ERR_INVALID_ARG, "cell_K must be finite and > 0");
  if (!(Ss > 0.0) || !(h > 0.0) || !std::isfinite(Ss) || !std::isfinite(h))
    return fail(SHK_ERR_INVALID_ARG, "Ss and h must be finite and > 0");
  SHK_HIP(hipGetDevice(&p->device));
  p->n = n;
  const int d = p->kind == Kind::FV3D ? 3 : 2;
  const double scale = std::pow(h, d - 2);
  p->m0 = Ss * std::pow(h, d);
  double* Kd = nullptr;
  if (dev_alloc(p, (void**)&Kd, n * sizeof(double), st) != hipSuccess) return fail(SHK_ERR_OOM, "cell field");
  SHK_HIP(hipMemcpyAsync(Kd, K, n * sizeof(double), hipMemcpyHostToDevice, st));
  const int axes = d;
  double** T[3] = {&p->tx, &p->ty, &p->tz};
  float** T32[3] = {&p->tx32, &p->ty32, &p->tz32};
  for (int a = 0; a < axes; ++a) {
    const long cnt = (long)(p->nx + (a == 0)) * (p->ny + (a == 1)) * (p->nz + (a == 2));
    if (dev_alloc(p, (void**)T[a], cnt * sizeof(double), st) != hipSuccess ||
        dev_alloc(p, (void**)T32[a], cnt * sizeof(float), st) != hipSuccess) {
      if (!p->bump) (void)hipFreeAsync(Kd, st);
      return fail(SHK_ERR_OOM, "face arrays");
    }
    k_faces<<<grid_items(cnt, 8192), BS, 0, st>>>(Kd, p->nx, p->ny, p->nz, a, scale, *T[a], *T32[a]);
    SHK_HIP(hipGetLastError());
  }
  if (dev_alloc(p, (void**)&p->dK, n * sizeof(double), st) != hipSuccess ||
      dev_alloc(p, (void**)&p->dK32, n * sizeof(float), st) != hipSuccess)
    return fail(SHK_ERR_OOM, "diagonal arrays");
  if (p->kind == Kind::FV3D) {
    Op3D<double> od{p->nx, p->ny, p->nz, p->tx, p->ty, p->tz, nullptr, p->m0};
    k_diag<<<grid_items(n, 8192), BS, 0, st>>>(od, n, p->dK, p->dK32);
  } else {
    Op2D<double> od{p->nx, p->ny, p->tx, p->ty, nullptr, p->m0};
    k_diag<<<grid_items(n, 8192), BS, 0, st>>>(od, n, p->dK, p->dK32);
  }
  SHK_HIP(hipGetLastError());
  p->cellK = Kd;   // kept for sensitivities
  SHK_TRY(mg_setup(p, st));
  SHK_HIP(hipStreamSynchronize(st));
  return SHK_OK;
}

int problem_setup_csr(shk_problem* p, const int* rowptr, const int* col, const double* val, const double* mdiag,
                      hipStream_t st) {
  const long n = p->n;
  if (rowptr[0] != 0) return fail(SHK_ERR_INVALID_ARG, "rowptr[0] must be 0");
  for (long i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return fail(SHK_ERR_INVALID_ARG, "rowptr not monotone");
  const long nnz = rowptr[n];
  std::vector<double> dg(n, 0.0);
  std::vector<float> v32(nnz);
  for (long i = 0; i < n; ++i)
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n) return fail(SHK_ERR_INVALID_ARG, "column index out of range");
      if (!std::isfinite(val[e])) return fail(SHK_ERR_INVALID_ARG, "non-finite K value");
      if (col[e] == i) dg[i] += val[e];
      v32[e] = (float)val[e];
    }
  for (long i = 0; i < n; ++i)
    if (!std::isfinite(mdiag[i])) return fail(SHK_ERR_INVALID_ARG, "non-finite mass");
  SHK_HIP(hipGetDevice(&p->device));
  p->nnz = nnz;
  p->nx = (int)std::ceil(std::sqrt((double)n));
  SHK_HIP(hipMallocAsync((void**)&p->rowptr, (n + 1) * sizeof(int), st));
  SHK_HIP(hipMallocAsync((void**)&p->col, std::max<long>(nnz, 1) * sizeof(int), st));
  SHK_HIP(hipMallocAsync((void**)&p->val, std::max<long>(nnz, 1) * sizeof(double), st));
  SHK_HIP(hipMallocAsync((void**)&p->val32, std::max<long>(nnz, 1) * sizeof(float), st));
  SHK_HIP(hipMallocAsync((void**)&p->diag, n * sizeof(double), st));
  SHK_HIP(hipMallocAsync((void**)&p->mdiag, n * sizeof(double), st));
  SHK_HIP(hipMallocAsync((void**)&p->dK, n * sizeof(double), st));
  SHK_HIP(hipMallocAsync((void**)&p->dK32, n * sizeof(float), st));
  SHK_HIP(hipMemcpyAsync(p->rowptr, rowptr, (n + 1) * sizeof(int), hipMemcpyHostToDevice, st));
  SHK_HIP(hipMemcpyAsync(p->col, col, nnz * sizeof(int), hipMemcpyHostToDevice, st));
  SHK_HIP(hipMemcpyAsync(p->val, val, nnz * sizeof(double), hipMemcpyHostToDevice, st));
  SHK_HIP(hipMemcpyAsync(p->val32, v32.data(), nnz * sizeof(float), hipMemcpyHostToDevice, st));
  SHK_HIP(hipMemcpyAsync(p->diag, dg.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
  SHK_HIP(hipMemcpyAsync(p->mdiag, mdiag, n * sizeof(double), hipMemcpyHostToDevice, st));
  std::vector<float> dg32(dg.begin(), dg.end());
  SHK_HIP(hipMemcpyAsync(p->dK, dg.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
  SHK_HIP(hipMemcpyAsync(p->dK32, dg32.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
  SHK_HIP(hipStreamSynchronize(st));
  return SHK_OK;
}

template <typename F> static const F* pick(const double* a, const float* b);
template <> const double* pick<double>(const double* a, const float*) { return a; }
template <> const float* pick<float>(const double*, const float* b) { return b; }

template <typename F> static Op2D<F> op2d(const shk_problem* p) {
  return Op2D<F>{p->nx, p->ny, pick<F>(p->tx, p->tx32), pick<F>(p->ty, p->ty32), nullptr, p->m0};
}
template <typename F> static Op3D<F> op3d(const shk_problem* p) {
  return Op3D<F>{p->nx, p->ny, p->nz, pick<F>(p->tx, p->tx32), pick<F>(p->ty, p->ty32), pick<F>(p->tz, p->tz32),
                 nullptr, p->m0};
}
template <typename F> static OpCSR<F> opcsr(const shk_problem* p) {
  return OpCSR<F>{(int)p->n, p->rowptr, p->col, pick<F>(p->val, p->val32), p->diag, p->mdiag, 0.0};
}

// Calls fn(op, opd): the operator with faces in precision F and in FP64.
template <typename F, typename Fn> static int with_ops(const shk_problem* p, Fn&& fn) {
  switch (p->kind) {
    case Kind::FV2D: return fn(op2d<F>(p), op2d<double>(p));
    case Kind::FV3D: return fn(op3d<F>(p), op3d<double>(p));
    default: return fn(opcsr<F>(p), opcsr<double>(p));
  }
}
template <typename F, typename Fn> static int with_op(const shk_problem* p, Fn&& fn) {
  return with_ops<F>(p, [&](auto op, auto) { return fn(op); });
}

// Launch and round settings of the solver, per workload class.  Defaults are
// the fastest measured on MI355X at the benchmarked workloads; the table
// below holds what shk_tune_set (the autotuner) picked for a class.
//  cgb         block size of the iteration kernels (256 or 512)
//  nt64, nt32  streaming (non-temporal) stores of the Jacobi step, per precision
//  sep_limit   partial count above which a separate kernel folds the partials
//  skew        bytes added between the large workspace arrays
//  round_tol   complex64 inner rounds: reduction per round (Jacobi / multigrid)
//  stall_*     stall rule of a round (no halving for max(min, mult x length))
//  tail_lds    LDS budget of the V-cycle's one-workgroup tail
//  tail_lanes  lanes per workgroup of that tail (0: all; else the lanes are
//              split over several workgroups, and the tail starts where the
//              levels of that many lanes fit)
//  mg_fuse     step fused with the finest restriction where it applies
//  post_lt, down_lt, up_lt   lanes per thread of the product and grid legs
//              (complex64, several lanes); lt64 the same on complex128
//  graph       inner iterations replayed from a captured HIP graph
//  mg_chain    2-D, one lane: up to 3 middle legs of each V-cycle direction in
//              one launch
//  asm_mfma    solution assembly X = Z Y on the FP64 matrix cores
//  tile3_post, post3_lt   3-D, several lanes, finest level plane-marching: the
//              product w = A u on the same tiles, post3_lt complex64 lanes per thread
//  rows, rows64, rows_yb   2-D levels of at least `rows` (complex64) or
//              `rows64` (complex128) cells, several lanes: legs marching
//              rows_yb rows per block
//  tile3, tile3_zb, tile3_lt   3-D levels of at least tile3 cells: plane-
//              marching grid legs, tile3_zb planes per block, tile3_lt complex64
//              lanes per thread
struct Tune {
  int cgb = 256;
  int nt64 = 0;
  int nt32 = 1;
  long sep_limit = 3072;
  size_t skew = 0;
  double round_tol = 1e-2;
  double round_tol_mg = 1e-3;
  int stall_min = 150, stall_mult = 3;
  int tail_lds = MG_TAIL_LDS;
  int tail_lanes = 1;  // lanes per tail workgroup (0: all lanes in one)
  int mg_fuse = 1;
  int post_lt = 2;
  int down_lt = 4, up_lt = 4;
  int lt64 = 2;
  int graph = 0;
  long tile3 = 262144;  // 3-D levels with at least this many cells use the plane-marching legs (0: none)
  int tile3_zb = 4;     // planes per block of those legs (even)
  int tile3_lt = 4;   // complex64 lanes per thread of those legs (4 or 8)
  int mg_chain = 0;   // 2-D one-lane V-cycle: chain up to 3 middle legs per launch
  int asm_mfma = 1;   // solution assembly on the FP64 matrix cores
  int tile3_post = 0; // the product w = A u on the plane-marching tiles too (3-D, several lanes)
  int post3_lt = 2;   // complex64 lanes per thread of that product (2 or 4)
  long rows = 0;        // 2-D levels of at least this many cells, several complex64 lanes: row-marching legs
  long rows64 = 16384;  // the same for complex128 lanes (0: none)
  int rows_yb = 4;      // rows per block of those legs (even)

  // Sets a knob by name; false for an unknown name or a value out of range.
  bool set(const std::string& k, double v) {
    const int iv = (int)v;
    auto chunk = [](int x) { return x >= 8 ? 8 : x >= 4 ? 4 : 2; };
    if (k == "cg_block") { if (iv != 256 && iv != 512) return false; cgb = iv; }
    else if (k == "nt_store") { nt64 = nt32 = iv != 0; }
    else if (k == "nt_store64") { nt64 = iv != 0; }
    else if (k == "nt_store32") { nt32 = iv != 0; }
    else if (k == "sep_limit") { if (v < 0) return false; sep_limit = (long)v; }
    else if (k == "ws_skew") { if (v < 0) return false; skew = (size_t)v & ~size_t(255); }
    else if (k == "round_tol") { if (!(v > 0 && v < 1)) return false; round_tol = v; }
    else if (k == "round_tol_mg") { if (!(v > 0 && v < 1)) return false; round_tol_mg = v; }
    else if (k == "stall_min") { if (iv < 0) return false; stall_min = iv; }
    else if (k == "stall_mult") { if (iv < 0) return false; stall_mult = iv; }
    else if (k == "tail_lds") { if (iv < 0 || iv > MG_TAIL_LDS_MAX) return false; tail_lds = iv; }
    else if (k == "tail_lanes") { if (iv < 0 || iv > 64 || (iv & (iv - 1))) return false; tail_lanes = iv; }
    else if (k == "mg_fuse") { mg_fuse = iv != 0; }
    else if (k == "post_lt") { post_lt = iv >= 8 ? 8 : iv >= 4 ? 4 : iv >= 2 ? 2 : 0; }
    else if (k == "down_lt") { down_lt = chunk(iv); }
    else if (k == "up_lt") { up_lt = chunk(iv); }
    else if (k == "lt64") { lt64 = iv >= 4 ? 4 : iv >= 2 ? 2 : 0; }
    else if (k == "graph") { graph = iv != 0; }
    else if (k == "tile3") { if (v < 0) return false; tile3 = (long)v; }
    else if (k == "tile3_zb") { if (iv < 2 || iv > 64 || (iv & 1)) return false; tile3_zb = iv; }
    else if (k == "tile3_lt") { if (iv != 2 && iv != 4 && iv != 8) return false; tile3_lt = iv; }
    else if (k == "mg_chain") { if (iv < 0 || iv > 1) return false; mg_chain = iv; }
    else if (k == "asm_mfma") { asm_mfma = iv != 0; }
    else if (k == "tile3_post") { tile3_post = iv != 0; }
    else if (k == "post3_lt") { if (iv != 2 && iv != 4) return false; post3_lt = iv; }
    else if (k == "rows") { if (v < 0) return false; rows = (long)v; }
    else if (k == "rows64") { if (v < 0) return false; rows64 = (long)v; }
    else if (k == "rows_yb") { if (iv < 2 || iv > 256 || (iv & 1)) return false; rows_yb = iv; }
    else return false;
    return true;
  }
  bool get(const std::string& k, double* v) const {
    if (k == "cg_block") *v = cgb;
    else if (k == "nt_store64") *v = nt64;
    else if (k == "nt_store32" || k == "nt_store") *v = nt32;
    else if (k == "sep_limit") *v = (double)sep_limit;
    else if (k == "ws_skew") *v = (double)skew;
    else if (k == "round_tol") *v = round_tol;
    else if (k == "round_tol_mg") *v = round_tol_mg;
    else if (k == "stall_min") *v = stall_min;
    else if (k == "stall_mult") *v = stall_mult;
    else if (k == "tail_lds") *v = tail_lds;
    else if (k == "tail_lanes") *v = tail_lanes;
    else if (k == "mg_fuse") *v = mg_fuse;
    else if (k == "post_lt") *v = post_lt;
    else if (k == "down_lt") *v = down_lt;
    else if (k == "up_lt") *v = up_lt;
    else if (k == "lt64") *v = lt64;
    else if (k == "graph") *v = graph;
    else if (k == "tile3") *v = (double)tile3;
    else if (k == "tile3_zb") *v = tile3_zb;
    else if (k == "tile3_lt") *v = tile3_lt;
    else if (k == "mg_chain") *v = mg_chain;
    else if (k == "asm_mfma") *v = asm_mfma;
    else if (k == "tile3_post") *v = tile3_post;
    else if (k == "post3_lt") *v = post3_lt;
    else if (k == "rows") *v = (double)rows;
    else if (k == "rows64") *v = (double)rows64;
    else if (k == "rows_yb") *v = rows_yb;
    else return false;
    return true;
  }
};
static const Tune g_tune_default;

// A workload class: operator kind, unknowns, lanes, precision, inner
// preconditioner.
struct TuneKey {
  int kind;
  long long n;
  int lanes, precision, precond;
  bool operator<(const TuneKey& o) const {
    if (kind != o.kind) return kind < o.kind;
    if (n != o.n) return n < o.n;
    if (lanes != o.lanes) return lanes < o.lanes;
    if (precision != o.precision) return precision < o.precision;
    return precond < o.precond;
  }
};
static std::mutex g_tune_mu;
static Tune g_tune_base;                  // every class without an entry of its own
static std::map<TuneKey, Tune> g_tune_table;
static thread_local const Tune* t_tune = &g_tune_default;

// The settings in force on this thread (those of the running solve's class).
static const Tune& tn() { return *t_tune; }

static int tune_kind(const shk_problem* p) { return p->kind == Kind::FV2D ? 0 : p->kind == Kind::FV3D ? 1 : 2; }

// Selects the settings of a class for the scope of a solve on this thread.
struct TuneScope {
  const Tune* prev;
  Tune local;
  TuneScope(int kind, long long n, int lanes, int precision, int precond) : prev(t_tune) {
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      auto it = g_tune_table.find(TuneKey{kind, n, lanes, precision, precond});
      local = it != g_tune_table.end() ? it->second : g_tune_base;
    }
    t_tune = &local;
  }
  ~TuneScope() { t_tune = prev; }
};

// kind < 0 addresses the settings of every class without an entry of its own.
int tune_set(int kind, long long n, int lanes, int precision, int precond, const char* knob, double value) {
  if (!knob) return fail(SHK_ERR_INVALID_ARG, "null knob name");
  std::lock_guard<std::mutex> g(g_tune_mu);
  if (kind < 0) {
    Tune t = g_tune_base;
    if (!t.set(knob, value)) return fail(SHK_ERR_INVALID_ARG, std::string("unknown knob or value: ") + knob);
    g_tune_base = t;
    return SHK_OK;
  }
  const TuneKey key{kind, n, lanes, precision, precond};
  auto it = g_tune_table.find(key);
  Tune t = it != g_tune_table.end() ? it->second : g_tune_base;
  if (!t.set(knob, value)) return fail(SHK_ERR_INVALID_ARG, std::string("unknown knob or value: ") + knob);
  g_tune_table[key] = t;
  return SHK_OK;
}
int tune_get(int kind, long long n, int lanes, int precision, int precond, const char* knob, double* value) {
  if (!knob || !value) return fail(SHK_ERR_INVALID_ARG, "null knob name or value");
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = kind < 0 ? g_tune_table.end() : g_tune_table.find(TuneKey{kind, n, lanes, precision, precond});
  const Tune& t = it != g_tune_table.end() ? it->second : g_tune_base;
  if (!t.get(knob, value)) return fail(SHK_ERR_INVALID_ARG, std::string("unknown knob: ") + knob);
  return SHK_OK;
}
int tune_reset() {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_table.clear();
  g_tune_base = g_tune_default;
  return SHK_OK;
}

// ------------------------------------------------ captured inner iterations --
// HIP graphs of two inner iterations (an even and an odd one: the parities
// alternate the vector buffers and partial-sum slots), one per tau, captured
// on the solve stream by the first inner solve with that tau and replayed for
// every pair of iterations after that.  Every argument of the captured
// launches is fixed for the life of a solve's workspace layout except tau: the
// settings are read from device memory and the right-hand side and iterate
// sit in fixed buffers.  Owned by one solve, destroyed after its stream has
// drained.
struct GraphSet {
  hipStream_t st = nullptr;
  std::vector<std::pair<c128, hipGraphExec_t>> execs;
  hipGraphExec_t find(c128 tau) const {
    for (const auto& e : execs)
      if (e.first.re == tau.re && e.first.im == tau.im) return e.second;
    return nullptr;
  }
  ~GraphSet() {
    if (execs.empty()) return;
    (void)hipStreamSynchronize(st);
    for (auto& e : execs) (void)hipGraphExecDestroy(e.second);
  }
};

// ----------------------------------------------------------- workspace -----
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T> T* take(size_t count) {
    T* r = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    if (count * sizeof(T) >= (1u << 20)) off += tn().skew;   // large arrays only
    return r;
  }
};

// Item-kernel grid and reduction mode.  Consumers sum the producer's block
// partials themselves while that is cheap (few blocks x lanes); otherwise a
// one-block-per-lane kernel folds them into totals first.
struct Grid {
  int G;          // blocks of the item kernels
  bool separate;  // fold partials with k_lane_totals before consumers read them
};
static Grid item_plan(long N, int S) {
  const int CGB = tn().cgb;
  long G = (N + CGB - 1) / CGB;
  G = std::max<long>(1, std::min<long>(G, 2048));
  Grid g{(int)G, G * 3 * S > tn().sep_limit};
  return g;
}

template <typename R> struct Buffers {
  cx<R>*V, *W, *cr[2], *cw[2], *cs[2], *cp;
  c128* Z;                // flexible basis (FP64 on both paths)
  c128 *cpart[2], *ctot[2], *part;
  cx<R>* dinv;            // inverse Jacobi diagonal of the current inner solve
  CgScal* sc;             // two buffers of S lanes
  int* all_done;
  CgCfg* cfgd;            // settings of the running inner solve
  // captured inner iterations: fixed right-hand side and iterate buffers
  // (the basis column in use is copied in and the iterate out)
  cx<R>* gv = nullptr;
  c128* gx = nullptr;
  double *beta0, *hn, *mz, *pn, *nzs;
  c128 *H, *h2, *taus, *sigma, *zs;
  int *seed, *nact;
  double* qmax;           // per rhs: largest relative quasi-residual of the running lanes
  LaneState* ls;
  double* rc;
  c128 *rs, *g, *Rp, *Yb, *Yt, *ascale, *extra;
  c128 *bint, *rsv, *X;
  c128* ostage = nullptr;     // device staging of host ROWS / FACTORED output
  long long* rows = nullptr;  // cells of ROWS output
  c128* rpart;      // residual partials [s][nf][Gr]
  c128* rrow;       // residual rows [s*nf]
  // multigrid inner preconditioner: u = B r, and per coarse level l >= 1 the
  // right-hand side, solution and inverse diagonal of the V-cycle
  cx<R>* u = nullptr;
  std::vector<cx<R>*> mb, mx, mdinv;
  unsigned* mpack = nullptr;   // the V-cycle tail's packed coefficients
  // block FGMRES-Sh (one basis shared by the S right-hand sides)
  c128* Hb = nullptr;          // block Hessenberg, ((m+1) S) x (m S) column-major
  void* gpart = nullptr;       // chunk partials of the block projections
  cx<R>* Cc = nullptr;         // this pass's projection coefficients, (m+1) blocks S x S
  cx<R>* Rinv = nullptr;       // inverse of a CholQR factor (S x S, row-major)
  c128 *Gm = nullptr, *Rrow = nullptr, *beta_blk = nullptr, *Rinv64 = nullptr;
  double* fro = nullptr;       // ||H_{k+1,k}||_F^2
  int* broke = nullptr;        // breakdown flag of the current step
  c128 *Rf = nullptr, *Vr = nullptr, *Gq = nullptr, *Yp = nullptr;
  c128 *Qb = nullptr, *Rdinv = nullptr, *Tile = nullptr, *Gw = nullptr;
  double *Tr = nullptr, *brho = nullptr;
  int* want = nullptr;
  size_t bytes;
};

// Chunk partials of one block projection: at most BLK_WAVES waves' S x S
// complex128 results.
constexpr int BLK_WAVES = 2048;

// Block-basis buffers (block FGMRES-Sh) for nf shifts, S columns, m steps.
template <typename R> static void carve_block(Carver& cv, Buffers<R>& b, int m, int nf, int S) {
  const size_t ldh = (size_t)(m + 1) * S, mS = (size_t)m * S;
  b.Hb = cv.take<c128>(ldh * mS);
  b.gpart = cv.take<c128>((size_t)BLK_WAVES * S * S);
  b.Cc = cv.take<cx<R>>((m + 1) * (size_t)S * S);
  b.Rinv = cv.take<cx<R>>((size_t)S * S);
  b.Gm = cv.take<c128>((size_t)S * S);
  b.Rrow = cv.take<c128>((size_t)S * S);
  b.beta_blk = cv.take<c128>((size_t)S * S);
  b.Rinv64 = cv.take<c128>((size_t)S * S);
  b.fro = cv.take<double>(2);
  b.broke = cv.take<int>(4);
  b.Rf = cv.take<c128>((size_t)nf * (mS * (mS + 1) / 2));
  b.Vr = cv.take<c128>((size_t)nf * S * (S + 1));
  b.Tr = cv.take<double>((size_t)nf * S);
  b.Qb = cv.take<c128>((size_t)nf * m * 4 * S * S);
  b.Rdinv = cv.take<c128>((size_t)nf * m * S * S);
  b.Tile = cv.take<c128>((size_t)nf * 2 * S * S);
  b.Gq = cv.take<c128>((size_t)nf * ldh * S);
  b.Yp = cv.take<c128>((size_t)nf * S * mS);
  b.Gw = cv.take<c128>((size_t)nf * S * mS);
  b.brho = cv.take<double>((size_t)nf * S);
  b.want = cv.take<int>((size_t)nf * S);
}

// Multigrid buffers for S lanes over the coarse levels of p (none: no levels).
template <typename R> static void carve_mg(Carver& cv, Buffers<R>& b, const shk_problem* p, long N, int S) {
  b.u = cv.take<cx<R>>(N);
  b.mb.clear(); b.mx.clear(); b.mdinv.clear();
  for (const MgLevel& l : p->mg) {
    b.mb.push_back(cv.take<cx<R>>((size_t)l.n * S));
    b.mx.push_back(cv.take<cx<R>>((size_t)l.n * S));
    b.mdinv.push_back(cv.take<cx<R>>((size_t)l.n));
  }
  b.mpack = cv.take<unsigned>(MG_TAIL_LDS_MAX / 4);
}

// Norms from block partials: one block for few lanes, one block per lane
// from 4 lanes up (a single block would leave BS / S threads per lane).
template <int NV>
static void launch_final_sqrt(const c128* part, int G, int S, double* out0, double* out1, c128* hcol,
                              hipStream_t st) {
  if (S >= 4) k_final_sqrt_lanes<NV><<<S, BS, 0, st>>>(part, G, S, out0, out1, hcol);
  else k_final_sqrt<NV><<<1, BS, 0, st>>>(part, G, S, out0, out1, hcol);
}

static int resid_grid(long n) { return grid_items(n, 256); }

// X (+)= Z Y (Algorithm 4, x = Z y): Y staged in LDS when the block's JT
// columns for every rhs lane fit in 64 KB, else read per item.
template <typename R>
static void launch_assemble(long n, int S, int s_real, int nf, int kc, int m, const cx<R>* Z, size_t cstride,
                            const c128* Yb, const c128* ascale, c128* X, int acc, hipStream_t st,
                            c128* Yt = nullptr) {
  const long N = n * S;
  if (tn().asm_mfma) {
    // matrix cores: a wave per (16 cells, lane, 64 shifts); with 4 lanes or
    // more the tiles go in groups of 8 (one per XCD slot) x S/4 lane groups
    const long tiles = (n + 15) / 16;
    const long blocks = S >= 4 ? (tiles + 7) / 8 * 8 * (S / 4) : (tiles * S + 3) / 4;
    const dim3 grid((unsigned)blocks, (unsigned)((nf + 63) / 64));
    k_assemble_mfma<R, 4><<<grid, 256, 0, st>>>(n, S, s_real, nf, kc, m, Z, cstride, Yb, ascale, X, acc);
    return;
  }
  const size_t lds = (size_t)kc * JT * S * sizeof(c128);
  if (lds <= 65536) {
    dim3 grid(grid_items((N + 1) / 2, 4096), (nf + JT - 1) / JT);
    k_assemble_lds<R><<<grid, BS, lds, st>>>(n, S, s_real, nf, kc, m, Z, cstride, Yb, ascale, X, acc);
  } else if (Yt && S > 1) {
    k_y_transpose<<<grid_items((long)nf * kc * S, 1024), BS, 0, st>>>(S, nf, kc, m, Yb, Yt);
    constexpr int CT = 4, JQ = 8;
    int lS = 0;
    while ((1 << lS) < S) ++lS;
    dim3 grid(grid_items((n + CT - 1) / CT * S, 4096), (nf + JQ - 1) / JQ);
    k_assemble_rb<R, CT, JQ><<<grid, BS, 0, st>>>(n, S, lS, s_real, nf, kc, m, Z, cstride, Yt, ascale, X, acc);
  } else {
    dim3 grid(grid_items(N, 4096), (nf + JT - 1) / JT);
    k_assemble<R><<<grid, BS, 0, st>>>(n, S, s_real, nf, kc, m, Z, cstride, Yb, ascale, X, acc);
  }
}

// Bases up to GIVW_MAXM columns: a wave per (shift, rhs) lane; longer ones a
// thread per lane.
static size_t givens_wave_lds(int m) {
  return ((size_t)m * (m + 1) / 2 + 2 * (size_t)m + 2) * sizeof(c128) + (size_t)m * sizeof(double);
}

static void launch_givens(const GivensArgs& a, hipStream_t st) {
  if (a.m <= GIVW_MAXM)
    k_givens_wave<<<a.L, 64, givens_wave_lds(a.m), st>>>(a);
  else
    k_givens<<<(a.L + BS - 1) / BS, BS, 0, st>>>(a);
}
// Items per block of the Gram-Schmidt dot kernel (at least 256): about 512
// blocks (two per CU) while the vectors are small and the launch is
// latency-bound; about 2048 from 4 Mi items up, where the kernel streams and
// needs more waves in flight.
static long dot_ipb(long N) {
  const long blocks = N >= (4L << 20) ? 2048 : 512;
  long ipb = (N + blocks - 1) / blocks;
  ipb = std::max<long>(256, (ipb + 255) / 256 * 256);
  return ipb;
}

// Gram-Schmidt of w against kc columns of V (Algorithm 3): CGS2, two block
// passes (dot products of every column, then one update), or the paper's MGS,
// one column at a time (its dot product, then its update).  H receives the kc
// coefficients (summed over the two CGS2 passes); the last update leaves the
// partials of ||w||^2 over the update's blocks in part for k_final_sqrt.
template <typename R>
static void gram_schmidt(long N, int S, int kc, cx<R>* V, cx<R>* w, c128* H, c128* h2, c128* part, bool mgs,
                         hipStream_t st) {
  const long ipb = dot_ipb(N);
  const int Gd = (int)((N + ipb - 1) / ipb);
  const int Gu = (int)((N + (long)BS * GSQ - 1) / ((long)BS * GSQ));
  if (!mgs) {
    for (int pass = 0; pass < 2; ++pass) {
      k_gs_dot<R><<<Gd, BS, 0, st>>>(N, S, kc, V, (size_t)N, w, part, ipb);
      k_gs_reduce<<<kc * S, BS, 0, st>>>(part, Gd, kc, S, H, h2, pass);
      k_gs_update<R><<<Gu, BS, 0, st>>>(N, S, kc, V, (size_t)N, h2, w, pass, part);
    }
    return;
  }
  for (int i = 0; i < kc; ++i) {
    cx<R>* Vi = V + (size_t)i * N;
    k_gs_dot<R><<<Gd, BS, 0, st>>>(N, S, 1, Vi, (size_t)N, w, part, ipb);
    k_gs_reduce<<<S, BS, 0, st>>>(part, Gd, 1, S, H + (size_t)i * S, h2, 0);
    k_gs_update<R><<<Gu, BS, 0, st>>>(N, S, 1, Vi, (size_t)N, h2, w, i == kc - 1 ? 1 : 0, part);
  }
}

// Where a group's solution goes.  X itself is formed in the caller's buffer
// for device FULL output, otherwise in the workspace; host ROWS / FACTORED
// output is staged on the device first.
struct OutPlan {
  int mode = SHK_OUT_FULL;
  bool internal_x = false;
  size_t stage = 0;    // complex elements of device staging (host ROWS / FACTORED output)
  int n_rows = 0;
  int kcap = 0;
};
static int factored_kcap(const shk_params* prm) {
  return prm->m_restart * (prm->max_restarts + 1) * (prm->max_refine + 1);
}
static OutPlan out_plan(const shk_params* prm, long n, int nf, int s_real, bool host_x) {
  OutPlan o;
  o.mode = prm->output;
  o.internal_x = host_x || o.mode != SHK_OUT_FULL;
  if (o.mode == SHK_OUT_ROWS) {
    o.n_rows = prm->n_out_rows;
    if (host_x) o.stage = (size_t)o.n_rows * nf * s_real;
  } else if (o.mode == SHK_OUT_FACTORED) {
    o.kcap = factored_kcap(prm);
    if (host_x) o.stage = (size_t)o.kcap * ((size_t)n + nf) * s_real;
  }
  return o;
}

template <typename R>
static Buffers<R> carve(char* base, const shk_problem* p, int m, int nf, int S, int s_real, const OutPlan& op,
                        bool mg, bool block = false) {
  Carver cv{base};
  const long n = p->n;
  Buffers<R> b{};
  const long N = n * S;
  const int L = nf * S;
  b.V = cv.take<cx<R>>((size_t)(m + 1) * N);
  b.Z = cv.take<c128>((size_t)m * N);
  b.W = cv.take<cx<R>>(N);
  for (int i = 0; i < 2; ++i) {
    b.cr[i] = cv.take<cx<R>>(N);
    b.cw[i] = cv.take<cx<R>>(N);
    b.cs[i] = cv.take<cx<R>>(N);
  }
  b.cp = cv.take<cx<R>>(N);
  b.dinv = cv.take<cx<R>>(n);
  const Grid gp = item_plan(N, S);
  const long ipb = dot_ipb(N);
  const long Gd = (N + ipb - 1) / ipb;
  const long Gu = (N + (long)BS * GSQ - 1) / ((long)BS * GSQ);
  for (int i = 0; i < 2; ++i) {
    b.cpart[i] = cv.take<c128>((size_t)gp.G * 3 * S);
    b.ctot[i] = cv.take<c128>((size_t)3 * S);
  }
  b.part = cv.take<c128>(std::max<size_t>({(size_t)1024 * 2 * S, (size_t)Gd * (m + 1) * S, (size_t)Gu * S}));
  b.sc = cv.take<CgScal>(2 * S);
  b.all_done = cv.take<int>(4);
  b.cfgd = cv.take<CgCfg>(1);
  if (tn().graph) {
    b.gv = cv.take<cx<R>>(N);
    b.gx = cv.take<c128>(N);
  }
  b.beta0 = cv.take<double>(S);
  b.hn = cv.take<double>(S);
  b.mz = cv.take<double>(S);
  b.nzs = cv.take<double>(S);
  b.pn = cv.take<double>((size_t)m * S);
  if (mg) carve_mg(cv, b, p, N, S);
  b.H = cv.take<c128>((size_t)m * (m + 2) * S);
  b.h2 = cv.take<c128>((size_t)(m + 1) * S);
  b.taus = cv.take<c128>(m);
  b.sigma = cv.take<c128>(nf);
  b.zs = cv.take<c128>((size_t)(m + 1) * S);
  b.seed = cv.take<int>(S);
  b.nact = cv.take<int>(S);
  b.qmax = cv.take<double>(S);
  b.ls = cv.take<LaneState>(L);
  b.rc = cv.take<double>((size_t)m * L);
  b.rs = cv.take<c128>((size_t)m * L);
  b.g = cv.take<c128>((size_t)(m + 1) * L);
  b.Rp = cv.take<c128>((size_t)m * (m + 1) / 2 * L);
  b.Yb = cv.take<c128>((size_t)L * m);
  b.Yt = S > 1 ? cv.take<c128>((size_t)L * m) : nullptr;
  b.ascale = cv.take<c128>(L);
  b.extra = cv.take<c128>(L);
  b.bint = cv.take<c128>(N);
  b.rsv = cv.take<c128>(N);
  b.X = op.internal_x ? cv.take<c128>((size_t)n * nf * s_real) : nullptr;
  b.ostage = op.stage ? cv.take<c128>(op.stage) : nullptr;
  b.rows = op.n_rows ? cv.take<long long>((size_t)op.n_rows) : nullptr;
  const int Gr = resid_grid(n);
  b.rpart = cv.take<c128>((size_t)s_real * nf * Gr);
  b.rrow = cv.take<c128>((size_t)s_real * nf);
  if (block) carve_block(cv, b, m, nf, S);
  b.bytes = cv.off;
  return b;
}

// Lanes of a group of n_rhs right-hand sides: the next power of two up to 64;
// the shared block basis takes at least 16 (the matrix-core tile width; the
// extra columns are zero and drop out of the basis).
static int lanes_of(int n_rhs, bool block = false) {
  const int s = std::min(64, next_pow2(std::max(1, n_rhs)));
  return block ? std::max(16, s) : s;
}

static size_t group_bytes(const shk_problem* p, int m, int nf, int S, int s_real, int precision, const OutPlan& op,
                          bool mg, bool block) {
  if (precision == SHK_MIXED) return carve<float>(nullptr, p, m, nf, S, s_real, op, mg, block).bytes;
  return carve<double>(nullptr, p, m, nf, S, s_real, op, mg, block).bytes;
}

// ------------------------------------------------------- lane totals -------
// One block per entry e = q*S + r (sum q, lane r): totals of NV partial sums
// over G blocks -> tot[e] (the layout of a single block's partials, so
// consumers read it with G=1).  The partials of a block are a row of NV*S
// entries; the 8 entries of each 128-byte line of a row go to blocks on one
// XCD (workgroups are dealt out to the XCDs round-robin, id mod 8), so each
// line comes from HBM into one XCD's L2 only: block i works entry
// ((i >> 6) * 8 + (i & 7)) * 8 + ((i >> 3) & 7), the grid rounded up to whole
// groups of 64 blocks (the blocks past the last entry return at once).  Each
// thread issues its first LTK loads together, then sums them in order (a
// strided loop takes blocks beyond LTK*BS), then a fixed-order block sum.
constexpr int LTK = 8;
static int lane_totals_grid(int entries) { return 64 * (((entries + 7) / 8 + 7) / 8); }
template <int NV>
__global__ void __launch_bounds__(BS) k_lane_totals(const c128* __restrict__ part, int G, int S,
                                                    c128* __restrict__ tot) {
  const int i = (int)blockIdx.x;
  const int e = (((i >> 6) * 8 + (i & 7)) * 8) + ((i >> 3) & 7);
  if (e >= NV * S) return;
  const int q = e / S, r = e - q * S;
  const c128* col = part + (size_t)q * S + r;
  const size_t stride = (size_t)NV * S;
  c128 v[LTK];
#pragma unroll
  for (int k = 0; k < LTK; ++k) {
    const int b = (int)threadIdx.x + k * BS;
    v[k] = b < G ? col[(size_t)b * stride] : c128{0.0, 0.0};
  }
  c128 a = v[0];
#pragma unroll
  for (int k = 1; k < LTK; ++k) a = a + v[k];
  for (int b = (int)threadIdx.x + LTK * BS; b < G; b += BS) a = a + col[(size_t)b * stride];
  a = block_sum_all(a);
  if (threadIdx.x == 0) tot[q * S + r] = a;
}

// --------------------------------------------------------------- solver ----
struct PassSpec {
  int m, max_restarts, inner_maxit;
  double tol, eps;
  const std::vector<c128>* taus;
  long long kglob0;   // tau schedule position
  double relax = 0.0, eps_max = 1e-2;   // relaxed inner tolerance (0: off)
  bool fom = false;                     // FOM projected problem and FOM restart
};

struct Snap {
  int all_done;
  int live;   // iteration launches that did work since the solve started
  int pad[2];
  CgScal sc[64];
};

// Pairs whose projected residual is within BLK_CAND x tol of the target get
// their least-squares solution and the eq. trueresidual test each step.
constexpr double BLK_CAND = 10.0;

static void blk_lsq_launch(const BlkLsqArgs& la, int S, int nf, hipStream_t st) {
  const size_t lds_prev = 2 * (size_t)(2 * S) * 16 * sizeof(c128);
  const size_t lds_new = 2 * (size_t)(S + 1) * sizeof(c128) + 2 * sizeof(double) + 2 * (size_t)S * S * sizeof(c128);
  const size_t lds_q = (size_t)S * (S + 1) * sizeof(c128) + S * sizeof(double);
  if (S == 64) k_blk_lsq_prev<64><<<dim3(nf, S / 16), 256, lds_prev, st>>>(la);
  else if (S == 32) k_blk_lsq_prev<32><<<dim3(nf, S / 16), 256, lds_prev, st>>>(la);
  else k_blk_lsq_prev<16><<<dim3(nf, S / 16), 256, lds_prev, st>>>(la);
  if (S == 64) k_blk_lsq_new<4, 1024><<<nf, 1024, lds_new, st>>>(la);
  else if (S == 32) k_blk_lsq_new<2, 1024><<<nf, 1024, lds_new, st>>>(la);
  else k_blk_lsq_new<1, 1024><<<nf, 1024, lds_new, st>>>(la);
  k_blk_lsq_q<<<dim3(nf, 3 * S / 16), 256, lds_q, st>>>(la);
}

static void blk_backsolve_launch(const BlkSolveArgs& sa, int S, int nf, hipStream_t st) {
  if (S == 64) k_blk_backsolve<64><<<dim3(nf, S / 16), 256, 0, st>>>(sa);
  else if (S == 32) k_blk_backsolve<32><<<dim3(nf, S / 16), 256, 0, st>>>(sa);
  else k_blk_backsolve<16><<<dim3(nf, S / 16), 256, 0, st>>>(sa);
}

// Block-basis operations on n x S blocks (block FGMRES-Sh), with the scratch
// they need: chunk partials, coefficients, CholQR factors.
template <typename R> struct BlkCtx {
  long n;
  int S;
  hipStream_t st;
  void* gpart;        // chunk partials (BLK_WAVES S x S complex128)
  cx<R>* Cc;          // projection coefficients, up to (m+1) S x S blocks
  cx<R>* Rinv;        // S x S
  c128 *Gm, *Rrow, *Rinv64;
  double* fro;

  // C = A^H B over nb blocks of A (astride apart) against one block B, summed
  // into Hcol (rows iS.., leading dimension ldh; add != 0 accumulates) and/or
  // rounded into Cc.  TAcc: accumulation of the matrix-core products.
  template <typename TIn, typename TAcc, int TM>
  void project_tm(const cx<TIn>* A, size_t astride, int nb, const cx<TIn>* Bm, c128* Hcol, int ldh, int add,
                  cx<R>* C) const {
    constexpr bool dbl = std::is_same<TAcc, double>::value;
    constexpr int TN = dbl ? 1 : TM, ZG = TM / TN;
    const long ncap = std::max<long>(1, (n + 63) / 64);
    long nch = std::max<long>(1, std::min<long>(ncap, BLK_WAVES / ((long)nb * ZG)));
    long ch = (n + nch - 1) / nch;
    ch = (ch + 3) & ~3L;
    nch = (n + ch - 1) / ch;
    auto* part = reinterpret_cast<cx<TAcc>*>(gpart);
    k_blk_gram<TIn, TAcc, TM, TN><<<dim3((unsigned)nch, (unsigned)nb, ZG), 64, 0, st>>>(A, astride, Bm, n, (int)ch,
                                                                                       part);
    k_blk_reduce<TAcc, R><<<dim3((unsigned)((S * S + BS - 1) / BS), (unsigned)nb), BS, 0, st>>>(part, (int)nch, S,
                                                                                                 Hcol, ldh, add, C);
  }
  template <typename TIn, typename TAcc>
  void project(const cx<TIn>* A, size_t astride, int nb, const cx<TIn>* Bm, c128* Hcol, int ldh, int add,
               cx<R>* C) const {
    if (S == 64) project_tm<TIn, TAcc, 4>(A, astride, nb, Bm, Hcol, ldh, add, C);
    else if (S == 32) project_tm<TIn, TAcc, 2>(A, astride, nb, Bm, Hcol, ldh, add, C);
    else project_tm<TIn, TAcc, 1>(A, astride, nb, Bm, Hcol, ldh, add, C);
  }
  // Out = beta In + sgn sum_i A_i C_i (C row-major S x S blocks)
  template <typename TIn, typename TC, typename TOut, int TM>
  void apply_tm(const cx<TIn>* A, size_t astride, int nb, const cx<TC>* C, const cx<TOut>* In, cx<TOut>* Out,
                double beta, double sgn) const {
    constexpr int TMC = std::is_same<TC, double>::value ? 1 : 2;
    const long cells = 4L * 16 * TMC;
    const size_t lds = (size_t)S * (S + 1) * sizeof(cx<TC>);
    k_blk_update<TIn, TC, TOut, TM, TMC><<<(unsigned)((n + cells - 1) / cells), 256, lds, st>>>(
        A, astride, nb, C, In, Out, n, (TC)beta, (TC)sgn);
  }
  template <typename TIn, typename TC, typename TOut>
  void apply(const cx<TIn>* A, size_t astride, int nb, const cx<TC>* C, const cx<TOut>* In, cx<TOut>* Out,
             double beta, double sgn) const {
    if (S == 64) apply_tm<TIn, TC, TOut, 4>(A, astride, nb, C, In, Out, beta, sgn);
    else if (S == 32) apply_tm<TIn, TC, TOut, 2>(A, astride, nb, C, In, Out, beta, sgn);
    else apply_tm<TIn, TC, TOut, 1>(A, astride, nb, C, In, Out, beta, sgn);
  }
  // Block classical Gram-Schmidt with one reorthogonalisation of W against
  // nb blocks of V: H(0:nb, col) = V^H W, W -= V H, twice (H summed).
  void cgs2(const cx<R>* V, size_t vstride, int nb, cx<R>* W, c128* Hcol, int ldh) const {
    for (int pass = 0; pass < 2; ++pass) {
      project<R, R>(V, vstride, nb, W, Hcol, ldh, pass, Cc);
      apply<R, R, R>(V, vstride, nb, Cc, W, W, 1.0, -1.0);
    }
  }
  // CholQR2 of the block W (n x S, precision TIn) into Vout (precision R):
  // two passes of G = W^H W (FP64 products), G = R^H R, W <- W R^{-1}.  R =
  // R2 R1 goes to Rout (column-major, leading dimension ldh; may be null) and
  // row-major to Rrow_out (may be null); ||R||_F^2 to fro.
  template <typename TIn> void qr(const cx<TIn>* W, cx<R>* Vout, c128* Rout, int ldh, c128* Rrow_out) const {
    const size_t lds = 2 * (size_t)S * S * sizeof(c128);
    cx<TIn>* rinv1 = reinterpret_cast<cx<TIn>*>(std::is_same<TIn, double>::value ? (void*)Rinv64 : (void*)Rinv);
    project<TIn, double>(W, 0, 1, W, Gm, S, 0, nullptr);
    k_blk_chol<TIn><<<1, 256, lds, st>>>(Gm, S, nullptr, nullptr, 0, Rrow, rinv1, nullptr);
    apply<TIn, TIn, R>(W, 0, 1, rinv1, nullptr, Vout, 0.0, 1.0);
    project<R, double>(Vout, 0, 1, Vout, Gm, S, 0, nullptr);
    k_blk_chol<R><<<1, 256, lds, st>>>(Gm, S, Rrow, Rout, ldh, Rrow_out, Rinv, fro);
    apply<R, R, R>(Vout, 0, 1, Rinv, nullptr, Vout, 0.0, 1.0);
  }
};

template <typename R, typename Op, typename OpD> struct Group {
  shk_problem* p;
  Op op;
  OpD opd;
  hipStream_t st;
  Buffers<R> B;
  long n, N;
  int S, s_real, nf, m, L;
  Grid gp;
  long long inner_its = 0;
  int outer_steps = 0;

  template <int CGB, bool NT, bool ONE, bool MULTI>
  void step_k(int G, c128 tau, int ni, int lS, const CgCfg& e, const c128* in, int Gin, const CgScal* scIn,
              CgScal* scOut, const CgVecs<R>& vec, int par, c128* out) {
    k_cg_step<Op, OpD, R, CGB, NT, ONE, MULTI><<<G, CGB, 0, st>>>(op, opd, B.dinv, tau, ni, lS, B.cfgd, cur_v, in, Gin,
                                                                  scIn, scOut, vec, par, out, B.all_done);
  }
  template <int CGB, bool NT>
  void step_nt(int G, c128 tau, int ni, int lS, const CgCfg& e, const c128* in, int Gin, const CgScal* scIn,
               CgScal* scOut, const CgVecs<R>& vec, int par, c128* out) {
    const bool multi = (long)G * CGB < N;
    if (lS == 0) {
      if (multi) step_k<CGB, NT, true, true>(G, tau, ni, lS, e, in, Gin, scIn, scOut, vec, par, out);
      else step_k<CGB, NT, true, false>(G, tau, ni, lS, e, in, Gin, scIn, scOut, vec, par, out);
    } else {
      if (multi) step_k<CGB, NT, false, true>(G, tau, ni, lS, e, in, Gin, scIn, scOut, vec, par, out);
      else step_k<CGB, NT, false, false>(G, tau, ni, lS, e, in, Gin, scIn, scOut, vec, par, out);
    }
  }
  template <int CGB>
  void step_cgb(int G, c128 tau, int ni, int lS, const CgCfg& e, const c128* in, int Gin, const CgScal* scIn,
                CgScal* scOut, const CgVecs<R>& vec, int par, c128* out) {
    if (std::is_same<R, float>::value ? tn().nt32 : tn().nt64)
      step_nt<CGB, true>(G, tau, ni, lS, e, in, Gin, scIn, scOut, vec, par, out);
    else
      step_nt<CGB, false>(G, tau, ni, lS, e, in, Gin, scIn, scOut, vec, par, out);
  }
  void launch_step(int G, c128 tau, int ni, int lS, const CgCfg& e, const c128* in, int Gin, const CgScal* scIn,
                   CgScal* scOut, const CgVecs<R>& vec, int par, c128* out) {
    if (tn().cgb == 512) step_cgb<512>(G, tau, ni, lS, e, in, Gin, scIn, scOut, vec, par, out);
    else step_cgb<256>(G, tau, ni, lS, e, in, Gin, scIn, scOut, vec, par, out);
  }

  // ---- multigrid V-cycle (inner preconditioner) ----
  bool mg = false;                // COCG preconditioned by the V-cycle
  double mg_omega = 0.8;
  MgTail mg_ta{};                 // tail arguments for the current inner solve
  const CgScal* vsc = nullptr;    // lane states the V-cycle's launches read (the step's output)
  // working launches of the last inner solve per tau (a handful of taus)
  std::vector<std::pair<c128, int>> mg_hist;
  int mg_hist_get(c128 tau) const {
    for (const auto& h : mg_hist)
      if (h.first.re == tau.re && h.first.im == tau.im) return h.second;
    return 0;
  }
  void mg_hist_put(c128 tau, int launches) {
    for (auto& h : mg_hist)
      if (h.first.re == tau.re && h.first.im == tau.im) {
        h.second = launches;
        return;
      }
    if (mg_hist.size() < 16) mg_hist.emplace_back(tau, launches);
  }
  int mg_lds = 0;                 // and its LDS bytes
  int mg_levels() const { return 1 + (int)p->mg.size(); }
  LevelDims mg_dims(int l) const {
    if (l == 0) return {p->nx, p->ny, p->nz};
    const MgLevel& L = p->mg[l - 1];
    return {L.nx, L.ny, L.nz};
  }
  // operator of level l in precision F (level 0: the problem's own)
  template <typename O, typename F> O mg_op(const O& base, int l) const {
    if (l == 0) return base;
    O o = base;
    if constexpr (O::NB > 0) {
      const MgLevel& L = p->mg[l - 1];
      auto faces = [&](int a) -> const F* {
        if constexpr (std::is_same<F, float>::value) return L.t32[a];
        else return L.t[a];
      };
      o.nx = L.nx; o.ny = L.ny; o.tx = faces(0); o.ty = faces(1);
      if constexpr (O::NB == 6) { o.nz = L.nz; o.tz = faces(2); }
      o.mdiag = L.mass; o.m0 = 0.0;
    }
    return o;
  }
  // inverse diagonals of the coarse levels for this tau
  void mg_prepare(c128 tau) {
    if constexpr (Op::NB > 0) {
      // D^-1 of every coarse level, MG_DINV_TAB levels per launch
      const int Lv = mg_levels();
      for (int l0 = 1; l0 < Lv; l0 += MG_DINV_TAB) {
        MgDinvTab<OpD, R> tab{};
        tab.nl = std::min(MG_DINV_TAB, Lv - l0);
        long tot = 0;
        for (int q = 0; q < tab.nl; ++q) {
          tab.start[q] = tot;
          tab.op[q] = mg_op<OpD, double>(opd, l0 + q);
          tab.out[q] = B.mdinv[l0 + q - 1];
          tot += mg_dims(l0 + q).n();
        }
        tab.start[tab.nl] = tot;
        k_mg_dinv_levels<OpD, R><<<grid_items(tot, 2048), BS, 0, st>>>(tab, tau);
      }
      const int t = mg_tail_level(ilog2(S));
      if (t < mg_levels()) {
        MgPack pk;
        mg_tail_layout(t, tail_lg(ilog2(S)), mg_ta, pk, mg_lds);
        k_mg_pack<<<pk.nseg, BS, 0, st>>>(pk, B.mpack);
      }
    }
  }
  // Face array lengths of level l along each axis.
  void mg_face_lens(int l, long (&len)[3]) const {
    const LevelDims d = mg_dims(l);
    len[0] = (long)(d.nx + 1) * d.ny * d.nz;
    len[1] = (long)d.nx * (d.ny + 1) * d.nz;
    len[2] = Op::NB == 6 ? (long)d.nx * d.ny * (d.nz + 1) : 0;
  }
  // LDS bytes of the tail started at level l: b and x of every level, and
  // the packed D^-1, masses and faces (each array on a 16-byte boundary).
  size_t mg_tail_bytes(int l, int lS) const {
    size_t vec = 0, pack = 0;
    for (int k = l; k < mg_levels(); ++k) {
      const size_t nk = (size_t)mg_dims(k).n();
      long len[3];
      mg_face_lens(k, len);
      vec += 2 * (nk << lS) * sizeof(cx<R>);
      pack += align16(nk * sizeof(cx<R>)) + align16(nk * sizeof(double));
      for (int a = 0; a < 3; ++a) pack += align16((size_t)len[a] * sizeof(R));
    }
    return align16(vec) + pack;
  }
  static size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }
  // log2 of the lanes one tail workgroup takes, for 2^lS lanes in all.
  static int tail_lg(int lS) {
    const int tl = tn().tail_lanes;
    return tl > 0 ? std::min(lS, ilog2(tl)) : lS;
  }
  // First level of the tail: the finest level from which all coarser levels
  // of one tail workgroup's lanes fit in its LDS.
  int mg_tail_level(int lS) const {
    const int Lv = mg_levels(), lg = tail_lg(lS);
    int t = Lv;
    for (int l = Lv - 1; l >= 0; --l) {
      if (mg_tail_bytes(l, lg) > (size_t)tn().tail_lds || Lv - l > MG_MAXL) break;
      t = l;
    }
    return t;   // Lv: not even the one-cell level fits (many lanes)
  }
  // Tail arguments and the segments of its packed block (offsets relative
  // to the pack for the segments, absolute LDS offsets in the arguments).
  void mg_tail_layout(int t, int lS, MgTail& a, MgPack& pk, int& lds_bytes) const {
    const int Lv = mg_levels();
    a = MgTail{};
    pk = MgPack{};
    a.T = Lv - t;
    size_t vec = 0;
    for (int k = 0; k < a.T; ++k) {
      const LevelDims d = mg_dims(t + k);
      a.lv[k].nx = d.nx;
      a.lv[k].ny = d.ny;
      a.lv[k].nz = d.nz;
      a.lv[k].lpx = ceil_log2(d.nx);
      a.lv[k].lpy = ceil_log2(d.ny);
      a.lv[k].off = (int)(vec / sizeof(cx<R>));
      vec += 2 * ((size_t)d.n() << lS) * sizeof(cx<R>);
    }
    a.pack_lds = (int)align16(vec);
    size_t off = 0;
    auto seg = [&](const void* src, size_t bytes, double fill) {
      MgSeg& sg = pk.seg[pk.nseg++];
      sg.src = src;
      sg.dst = (int)off;
      sg.words = (int)(bytes / 4);
      sg.fill = fill;
      const int at = a.pack_lds + (int)off;
      off += align16(bytes);
      return at;
    };
    for (int k = 0; k < a.T; ++k) {
      const int l = t + k;
      const size_t nk = (size_t)mg_dims(l).n();
      const Op o = mg_op<Op, R>(op, l);
      a.lv[k].doff = seg(l == 0 ? (const void*)B.dinv : (const void*)B.mdinv[l - 1], nk * sizeof(cx<R>), 0.0);
      a.lv[k].moff = seg(o.mdiag, nk * sizeof(double), o.m0);
      long len[3];
      mg_face_lens(l, len);
      a.lv[k].foff[0] = seg(o.tx, (size_t)len[0] * sizeof(R), 0.0);
      a.lv[k].foff[1] = seg(o.ty, (size_t)len[1] * sizeof(R), 0.0);
      if constexpr (Op::NB == 6) a.lv[k].foff[2] = seg(o.tz, (size_t)len[2] * sizeof(R), 0.0);
    }
    a.pack_words = (int)(off / 4);
    lds_bytes = a.pack_lds + (int)off;
  }
  // uout = B b0 (one V-cycle over every level)
  // (from = 1: the finest restriction was done by the fused step kernel)
  // Grid legs for several lanes: chunks of up to 4 lanes per thread on the
  // complex64 path and of 2 on the complex128 path (each measured faster
  // than the other sizes and than a lane per thread).
  static constexpr bool c64 = std::is_same<R, float>::value;
  bool lane_chunks() const { return c64 || tn().lt64 >= 2; }
  // row-marching 2-D legs (several lanes, levels of at least `rows` cells)
  bool rows_for(const LevelDims& f, int lNC) const {
    const long th = c64 ? tn().rows : tn().rows64;
    return Op::NB == 4 && th > 0 && (long)f.n() >= th && lNC <= 5;
  }
  template <bool UP, int LT>
  void leg_rows(int l, const LevelDims& f, const LevelDims& c, c128 tau, int lS, int lNC, const cx<R>* bl,
                const cx<R>* dl, const cx<R>* xcoarse, cx<R>* out) {
    if constexpr (Op::NB == 4 && LT * sizeof(cx<R>) <= 32) {
      const int SW = BS >> lNC, YB = tn().rows_yb;
      const long G = (long)((f.nx + SW - 1) / SW) * ((f.ny + YB - 1) / YB);
      k_mg_leg_rows<Op, R, LT, UP><<<(unsigned)G, BS, 0, st>>>(mg_op<Op, R>(op, l), f, c, tau, mg_omega, lS, lNC, YB,
                                                               bl, dl, xcoarse, out, vsc, B.all_done);
    }
  }
  template <int LT>
  void mg_down_lt(int l, const LevelDims& f, const LevelDims& c, c128 tau, int lS, const cx<R>* bl, const cx<R>* dl,
                  cx<R>* out) {
    const int lNC = lS - ilog2(LT);
    if (LT * sizeof(cx<R>) <= 32 && rows_for(f, lNC)) {
      leg_rows<false, LT>(l, f, c, tau, lS, lNC, bl, dl, nullptr, out);
      return;
    }
    const dim3 g((unsigned)((((long)c.nx << (lNC + Op::NB / 2)) + BS - 1) / BS), (unsigned)c.ny, (unsigned)c.nz);
    k_mg_down_lanes<Op, R, LT><<<g, BS, 0, st>>>(mg_op<Op, R>(op, l), f, c, tau, mg_omega, lS, lNC, bl, dl, out,
                                                 vsc, B.all_done);
  }
  void mg_down_lanes(int l, const LevelDims& f, const LevelDims& c, c128 tau, int lS, const cx<R>* bl,
                     const cx<R>* dl, cx<R>* out) {
    const int lt = std::min(c64 ? tn().down_lt : tn().lt64, 1 << lS);
    if (lt == 2) mg_down_lt<2>(l, f, c, tau, lS, bl, dl, out);
    else if (lt == 4) mg_down_lt<4>(l, f, c, tau, lS, bl, dl, out);
    else mg_down_lt<8>(l, f, c, tau, lS, bl, dl, out);
  }
  template <int LT>
  void mg_up_lt(int l, const LevelDims& f, const LevelDims& c, c128 tau, int lS, const cx<R>* bl, const cx<R>* dl,
                const cx<R>* xcoarse, cx<R>* out) {
    const int lNC = lS - ilog2(LT);
    if (LT * sizeof(cx<R>) <= 32 && rows_for(f, lNC)) {
      leg_rows<true, LT>(l, f, c, tau, lS, lNC, bl, dl, xcoarse, out);
      return;
    }
    const dim3 g((unsigned)((((long)f.nx << lNC) + BS - 1) / BS), (unsigned)f.ny, (unsigned)f.nz);
    k_mg_up_lanes<Op, R, LT><<<g, BS, 0, st>>>(mg_op<Op, R>(op, l), f, c, tau, mg_omega, lS, lNC, bl, dl, xcoarse,
                                               out, vsc, B.all_done);
  }
  void mg_up_lanes(int l, const LevelDims& f, const LevelDims& c, c128 tau, int lS, const cx<R>* bl,
                   const cx<R>* dl, const cx<R>* xcoarse, cx<R>* out) {
    const int lt = std::min(c64 ? tn().up_lt : tn().lt64, 1 << lS);
    if (lt == 2) mg_up_lt<2>(l, f, c, tau, lS, bl, dl, xcoarse, out);
    else if (lt == 4) mg_up_lt<4>(l, f, c, tau, lS, bl, dl, xcoarse, out);
    else mg_up_lt<8>(l, f, c, tau, lS, bl, dl, xcoarse, out);
  }
  // plane-marching 3-D legs: a chunk of tile3_lt (complex64) or 2 (complex128)
  // lanes per block
  bool tile3_for(const LevelDims& f) const {
    return Op::NB == 6 && tn().tile3 > 0 && (long)f.n() >= tn().tile3;
  }
  template <bool UP, int LT>
  void leg_tile3_lt(const LevelDims& f, const LevelDims& c, const Op& o, c128 tau, int lS, const cx<R>* bl,
                    const cx<R>* dl, const cx<R>* xcoarse, cx<R>* out) {
    if constexpr (Op::NB == 6) {
      const int C = (1 << lS) / LT, ZB = tn().tile3_zb;
      const dim3 g((unsigned)(((f.nx + T3X - 1) / T3X) * C), (unsigned)((f.ny + T3Y - 1) / T3Y),
                   (unsigned)((f.nz + ZB - 1) / ZB));
      k_mg_leg_tile3<Op, R, LT, UP><<<g, T3T, 0, st>>>(o, f, c, tau, mg_omega, lS, C, ZB, bl, dl, xcoarse, out,
                                                        vsc, B.all_done);
    }
  }
  template <bool UP>
  void leg_tile3(int l, const LevelDims& f, const LevelDims& c, c128 tau, int lS, const cx<R>* bl, const cx<R>* dl,
                 const cx<R>* xcoarse, cx<R>* out) {
    const Op o = mg_op<Op, R>(op, l);
    const int lt = std::min(1 << lS, c64 ? tn().tile3_lt : 2);
    if (lt == 1) leg_tile3_lt<UP, 1>(f, c, o, tau, lS, bl, dl, xcoarse, out);
    else if (lt == 2) leg_tile3_lt<UP, 2>(f, c, o, tau, lS, bl, dl, xcoarse, out);
    else if (lt == 4) leg_tile3_lt<UP, 4>(f, c, o, tau, lS, bl, dl, xcoarse, out);
    else if constexpr (c64) leg_tile3_lt<UP, 8>(f, c, o, tau, lS, bl, dl, xcoarse, out);
  }
  // chains of middle legs (2-D, one lane)
  bool chain_ok(int lS) const { return Op::NB == 4 && lS == 0 && tn().mg_chain > 0; }
  const cx<R>* lvl_dinv(int l) const { return l == 0 ? B.dinv : B.mdinv[l - 1]; }
  MgChain<Op, R> chain_args(int a, int nl) const {
    MgChain<Op, R> c{};
    c.nl = nl;
    for (int k = 0; k <= nl; ++k) {
      c.d[k] = mg_dims(a + k);
      c.dinv[k] = lvl_dinv(a + k);
    }
    for (int k = 0; k < nl; ++k) c.op[k] = mg_op<Op, R>(op, a + k);
    return c;
  }
  // restrictions a -> a + nl: right-hand side of level a in, of levels a+1..a+nl out
  void down_chain(int a, int nl, c128 tau, const cx<R>* bin) {
    if constexpr (Op::NB == 4) {
      MgChain<Op, R> c = chain_args(a, nl);
      c.b[0] = bin;
      for (int k = 1; k <= nl; ++k) c.out[k] = B.mb[a + k - 1];
      const LevelDims d = c.d[nl];
      const dim3 g((unsigned)((d.nx + 1) / 2), (unsigned)((d.ny + 1) / 2));
      k_mg_down_chain2d<Op, R, 2><<<g, BS, 0, st>>>(c, tau, mg_omega, B.all_done);
    }
  }
  // prolongations a + nl -> a: x of level a + nl in, x of level a out
  void up_chain(int a, int nl, c128 tau, const cx<R>* b0, const cx<R>* xcoarse, cx<R>* xout) {
    if constexpr (Op::NB == 4) {
      MgChain<Op, R> c = chain_args(a, nl);
      for (int k = 0; k < nl; ++k) c.b[k] = a + k == 0 ? b0 : B.mb[a + k - 1];
      c.xc = xcoarse;
      c.out[0] = xout;
      const LevelDims d = c.d[0];
      const dim3 g((unsigned)((d.nx + 15) / 16), (unsigned)((d.ny + 15) / 16));
      k_mg_up_chain2d<Op, R, 16><<<g, BS, 0, st>>>(c, tau, mg_omega, B.all_done);
    }
  }
  void mg_vcycle(const cx<R>* b0, c128 tau, int lS, cx<R>* uout, int from = 0) {
    if constexpr (Op::NB > 0) {
      const int Lv = mg_levels();
      const int S_ = 1 << lS;
      const int t = mg_tail_level(lS);
      const int gdown = std::min(t, Lv - 1);   // levels whose down leg runs on the grid
      const cx<R>* bl = from > 0 ? B.mb[from - 1] : b0;
      // the last legs above the tail as one chain
      const int dchain = chain_ok(lS) && gdown - from >= 2 ? std::min(MGC_F, gdown - from) : 0;
      for (int l = from; l < gdown - dchain; ++l) {
        const LevelDims f = mg_dims(l), c = mg_dims(l + 1);
        const cx<R>* dl = l == 0 ? B.dinv : B.mdinv[l - 1];
        if (tile3_for(f)) {
          leg_tile3<false>(l, f, c, tau, lS, bl, dl, nullptr, B.mb[l]);
        } else if (lS > 0 && lane_chunks()) {
          mg_down_lanes(l, f, c, tau, lS, bl, dl, B.mb[l]);
        } else {
          const dim3 g((unsigned)((((long)c.nx * S_ << (Op::NB / 2)) + BS - 1) / BS), (unsigned)c.ny, (unsigned)c.nz);
          k_mg_down<Op, R><<<g, BS, 0, st>>>(mg_op<Op, R>(op, l), f, c, tau, mg_omega, lS, bl, dl, B.mb[l],
                                              B.all_done);
        }
        bl = B.mb[l];
      }
      if (dchain > 0) {
        down_chain(gdown - dchain, dchain, tau, bl);
        bl = B.mb[gdown - 1];
      }
      if (t < Lv) {
        cx<R>* xt = t == 0 ? uout : B.mx[t - 1];   // mg_ta, mg_lds: laid out by mg_prepare
        const int lg = tail_lg(lS);
        const unsigned gt = 1u << (lS - lg);
        if (mg_lds > MG_TAIL_LDS)
          k_mg_tail<Op, R, MG_TAIL_LDS_MAX><<<gt, MG_TAIL_THREADS, (size_t)mg_lds, st>>>(
              mg_ta, tau, mg_omega, lg, lS, B.mpack, bl, xt, vsc, B.all_done);
        else
          k_mg_tail<Op, R, MG_TAIL_LDS><<<gt, MG_TAIL_THREADS, (size_t)mg_lds, st>>>(mg_ta, tau, mg_omega, lg, lS,
                                                                                   B.mpack, bl, xt, vsc, B.all_done);
      } else {
        // the coarsest level alone exceeds the tail: solve it on the grid
        const int l = Lv - 1;
        k_mg_scale_grid<R><<<grid_items((long)S_, 8192), BS, 0, st>>>((long)mg_dims(l).n() << lS, lS,
                                                                       B.mdinv[l - 1], bl, B.mx[l - 1], B.all_done);
      }
      int ltop = std::min(t, Lv - 1) - 1;
      // the first legs below the tail (not the finest) as one chain
      if (chain_ok(lS) && ltop >= 2) {
        const int nl = std::min(MGC_F, ltop);
        const int a = ltop - nl + 1;
        up_chain(a, nl, tau, b0, B.mx[a + nl - 1], a == 0 ? uout : B.mx[a - 1]);
        ltop = a - 1;
      }
      for (int l = ltop; l >= 0; --l) {
        const LevelDims f = mg_dims(l), c = mg_dims(l + 1);
        const cx<R>* bl2 = l == 0 ? b0 : B.mb[l - 1];
        const cx<R>* dl = l == 0 ? B.dinv : B.mdinv[l - 1];
        cx<R>* out = l == 0 ? uout : B.mx[l - 1];
        if (tile3_for(f)) {
          leg_tile3<true>(l, f, c, tau, lS, bl2, dl, B.mx[l], out);
        } else if (lS > 0 && lane_chunks()) {
          mg_up_lanes(l, f, c, tau, lS, bl2, dl, B.mx[l], out);
        } else {
          const dim3 g((unsigned)(((long)f.nx * S_ + BS - 1) / BS), (unsigned)f.ny, (unsigned)f.nz);
          k_mg_up<Op, R><<<g, BS, 0, st>>>(mg_op<Op, R>(op, l), f, c, tau, mg_omega, lS, bl2, dl, B.mx[l], out,
                                            B.all_done);
        }
      }
    }
  }
  // The product on the plane-marching tiles (3-D, several lanes, separate fold
  // of the partials); Gpost = the partial rows it writes.
  int Gpost = 0;
  bool post_tile3(c128 tau, int lS, const CgScal* sc, const cx<R>* r, cx<R>* w, c128* out) {
    if constexpr (Op::NB == 6) {
      const LevelDims f = mg_dims(0);
      if (!tn().tile3_post || !tile3_for(f) || !gp.separate || lS == 0) return false;
      const int lt = std::min(1 << lS, c64 ? tn().post3_lt : 2);
      const int C = (1 << lS) / lt, ZB = tn().tile3_zb;
      const int gx = (f.nx + T3X - 1) / T3X, gy = (f.ny + T3Y - 1) / T3Y, gz = (f.nz + ZB - 1) / ZB;
      if ((long)gx * gy * gz > gp.G) return false;   // the partial rows must fit
      Gpost = gx * gy * gz;
      const dim3 g((unsigned)(gx * C), (unsigned)gy, (unsigned)gz);
      if (lt == 2)
        k_cgmg_post_tile3<Op, R, 2><<<g, T3T, 0, st>>>(op, f, tau, lS, C, ZB, sc, r, B.u, w, out, B.all_done);
      else if (lt == 4)
        k_cgmg_post_tile3<Op, R, 4><<<g, T3T, 0, st>>>(op, f, tau, lS, C, ZB, sc, r, B.u, w, out, B.all_done);
      return true;
    }
    return false;
  }
  // w = A u and the forms with r, on the iteration kernels' grid
  // Several lanes: a thread per cell and chunk of lanes.
  template <int CGB>
  bool mg_post_lanes(int G, c128 tau, int ni, int lS, const CgScal* sc, const cx<R>* r, cx<R>* w, c128* out) {
    if constexpr (Op::NB > 0) {
      const int lt = std::min(c64 ? tn().post_lt : std::min(tn().lt64, 2), 1 << lS);
      if (lS == 0 || lt < 2) return false;
      if (lt == 2) {
        k_cgmg_post_lanes<Op, R, CGB, 2><<<G, CGB, 0, st>>>(op, tau, ni, lS, sc, r, B.u, w, out, B.all_done);
      } else if constexpr (c64) {
        if (lt == 4) k_cgmg_post_lanes<Op, R, CGB, 4><<<G, CGB, 0, st>>>(op, tau, ni, lS, sc, r, B.u, w, out, B.all_done);
        else k_cgmg_post_lanes<Op, R, CGB, 8><<<G, CGB, 0, st>>>(op, tau, ni, lS, sc, r, B.u, w, out, B.all_done);
      }
      return true;
    }
    return false;
  }
  template <int CGB>
  void mg_post_cgb(int G, c128 tau, int ni, int lS, const CgScal* sc, const cx<R>* r, cx<R>* w, c128* out) {
    if constexpr (Op::NB > 0) {
      const bool multi = (long)G * CGB < N;
      if (mg_post_lanes<CGB>(G, tau, ni, lS, sc, r, w, out)) return;
      if (lS == 0) {
        if (multi) k_cgmg_post<Op, R, CGB, true, true><<<G, CGB, 0, st>>>(op, tau, ni, lS, sc, r, B.u, w, out, B.all_done);
        else k_cgmg_post<Op, R, CGB, true, false><<<G, CGB, 0, st>>>(op, tau, ni, lS, sc, r, B.u, w, out, B.all_done);
      } else {
        if (multi) k_cgmg_post<Op, R, CGB, false, true><<<G, CGB, 0, st>>>(op, tau, ni, lS, sc, r, B.u, w, out, B.all_done);
        else k_cgmg_post<Op, R, CGB, false, false><<<G, CGB, 0, st>>>(op, tau, ni, lS, sc, r, B.u, w, out, B.all_done);
      }
    }
  }
  void mg_post(int G, c128 tau, int ni, int lS, const CgScal* sc, const cx<R>* r, cx<R>* w, c128* out) {
    if (post_tile3(tau, lS, sc, r, w, out)) return;
    if (tn().cgb == 512) mg_post_cgb<512>(G, tau, ni, lS, sc, r, w, out);
    else mg_post_cgb<256>(G, tau, ni, lS, sc, r, w, out);
  }
  // The step fused with the finest restriction: one lane, the default block
  // size, the finest down leg on the grid, and few enough blocks that each
  // summing every partial stays cheap.
  bool mg_fused(int lS) const {
    if (Op::NB == 0 || lS != 0 || tn().cgb != BS || !tn().mg_fuse) return false;
    if (mg_levels() < 2 || mg_tail_level(lS) < 1) return false;
    const LevelDims c = mg_dims(1);
    const long blocks = ((long)c.nx * (1 << (Op::NB / 2)) + BS - 1) / BS * c.ny * c.nz;
    return blocks <= 2048;
  }
  template <int CGB, bool ONE, bool MULTI>
  void mg_iter_k(int G, c128 tau, int ni, int lS, const CgCfg& cfg, const c128* in, int Gin, const CgScal* scIn,
                 CgScal* scOut, const CgVecs<R>& vec, int par, c128* out) {
    if constexpr (Op::NB > 0) {
      if (mg_fused(lS)) {
        const LevelDims f = mg_dims(0), c = mg_dims(1);
        const dim3 g((unsigned)(((long)c.nx * (1 << (Op::NB / 2)) + BS - 1) / BS), (unsigned)c.ny, (unsigned)c.nz);
        k_cgmg_step_down<Op, OpD, R><<<g, BS, 0, st>>>(op, opd, f, c, tau, mg_omega, B.cfgd, cur_v, B.u, in, Gin, scIn,
                                                       scOut, vec, par, B.dinv, B.mb[0], B.all_done);
        vsc = scOut;
        mg_vcycle(vec.r[par ^ 1], tau, lS, B.u, 1);
      } else {
        k_cgmg_step<Op, OpD, R, CGB, ONE, MULTI><<<G, CGB, 0, st>>>(opd, tau, ni, lS, B.cfgd, cur_v, B.u, in, Gin, scIn,
                                                                    scOut, vec, par, B.all_done);
        vsc = scOut;
        mg_vcycle(vec.r[par ^ 1], tau, lS, B.u);
      }
      if (!post_tile3(tau, lS, scOut, vec.r[par ^ 1], vec.w[par ^ 1], out) &&
          !mg_post_lanes<CGB>(G, tau, ni, lS, scOut, vec.r[par ^ 1], vec.w[par ^ 1], out))
        k_cgmg_post<Op, R, CGB, ONE, MULTI><<<G, CGB, 0, st>>>(op, tau, ni, lS, scOut, vec.r[par ^ 1], B.u,
                                                               vec.w[par ^ 1], out, B.all_done);
    }
  }
  template <int CGB>
  void mg_iter_cgb(int G, c128 tau, int ni, int lS, const CgCfg& cfg, const c128* in, int Gin, const CgScal* scIn,
                   CgScal* scOut, const CgVecs<R>& vec, int par, c128* out) {
    const bool multi = (long)G * CGB < N;
    if (lS == 0) {
      if (multi) mg_iter_k<CGB, true, true>(G, tau, ni, lS, cfg, in, Gin, scIn, scOut, vec, par, out);
      else mg_iter_k<CGB, true, false>(G, tau, ni, lS, cfg, in, Gin, scIn, scOut, vec, par, out);
    } else {
      if (multi) mg_iter_k<CGB, false, true>(G, tau, ni, lS, cfg, in, Gin, scIn, scOut, vec, par, out);
      else mg_iter_k<CGB, false, false>(G, tau, ni, lS, cfg, in, Gin, scIn, scOut, vec, par, out);
    }
  }
  // one multigrid-COCG iteration: vector updates, V-cycle, operator product
  void mg_iteration(int G, c128 tau, int ni, int lS, const CgCfg& cfg, const c128* in, int Gin,
                    const CgScal* scIn, CgScal* scOut, const CgVecs<R>& vec, int par, c128* out) {
    if (tn().cgb == 512) mg_iter_cgb<512>(G, tau, ni, lS, cfg, in, Gin, scIn, scOut, vec, par, out);
    else mg_iter_cgb<256>(G, tau, ni, lS, cfg, in, Gin, scIn, scOut, vec, par, out);
  }

  // ---- inner solve of (K + tau M) z = v (section 4) into z, w = M z ----
  const cx<R>* cur_v = nullptr;   // right-hand side of the running inner solve
  GraphSet graphs;                // captured iterations, per tau
  int inner(c128 tau, const cx<R>* v, c128* z, double eps, int maxit, int fixed, double* pn_out) {
    const int G = gp.G;
    const bool rounds = std::is_same<R, float>::value && fixed <= 0;
    const double e = fixed > 0 ? -1.0 : eps;
    const int cap = fixed > 0 ? fixed : maxit;
    const int lS = ilog2(S);
    const int ni = (int)n;
    // captured iterations: not while the per-iteration timer runs, and not
    // on the legacy default stream (it cannot be captured)
    const bool timing = g_timer.on;
    const bool use_graph = tn().graph && B.gx && !timing && st != nullptr;
    cur_v = v;
    CgVecs<R> vec{{B.cr[0], B.cr[1]}, {B.cw[0], B.cw[1]}, {B.cs[0], B.cs[1]}, B.cp, z};
    if (use_graph) {
      SHK_HIP(hipMemcpyAsync(B.gv, v, (size_t)N * sizeof(cx<R>), hipMemcpyDeviceToDevice, st));
      cur_v = B.gv;
      vec.x = B.gx;
    }
    k_dinv<OpD, R><<<grid_items(n, 2048), BS, 0, st>>>(opd, p->dK, tau, ni, B.dinv);
    // partials of launch L live in cpart[L & 1] (totals in ctot[L & 1])
    auto totals = [&](int slot) -> const c128* {
      if (!gp.separate) return B.cpart[slot];
      k_lane_totals<3><<<lane_totals_grid(3 * S), BS, 0, st>>>(B.cpart[slot], Gpost > 0 ? Gpost : G, S,
                                                              B.ctot[slot]);
      return B.ctot[slot];
    };
    const int Gin = gp.separate ? 1 : G;
    CgCfg cfg{};
    cfg.eps = fixed > 0 ? -1.0 : eps;
    cfg.maxit = cap;
    cfg.trust = rounds ? 0 : 1;
    const double rtol = mg ? tn().round_tol_mg : tn().round_tol;
    cfg.round_tol = rounds ? rtol : 0.0;
    cfg.stall_min = tn().stall_min;
    cfg.stall_mult = tn().stall_mult;
    cfg.fused_start = mg ? 1 : 0;
    k_set_cfg<<<1, 64, 0, st>>>(B.cfgd, cfg);
    k_cg_init<Op, R><<<G, BS, 0, st>>>(op, B.dinv, tau, ni, lS, cur_v, vec, B.cpart[0], B.sc, B.all_done);
    if (mg) {
      if constexpr (Op::NB > 0) {
        // the first round's u = B v, w = A u and forms
        mg_prepare(tau);
        vsc = B.sc;   // the states k_cg_init wrote: every lane running
        mg_vcycle(vec.r[0], tau, lS, B.u);
        mg_post(G, tau, ni, lS, B.sc, vec.r[0], vec.w[0], B.cpart[0]);
      }
    }
    const c128* in = totals(0);
    SHK_HIP(hipGetLastError());
    long it = 0;
    int chunk = std::min(cap + 1, 16);
    // Multigrid: an idle iteration (launched past the end of the solve) costs
    // about half a working one, so the first chunk is the working launch
    // count of the last inner solve with this tau, when there was one (the
    // shifts repeat cyclically and so do the counts, give or take a few),
    // plus the launch that finds every lane done.
    const int hist = mg && fixed <= 0 ? mg_hist_get(tau) : 0;
    if (hist > 0) chunk = std::min(cap + 1, hist + 1);
    static_assert(sizeof(Snap) <= 32768, "staging layout");
    Snap* snap = (Snap*)g_pinned.get(65536);
    if (!snap) return fail(SHK_ERR_OOM, "pinned staging");
    // Timer (profiling only).  At each poll the launches that did work are
    // the chunk's first `live` ones.  Multigrid: an event after every
    // iteration (its step, V-cycle and product launches), and the time from
    // the end of the chunk's first to the end of its last working iteration.
    // Jacobi (one short kernel per iteration, where an event each would
    // slow the loop): events around the chunk, counted when every launch of
    // it worked.  Either way kernel time plus the back-to-back gaps.
    int live_before = 0;
    // per lane: iteration count and residual norm seen at the previous poll
    std::vector<int> prev_its(S, 0);
    std::vector<double> prev_rn(S, 0.0);
    const double lrt = std::log(std::max(rtol, 1e-12));
    while (true) {
      if (timing) {
        g_timer.ensure((size_t)chunk / 2 + 1);
        if (!mg) (void)hipEventRecord(g_timer.ev[0], st);
      }
      if (use_graph) {
        // pairs of iterations from the captured graph (it stays even)
        chunk += chunk & 1;
        hipGraphExec_t ex = graphs.find(tau);
        if (!ex) {
          hipGraph_t gr = nullptr;
          SHK_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
          const c128* in2 = in;
          for (int par = 0; par < 2; ++par) {
            const CgScal* scIn = B.sc + (size_t)par * S;
            CgScal* scOut = B.sc + (size_t)(par ^ 1) * S;
            if (mg) mg_iteration(G, tau, ni, lS, cfg, in2, Gin, scIn, scOut, vec, par, B.cpart[par ^ 1]);
            else launch_step(G, tau, ni, lS, cfg, in2, Gin, scIn, scOut, vec, par, B.cpart[par ^ 1]);
            in2 = totals(par ^ 1);
          }
          const hipError_t ce = hipStreamEndCapture(st, &gr);
          if (ce != hipSuccess) return fail(SHK_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
          const hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
          (void)hipGraphDestroy(gr);
          if (ie != hipSuccess) return fail(SHK_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
          graphs.st = st;
          graphs.execs.emplace_back(tau, ex);
        }
        for (int c = 0; c < chunk; c += 2) SHK_HIP(hipGraphLaunch(ex, st));
        it += chunk;
      } else {
        for (int c = 0; c < chunk; ++c, ++it) {
          const CgScal* scIn = B.sc + (size_t)(it & 1) * S;
          CgScal* scOut = B.sc + (size_t)((it + 1) & 1) * S;
          const int out = (int)((it + 1) & 1);
          if (mg) mg_iteration(G, tau, ni, lS, cfg, in, Gin, scIn, scOut, vec, (int)(it & 1), B.cpart[out]);
          else launch_step(G, tau, ni, lS, cfg, in, Gin, scIn, scOut, vec, (int)(it & 1), B.cpart[out]);
          in = totals(out);
          if (timing && mg) (void)hipEventRecord(g_timer.ev[c + 1], st);
        }
      }
      if (timing && !mg) (void)hipEventRecord(g_timer.ev[1], st);
      SHK_HIP(hipGetLastError());
      SHK_HIP(hipMemcpyAsync(&snap->all_done, B.all_done, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
      SHK_HIP(hipMemcpyAsync(snap->sc, B.sc + (size_t)(it & 1) * S, S * sizeof(CgScal), hipMemcpyDeviceToHost, st));
      SHK_HIP(hipStreamSynchronize(st));
      if (timing) {
        const int live = snap->live - live_before;
        float ms = 0.f;
        if (mg && live >= 2 && hipEventElapsedTime(&ms, g_timer.ev[1], g_timer.ev[live]) == hipSuccess) {
          g_timer.total_ms += ms;
          g_timer.launches += live - 1;
          g_timer.total_bytes += (double)(live - 1) * mg_iteration_bytes();
        } else if (!mg && live == chunk && hipEventElapsedTime(&ms, g_timer.ev[0], g_timer.ev[1]) == hipSuccess) {
          g_timer.total_ms += ms;
          g_timer.launches += chunk;
          g_timer.total_bytes += (double)chunk * n * S * step_bytes_per_cell();
        }
      }
      live_before = snap->live;
      if (snap->all_done) break;
      // hang guard only: every lane stops itself after cap iterations and a
      // bounded number of round changes; the rest are the tails of chunks
      if (it > 8L * cap + 16L * 512) break;
      // Launches to the end of the solve: each running lane's rate (the mean
      // of its rate since the start and since the previous poll), two more
      // launches per remaining refinement round, and never more than the
      // iterations already taken (a poll costs about as much as a few idle
      // launches; an early overestimate of a slow start far more).
      int need = mg ? 2 : 4;
      for (int r = 0; r < S; ++r) {
        const CgScal& s = snap->sc[r];
        int rem = 16;
        if (e < 0.0) {
          rem = cap - s.its + 1;   // fixed iteration count
        } else if (!s.done && s.its >= 4 && s.rnorm > 0.0 && s.rnorm < s.vnorm) {
          const double target = e * s.vnorm;
          double rate = std::log(s.rnorm / s.vnorm) / s.its;
          const int kw = s.its - prev_its[r];
          if (kw >= 8 && s.rnorm < prev_rn[r]) rate = 0.5 * (rate + std::log(s.rnorm / prev_rn[r]) / kw);
          if (s.rnorm <= target) {
            rem = 2;
          } else {
            const double lr = std::log(target / s.rnorm);
            rem = (int)std::ceil(lr / rate * 1.05) + 1;
            if (!cfg.trust) rem += 2 * (int)std::ceil(lr / lrt);
          }
          rem = std::min(rem, std::max(16, s.its));
        }
        prev_its[r] = s.its;
        prev_rn[r] = s.rnorm;
        if (s.done) continue;
        rem = std::min(rem, cap - s.its + 8);
        need = std::max(need, std::min(rem, 512));
      }
      chunk = need;
    }
    long long its_max = 0;
    for (int r = 0; r < S; ++r) its_max = std::max<long long>(its_max, snap->sc[r].its);
    inner_its += its_max;
    if (mg && fixed <= 0) mg_hist_put(tau, snap->live);
    if (use_graph) SHK_HIP(hipMemcpyAsync(z, B.gx, (size_t)N * sizeof(c128), hipMemcpyDeviceToDevice, st));
    const int Gf = grid_items(N, 1024);
    k_cocg_finish<OpD, R><<<Gf, BS, 0, st>>>(opd, tau, n, S, v, z, B.W, B.part);
    launch_final_sqrt<2>(B.part, Gf, S, pn_out, B.mz, nullptr, st);
    SHK_HIP(hipGetLastError());
    return SHK_OK;
  }

  // ---- Gram-Schmidt step of Algorithm 3 (CGS2, or MGS when mgs is set) ----
  bool mgs = false;
  int orthogonalize(int k, cx<R>* w) {
    const int kc = k + 1;
    const int Gu = (int)((N + (long)BS * GSQ - 1) / ((long)BS * GSQ));
    c128* Hk = B.H + (size_t)k * (m + 2) * S;
    gram_schmidt<R>(N, S, kc, B.V, w, Hk, B.h2, B.part, mgs, st);
    launch_final_sqrt<1>(B.part, Gu, S, B.hn, nullptr, Hk + (size_t)(k + 1) * S, st);
    k_scale_col<R><<<grid_items(N, 4096), BS, 0, st>>>(N, S, w, B.hn, B.mz, B.V + (size_t)(k + 1) * N);
    SHK_HIP(hipGetLastError());
    return SHK_OK;
  }

  // Algorithmic bytes per cell and lane of one k_cg_step: r, w, s read and
  // written (6 vectors), p read and written, x (FP64) read and written, the
  // complex inverse diagonal and the cell's share of the faces read once.
  double step_bytes_per_cell() const {
    const double wv = sizeof(cx<R>);
    double faces;
    if (p->kind == Kind::FV2D) faces = 2.0 * sizeof(R);
    else if (p->kind == Kind::FV3D) faces = 3.0 * sizeof(R);
    else faces = (double)p->nnz / (double)p->n * (sizeof(R) + sizeof(int));
    return 8.0 * wv + 32.0 + (2.0 * sizeof(R) + faces) / S;
  }

  // Algorithmic bytes of one multigrid-COCG iteration (all its launches):
  // k_cgmg_step reads r, w, s, u, p and writes r, s, p, and reads and writes
  // the FP64 x every other iteration (the deferred update); on every
  // level above the tail the down leg reads b, D^-1, the faces (and the mass
  // on coarse levels) and writes the coarse b, and the up leg reads b, D^-1,
  // the faces, the mass and the coarse x and writes x; the tail reads its top
  // level's b and writes its x (its own levels stay in LDS); k_cgmg_post reads
  // u, r and the faces and writes w.  Faces count once per cell.
  double mg_iteration_bytes() const {
    const double w = sizeof(cx<R>);
    const double fpc = (p->kind == Kind::FV3D ? 3.0 : 2.0) * sizeof(R);
    const int lS = ilog2(S);
    const int Lv = mg_levels(), t = mg_tail_level(lS);
    double bytes = (double)N * (8.0 * w + 16.0);                       // vector updates (FP64 x every other)
    if (mg_fused(lS)) bytes -= (double)N * w;                           // fused: r' not read back
    for (int l = 0; l < std::min(t, Lv - 1); ++l) {
      const double nl = mg_dims(l).n(), nc = mg_dims(l + 1).n();
      const double mass = l == 0 ? 0.0 : 8.0;
      bytes += nl * (S * w + w + fpc + mass) + nc * S * w;              // down
      bytes += nl * (S * w + w + fpc + mass + S * w) + nc * S * w;      // up
    }
    if (t < Lv) bytes += 2.0 * mg_dims(t).n() * S * w + 4.0 * mg_ta.pack_words;   // tail in/out, coefficients
    bytes += (double)N * 3.0 * w + (double)n * fpc;                     // product
    return bytes;
  }

  GivensArgs gargs(int k, int cycle, int kglob, double tol) {
    GivensArgs a{};
    a.L = L; a.S = S; a.m = m; a.k = k; a.cycle = cycle; a.kglob = kglob;
    a.tol = tol; a.inexact_ratio = 0.1; a.breakdown_rel = 1e-14;
    a.Hk = B.H + (size_t)k * (m + 2) * S;
    a.hn = B.hn; a.mz = B.mz; a.pn = B.pn; a.beta0 = B.beta0; a.sigma = B.sigma; a.taus = B.taus;
    a.ls = B.ls; a.rc = B.rc; a.rs = B.rs; a.g = B.g; a.Rp = B.Rp; a.Yb = B.Yb;
    return a;
  }

  // factored output (SHK_OUT_FACTORED): every assembly also appends its basis
  // vectors and scaled coefficients at column fz_off
  c128 *fz = nullptr, *fy = nullptr;
  int fz_cap = 0, fz_off = 0;

  int assemble(int kc, int cycle, const c128* extra, c128* X, bool accumulate) {
    const int Lb = (L + BS - 1) / BS;
    k_asm_scale<<<Lb, BS, 0, st>>>(L, cycle, B.ls, extra, B.ascale);
    launch_assemble<double>(n, S, s_real, nf, kc, m, B.Z, (size_t)N, B.Yb, B.ascale, X, accumulate ? 1 : 0, st,
                            B.Yt);
    if (fz) {
      if (fz_off + kc > fz_cap) return fail(SHK_ERR_WORKSPACE, "factored output capacity exceeded");
      k_factored_out<<<grid_items((long)(n + nf) * kc * s_real, 4096), BS, 0, st>>>(
          n, S, s_real, nf, kc, m, B.Z, (size_t)N, B.Yb, B.ascale, fz, fy, fz_cap, fz_off);
      fz_off += kc;
    }
    SHK_HIP(hipGetLastError());
    return SHK_OK;
  }

  // One FGMRES-Sh solve of all shifts for the rhs block `rhs` (interleaved
  // c128), results written or added to X (ABI layout).
  int pass(const c128* rhs, const PassSpec& ps, c128* X, bool accumulate, const c128* extra) {
    const int Lb = (L + BS - 1) / BS;
    SHK_HIP(hipMemsetAsync(B.Yb, 0, sizeof(c128) * (size_t)L * m, st));
    const int Gn = grid_items(N, 1024);
    k_norm2<double><<<Gn, BS, 0, st>>>(rhs, N, S, B.part);
    launch_final_sqrt<1>(B.part, Gn, S, B.beta0, nullptr, nullptr, st);
    k_scale_conv<R><<<grid_items(N, 4096), BS, 0, st>>>(rhs, N, S, B.beta0, B.V);
    k_lanes_init<<<Lb, BS, 0, st>>>(L, S, s_real, B.beta0, B.ls, B.g);
    SHK_HIP(hipGetLastError());
    g_phase.mark(st, PH_START);
    const std::vector<c128>& taus = *ps.taus;
    long long kglob = ps.kglob0;
    std::vector<c128> tcyc(m);
    char* stage = (char*)g_pinned.get(65536);
    int* nact = stage ? (int*)(stage + 32768) : nullptr;
    if (!nact) return fail(SHK_ERR_OOM, "pinned staging");
    double* qmax = (double*)(stage + 32768 + 64 * sizeof(int));   // per rhs: largest running quasi-residual / ||b||
    double eps_k = ps.eps;
    bool first_write = !accumulate;
    for (int cycle = 0; cycle <= ps.max_restarts; ++cycle) {
      for (int k = 0; k < m; ++k) tcyc[k] = taus[(size_t)((kglob + k) % (long long)taus.size())];
      SHK_HIP(hipMemcpyAsync(B.taus, tcyc.data(), m * sizeof(c128), hipMemcpyHostToDevice, st));
      int kend = 0;
      bool any_active = true;
      for (int k = 0; k < m; ++k) {
        g_phase.mark(st, PH_TURN);
        SHK_TRY(inner(tcyc[k], B.V + (size_t)k * N, B.Z + (size_t)k * N, eps_k, ps.inner_maxit, 0,
                      B.pn + (size_t)k * S));
        g_phase.mark(st, PH_INNER);
        SHK_TRY(orthogonalize(k, B.W));
        g_phase.mark(st, PH_GS);
        GivensArgs a = gargs(k, cycle, (int)(kglob - ps.kglob0), ps.tol);
        a.fom = ps.fom ? 1 : 0;
        launch_givens(a, st);
        k_count_active<<<1, BS, 0, st>>>(S, nf, B.ls, B.beta0, B.nact, B.qmax);
        SHK_HIP(hipGetLastError());
        SHK_HIP(hipMemcpyAsync(nact, B.nact, S * sizeof(int), hipMemcpyDeviceToHost, st));
        if (ps.relax > 0.0) SHK_HIP(hipMemcpyAsync(qmax, B.qmax, S * sizeof(double), hipMemcpyDeviceToHost, st));
        g_phase.mark(st, PH_LSQ);
        SHK_HIP(hipStreamSynchronize(st));
        if (ps.relax > 0.0) {
          // relaxed inner tolerance for the next step: the outer residual has
          // fallen to q, so the next preconditioner solve may be looser
          double q = 0.0;
          for (int r = 0; r < S; ++r) q = std::max(q, qmax[r]);
          if (q > 0.0) eps_k = std::min(ps.eps_max, std::max(ps.eps, ps.relax * ps.tol / q));
        }
        ++kglob;
        ++outer_steps;
        kend = k + 1;
        int tot = 0;
        for (int r = 0; r < S; ++r) tot += nact[r];
        if (tot == 0) {
          any_active = false;
          break;
        }
      }
      if (!any_active || cycle == ps.max_restarts) {
        // final cycle: lanes still active keep their last least-squares y
        g_phase.mark(st, PH_TURN);
        SHK_TRY(assemble(kend, cycle, extra, X, !first_write));
        if (any_active) k_finalize_active<<<Lb, BS, 0, st>>>(L, B.ls);
        SHK_HIP(hipGetLastError());
        g_phase.mark(st, PH_ASM);
        break;
      }
      GivensArgs a = gargs(m - 1, cycle, 0, ps.tol);
      if (ps.fom) {
        // ---- FOM restart: every residual lies along v_{m+1} ----
        k_restart_fom<<<Lb, BS, 0, st>>>(a);
        SHK_HIP(hipGetLastError());
        SHK_TRY(assemble(m, cycle, extra, X, !first_write));
        first_write = false;
        k_copy<R><<<grid_items(N, 4096), BS, 0, st>>>(B.V + (size_t)m * N, N, B.V);
        SHK_HIP(hipGetLastError());
        continue;
      }
      // ---- GMRES restart with collinear residuals ----
      k_restart_seed<<<1, 64, 0, st>>>(S, nf, m, B.ls, B.rc, B.rs, B.g, B.seed, B.zs, B.nzs);
      k_restart_lanes<<<Lb, BS, 0, st>>>(a, B.seed, B.zs, B.nzs);
      SHK_HIP(hipGetLastError());
      SHK_TRY(assemble(m, cycle, extra, X, !first_write));
      first_write = false;
      k_basis_combine<R><<<grid_items(N, 4096), BS, 0, st>>>(N, S, m + 1, B.V, (size_t)N, B.zs, B.W);
      k_copy<R><<<grid_items(N, 4096), BS, 0, st>>>(B.W, N, B.V);
      SHK_HIP(hipGetLastError());
      g_phase.mark(st, PH_ASM);
    }
    return SHK_OK;
  }

  // ---- block FGMRES-Sh: one basis shared by the S right-hand sides ----
  BlkCtx<R> blk() const {
    return BlkCtx<R>{n, S, st, B.gpart, B.Cc, B.Rinv, B.Gm, B.Rrow, B.Rinv64, B.fro};
  }

  // One block FGMRES-Sh pass for the S right-hand sides in `rhs` (interleaved
  // c128): block flexible Arnoldi with block CGS2 and CholQR2, each shift's
  // block least squares updated per step, per-(shift, rhs) freezing by the
  // rule of eq. trueresidual, no restart (pairs still running after m block
  // steps keep their least-squares iterate), then X (+)= scale Z y.
  int pass_block(const c128* rhs, const PassSpec& ps, c128* X, bool accumulate, const c128* extra) {
    const int Lb = (L + BS - 1) / BS;
    const int ldh = (m + 1) * S, mS = m * S;
    const int Gn = grid_items(N, 1024);
    k_norm2<double><<<Gn, BS, 0, st>>>(rhs, N, S, B.part);
    launch_final_sqrt<1>(B.part, Gn, S, B.beta0, nullptr, nullptr, st);
    k_lanes_init<<<Lb, BS, 0, st>>>(L, S, s_real, B.beta0, B.ls, B.g);
    // pairs that stop early keep zeros beyond their own basis length
    SHK_HIP(hipMemsetAsync(B.Yp, 0, sizeof(c128) * (size_t)L * mS, st));
    // start block: rhs = V_1 beta
    const BlkCtx<R> bc = blk();
    bc.template qr<double>(rhs, B.V, nullptr, 0, B.beta_blk);
    k_blk_g_init<<<grid_items((long)nf * ldh * S, 4096), BS, 0, st>>>(S, ldh, nf, B.beta_blk, B.Gq);
    SHK_HIP(hipGetLastError());
    const std::vector<c128>& taus = *ps.taus;
    char* stage = (char*)g_pinned.get(65536);
    int* nact = stage ? (int*)(stage + 32768) : nullptr;
    if (!nact) return fail(SHK_ERR_OOM, "pinned staging");
    double* qmax = (double*)(stage + 32768 + 64 * sizeof(int));
    double eps_k = ps.eps;
    int kend = 0;
    long long kglob = ps.kglob0;
    for (int k = 0; k < m; ++k) {
      const c128 tau = taus[(size_t)(kglob % (long long)taus.size())];
      ++kglob;
      cx<R>* Vk = B.V + (size_t)k * N;
      SHK_TRY(inner(tau, Vk, B.Z + (size_t)k * N, eps_k, ps.inner_maxit, 0, B.pn + (size_t)k * S));
      // block CGS2: H(0:k, k) = V^H W, W -= V H, twice
      c128* Hcol = B.Hb + (size_t)ldh * k * S;
      const bool timing = g_timer.on;
      if (timing) {
        if (!g_btimer.e0) {
          SHK_HIP(hipEventCreate(&g_btimer.e0));
          SHK_HIP(hipEventCreate(&g_btimer.e1));
        }
        SHK_HIP(hipEventRecord(g_btimer.e0, st));
      }
      bc.cgs2(B.V, (size_t)N, k + 1, B.W, Hcol, ldh);
      if (timing) SHK_HIP(hipEventRecord(g_btimer.e1, st));
      // W = V_{k+1} H(k+1, k)
      bc.template qr<R>(B.W, B.V + (size_t)(k + 1) * N, Hcol + (size_t)(k + 1) * S, ldh, nullptr);
      k_blk_breakdown<<<1, 64, 0, st>>>(B.fro, B.mz, S, B.broke);
      // each shift's block least squares, then the pairs near their target
      const BlkLsqArgs la = lsq_args(k, tau);
      blk_lsq_step(la);
      const bool last = k == m - 1;
      k_blk_mark<<<Lb, BS, 0, st>>>(L, S, B.brho, B.beta0, BLK_CAND * ps.tol, last ? 1 : 0, B.broke,
                                    outer_steps + 1, B.ls, B.want);
      BlkSolveArgs sa{S, m, k + 1, nf, ldh, outer_steps + 1, last ? 1 : 0, B.Rf, B.Rdinv, B.Gq, B.want, B.Yp,
                      B.Gw, B.pn, B.brho, B.beta0, ps.tol, 0.1, B.broke, B.ls};
      blk_backsolve_launch(sa, S, nf, st);
      k_count_active<<<1, BS, 0, st>>>(S, nf, B.ls, B.beta0, B.nact, B.qmax);
      SHK_HIP(hipGetLastError());
      int brk = 0;
      SHK_HIP(hipMemcpyAsync(nact, B.nact, S * sizeof(int), hipMemcpyDeviceToHost, st));
      SHK_HIP(hipMemcpyAsync(qmax, B.qmax, S * sizeof(double), hipMemcpyDeviceToHost, st));
      SHK_HIP(hipMemcpyAsync(&brk, B.broke, sizeof(int), hipMemcpyDeviceToHost, st));
      SHK_HIP(hipStreamSynchronize(st));
      if (timing) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, g_btimer.e0, g_btimer.e1) == hipSuccess) {
          g_btimer.calls += 1;
          g_btimer.ms += ms;
          g_btimer.flops += 4.0 * 8.0 * (double)n * (k + 1) * S * S;
        }
      }
      ++outer_steps;
      kend = k + 1;
      if (ps.relax > 0.0) {
        double q = 0.0;
        for (int r = 0; r < S; ++r) q = std::max(q, qmax[r]);
        if (q > 0.0) eps_k = std::min(ps.eps_max, std::max(ps.eps, ps.relax * ps.tol / q));
      }
      int tot = 0;
      for (int r = 0; r < S; ++r) tot += nact[r];
      if (tot == 0 || brk) break;
    }
    // pairs still running (breakdown with some pair undecided cannot happen:
    // a breakdown step decides every active pair)
    k_finalize_active<<<Lb, BS, 0, st>>>(L, B.ls);
    assemble_block(kend, extra, X, accumulate);
    SHK_HIP(hipGetLastError());
    return SHK_OK;
  }
  BlkLsqArgs lsq_args(int k, c128 tau) const {
    return BlkLsqArgs{S, m, k, nf, (m + 1) * S, B.Hb, B.sigma, tau, B.Rf, B.Vr, B.Tr, B.Qb, B.Rdinv, B.Tile, B.Gq,
                      B.brho};
  }
  // Step k of every shift's block least squares: earlier blocks' reflectors
  // on the new block column, the new block's QR, its reflectors' product.
  void blk_lsq_step(const BlkLsqArgs& la) { blk_lsq_launch(la, S, nf, st); }
  // X[:, j, r] (+)= extra_{j,r} Z y_{j,r} over kc block columns (FP64, matrix cores).
  void assemble_block(int kc, const c128* extra, c128* X, bool accumulate) {
    const int mS = m * S;
    const size_t lds = (size_t)S * (S + 1) * sizeof(c128);
    const dim3 g((unsigned)((n + 63) / 64), (unsigned)nf);
    const int acc = accumulate ? 1 : 0;
    if (S == 64) k_blk_assemble<4, 1><<<g, 256, lds, st>>>(B.Z, (size_t)N, kc, mS, B.Yp, extra, n, nf, s_real, X, acc);
    else if (S == 32) k_blk_assemble<2, 1><<<g, 256, lds, st>>>(B.Z, (size_t)N, kc, mS, B.Yp, extra, n, nf, s_real, X, acc);
    else k_blk_assemble<1, 1><<<g, 256, lds, st>>>(B.Z, (size_t)N, kc, mS, B.Yp, extra, n, nf, s_real, X, acc);
  }
};

// FP64 true residual norms ||b_r - (K + sigma_j M) x_{j,r}||, rows [r][j].
template <typename OpD>
static int residual_rows(const OpD& opd, long n, int S, int s_real, int nf, const c128* sigma, const c128* bint,
                         const c128* X, const c128* rs, int mode, c128* rpart, c128* rrow, hipStream_t st) {
  const int Gr = resid_grid(n);
  if (S >= 4) {
    constexpr int JR = 8;
    k_resid_jr<OpD, JR><<<dim3(Gr, (nf + JR - 1) / JR, s_real), BS, 0, st>>>(opd, n, S, nf, sigma, bint, X, rs, mode,
                                                                          rpart);
  } else {
    k_resid<OpD><<<dim3(Gr, nf, s_real), BS, 0, st>>>(opd, n, S, nf, sigma, bint, X, rs, mode, rpart);
  }
  k_rows_reduce<<<s_real * nf, BS, 0, st>>>(rpart, Gr, rrow);
  SHK_HIP(hipGetLastError());
  return SHK_OK;
}

// Output destinations of one group: x (FULL, ROWS) or the Z and Y parts of
// the factored output, host or device per ptr_kind.
struct GroupOut {
  c128* x = nullptr;
  c128* fz = nullptr;
  c128* fy = nullptr;
};

template <typename R>
static int solve_group(shk_problem* p, const shk_params* prm, int nf, const c128* sigma_h, int s_real,
                       const c128* b_src, int ptr_kind, const GroupOut& dst, shk_status* st_out, char* ws,
                       hipStream_t st) {
  const bool blk = prm->rhs_mode == SHK_RHS_BLOCK;
  const int S = lanes_of(s_real, blk);
  const int m = prm->m_restart;
  const long n = p->n;
  const bool host_x = ptr_kind == SHK_PTR_HOST;
  const bool use_mg = prm->inner_precond == SHK_PRECOND_MULTIGRID;
  const TuneScope ts(tune_kind(p), p->n, S, prm->precision, prm->inner_precond);
  const OutPlan op = out_plan(prm, n, nf, s_real, host_x);
  Buffers<R> B = carve<R>(ws, p, m, nf, S, s_real, op, use_mg, blk);
  c128* X = op.internal_x ? B.X : dst.x;
  // factored output: device destinations (the caller's, or staging for host)
  c128* fz = nullptr;
  c128* fy = nullptr;
  if (op.mode == SHK_OUT_FACTORED) {
    fz = host_x ? B.ostage : dst.fz;
    fy = host_x ? B.ostage + (size_t)op.kcap * n * s_real : dst.fy;
    SHK_HIP(hipMemsetAsync(fz, 0, sizeof(c128) * (size_t)op.kcap * n * s_real, st));
    SHK_HIP(hipMemsetAsync(fy, 0, sizeof(c128) * (size_t)op.kcap * nf * s_real, st));
  }
  if (op.mode == SHK_OUT_ROWS)
    SHK_HIP(hipMemcpyAsync(B.rows, prm->out_rows, sizeof(long long) * op.n_rows, hipMemcpyHostToDevice, st));
  const long N = n * S;
  // rhs into interleaved c128
  const c128* bdev = b_src;
  if (host_x) {
    SHK_HIP(hipMemcpyAsync(B.rsv, b_src, sizeof(c128) * n * s_real, hipMemcpyHostToDevice, st));
    bdev = B.rsv;
  }
  k_interleave<<<grid_items(N, 4096), BS, 0, st>>>(bdev, n, s_real, S, B.bint);
  SHK_HIP(hipMemcpyAsync(B.sigma, sigma_h, nf * sizeof(c128), hipMemcpyHostToDevice, st));
  SHK_HIP(hipGetLastError());

  std::vector<c128> taus(prm->n_tau);
  for (int i = 0; i < prm->n_tau; ++i) taus[i] = c128{prm->tau_seq[i].re, prm->tau_seq[i].im};
  const int maxit = prm->inner_maxit > 0 ? prm->inner_maxit : 20 * p->max_dim();

  std::vector<LaneState> lanes(nf * S);
  std::vector<double> bnorm(S);
  long long inner_total = 0;
  int rc = with_ops<R>(p, [&](auto op, auto opd) -> int {
    using Op = decltype(op);
    using OpD = decltype(opd);
    Group<R, Op, OpD> g{p, op, opd, st, B, n, N, S, s_real, nf, m, nf * S, item_plan(N, S)};
    g.mg = use_mg;
    g.mg_omega = prm->mg_omega;
    g.mgs = prm->ortho == SHK_MGS;
    g.fz = fz;
    g.fy = fy;
    g.fz_cap = factored_kcap(prm);
    PassSpec ps{m, prm->max_restarts, maxit, prm->tol, prm->eps_inner, &taus, 0, prm->inner_relax, prm->inner_eps_max,
                prm->variant == SHK_FOM};
    g_phase.mark(st, -1);
    SHK_TRY(blk ? g.pass_block(B.bint, ps, X, false, nullptr) : g.pass(B.bint, ps, X, false, nullptr));
    if (blk) g_phase.mark(st, PH_BLOCK);
    SHK_HIP(hipMemcpyAsync(lanes.data(), B.ls, sizeof(LaneState) * nf * S, hipMemcpyDeviceToHost, st));
    SHK_HIP(hipMemcpyAsync(bnorm.data(), B.beta0, sizeof(double) * S, hipMemcpyDeviceToHost, st));
    SHK_HIP(hipStreamSynchronize(st));
    // ---- FP64 true residuals and collinear refinement ----
    std::vector<c128> rows(s_real * nf);
    std::vector<double> rel(s_real * nf);
    std::vector<c128> extra(nf * S);
    std::vector<int> seeds(S);
    int sweeps = 0;
    auto measure = [&]() -> int {
      g_phase.mark(st, PH_TURN);
      SHK_TRY(residual_rows(opd, n, S, s_real, nf, B.sigma, B.bint, X, nullptr, 0, B.rpart, B.rrow, st));
      SHK_HIP(hipMemcpyAsync(rows.data(), B.rrow, sizeof(c128) * rows.size(), hipMemcpyDeviceToHost, st));
      g_phase.mark(st, PH_RESID);
      SHK_HIP(hipStreamSynchronize(st));
      for (int r = 0; r < s_real; ++r)
        for (int j = 0; j < nf; ++j) {
          const double nb = bnorm[r];
          rel[r * nf + j] = nb > 0.0 ? std::sqrt(rows[r * nf + j].re) / nb : std::sqrt(rows[r * nf + j].re);
        }
      return SHK_OK;
    };
    SHK_TRY(measure());
    for (; sweeps < prm->max_refine; ++sweeps) {
      bool any_bad = false;
      for (int r = 0; r < S; ++r) {
        seeds[r] = -1;
        if (r >= s_real) continue;
        double best = -1.0;
        bool bad_r = false;
        for (int j = 0; j < nf; ++j) {
          const double v = rel[r * nf + j];
          if (v > prm->tol && std::isfinite(v)) bad_r = true;
          if (v > best) { best = v; seeds[r] = j; }
        }
        any_bad |= bad_r;
        if (!bad_r) seeds[r] = -1;
      }
      if (!any_bad) break;
      g_phase.mark(st, PH_TURN);
      SHK_HIP(hipMemcpyAsync(B.seed, seeds.data(), sizeof(int) * S, hipMemcpyHostToDevice, st));
      k_resid_vec<OpD><<<grid_items(N, 4096), BS, 0, st>>>(opd, n, S, s_real, nf, B.sigma, B.seed, B.bint, X, B.rsv);
      SHK_HIP(hipGetLastError());
      SHK_TRY(residual_rows(opd, n, S, s_real, nf, B.sigma, B.bint, X, B.rsv, 1, B.rpart, B.rrow, st));
      SHK_HIP(hipMemcpyAsync(rows.data(), B.rrow, sizeof(c128) * rows.size(), hipMemcpyDeviceToHost, st));
      g_phase.mark(st, PH_RESID);
      SHK_HIP(hipStreamSynchronize(st));
      for (int r = 0; r < S; ++r)
        for (int j = 0; j < nf; ++j) {
          c128 gmm{0.0, 0.0};
          if (r < s_real && seeds[r] >= 0 && rel[r * nf + j] > prm->tol) {
            const c128 den = rows[r * nf + seeds[r]];
            gmm = cdiv(rows[r * nf + j], c128{den.re, 0.0});
          }
          extra[j * S + r] = gmm;
        }
      SHK_HIP(hipMemcpyAsync(B.extra, extra.data(), sizeof(c128) * nf * S, hipMemcpyHostToDevice, st));
      g_phase.mark(st, PH_TURN);
      PassSpec pr{m, prm->max_restarts, maxit, prm->refine_tol, prm->refine_eps_inner, &taus, 0, prm->inner_relax,
                  prm->inner_eps_max, prm->variant == SHK_FOM};
      SHK_TRY(blk ? g.pass_block(B.rsv, pr, X, true, B.extra) : g.pass(B.rsv, pr, X, true, B.extra));
      if (blk) g_phase.mark(st, PH_BLOCK);
      SHK_TRY(measure());
    }
    inner_total = g.inner_its;
    const int basis_cols = blk ? g.outer_steps * S : (fz ? g.fz_off : g.outer_steps);
    for (int r = 0; r < s_real; ++r)
      for (int j = 0; j < nf; ++j) {
        const LaneState& ls = lanes[j * S + r];
        shk_status& o = st_out[j + (long)nf * r];
        o.outer_its = ls.outer_its;
        o.restarts = ls.restarts;
        o.refine_sweeps = sweeps;
        o.basis_cols = basis_cols;
        o.reserved = 0;
        o.inner_its = inner_total;
        o.quasi_relres = bnorm[r] > 0 ? ls.rho / bnorm[r] : 0.0;
        o.bound_relres = bnorm[r] > 0 ? ls.bound / bnorm[r] : 0.0;
        o.true_relres = rel[r * nf + j];
        int s = ls.status;
        if (!std::isfinite(o.true_relres)) s = SHK_NAN;
        else if (o.true_relres <= prm->tol) s = (s == SHK_BREAKDOWN_EXACT) ? s : SHK_CONVERGED;
        else if (prm->max_refine > 0 || s == SHK_CONVERGED || s == SHK_BREAKDOWN_EXACT) s = SHK_NOT_CONVERGED;
        o.status = s;
      }
    return SHK_OK;
  });
  SHK_TRY(rc);
  if (op.mode == SHK_OUT_FULL) {
    if (host_x) SHK_HIP(hipMemcpyAsync(dst.x, X, sizeof(c128) * n * nf * s_real, hipMemcpyDeviceToHost, st));
  } else if (op.mode == SHK_OUT_ROWS) {
    const long cols = (long)nf * s_real;
    c128* out = host_x ? B.ostage : dst.x;
    k_gather_rows<<<grid_items((long)op.n_rows * cols, 4096), BS, 0, st>>>(X, n, cols, B.rows, op.n_rows, out);
    SHK_HIP(hipGetLastError());
    if (host_x)
      SHK_HIP(hipMemcpyAsync(dst.x, out, sizeof(c128) * (size_t)op.n_rows * cols, hipMemcpyDeviceToHost, st));
  } else if (host_x) {
    SHK_HIP(hipMemcpyAsync(dst.fz, fz, sizeof(c128) * (size_t)op.kcap * n * s_real, hipMemcpyDeviceToHost, st));
    SHK_HIP(hipMemcpyAsync(dst.fy, fy, sizeof(c128) * (size_t)op.kcap * nf * s_real, hipMemcpyDeviceToHost, st));
  }
  SHK_HIP(hipStreamSynchronize(st));
  g_phase.flush();
  return SHK_OK;
}

static int check_params(const shk_problem* p, const shk_params* prm, int nf, int n_rhs) {
  if (!p || !prm) return fail(SHK_ERR_INVALID_ARG, "null problem or params");
  if (nf < 1 || n_rhs < 1) return fail(SHK_ERR_INVALID_ARG, "n_shifts and n_rhs must be >= 1");
  if (prm->m_restart < 1 || prm->m_restart > 400) return fail(SHK_ERR_INVALID_ARG, "m_restart must be in [1, 400]");
  if (prm->max_restarts < 0 || prm->max_refine < 0) return fail(SHK_ERR_INVALID_ARG, "negative restart/refine count");
  if (prm->n_tau < 1 || !prm->tau_seq) return fail(SHK_ERR_INVALID_ARG, "tau_seq must hold n_tau >= 1 values");
  if (!(prm->tol > 0.0) || !(prm->eps_inner >= 0.0)) return fail(SHK_ERR_INVALID_ARG, "tol must be > 0, eps >= 0");
  if (prm->variant != SHK_GMRES && prm->variant != SHK_FOM) return fail(SHK_ERR_INVALID_ARG, "variant");
  if (prm->ortho != SHK_CGS2 && prm->ortho != SHK_MGS) return fail(SHK_ERR_INVALID_ARG, "ortho");
  if (prm->precision != SHK_FP64 && prm->precision != SHK_MIXED) return fail(SHK_ERR_INVALID_ARG, "precision");
  if (prm->inner_precond != SHK_PRECOND_JACOBI && prm->inner_precond != SHK_PRECOND_MULTIGRID)
    return fail(SHK_ERR_INVALID_ARG, "inner_precond");
  if (prm->inner_precond == SHK_PRECOND_MULTIGRID) {
    if (p->kind == Kind::CSR) return fail(SHK_ERR_UNSUPPORTED, "multigrid needs a finite-volume problem");
    if (!mg_grid_ok(p)) return fail(SHK_ERR_UNSUPPORTED, "multigrid: ny and nz must be at most 65535");
    if (prm->mg_sweeps != 1) return fail(SHK_ERR_UNSUPPORTED, "mg_sweeps must be 1");
    if (!(prm->mg_omega > 0.0 && prm->mg_omega <= 1.0)) return fail(SHK_ERR_INVALID_ARG, "mg_omega must be in (0, 1]");
  }
  if (prm->rhs_mode != SHK_RHS_LOCKSTEP && prm->rhs_mode != SHK_RHS_BLOCK) return fail(SHK_ERR_INVALID_ARG, "rhs_mode");
  if (prm->output != SHK_OUT_FULL && prm->output != SHK_OUT_ROWS && prm->output != SHK_OUT_FACTORED)
    return fail(SHK_ERR_INVALID_ARG, "output");
  if (prm->output == SHK_OUT_ROWS) {
    if (prm->n_out_rows < 1 || !prm->out_rows) return fail(SHK_ERR_INVALID_ARG, "SHK_OUT_ROWS needs out_rows");
    for (int q = 0; q < prm->n_out_rows; ++q)
      if (prm->out_rows[q] < 0 || prm->out_rows[q] >= p->n) return fail(SHK_ERR_INVALID_ARG, "out_rows outside [0, n)");
  }
  if (prm->output == SHK_OUT_FACTORED && prm->rhs_mode == SHK_RHS_BLOCK)
    return fail(SHK_ERR_UNSUPPORTED, "factored output is provided for lockstep bases only");
  if (prm->rhs_mode == SHK_RHS_BLOCK) {
    if (prm->variant != SHK_GMRES) return fail(SHK_ERR_UNSUPPORTED, "the shared block basis solves least squares (GMRES) only");
    if (prm->ortho != SHK_CGS2) return fail(SHK_ERR_UNSUPPORTED, "the shared block basis uses block CGS2");
    if (prm->m_restart > 100) return fail(SHK_ERR_INVALID_ARG, "m_restart must be <= 100 with the shared block basis");
  }
  if (!(prm->inner_relax >= 0.0) || !std::isfinite(prm->inner_relax))
    return fail(SHK_ERR_INVALID_ARG, "inner_relax must be finite and >= 0");
  if (prm->inner_relax > 0.0 && !(prm->inner_eps_max >= prm->eps_inner && prm->inner_eps_max < 1.0))
    return fail(SHK_ERR_INVALID_ARG, "inner_eps_max must be in [eps_inner, 1)");
  for (int i = 0; i < prm->n_tau; ++i)
    if (!std::isfinite(prm->tau_seq[i].re) || !std::isfinite(prm->tau_seq[i].im))
      return fail(SHK_ERR_INVALID_ARG, "non-finite tau");
  return SHK_OK;
}

int tune_class(const shk_problem* p, const shk_params* prm, int n_rhs, int* kind, long long* n, int* lanes) {
  if (!p || !prm || !kind || !n || !lanes || n_rhs < 1) return fail(SHK_ERR_INVALID_ARG, "tune class arguments");
  *kind = tune_kind(p);
  *n = p->n;
  *lanes = lanes_of(std::min(n_rhs, 64), prm->rhs_mode == SHK_RHS_BLOCK);
  return SHK_OK;
}

size_t workspace_bytes(const shk_problem* p, const shk_params* prm, int nf, int n_rhs, bool host_x) {
  const int s_real = std::min(n_rhs, 64);
  const bool blk = prm->rhs_mode == SHK_RHS_BLOCK;
  const TuneScope ts(tune_kind(p), p->n, lanes_of(s_real, blk), prm->precision, prm->inner_precond);
  return group_bytes(p, prm->m_restart, nf, lanes_of(s_real, blk), s_real, prm->precision,
                     out_plan(prm, p->n, nf, s_real, host_x), prm->inner_precond == SHK_PRECOND_MULTIGRID, blk);
}

size_t output_elems(const shk_params* prm, long n, int nf, int n_rhs, int* kcap) {
  if (kcap) *kcap = prm->output == SHK_OUT_FACTORED ? factored_kcap(prm) : 0;
  if (prm->output == SHK_OUT_ROWS) return (size_t)prm->n_out_rows * nf * n_rhs;
  if (prm->output == SHK_OUT_FACTORED) return (size_t)factored_kcap(prm) * ((size_t)n + nf) * n_rhs;
  return (size_t)n * nf * n_rhs;
}

int solve_all(shk_problem* p, const shk_params* prm, int nf, const c128* sigma, int n_rhs, const c128* b, c128* x,
              shk_status* stat, void* ws, size_t ws_bytes, hipStream_t st, int ptr_kind) {
  SHK_TRY(check_params(p, prm, nf, n_rhs));
  if (!sigma || !b || !x || !stat) return fail(SHK_ERR_INVALID_ARG, "null sigma/b/x/status");
  for (int j = 0; j < nf; ++j)
    if (!std::isfinite(sigma[j].re) || !std::isfinite(sigma[j].im)) return fail(SHK_ERR_INVALID_ARG, "non-finite shift");
  const bool host_x = ptr_kind == SHK_PTR_HOST;
  const size_t need = workspace_bytes(p, prm, nf, n_rhs, host_x);
  void* own = nullptr;
  if (!ws) {
    if (hipMalloc(&own, need) != hipSuccess) return fail(SHK_ERR_OOM, "workspace allocation failed");
    ws = own;
  } else if (ws_bytes < need) {
    return fail(SHK_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  int rc = SHK_OK;
  const long n = p->n;
  const int kcap = prm->output == SHK_OUT_FACTORED ? factored_kcap(prm) : 0;
  for (int r0 = 0; r0 < n_rhs && rc == SHK_OK; r0 += 64) {
    const int s_real = std::min(64, n_rhs - r0);
    const c128* bg = b + (size_t)n * r0;
    GroupOut go;
    if (prm->output == SHK_OUT_FULL) {
      go.x = x + (size_t)n * nf * r0;
    } else if (prm->output == SHK_OUT_ROWS) {
      go.x = x + (size_t)prm->n_out_rows * nf * r0;
    } else {
      go.fz = x + (size_t)n * kcap * r0;
      go.fy = x + (size_t)n * kcap * n_rhs + (size_t)kcap * nf * r0;
    }
    shk_status* sg = stat + (size_t)nf * r0;
    if (prm->precision == SHK_MIXED)
      rc = solve_group<float>(p, prm, nf, sigma, s_real, bg, ptr_kind, go, sg, (char*)ws, st);
    else
      rc = solve_group<double>(p, prm, nf, sigma, s_real, bg, ptr_kind, go, sg, (char*)ws, st);
  }
  if (own) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(own);
  }
  return rc;
}

// ---------------------------------------------------------- step level -----
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

int step_apply(shk_problem* p, c128 sigma, int S, const void* x, void* y, int precision, hipStream_t st) {
  if (!p || !x || !y || S < 1 || S > 64 || (S & (S - 1))) return fail(SHK_ERR_INVALID_ARG, "apply arguments");
  const long N = p->n * S;
  auto run = [&](auto tag) -> int {
    using R = decltype(tag);
    return with_op<R>(p, [&](auto op) -> int {
      k_apply<decltype(op), R><<<grid_items(N, 4096), BS, 0, st>>>(op, sigma, p->n, S, (const cx<R>*)x, (cx<R>*)y);
      SHK_HIP(hipGetLastError());
      SHK_HIP(hipStreamSynchronize(st));
      return SHK_OK;
    });
  };
  return precision == SHK_MIXED ? run(float{}) : run(double{});
}

int step_inner(shk_problem* p, c128 tau, int S, const void* v, void* z, void* w, double eps, int maxit,
               int fixed_iters, int precision, int precond, int* its, double* pnorm, hipStream_t st) {
  if (!p || !v || !z || S < 1 || S > 64 || (S & (S - 1))) return fail(SHK_ERR_INVALID_ARG, "inner arguments");
  if (precond != SHK_PRECOND_JACOBI && precond != SHK_PRECOND_MULTIGRID) return fail(SHK_ERR_INVALID_ARG, "precond");
  if (precond == SHK_PRECOND_MULTIGRID && p->kind == Kind::CSR)
    return fail(SHK_ERR_UNSUPPORTED, "multigrid needs a finite-volume problem");
  if (precond == SHK_PRECOND_MULTIGRID && !mg_grid_ok(p))
    return fail(SHK_ERR_UNSUPPORTED, "multigrid: ny and nz must be at most 65535");
  const bool use_mg = precond == SHK_PRECOND_MULTIGRID;
  if (maxit <= 0) maxit = 20 * p->max_dim();
  const TuneScope ts(tune_kind(p), p->n, S, precision, precond);
  auto run = [&](auto tag) -> int {
    using R = decltype(tag);
    const long N = p->n * S;
    const Grid gp = item_plan(N, S);
    auto lay = [&](Carver& c, Buffers<R>& b) {
      b.W = c.take<cx<R>>(N);
      for (int i = 0; i < 2; ++i) {
        b.cr[i] = c.take<cx<R>>(N); b.cw[i] = c.take<cx<R>>(N); b.cs[i] = c.take<cx<R>>(N);
        b.cpart[i] = c.take<c128>((size_t)gp.G * 3 * S); b.ctot[i] = c.take<c128>((size_t)3 * S);
      }
      b.cp = c.take<cx<R>>(N);
      b.dinv = c.take<cx<R>>(p->n);
      b.part = c.take<c128>((size_t)grid_items(N, 1024) * 2 * S);
      b.sc = c.take<CgScal>(2 * S); b.all_done = c.take<int>(4);
      b.cfgd = c.take<CgCfg>(1);
      if (tn().graph) {
        b.gv = c.take<cx<R>>(N);
        b.gx = c.take<c128>(N);
      }
      b.mz = c.take<double>(S); b.pn = c.take<double>(S);
      if (use_mg) carve_mg(c, b, p, N, S);
    };
    Carver cv{nullptr};
    Buffers<R> b0{};
    lay(cv, b0);
    DevBuf mem;
    SHK_HIP(hipMalloc(&mem.p, cv.off));
    SHK_HIP(hipMemsetAsync(mem.p, 0, cv.off, st));
    Carver c2{(char*)mem.p};
    Buffers<R> b{};
    lay(c2, b);
    return with_ops<R>(p, [&](auto op, auto opd) -> int {
      using Op = decltype(op);
      using OpD = decltype(opd);
      Group<R, Op, OpD> g{p, op, opd, st, b, p->n, N, S, S, 1, 1, S, gp};
      g.mg = use_mg;
      SHK_TRY(g.inner(tau, (const cx<R>*)v, (c128*)z, eps, maxit, fixed_iters, b.pn));
      if (w) {
        k_copy<R><<<grid_items(N, 4096), BS, 0, st>>>(b.W, N, (cx<R>*)w);
        SHK_HIP(hipGetLastError());
      }
      Snap* snap = (Snap*)g_pinned.get(65536);
      std::vector<double> pn(S);
      SHK_HIP(hipMemcpyAsync(pn.data(), b.pn, sizeof(double) * S, hipMemcpyDeviceToHost, st));
      SHK_HIP(hipStreamSynchronize(st));
      for (int r = 0; r < S; ++r) {
        if (its) its[r] = snap->sc[r].its;
        if (pnorm) pnorm[r] = pn[r];
      }
      return SHK_OK;
    });
  };
  return precision == SHK_MIXED ? run(float{}) : run(double{});
}

int step_orth(long long n, int S, int k, void* V, void* w, c128* h, int precision, int ortho, hipStream_t st) {
  if (!V || !w || !h || k < 1 || S < 1 || S > 64 || (S & (S - 1))) return fail(SHK_ERR_INVALID_ARG, "orth arguments");
  if (ortho != SHK_CGS2 && ortho != SHK_MGS) return fail(SHK_ERR_INVALID_ARG, "ortho");
  auto run = [&](auto tag) -> int {
    using R = decltype(tag);
    const long N = (long)n * S;
    const long ipb = dot_ipb(N);
    const long Gd = (N + ipb - 1) / ipb;
    const long Gu = (N + (long)BS * GSQ - 1) / ((long)BS * GSQ);
    auto lay = [&](Carver& c, Buffers<R>& b) {
      b.part = c.take<c128>(std::max<size_t>((size_t)Gd * (k + 1) * S, (size_t)Gu * S));
      b.H = c.take<c128>((size_t)(k + 2) * S); b.h2 = c.take<c128>((size_t)(k + 1) * S);
      b.hn = c.take<double>(S); b.mz = c.take<double>(S);
    };
    Carver cv{nullptr};
    Buffers<R> b0{};
    lay(cv, b0);
    DevBuf mem;
    SHK_HIP(hipMalloc(&mem.p, cv.off));
    SHK_HIP(hipMemsetAsync(mem.p, 0, cv.off, st));
    Carver c2{(char*)mem.p};
    Buffers<R> b{};
    lay(c2, b);
    std::vector<double> tiny(S, 1e-300);
    SHK_HIP(hipMemcpyAsync(b.mz, tiny.data(), sizeof(double) * S, hipMemcpyHostToDevice, st));
    cx<R>* Vp = (cx<R>*)V;
    const int kc = k;
    gram_schmidt<R>(N, S, kc, Vp, (cx<R>*)w, b.H, b.h2, b.part, ortho == SHK_MGS, st);
    launch_final_sqrt<1>(b.part, (int)Gu, S, b.hn, nullptr, b.H + (size_t)kc * S, st);
    k_scale_col<R><<<grid_items(N, 4096), BS, 0, st>>>(N, S, (const cx<R>*)w, b.hn, b.mz, Vp + (size_t)kc * N);
    SHK_HIP(hipGetLastError());
    std::vector<c128> hh((size_t)(k + 1) * S);
    SHK_HIP(hipMemcpyAsync(hh.data(), b.H, sizeof(c128) * (k + 1) * S, hipMemcpyDeviceToHost, st));
    SHK_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < S; ++r)
      for (int i = 0; i <= k; ++i) h[i + (size_t)(k + 1) * r] = hh[(size_t)i * S + r];
    return SHK_OK;
  };
  return precision == SHK_MIXED ? run(float{}) : run(double{});
}

// Block orthogonalisation step (block CGS2 + CholQR2) on device blocks.
int step_block_orth(long long n, int S, int k, void* V, void* W, c128* h, int precision, hipStream_t st) {
  if (!V || !W || !h || k < 0 || n < 1 || (S != 16 && S != 32 && S != 64))
    return fail(SHK_ERR_INVALID_ARG, "block orthogonalisation arguments (S in {16, 32, 64})");
  auto run = [&](auto tag) -> int {
    using R = decltype(tag);
    const long N = (long)n * S;
    const int ldh = (k + 1) * S;
    auto lay = [&](Carver& c, Buffers<R>& b) {
      b.gpart = c.take<c128>((size_t)BLK_WAVES * S * S);
      b.Cc = c.take<cx<R>>((size_t)(k + 1) * S * S);
      b.Rinv = c.take<cx<R>>((size_t)S * S);
      b.Gm = c.take<c128>((size_t)S * S); b.Rrow = c.take<c128>((size_t)S * S);
      b.Rinv64 = c.take<c128>((size_t)S * S); b.fro = c.take<double>(2);
      b.Hb = c.take<c128>((size_t)ldh * S);
    };
    Carver cv{nullptr};
    Buffers<R> b0{};
    lay(cv, b0);
    DevBuf mem;
    SHK_HIP(hipMalloc(&mem.p, cv.off));
    Carver c2{(char*)mem.p};
    Buffers<R> b{};
    lay(c2, b);
    const BlkCtx<R> bc{(long)n, S, st, b.gpart, b.Cc, b.Rinv, b.Gm, b.Rrow, b.Rinv64, b.fro};
    cx<R>* Vp = (cx<R>*)V;
    if (k > 0) bc.cgs2(Vp, (size_t)N, k, (cx<R>*)W, b.Hb, ldh);
    bc.template qr<R>((cx<R>*)W, Vp + (size_t)k * N, b.Hb + (size_t)k * S, ldh, nullptr);
    SHK_HIP(hipGetLastError());
    SHK_HIP(hipMemcpyAsync(h, b.Hb, sizeof(c128) * (size_t)ldh * S, hipMemcpyDeviceToHost, st));
    SHK_HIP(hipStreamSynchronize(st));
    return SHK_OK;
  };
  return precision == SHK_MIXED ? run(float{}) : run(double{});
}

// Block least squares of every shift for a given block Hessenberg (host).
int step_block_lsq(int K, int S, const c128* H, const c128* taus, int nf, const c128* sigma, const c128* beta,
                   c128* y, double* rho) {
  if (K < 1 || nf < 1 || !H || !taus || !sigma || !beta || !y || !rho || (S != 16 && S != 32 && S != 64))
    return fail(SHK_ERR_INVALID_ARG, "block least-squares arguments (S in {16, 32, 64})");
  const int m = K, ldh = (m + 1) * S, mS = m * S, L = nf * S;
  Carver cv{nullptr};
  Buffers<double> b0{};
  auto lay = [&](Carver& c, Buffers<double>& b) {
    b.Hb = c.take<c128>((size_t)ldh * mS); b.sigma = c.take<c128>(nf); b.beta_blk = c.take<c128>((size_t)S * S);
    b.Rf = c.take<c128>((size_t)nf * rpk(0, mS)); b.Vr = c.take<c128>((size_t)nf * S * (S + 1));
    b.Tr = c.take<double>((size_t)nf * S); b.Gq = c.take<c128>((size_t)nf * ldh * S);
    b.Qb = c.take<c128>((size_t)nf * m * 4 * S * S); b.Rdinv = c.take<c128>((size_t)nf * m * S * S);
    b.Tile = c.take<c128>((size_t)nf * 2 * S * S); b.Gw = c.take<c128>((size_t)L * mS);
    b.Yp = c.take<c128>((size_t)L * mS); b.brho = c.take<double>(L); b.want = c.take<int>(L);
    b.pn = c.take<double>((size_t)mS); b.beta0 = c.take<double>(S); b.ls = c.take<LaneState>(L);
    b.broke = c.take<int>(4); b.g = c.take<c128>(L);
  };
  lay(cv, b0);
  DevBuf mem;
  SHK_HIP(hipMalloc(&mem.p, cv.off));
  SHK_HIP(hipMemset(mem.p, 0, cv.off));
  Carver c2{(char*)mem.p};
  Buffers<double> b{};
  lay(c2, b);
  SHK_HIP(hipMemcpy(b.Hb, H, sizeof(c128) * (size_t)ldh * mS, hipMemcpyHostToDevice));
  SHK_HIP(hipMemcpy(b.sigma, sigma, sizeof(c128) * nf, hipMemcpyHostToDevice));
  // beta: column-major on the host, row-major for the start of G
  std::vector<c128> brow((size_t)S * S);
  std::vector<double> bn(S, 0.0);
  for (int r = 0; r < S; ++r)
    for (int i = 0; i < S; ++i) {
      brow[(size_t)i * S + r] = beta[i + (size_t)S * r];
      bn[r] += beta[i + (size_t)S * r].re * beta[i + (size_t)S * r].re + beta[i + (size_t)S * r].im * beta[i + (size_t)S * r].im;
    }
  for (int r = 0; r < S; ++r) bn[r] = std::sqrt(bn[r]);
  SHK_HIP(hipMemcpy(b.beta_blk, brow.data(), sizeof(c128) * brow.size(), hipMemcpyHostToDevice));
  SHK_HIP(hipMemcpy(b.beta0, bn.data(), sizeof(double) * S, hipMemcpyHostToDevice));
  k_lanes_init<<<(L + BS - 1) / BS, BS>>>(L, S, S, b.beta0, b.ls, b.g);
  k_blk_g_init<<<grid_items((long)nf * ldh * S, 4096), BS>>>(S, ldh, nf, b.beta_blk, b.Gq);
  std::vector<double> hr(L);
  for (int k = 0; k < K; ++k) {
    BlkLsqArgs la{S, m, k, nf, ldh, b.Hb, b.sigma, taus[k], b.Rf, b.Vr, b.Tr, b.Qb, b.Rdinv, b.Tile, b.Gq, b.brho};
    blk_lsq_launch(la, S, nf, nullptr);
    SHK_HIP(hipGetLastError());
    SHK_HIP(hipMemcpy(hr.data(), b.brho, sizeof(double) * L, hipMemcpyDeviceToHost));
    for (int p = 0; p < L; ++p) rho[p + (size_t)L * k] = hr[p];
  }
  k_blk_mark<<<(L + BS - 1) / BS, BS>>>(L, S, b.brho, b.beta0, 0.0, 1, b.broke, K, b.ls, b.want);
  BlkSolveArgs sa{S, m, K, nf, ldh, K, 1, b.Rf, b.Rdinv, b.Gq, b.want, b.Yp, b.Gw, b.pn, b.brho, b.beta0, 0.0, -1.0,
                  b.broke, b.ls};
  blk_backsolve_launch(sa, S, nf, nullptr);
  SHK_HIP(hipGetLastError());
  SHK_HIP(hipMemcpy(y, b.Yp, sizeof(c128) * (size_t)L * mS, hipMemcpyDeviceToHost));
  return SHK_OK;
}

int step_lsq(int K, const c128* H, const c128* taus, int nf, const c128* sigma, double beta, c128* y, double* rho,
             int variant) {
  if (K < 1 || nf < 1 || !H || !taus || !sigma || !y || !rho) return fail(SHK_ERR_INVALID_ARG, "lsq arguments");
  if (variant != SHK_GMRES && variant != SHK_FOM) return fail(SHK_ERR_INVALID_ARG, "variant");
  const int m = K, S = 1, L = nf;
  Carver cv{nullptr};
  Buffers<double> b0{};
  auto lay = [&](Carver& c, Buffers<double>& b) {
    b.H = c.take<c128>((size_t)m * (m + 2)); b.hn = c.take<double>(1); b.mz = c.take<double>(1);
    b.pn = c.take<double>(m); b.beta0 = c.take<double>(1); b.sigma = c.take<c128>(nf); b.taus = c.take<c128>(m);
    b.ls = c.take<LaneState>(L); b.rc = c.take<double>((size_t)m * L); b.rs = c.take<c128>((size_t)m * L);
    b.g = c.take<c128>((size_t)(m + 1) * L); b.Rp = c.take<c128>((size_t)m * (m + 1) / 2 * L);
    b.Yb = c.take<c128>((size_t)L * m);
  };
  lay(cv, b0);
  DevBuf mem;
  SHK_HIP(hipMalloc(&mem.p, cv.off));
  SHK_HIP(hipMemset(mem.p, 0, cv.off));
  Carver c2{(char*)mem.p};
  Buffers<double> b{};
  lay(c2, b);
  // Hbar column k at H[k*(m+2) + i]
  std::vector<c128> Hd((size_t)m * (m + 2), c128{0, 0});
  for (int k = 0; k < K; ++k)
    for (int i = 0; i <= k + 1; ++i) Hd[(size_t)k * (m + 2) + i] = H[i + (size_t)(K + 1) * k];
  SHK_HIP(hipMemcpy(b.H, Hd.data(), sizeof(c128) * Hd.size(), hipMemcpyHostToDevice));
  SHK_HIP(hipMemcpy(b.sigma, sigma, sizeof(c128) * nf, hipMemcpyHostToDevice));
  SHK_HIP(hipMemcpy(b.taus, taus, sizeof(c128) * K, hipMemcpyHostToDevice));
  SHK_HIP(hipMemcpy(b.beta0, &beta, sizeof(double), hipMemcpyHostToDevice));
  const double one = 1.0;
  SHK_HIP(hipMemcpy(b.mz, &one, sizeof(double), hipMemcpyHostToDevice));
  k_lanes_init<<<(L + BS - 1) / BS, BS>>>(L, 1, 1, b.beta0, b.ls, b.g);
  std::vector<LaneState> ls(L);
  for (int k = 0; k < K; ++k) {
    const double hnk = Hd[(size_t)k * (m + 2) + k + 1].re;
    SHK_HIP(hipMemcpy(b.hn, &hnk, sizeof(double), hipMemcpyHostToDevice));
    GivensArgs a{};
    a.L = L; a.S = S; a.m = m; a.k = k; a.cycle = 0; a.kglob = k; a.fom = variant == SHK_FOM ? 1 : 0;
    a.tol = 0.0; a.inexact_ratio = -1.0; a.breakdown_rel = 0.0;
    a.Hk = b.H + (size_t)k * (m + 2); a.hn = b.hn; a.mz = b.mz; a.pn = b.pn; a.beta0 = b.beta0;
    a.sigma = b.sigma; a.taus = b.taus; a.ls = b.ls; a.rc = b.rc; a.rs = b.rs; a.g = b.g; a.Rp = b.Rp; a.Yb = b.Yb;
    launch_givens(a, nullptr);
    SHK_HIP(hipGetLastError());
    SHK_HIP(hipMemcpy(ls.data(), b.ls, sizeof(LaneState) * L, hipMemcpyDeviceToHost));
    for (int j = 0; j < nf; ++j) rho[j + (size_t)nf * k] = ls[j].rho;
  }
  std::vector<c128> Y((size_t)L * m);
  SHK_HIP(hipMemcpy(Y.data(), b.Yb, sizeof(c128) * Y.size(), hipMemcpyDeviceToHost));
  for (int j = 0; j < nf; ++j)
    for (int i = 0; i < K; ++i) y[i + (size_t)K * j] = Y[(size_t)j * m + i];
  return SHK_OK;
}

int step_assemble(long long n, int k, int nf, const void* Z, const c128* Y, c128* X, int acc, int precision,
                  hipStream_t st) {
  if (!Z || !Y || !X || k < 1 || nf < 1 || n < 1) return fail(SHK_ERR_INVALID_ARG, "assemble arguments");
  DevBuf ones;
  SHK_HIP(hipMalloc(&ones.p, sizeof(c128) * nf));
  std::vector<c128> o(nf, c128{1.0, 0.0});
  SHK_HIP(hipMemcpyAsync(ones.p, o.data(), sizeof(c128) * nf, hipMemcpyHostToDevice, st));
  auto run = [&](auto tag) -> int {
    using R = decltype(tag);
    launch_assemble<R>((long)n, 1, 1, nf, k, k, (const cx<R>*)Z, (size_t)n, Y, (const c128*)ones.p, X, acc, st);
    SHK_HIP(hipGetLastError());
    SHK_HIP(hipStreamSynchronize(st));
    return SHK_OK;
  };
  return precision == SHK_MIXED ? run(float{}) : run(double{});
}

int step_sensitivity(shk_problem* p, int nf, int ns, const c128* phi, int nr, const c128* psi, void* J, int precision,
                     hipStream_t st) {
  if (!p || !phi || !psi || !J || nf < 1 || ns < 1 || nr < 1) return fail(SHK_ERR_INVALID_ARG, "sensitivity arguments");
  if (p->kind == Kind::CSR || !p->cellK) return fail(SHK_ERR_UNSUPPORTED, "sensitivities need a finite-volume problem");
  if (precision != SHK_FP64 && precision != SHK_MIXED) return fail(SHK_ERR_INVALID_ARG, "precision");
  constexpr int TS = 4;
  const long gx = (p->n + BS - 1) / BS * ((ns + TS - 1) / TS);
  if (nf > 65535 || gx * nf > 0x7fffffffL) return fail(SHK_ERR_INVALID_ARG, "too many shifts or sources for one launch");
  SensArgs a{p->nx, p->ny, p->nz, p->tx, p->ty, p->tz, p->cellK, phi, psi, nf, ns, nr};
  const dim3 g((unsigned)gx, (unsigned)nf);
  const bool d3 = p->kind == Kind::FV3D;
  if (precision == SHK_FP64) {
    if (d3) k_sensitivity<double, TS, 6><<<g, BS, 0, st>>>(a, (c128*)J);
    else k_sensitivity<double, TS, 4><<<g, BS, 0, st>>>(a, (c128*)J);
  } else {
    if (d3) k_sensitivity<float, TS, 6><<<g, BS, 0, st>>>(a, (c64*)J);
    else k_sensitivity<float, TS, 4><<<g, BS, 0, st>>>(a, (c64*)J);
  }
  SHK_HIP(hipGetLastError());
  return SHK_OK;
}

// Scratch of the true-residual entry points, carved from base (nullptr: sizes
// only): the shifts, residual partials [nf][Gr], residual rows [nf], partials
// of ||b||^2 [Gn] and ||b||.  Every slot is written before it is read.
struct ResidScratch {
  c128 *sg, *part, *rows, *npart;
  double* nbd;
  size_t bytes;
};
static ResidScratch resid_scratch(char* base, long n, int nf) {
  Carver c{base};
  ResidScratch r{};
  r.sg = c.take<c128>(nf);
  r.part = c.take<c128>((size_t)nf * resid_grid(n));
  r.rows = c.take<c128>(nf);
  r.npart = c.take<c128>(grid_items(n, 1024));
  r.nbd = c.take<double>(2);
  r.bytes = c.off;
  return r;
}

static int check_resid_args(shk_problem* p, int nf, const c128* sigma, const c128* b, const c128* x,
                            const double* relres) {
  if (!p || !sigma || !b || !x || !relres || nf < 1) return fail(SHK_ERR_INVALID_ARG, "residual arguments");
  if (nf > 65535) return fail(SHK_ERR_INVALID_ARG, "at most 65535 shifts per residual call");
  return SHK_OK;
}

// ||b - (K + sigma_j M) x_j|| / ||b|| with the scratch at base (device).
static int true_residual_in(shk_problem* p, int nf, const c128* sigma, const c128* b, const c128* x, double* relres,
                            hipStream_t st, char* base) {
  const long n = p->n;
  const int Gn = grid_items(n, 1024);
  const ResidScratch r = resid_scratch(base, n, nf);
  SHK_HIP(hipMemcpyAsync(r.sg, sigma, sizeof(c128) * nf, hipMemcpyHostToDevice, st));
  k_norm2<double><<<Gn, BS, 0, st>>>(b, n, 1, r.npart);
  k_final_sqrt<1><<<1, BS, 0, st>>>(r.npart, Gn, 1, r.nbd, nullptr, nullptr);
  SHK_TRY(with_op<double>(p, [&](auto opd) -> int {
    return residual_rows(opd, n, 1, 1, nf, r.sg, b, x, nullptr, 0, r.part, r.rows, st);
  }));
  std::vector<c128> hr(nf);
  double bn = 0.0;
  SHK_HIP(hipMemcpyAsync(hr.data(), r.rows, sizeof(c128) * nf, hipMemcpyDeviceToHost, st));
  SHK_HIP(hipMemcpyAsync(&bn, r.nbd, sizeof(double), hipMemcpyDeviceToHost, st));
  SHK_HIP(hipStreamSynchronize(st));
  for (int j = 0; j < nf; ++j) relres[j] = bn > 0 ? std::sqrt(hr[j].re) / bn : std::sqrt(hr[j].re);
  return SHK_OK;
}

int step_true_residual(shk_problem* p, int nf, const c128* sigma, const c128* b, const c128* x, double* relres,
                       hipStream_t st) {
  SHK_TRY(check_resid_args(p, nf, sigma, b, x, relres));
  DevBuf mem;
  SHK_HIP(hipMalloc(&mem.p, resid_scratch(nullptr, p->n, nf).bytes));
  return true_residual_in(p, nf, sigma, b, x, relres, st, (char*)mem.p);
}

// ------------------------------------------- allocation-free residual ------
// The same residual with its scratch in a fixed device array: for callers that
// cannot allocate device memory.  Each device holds its own copy of the array
// for the life of the process; its address is looked up once per device, with
// that device current, on the first call there.  Calls that overlap on one
// device share the array and race.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_addr[64] = {};

static int scratch_address(void** out) {
  int dev = 0;
  SHK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(SHK_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    SHK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(SHK_ERR_HIP, "no device address for the residual scratch");
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return SHK_OK;
}

int step_true_residual_noalloc(shk_problem* p, int nf, const c128* sigma, const c128* b, const c128* x,
                               double* relres, hipStream_t st) {
  SHK_TRY(check_resid_args(p, nf, sigma, b, x, relres));
  const size_t need = resid_scratch(nullptr, p->n, nf).bytes;
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(SHK_ERR_WORKSPACE, "residual scratch of " + std::to_string(need) + " bytes exceeds the fixed " +
                                       std::to_string(NOALLOC_SCRATCH_BYTES) + " (fewer shifts per call)");
  void* base = nullptr;
  SHK_TRY(scratch_address(&base));
  return true_residual_in(p, nf, sigma, b, x, relres, st, (char*)base);
}

}  // namespace shk
