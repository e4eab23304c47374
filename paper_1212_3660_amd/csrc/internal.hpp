// Internal host-side declarations of the shifted-Krylov library.
#pragma once
#include <string>
#include <vector>
#include "common.hpp"
#include "ops.hpp"
#include "../../include/shk.h"

namespace shk {

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define SHK_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return ::shk::fail(SHK_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define SHK_TRY(call)         \
  do {                        \
    int rc_ = (call);         \
    if (rc_ != SHK_OK) return rc_; \
  } while (0)

enum class Kind { FV2D, FV3D, CSR };

// Bump allocation from a caller-owned device region (the solve server's
// per-request region): 256-byte aligned, nothing freed individually.
struct Bump {
  char* base = nullptr;
  size_t off = 0, cap = 0;
  void* take(size_t bytes) {
    const size_t o = (off + 255) & ~size_t(255);
    if (o + bytes > cap) return nullptr;
    off = o + bytes;
    return base + o;
  }
};

// One coarse level of the multigrid hierarchy (level 0 is the problem's own
// grid): cells, faces (FP64 and FP32) and per-cell mass on the device.
struct MgLevel {
  int nx = 1, ny = 1, nz = 1;
  long long n = 0;
  double* t[3] = {nullptr, nullptr, nullptr};
  float* t32[3] = {nullptr, nullptr, nullptr};
  double* mass = nullptr;
};

}  // namespace shk

// The problem: device copies of the operator coefficients in FP64 (and FP32
// for the complex64 path).  Owned by the handle.
struct shk_problem {
  shk::Kind kind;
  int nx = 1, ny = 1, nz = 1;
  long long n = 0;
  double m0 = 0.0;                  // uniform mass value (FV problems)
  int device = 0;
  // finite volume faces
  double* tx = nullptr; double* ty = nullptr; double* tz = nullptr;
  float* tx32 = nullptr; float* ty32 = nullptr; float* tz32 = nullptr;
  // CSR
  int* rowptr = nullptr; int* col = nullptr;
  double* val = nullptr; float* val32 = nullptr;
  double* diag = nullptr;           // diagonal of K (CSR only)
  double* cellK = nullptr;          // cell conductivity (finite-volume problems; sensitivities)
  double* dK = nullptr;             // diagonal of K, every kind (Jacobi preconditioner)
  float* dK32 = nullptr;
  double* mdiag = nullptr;          // per-row mass (CSR only)
  long long nnz = 0;
  std::vector<shk::MgLevel> mg;     // coarse levels (finite-volume problems)
  shk::Bump* bump = nullptr;        // device arrays from this region instead of the HIP allocator
  int max_dim() const { return nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz); }
};

namespace shk {

int solve_all(shk_problem* p, const shk_params* prm, int n_shifts, const c128* sigma, int n_rhs,
              const c128* b, c128* x, shk_status* st, void* ws, size_t ws_bytes,
              hipStream_t stream, int ptr_kind);

int step_apply(shk_problem* p, c128 sigma, int S, const void* x, void* y, int precision,
               hipStream_t stream);
int step_inner(shk_problem* p, c128 tau, int S, const void* v, void* z, void* w, double eps,
               int maxit, int fixed_iters, int precision, int precond, int* its, double* pnorm,
               hipStream_t stream);
int step_orth(long long n, int S, int k, void* V, void* w, c128* h, int precision, int ortho,
              hipStream_t stream);
int step_lsq(int k, const c128* H, const c128* taus, int nf, const c128* sigma, double beta,
             c128* y, double* rho, int variant);
int step_block_orth(long long n, int S, int k, void* V, void* W, c128* h, int precision, hipStream_t stream);
int step_block_lsq(int k, int S, const c128* H, const c128* taus, int nf, const c128* sigma, const c128* beta,
                   c128* y, double* rho);
int step_assemble(long long n, int k, int nf, const void* Z, const c128* Y, c128* X, int acc,
                  int precision, hipStream_t stream);
int step_sensitivity(shk_problem* p, int nf, int ns, const c128* phi, int nr, const c128* psi, void* J, int precision,
                     hipStream_t st);
int step_true_residual(shk_problem* p, int nf, const c128* sigma, const c128* b, const c128* x,
                       double* relres, hipStream_t stream);
// Bytes of the fixed device array behind shk_true_residual_noalloc.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(9) << 20;
int step_true_residual_noalloc(shk_problem* p, int nf, const c128* sigma, const c128* b, const c128* x,
                               double* relres, hipStream_t stream);

int problem_setup_fv(shk_problem* p, const double* cellK_host, double Ss, double h, hipStream_t st);
int problem_setup_csr(shk_problem* p, const int* rowptr, const int* col, const double* val,
                      const double* mdiag, hipStream_t st);
void problem_free(shk_problem* p, hipStream_t st);
size_t problem_bytes(const shk_problem* p);
void problem_plan_levels(shk_problem* p);
size_t workspace_bytes(const shk_problem* p, const shk_params* prm, int nf, int n_rhs, bool host_x);
size_t output_elems(const shk_params* prm, long n, int nf, int n_rhs, int* kcap);
const char* last_error_text();
int profile_enable(int on);
int profile_read(long long* launches, double* ms, double* bytes);
int profile_read_block(long long* calls, double* ms, double* flops);
int profile_read_phases(double* ms, int n);
int tune_set(int kind, long long n, int lanes, int precision, int precond, const char* knob, double value);
int tune_get(int kind, long long n, int lanes, int precision, int precond, const char* knob, double* value);
int tune_reset();
int tune_class(const shk_problem* p, const shk_params* prm, int n_rhs, int* kind, long long* n, int* lanes);

}  // namespace shk
