// extern "C" entry points of the shifted-Krylov library (declared in shk.h).
#include <cmath>
#include <new>
#include <string>

#include "internal.hpp"

using shk::c128;

extern "C" {

void shk_params_default(shk_params* p) {
  if (!p) return;
  p->m_restart = 50;
  p->max_restarts = 20;
  p->max_refine = 2;
  p->inner_maxit = 0;
  p->tol = 1e-8;
  p->eps_inner = 1e-10;
  p->n_tau = 0;
  p->tau_seq = nullptr;
  p->variant = SHK_GMRES;
  p->precision = SHK_FP64;
  p->refine_tol = 0.05;
  p->refine_eps_inner = 5e-3;
  p->inner_precond = SHK_PRECOND_JACOBI;
  p->mg_sweeps = 1;
  p->mg_omega = 0.8;
  p->inner_relax = 0.0;
  p->inner_eps_max = 1e-2;
  p->ortho = SHK_CGS2;
  p->rhs_mode = SHK_RHS_LOCKSTEP;
  p->output = SHK_OUT_FULL;
  p->n_out_rows = 0;
  p->out_rows = nullptr;
}

static int create_fv(int nx, int ny, int nz, shk::Kind kind, const double* cell_K, double Ss, double h,
                     shk_problem** out) {
  if (!out || !cell_K) return shk::fail(SHK_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1) return shk::fail(SHK_ERR_INVALID_ARG, "grid dimensions must be >= 1");
  if ((double)nx * ny * nz > 2.0e9) return shk::fail(SHK_ERR_INVALID_ARG, "grid too large");
  shk_problem* p = new (std::nothrow) shk_problem();
  if (!p) return shk::fail(SHK_ERR_OOM, "host allocation");
  p->kind = kind;
  p->nx = nx;
  p->ny = ny;
  p->nz = nz;
  const int rc = shk::problem_setup_fv(p, cell_K, Ss, h, nullptr);
  if (rc != SHK_OK) {
    shk::problem_free(p, nullptr);
    delete p;
    return rc;
  }
  *out = p;
  return SHK_OK;
}

int shk_problem_create_fv2d(int nx, int ny, const double* cell_K, double Ss, double h, shk_problem** out) {
  return create_fv(nx, ny, 1, shk::Kind::FV2D, cell_K, Ss, h, out);
}

int shk_problem_create_fv3d(int nx, int ny, int nz, const double* cell_K, double Ss, double h,
                            shk_problem** out) {
  return create_fv(nx, ny, nz, shk::Kind::FV3D, cell_K, Ss, h, out);
}

int shk_problem_create_csr(int n, const int* rowptr, const int* col, const double* K_val, const double* M_diag,
                           shk_problem** out) {
  if (!out || !rowptr || !col || !K_val || !M_diag) return shk::fail(SHK_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (n < 1) return shk::fail(SHK_ERR_INVALID_ARG, "n must be >= 1");
  shk_problem* p = new (std::nothrow) shk_problem();
  if (!p) return shk::fail(SHK_ERR_OOM, "host allocation");
  p->kind = shk::Kind::CSR;
  p->n = n;
  const int rc = shk::problem_setup_csr(p, rowptr, col, K_val, M_diag, nullptr);
  if (rc != SHK_OK) {
    shk::problem_free(p, nullptr);
    delete p;
    return rc;
  }
  *out = p;
  return SHK_OK;
}

void shk_problem_destroy(shk_problem* p) {
  if (!p) return;
  shk::problem_free(p, nullptr);
  delete p;
}

long long shk_problem_size(const shk_problem* p) { return p ? p->n : 0; }

int shk_workspace_bytes(const shk_problem* p, const shk_params* prm, int n_shifts, int n_rhs, size_t* bytes) {
  if (!p || !prm || !bytes || n_shifts < 1 || n_rhs < 1 || prm->m_restart < 1)
    return shk::fail(SHK_ERR_INVALID_ARG, "workspace arguments");
  *bytes = shk::workspace_bytes(p, prm, n_shifts, n_rhs, false);
  return SHK_OK;
}

int shk_output_elems(const shk_problem* p, const shk_params* prm, int n_shifts, int n_rhs, size_t* elems,
                     int* k_cap) {
  if (!p || !prm || !elems || n_shifts < 1 || n_rhs < 1) return shk::fail(SHK_ERR_INVALID_ARG, "output_elems arguments");
  *elems = shk::output_elems(prm, p->n, n_shifts, n_rhs, k_cap);
  return SHK_OK;
}

int fgmres_sh_solve(shk_problem* p, const shk_params* prm, int n_shifts, const shk_c128* sigma, int n_rhs,
                    const shk_c128* b, shk_c128* x, shk_status* st, void* workspace, size_t ws_bytes,
                    void* hip_stream, int ptr_kind) {
  if (ptr_kind != SHK_PTR_HOST && ptr_kind != SHK_PTR_DEVICE) return shk::fail(SHK_ERR_INVALID_ARG, "ptr_kind");
  if (ptr_kind == SHK_PTR_HOST && workspace) {
    // host x needs the device staging area that the host-layout workspace includes
    if (ws_bytes < shk::workspace_bytes(p, prm, n_shifts, n_rhs, true))
      return shk::fail(SHK_ERR_WORKSPACE, "host pointers need a larger workspace; pass NULL to let the library allocate");
  }
  return shk::solve_all(p, prm, n_shifts, reinterpret_cast<const c128*>(sigma), n_rhs,
                        reinterpret_cast<const c128*>(b), reinterpret_cast<c128*>(x), st, workspace, ws_bytes,
                        (hipStream_t)hip_stream, ptr_kind);
}

int shk_apply_shifted(shk_problem* p, shk_c128 sigma, int n_rhs, const void* x, void* y, int precision,
                      void* hip_stream) {
  return shk::step_apply(p, c128{sigma.re, sigma.im}, n_rhs, x, y, precision, (hipStream_t)hip_stream);
}

int shk_inner_solve(shk_problem* p, shk_c128 tau, int n_rhs, const void* v, void* z, void* w, double eps, int maxit,
                    int fixed_iters, int precision, int precond, int* its, double* pnorm, void* hip_stream) {
  return shk::step_inner(p, c128{tau.re, tau.im}, n_rhs, v, z, w, eps, maxit, fixed_iters, precision, precond, its,
                         pnorm, (hipStream_t)hip_stream);
}

int shk_orthogonalize(long long n, int n_rhs, int k, void* V, void* w, shk_c128* h, int precision, int ortho,
                      void* hip_stream) {
  return shk::step_orth(n, n_rhs, k, V, w, reinterpret_cast<c128*>(h), precision, ortho, (hipStream_t)hip_stream);
}

int shk_shifted_lsq(int k, const shk_c128* Hbar, const shk_c128* taus, int n_shifts, const shk_c128* sigma,
                    double beta, shk_c128* y, double* rho, int variant) {
  return shk::step_lsq(k, reinterpret_cast<const c128*>(Hbar), reinterpret_cast<const c128*>(taus), n_shifts,
                       reinterpret_cast<const c128*>(sigma), beta, reinterpret_cast<c128*>(y), rho, variant);
}

int shk_block_orthogonalize(long long n, int n_rhs, int k, void* V, void* W, shk_c128* h, int precision,
                            void* hip_stream) {
  return shk::step_block_orth(n, n_rhs, k, V, W, reinterpret_cast<c128*>(h), precision, (hipStream_t)hip_stream);
}

int shk_block_shifted_lsq(int k, int n_rhs, const shk_c128* Hbar, const shk_c128* taus, int n_shifts,
                          const shk_c128* sigma, const shk_c128* beta, shk_c128* y, double* rho) {
  return shk::step_block_lsq(k, n_rhs, reinterpret_cast<const c128*>(Hbar), reinterpret_cast<const c128*>(taus),
                             n_shifts, reinterpret_cast<const c128*>(sigma), reinterpret_cast<const c128*>(beta),
                             reinterpret_cast<c128*>(y), rho);
}

int shk_assemble(long long n, int k, int n_shifts, const void* Z, const shk_c128* Y, shk_c128* X, int accumulate,
                 int precision, void* hip_stream) {
  return shk::step_assemble(n, k, n_shifts, Z, reinterpret_cast<const c128*>(Y), reinterpret_cast<c128*>(X),
                            accumulate, precision, (hipStream_t)hip_stream);
}

int shk_sensitivity(shk_problem* p, int n_shifts, int n_src, const shk_c128* phi, int n_rec, const shk_c128* psi,
                    void* J, int precision, void* hip_stream) {
  return shk::step_sensitivity(p, n_shifts, n_src, reinterpret_cast<const c128*>(phi), n_rec,
                               reinterpret_cast<const c128*>(psi), J, precision, (hipStream_t)hip_stream);
}

int shk_true_residual(shk_problem* p, int n_shifts, const shk_c128* sigma, const shk_c128* b, const shk_c128* x,
                      double* relres, void* hip_stream) {
  return shk::step_true_residual(p, n_shifts, reinterpret_cast<const c128*>(sigma), reinterpret_cast<const c128*>(b),
                                 reinterpret_cast<const c128*>(x), relres, (hipStream_t)hip_stream);
}

int shk_true_residual_noalloc(shk_problem* p, int n_shifts, const shk_c128* sigma, const shk_c128* b,
                              const shk_c128* x, double* relres, void* hip_stream) {
  return shk::step_true_residual_noalloc(p, n_shifts, reinterpret_cast<const c128*>(sigma),
                                         reinterpret_cast<const c128*>(b), reinterpret_cast<const c128*>(x), relres,
                                         (hipStream_t)hip_stream);
}

int shk_profile_read_phases(double* ms, int n) { return shk::profile_read_phases(ms, n); }

int shk_tune_set(int kind, long long n, int lanes, int precision, int inner_precond, const char* knob,
                 double value) {
  return shk::tune_set(kind, n, lanes, precision, inner_precond, knob, value);
}
int shk_tune_get(int kind, long long n, int lanes, int precision, int inner_precond, const char* knob,
                 double* value) {
  return shk::tune_get(kind, n, lanes, precision, inner_precond, knob, value);
}
int shk_tune_reset(void) { return shk::tune_reset(); }
int shk_tune_class(const shk_problem* p, const shk_params* prm, int n_rhs, int* kind, long long* n, int* lanes) {
  return shk::tune_class(p, prm, n_rhs, kind, n, lanes);
}

const char* shk_status_string(int code) {
  switch (code) {
    case SHK_CONVERGED: return "converged";
    case SHK_NOT_CONVERGED: return "not converged";
    case SHK_INNER_LIMITED: return "inner-solve limited";
    case SHK_BREAKDOWN_EXACT: return "breakdown (exact solution)";
    case SHK_NAN: return "non-finite value";
    case SHK_ERR_INVALID_ARG: return "invalid argument";
    case SHK_ERR_OOM: return "out of memory";
    case SHK_ERR_HIP: return "HIP runtime error";
    case SHK_ERR_NOT_READY: return "not ready";
    case SHK_ERR_UNSUPPORTED: return "unsupported";
    case SHK_ERR_WORKSPACE: return "workspace too small";
    case SHK_ERR_REJECTED: return "request rejected";
    default: return "unknown code";
  }
}

const char* shk_last_error(void) { return shk::last_error_text(); }

int shk_profile_enable(int on) { return shk::profile_enable(on); }
int shk_profile_read(long long* launches, double* total_ms, double* total_bytes) {
  return shk::profile_read(launches, total_ms, total_bytes);
}
int shk_profile_read_block(long long* calls, double* total_ms, double* total_flops) {
  return shk::profile_read_block(calls, total_ms, total_flops);
}

}  // extern "C"
