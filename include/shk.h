/*
 * shk.h - C ABI of the MI355X flexible Krylov solver for shifted systems.
 *
 * Method: Saibaba, Bakhos, Kitanidis, "A Flexible Krylov Solver for Shifted
 * Systems with Application to Oscillatory Hydraulic Tomography" (arXiv
 * 1212.3660).  The library solves the family
 *
 *     (K + sigma_j M) x_j = b,   j = 1..n_f                  (section 2, eq. multipleshifted)
 *
 * with one flexible Arnoldi basis built from preconditioners K + tau_k M
 * (Algorithm 3), a per-shift projected problem (Algorithm 4, GMRES or FOM),
 * inexact inner solves of the preconditioner systems (section 4, eq.
 * zmmoditer) and the true-residual bound of eq. trueresidual as stopping test.
 * K is real symmetric positive definite, M real diagonal (lumped mass), the
 * shifts complex (sigma = i omega for the phasor equation, section 5.1).
 *
 * Conventions shared by every entry point
 *  - Complex numbers are shk_c128 {re, im} (complex128) unless a call says
 *    complex64 ({float re, im}).
 *  - Cells are numbered x fastest: c = x + nx*(y + ny*z).
 *  - A block of vectors "n x k column-major" stores element (i, j) at i + n*j.
 *  - "device" pointers are HIP device allocations on the current device; "host"
 *    pointers are ordinary memory.  The library never frees caller memory.
 *  - Return value: SHK_OK (0) or a negative SHK_ERR_* code; shk_last_error()
 *    then returns a thread-local message.  Non-convergence is not a call
 *    error: it is reported per (shift, rhs) in shk_status.status.
 *  - hip_stream may be NULL (the default stream).  Calls are stream-ordered
 *    and synchronise that stream before returning unless stated otherwise.
 */
#ifndef SHK_H
#define SHK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } shk_c128;
typedef struct { float re, im; } shk_c64;
typedef struct shk_problem shk_problem;
typedef struct shk_server shk_server;

/* call errors */
#define SHK_OK 0
#define SHK_ERR_INVALID_ARG (-1)
#define SHK_ERR_OOM (-2)
#define SHK_ERR_HIP (-3)
#define SHK_ERR_NOT_READY (-4)
#define SHK_ERR_UNSUPPORTED (-5)
#define SHK_ERR_WORKSPACE (-6)
#define SHK_ERR_REJECTED (-7)

/* per-(shift, rhs) solve status (section 4 stopping test, section 3 breakdown) */
#define SHK_CONVERGED 0        /* FP64 true relative residual <= tol            */
#define SHK_NOT_CONVERGED 1    /* restart / refinement budget exhausted          */
#define SHK_INNER_LIMITED 2    /* quasi-residual below the inexact-inner term of
                                  eq. trueresidual; refinement decides the rest */
#define SHK_BREAKDOWN_EXACT 3  /* h_{k+1,k} = 0: exact solution (section 3)      */
#define SHK_NAN 4              /* non-finite input or arithmetic                  */

/* parameter values */
#define SHK_GMRES 0
#define SHK_FOM 1
#define SHK_CGS2 0
#define SHK_MGS 1
#define SHK_FP64 0   /* every vector complex128                                       */
#define SHK_MIXED 1  /* Arnoldi basis V and the inner solve's vectors stored in
                        complex64, the operator's products in FP32 arithmetic; the
                        inner iterate, the flexible basis Z and x in complex128;
                        every inner product and Gram-Schmidt projection formed from
                        exact FP64 products of the complex64 values and summed in
                        FP64 (SHK_RHS_BLOCK: the block projections V^H W and
                        W - V C on the matrix cores in FP32, the CholQR Gram in
                        FP64); Hessenberg least squares, basis norms, true
                        residual and refinement in FP64                             */
#define SHK_PTR_HOST 0
#define SHK_PTR_DEVICE 1
#define SHK_RHS_LOCKSTEP 0  /* one flexible basis per right-hand side, the bases
                               built in lockstep (the paper's choice, section 5)  */
#define SHK_RHS_BLOCK 1     /* one block basis shared by a group's right-hand
                               sides (block FGMRES-Sh)                           */
#define SHK_OUT_FULL 0      /* x: every x_{j,r} in full                                 */
#define SHK_OUT_ROWS 1      /* x: x_{j,r} at the cells out_rows only                    */
#define SHK_OUT_FACTORED 2  /* x: Z and y with x_{j,r} = Z_r y_{j,r} (see shk_params)  */
#define SHK_PRECOND_JACOBI 0     /* inner COCG with D = diag(K + tau M)              */
#define SHK_PRECOND_MULTIGRID 1  /* inner COCG preconditioned by a geometric
                                    aggregation multigrid V-cycle (structured
                                    finite-volume problems only)                  */

/*
 * Solver parameters (inputs of Algorithm 4 plus library knobs).
 *  m_restart      basis length m before a restart (section 2.2.2); >= 1.
 *  max_restarts   number of restarts allowed (0 = a single cycle).
 *  max_refine     FP64 refinement sweeps after the solve (0 = none).
 *  tol            target ||b - (K + sigma_j M) x_j|| / ||b|| per (shift, rhs)
 *                 (section 6.1 stopping rule, with x_0 = 0).
 *  eps_inner      inner tolerance eps: each preconditioner solve stops at
 *                 ||v_k - (K + tau_k M) z_k|| <= eps ||v_k|| (section 4).
 *  inner_maxit    cap on inner iterations per solve (0 = 20 * largest grid dim).
 *  n_tau, tau_seq tau_k used cyclically over the outer step counter (host
 *                 array of n_tau complex values; section 2.2.1 and the recycled
 *                 schedule of section 6.1).  A blocked schedule is expressed by
 *                 repeating entries.
 *  variant        SHK_GMRES: y_j minimises ||beta e_1 - Hbar(sigma_j;T) y||;
 *                 restarts keep the residuals collinear with the largest one
 *                 (section 2.2.2).  SHK_FOM: y_j solves the square system
 *                 H_m(sigma_j;T) y = beta e_1 (Algorithm 4, FOM); every
 *                 residual is a multiple of v_{m+1} (proof of Prop. 2), which
 *                 starts the next cycle.  A (shift, rhs) whose square system is
 *                 exactly singular at the end of a cycle stops NOT_CONVERGED
 *                 with its least-squares iterate.  Other values: INVALID_ARG.
 *  precision      SHK_FP64 or SHK_MIXED.
 *  refine_tol     relative accuracy asked of each refinement correction solve.
 *  refine_eps_inner  inner tolerance of the correction solves.
 *  inner_precond  preconditioner of the inner COCG: SHK_PRECOND_JACOBI, or
 *                 SHK_PRECOND_MULTIGRID (section 6 preconditions the paper's
 *                 inner solver with multigrid): cells grouped 2^d per level
 *                 down to one cell, coarse faces half the sum of the fine
 *                 faces they cover, coarse mass the sum, one V-cycle with
 *                 mg_sweeps damped Jacobi sweeps of weight mg_omega before and
 *                 after the coarse correction; a call error (UNSUPPORTED) for
 *                 CSR problems and for grids with ny or nz above 65535.
 *  mg_sweeps      1 (the only value provided; others are a call error).
 *  mg_omega       Jacobi damping of the smoother, in (0, 1].
 *  inner_relax    0: every inner solve asks for eps_inner.  > 0: relaxed inner
 *                 tolerance (the Simoncini-Szyld idea section 4 cites without
 *                 pursuing it): after each outer step the next inner solve asks
 *                 for min(inner_eps_max, max(eps, inner_relax * tol / q)), q the
 *                 largest relative quasi-residual of the (shift, rhs) pairs
 *                 still running; the stopping bound keeps using the measured
 *                 inner residuals.  0.1 keeps every shift CONVERGED on the
 *                 workloads here.
 *  inner_eps_max  cap of the relaxed inner tolerance, in [eps_inner, 1).
 *  ortho          orthogonalisation of each new basis vector (Algorithm 3):
 *                 SHK_CGS2 (default): classical Gram-Schmidt with one
 *                 reorthogonalisation, two passes over the basis;
 *                 SHK_MGS: the paper's modified Gram-Schmidt, one column at a
 *                 time (k + 1 sequential passes at step k).  Other values:
 *                 INVALID_ARG.
 *  rhs_mode       how the right-hand sides of a group (up to 64 per call group)
 *                 share the work.  SHK_RHS_LOCKSTEP (default): each has its
 *                 own flexible basis (Algorithms 3 and 4 per rhs); the bases
 *                 are built side by side so the operator is read once for all.
 *                 SHK_RHS_BLOCK: one block basis for the group (the block
 *                 extension for several right-hand sides the paper points to in
 *                 sections 5 and 7): B = V_1 beta; per step the S columns of V_k
 *                 get their inner solves, W = M Z_k is orthogonalised against
 *                 V_1..V_k by block CGS2 on the matrix cores and factored W =
 *                 V_{k+1} H_{k+1,k} (CholQR2, FP64 Gram); each (shift, rhs)
 *                 takes the least-squares solution of the block form of eq.
 *                 shiftedarnoldimod with the stopping rule of eq.
 *                 trueresidual (one inner residual per basis column).  The
 *                 group is padded to at least 16 columns.  No restarts: pairs
 *                 still running after m_restart block steps keep their
 *                 least-squares iterate and go to refinement.  Requires
 *                 variant SHK_GMRES and ortho SHK_CGS2 (else UNSUPPORTED) and
 *                 m_restart <= 100; workspace grows as n_shifts (m S)^2.
 *  output         what fgmres_sh_solve writes to x (section 2: the family of
 *                 solutions x_j, eq. multipleshifted, and its Krylov form x_j =
 *                 Z y_j of Algorithm 4).  The FP64 true residuals and the
 *                 refinement need every x_j, so the library forms them in its
 *                 workspace whatever is returned; the modes shrink the output
 *                 and its copy to the host, not the device working set.
 *    SHK_OUT_FULL      x: n x n_shifts x n_rhs, x[c + n (j + n_shifts r)].
 *    SHK_OUT_ROWS      x: n_out_rows x n_shifts x n_rhs, x[q + n_out_rows (j +
 *                      n_shifts r)] = x_{j,r} at cell out_rows[q] (host array of
 *                      n_out_rows cell indices in [0, n), repeats allowed).
 *    SHK_OUT_FACTORED  x holds Z (n x k_cap x n_rhs, Z[c + n (i + k_cap r)])
 *                      followed by Y (k_cap x n_shifts x n_rhs, Y[i + k_cap (j +
 *                      n_shifts r)]) with x_{j,r} = sum_i Z[:, i, r] Y[i, j, r]:
 *                      the flexible basis vectors z_i of every cycle and
 *                      refinement pass in the order they were built, and their
 *                      coefficients (zero for the cycles a pair did not use).
 *                      k_cap = m_restart (max_restarts + 1) (max_refine + 1);
 *                      columns past shk_status.basis_cols are zero.  Lockstep
 *                      bases only (UNSUPPORTED with SHK_RHS_BLOCK).
 *                 shk_output_elems gives the size of x for each mode.
 *  n_out_rows, out_rows  cells of SHK_OUT_ROWS (ignored otherwise).
 */
typedef struct {
  int m_restart;
  int max_restarts;
  int max_refine;
  int inner_maxit;
  double tol;
  double eps_inner;
  int n_tau;
  const shk_c128* tau_seq;
  int variant;
  int precision;
  double refine_tol;
  double refine_eps_inner;
  int inner_precond;
  int mg_sweeps;
  double mg_omega;
  double inner_relax;
  double inner_eps_max;
  int ortho;
  int rhs_mode;
  int output;
  int n_out_rows;
  const long long* out_rows;
} shk_params;

/* Per-(shift, rhs) result, host memory, n_shifts x n_rhs column-major. */
typedef struct {
  int status;          /* SHK_CONVERGED ...                                    */
  int outer_its;       /* outer steps taken when the shift was frozen          */
  int restarts;        /* restarts before it was frozen                        */
  int refine_sweeps;   /* refinement sweeps applied                            */
  int basis_cols;      /* basis vectors built for this rhs (all cycles and
                          refinement passes; the used columns of SHK_OUT_FACTORED) */
  int reserved;
  long long inner_its; /* inner iterations of the whole solve (shared)         */
  double quasi_relres; /* ||beta e_1 - Hbar(sigma;T) y|| / ||b|| at freeze      */
  double bound_relres; /* eq. trueresidual bound / ||b|| at freeze             */
  double true_relres;  /* FP64 ||b - (K + sigma M) x|| / ||b|| on return        */
} shk_status;

/* Fill *p with defaults: m 50, 20 restarts, 2 refinement sweeps, tol 1e-8,
 * eps 1e-10, GMRES, FP64, refine_tol 0.05, refine_eps_inner 5e-3, no tau,
 * Jacobi inner preconditioner (multigrid settings 1 sweep, omega 0.8). */
void shk_params_default(shk_params* p);

/*
 * Problem setup (section 5.1, eq. phasor1 discretised by cell-centred finite
 * volumes): face transmissivity T = 2 K_a K_b / (K_a + K_b) h^(d-2) (harmonic
 * mean), boundary faces T = K_cell h^(d-2) against a Dirichlet ghost value 0,
 * K_ii = sum of the cell's face T, K_ij = -T; lumped mass M = Ss h^d.
 *  cell_K  host, nx*ny (or nx*ny*nz) positive conductivities, x fastest.
 *  Ss, h   specific storage (> 0) and grid spacing (> 0).
 * The face arrays are computed on the device and owned by the problem, which
 * also keeps a complex64-path copy.  Errors: INVALID_ARG (sizes, non-positive
 * or non-finite K), OOM, HIP.
 */
int shk_problem_create_fv2d(int nx, int ny, const double* cell_K, double Ss, double h,
                            shk_problem** out);
int shk_problem_create_fv3d(int nx, int ny, int nz, const double* cell_K, double Ss, double h,
                            shk_problem** out);
/* General K given as CSR (host arrays, 0-based, n rows, K must be symmetric so
 * the inner COCG applies) and a diagonal mass (host, n entries). */
int shk_problem_create_csr(int n, const int* rowptr, const int* col, const double* K_val,
                           const double* M_diag, shk_problem** out);
void shk_problem_destroy(shk_problem* p);
/* Number of unknowns n of the problem. */
long long shk_problem_size(const shk_problem* p);

/* Number of complex128 elements fgmres_sh_solve writes to x for prm->output
 * (FULL: n n_shifts n_rhs; ROWS: n_out_rows n_shifts n_rhs; FACTORED: k_cap
 * (n + n_shifts) n_rhs) and, for FACTORED, k_cap (0 otherwise; k_cap may be
 * NULL).  Errors: INVALID_ARG. */
int shk_output_elems(const shk_problem* p, const shk_params* prm, int n_shifts, int n_rhs, size_t* elems,
                     int* k_cap);

/* Bytes of device workspace fgmres_sh_solve needs for these sizes. */
int shk_workspace_bytes(const shk_problem* p, const shk_params* prm, int n_shifts, int n_rhs,
                        size_t* bytes);

/*
 * Solve (K + sigma_j M) x_{j,r} = b_r for all shifts j and right-hand sides r
 * (Algorithms 3 and 4; independent flexible bases per rhs, run in lockstep so
 * the operator is read once for all of them).
 *  sigma      host, n_shifts complex shifts.
 *  b          n x n_rhs column-major complex128 (host or device per ptr_kind).
 *  x          complex128 output per prm->output (host or device per ptr_kind);
 *             SHK_OUT_FULL: n x n_shifts x n_rhs column-major, x[c + n*(j +
 *             n_shifts*r)]; the other modes as described with shk_params.
 *  st         host, n_shifts x n_rhs statuses, st[j + n_shifts*r].
 *  workspace  device buffer of >= shk_workspace_bytes(); NULL lets the library
 *             allocate and free it inside the call.
 * Errors: INVALID_ARG, UNSUPPORTED (multigrid on a CSR problem or an oversized
 * grid), WORKSPACE (too small), OOM, HIP.
 */
int fgmres_sh_solve(shk_problem* p, const shk_params* prm, int n_shifts, const shk_c128* sigma,
                    int n_rhs, const shk_c128* b, shk_c128* x, shk_status* st, void* workspace,
                    size_t ws_bytes, void* hip_stream, int ptr_kind);

/* ---------------------------------------------------------------------------
 * Step-level entry points: each runs one row of the method on device buffers
 * (all pointers device, vectors of n_rhs right-hand sides stored interleaved:
 * element (cell c, rhs r) at c*n_rhs + r; n_rhs a power of two <= 64).
 * precision selects complex128 (SHK_FP64) or complex64 (SHK_MIXED) vectors.
 * ------------------------------------------------------------------------ */

/* y = (K + sigma M) x (operator of eq. multipleshifted). */
int shk_apply_shifted(shk_problem* p, shk_c128 sigma, int n_rhs, const void* x, void* y,
                      int precision, void* hip_stream);

/* Inner preconditioner solve z ~ (K + tau M)^{-1} v (section 4, eq. zmmoditer):
 * COCG from z = 0 preconditioned by precond (SHK_PRECOND_JACOBI, or
 * SHK_PRECOND_MULTIGRID: the V-cycle of shk_params with one sweep, omega 0.8),
 * stopped when the residual satisfies
 * ||r|| <= eps ||v|| or after maxit iterations (0: 20 * largest grid dim);
 * fixed_iters > 0 runs exactly that many iterations instead.  v and w use the
 * vector precision; the iterate z is always complex128 (on the complex64 path
 * it accumulates in FP64 and the residual is recomputed in FP64 before the
 * solve is accepted).  Outputs (host, n_rhs each): its[r], true residual norm
 * pnorm[r] = ||v - (K + tau M) z|| (FP64).  Also writes w = M z in the vector
 * precision (device, may be NULL). */
int shk_inner_solve(shk_problem* p, shk_c128 tau, int n_rhs, const void* v, void* z, void* w,
                    double eps, int maxit, int fixed_iters, int precision, int precond, int* its,
                    double* pnorm, void* hip_stream);

/* One orthogonalisation step of Algorithm 3: V holds k orthonormal columns
 * (column stride n*n_rhs elements), w is orthogonalised against them in place
 * (ortho = SHK_CGS2: classical Gram-Schmidt with one reorthogonalisation;
 * SHK_MGS: modified Gram-Schmidt) and normalised into V column k.  h (host,
 * (k+1) x n_rhs, h[i + (k+1)*r]) receives the coefficients of v_i for i < k
 * and ||w|| at i = k (the new Hessenberg column).  Errors: INVALID_ARG. */
int shk_orthogonalize(long long n, int n_rhs, int k, void* V, void* w, shk_c128* h,
                      int precision, int ortho, void* hip_stream);

/* Per-shift projected problem of Algorithm 4: given Hbar ((k+1) x k, host,
 * column-major, one rhs), taus (host, k) and shifts (host, n_shifts), with
 * Hbar(sigma;T) = [I;0] + Hbar (sigma I - T) (eq. shiftedarnoldimod), on the
 * device with Givens rotations:
 *   variant SHK_GMRES: y = argmin ||beta e_1 - Hbar(sigma_j;T) y||;
 *   variant SHK_FOM:   y solves H_k(sigma_j;T) y = beta e_1 (the first k rows).
 * Outputs (host): y (k x n_shifts column-major) and quasi-residual norms
 * ||beta e_1 - Hbar(sigma_j;T) y|| after each step s = 0..k-1 at
 * rho[j + n_shifts*s] (FOM: |hbar_{s+1,s}(sigma_j)| |y_s|; +inf where the
 * square system of that step is exactly singular).  Errors: INVALID_ARG. */
int shk_shifted_lsq(int k, const shk_c128* Hbar, const shk_c128* taus, int n_shifts,
                    const shk_c128* sigma, double beta, shk_c128* y, double* rho, int variant);

/* One step of the shared block basis (block form of Algorithm 3): V holds k
 * blocks of n_rhs columns (device, n x n_rhs each, element (c, r) at c*n_rhs
 * + r, block stride n*n_rhs), orthonormal; W (device, one such block) is
 * orthogonalised against them by block classical Gram-Schmidt with one
 * reorthogonalisation (projections on the matrix cores, FP32 products summed
 * in FP64 for SHK_MIXED, FP64 for SHK_FP64) and factored W = V_{k+1} R
 * (CholQR twice, FP64 Gram matrices; R upper triangular with a real positive
 * diagonal; a dependent column gives a zero column of V_{k+1}), V_{k+1}
 * written as block k of V.  h (host, ((k+1) n_rhs) x n_rhs column-major)
 * receives the coefficients of V_1..V_k in rows 0..k n_rhs and R below.
 * n_rhs in {16, 32, 64}.  Overwrites W.  Errors: INVALID_ARG. */
int shk_block_orthogonalize(long long n, int n_rhs, int k, void* V, void* W, shk_c128* h, int precision,
                            void* hip_stream);

/* Per-shift block least squares of the shared block basis (FP64, on the
 * device): Hbar ((k+1) s x k s, host, column-major, s = n_rhs in {16, 32,
 * 64}), taus (host, k: block column i uses tau_i), beta (host, s x s
 * column-major, upper triangular: B = V_1 beta), shifts (host).  For every
 * shift j and column r, y minimises ||E_1 beta e_r - Hbar(sigma_j;T) y|| with
 * Hbar(sigma;T) = [I;0] + Hbar (sigma I - T), T = diag(tau_i I_s) (the block
 * form of eq. shiftedarnoldimod).  Outputs (host): y[row + k s (r + s j)]
 * (k s rows), and the projected residual norm after each block column i at
 * rho[r + s (j + n_shifts i)].  Errors: INVALID_ARG. */
int shk_block_shifted_lsq(int k, int n_rhs, const shk_c128* Hbar, const shk_c128* taus, int n_shifts,
                          const shk_c128* sigma, const shk_c128* beta, shk_c128* y, double* rho);

/* Solution assembly x_j = Z y_j (Algorithm 4): Z is k columns of n complex
 * values (column stride n, complex128 or complex64 per precision, device), Y
 * (device, k x n_shifts column-major complex128), X (device, n x n_shifts
 * column-major complex128); accumulate != 0 adds to X. */
int shk_assemble(long long n, int k, int n_shifts, const void* Z, const shk_c128* Y, shk_c128* X,
                 int accumulate, int precision, void* hip_stream);

/* FP64 true relative residuals ||b - (K + sigma_j M) x_j|| / ||b|| (device b:
 * n, device x: n x n_shifts column-major; host relres: n_shifts). */
int shk_true_residual(shk_problem* p, int n_shifts, const shk_c128* sigma, const shk_c128* b,
                      const shk_c128* x, double* relres, void* hip_stream);

/* The residuals of shk_true_residual computed without allocating device
 * memory, for callers that cannot allocate (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  Its scratch (shifts,
 * per-block partial sums, ||b||) lives in a fixed 9 MiB device array that the
 * library holds on each device it runs on until the process ends; the array's
 * device address is looked up on the first call on a device.  Same arguments,
 * layout and results as shk_true_residual (bitwise: same kernels, same
 * summation order).  Errors: INVALID_ARG as shk_true_residual; WORKSPACE when
 * n_shifts x (the residual kernel's block count, at most 256) x 16 bytes plus
 * small terms exceeds the array (about 2,280 shifts at n >= 65,536 cells:
 * split the shifts over calls).  Calls that overlap on one device share the
 * array and race; calls on different devices do not. */
int shk_true_residual_noalloc(shk_problem* p, int n_shifts, const shk_c128* sigma, const shk_c128* b,
                              const shk_c128* x, double* relres, void* hip_stream);

/* Sensitivities of point measurements to the log-conductivity field (section
 * 5, eq. sensitivity; step 3 of Algorithm 6), finite-volume problems only.
 * phi: forward solutions, device, n x n_shifts x n_src column-major complex128
 * (the layout fgmres_sh_solve writes), A_j phi_{j,s} = b_s; psi: adjoint
 * solutions, same layout with n_rec columns per shift, A_j psi_{j,r} = e_{m_r}
 * (unit source at the measurement cell; the paper's adjoint has source -delta,
 * i.e. it is -psi).  Writes, for every shift j, source s, receiver r and cell
 * c, J[c + n*(r + n_rec*(s + n_src*j))] = d h / d(ln K_c) with h = e_{m_r}^T
 * phi_{j,s}:  J = -sum over the faces f of c of (dT_f / d ln K_c)
 * (g_f^T psi)(g_f^T phi), g_f the face's difference operator (Dirichlet
 * ghost 0 at the boundary).  Real and imaginary parts are the paper's two
 * measurements per location and frequency.  J: device, complex128 for
 * SHK_FP64, complex64 for SHK_MIXED (computed in FP64, rounded once); the
 * caller owns all buffers.  Asynchronous on hip_stream.  UNSUPPORTED for CSR
 * problems; INVALID_ARG for null pointers, non-positive counts or more than
 * 65535 shifts. */
int shk_sensitivity(shk_problem* p, int n_shifts, int n_src, const shk_c128* phi, int n_rec, const shk_c128* psi,
                    void* J, int precision, void* hip_stream);

/* Instrumentation of the inner iteration (the hot loop of section 4's inner
 * solves).  When enabled, the solve stream carries HIP events and the library
 * accumulates, over the iterations that did work, their duration, their count
 * and their algorithmic bytes:
 *  - Jacobi inner solve: one kernel per iteration; events bracket each batch of
 *    launches between two host polls, and a batch counts when every launch in
 *    it iterated (bytes per cell: r, w, s read and written, p and the FP64
 *    iterate read and written, inverse diagonal and faces read);
 *  - multigrid inner solve: an event after every iteration (step, V-cycle and
 *    product launches); the count is iterations, the time runs from the end of
 *    a batch's first to the end of its last working iteration, and the bytes
 *    follow the byte model of one iteration (the step's vector updates, every
 *    V-cycle leg's operands and output, the tail's coefficients, the product).
 * launches: the count (kernel launches or iterations); total_ms: summed time;
 * total_bytes: summed algorithmic bytes.  Process-wide; enable/disable/read are
 * not meant to race with solves on other threads.
 * on: bit 0 this iteration instrumentation, bit 1 the phase timer
 * (shk_profile_read_phases); each call resets the totals. */
int shk_profile_enable(int on);
int shk_profile_read(long long* launches, double* total_ms, double* total_bytes);
/* With the instrumentation on, each block Gram-Schmidt of the shared block
 * basis (SHK_RHS_BLOCK: two projections V^H W and two updates W -= V C over
 * the k + 1 blocks of step k) is bracketed by HIP events on the solve stream:
 * calls, their summed time and their flops (4 x 8 n (k+1) s^2 real flops per
 * call, s the block width).  Reset by shk_profile_enable. */
int shk_profile_read_block(long long* calls, double* total_ms, double* total_flops);
/* Phase timer (shk_profile_enable bit 1): HIP events on the solve stream at the
 * boundaries of a solve's phases; the GPU time between two marks is charged to
 * the phase the later mark closes, so time the GPU spends waiting for the host
 * falls into the phase whose launches follow the wait.  ms[0..n-1] receives the
 * totals since the last enable, in this order: 0 start of a pass (norms, lane
 * set-up); 1 inner solves (set-up, iterations, the host's polls, finish); 2
 * Gram-Schmidt; 3 shifted least squares and the outer step's test (up to the
 * copy of the active counts); 4 turnaround (the host's wait on that copy and its
 * launch of the next phase: between outer steps, before the assembly and
 * around the true-residual checks); 5 assembly and restarts; 6 true residuals
 * and the refinement's residual; 7 whole block-basis passes (SHK_RHS_BLOCK is
 * timed as one phase).  For one solve at a time (lockstep or block path).
 * Returns the number of phases (8), or INVALID_ARG for a null ms. */
int shk_profile_read_phases(double* ms, int n);

/* ---------------------------------------------------------------------------
 * Tuning table.  Launch and round settings (block sizes, lanes per thread,
 * round tolerances, captured iterations, ...) are kept per workload class:
 * (kind, n, lanes, precision, inner_precond), kind 0 = 2D finite volume, 1 =
 * 3D finite volume, 2 = CSR; lanes = the power-of-two lane count of a group of
 * right-hand sides (at least 16 with SHK_RHS_BLOCK).  A solve reads its class's
 * entry once at its start; a class without an entry takes the shared settings,
 * which kind < 0 addresses (the other key fields are then ignored).  Settings
 * change the launch shapes and the inner solve's rounds only, never what the
 * method computes: a solve converges to the same tolerance under any of them.
 * The autotuner in the Python package fills the table from a measured search.
 * Knobs (value ranges are checked; an unknown name or a bad value returns
 * INVALID_ARG):
 *   cg_block 256|512        block size of the inner iteration kernels
 *   nt_store, nt_store32, nt_store64  0|1  streaming stores of the Jacobi step
 *   sep_limit >= 0          partial-sum count above which a kernel folds them
 *   ws_skew >= 0            bytes between the large workspace arrays
 *   round_tol, round_tol_mg (0,1)  reduction per complex64 inner round
 *                           (Jacobi / multigrid inner preconditioner)
 *   stall_min, stall_mult >= 0  a round ends after max(min, mult x its
 *                           productive length) iterations without halving
 *   tail_lds                LDS bytes of a workgroup of the V-cycle's tail
 *   tail_lanes 0|1|2|..|64  lanes per tail workgroup (default 1; 0: all in
 *                           one): the lanes are split over workgroups and the
 *                           tail starts at the finest level where the coarser
 *                           levels of that many lanes fit
 *   mg_fuse 0|1             step fused with the finest restriction
 *   post_lt, down_lt, up_lt 2|4|8  lanes per thread (complex64, several lanes)
 *   lt64 0|2|4              lanes per thread on complex128
 *   rows, rows64 >= 0       2-D levels of at least this many cells, several
 *                           lanes, complex64 / complex128: grid legs marching
 *                           the rows (0: none; defaults 0 and 16384)
 *   rows_yb 2..256, even    rows per block of those legs (default 4)
 *   graph 0|1               inner iterations replayed from a HIP graph captured
 *                           on the solve stream (needs a non-null stream)
 *   mg_chain 0|1            2-D, one lane: up to 3 middle legs of each direction
 *                           of the V-cycle in one launch
 *   asm_mfma 0|1            solution assembly X = Z Y on the FP64 matrix cores
 *   tile3_post 0|1          the product w = A u on the plane-marching tiles too
 *   post3_lt 2|4            complex64 lanes per thread of that product
 *   tile3 >= 0              3-D levels with at least this many cells run the
 *                           plane-marching V-cycle legs (0: none)
 *   tile3_zb 2..64, even    planes per block of those legs
 *   tile3_lt 2|4|8          complex64 lanes per thread of those legs
 * The table is process-wide and guarded by a lock; a solve in flight keeps the
 * settings it started with.
 */
int shk_tune_set(int kind, long long n, int lanes, int precision, int inner_precond, const char* knob,
                 double value);
int shk_tune_get(int kind, long long n, int lanes, int precision, int inner_precond, const char* knob,
                 double* value);
/* Removes every entry and restores the shared settings' defaults. */
int shk_tune_reset(void);
/* The class key of a solve of p with prm and n_rhs right-hand sides (the first
 * group of 64 when n_rhs > 64).  Errors: INVALID_ARG. */
int shk_tune_class(const shk_problem* p, const shk_params* prm, int n_rhs, int* kind, long long* n, int* lanes);

/* Text for a status or error code; last error message of the calling thread. */
const char* shk_status_string(int code);
const char* shk_last_error(void);

/* ---------------------------------------------------------------------------
 * Solve server: requests (field, shifts, right-hand sides) arrive at any time.
 * Every device byte a request needs (operator and multigrid hierarchy, Krylov
 * workspace, right-hand sides, its output) is one contiguous region of the
 * server's device arena.  Worker threads, one per slot and each with its own
 * HIP stream, take the oldest pending request for which a region is free
 * (first fit), so requests are admitted as slots and memory free up and run
 * concurrently with the ones already on the device; arrival, start and
 * completion times are recorded.  The server calls no device allocator per
 * request.  Only 2-D finite-volume requests are served.
 * ------------------------------------------------------------------------ */
typedef struct {
  int nx, ny;              /* 2-D finite-volume grid                             */
  const double* cell_K;    /* host, nx*ny, copied at submit                      */
  double Ss, h;
  int n_shifts;
  const shk_c128* sigma;   /* host, copied                                       */
  int n_rhs;
  const shk_c128* b;       /* host, n x n_rhs, copied                            */
  shk_params params;       /* tau_seq and out_rows copied; params.output selects
                              what the request returns (shk_params)              */
  int keep_solution;       /* 1: keep the output for shk_server_poll; 0: statuses
                              only                                               */
} shk_request;

typedef struct {
  int done;                /* 1 when finished                                    */
  int error;               /* call error of the solve (SHK_OK on success)        */
  double t_arrival, t_start, t_done;  /* seconds on the server clock           */
  int n_converged;         /* (shift, rhs) pairs with SHK_CONVERGED              */
  double max_true_relres;
} shk_result;

/* device_arena: a device buffer of mem_budget_bytes (256-byte aligned) that
 * the caller owns and keeps alive until shk_server_destroy returns, from which
 * every request's memory is taken; NULL makes the server allocate the arena
 * once here and free it at destroy.  max_slots (1..16) bounds the number of
 * concurrent requests (streams).  Errors: INVALID_ARG, OOM, HIP. */
int shk_server_create(size_t mem_budget_bytes, int max_slots, void* device_arena, shk_server** out);
/* Copies the request, returns a ticket.  REJECTED if its region can never fit
 * the arena; INVALID_ARG for bad sizes or out_rows. */
int shk_server_submit(shk_server* s, const shk_request* req, long long* ticket);
/* Non-blocking: NOT_READY until done; then fills *res.  With x != NULL (host,
 * shk_output_elems complex128 values for the request's output mode) and st !=
 * NULL (host, n_shifts x n_rhs) copies the output and statuses out. */
int shk_server_poll(shk_server* s, long long ticket, shk_result* res, shk_c128* x, shk_status* st);
/* Blocks until every submitted request is done. */
int shk_server_drain(shk_server* s);
/* Current server clock in seconds (the time base of shk_result). */
double shk_server_clock(shk_server* s);
int shk_server_destroy(shk_server* s);

#ifdef __cplusplus
}
#endif
#endif /* SHK_H */
