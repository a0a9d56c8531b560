/*
 * rte.h -- C ABI of the MI355X (gfx950) library for the rank-adaptive,
 * sweep-based SI-DSA of the steady first-order radiative transfer equation
 * (W. Guo, Z. Peng, arXiv 2603.25233).
 *
 * Problem (paper Sec. 2, eq. (rte)): mono-energetic, isotropic scattering,
 *     Omega . grad psi + sigma_t psi = sigma_s phi + G,  phi = (1/4pi) int psi,
 * on a rectangle [x0,x1] x [y0,y1] with isotropic inflow data g (vacuum: g = 0).
 * Discretisation (Sec. 2.1, Appendix A/B): discrete ordinates with normalised
 * weights (sum w_j = 1) and upwind DG-Q1 on a uniform nx x ny Cartesian mesh, giving
 * eq. (mat-vec-a):  (D_j + Sigma_t) psi_j = Sigma_s phi + G + g_j^bc.
 *
 * Conventions shared by every entry point
 *   - Cell (a, b) (a along x, b along y) has index c = b*nx + a; a scalar field is
 *     [ny][nx]; a DG field is [ny][nx][4] (ndof = 4*nx*ny).  The cell basis is
 *     orthonormal: eta_{pq} = l_p(x) l_q(y), l_0 = 1/sqrt(h), l_1 = sqrt(3) xi/sqrt(h)
 *     with xi in [-1,1] the cell-local coordinate, local index k = 2q + p.
 *   - Inflow data g: [4][max(nx,ny)][2] face moments g_m = int_face g l_m(s) ds on
 *     the sides L (x = x0), R (x = x1), B (y = y0), T (y = y1); s = y on L/R and
 *     s = x on B/T, l_1 increasing with s.  NULL means vacuum.
 *   - "HOST" pointers are read on the host during the call.  "DEV" pointers are
 *     device (HBM) pointers owned by the caller; the library never frees them.
 *   - `stream` is a hipStream_t (NULL = the null stream).  rte_sweep_execute is
 *     asynchronous on it; the other calls that take a stream return after their
 *     work on `stream` has finished (the solver takes its sampling and stopping
 *     decisions on the host).
 *   - Every call returns an rte_status; on error nothing is thrown or aborted and
 *     rte_last_error() gives a message (thread-local, valid until the next call
 *     from the same thread).
 *   - Workspace of the calls that take a stream comes from device memory the library
 *     keeps between calls (blocks of the same rounded size are reused; at most an
 *     eighth of the device's memory is kept; see rte_release_cached_memory).  Sweep
 *     plans hold their own hipMalloc'd workspace until rte_sweep_plan_destroy.
 *   - The library runs on the current HIP device.
 */
#ifndef RTE_H
#define RTE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RTE_OK = 0,
  RTE_ENOCONV = 1,       /* iteration cap reached: outputs hold the last iterate      */
  RTE_EINVAL = -1,       /* invalid argument (message says which)                     */
  RTE_ENOMEM = -2,       /* device or host allocation failed                          */
  RTE_EHIP = -3,         /* a HIP runtime call failed                                 */
  RTE_ERAND = -4         /* the caller's random stream ran out                        */
} rte_status;

typedef enum {
  RTE_FP64 = 0,          /* every step in float64                                     */
  RTE_MIXED = 1          /* rte_sweep: float32 throughout.  Solver: float32 basis X
                            (half the bytes of every pass over it), with float64
                            snapshots, projections accumulated in float64, reduced
                            solves, residuals, SVD, convergence tests and DSA; the
                            full-rank form sweeps the whole source in float64 until the
                            SI change is 1e-3 of the flux, then only the change of the
                            scattering source, in float32, added in float64          */
} rte_precision;

/* The discrete problem, eq. (mat-vec-a).                                           */
typedef struct {
  int32_t nx, ny;              /* cells along x, y (1 <= ny <= 1024 for the sweep)   */
  double x0, x1, y0, y1;       /* domain, x0 < x1, y0 < y1                            */
  int32_t n_dirs;              /* number of ordinates N_Omega                         */
  const double* dirs;          /* HOST [n_dirs][3] unit vectors Omega_j               */
  const double* wts;           /* HOST [n_dirs] weights, sum within 1e-12 of 1        */
  const double* sigma_t;       /* DEV [ny][nx] total cross section, in [1e-30, 1e30]  */
  const double* sigma_s;       /* DEV [ny][nx] scattering, 0 <= sigma_s <= sigma_t    */
  const double* G;             /* DEV [ny][nx][4] moments int_cell G eta_k, or NULL   */
  const double* bc;            /* DEV [4][max(nx,ny)][2] inflow face moments, or NULL */
} rte_problem;

/*
 * Transport sweep (paper Sec. 2.2, "Transport sweeps"; eqs. (SI), (sampled-sweep)).
 * For each selected ordinate j = dir_idx[i] solves
 *     (D_j + Sigma_t) psi_i = src + g_j^bc
 * exactly, by one pass over the cells in upwind order.
 *   dir_idx  HOST [n_sel] ordinate indices in [0, n_dirs)  (repeats allowed).
 *   src      DEV  [ny][nx][4] isotropic right-hand side (e.g. Sigma_s phi + G);
 *            float64, or float32 when prec == RTE_MIXED.
 *   psi      DEV  [n_sel][ny][nx][4] output (same type as src), or NULL.
 *   phi      DEV  [ny][nx][4] output (same type): overwritten with
 *            sum_i wts[dir_idx[i]] psi_i, or NULL.  At least one of psi, phi.
 * prob->G is not used (src is the whole isotropic right-hand side); prob->bc is.
 */
rte_status rte_sweep(const rte_problem* prob, const int32_t* dir_idx, int32_t n_sel,
                     const void* src, void* psi, void* phi, rte_precision prec,
                     void* stream);

/*
 * Allocation-free rte_sweep, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Arguments, results and errors as rte_sweep; the caller still owns src, psi and phi.
 * The workspace (direction table, anti-diagonal input copies, per-workgroup partial
 * sums of the scalar flux) comes from a 256 MiB static device array that each device
 * holds until the process ends, so the call makes no hipMalloc/hipFree.  A sweep whose
 * workspace exceeds 256 MiB returns RTE_EINVAL (roughly: psi only up to ~1.5M cells in
 * FP64; with phi, (number of workgroups + 2) * ndof * 8 bytes must fit).  All calls
 * on one device share the array: calls that overlap in time on one device (other
 * streams or host threads) race.  The call returns after its kernels have finished.
 */
rte_status rte_sweep_noalloc(const rte_problem* prob, const int32_t* dir_idx, int32_t n_sel,
                             const void* src, void* psi, void* phi, rte_precision prec,
                             void* stream);

/*
 * Adjoint sweep: solves (D_j + Sigma_t)^T mu_i = src + b_j for each j = dir_idx[i],
 * where b_j holds |Omega_j . n| int_face g eta_k on the OUTFLOW sides of Omega_j
 * (g = prob->bc): the right-hand side of the adjoint of an exit-current functional.
 * The transposed operator is taken in downwind order with transposed cell blocks
 * and couplings (D(Omega)^T = D(-Omega) for upwind DG).  Arguments as rte_sweep.
 */
rte_status rte_adjoint_sweep(const rte_problem* prob, const int32_t* dir_idx,
                             int32_t n_sel, const void* src, void* psi, void* phi,
                             rte_precision prec, void* stream);

/*
 * Persistent sweep plan for repeated sweeps of the same ordinate list (e.g. one SI
 * step per call): the direction tables and the workspace (anti-diagonal copies of
 * the source and cross section, per-group partial sums) are built and allocated
 * once, so rte_sweep_execute only enqueues the sweep's kernels: the input reordering,
 * the sweep and, when phi is requested, the fixed-order reduction of the per-group
 * partial sums.  The plan keeps one direction table per output combination (psi
 * only, phi only, both): large ordinate sets batch several ordinates of one quadrant
 * per workgroup, except when psi and phi are both written.
 *   rte_sweep_plan_create: arguments as rte_sweep (prob->dirs/wts/bc and the device
 *     pointers in prob are captured and must stay valid for the plan's lifetime);
 *     want_phi != 0 reserves the scalar-flux workspace; adjoint != 0 plans
 *     rte_adjoint_sweep semantics.  *plan receives an opaque handle.
 *   rte_sweep_execute: asynchronous on `stream`; src/psi/phi as in rte_sweep.
 *   rte_sweep_plan_destroy: frees the plan (synchronises the device).
 */
typedef struct rte_sweep_plan_s* rte_sweep_plan;
rte_status rte_sweep_plan_create(const rte_problem* prob, const int32_t* dir_idx,
                                 int32_t n_sel, rte_precision prec, int32_t want_phi,
                                 int32_t adjoint, rte_sweep_plan* plan);
rte_status rte_sweep_execute(rte_sweep_plan plan, const void* src, void* psi, void* phi,
                             void* stream);
rte_status rte_sweep_plan_destroy(rte_sweep_plan plan);

/*
 * Frees the device memory the library keeps for the workspace of later calls (not part
 * of the method: repeated solves reuse their buffers instead of paying hipMalloc /
 * hipFree every call).  Safe at any time no call of the library is running; always
 * returns RTE_OK.  A hipMalloc that runs out of memory inside a call empties the cache
 * by itself before it gives up.
 */
rte_status rte_release_cached_memory(void);

/* Solver settings (paper Sec. 2.2, Alg. 1, Sec. 3.2-3.4 and the settings of Sec. 4). */
typedef struct {
  int32_t full_rank;     /* 1: full-rank SI-DSA (every ordinate swept per outer step) */
  int32_t adjoint;       /* 1: solve the adjoint system with adjoint sweeps
                            (full_rank only); G must be NULL                          */
  int32_t use_dsa;       /* 1: apply the diffusion correction (default 1)            */
  int32_t p;             /* angles added per inner iteration (>= 1)                   */
  int32_t q;             /* random candidates per inner iteration (p <= q <= number of
                            ordinate classes; q >= the unsampled count makes every
                            unsampled class a candidate: fully greedy selection)      */
  int32_t m_max;         /* MGS2-A cleanup passes (Alg. 2), 4 in the paper            */
  int32_t max_outer;     /* cap on outer iterations                                   */
  int32_t max_rank;      /* cap on the basis size (0: number of distinct angles)      */
  double eps_si;         /* outer test ||phi^{n,*} - phi^{n-1}||_inf <= eps_si        */
  double eps_res;        /* inner residual threshold, eq. (residual-chk)              */
  double eps_diff;       /* inner phi-difference threshold, eq. (phi-diff)            */
  double eps_svd;        /* truncation tolerance (l1 tail of singular values)         */
  double eps_mgs;        /* MGS2-A orthogonality threshold                            */
  double eps_dsa;        /* relative residual of the DSA conjugate gradient           */
  rte_precision prec;
  const uint64_t* rand;  /* HOST random stream consumed by the sampling (low rank)     */
  int64_t n_rand;
  const int32_t* replay; /* HOST optional forced samples (angle classes): for each outer
                            iteration, groups "count, id, id, ..." (one per inner
                            iteration) followed by a 0; when an outer iteration's
                            groups run out the greedy choice is used; NULL = greedy    */
  int64_t n_replay;
  double* phi_checkpoints;  /* DEV [max_outer][ny][nx][4]: phi^{n,*} of every outer
                               iteration, or NULL                                     */
  int32_t fold_classes;  /* full rank: 1 sweeps one ordinate per class of equal
                            (Omega_x, Omega_y) with the class's summed weight (the
                            Omega_z twins of X-Y geometry have identical sweeps, so phi
                            is unchanged up to rounding); 0 sweeps every ordinate     */
  int32_t basis_update;  /* low rank: 0 MGS2-A (Alg. 2); 1 MGS-QR; 2 full QR (the
                            basis-update variants compared in Sec. 4.2)             */
  int32_t sampling;      /* low rank: 0 greedy random subsampling (Sec. 3.2); 1 DEIM
                            points of the angular basis V of C = U S V^T (the
                            alternative of the Remark in Sec. 3.2): the next p samples
                            are the first p unsampled DEIM points of the leading r'
                            columns of V (r' by the eps_svd rule), completed from the
                            candidates in residual order; the stopping test keeps the
                            q random candidates                                      */
} rte_solve_params;

/* What the solver reports (all HOST; optional arrays may be NULL).                    */
typedef struct {
  int32_t outer_iters;   /* SI steps taken, counting the last one                     */
  int32_t converged;
  int32_t rank;          /* r' after the single truncation of the last outer step    */
  int32_t n_swept;       /* angles swept over all outer iterations (low rank)         */
  int32_t mgs_failures;  /* Alg. 2 orthogonality failures                             */
  int32_t breakdowns;    /* snapshots already in span(X) (not appended)               */
  int32_t dsa_iters;     /* conjugate-gradient iterations over all DSA solves          */
  double* history;       /* [max_outer] ||phi^{n,*} - phi^{n-1}||_inf per outer step   */
  int32_t* ranks;        /* [max_outer] basis size r_k before truncation (low rank)    */
  int32_t* swept;        /* [max_outer] angles swept per outer step (low rank)         */
  int32_t* sample_log;   /* [sample_log_cap] angle classes in the order swept          */
  int32_t sample_log_cap, sample_log_len;
  double* resid_log;     /* [resid_log_cap] candidate residual norms in draw order     */
  int32_t resid_log_cap, resid_log_len;
  double ms_sweep, ms_lowrank, ms_dsa, ms_total;   /* phase wall times               */
  int32_t* trunc_ranks;  /* [max_outer] r' of the truncated SVD after each outer step
                            (low rank; NULL: truncate after the last step only)       */
  int32_t full_qrs;      /* full QR factorisations of the basis (basis_update 1, 2)  */
  int32_t fp64_sweeps;   /* full rank, RTE_MIXED: outer iterations that swept the whole
                            source in FP64 before the switch to FP32 increment sweeps */
} rte_solve_result;

/*
 * SI-DSA (paper Alg. 1).  full_rank = 1: the SI step sweeps all ordinates and
 * phi^{n,*} = sum_j w_j psi_j (Sec. 2.2).  full_rank = 0: the low-rank SI of
 * Sec. 3 (greedy random angle sampling, MGS2-A, incremental projected operators,
 * inner stopping test, one truncated SVD after the inner loop).  The outer test
 * is taken before the DSA step; the returned phi is phi^{n,*} of the last step.
 *   phi0     DEV [ny][nx][4] initial scalar flux, or NULL (zero).
 *   phi_out  DEV [ny][nx][4] result.
 *   X, S, V  DEV optional low-rank factors of the last outer step (Sec. 3.3):
 *            X [max_rank][ny*nx*4] (column i contiguous), S [max_rank],
 *            V [max_rank][n_dirs] (column i contiguous); res->rank columns are set.
 * Returns RTE_OK, RTE_ENOCONV (outputs hold the last iterate), or an error.
 */
rte_status rte_lowrank_si_dsa_solve(const rte_problem* prob, const rte_solve_params* params,
                                    const double* phi0, double* phi_out, double* X,
                                    double* S, double* V, rte_solve_result* res,
                                    void* stream);

/*
 * One backward Euler step of size dt of the time-dependent equation with unit speed,
 *   d psi/dt + Omega . grad psi + sigma_t psi = sigma_s phi + Q
 * (the implicit time marching outlined in Sec. 3.7): the steady problem with
 * sigma_t + 1/dt per cell and the angular source psi_j^m / dt (the mass matrix of the
 * orthonormal DG basis is the identity), solved by the full-rank SI-DSA (params->full_rank
 * = 1) or the low-rank SI-DSA of Sec. 3 (0), with the DSA on the step's cross sections.
 * FP64 only (params->prec = RTE_FP64), forward only; the other settings as for
 * rte_lowrank_si_dsa_solve.
 *   dt             > 0, finite.
 *   r_prev, X_prev, S_prev, V_prev
 *                  psi^m = X_prev diag(S_prev) V_prev^T, DEV X_prev [r_prev][ny*nx*4]
 *                  (column i contiguous), S_prev [r_prev], V_prev [r_prev][n_dirs] (the
 *                  layout of the X, S, V this call returns, so that steps chain);
 *                  r_prev = 0: psi^m = 0 (the pointers are not read).  V_prev must be
 *                  equal on ordinates of equal (Omega_x, Omega_y) (as every V returned
 *                  here is), else RTE_EINVAL.
 *   phi0           DEV initial scalar flux of the SI, or NULL (zero).
 *   phi_out        DEV [ny][nx][4] phi^{m+1}.
 *   X, S, V        DEV psi^{m+1} in the same factor form (required; X must not overlap
 *                  X_prev): low rank, the truncated factors of the last outer iteration
 *                  (res->rank columns); full rank, the psi of the last SI sweep per class
 *                  of equal (Omega_x, Omega_y) as K columns of X with S = 1 and V the class
 *                  indicator (res->rank = K; needs max_rank = 0 or >= K).
 * Returns RTE_OK, RTE_ENOCONV (outputs hold the last iterate), or an error.
 */
rte_status rte_backward_euler_step(const rte_problem* prob, const rte_solve_params* params,
                                   double dt, int32_t r_prev, const double* X_prev,
                                   const double* S_prev, const double* V_prev, const double* phi0,
                                   double* phi_out, double* X, double* S, double* V,
                                   rte_solve_result* res, void* stream);

/*
 * Exit partial currents of a converged scalar flux: regenerates psi_j by one sweep
 * of Sigma_s phi + G (+ inflow) and returns, for every boundary face e,
 *     J_e = sum_j w_j (Omega_j . n_e)^+ |e|^{-1} int_e psi_j ds.
 *   phi  DEV [ny][nx][4];  J  DEV [4][max(nx,ny)] (unused tail entries set to 0).
 */
rte_status rte_exit_currents(const rte_problem* prob, const double* phi, double* J,
                             void* stream);

/*
 * Boundary-detector misfit of exit currents (project addition, the functional whose
 * gradient rte_cross_section_gradient returns): L = 1/2 sum_e (J_e - J_obs,e)^2 over
 * every boundary face, and the adjoint boundary data it induces, an isotropic inflow
 * (J_e - J_obs,e) / |e| on face e, as face moments bc_adj[e] = ((J_e - J_obs,e) /
 * sqrt|e|, 0).
 *   J, J_obs DEV [4][max(nx,ny)] (tail entries ignored); bc_adj DEV [4][max(nx,ny)][2]
 *   (written; tail entries 0); loss HOST (written).  Synchronous on `stream`.
 */
rte_status rte_detector_misfit(const rte_problem* prob, const double* J, const double* J_obs,
                               double* bc_adj, double* loss, void* stream);

/*
 * Cross-section gradients by the discrete adjoint.  With psi_j regenerated from
 * the forward flux phi and mu_j from the adjoint flux phi_adj (adjoint sweeps with
 * boundary data bc_adj), per cell c:
 *     grad_sigma_a[c] = - sum_j w_j <mu_j, psi_j>_c
 *     grad_sigma_s[c] = grad_sigma_a[c] + <phi_adj, phi>_c.
 *   phi, phi_adj DEV [ny][nx][4]; bc_adj DEV [4][max(nx,ny)][2];
 *   grad_sigma_a, grad_sigma_s DEV [ny][nx].
 */
rte_status rte_cross_section_gradient(const rte_problem* prob, const double* phi,
                                      const double* phi_adj, const double* bc_adj,
                                      double* grad_sigma_a, double* grad_sigma_s,
                                      void* stream);

/* Chebyshev-Legendre rule CL(n_theta, n_z) (Appendix A): dirs HOST [n][3], wts HOST [n],
 * n = n_theta * n_z, index j = j2 * n_theta + j1 (j2 over ascending Omega_z).       */
rte_status rte_cl_quadrature(int32_t n_theta, int32_t n_z, double* dirs, double* wts);

/* Adds the moments of G = value on the box [bx0,bx1] x [by0,by1] to G_host
 * [ny][nx][4] (Appendix B, G(k) = int_cell G eta_k), integrated exactly.            */
rte_status rte_box_source_moments(int32_t nx, int32_t ny, double x0, double x1, double y0,
                                  double y1, double value, double bx0, double bx1,
                                  double by0, double by1, double* G_host);

/* Adds the face moments of a constant isotropic inflow g = value on boundary face
 * `index` of side `side` (0 L, 1 R, 2 B, 3 T; index along y on L/R, along x on B/T) to
 * bc_host [4][max(nx,ny)][2] (Appendix B, g_m = int_face g l_m ds): (value sqrt(h), 0)
 * for a face of length h.  Out-of-range side or index gives RTE_EINVAL.              */
rte_status rte_inflow_face_moments(int32_t nx, int32_t ny, double x0, double x1, double y0,
                                   double y1, int32_t side, int32_t index, double value,
                                   double* bc_host);

/* Adds the moments of the Gaussian source G = amp exp(-alpha ((x-cx)^2 + (y-cy)^2))
 * (the source of the examples of Sec. 4: amp = 1, alpha = 100, centre 0) to G_host
 * [ny][nx][4] (Appendix B, G(k) = int_cell G eta_k): the source is separable, so each
 * moment is a product of one-axis integrals, evaluated in closed form (error function).
 * alpha > 0; the mesh and the inputs must be finite.                                 */
rte_status rte_gaussian_source_moments(int32_t nx, int32_t ny, double x0, double x1, double y0,
                                       double y1, double amp, double alpha, double cx,
                                       double cy, double* G_host);

const char* rte_last_error(void);
int32_t rte_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RTE_H */
