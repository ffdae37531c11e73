/*
 * taps.h -- C ABI of the TAPS slab-solve hot path on MI355X (gfx950).
 *
 * TAPS (Guo et al., tensor-decomposition-based a priori surrogate) solves the
 * Galerkin form of a space-parameter-time PDE in CP-decomposed form
 * u(x) = sum_m prod_d U_d[:, m]  (Sec. 2.2-2.3), one dimension at a time
 * (Sec. 2.6, Algorithm 1).  This library holds every data-parallel step of
 * that loop as HIP kernels:
 *
 *   taps_gauss_points / taps_shape1d     1D C-HiDeNN basis at points      (Sec. 2.1)
 *   taps_source1d                        separable source factors           (Sec. 2.4)
 *   taps_assemble1d                      1D quadrature matrices and loads  (Sec. 2.5)
 *   taps_load1d                          loads from shape values held by the caller
 *   taps_band_apply                      banded 1D matrix x factor columns
 *   taps_contract                        Grams, Hadamard couplings, force  (Sec. 2.5)
 *   taps_solve_dim                       block-banded (n_d M) dim solve    (Sec. 2.6)
 *   taps_residual / taps_balance         projected residual, mode balance  (Sec. 2.5-2.6)
 *   taps_sweep / taps_als                Algorithm 1 driver                (Sec. 2.6)
 *   taps_als_batched, taps_autotune      many problems at once, HIP graphs
 *   taps_interp1d / taps_reconstruct     TD interpolation on grids         (Sec. 2.3)
 *   taps_canonicalize, taps_mlp_*,       learned warm start of a slab's factors
 *   taps_adam_step
 *
 * Conventions (every call):
 *   - Pointers named d_* are device memory owned by the caller; everything else
 *     is host memory read during the call only.
 *   - Dense matrices are row-major.  Factors U_d are n_d x M, node-major
 *     (U[i*M + m]).  1D banded matrices are stored as n x (2w+1) with
 *     w = 2s+1 the half-bandwidth: band[i*(2w+1) + (j - i + w)] = A[i][j]
 *     (test index i first, trial index j second).
 *   - Work is enqueued on `stream` and is asynchronous to the host unless the
 *     description says otherwise.  Arguments are validated on the host before
 *     anything is enqueued: a bad argument returns TAPS_ERR_INVALID or
 *     TAPS_ERR_UNSUPPORTED and enqueues nothing; taps_last_error() tells why.
 *   - A handle owns a device workspace that grows on demand (hipMalloc after a
 *     stream synchronisation), and taps_als_batched a pinned host staging area
 *     (hipHostMalloc).  Call taps_reserve() up front to keep later
 *     single-problem calls allocation-free.  A handle is not thread-safe; use
 *     one per host thread.
 *   - Numerical breakdown (zero or NaN pivot) never aborts: it is reported in a
 *     device info word (LAPACK style) and the outputs are then unspecified.
 *   - Everything is FP64 except the precision argument of taps_reconstruct.
 */
#ifndef TAPS_H
#define TAPS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TAPS_OK = 0,
  TAPS_ERR_INVALID = -1,      /* bad argument (null pointer, size, range) */
  TAPS_ERR_UNSUPPORTED = -2,  /* valid but outside what the kernels handle */
  TAPS_ERR_ALLOC = -3,        /* device allocation failed */
  TAPS_ERR_HIP = -4           /* a HIP runtime call or launch failed */
} taps_status;

typedef struct taps_handle* taps_handle_t;

#define TAPS_MAX_DIMS 8
#define TAPS_MAX_TERMS 32
#define TAPS_MAX_KINDS 8
#define TAPS_MAX_M 64
#define TAPS_MAX_S 3
#define TAPS_MAX_GAUSS 8

/* Handle with an empty workspace.  Returns TAPS_ERR_INVALID for a null out-pointer. */
taps_status taps_create(taps_handle_t* out);
/* Frees the workspace (after synchronising the device).  Null is accepted. */
taps_status taps_destroy(taps_handle_t h);
/* Message of the last failed call on this handle ("" if none).  Owned by the handle. */
const char* taps_last_error(taps_handle_t h);
/* Grow the workspace to at least `bytes` now (synchronises the device). */
taps_status taps_reserve(taps_handle_t h, size_t bytes);
/* Bytes the workspace holds. */
size_t taps_workspace_bytes(taps_handle_t h);

/* ------------------------------------------------------------------------ */
/* 1D C-HiDeNN basis (Sec. 2.1, the C-HiDeNN interpolation equation).
 * Readings (the paper defers the patch function to its references):
 *   patch of node i = nodes max(0,i-s)..min(n-1,i+s); W^i_j = cardinal
 *   functions of radial-basis interpolation with degree-p polynomial
 *   reproduction on that patch, kernel = cubic B-spline of |x-x_j|/(a h_i),
 *   h_i = mean node spacing of the patch (for s = 0: of the adjacent elements),
 *   polynomial basis in (x-x_i)/h_i.  Ntilde_k = sum over the element's two
 *   nodes of (linear hat) * W.  A point on an interior node belongs to the
 *   element on its right, the last node to the last element.             */
typedef struct {
  int32_t n_nodes;     /* >= max(2, 2s+2) */
  const double* d_x;   /* device, n_nodes strictly increasing coordinates */
  int32_t s;           /* patch size, 0..TAPS_MAX_S */
  double a;            /* dilation, > 0 */
  int32_t p;           /* reproducing order, 0 <= p <= s (p = 0 allowed for s = 0) */
  int32_t n_gauss;     /* Gauss points per element, 1..TAPS_MAX_GAUSS */
} taps_basis1d_t;

/* Gauss-Legendre points and weights (Jacobian included) of every element,
 * element-major: point g of element e at e*n_gauss+g.  d_xg, d_wg hold
 * (n_nodes-1)*n_gauss doubles.  (Sec. 2.1: Gaussian integration.) */
taps_status taps_gauss_points(taps_handle_t h, const taps_basis1d_t* b,
                              double* d_xg, double* d_wg, hipStream_t stream);

/* Shape values and derivatives at n_pts points (Sec. 2.5, the 1D shape
 * functions Ntilde and their derivatives Btilde = dNtilde/dx).  Per point p:
 * d_first[p] = first node of the window of L = 2s+2 nodes
 * (clamped to [0, n-L]), d_N[p*L + l] = Ntilde_{first+l}(x_p), same for d_dN
 * (nullable).  Points outside [x_0, x_{n-1}] are clamped onto the end elements
 * (extrapolation). */
taps_status taps_shape1d(taps_handle_t h, const taps_basis1d_t* b, int32_t n_pts,
                         const double* d_pts, double* d_N, double* d_dN,
                         int32_t* d_first, hipStream_t stream);

/* Separable source factors evaluated at points (the forcing of Sec. 2.4 in
 * separated form).  d_out[c*n_pts + p] = f_c(x_p) for c < n_cols.
 *   TAPS_SRC_GAUSS:    params[0]*exp(-2 (x - d_centers[c])^2 / params[1]^2)
 *                      (moving Gaussian beam profile, radius params[1])
 *   TAPS_SRC_TOPLAYER: 1 if params[0] - x <= params[1] else 0 (top layer of
 *                      depth params[1] below the surface x = params[0])
 *   TAPS_SRC_POLY:     sum_q params[q] x^q, q < n_params (n_cols must be 1)
 *   TAPS_SRC_SIN:      params[0]*sin(params[1]*x)      (n_cols must be 1)
 *   TAPS_SRC_NODAL:    Ntilde_c(x) of `basis` (time interpolation of a
 *                      non-separable source; n_cols = basis->n_nodes)
 *   TAPS_SRC_EXPQUAD:  (p0 + p1 xi + p2 xi^2) exp(-beta xi^2 + lambda x)
 *                      + q0 + q1 x with xi = x - s, per column c from
 *                      d_centers[8c .. 8c+7] = {s, beta, lambda, p0, p1, p2,
 *                      q0, q1} (factors of closed-form test fields and
 *                      their sources: Gaussians and exponentials times
 *                      quadratics)
 * d_centers is used by GAUSS and EXPQUAD only; basis by NODAL only. */
typedef enum { TAPS_SRC_GAUSS = 0, TAPS_SRC_TOPLAYER = 1, TAPS_SRC_POLY = 2,
               TAPS_SRC_SIN = 3, TAPS_SRC_NODAL = 4, TAPS_SRC_EXPQUAD = 5 } taps_source_kind;
taps_status taps_source1d(taps_handle_t h, taps_source_kind kind, int32_t n_pts,
                          const double* d_pts, int32_t n_cols, int32_t n_params,
                          const double* params, const double* d_centers,
                          const taps_basis1d_t* basis, double* d_out, hipStream_t stream);

/* 1D matrices and load vectors by Gauss quadrature (Sec. 2.5, the 1D
 * integrals of the spatial, parametric and temporal terms; Appendix A, the
 * solution-dependent coefficients):
 *   TAPS_MASS   int Ntilde_i Ntilde_j        TAPS_STIFF int Btilde_i Btilde_j
 *   TAPS_DDT    int Ntilde_i Btilde_j        TAPS_WMASS int c(x) Ntilde_i Ntilde_j
 *   TAPS_BMASS  e_b e_b^T (boundary point mass of node bnode[k])
 *   TAPS_WSTIFF int c(x) Btilde_i Btilde_j
 *   TAPS_WDDT   int Ntilde_i d/dx (c(x) Ntilde_j) = int Ntilde_i (c' Ntilde_j + c Btilde_j)
 * d_band: n_kinds (<= 8) bands of n_nodes*(4s+3) doubles, in the order of kinds[].
 * d_coef_g: c at the Gauss points ((n_nodes-1)*n_gauss) for WMASS and WSTIFF;
 * for WDDT c followed by c' (2 (n_nodes-1) n_gauss).  The weighted kinds of
 * one call share d_coef_g.
 * Loads: d_F[i*n_loads + r] = int Ntilde_i f_r with f_r given at the Gauss
 * points as d_f_g[r*n_gpts + g] (n_gpts = (n_nodes-1)*n_gauss).
 * n_loads = 0 skips the loads. */
typedef enum { TAPS_MASS = 0, TAPS_STIFF = 1, TAPS_DDT = 2, TAPS_WMASS = 3,
               TAPS_BMASS = 4, TAPS_WSTIFF = 5, TAPS_WDDT = 6 } taps_kind;
taps_status taps_assemble1d(taps_handle_t h, const taps_basis1d_t* b, int32_t n_kinds,
                            const int32_t* kinds, const double* d_coef_g,
                            const int32_t* bnode, double* d_band, int32_t n_loads,
                            const double* d_f_g, double* d_F, hipStream_t stream);

/* The loads of taps_assemble1d from shape values the caller already holds,
 * for many load sets on one grid (the shape functions are then computed
 * once): d_N (n_gpts x (2s+2)) and d_first (n_gpts) are taps_shape1d at the
 * Gauss points of taps_gauss_points (whose weights are d_wg, n_gpts =
 * (n_nodes-1)*n_gauss); d_f_g and d_F as for taps_assemble1d:
 *   d_F[i*n_loads + r] = sum_g d_wg[g] Ntilde_i(x_g) d_f_g[r*n_gpts + g]
 * (Sec. 2.5, the forcing integrals).  Needs n_nodes >= max(2, 2s+2). */
taps_status taps_load1d(taps_handle_t h, int32_t n_nodes, int32_t s, int32_t n_gauss, const double* d_N,
                        const int32_t* d_first, const double* d_wg, int32_t n_loads, const double* d_f_g,
                        double* d_F, hipStream_t stream);

/* Banded 1D matrix times a block of columns (Sec. 2.5: the 1D matrices act on
 * factor columns; the slab chain builds its carried-field loads A_d V_d and the
 * mode-compression loads M_d W_d this way):
 *   d_Y[i*ldy + c] = alpha * scale[c] * sum_j A[i][j] d_X[j*ldx + c],
 * i < n, c < n_cols, A one band of taps_assemble1d (n x (4s+3), half-bandwidth
 * w = 2s+1), scale = d_scale (device, n_cols values) or all ones when NULL.
 * ldx, ldy >= n_cols; X and Y must not overlap.  TAPS_ERR_INVALID for null
 * pointers, n < 1, n_cols < 0, s outside 0..TAPS_MAX_S or short leading
 * dimensions; n_cols = 0 enqueues nothing. */
taps_status taps_band_apply(taps_handle_t h, int32_t n, int32_t s, const double* d_band,
                            int32_t n_cols, const double* d_X, int32_t ldx, const double* d_scale,
                            double alpha, double* d_Y, int32_t ldy, hipStream_t stream);

/* Inner product of two TD fields a = sum_m prod_d A_d[:, m] and
 * b = sum_m prod_d B_d[:, m] in the metric of one banded 1D matrix per dim
 * (the mass matrices give the L2 inner product of the interpolated fields,
 * Sec. 2.3): d_out[m*Mb + m'] = prod_d A_d[:, m]^T S_d B_d[:, m'] and
 * d_out[Ma*Mb] = the sum of those entries, (a, b).  A_d: n[d] x Ma, B_d:
 * n[d] x Mb row-major, S_d = d_band[d], one band of taps_assemble1d with
 * patch size s[d].  Used for the change of a field between iterations
 * (||a - b||^2 = (a,a) + (b,b) - 2 (a,b)).  d_out holds Ma*Mb + 1 doubles. */
taps_status taps_td_inner(taps_handle_t h, int32_t D, const int32_t* n, const int32_t* s,
                          const double* const* d_band, int32_t Ma, const double* const* d_A, int32_t Mb,
                          const double* const* d_B, double* d_out, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Separated problem (Sec. 2.5): operator sum_tau gamma_tau (x)_d A^{tau}_d
 * with A^{tau}_d = band number term_kind[tau][d] of dim d, and load
 * sum_r (x)_d F_d[:, col_d(r)].  Host struct, read during each call; the
 * device arrays it points to must stay valid while work using them runs.  */
typedef struct {
  int32_t D;                                  /* dims, 1..TAPS_MAX_DIMS */
  int32_t M;                                  /* modes, 1..TAPS_MAX_M */
  int32_t T;                                  /* operator terms, 1..TAPS_MAX_TERMS */
  int32_t R;                                  /* load terms, >= 1 */
  int32_t n[TAPS_MAX_DIMS];                   /* nodes per dim */
  int32_t s[TAPS_MAX_DIMS];                   /* patch size per dim (band half-width 2s+1) */
  int32_t n_kinds[TAPS_MAX_DIMS];             /* bands per dim, 1..TAPS_MAX_KINDS */
  int32_t term_kind[TAPS_MAX_TERMS][TAPS_MAX_DIMS];
  double gamma[TAPS_MAX_TERMS];
  const double* d_band[TAPS_MAX_DIMS];        /* n_kinds[d] * n[d] * (4s+3) */
  int32_t R_cols[TAPS_MAX_DIMS];              /* columns of F_d */
  const double* d_F[TAPS_MAX_DIMS];           /* n[d] * R_cols[d] */
  /* load-term -> column map of dim d (R entries) and its inverse grouped by
     column (CSR: d_load_ptr R_cols+1 entries, d_load_idx R entries).  All three
     NULL means the identity map (R_cols[d] must equal R). */
  const int32_t* d_load_col[TAPS_MAX_DIMS];
  const int32_t* d_load_ptr[TAPS_MAX_DIMS];
  const int32_t* d_load_idx[TAPS_MAX_DIMS];
  const uint8_t* d_fixed[TAPS_MAX_DIMS];      /* n[d] bytes, 1 = node held at 0; NULL = none */
} taps_problem_t;

/* Couplings and force of dim d (Sec. 2.5: the coefficient matrices of the
 * other dimensions multiplied entrywise, then the per-dim system).
 *   Gram   G^k_e[m][n] = U_e[:,m]^T A^k_e U_e[:,n]   (test mode m first)
 *   Lgram  L_e[c][m]   = F_e[:,c] . U_e[:,m]
 *   d_C[k*M*M + m*M + n] = sum_{tau: term_kind[tau][d] = k} gamma_tau
 *                           prod_{e != d} G^{term_kind[tau][e]}_e[m][n]
 *   d_Q[i*M + m] = sum_r F_d[i][col_d(r)] prod_{e != d} L_e[col_e(r)][m]
 * (all rows, fixed ones included).  Grams of dims whose bit is set in
 * stale_mask are recomputed from d_U and cached in the handle; the others are
 * taken from the cache, which belongs to the last problem contracted on the
 * handle (pass all bits after changing the problem). */
taps_status taps_contract(taps_handle_t h, const taps_problem_t* prob, int32_t d,
                          uint32_t stale_mask, const double* const* d_U,
                          double* d_C, double* d_Q, hipStream_t stream);

/* Backward-error limit above which a dim solve counts as a breakdown. */
#define TAPS_BERR_LIMIT 1e-8

/* Solve the dim-d system sum_k A^k_d X (C^k)^T = Q (Sec. 2.6, the linear
 * system in the subspace iteration; node-major (n_d M) block-banded matrix
 * with M x M blocks sum_k A^k_d[i][j] C^k and block half-bandwidth 2s+1).
 * Rows of fixed nodes are X = 0.  Block LU without pivoting (valid when the
 * symmetric part of the system is positive definite, which holds for the
 * heat and Poisson operators with at least one Dirichlet or initial-condition
 * row), pivot blocks inverted by Gauss-Jordan.  *d_info = 0 on success, or
 * 1 + the block row of the first zero / non-finite pivot.  Without pivoting
 * the factorisation is not backward stable when the couplings are
 * (near-)singular (more modes than the field's effective rank); d_berr
 * (nullable, one double) receives the relative backward error
 * ||sum_k A^k X C^k^T - Q||_F / ||Q||_F over free rows, computed after the
 * solve, so callers can detect that case (TAPS_BERR_LIMIT). */
taps_status taps_solve_dim(taps_handle_t h, const taps_problem_t* prob, int32_t d,
                           const double* d_C, const double* d_Q, double* d_X,
                           int32_t* d_info, double* d_berr, hipStream_t stream);

/* Projected Galerkin residual of every dim (the block-diagonal system of
 * Sec. 2.5; zero at a fixed point of Algorithm 1):
 *   R_d = sum_k A^k_d U_d (C^k_d)^T - Q_d on free rows, Grams from d_U.
 * d_out (D+2 doubles): [d] = ||R_d||_F^2, [D] = sum_d ||Q_d||_F^2 (free rows),
 * [D+1] = rho = sqrt(sum_d ||R_d||^2 / sum_d ||Q_d||^2).  Refreshes the cache. */
taps_status taps_residual(taps_handle_t h, const taps_problem_t* prob,
                          const double* const* d_U, double* d_out, hipStream_t stream);

/* Equalise the per-mode column norms across dims in place (the field is
 * unchanged): U_e[:,m] *= g_m / ||U_e[:,m]||, g_m = geometric mean over e;
 * skipped for a mode with any norm below 1e-300. */
taps_status taps_balance(taps_handle_t h, const taps_problem_t* prob,
                         double* const* d_U, hipStream_t stream);

/* One sweep of Algorithm 1 (Sec. 2.6): for d = 0..D-1 contract, solve into
 * d_U[d]; then balance.  d_info (nullable): one int32 (first failing block
 * row + 1, from the first dim that failed; 0 = ok).  d_berr (nullable): D
 * doubles, backward error of each dim solve. */
taps_status taps_sweep(taps_handle_t h, const taps_problem_t* prob, double* const* d_U,
                       int32_t* d_info, double* d_berr, hipStream_t stream);

/* Algorithm 1 to tolerance (Sec. 2.6).  Stops after the first sweep whose
 * projected residual rho <= tol, or -- the paper's own rule -- whose relative
 * change of all factors
 *   change = sqrt(sum_d ||U_d - U_d^prev||_F^2 / sum_d ||U_d||_F^2)
 * (balanced factors after the sweep against those at its start) is at or
 * below change_tol > 0 (0 disables that rule), or after iter_max sweeps.
 * Synchronises the stream once per sweep to read rho and the change.  Host
 * outputs: *sweeps, *rho (last), *change (last; nullable), history[k] = rho
 * and change_history[k] = change after sweep k (nullable, iter_max entries
 * each).  Returns TAPS_OK even if not converged (compare *rho with tol); a
 * breakdown in a dim solve (zero pivot, or backward error above
 * TAPS_BERR_LIMIT) ends the loop with *rho = *change = NaN and
 * taps_last_error() naming the dim.  The change is measured (a copy of the
 * factors, sum_d n_d M doubles of workspace, per sweep) only when change or
 * change_history is non-null or change_tol > 0. */
taps_status taps_als(taps_handle_t h, const taps_problem_t* prob, double* const* d_U,
                     double tol, double change_tol, int32_t iter_max, int32_t* sweeps, double* rho,
                     double* change, double* history, double* change_history, hipStream_t stream);

/* Algorithm 1 over a batch of B independent problems (slabs, parameter
 * queries) sharing D, M and the patch size of each dim; grid sizes, term
 * tables and loads may differ.  d_U holds B*D factor pointers,
 * problem-major (d_U[b*D + d]).  Each step of a sweep is one launch over
 * every active problem: Gram and load-Gram refreshes, couplings, forces, the
 * dim solves (the solver of taps_set_tuning: fast diagonalisation for dims
 * with two matrix kinds and M <= 64, block LU on the matrix cores otherwise;
 * one workgroup per system), backward errors, balancing with the relative
 * change, and the residual.  After each sweep (or each replay of a captured
 * graph of sweeps, taps_set_tuning) the host reads every problem's residual,
 * change and backward errors and drops the problems that reached tol or
 * change_tol (same rules as taps_als) or broke down.  Host outputs:
 * sweeps[b], rho[b] and change[b] (nullable) after the last sweep run, NaN
 * after a breakdown.  The change is measured (one copy of the factors per
 * sweep) only when change is non-null or change_tol > 0.  Synchronises the
 * stream once per sweep (or replay).  The per-call device records (problem
 * layout, coupling term tables, solve arguments, the active list and its
 * work-item prefix tables) are written into pinned host staging that the
 * handle keeps (hipHostMalloc, grown on demand) and sent in stream-ordered
 * copies; an event recorded behind the last copy guards the staging's reuse
 * by the next call.  probs is read during the call only.
 * TAPS_ERR_UNSUPPORTED when a block-LU dim does not fit LDS (M, s). */
taps_status taps_als_batched(taps_handle_t h, int32_t B, const taps_problem_t* probs,
                             double* const* d_U, double tol, double change_tol, int32_t iter_max,
                             int32_t* sweeps, double* rho, double* change, hipStream_t stream);

/* Tuning of the dim solves and of the batched driver.
 *
 * lgram_rows is the row split of the batched load-Gram kernel: each work
 * item contracts 64 load columns over lgram_rows rows (a multiple of 16,
 * 16..4096; 0 = 256), and the partials of the ceil(n/lgram_rows) splits are
 * summed afterwards -- fewer, longer items stream F with less partial
 * traffic, more, shorter ones spread a small problem over more workgroups.
 *
 * graph_sweeps = 0 launches every kernel of a sweep from the host; K > 0
 * captures K consecutive sweeps (every launch, no host work in between) into
 * one HIP graph, replays it, and checks the residuals after each replay, so a
 * slab that reaches tol mid-graph runs up to K-1 extra sweeps and sweeps[b]
 * counts in steps of K.  The graph is re-captured when the set of unconverged
 * slabs, the batch layout or the solver changes, and kept on the handle
 * otherwise (across calls).  Graphs are not used while kernel timing is
 * enabled.  Valid K: 0..16.
 *
 * solver selects how a dim system sum_k A^k X C^(k)T = Q (a Sylvester equation, Sec. 2.6) is
 * solved, in taps_solve_dim, taps_als and taps_als_batched alike:
 *   0  block LU over the block-banded operator (any number of kinds);
 *   1  fast diagonalisation / complex Schur (Sec. 2.6): for a dim with two kinds,
 *      E = C^(1)T C^(0)-T is brought to complex Schur form and its
 *      eigenvectors P, and the system decouples into M banded complex
 *      systems (A^0 + lambda_m A^1) y_m = (Q C^(0)-T P)_m, X = Re(Y P^-1).
 *      Needs M <= 64 (kernels laid out for M <= 48 and for M <= 64; above
 *      56 the complex Schur vectors of the last eigen kernel go through the
 *      workspace instead of LDS); dims with another number of kinds, or
 *      larger M, use the block LU.  Failure codes in the info word: -1 C^(0) singular,
 *      -2 the QR iteration did not converge (40 M iterations), k > 0 a zero
 *      pivot in row k-1 of a banded system.  Same backward-error check as
 *      the block LU.
 * Valid solver: 0, 1. */
typedef struct {
  int32_t graph_sweeps;
  int32_t solver;
  int32_t lgram_rows;   /* rows per partial of the batched load Gram (0 = 256) */
} taps_tuning_t;
taps_status taps_set_tuning(taps_handle_t h, const taps_tuning_t* t);
taps_status taps_get_tuning(taps_handle_t h, taps_tuning_t* t);

/* Timing autotuner of the batched driver (coordinate search).  First the
 * load-Gram row split lgram_rows in {128, 256, 512, 1024} with host launches
 * (the fastest is kept), then graph_sweeps in {0, 1, 2, 4} with that split
 * (the smallest K within 3 % of the fastest is kept); each candidate is
 * timed on this batch (4 sweeps after one untimed run that also captures the
 * graph; HIP events on `stream`).  The choice is applied to the handle and
 * returned in *chosen; ms_per_sweep (nullable, 8 doubles) receives the
 * measured times, row splits first.  The factors d_U are saved first and
 * restored before returning (device copies, allocated here).  With
 * cache_path non-NULL the choice is looked up in, or appended to, a JSON
 * file keyed by the batch shape (B, D, M, solver, s, and per dim the largest
 * n, R_cols and n_kinds); a key already there is applied without timing
 * (ms_per_sweep then all -1). */
taps_status taps_autotune(taps_handle_t h, int32_t B, const taps_problem_t* probs, double* const* d_U,
                          const char* cache_path, taps_tuning_t* chosen, double* ms_per_sweep,
                          hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Kernel timing.  While enabled, each launch of a timed kernel family is
 * bracketed by HIP events recorded on the stream it runs on, and the
 * family's algorithmic work per launch is added up on the host:
 *   TAPS_PROF_SOLVE    block LU of the dim system: flops = sum over block rows
 *                      of 2/3 M^3 + 2 wa M^3 + 2 wa^2 M^3 + (2 + 4 wa) M^2,
 *                      wa = min(w, n-1-k) (pivot factorisation, row panel,
 *                      trailing update, right-hand side, back substitution);
 *                      bytes = band + couplings + Q read, X written.
 *                      Fast diagonalisation (solver 1), its banded stage:
 *                      flops = 8 n M^2 (the two complex transforms) +
 *                      8 n M (w+1)(w+2) (elimination and back substitution);
 *                      bytes = what the method moves: bands and Q read, X
 *                      written, the two complex M x M transforms read (the
 *                      kernel's own scratch -- complex right-hand sides and
 *                      pivot-scaled U rows written and read back -- is not
 *                      counted).
 *   TAPS_PROF_EIG      fast diagonalisation, its eigen stage: flops = 44 M^3
 *                      per system (inverse 2, E 2, Schur form with Schur
 *                      vectors 25, triangular eigenvectors and their inverse
 *                      2 x 4/3, H3 4, Z Wv 4, H2 4, in units of M^3); bytes =
 *                      couplings read, transforms and inverse written.
 *   TAPS_PROF_SCHUR    the same stage's real Schur kernel alone (timed inside
 *                      the eigen-stage bracket): flops = 25 M^3 per system
 *                      (Hessenberg reduction and Francis QR with the Schur
 *                      vectors accumulated); bytes = 24 M^2 (E read, the
 *                      Schur form and its vectors written).
 *   TAPS_PROF_CONTRACT Grams, load Grams, couplings and force: flops of the
 *                      products; bytes = what the method moves: U read once
 *                      for all kinds of a dim and the Grams written, F and U
 *                      read and the load Grams written, F read and Q written
 *                      for the force (the banded 1D matrices are not counted:
 *                      they are Toeplitz inside a uniform grid; a load matrix
 *                      that several problems of one batched launch share is
 *                      counted once).
 *   TAPS_PROF_RECON    FP32/BF16 reconstruction on the matrix cores: flops =
 *                      2 n0 n1 n2 M (the method's modes; the matrix cores
 *                      execute M padded to their inner size), bytes = field
 *                      written (STORE) + factors read once.
 * taps_profile_enable(h, 1) clears the counters and starts recording,
 * (h, 0) stops; each call also launches one empty kernel (k_prof_mark) on
 * the null stream, so that a kernel trace or counter run of the process can
 * find the profiled region between the two dispatches.  taps_profile_read synchronises on the recorded events and
 * returns launches, summed kernel milliseconds, flops and bytes of one family. */
typedef enum {
  TAPS_PROF_SOLVE = 0,
  TAPS_PROF_CONTRACT = 1,
  TAPS_PROF_RECON = 2,
  TAPS_PROF_EIG = 3,
  TAPS_PROF_SCHUR = 4
} taps_prof_family;
taps_status taps_profile_enable(taps_handle_t h, int32_t enable);
taps_status taps_profile_read(taps_handle_t h, taps_prof_family family, int32_t* launches,
                              double* total_ms, double* flops, double* bytes);

/* ------------------------------------------------------------------------ */
/* TD interpolation (Sec. 2.3): Phi = Ntilde(pts) U with the shape window of
 * taps_shape1d (L values per point starting at d_first[p]):
 * d_Phi[p*M + m] = sum_l d_N[p*L + l] * d_U[(d_first[p]+l)*M + m]. */
taps_status taps_interp1d(taps_handle_t h, int32_t n_pts, int32_t L, const double* d_N,
                          const int32_t* d_first, int32_t n_nodes, int32_t M,
                          const double* d_U, double* d_Phi, hipStream_t stream);

/* Rank-M field on a 3D grid (Sec. 2.3, TD interpolation):
 *   u[i][j][k] = sum_m w_m Phi_0[i][m] Phi_1[j][m] Phi_2[k][m]
 * (w = d_mode_w or all ones; e.g. Phi_t(t*) folds the time factor in).
 * Precision: TAPS_FP64 (plain FP64), TAPS_FP32 (FP32 factors, FP32 MFMA
 * accumulate), TAPS_BF16 (BF16 factors, FP32 MFMA accumulate).
 * TAPS_STORE writes the field: d_out = n0*n1*n2 values (double for FP64,
 * float otherwise), plane-major: u[i][j][k] at d_out[(k*n0 + i)*n1 + j].
 * TAPS_REDUCE writes per z-plane k (n2 entries of 4 doubles):
 *   {max_ij u, sum_ij u^2, count_ij(u > thr), 0}. */
typedef enum { TAPS_FP64 = 0, TAPS_FP32 = 1, TAPS_BF16 = 2 } taps_prec;
typedef enum { TAPS_STORE = 0, TAPS_REDUCE = 1 } taps_recon_mode;
taps_status taps_reconstruct(taps_handle_t h, const int32_t* n_pts, const double* const* d_Phi,
                             int32_t M, const double* d_mode_w, taps_prec prec,
                             taps_recon_mode mode, void* d_out, double thr, hipStream_t stream);

/* B fields of one grid shape in one call (the same kernels as
 * taps_reconstruct, with a field index in the launch grid, so every field's
 * output is bit-identical to its own taps_reconstruct call).  d_Phi: 3*B
 * device pointers, field b's factors at d_Phi[3b .. 3b+2]; d_mode_w: B
 * pointers (entries may be null) or null; d_out: B outputs, each laid out as
 * for taps_reconstruct.  The pointer arrays are host arrays; FP32 and BF16
 * upload per-field tables to the handle workspace (one host-to-device copy),
 * FP64 runs the fields one after the other.  B <= 65535. */
taps_status taps_reconstruct_batched(taps_handle_t h, int32_t B, const int32_t* n_pts,
                                     const double* const* d_Phi, int32_t M, const double* const* d_mode_w,
                                     taps_prec prec, taps_recon_mode mode, void* const* d_out, double thr,
                                     hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * reconstruction as taps_reconstruct (same kernels, bit-identical outputs,
 * every precision and mode), with its scratch -- the staged reduced-precision
 * factors and the per-block partial records -- in a static device array of
 * TAPS_NOALLOC_SCRATCH_BYTES per GPU instead of the handle's workspace.  It
 * calls no allocation routine and times no kernel.  The array is looked up
 * by taps_create on the handle's GPU, which must be current; every call on a
 * GPU shares that GPU's array and overwrites it (nothing in it needs to
 * start at zero), so calls that overlap on one GPU -- on concurrent streams
 * or from several host threads -- race.  Sizes whose scratch exceeds the
 * array return TAPS_ERR_UNSUPPORTED before anything is enqueued: FP32/BF16
 * need 4 n0 Mp + (2 or 4) n1 Mp bytes (Mp = M padded to 32 for BF16, 16 for
 * FP32) plus 32 n2 ceil(n0/256) for REDUCE; FP64 REDUCE needs
 * 32 n2 ceil(n0/16) ceil(n1/16); FP64 STORE needs none. */
#define TAPS_NOALLOC_SCRATCH_BYTES (8u << 20)
taps_status taps_reconstruct_noalloc(taps_handle_t h, const int32_t* n_pts, const double* const* d_Phi,
                                     int32_t M, const double* d_mode_w, taps_prec prec, taps_recon_mode mode,
                                     void* d_out, double thr, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Learned warm start.  A slab's converged factors are stored in a canonical
 * form before a network learns them, and the network's coarse factors are
 * prolongated with taps_shape1d + taps_interp1d.
 *
 * Canonical form of a CP field u = sum_m prod_d U_d[:, m] (the field is
 * unchanged): modes ordered by lambda_m = prod_d ||U_d[:, m]||_2, largest
 * first (ties keep the lower index first); for d >= 1 every column scaled to
 * unit 2-norm with the sign that makes its largest-magnitude entry positive
 * (the first such entry on ties); scale and sign go into U_0.  A mode with a
 * zero column is left unscaled.  d_U[d] (n[d] x M) in, d_out[d] out (distinct
 * buffers).  One workgroup; D <= TAPS_MAX_DIMS, M <= TAPS_MAX_M. */
taps_status taps_canonicalize(taps_handle_t h, int32_t D, const int32_t* n, int32_t M,
                              const double* const* d_U, double* const* d_out, hipStream_t stream);

/* Multilayer perceptron x_{l+1} = GELU(W_l x_l + b_l), last layer linear,
 * GELU(z) = z Phi(z).  Weights are BF16 (bit patterns, uint16), row-major
 * width[l+1] x ldw(l) with ldw(l) = width[l] rounded up to a multiple of 32
 * and zero padding; biases FP32.  Each layer's input is rounded to BF16
 * (nearest, ties to even) and multiplied on the matrix cores with FP32
 * accumulation (v_mfma_f32_16x16x32_bf16); the gradients are FP32 (FP32
 * matrix-core products), the BF16 rounding passed through unchanged. */
#define TAPS_MLP_MAX_LAYERS 8
typedef struct {
  int32_t n_layers;                              /* 1..TAPS_MLP_MAX_LAYERS */
  int32_t width[TAPS_MLP_MAX_LAYERS + 1];        /* width[0] inputs .. width[L] outputs, <= 4096 */
  const uint16_t* d_W[TAPS_MLP_MAX_LAYERS];      /* BF16 weights (device) */
  const float* d_b[TAPS_MLP_MAX_LAYERS];         /* FP32 biases (device) */
} taps_mlp_t;
/* Bytes of the activation cache a forward pass leaves for the backward pass
 * with batch B.  Layout, layer by layer, each block starting on a 256-byte
 * boundary: the layer's BF16 input (B x ldw(l), zero padded), then its FP32
 * pre-activation z (B x width[l+1]). */
size_t taps_mlp_cache_bytes(const taps_mlp_t* net, int32_t B);
/* Forward: d_X (B x width[0], FP32, row-major) -> d_Y (B x width[L], FP32);
 * d_cache (taps_mlp_cache_bytes) receives what the backward pass needs. */
taps_status taps_mlp_forward(taps_handle_t h, const taps_mlp_t* net, int32_t B, const float* d_X,
                             void* d_cache, float* d_Y, hipStream_t stream);
/* Backward from dL/dY (B x width[L], FP32): d_gW[l] (width[l+1] x ldw(l),
 * FP32, padding written as 0) and d_gb[l] (width[l+1]) receive the gradients.
 * Uses the handle's workspace for the intermediate input gradients. */
taps_status taps_mlp_backward(taps_handle_t h, const taps_mlp_t* net, int32_t B, const void* d_cache,
                              const float* d_dY, float* const* d_gW, float* const* d_gb, hipStream_t stream);
/* Mean squared error over n entries: d_loss[0] = sum (Y-T)^2 / n (FP64),
 * d_dY = 2 (Y - T) / n (FP32). */
taps_status taps_mlp_mse(taps_handle_t h, int64_t n, const float* d_Y, const float* d_T, float* d_dY,
                         double* d_loss, hipStream_t stream);
/* One Adam step (bias-corrected, step number t >= 1) on n FP32 master values:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps);
 * d_p16 (nullable) receives the updated values rounded to BF16. */
taps_status taps_adam_step(taps_handle_t h, int64_t n, float* d_p, const float* d_g, float* d_m, float* d_v,
                           double lr, double b1, double b2, double eps, int32_t t, uint16_t* d_p16,
                           hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* TAPS_H */
