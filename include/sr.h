/*
 * libsr: matrix-free stochastic reconfiguration (SR) and linear-method (LM) products on
 * AMD Instinct MI355X (gfx950).
 *
 * The method (Neuscamman, Umrigar and Chan, arXiv:1108.0900, Sec. II.A and II.B) never
 * forms the N_p x N_p overlap matrix.  It keeps the per-sample derivative ratios
 * O[k][i] = Psi^i_n / Psi_n (one row per sample, Eq. sr_overlap) and applies
 *     S v = (1/N_s) Oc^T (Oc v),   Oc = O - 1 obar^T,   obar = column mean of O
 * by interchanging the sums over samples and parameters (Eq. sr_multiply_2), inside a
 * conjugate-gradient solve of (S + eps I) x = g (Eq. sr_lin_eq in its centred form).
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers on the current HIP device, owned by the
 *    caller; the library never frees them.  Host pointers are marked "host".
 *  - Matrices are row-major: element (k, i) of O is at O + k*ld + i, with ld >= n_p.
 *    The allocation must span n_s*ld elements, O must be 16-byte aligned and
 *    ld * (element size) must be a multiple of 16 bytes (columns n_p..ld-1 are padding
 *    and are never used in the arithmetic).
 *  - Vectors of length n_p are float64 and contiguous.
 *  - Every call is asynchronous on `stream` unless stated otherwise, and runs its work
 *    in one or more kernels on that stream.  Calls that share a device and a stream
 *    share the library's workspace for that (device, stream) pair; calls that overlap
 *    in time on two different streams use two workspaces.
 *  - Return value: an sr_status code.  Negative codes are errors; no kernel has been
 *    launched when SR_ERR_INVALID is returned.  The thread-local text of the last error
 *    is available from sr_last_error().
 */
#ifndef SR_H
#define SR_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum sr_status {
  SR_OK = 0,
  SR_NOT_CONVERGED = 1,   /* CG reached max_iter; x holds the last iterate           */
  SR_BREAKDOWN = 2,       /* CG found p.(S+eps I)p <= 0; x holds the last iterate     */
  SR_ERR_INVALID = -1,    /* bad argument, detected on the host before any launch    */
  SR_ERR_NOMEM = -2,      /* workspace allocation failed                              */
  SR_ERR_HIP = -3,        /* a HIP runtime call failed (text in sr_last_error)        */
  SR_ERR_NONFINITE = -4,  /* CG met a NaN or infinity in a scalar                      */
  SR_ERR_NODEVICE = -5,   /* no HIP device, or the device is not gfx950              */
  SR_ERR_TIMEOUT = -6     /* a cross-workgroup wait exceeded its bound (kernel exited) */
};

/* Storage type of the derivative-ratio matrix. */
enum sr_dtype {
  SR_F64 = 0,    /* float64; arithmetic in float64                                   */
  SR_F32 = 1,    /* float32; arithmetic in float64                                   */
  SR_BF16 = 2,   /* bfloat16 codes q with float32 column scales s: O = s_j * q_kj;   */
                 /* products accumulate in float32, vectors and CG scalars float64    */
  SR_F16 = 3     /* float16 codes with float32 column scales, as SR_BF16             */
};

/* Non-owning view of a derivative-ratio matrix: the per-sample ratios of Eq. sr_overlap,
 * computed once per sample set and kept for every product (Sec. II.A, Eq. sr_multiply_2). */
typedef struct sr_matrix {
  int64_t n_s;               /* rows = samples, >= 1                                   */
  int64_t n_p;               /* columns = parameters, >= 1                             */
  int64_t ld;                /* row stride in elements, >= n_p                         */
  int32_t dtype;             /* enum sr_dtype                                          */
  int32_t reserved;          /* must be 0                                              */
  const void *O;             /* [n_s][ld] device                                       */
  const void *O_lo;          /* SR_BF16/SR_F16 only, optional: second code plane holding */
                             /* the quantisation remainder, so the stored value is       */
                             /* s_j*(q_kj + lo_kj).  Full plane (lo_cols NULL): [n_s][ld], */
                             /* same dtype and ld as O.  Compact plane (lo_cols given):   */
                             /* [n_s][ld_lo], column i holding the remainder of parameter */
                             /* lo_cols[i]; every other parameter is stored as s_j*q_kj.  */
                             /* NULL: single plane                                       */
  const float *col_scale;    /* [n_p] device; required for SR_BF16/SR_F16, else NULL   */
  const double *col_mean;    /* [n_p] device column means of the STORED values         */
                             /* (s_j*q_kj for scaled types); NULL: computed by the call */
  const int32_t *lo_cols;    /* [n_lo] device, strictly increasing parameter indices in  */
                             /* [0, n_p) (sr_remainder_columns writes such a list; other */
                             /* lists give wrong results but no out-of-bounds access), or */
                             /* NULL: O_lo, if given, is a full plane                    */
  int64_t n_lo;              /* columns of the compact plane (0 with lo_cols NULL)      */
  int64_t ld_lo;             /* row stride of the compact plane in elements, >= n_lo,   */
                             /* ld_lo * 2 a multiple of 16 bytes                         */
} sr_matrix;

/* Conjugate-gradient options (Sec. II.A: iterate until the requested accuracy). */
typedef struct sr_cg_opts {
  double rtol;               /* stop when ||r|| <= rtol ||g|| (recurrence residual,    */
                             /* confirmed by the true residual g - (S+eps I)x); > 0     */
  int32_t max_iter;          /* <= 0: n_p + 100                                        */
  int32_t refresh_every;     /* m > 0: every m-th iteration r <- g - (S+eps I)x; 0: never */
  int32_t use_x0;            /* 1: x holds the starting guess on entry; 0: start at 0  */
  int32_t restart_on_refresh;/* 1: also reset p <- r at each refresh (restarted CG);   */
                             /* 0: keep p (residual replacement)                       */
  double *res_history;       /* optional device [max_iter+1]: ||r||/||g|| per iteration */
  double refresh_drop;       /* in [0, 1): > 0 also refreshes as soon as ||r|| has      */
                             /* fallen below refresh_drop times its value at the last   */
                             /* refresh (or start); 0: periodic refreshes only          */
  int32_t precond;           /* 1: Jacobi preconditioner, z = r / (diag S + eps) (one  */
                             /* extra prepare pass computes diag S); SR_F64 / SR_F32    */
                             /* storage only; 0: none                                  */
  int32_t search_f64;        /* SR_BF16/SR_F16 with one plane or a compact plane: 1:   */
                             /* search-direction products accumulate in float64 too     */
                             /* (robust to tight rtol when eps is far below the spread */
                             /* of S); 0: float32.  Ignored for other storage           */
  int32_t reserved;          /* must be 0                                              */
} sr_cg_opts;

/* CG outcome, written to host memory. */
typedef struct sr_cg_info {
  int32_t iters;             /* CG iterations performed                                */
  int32_t refreshes;         /* true-residual replacements (periodic and at exit)      */
  int32_t status;            /* same value the call returns                            */
  int32_t products;          /* products with (S + eps I) performed                    */
  double rel_res_recur;      /* ||r||/||g|| of the recurrence residual at exit         */
  double rel_res_true;       /* ||g - (S+eps I)x|| / ||g|| at exit                      */
} sr_cg_info;

/* ------------------------------------------------------------------------------------
 * sr_grad: one pass over O (and E) giving the sampled quantities of the centred SR
 * system (Sec. II.A, Eq. sr_lin_eq with Psi^0 eliminated; Eq. sr_overlap for the means):
 *   E_mean       = (1/n_s) sum_k E_k                                   (device scalar)
 *   col_mean_i   = (1/n_s) sum_k O_ki                                  [n_p]
 *   diagS_i      = (1/n_s) sum_k (O_ki - col_mean_i)^2                 [n_p]
 *   g_i          = (2/n_s) sum_k (E_k - E_mean)(O_ki - col_mean_i)     [n_p]
 * E: [n_s] float64.  Any of E_mean, col_mean_out, diagS_out may be NULL.  g may be NULL
 * only if E is NULL too (then only the column statistics are produced).
 * The matrix's own col_mean field is ignored.
 * ------------------------------------------------------------------------------------ */
int sr_grad(const sr_matrix *O, const double *E, double *g, double *E_mean,
            double *col_mean_out, double *diagS_out, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * sr_sv_product: y = (S + eps I) v with S = (1/n_s) Oc^T Oc applied by interchanging the
 * sums over samples and parameters (Sec. II.A, Eq. sr_multiply_2): for each row,
 * w_k = Oc_k . v, then y = (1/n_s) sum_k w_k Oc_k + eps v.  O is read once.
 * v, y: [n_p] float64, must not overlap.  eps >= 0.  With a second code plane the
 * product is that of the two-plane values, accumulated in float64.
 * Asynchronous: if a cross-workgroup wait of the kernel gives up (SR_ERR_TIMEOUT in the
 * synchronous calls) y is filled with NaN.  The same holds for lm_hv_product.
 * ------------------------------------------------------------------------------------ */
int sr_sv_product(const sr_matrix *O, const double *v, double *y, double eps, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * sr_sv_product_noalloc: sr_sv_product for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * kernels and result; it calls no hipMalloc, hipFree or allocating routine.  Its scratch
 * (barrier flags, partial-dot exchange, row-group partials) is a 36 MiB array the library
 * holds on each device for the life of the process; a product that would need more returns
 * SR_ERR_INVALID (no built tile plans more than 33 MiB).  O->col_mean is required (the call
 * runs no prepare pass).  Calls that overlap in time on one device share that array and
 * race: serialize them (one stream, or events).
 * ------------------------------------------------------------------------------------ */
int sr_sv_product_noalloc(const sr_matrix *O, const double *v, double *y, double eps, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * sr_cg_solve: conjugate gradient on (S + eps I) x = g with S applied only through the
 * product above (Sec. II.A).  One stored plane without a preconditioner (bf16/f16
 * storage, or float64/float32 products of at least 2^31 bytes) runs split: one launch per
 * search iteration plus residual-phase launches; every other solve is one persistent launch.
 * g: [n_p] float64 right-hand side.  x: [n_p] float64 solution (starting guess on
 * entry if opt->use_x0).  opt: host, may be NULL (rtol 1e-10, defaults otherwise).
 * info: host, may be NULL.  eps >= 0; with eps = 0 and a singular S the result is the
 * minimum-norm solution when g lies in the range of S.
 * Residual refreshes and the exit check use products accumulated in float64 for every
 * storage type, so for bf16/f16 storage the iteration converges to the solution of the
 * stored (dequantized) system although its search-direction products accumulate in
 * float32 (mixed-precision residual replacement; opt->search_f64 makes them float64
 * too).  With a second code plane (O_lo, full or compact) the stored system is the
 * two-plane one and every product reads the remainder codes; a full plane's products
 * all accumulate in float64.  Float32 search products inject rounding errors of about
 * 1e-7 of the largest eigenvalue of S into every direction, including the null space of
 * S where the system is only eps: with N_s < N_p and eps far below the spread of S,
 * tolerances much below 1e-6 need search_f64.
 * Below the accuracy float64 arithmetic can attain (about kappa * 1e-16) the iteration
 * drifts; a refresh or exit check whose true residual exceeds 1000 times the best one seen
 * ends the solve with SR_NOT_CONVERGED (x is that iterate) instead of letting it grow.
 * This call synchronizes `stream` before returning (it reads the outcome back).
 * Returns SR_OK, SR_NOT_CONVERGED, SR_BREAKDOWN or an error code.
 * ------------------------------------------------------------------------------------ */
int sr_cg_solve(const sr_matrix *O, const double *g, double eps, double *x,
                const sr_cg_opts *opt, sr_cg_info *info, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * sr_cg_solve_async: sr_cg_solve without waiting for the solve: the outcome goes to device
 * memory, info_dev [16] float64: iters, refreshes, status (an sr_status value), products,
 * rel_res_recur, rel_res_true, then words the kernel uses for itself.  The whole solve is
 * one persistent launch (for bf16/f16 storage with float32 search products that kernel
 * holds both product codes and runs slower than the split solve sr_cg_solve uses).  Only a
 * workspace that has to grow synchronizes `stream` (sr_workspace_reserve avoids it).
 * Returns SR_OK once the work is queued, or an error detected before any launch.
 * ------------------------------------------------------------------------------------ */
int sr_cg_solve_async(const sr_matrix *O, const double *g, double eps, double *x,
                      const sr_cg_opts *opt, double *info_dev, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * lm_hv_product: the linear method's Hamiltonian product in the basis
 * {Psi, Psi^i - obar_i Psi} (Sec. II.B, Eq. linear_eigen), estimated from local energies
 * E and their parameter derivatives D (D_kj = d E_L / d alpha_j on sample k):
 *   t_k = Oc_k . v[1:],  u_k = D_k . v[1:],  z_k = E_k (v_0 + t_k) + u_k
 *   y_0 = E_mean v_0 + (1/n_s) sum_k (E_k t_k + u_k)
 *   y_i = (1/n_s) sum_k Oc_ki z_k                                       (i >= 1)
 * O and D: same n_s, n_p and dtype (their ld and scales may differ), single code plane
 * (O_lo = NULL).  E: [n_s] float64.
 * v, y: [n_p + 1] float64, must not overlap.  The companion overlap is 1 (+) S.
 * ------------------------------------------------------------------------------------ */
int lm_hv_product(const sr_matrix *O, const double *E, const sr_matrix *D,
                  const double *v, double *y, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Several right-hand sides and batches of systems (the batched form; the paper solves
 * one system at a time).  Up to SR_BATCH_MAX_RHS columns share each product:
 *   Y = (S + diag(eps)) V,  i.e. W = Oc V, Y = (1/n_s) Oc^T W + V diag(eps),
 * computed in two passes over O (the row dots W by row blocks, then Oc^T W by column
 * blocks), every sum accumulated in float64.
 * sr_svk_product: V, Y: device [k][n_p] float64 (column i at V + i n_p), must not
 * overlap; eps: host [k].  exact must be 0 or 1; both accumulate in float64 (the flag
 * is kept so that a faster inexact product can be added behind it).  Storage SR_F64 or
 * SR_F32, one code plane.  Synchronizes `stream` (its launch descriptor is copied from
 * host memory).
 * sr_cg_solve_batched: n_sys independent systems (each its own O, k right-hand sides g
 * and shifts eps), all solved in one persistent launch, system after system; within a
 * system the k CG iterations share each product.  Each column stops when its true
 * residual reaches opt->rtol (checked with a product from x whenever its recurrence
 * residual gets there, every opt->refresh_every iterations, once it fell by
 * opt->refresh_drop since the last check if refresh_drop > 0, and at max_iter).
 * sys: host [n_sys]; every O has the same dtype (SR_F64 or SR_F32).  info: host
 * [n_sys * k] (system-major) or NULL; its `refreshes` is 0 and rel_res_recur repeats
 * rel_res_true.  opt->use_x0, restart_on_refresh, precond, search_f64 and res_history are
 * not used.
 * Synchronizes `stream`.  Returns SR_OK if every column converged, else
 * SR_NOT_CONVERGED / SR_BREAKDOWN (the first such status met) or an error code.
 * ------------------------------------------------------------------------------------ */
#define SR_BATCH_MAX_RHS 8
typedef struct sr_batch_system {
  sr_matrix O;               /* the system's matrix; col_mean may be NULL (computed)    */
  const double *g;           /* device [k][n_p] right-hand sides                        */
  double *x;                 /* device [k][n_p] solutions                               */
  double eps[SR_BATCH_MAX_RHS]; /* shift of each right-hand side, >= 0                 */
} sr_batch_system;

int sr_svk_product(const sr_matrix *O, int32_t k, const double *V, const double *eps, double *Y, int32_t exact,
                   hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * sr_cg_solve_shifts: (S + eps_i I) x_i = g for up to SR_BATCH_MAX_RHS shifts eps_i and
 * one right-hand side g, by multi-shift CG (not in the paper): Krylov spaces do not
 * depend on the shift, so one CG sequence of the smallest shift, one fused product per
 * iteration, serves every shift through scalar recurrences (x_i and its direction are
 * the only per-shift vectors).  A shift stops once its recurrence residual reaches
 * opt->rtol; afterwards every shift's true residual is computed with a float64 product,
 * and a shift that missed rtol continues with sr_cg_solve from its x_i (warm start,
 * refresh_every of opt, 20 if 0).  Storage SR_F64 or SR_F32, one code plane.
 * g: device [n_p]; eps: host [k], finite, >= 0, any order; X: device [k][n_p] (row i for
 * eps_i), must not overlap g.  info: host [k] or NULL (iters and products include the
 * shared sequence, the residual check and any continuation).  opt->use_x0, search_f64,
 * precond and res_history are not used.  Synchronizes `stream`.  Returns SR_OK if every
 * shift converged, else the first non-OK status or an error code.
 * ------------------------------------------------------------------------------------ */
int sr_cg_solve_shifts(const sr_matrix *O, const double *g, int32_t k, const double *eps, double *X,
                       const sr_cg_opts *opt, sr_cg_info *info, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * sr_cg_solve_shifts_batched: n_sys independent systems, each with one right-hand side g
 * and k shifts, all by multi-shift CG in one persistent launch, system after system (one
 * fused single-vector product per iteration per system; each system's true residuals
 * checked with one float64 product per shift inside the launch).  Per system as
 * sr_cg_solve_shifts (a shift that missed rtol continues with sr_cg_solve afterwards).
 * sys: host [n_sys]; every O has the same dtype (SR_F64 or SR_F32, one plane).  info:
 * host [n_sys * k] (system-major) or NULL.  Synchronizes `stream`.
 * ------------------------------------------------------------------------------------ */
typedef struct sr_shift_system {
  sr_matrix O;               /* the system's matrix; col_mean may be NULL (computed)    */
  const double *g;           /* device [n_p] right-hand side                            */
  double *X;                 /* device [k][n_p] solutions, row i for eps[i]             */
  double eps[SR_BATCH_MAX_RHS]; /* shifts, finite and >= 0, any order                   */
} sr_shift_system;
int sr_cg_solve_shifts_batched(int32_t n_sys, const sr_shift_system *sys, int32_t k, const sr_cg_opts *opt,
                               sr_cg_info *info, hipStream_t stream);
int sr_cg_solve_batched(int32_t n_sys, const sr_batch_system *sys, int32_t k, const sr_cg_opts *opt,
                        sr_cg_info *info, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * sr_adjoint: gradients of a loss L(x) through the SR solve x = (S + eps I)^{-1} g with
 * S and g the sampled quantities of sr_grad (Sec. II.A, Eq. sr_overlap and the right-hand
 * side of Eq. sr_lin_eq), given x and lambda = (S + eps I)^{-1} dL/dx (a second
 * sr_cg_solve).  One read of O gives p1 = Oc x and p2 = Oc lambda; then
 *   dE_k      = (2/n_s) p2_k                                              [n_s]
 *   dO_kj     = (1/n_s) [ (2 (E_k - E_mean) - p1_k) lambda_j - p2_k x_j ]   [n_s][ld_dO]
 *   deps      = -lambda . x                                               (device scalar)
 * (dL/dg = lambda needs no kernel).  The derivative is taken
 * with respect to the stored values of O (s_j q_kj for scaled storage), the column means
 * depending on O included.
 * O: single code plane (O_lo = NULL); col_mean may be NULL (computed).  E, x, lam:
 * device float64 [n_s], [n_p], [n_p].  dE: device [n_s] float64 or NULL.  deps: device
 * float64 scalar or NULL (with dE, dO and p12 all NULL only deps is computed, without a
 * pass over O).  dO: device,
 * dO_dtype SR_F64 or SR_F32, row stride ld_dO >= n_p elements with 16-byte aligned rows,
 * or NULL (columns >= n_p are not written).  p12: device [2 n_s] float64 (p1 then p2) or
 * NULL.  Outputs must not overlap the inputs.  Asynchronous on `stream`.
 * ------------------------------------------------------------------------------------ */
int sr_adjoint(const sr_matrix *O, const double *E, const double *x, const double *lam, double *dE,
               void *dO, int32_t dO_dtype, int64_t ld_dO, double *p12, double *deps, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * lm_davidson: lowest eigenpair of the linear method's generalized eigenproblem
 * H c = theta S c (Sec. II.B, Eq. linear_eigen; the paper solves it with a generalized
 * Davidson method on H.x and S.x products), with H the sampled matrix of lm_hv_product and
 * S = 1 (+) S_c (the overlap in the basis {Psi, Psi^i - <O_i> Psi}).  Each iteration takes
 * one H product (lm_hv_product, one read of O and D) and one S product (sr_sv_product,
 * one read of O); the subspace basis is S-orthonormal (classical Gram-Schmidt, twice),
 * the projected matrix is solved on the host (Hessenberg QR), the new direction is the
 * Ritz residual r = H c - theta S c, and the subspace restarts from the Ritz vector when
 * it reaches opt->max_sub vectors.  With opt->precond the new direction is Davidson's
 * diagonal correction (diag H - theta diag S)^{-1} r: precond = 2 with the sampled
 * diag H (H_00 = <E>, H_jj = <Oc_j E Oc_j> + <Oc_j D_j>; one extra pass over O and D and
 * one prepare pass over O), precond = 1 with diag H approximated by <E> diag S, i.e. r_0
 * and r_i / S_ii (one prepare pass).  Near-zero denominators are kept at 1e-8 of their
 * terms' size.  The start vector is Psi itself, c = (1, 0, ..., 0).
 * O, D, E: as lm_hv_product (same n_s, n_p, dtype; single code plane).  c: device
 * [n_p + 1] float64, receives the Ritz vector (S-normalized, c^T S c = 1).  info: host,
 * required.  opt: NULL for the defaults (tol 1e-8, max_iter 1000, max_sub 40, precond 0); converged
 * when ||H c - theta S c|| <= tol |theta|.  Needs S positive definite on the explored
 * subspace (a direction of S-norm <= 1e-28 relative ends the iteration).  Synchronizes
 * `stream`.  Returns SR_OK when converged, SR_NOT_CONVERGED otherwise (c then holds the
 * last Ritz vector), SR_BREAKDOWN if the projected eigenproblem's QR iteration did not
 * converge, or an error code.
 * ------------------------------------------------------------------------------------ */
typedef struct lm_davidson_opts {
  double tol;                /* > 0 */
  int32_t max_iter;          /* H products, >= 1 */
  int32_t max_sub;           /* subspace size before a restart, in [2, 64] */
  int32_t precond;           /* 0: the residual; 1: approximate, 2: exact diagonal correction */
  int32_t reserved;          /* 0 */
} lm_davidson_opts;
typedef struct lm_davidson_info {
  int32_t iters;             /* iterations (each one H and one S product) */
  int32_t restarts;
  int32_t status;
  int32_t reserved;
  double theta;              /* Ritz value */
  double res_norm;           /* ||H c - theta S c|| */
} lm_davidson_info;
int lm_davidson(const sr_matrix *O, const double *E, const sr_matrix *D, const lm_davidson_opts *opt,
                double *c, lm_davidson_info *info, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * sr_quantize: storage conversion of a float64 or float32 matrix to SR_BF16 or SR_F16
 * codes with per-column float32 scales (not in the paper; the precision form):
 *   s_j = float32(max_k |O_kj|)  (1 for an all-zero column)
 *   q_kj = round-to-nearest-even of O_kj / s_j (the quotient taken in float64).
 * in: [n_s][ld_in] of in_dtype (SR_F64 or SR_F32).  q: [n_s][ld_out] of out_dtype
 * (columns n_p..ld_out-1 are set to zero).  scale: [n_p] float32.
 * q_lo: NULL, or [n_s][ld_out] of out_dtype receiving the second plane, the nearest code
 * of the remainder O_kj/s_j - q_kj (in float64).
 * Same alignment rules as sr_matrix for both matrices.
 * ------------------------------------------------------------------------------------ */
int sr_quantize(int64_t n_s, int64_t n_p, const void *in, int64_t ld_in, int32_t in_dtype,
                void *q, void *q_lo, int64_t ld_out, int32_t out_dtype, float *scale, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Compact remainder plane (the precision form, not in the paper): a second code only for
 * the columns whose single-plane codes are not accurate enough.
 * sr_remainder_columns: with `scale` the column scales sr_quantize wrote for `in`, selects
 * the columns j with  max_k |O_kj / s_j - q_kj| > tol  (quotient and difference in
 * float64, q_kj the out_dtype code of O_kj / s_j) and writes them in increasing order to
 * lo_cols (device [n_p]); their number goes to *n_lo (host).  A tol equal to the two-plane
 * error bound (bf16: 2^-17, f16: 2^-21) selects exactly the columns a second plane
 * improves; the stored values then meet that bound everywhere.  Synchronizes `stream`.
 * sr_quantize_remainder: writes the compact plane q_lo (device [n_s][ld_lo], ld_lo >= n_lo,
 * ld_lo * 2 a multiple of 16 bytes, padding columns set to zero): q_lo_ki = the nearest code
 * of O_kj / s_j - q_kj with j = lo_cols[i] (as the second plane of sr_quantize).
 * Same input rules as sr_quantize.  Pass the plane with lo_cols, n_lo, ld_lo in sr_matrix.
 * ------------------------------------------------------------------------------------ */
int sr_remainder_columns(int64_t n_s, int64_t n_p, const void *in, int64_t ld_in, int32_t in_dtype,
                         int32_t out_dtype, const float *scale, double tol, int32_t *lo_cols, int64_t *n_lo,
                         hipStream_t stream);
int sr_quantize_remainder(int64_t n_s, int64_t n_p, const void *in, int64_t ld_in, int32_t in_dtype,
                          int32_t out_dtype, const float *scale, const int32_t *lo_cols, int64_t n_lo, void *q_lo,
                          int64_t ld_lo, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Tuning hooks (not in the paper).  The fused product is built for a few tile
 * configurations: nv 16-byte vectors per thread and row, `rows` rows per tile, `lookahead`
 * tiles of loads in flight, a `poll_delay` (poll depth) of steps between issuing the
 * reads of the other column groups' partial dots of a tile and using them, and
 * `threads` per workgroup.
 * sr_tile_configs: writes up to `max` configurations built for `dtype` (kind 0: SR
 * products and CG, kind 1: linear-method products) as int32 quintuples
 * (nv, rows, lookahead, poll_delay, threads) to the host array `out`; returns how many
 * exist.  The first one listed is the default.
 * sr_set_tile_config: process-wide override of the automatic choice for every later call
 * with storage type `dtype` and product kind `kind` (nv = 0 restores the automatic
 * choice; dtype = -1 with nv = 0 restores it for all); col_groups = 0 keeps the
 * automatic number of column groups, otherwise it must be a power of two (used when
 * larger than the minimum).  Not synchronized with calls running on other threads.
 * SR_ERR_INVALID if no kernel of that type and kind has that configuration.
 * ------------------------------------------------------------------------------------ */
int sr_tile_configs(int32_t dtype, int32_t kind, int32_t *out, int32_t max);
/* Geometry of the batched products (sr_svk_product, sr_cg_solve_batched), process-wide:
 * split_rows = the most rows per split of the update pass (a power of two in
 * [128, 1024]; fewer rows give more, shorter tasks and more partial traffic), tasks = the
 * tasks per workgroup aimed at when choosing column parts and splits (1..8).  (0, 0)
 * restores the defaults (1024, 2).  Returns SR_ERR_INVALID otherwise. */
int sr_set_batch_config(int32_t split_rows, int32_t tasks);
int sr_set_tile_config(int32_t dtype, int32_t kind, int32_t nv, int32_t rows, int32_t lookahead,
                       int32_t poll_delay, int32_t threads, int32_t col_groups);

/* ------------------------------------------------------------------------------------
 * Index-coded correlator-product-state (CPS) storage (Sec. II.C, Eq. ansatz; parameter
 * layout of Sec. III.A).  A sample occupies exactly one state of each correlator, so the
 * derivative ratio of correlator p's parameter for state s is val[p*n_states + s] (the
 * inverse of that correlator entry) when the sample is in state s, and 0 otherwise: one
 * nonzero per correlator per row, its value fixed by the column.  The storage keeps
 *   idx    one byte per correlator per sample, correlator-major: idx[p*ld_idx + k] is the
 *          state of correlator p in sample k (a state >= n_states selects no column);
 *   val    the value of each correlator column;
 *   dense  the remaining parameters (the pairing block) as an ordinary matrix,
 * with the parameters ordered [correlator 0's n_states columns | correlator 1 | ... |
 * dense columns], n_p = n_corr * n_states + dense.n_p.  Every entry point below computes
 * exactly what the sr_* entry point of the same name computes on the expanded n_s x n_p
 * matrix.  At 32768 samples, 2048 correlators of 240 states and 8480 dense columns a
 * product reads 67 MB of states and the dense block (556 MB in bf16) instead of a
 * 32768 x 500000 matrix.
 * ------------------------------------------------------------------------------------ */
typedef struct sr_cps_matrix {
  int64_t n_s;               /* samples, >= 1                                          */
  int64_t n_corr;            /* correlators, >= 0                                      */
  int32_t n_states;          /* states (columns) per correlator, 1..256                */
  int32_t reserved;          /* must be 0                                              */
  const uint8_t *idx;        /* [n_corr][ld_idx] device, 16-byte aligned               */
  int64_t ld_idx;            /* >= n_s, a multiple of 16                               */
  const double *val;         /* [n_corr * n_states] device                             */
  sr_matrix dense;           /* dense block, n_s rows and dense.n_p >= 0 columns (0: no */
                             /* block; dense.O may then be NULL); SR_F64, SR_F32 or     */
                             /* SR_BF16 with one plane (no O_lo, no lo_cols); at most  */
                             /* 32768 (bf16; 16384 with search_f64), 16384 (f32, f64)   */
                             /* columns; dense.col_mean is ignored                      */
  const double *col_mean;    /* [n_p] device column means (only the dense entries are  */
                             /* read), or NULL: computed by the call                    */
} sr_cps_matrix;

/* sr_grad of the expanded matrix.  The correlator columns' statistics come from per-state
 * counts and per-state energy sums (int64 fixed point: the same bits on every run):
 * mean = val f, diag S = val^2 f (1 - f), g = (2/n_s) val (B_s - f B) with e = E - E_mean,
 * B_s the sum of e over the samples in the state, B over all samples and f the fraction of
 * samples in the state. */
int sr_cps_grad(const sr_cps_matrix *M, const double *E, double *g, double *E_mean, double *col_mean_out,
                double *diagS_out, hipStream_t stream);
/* sr_sv_product of the expanded matrix, one cooperative launch: the row values
 * w_k = (sum of the u = val*v entries of the sample's states) + dense_k . v - obar . v,
 * then per correlator the sums of w_k - mean(w) over the samples in each state (int64
 * fixed point, so the result is the same bit for bit on every run), and the dense block's
 * O^T w.  The dense block is read once; idx is read twice.  bf16 dense blocks accumulate
 * in float32, the rest in float64. */
int sr_cps_sv_product(const sr_cps_matrix *M, const double *v, double *y, double eps, hipStream_t stream);
/* sr_cg_solve of the expanded matrix (same options, outcome and status codes; precond
 * must be 0; search_f64 applies to a bf16 dense block; residual refreshes accumulate in
 * float64). */
int sr_cps_cg_solve(const sr_cps_matrix *M, const double *g, double eps, double *x, const sr_cg_opts *opt,
                    sr_cg_info *info, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Products during sampling (Sec. I: each sampled configuration contributes an outer
 * product, so S can be applied while the samples are generated, without keeping O).
 * The caller owns the accumulators (device memory) and feeds batches of sample rows as its
 * sampler produces them; only one batch need exist at a time.  After the batches of n
 * samples in total, with obar = s1 / n:
 *   Y_i = A_i / n - obar (s1 . z_i) / n + eps z_i = ((S + eps I) z_i)   (centred S of all n),
 *   g = 2 (se / n - <E> obar),  col_mean = obar,  E_mean = <E>.
 * The sums are uncentred (the means are not known before the last sample), so when a
 * column's mean is large against its spread the subtraction loses the corresponding
 * digits; each batch's own contributions are computed by the fused kernels of sr_grad /
 * sr_sv_product (dense rows) or sr_cps_grad / sr_cps_sv_product (index-coded rows), one
 * read of the batch for its statistics and one per vector.
 * ------------------------------------------------------------------------------------ */
typedef struct sr_stream_acc {
  int64_t n_p;               /* parameters, >= 1                                       */
  int32_t m;                 /* vectors z_i, 1..8                                      */
  int32_t reserved;          /* must be 0                                              */
  double *A;                 /* [m][n_p] device: sum over samples of O_k (O_k . z_i)   */
  double *s1;                /* [n_p] device: sum of O_k                               */
  double *se;                /* [n_p] device: sum of E_k O_k, or NULL (no energies)    */
  double *scal;              /* [4] device: samples, sum of E_k, two reserved words    */
} sr_stream_acc;
/* Zero the accumulators. */
int sr_stream_begin(const sr_stream_acc *acc, hipStream_t stream);
/* Add one batch: exactly one of O (dense rows, one plane) and C (index-coded rows) is
 * non-NULL, with n_p columns; E: [batch samples] energies or NULL; Z: [m][n_p] the vectors
 * (the same for every batch of one product). */
int sr_stream_accumulate(const sr_stream_acc *acc, const sr_matrix *O, const sr_cps_matrix *C, const double *E,
                         const double *Z, hipStream_t stream);
/* Y: [m][n_p] (S + eps I) z_i; g, col_mean: [n_p] and E_mean: scalar, each may be NULL (g
 * needs se). */
int sr_stream_finish(const sr_stream_acc *acc, const double *Z, double eps, double *Y, double *g, double *col_mean,
                     double *E_mean, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Workspace (the library's own memory for partials, exchange words and CG vectors; one per
 * device and stream, grown on demand by reallocation, which synchronizes the stream).
 * sr_workspace_bytes: bytes that workspace must hold for `call` (enum sr_call) on the
 * matrix O on the current device (tile choices in effect included; a call with
 * O->col_mean NULL also runs the prepare pass, counted here, and keeps the n_p column
 * means in a separate small buffer of n_p * 8 bytes).  Negative: an sr_status error.
 * sr_workspace_reserve: grows the (current device, stream) workspace to at least `bytes`
 * now, so that later calls within that size allocate nothing there.
 * sr_workspace_held: bytes the (current device, stream) workspace holds (0 if none).
 * ------------------------------------------------------------------------------------ */
enum sr_call { SR_CALL_GRAD = 0, SR_CALL_SV_PRODUCT = 1, SR_CALL_CG_SOLVE = 2, SR_CALL_LM_HV_PRODUCT = 3,
               SR_CALL_ADJOINT = 4 };
int64_t sr_workspace_bytes(const sr_matrix *O, int32_t call);
int sr_workspace_reserve(int64_t bytes, hipStream_t stream);
int64_t sr_workspace_held(hipStream_t stream);

/* Kernel timing (measurement, not in the paper).  sr_timing(1) clears the totals and has
 * the CG solves record HIP events, on their stream, around their launches; sr_timing(0)
 * stops it.  sr_timing_read gives the total milliseconds and the number of launches of a
 * class: 0 the search steps of a split solve (one stored plane, no preconditioner, the
 * storage type's own accumulation) that ran a product, 1 its residual phases that ran one,
 * 2 single-launch solves (two planes, Jacobi, float64 search products, float64/float32
 * products below 2^31 bytes).  Split solves time their launches only where they check the state after every
 * launch (products of at least 2^30 streamed bytes).  Timing adds a synchronization per
 * timed launch. */
int sr_timing(int32_t enable);
int sr_timing_read(int32_t cls, double *ms, int64_t *count);

/* Measurement helper (not in the paper): reads `bytes` (a multiple of 16) at p (16-byte
 * aligned, device) with the products' non-temporal 16-byte loads, `unroll` (2, 4 or 8)
 * loads in flight per thread, blocks_per_cu (1..8) workgroups of 512 threads per compute
 * unit, and writes one folded word per workgroup to sink (device, [CUs * blocks_per_cu]
 * uint32).  Its duration gives the streaming-read ceiling the products are compared
 * with.  Asynchronous on `stream`. */
int sr_stream_read(const void *p, int64_t bytes, int32_t blocks_per_cu, int32_t unroll, uint32_t *sink,
                   hipStream_t stream);

/* Frees every workspace the library holds (all devices, all streams).  Must not be
 * called while library work is pending on any stream. */
int sr_release(void);

/* Static text for a status code. */
const char *sr_status_string(int status);

/* Thread-local text describing the last error returned on this thread ("" if none). */
const char *sr_last_error(void);

/* Library ABI version (major*10000 + minor*100 + patch). */
int sr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SR_H */
