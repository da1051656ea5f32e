// Kernel argument blocks and the kernel registry shared by the kernels and the host API.
#pragma once
#include "sr_product.hpp"

namespace sr {

struct SyncBufs {
  uint32_t *flags;      // [G] grid-barrier epochs (zeroed before each launch)
  uint32_t *abort;      // [1]
  double *red;          // [4][2][G] grid reductions
};

struct SvArgs {
  ProdGeom pg;
  ProdBufs pb;
  SyncBufs sb;
  Operand op;
  const double *mean;
  const double *v;
  double *y;
  double eps;
};

struct LmArgs {
  ProdGeom pg;
  ProdBufs pb;
  SyncBufs sb;
  Operand ops[2];       // O, D
  const double *mean;   // column mean of O
  const double *E;      // [n_s]
  const double *v;      // [n_p + 1]
  double *y;            // [n_p + 1]
};

// Index-coded correlator-product-state storage (one state per correlator per sample plus
// a dense block): the operand of the CPS product and of the CG solves over it.
struct CpsOp {
  const unsigned char *idx;   // [n_corr][ld_idx] state of correlator p in sample k at p*ld_idx + k
  int64_t ld_idx;             // bytes, multiple of 16
  const double *val;          // [n_sp] value of each correlator column
  int64_t n_corr;
  int32_t n_states;           // columns per correlator (states >= n_states select no column)
  int32_t tiles;              // row tiles of tile_rows rows
  int32_t raw;                // 1: uncentred product O^T (O v) / n_s (with zero dense means)
  int32_t tile_rows;          // rows per tile of the row pass: kCpsTileRows, or a smaller
                              // power of two (>= kCpsMinTileRows) so that every workgroup
                              // has a tile when there are few samples
  int64_t n_sp, n_d;          // correlator columns (n_corr * n_states) and dense columns
  const unsigned char *dO;    // dense block [n_s][ld_d] (nullptr when n_d == 0)
  const float *dscale;        // [n_d] column scales (bf16 / f16 dense block) or nullptr
  int64_t ldb_d;              // row stride of the dense block in bytes, multiple of 16
  double *w;                  // [n_s] w_k of the current product
  void *part_sp;              // [n_grp][n_s] partial row sums of the correlator groups (accumulation type)
  int32_t n_grp, cpg;         // correlator groups, correlators per group (LDS table of cpg * n_states)
  int32_t n_items;            // (group, row range) work items of the partial sums
  int32_t rpr;                // rows per range (a multiple of kCpsTileRows)
  void *part;                 // [G][n_dp] dense partial sums (accumulation type)
  int64_t n_dp;               // row stride of part (n_d rounded up to the vector width)
  double *red;                // [4][2][G] grid reductions of the product
};
constexpr int kCpsTileRows = 128;   // rows per tile of the row pass (64 lanes x 2 rows)
constexpr int kCpsMinTileRows = 16; // the smallest tile (its rows' sums come from NT / 16 slices)
constexpr int kCpsTableBytes = 65536;   // LDS table of one correlator group (float64 entries: 8192)

struct CgArgs {
  ProdGeom pg;
  ProdBufs pb;
  SyncBufs sb;
  Operand op;
  const double *mean;
  const double *g;
  double *x, *r, *p, *q;
  double eps, rtol;
  int max_iter, refresh_every, use_x0, restart_on_refresh;
  double refresh_drop2;       // squared relative drop that triggers a refresh; 0: off
  double *hist;         // [max_iter + 1] or nullptr
  double *info;         // [16]: outcome, then the state between the launches of a split solve
  const double *diag;   // [n_p] diag S (Jacobi-preconditioned CG), else nullptr
  CpsOp cps;            // index-coded storage (CPS products only)
};

// A CG solve split over launches (one stored plane, no preconditioner), so that no kernel
// holds more than one product code and the state machine around it (two product codes, or
// the whole state machine, in one kernel cost register spills in the streaming loop):
// k_cg_init starts the solve, k_cg_step runs one search-direction iteration per launch,
// k_cg<..., kPhResidual> runs the residual products (refresh, exit check, warm start;
// float64 accumulation for scaled storage) and returns at the next search step; kPhAll
// runs a whole solve in one launch.  Between launches the state lives in CgArgs::info.
enum { kPhAll = 0, kPhResidual = 2 };
// Layout of CgArgs::info: outcome (read by the host) then the state of a split solve.
enum { kInfoIters = 0, kInfoRefreshes, kInfoStatus, kInfoProducts, kInfoRelRecur, kInfoRelTrue, kInfoOk,
       kInfoMode, kInfoRho, kInfoGg, kInfoRhoRef, kInfoRz, kInfoXstep, kInfoRelBest, kInfoWords = 16 };
// A refresh or exit check whose true residual exceeds this multiple of the best one seen
// ends the solve as not converged (the iteration is past the attainable accuracy).
constexpr double kCgDivergence = 1e3;
enum { kCgModeInit = 0, kCgModeP, kCgModeRefresh, kCgModeConfirm, kCgModeFinal, kCgModeX0, kCgModeDone };

struct GradArgs {
  ProdGeom pg;          // wslice / C / RG for the column reduction (R unused)
  ProdBufs pb;          // ypart holds [RG][3][n_p]
  SyncBufs sb;
  Operand op;
  const double *E;      // [n_s] or nullptr
  double *g_out, *mean_out, *diag_out, *Emean_out;
};

struct QuantArgs {
  ProdGeom pg;
  ProdBufs pb;          // ypart holds [RG][n_p] partial maxima
  SyncBufs sb;
  const unsigned char *in;
  int64_t ldb_in;       // bytes
  unsigned char *out;
  unsigned char *out_lo;  // second code plane or nullptr
  int64_t ld_out;       // elements (16-bit codes)
  float *scale;
};

// Tile configurations (NV 16-byte vectors per data thread, R rows per tile) built for
// each storage type: SR products (k_sv, k_cg) and linear-method products (k_lm, which
// streams two matrices and so uses half the tile).
// X(NV, R, LOOKAHEAD, POLL_DEPTH, THREADS) per storage type; the first SR entry is the
// default (chosen by the tile sweep on MI355X), the others are selectable for tuning.
#define SR_SR_CONFIGS_F64(X) X(4, 1, 1, 1, 512) X(4, 1, 2, 1, 512) X(2, 1, 2, 1, 512) X(2, 2, 1, 1, 512) \
  X(4, 1, 1, 2, 512) X(4, 1, 3, 2, 512)
#define SR_SR_CONFIGS_F32(X) X(4, 1, 1, 1, 512) X(2, 1, 2, 1, 512) X(2, 2, 1, 1, 512)
#define SR_SR_CONFIGS_BF16(X) X(2, 2, 1, 0, 512) X(2, 1, 2, 1, 512) X(2, 1, 3, 1, 512) X(4, 1, 1, 1, 512) \
  X(2, 2, 2, 1, 512) X(1, 4, 1, 1, 512)
#define SR_SR_CONFIGS_F16(X) X(2, 2, 1, 1, 512) X(2, 1, 2, 1, 512) X(4, 1, 1, 1, 512)
#define SR_LM_CONFIGS(X) X(2, 1, 2, 1, 512) X(4, 1, 2, 1, 256)

// Batched solves: K right-hand sides per system, systems one after another in one
// persistent launch.  A product (S + diag(eps)) V takes two passes over O: row dots
// W = O_c V by row blocks (V staged through LDS chunk by chunk), then O^T W by column
// blocks and row splits (the split's rows of W held in LDS).
constexpr int kBatchK = 8;           // right-hand sides per product of the batched kernels
constexpr int kBatchRows = 4;        // rows per wave in the row-dot pass
constexpr int kBatchSplitRows = 1024;   // most rows per split of the update pass (LDS)
constexpr int kBatchNT = 512;        // threads per workgroup of the batched kernels

struct BatchGeom {
  int64_t n_s, n_p;
  int64_t n_rb;                      // row blocks of the row-dot pass (waves * kBatchRows rows)
  int64_t pw;                        // columns per part of the row-dot pass (chunk multiple)
  int P;                             // column parts of the row-dot pass
  int C;                             // column blocks of the update pass (threads * VEC columns)
  int SP;                            // row splits of the update pass
  int64_t rs;                        // rows per split (<= kBatchSplitRows)
};
struct BatchSys {
  Operand op;
  const double *mean;                // [n_p] column means
  const double *g;                   // [k][n_p] right-hand sides
  double *x;                         // [k][n_p] solutions
  BatchGeom bg;                      // geometry of this system's products
  int k;                             // right-hand sides in use (<= kBatchK)
  double eps[kBatchK];               // shift of each right-hand side
};
struct BatchArgs {
  const BatchSys *sys;               // [n_sys] device table
  int n_sys;
  SyncBufs sb;
  double *red;                       // [4][K][G] grid reductions
  double *vs;                        // [K][vstride] scaled operand s_j v_kj
  double *wp;                        // [P][n_s][K] row dots per column part (largest system)
  double *yp;                        // [SP][K][n_p] update-pass partials (largest system)
  double *swp;                       // [SP][K] sums of the centred row dots per split
  double *x, *r, *p, *q;             // [K][vstride]
  int64_t vstride;                   // max n_p (stride of the K vectors)
  double rtol;
  int max_iter, refresh_every;
  double refresh_drop2;              // squared residual drop that triggers a refresh; 0: off
  double *info;                      // [n_sys][K][4]: iterations, status, rel. true residual,
                                     // products; then [1]: 1 if no wait gave up
};

// The batched kernels of a storage type (float64 and float32 only).
struct BatchEntry {
  const void *cg, *sv;
  int nt;
};
const BatchEntry *batched_entry(int dt);   // nullptr if the type has none

// Adjoint backward (row dots, finish, rank-2 write).
struct RowDotsArgs {
  const unsigned char *O;
  int64_t ldb;                       // row stride in bytes
  const float *scale;                // column scales (scaled storage) or nullptr
  const double *mean, *x, *lam;
  int64_t n_s, n_p, wslice;
  int C, RG;
  double *part;                      // [C][n_s][2]
};
struct AdjFinishArgs {
  const double *E, *part;
  int64_t n_s;
  int C;
  double *coef, *dE, *p12;
  const double *x, *lam;             // [n_p]
  int64_t n_p;
  double *deps;                      // device scalar -lambda . x, or nullptr
};
struct Rank2Args {
  const double *coef, *lam, *x;
  int64_t n_s, n_p, ld;              // ld in elements of the output type
  void *dO;
};
const void *rowdots_kernel(int dt, int nv);
const void *adjoint_finish_kernel();
const void *rank2_kernel(int out_dt);
int adjoint_threads();
int adjoint_rows_per_block();

struct KernelEntry {
  int dt, nv, r, look, poll, nt;
  int kind;              // 0: SR (sv + cg), 1: LM
  const void *sv, *cg, *lm;
  const void *sv2;       // two-code-plane product (scaled storage), or nullptr
  const void *cg2;       // CG over two code planes (scaled storage), or nullptr
  const void *cgj;       // Jacobi-preconditioned CG (float64 / float32 storage), or nullptr
  const void *cgx;       // CG with float64-accumulated search products (scaled storage), or nullptr
  const void *cgs, *cgr; // split CG (one plane): search step and residual phase, or nullptr
  const void *cgi;       // split CG: its first launch (initial state), or nullptr
  int ring_bytes;        // dynamic LDS of the launch
};

const KernelEntry *kernel_table(int dt, int *count);

// Index-coded CPS storage: kernels per dense storage type and register tile (nvt 16-byte
// vectors of a dense row per thread, 512 threads).
struct CpsEntry {
  int dt, nvt;
  const void *sv, *init, *step, *stepx, *resid;   // stepx: float64 search products, or nullptr
};
const CpsEntry *cps_table(int dt, int *count);

// Column statistics of the correlator columns of CPS storage.
struct CpsStatsArgs {
  const unsigned char *idx;   // [n_corr][ld_idx]
  int64_t ld_idx, n_corr, n_s;
  const double *val;          // [n_corr * n_states]
  const double *E;            // [n_s] or nullptr
  double *mean, *diag, *g;    // [n_corr * n_states], each may be nullptr (g needs E)
  double *Emean;              // device scalar or nullptr
  int32_t n_states, pad;
};
const void *cps_stats_kernel();

// Products during sampling: accumulators of streamed sample batches and their finish.
struct StreamArgs {
  int64_t n_p;
  int32_t m, i;               // vectors; the vector of a product batch (k_stream_addy)
  double B;                   // samples in the batch
  double *A, *s1, *se, *scal; // accumulators: [m][n_p], [n_p], [n_p] or nullptr, [4]
  const double *mean_b, *g_b, *Emean_b, *y_b;   // batch statistics and raw product
  const double *Z;            // [m][n_p] vectors
  double eps;
  double *Y, *g, *col_mean, *E_mean;            // finish outputs (any but Y may be nullptr)
  double *dots;               // [m] s1 . z_i
};
const void *stream_kernel(int which);   // 0 stats, 1 addy, 2 dots, 3 finish
const void *grad_kernel(int dt);
int grad_nv(int dt);
int grad_threads(int dt);
int grad_rows(int dt);
const void *absmax_kernel(int in_dt);
const void *quantize_kernel(int in_dt, int out_dt);
const void *fill_kernel();

// Compact remainder plane: prepare pass of its columns, column selection and codes.
struct GradLoArgs {
  const unsigned char *Q, *LO;       // first code plane, compact remainder plane
  int64_t ldb, ldb_lo;               // their row strides in bytes
  const int32_t *cols;               // [n_lo] parameter of each remainder column
  int64_t n_lo, n_s, n_p;
  const float *scale;                // [n_p]
  const double *E;                   // [n_s] or nullptr
  const double *Emean;               // device scalar <E> (when E is given)
  int64_t rows_per_block;
  int n_rb;                          // row blocks
  double *part;                      // [n_rb][4][n_lo]: sums of x - K, (x - K)^2, e (x - K), e
  double *g_out, *mean_out, *diag_out;   // [n_p] (entries of the remainder columns rewritten)
};
constexpr int kGradLoRows = 256;     // rows per block of the remainder columns' prepare pass
const void *gradlo_part_kernel(int dt);
const void *gradlo_finish_kernel(int dt);

struct RemArgs {
  ProdGeom pg;
  ProdBufs pb;                       // ypart holds [RG][n_p] partial maxima
  SyncBufs sb;
  const unsigned char *in;
  int64_t ldb_in;                    // bytes
  const float *scale;                // [n_p]
  double *err;                       // [n_p] max_k |O_kj / s_j - q_kj|
};
struct SelectArgs {
  const double *err;                 // [n_p]
  int64_t n_p;
  double tol;
  int32_t *cols;                     // [n_p] selected columns, increasing
  int64_t *count;                    // device scalar
};
struct QuantLoArgs {
  const unsigned char *in;
  int64_t ldb_in, n_s, n_p, n_lo, ld_lo;   // ld_lo in codes (multiple of 8)
  const float *scale;
  const int32_t *cols;
  unsigned char *out;
};
const void *stream_read_kernel(int unroll);   // 512 threads per workgroup
const void *remmax_kernel(int in_dt, int out_dt);
const void *select_kernel();
const void *quantize_lo_kernel(int in_dt, int out_dt);

}  // namespace sr
