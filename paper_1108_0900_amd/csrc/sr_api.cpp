// libsr C-ABI: argument validation, launch planning, per-(device, stream) workspace and
// cooperative launches of the kernels.  Declarations and the contract are in sr.h.
#include "sr.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "sr_launch.hpp"
#include "sr_lm.hpp"
#include "sr_shifts.hpp"

namespace {

using namespace sr;

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(SR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int elem_bytes(int dt) { return dt == SR_F64 ? 8 : dt == SR_F32 ? 4 : 2; }
int vec_of(int dt) { return 16 / elem_bytes(dt); }
bool scaled(int dt) { return dt == SR_BF16 || dt == SR_F16; }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t round_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }
int64_t pow2_ceil(int64_t a) {
  int64_t p = 1;
  while (p < a) p <<= 1;
  return p;
}

// ------------------------------------------------------------------------------------
// Argument checks (host only; no HIP call)
// ------------------------------------------------------------------------------------
int check_matrix(const sr_matrix *m, const char *name) {
  if (m == nullptr) return fail(SR_ERR_INVALID, "%s: null sr_matrix", name);
  if (m->dtype < SR_F64 || m->dtype > SR_F16) return fail(SR_ERR_INVALID, "%s: unknown dtype %d", name, m->dtype);
  if (m->reserved != 0) return fail(SR_ERR_INVALID, "%s: reserved field must be 0", name);
  if (m->n_s < 1) return fail(SR_ERR_INVALID, "%s: n_s must be >= 1 (got %lld)", name, (long long)m->n_s);
  if (m->n_p < 1) return fail(SR_ERR_INVALID, "%s: n_p must be >= 1 (got %lld)", name, (long long)m->n_p);
  if (m->ld < m->n_p) return fail(SR_ERR_INVALID, "%s: ld (%lld) < n_p (%lld)", name, (long long)m->ld, (long long)m->n_p);
  if (m->n_s > (int64_t)1 << 40 || m->n_p > (int64_t)1 << 31)
    return fail(SR_ERR_INVALID, "%s: dimensions out of range", name);
  if (m->O == nullptr) return fail(SR_ERR_INVALID, "%s: O is null", name);
  if (((uintptr_t)m->O) % 16 != 0) return fail(SR_ERR_INVALID, "%s: O must be 16-byte aligned", name);
  if ((m->ld * elem_bytes(m->dtype)) % 16 != 0)
    return fail(SR_ERR_INVALID, "%s: ld * element size must be a multiple of 16 bytes", name);
  if (scaled(m->dtype) && m->col_scale == nullptr)
    return fail(SR_ERR_INVALID, "%s: col_scale is required for bf16/f16 storage", name);
  if (!scaled(m->dtype) && m->col_scale != nullptr)
    return fail(SR_ERR_INVALID, "%s: col_scale must be NULL for f64/f32 storage", name);
  if (m->O_lo != nullptr && !scaled(m->dtype))
    return fail(SR_ERR_INVALID, "%s: a second code plane (O_lo) needs bf16/f16 storage", name);
  if (((uintptr_t)m->O_lo) % 16 != 0) return fail(SR_ERR_INVALID, "%s: O_lo must be 16-byte aligned", name);
  if (m->lo_cols != nullptr) {
    if (!scaled(m->dtype)) return fail(SR_ERR_INVALID, "%s: a compact remainder plane needs bf16/f16 storage", name);
    if (m->n_lo < 0 || m->n_lo > m->n_p)
      return fail(SR_ERR_INVALID, "%s: n_lo must be in [0, n_p] (got %lld)", name, (long long)m->n_lo);
    if (m->n_lo > 0 && m->O_lo == nullptr) return fail(SR_ERR_INVALID, "%s: lo_cols given without O_lo", name);
    if (m->n_lo > 0 && (m->ld_lo < m->n_lo || (m->ld_lo * 2) % 16 != 0))
      return fail(SR_ERR_INVALID, "%s: ld_lo must be >= n_lo with ld_lo * 2 a multiple of 16 bytes", name);
    if (round_up(m->n_p, 8) + m->n_lo >= ((int64_t)1 << 31) - 64)
      return fail(SR_ERR_INVALID, "%s: n_p + n_lo out of range", name);
  } else if (m->n_lo != 0 || m->ld_lo != 0) {
    return fail(SR_ERR_INVALID, "%s: n_lo and ld_lo must be 0 without lo_cols", name);
  }
  return SR_OK;
}

// A compact remainder plane with at least one column.
bool compact(const sr_matrix *m) { return m->lo_cols != nullptr && m->n_lo > 0; }
// A full second code plane.
bool two_planes(const sr_matrix *m) { return m->O_lo != nullptr && m->lo_cols == nullptr; }
// Columns a single-plane product streams: the parameters, then (compact plane) its columns
// starting at n_p rounded up to whole 16-byte vectors.
int64_t streamed_cols(const sr_matrix *m) {
  return compact(m) ? round_up(m->n_p, vec_of(m->dtype)) + m->n_lo : m->n_p;
}

bool ranges_overlap(const void *a, int64_t na, const void *b, int64_t nb) {
  const char *pa = (const char *)a, *pb = (const char *)b;
  return pa < pb + nb && pb < pa + na;
}

// ------------------------------------------------------------------------------------
// Device state
// ------------------------------------------------------------------------------------
struct DeviceInfo {
  bool ok = false;
  int cus = 0;
  int grid = 0;     // persistent grid size: 8 * (largest power of two <= CUs/8)
};

std::mutex g_mu;
// Geometry of the batched products, tunable: the most rows per update split (a power of
// two in [128, kBatchSplitRows]) and the tasks per workgroup aimed at in each pass (1..8);
// set by sr_set_batch_config.
int g_batch_split_rows = kBatchSplitRows;
int g_batch_tasks = 2;
std::map<int, DeviceInfo> g_dev;

struct Workspace {
  void *ptr = nullptr;
  size_t bytes = 0;
};
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

int device_check(int *dev_out, DeviceInfo *info_out) {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n < 1) {
    (void)hipGetLastError();
    return fail(SR_ERR_NODEVICE, "no HIP device available");
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_dev.find(dev);
  if (it == g_dev.end()) {
    hipDeviceProp_t p;
    HIP_TRY(hipGetDeviceProperties(&p, dev));
    DeviceInfo di;
    di.ok = std::strncmp(p.gcnArchName, "gfx950", 6) == 0;
    di.cus = p.multiProcessorCount;
    int coop = 0;
    HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) di.ok = false;
    int L = 1;
    while (L * 2 <= di.cus / 8) L *= 2;
    di.grid = 8 * L;
    it = g_dev.emplace(dev, di).first;
  }
  if (!it->second.ok) return fail(SR_ERR_NODEVICE, "device %d is not a gfx950 device with cooperative launch", dev);
  *dev_out = dev;
  *info_out = it->second;
  return SR_OK;
}

// Workspace of at least `bytes` for (dev, stream); grows by reallocation (after the
// stream has drained).
int get_workspace(int dev, hipStream_t s, size_t bytes, void **out,
                  std::map<std::pair<int, hipStream_t>, Workspace> &table = g_ws) {
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace &w = table[std::make_pair(dev, s)];
  if (w.bytes < bytes) {
    if (w.ptr) {
      HIP_TRY(hipStreamSynchronize(s));
      HIP_TRY(hipFree(w.ptr));
      w.ptr = nullptr;
      w.bytes = 0;
    }
    const size_t want = (size_t)round_up((int64_t)bytes, (int64_t)1 << 20);
    hipError_t e = hipMalloc(&w.ptr, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      w.ptr = nullptr;
      return fail(SR_ERR_NOMEM, "workspace allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
    }
    w.bytes = want;
  }
  *out = w.ptr;
  return SR_OK;
}

// Bump allocator over the workspace (256-byte aligned pieces).
struct Carve {
  char *base;
  size_t off = 0;
  explicit Carve(void *b) : base((char *)b) {}
  template <typename T> T *take(int64_t n) {
    off = (size_t)round_up((int64_t)off, 256);
    T *p = (T *)(base + off);
    off += (size_t)n * sizeof(T);
    return p;
  }
};

// ------------------------------------------------------------------------------------
// Launch planning
// ------------------------------------------------------------------------------------
struct Plan {
  const KernelEntry *ke = nullptr;
  ProdGeom pg{};
  int words = 0;   // exchange words per column group per tile
};

// Tile overrides per (storage type, product kind) set by sr_set_tile_config (tuning):
// tile shape, pipeline depths, workgroup size and, optionally, a larger power-of-two
// number of column groups.  nv = 0: automatic.
struct TileForce {
  int nv, r, look, poll, nt, c;
};
TileForce g_force[4][2] = {};

// Column groups and slices over the n_v streamed columns (n_v < 0: n_v = n_p).  C is a
// power of two (RG = G / C), or with any_c the least number of column groups that holds
// the columns when that gives more row groups: each XCD holds (G/8)/C row groups and
// leaves its other workgroups idle (a product's time goes with its rows per row group,
// not with how full a workgroup's slice is).
int geometry(int G, int64_t n_s, int64_t n_p, int cols_per_wg, int vec, int r, int force_c, ProdGeom *pg,
             int64_t n_v = -1, bool any_c = false) {
  if (n_v < 0) n_v = n_p;
  const int64_t cmin = cdiv(n_v, cols_per_wg);
  int64_t C = pow2_ceil(cmin);
  int RG = C <= G ? G / (int)C : 0;
  if (force_c > 0 && force_c >= C) {
    C = force_c;
    RG = G / (int)C;
  } else if (any_c && G % 8 == 0 && cmin < C && cmin <= G / 8 && 8 * ((G / 8) / cmin) > RG) {
    C = cmin;
    RG = 8 * ((G / 8) / (int)cmin);
  }
  if (C > G) return fail(SR_ERR_INVALID, "%lld columns exceed the column capacity of the built tiles (%lld)",
                         (long long)n_v, (long long)G * cols_per_wg);
  pg->G = G;
  pg->C = (int)C;
  pg->RG = RG;
  pg->n_s = n_s;
  pg->n_p = n_p;
  pg->n_v = n_v;
  pg->wslice = round_up(cdiv(n_v, C), vec);
  pg->n_tiles = (int)cdiv(n_s, r);
  return SR_OK;
}

int make_plan(int dt, int G, int64_t n_s, int64_t n_p, int ndot, Plan *plan, int64_t n_v = -1) {
  int count = 0;
  const KernelEntry *tab = kernel_table(dt, &count);
  const int vec = vec_of(dt);
  const int kind = ndot == 1 ? 0 : 1;
  const TileForce &f = g_force[dt][kind];
  const KernelEntry *pick = nullptr;
  if (f.nv > 0) {
    for (int i = 0; i < count; ++i)
      if (tab[i].kind == kind && tab[i].nv == f.nv && tab[i].r == f.r && tab[i].look == f.look &&
          tab[i].poll == f.poll && tab[i].nt == f.nt)
        pick = &tab[i];
  }
  if (pick == nullptr) {
    // Default: the first configuration listed for the kind (the tuned one); the
    // tuning hooks select others.
    for (int i = 0; i < count && pick == nullptr; ++i)
      if (tab[i].kind == kind) pick = &tab[i];
  }
  plan->ke = pick;
  const int cols = pick->nv * vec * pick->nt;
  // uneven column groups by default for 4- and 2-byte storage (measured faster there);
  // float64 keeps powers of two (on CPS 65536 x 24512 six groups ran 5-14 % slower than
  // eight); the tuning hook forces either
  int rc = geometry(G, n_s, n_p, cols, vec, pick->r, f.nv > 0 && pick->nv == f.nv ? f.c : 0, &plan->pg, n_v,
                    dt != DT_F64);
  if (rc) return rc;
  plan->words = ndot * pick->r * 2;   // float64 partials (two tagged words each)
  return SR_OK;
}

// Workspace pieces used by a product-type launch.
struct ProdWs {
  SyncBufs sb;
  ProdBufs pb;
  uint32_t *zero_base;   // start of the region zeroed before each launch
  int64_t zero_words;    // its length in 32-bit words
};

void carve_prod(Carve &cv, const Plan &pl, int64_t ypart_doubles, ProdWs *w) {
  const ProdGeom &pg = pl.pg;
  // zeroed region: flags, abort, exchange ring
  const size_t start = (size_t)round_up((int64_t)cv.off, 256);
  w->sb.flags = cv.take<uint32_t>(pg.G);
  w->sb.abort = cv.take<uint32_t>(64);
  // the ring is sized for G workgroups (RG * C <= G), so that plans of one launch with
  // different geometries keep one layout
  w->pb.xchg = cv.take<u64>((int64_t)pg.G * kRing * (pl.words > 0 ? pl.words : 1));
  const size_t end = cv.off;
  w->zero_base = (uint32_t *)(cv.base + start);
  w->zero_words = (int64_t)((end - start + 3) / 4);
  w->sb.red = cv.take<double>(4 * 2 * pg.G);
  w->pb.sink = cv.take<u64>((int64_t)pg.G * (pl.words > 0 ? pl.words : 1));
  w->pb.ypart = cv.take<double>(ypart_doubles);
  w->pb.spart = cv.take<double>((int64_t)pg.RG * 2);
}

size_t prod_ws_bytes(const Plan &pl, int64_t ypart_doubles) {
  const ProdGeom &pg = pl.pg;
  size_t b = 0;
  auto add = [&](size_t n) { b = (size_t)round_up((int64_t)b, 256) + n; };
  add(pg.G * 4);
  add(64 * 4);
  add((size_t)pg.G * kRing * (pl.words > 0 ? pl.words : 1) * 8);
  add((size_t)4 * 2 * pg.G * 8);
  add((size_t)pg.G * (pl.words > 0 ? pl.words : 1) * 8);
  add((size_t)ypart_doubles * 8);
  add((size_t)pg.RG * 2 * 8);
  return b + 256;
}

int zero_sync(const ProdWs &w, hipStream_t s) {
  int64_t n = w.zero_words;
  uint32_t v = 0;
  uint32_t *p = w.zero_base;
  void *args[] = {&p, &n, &v};
  const int blocks = (int)std::min<int64_t>(1024, cdiv(n, 256));
  HIP_TRY(hipLaunchKernel(fill_kernel(), dim3(blocks > 0 ? blocks : 1), dim3(256), args, 0, s));
  return SR_OK;
}

int launch_coop(const void *fn, int G, void *argp, hipStream_t s, int block = kNT, int shmem = 0) {
  void *args[] = {argp};
  if (shmem > 0) HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, shmem));
  HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(G), dim3(block), args, (unsigned)shmem, s));
  return SR_OK;
}

Operand make_operand(const sr_matrix *m) {
  Operand op;
  op.O = (const unsigned char *)m->O;
  op.lo = (const unsigned char *)m->O_lo;
  op.lo_cols = nullptr;
  op.n_lo = 0;
  op.ldb_lo = 0;
  op.n_q = (int64_t)1 << 62;
  if (compact(m)) {
    op.lo_cols = m->lo_cols;
    op.n_lo = m->n_lo;
    op.ldb_lo = m->ld_lo * elem_bytes(m->dtype);
    op.n_q = round_up(m->n_p, vec_of(m->dtype));
  } else if (m->lo_cols != nullptr) {
    op.lo = nullptr;     // an empty compact plane: single plane
  }
  op.ldb = m->ld * elem_bytes(m->dtype);
  op.scale = m->col_scale;
  return op;
}

// Column statistics / gradient pass.  Any output pointer may be null.
int run_grad(const sr_matrix *m, const double *E, double *g, double *Emean, double *mean, double *diag, int dev,
             const DeviceInfo &di, hipStream_t s) {
  const int dt = m->dtype;
  const int vec = vec_of(dt);
  Plan pl;
  pl.words = 0;
  int rc = geometry(di.grid, m->n_s, m->n_p, grad_nv(dt) * vec * grad_threads(dt), vec, grad_rows(dt), 0, &pl.pg);
  if (rc) return rc;
  const int64_t ypd = (int64_t)pl.pg.RG * 3 * m->n_p;
  // a compact remainder plane: the pass over the first plane gives every column, then the
  // remainder columns are redone from both planes (row blocks, then a fixed-order sum)
  const bool cmp = compact(m);
  const int64_t n_rb = cmp ? cdiv(m->n_s, kGradLoRows) : 0;
  const size_t extra = cmp ? (size_t)(4 * n_rb * m->n_lo + 64) * 8 + 512 : 0;
  void *base = nullptr;
  rc = get_workspace(dev, s, prod_ws_bytes(pl, ypd) + extra, &base);
  if (rc) return rc;
  Carve cv(base);
  ProdWs w;
  carve_prod(cv, pl, ypd, &w);
  GradArgs a{};
  a.pg = pl.pg;
  a.pb = w.pb;
  a.sb = w.sb;
  a.op = make_operand(m);
  if (cmp) a.op.lo = nullptr;
  a.E = E;
  a.g_out = g;
  a.mean_out = mean;
  a.diag_out = diag;
  a.Emean_out = Emean;
  double *emean_ws = nullptr, *part = nullptr;
  if (cmp) {
    emean_ws = cv.take<double>(8);
    part = cv.take<double>(4 * n_rb * m->n_lo);
    if (a.Emean_out == nullptr) a.Emean_out = emean_ws;
  }
  rc = zero_sync(w, s);
  if (rc) return rc;
  rc = launch_coop(grad_kernel(dt), pl.pg.G, &a, s, grad_threads(dt));
  if (rc || !cmp) return rc;
  GradLoArgs b{};
  b.Q = (const unsigned char *)m->O;
  b.LO = (const unsigned char *)m->O_lo;
  b.ldb = m->ld * elem_bytes(dt);
  b.ldb_lo = m->ld_lo * elem_bytes(dt);
  b.cols = m->lo_cols;
  b.n_lo = m->n_lo;
  b.n_s = m->n_s;
  b.n_p = m->n_p;
  b.scale = m->col_scale;
  b.E = E;
  b.Emean = a.Emean_out;
  b.rows_per_block = kGradLoRows;
  b.n_rb = (int)n_rb;
  b.part = part;
  b.g_out = g;
  b.mean_out = mean;
  b.diag_out = diag;
  void *args[] = {&b};
  const int nb = (int)cdiv(m->n_lo, kNT);
  HIP_TRY(hipLaunchKernel(gradlo_part_kernel(dt), dim3(nb, (unsigned)n_rb), dim3(kNT), args, 0, s));
  HIP_TRY(hipLaunchKernel(gradlo_finish_kernel(dt), dim3(nb), dim3(kNT), args, 0, s));
  return SR_OK;
}

// Column means into `mean` when the matrix does not carry them.
int ensure_mean(const sr_matrix *m, double *scratch, const double **mean_out, int dev, const DeviceInfo &di,
                hipStream_t s) {
  if (m->col_mean) {
    *mean_out = m->col_mean;
    return SR_OK;
  }
  int rc = run_grad(m, nullptr, nullptr, nullptr, scratch, nullptr, dev, di, s);
  if (rc) return rc;
  *mean_out = scratch;
  return SR_OK;
}

// Separate small allocation for means computed on behalf of the caller, so they survive
// the workspace being re-carved by the product launch that follows.
std::map<std::pair<int, hipStream_t>, Workspace> g_mean_ws;
// Buffers of the batched calls (kept apart from g_ws, which the prepare passes they
// launch first carve for themselves).
std::map<std::pair<int, hipStream_t>, Workspace> g_batch_ws;
// Scratch of the streamed (during-sampling) products: batch statistics, one product.
std::map<std::pair<int, hipStream_t>, Workspace> g_stream_ws;

int get_mean_scratch(int dev, hipStream_t s, int64_t n, double **out) {
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace &w = g_mean_ws[std::make_pair(dev, s)];
  const size_t bytes = (size_t)n * 8 + 256;
  if (w.bytes < bytes) {
    if (w.ptr) {
      HIP_TRY(hipStreamSynchronize(s));
      HIP_TRY(hipFree(w.ptr));
      w.ptr = nullptr;
      w.bytes = 0;
    }
    hipError_t e = hipMalloc(&w.ptr, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      w.ptr = nullptr;
      return fail(SR_ERR_NOMEM, "mean scratch allocation failed");
    }
    w.bytes = bytes;
  }
  *out = (double *)w.ptr;
  return SR_OK;
}

// Buffers of the Davidson solver (its products carve g_ws for themselves).
std::map<std::pair<int, hipStream_t>, Workspace> g_lm_ws;
// Solutions, directions and checks of the multi-shift solve (kept apart from g_ws, which
// its launch and the residual checks carve).
std::map<std::pair<int, hipStream_t>, Workspace> g_shift_ws;

// ------------------------------------------------------------------------------------
// Small dense eigenproblem of the Davidson subspace (host)
// ------------------------------------------------------------------------------------
typedef std::complex<double> cplx;

// Eigenvalues of the real m x m matrix A (row-major): Householder reduction to upper
// Hessenberg form, then single-shift QR in complex arithmetic with Wilkinson shifts
// (Givens rotations on the active block, deflation at negligible subdiagonals).
bool hessenberg_qr_eigenvalues(const std::vector<double> &A, int m, std::vector<cplx> &ev) {
  std::vector<cplx> H(A.begin(), A.end());
  auto h = [&](int i, int j) -> cplx & { return H[(size_t)i * m + j]; };
  for (int k = 0; k + 2 < m; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < m; ++i) alpha += std::norm(h(i, k));
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    std::vector<cplx> v(m, 0.0);
    const cplx x0 = h(k + 1, k);
    const cplx ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cplx(1.0);
    for (int i = k + 1; i < m; ++i) v[i] = h(i, k);
    v[k + 1] += ph * alpha;
    double vn = 0.0;
    for (int i = k + 1; i < m; ++i) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    // H <- P H P with P = I - 2 v v^H / (v^H v)
    for (int j = 0; j < m; ++j) {
      cplx d = 0.0;
      for (int i = k + 1; i < m; ++i) d += std::conj(v[i]) * h(i, j);
      d *= 2.0 / vn;
      for (int i = k + 1; i < m; ++i) h(i, j) -= v[i] * d;
    }
    for (int i = 0; i < m; ++i) {
      cplx d = 0.0;
      for (int j = k + 1; j < m; ++j) d += h(i, j) * v[j];
      d *= 2.0 / vn;
      for (int j = k + 1; j < m; ++j) h(i, j) -= d * std::conj(v[j]);
    }
  }
  const double ulp = 2.220446049250313e-16;
  int hi = m - 1, iter = 0, total = 0;
  while (hi > 0) {
    if (std::abs(h(hi, hi - 1)) <= ulp * (std::abs(h(hi, hi)) + std::abs(h(hi - 1, hi - 1)))) {
      h(hi, hi - 1) = 0.0;
      --hi;
      iter = 0;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::abs(h(lo, lo - 1)) > ulp * (std::abs(h(lo, lo)) + std::abs(h(lo - 1, lo - 1)))) --lo;
    const cplx a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
    const cplx tr = a + d, det = a * d - b * c, disc = std::sqrt(tr * tr / 4.0 - det);
    const cplx m1 = tr / 2.0 + disc, m2 = tr / 2.0 - disc;
    cplx mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    if (iter > 0 && iter % 10 == 0) mu += std::abs(h(hi, hi - 1));     // exceptional shift
    for (int k = lo; k <= hi; ++k) h(k, k) -= mu;
    std::vector<double> cs(m);
    std::vector<cplx> sn(m);
    for (int k = lo; k < hi; ++k) {           // H - mu I = Q R
      const cplx x = h(k, k), y = h(k + 1, k);
      const double r = std::sqrt(std::norm(x) + std::norm(y));
      double cc;
      cplx ss;
      if (r == 0.0) {
        cc = 1.0;
        ss = 0.0;
      } else if (std::abs(x) == 0.0) {
        cc = 0.0;
        ss = std::conj(y) / std::abs(y);
      } else {
        cc = std::abs(x) / r;
        ss = (x / std::abs(x)) * std::conj(y) / r;
      }
      cs[k] = cc;
      sn[k] = ss;
      for (int j = k; j <= hi; ++j) {
        const cplx p = h(k, j), q = h(k + 1, j);
        h(k, j) = cc * p + ss * q;
        h(k + 1, j) = -std::conj(ss) * p + cc * q;
      }
    }
    for (int k = lo; k < hi; ++k) {           // R Q
      const double cc = cs[k];
      const cplx ss = sn[k];
      for (int i = lo; i <= std::min(k + 1, hi); ++i) {
        const cplx p = h(i, k), q = h(i, k + 1);
        h(i, k) = p * cc + q * std::conj(ss);
        h(i, k + 1) = -p * ss + q * cc;
      }
    }
    for (int k = lo; k <= hi; ++k) h(k, k) += mu;
    ++iter;
    if (++total > 200 * m) return false;
  }
  ev.resize(m);
  for (int i = 0; i < m; ++i) ev[i] = h(i, i);
  return true;
}

// Eigenvector of A for the eigenvalue theta by inverse iteration (complex LU with partial
// pivoting of A - theta I, nudged off exact singularity); real part, unit norm, sign fixed
// by the largest component.
void inverse_iteration(const std::vector<double> &A, int m, cplx theta, std::vector<double> &y) {
  double scale = 0.0;
  for (double v : A) scale = std::max(scale, std::abs(v));
  const cplx shift = theta + cplx(1e-13 * std::max(scale, 1e-300), 0.0);
  std::vector<cplx> L((size_t)m * m);
  std::vector<int> piv(m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) L[(size_t)i * m + j] = A[(size_t)i * m + j] - (i == j ? shift : cplx(0.0));
  for (int k = 0; k < m; ++k) {
    int p = k;
    for (int i = k + 1; i < m; ++i)
      if (std::abs(L[(size_t)i * m + k]) > std::abs(L[(size_t)p * m + k])) p = i;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < m; ++j) std::swap(L[(size_t)k * m + j], L[(size_t)p * m + j]);
    if (std::abs(L[(size_t)k * m + k]) == 0.0) L[(size_t)k * m + k] = 1e-300;
    for (int i = k + 1; i < m; ++i) {
      const cplx f = L[(size_t)i * m + k] / L[(size_t)k * m + k];
      L[(size_t)i * m + k] = f;
      for (int j = k + 1; j < m; ++j) L[(size_t)i * m + j] -= f * L[(size_t)k * m + j];
    }
  }
  std::vector<cplx> z(m, cplx(1.0 / std::sqrt((double)m)));
  for (int sweep = 0; sweep < 3; ++sweep) {
    for (int k = 0; k < m; ++k) std::swap(z[k], z[piv[k]]);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < i; ++j) z[i] -= L[(size_t)i * m + j] * z[j];
    for (int i = m - 1; i >= 0; --i) {
      for (int j = i + 1; j < m; ++j) z[i] -= L[(size_t)i * m + j] * z[j];
      z[i] /= L[(size_t)i * m + i];
    }
    double nz = 0.0;
    for (const cplx &v : z) nz += std::norm(v);
    nz = std::sqrt(nz);
    for (cplx &v : z) v /= nz;
  }
  int big = 0;
  for (int i = 1; i < m; ++i)
    if (std::abs(z[i]) > std::abs(z[big])) big = i;
  const cplx ph = std::conj(z[big]) / std::abs(z[big]);
  y.assign(m, 0.0);
  double ny = 0.0;
  for (int i = 0; i < m; ++i) {
    y[i] = std::real(z[i] * ph);
    ny += y[i] * y[i];
  }
  ny = std::sqrt(ny);
  for (double &v : y) v /= ny;
}

// The lowest eigenvalue of A (least real part; real ones preferred) and its vector.
bool lowest_eigenpair(const std::vector<double> &A, int m, double *theta, std::vector<double> &y) {
  std::vector<cplx> ev;
  if (!hessenberg_qr_eigenvalues(A, m, ev)) return false;
  double scale = 0.0;
  for (const cplx &e : ev) scale = std::max(scale, std::abs(e));
  int best = -1;
  for (int pass = 0; pass < 2 && best < 0; ++pass)
    for (int i = 0; i < m; ++i) {
      if (pass == 0 && std::abs(std::imag(ev[i])) > 1e-10 * std::max(scale, 1e-300)) continue;
      if (best < 0 || std::real(ev[i]) < std::real(ev[best])) best = i;
    }
  inverse_iteration(A, m, ev[best], y);
  *theta = std::real(ev[best]);
  return true;
}

// ------------------------------------------------------------------------------------
// Device vector operations of the Davidson solver
// ------------------------------------------------------------------------------------
struct LmBufs {
  double *part, *dots;             // [nb][kLmMaxSub], [kLmMaxSub]
  int nb;
};
// out_dev[i] = X[i] . w for i < m in device memory (fixed-order reduction), queued only.
int lm_mdot_dev(const LmBufs &b, const double *X, int64_t ld, int m, const double *w, int64_t n, double *out_dev,
                hipStream_t s) {
  MdotArgs a{};
  a.X = X;
  a.ld = ld;
  a.n = n;
  a.m = m;
  a.nb = b.nb;
  a.w = w;
  a.part = b.part;
  a.out = out_dev;
  void *args[] = {&a};
  HIP_TRY(hipLaunchKernel(mdot_part_kernel(), dim3(b.nb, m), dim3(lm_threads()), args, 0, s));
  HIP_TRY(hipLaunchKernel(mdot_final_kernel(), dim3(1), dim3(64), args, 0, s));
  return SR_OK;
}
// out_host[i] = X[i] . w for i < m (device reduction in fixed order, then a copy).
int lm_mdot(const LmBufs &b, const double *X, int64_t ld, int m, const double *w, int64_t n, double *out_host,
            hipStream_t s) {
  int rc = lm_mdot_dev(b, X, ld, m, w, n, b.dots, s);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(out_host, b.dots, (size_t)m * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return SR_OK;
}
// out = beta out + sign * sum_i cdev[i] X[i] with cdev in device memory, or (X = nullptr,
// bdev given) out = out / sqrt(*bdev).
int lm_lincomb_dev(const double *X, const double *cdev, double sign, int mx, const double *bdev, int64_t ld,
                   double beta, double *out, int64_t n, hipStream_t s) {
  LincombArgs a{};
  a.X = X;
  a.mx = mx;
  a.ld = ld;
  a.n = n;
  a.beta = beta;
  a.out = out;
  a.cdev = cdev;
  a.cdev_sign = sign;
  a.bdev = bdev;
  void *args[] = {&a};
  const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(n, lm_threads())));
  HIP_TRY(hipLaunchKernel(lincomb_kernel(), dim3(blocks), dim3(lm_threads()), args, 0, s));
  return SR_OK;
}
// out = beta out + sum_i ca[i] X[i] + sum_i cz[i] Z[i].
int lm_lincomb(const double *X, const double *ca, int mx, const double *Z, const double *cz, int mz, int64_t ld,
               double beta, double *out, int64_t n, hipStream_t s) {
  LincombArgs a{};
  a.X = X;
  a.Z = Z;
  a.mx = mx;
  a.mz = mz;
  a.ld = ld;
  a.n = n;
  a.beta = beta;
  a.out = out;
  for (int i = 0; i < mx; ++i) a.ca[i] = ca[i];
  for (int i = 0; i < mz; ++i) a.cz[i] = cz[i];
  void *args[] = {&a};
  const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(n, lm_threads())));
  HIP_TRY(hipLaunchKernel(lincomb_kernel(), dim3(blocks), dim3(lm_threads()), args, 0, s));
  return SR_OK;
}

// Products of at least this many streamed bytes run their split solve with a state check
// after every launch.
constexpr int64_t kStepSyncBytes = (int64_t)1 << 30;
// Float64 / float32 storage: products below this many bytes run the persistent solve (one
// launch; per-launch costs outweigh the split form's register savings there: 136 against
// 160 us per product at 8192 x 4000 float64, 269 against 285 at 16384 x 16384 float32,
// equal from about 6 GB on).
constexpr int64_t kSplitMinBytes = (int64_t)2 << 30;

// Kernel timing (sr_timing): HIP events around the launches of the CG solves, on their
// stream; accumulated per class while enabled.
enum { kTimeSearchStep = 0, kTimeResidualPhase = 1, kTimeSolveLaunch = 2, kTimeClasses = 3 };
struct TimingTotals {
  bool on = false;
  double ms[kTimeClasses] = {0.0, 0.0, 0.0};
  int64_t count[kTimeClasses] = {0, 0, 0};
};
TimingTotals g_timing;

// Events around one launch when timing is enabled; record() (after the stream has passed
// the end event) adds the elapsed time to a class.
struct TimedLaunch {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStream_t s;
  explicit TimedLaunch(hipStream_t s_) : s(s_) {
    bool on;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      on = g_timing.on;
    }
    if (on && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
      (void)hipEventRecord(e0, s);
    } else {
      (void)hipGetLastError();
      release();
    }
  }
  void stop() {
    if (e1) (void)hipEventRecord(e1, s);
  }
  void record(int cls) {
    if (!e0 || !e1) return;
    float ms = 0.0f;
    if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
      std::lock_guard<std::mutex> lk(g_mu);
      g_timing.ms[cls] += ms;
      g_timing.count[cls] += 1;
    }
    (void)hipGetLastError();
  }
  void release() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    e0 = e1 = nullptr;
  }
  ~TimedLaunch() { release(); }
};

// Column layout of the adjoint's row-dot pass: NV 16-byte vectors per thread (more for wide
// matrices), column groups of NV * VEC * threads columns.
int adjoint_nv(const sr_matrix *O) {
  const int64_t vec = vec_of(O->dtype), nt = adjoint_threads();
  return O->n_p >= 4 * vec * nt * 8 ? 4 : (O->n_p >= 2 * vec * nt * 8 ? 2 : 1);
}
int64_t adjoint_column_groups(const sr_matrix *O) {
  const int64_t cols = (int64_t)adjoint_nv(O) * vec_of(O->dtype) * adjoint_threads();
  return std::min<int64_t>(cdiv(O->n_p, cols), 1 << 20);
}

// Scratch of sr_sv_product_noalloc: barrier flags, exchange ring, row-group partials.  The
// largest product any built tile plans needs G * (widest column slice) float64 partials,
// 256 * 16384 * 8 bytes = 32 MiB, plus under 0.5 MiB of synchronisation data.  Each device
// holds its own copy for the life of the process.  In host code the name is not a device
// address; scratch_address gives the device's.
constexpr size_t kNoAllocScratchBytes = (size_t)36 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::map<int, void *> g_scratch_ptr;

// Device address of `scratch` on device `dev` (the current device), looked up once.
int scratch_address(int dev, void **out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return fail(SR_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    }
    it = g_scratch_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return SR_OK;
}

}  // namespace

// ======================================================================================
// C ABI
// ======================================================================================
extern "C" {

int sr_version(void) { return 1 * 10000 + 0 * 100 + 0; }

const char *sr_last_error(void) { return g_last_error.c_str(); }

const char *sr_status_string(int status) {
  switch (status) {
    case SR_OK: return "SR_OK";
    case SR_NOT_CONVERGED: return "SR_NOT_CONVERGED: CG reached max_iter";
    case SR_BREAKDOWN: return "SR_BREAKDOWN: p.(S+eps I)p <= 0";
    case SR_ERR_INVALID: return "SR_ERR_INVALID: invalid argument";
    case SR_ERR_NOMEM: return "SR_ERR_NOMEM: workspace allocation failed";
    case SR_ERR_HIP: return "SR_ERR_HIP: HIP runtime error";
    case SR_ERR_NONFINITE: return "SR_ERR_NONFINITE: non-finite value in CG";
    case SR_ERR_NODEVICE: return "SR_ERR_NODEVICE: no gfx950 device";
    case SR_ERR_TIMEOUT: return "SR_ERR_TIMEOUT: cross-workgroup wait exceeded its bound";
    default: return "unknown status";
  }
}

int64_t sr_workspace_bytes(const sr_matrix *O, int32_t call) {
  int rc = check_matrix(O, "sr_workspace_bytes");
  if (rc) return rc;
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  const int dt = O->dtype, vec = vec_of(dt);
  // the prepare pass (also run by the products and the solve when col_mean is NULL)
  Plan gp;
  gp.words = 0;
  rc = geometry(di.grid, O->n_s, O->n_p, grad_nv(dt) * vec * grad_threads(dt), vec, grad_rows(dt), 0, &gp.pg);
  if (rc) return rc;
  size_t grad = prod_ws_bytes(gp, (int64_t)gp.pg.RG * 3 * O->n_p);
  if (compact(O)) grad += (size_t)(4 * cdiv(O->n_s, kGradLoRows) * O->n_lo + 64) * 8 + 512;
  const size_t pre = O->col_mean ? 0 : grad;
  switch (call) {
    case SR_CALL_GRAD: return (int64_t)grad;
    case SR_CALL_SV_PRODUCT:
    case SR_CALL_CG_SOLVE: {
      Plan pl;
      rc = make_plan(dt, di.grid, O->n_s, O->n_p, 1, &pl, streamed_cols(O));
      if (rc) return rc;
      size_t b = prod_ws_bytes(pl, (int64_t)pl.pg.RG * pl.pg.n_v);
      if (call == SR_CALL_CG_SOLVE) b += (size_t)3 * (O->n_p * 8 + 256) + 2048;
      return (int64_t)std::max(b, pre);
    }
    case SR_CALL_LM_HV_PRODUCT: {
      if (O->O_lo != nullptr) return fail(SR_ERR_INVALID, "sr_workspace_bytes: lm_hv_product takes one code plane");
      Plan pl;
      rc = make_plan(dt, di.grid, O->n_s, O->n_p, 2, &pl);
      if (rc) return rc;
      return (int64_t)std::max(prod_ws_bytes(pl, (int64_t)pl.pg.RG * O->n_p), pre);
    }
    case SR_CALL_ADJOINT: {
      if (O->O_lo != nullptr) return fail(SR_ERR_INVALID, "sr_workspace_bytes: sr_adjoint takes one code plane");
      const int64_t C = adjoint_column_groups(O);
      return (int64_t)std::max((size_t)C * O->n_s * 16 + (size_t)O->n_s * 16 + 1024, pre);
    }
    default: return fail(SR_ERR_INVALID, "sr_workspace_bytes: unknown call %d", call);
  }
}

int sr_workspace_reserve(int64_t bytes, hipStream_t stream) {
  if (bytes < 0) return fail(SR_ERR_INVALID, "sr_workspace_reserve: bytes must be >= 0");
  int dev;
  DeviceInfo di;
  int rc = device_check(&dev, &di);
  if (rc) return rc;
  void *base = nullptr;
  return bytes == 0 ? SR_OK : get_workspace(dev, stream, (size_t)bytes, &base);
}

int sr_timing(int32_t enable) {
  if (enable != 0 && enable != 1) return fail(SR_ERR_INVALID, "sr_timing: enable must be 0 or 1");
  std::lock_guard<std::mutex> lk(g_mu);
  g_timing = TimingTotals{};
  g_timing.on = enable != 0;
  return SR_OK;
}

int sr_timing_read(int32_t cls, double *ms, int64_t *count) {
  if (cls < 0 || cls >= kTimeClasses || ms == nullptr || count == nullptr)
    return fail(SR_ERR_INVALID, "sr_timing_read: bad argument");
  std::lock_guard<std::mutex> lk(g_mu);
  *ms = g_timing.ms[cls];
  *count = g_timing.count[cls];
  return SR_OK;
}

int64_t sr_workspace_held(hipStream_t stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SR_ERR_NODEVICE, "no HIP device available");
  }
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find(std::make_pair(dev, stream));
  return it == g_ws.end() ? 0 : (int64_t)it->second.bytes;
}

int sr_stream_read(const void *p, int64_t bytes, int32_t blocks_per_cu, int32_t unroll, uint32_t *sink,
                   hipStream_t stream) {
  if (p == nullptr || sink == nullptr) return fail(SR_ERR_INVALID, "sr_stream_read: null pointer");
  if (((uintptr_t)p) % 16 || bytes < 16 || bytes % 16)
    return fail(SR_ERR_INVALID, "sr_stream_read: p must be 16-byte aligned and bytes a positive multiple of 16");
  if (blocks_per_cu < 1 || blocks_per_cu > 8) return fail(SR_ERR_INVALID, "sr_stream_read: blocks_per_cu in [1, 8]");
  const void *fn = stream_read_kernel(unroll);
  if (fn == nullptr) return fail(SR_ERR_INVALID, "sr_stream_read: unroll must be 2, 4 or 8");
  int dev;
  DeviceInfo di;
  int rc = device_check(&dev, &di);
  if (rc) return rc;
  const unsigned char *src = (const unsigned char *)p;
  int64_t n_vec = bytes / 16;
  void *args[] = {&src, &n_vec, &sink};
  HIP_TRY(hipLaunchKernel(fn, dim3(di.cus * blocks_per_cu), dim3(512), args, 0, stream));
  return SR_OK;
}

int sr_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = SR_OK;
  for (auto *mp : {&g_ws, &g_mean_ws, &g_batch_ws, &g_lm_ws, &g_shift_ws, &g_stream_ws}) {
    for (auto &kv : *mp) {
      if (kv.second.ptr) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(kv.first.first);
        if (hipFree(kv.second.ptr) != hipSuccess) rc = fail(SR_ERR_HIP, "hipFree failed in sr_release");
        (void)hipSetDevice(cur);
      }
    }
    mp->clear();
  }
  return rc;
}

int sr_set_batch_config(int32_t split_rows, int32_t tasks) {
  if (split_rows == 0 && tasks == 0) {
    g_batch_split_rows = kBatchSplitRows;
    g_batch_tasks = 2;
    return SR_OK;
  }
  if (split_rows < 128 || split_rows > kBatchSplitRows || (split_rows & (split_rows - 1)) != 0)
    return fail(SR_ERR_INVALID, "sr_set_batch_config: split_rows must be a power of two in [128, %d]",
                kBatchSplitRows);
  if (tasks < 1 || tasks > 8) return fail(SR_ERR_INVALID, "sr_set_batch_config: tasks must be in [1, 8]");
  g_batch_split_rows = split_rows;
  g_batch_tasks = tasks;
  return SR_OK;
}

int sr_set_tile_config(int32_t dtype, int32_t kind, int32_t nv, int32_t rows, int32_t lookahead,
                       int32_t poll_delay, int32_t threads, int32_t col_groups) {
  if (nv == 0 && dtype == -1) {
    for (auto &row : g_force)
      for (auto &f : row) f = TileForce{};
    return SR_OK;
  }
  if (dtype < SR_F64 || dtype > SR_F16 || (kind != 0 && kind != 1))
    return fail(SR_ERR_INVALID, "sr_set_tile_config: bad dtype or kind");
  if (nv == 0) {
    g_force[dtype][kind] = TileForce{};
    return SR_OK;
  }
  if (col_groups < 0 || (col_groups & (col_groups - 1)))
    return fail(SR_ERR_INVALID, "sr_set_tile_config: col_groups must be 0 or a power of two");
  bool found = false;
  int count = 0;
  const KernelEntry *tab = kernel_table(dtype, &count);
  for (int i = 0; i < count; ++i)
    if (tab[i].kind == kind && tab[i].nv == nv && tab[i].r == rows && tab[i].look == lookahead &&
        tab[i].poll == poll_delay && tab[i].nt == threads)
      found = true;
  if (!found)
    return fail(SR_ERR_INVALID, "sr_set_tile_config: no kernel built for (%d, %d, %d, %d, %d) of this type and kind",
                nv, rows, lookahead, poll_delay, threads);
  g_force[dtype][kind] = TileForce{nv, rows, lookahead, poll_delay, threads, col_groups};
  return SR_OK;
}

int sr_tile_configs(int32_t dtype, int32_t kind, int32_t *out, int32_t max) {
  if (dtype < SR_F64 || dtype > SR_F16 || (kind != 0 && kind != 1) || max < 0 || (max > 0 && out == nullptr))
    return fail(SR_ERR_INVALID, "sr_tile_configs: bad argument");
  int count = 0, n = 0;
  const KernelEntry *tab = kernel_table(dtype, &count);
  for (int i = 0; i < count; ++i) {
    if (tab[i].kind != kind) continue;
    if (n < max) {
      out[5 * n + 0] = tab[i].nv;
      out[5 * n + 1] = tab[i].r;
      out[5 * n + 2] = tab[i].look;
      out[5 * n + 3] = tab[i].poll;
      out[5 * n + 4] = tab[i].nt;
    }
    n++;
  }
  return n;
}

int sr_grad(const sr_matrix *O, const double *E, double *g, double *E_mean, double *col_mean_out,
            double *diagS_out, hipStream_t stream) {
  int rc = check_matrix(O, "sr_grad");
  if (rc) return rc;
  if (g != nullptr && E == nullptr) return fail(SR_ERR_INVALID, "sr_grad: g requires E");
  if (E_mean != nullptr && E == nullptr) return fail(SR_ERR_INVALID, "sr_grad: E_mean requires E");
  if (g == nullptr && E_mean == nullptr && col_mean_out == nullptr && diagS_out == nullptr)
    return fail(SR_ERR_INVALID, "sr_grad: no output requested");
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  return run_grad(O, E, g, E_mean, col_mean_out, diagS_out, dev, di, stream);
}

static int check_sv_args(const sr_matrix *O, const double *v, double *y, double eps, const char *name) {
  int rc = check_matrix(O, name);
  if (rc) return rc;
  if (v == nullptr || y == nullptr) return fail(SR_ERR_INVALID, "%s: null v or y", name);
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(SR_ERR_INVALID, "%s: eps must be finite and >= 0", name);
  if (ranges_overlap(v, O->n_p * 8, y, O->n_p * 8)) return fail(SR_ERR_INVALID, "%s: v and y overlap", name);
  return SR_OK;
}

// The product's launch over a caller-provided workspace of prod_ws_bytes(pl, RG * n_v).
static int launch_sv(const sr_matrix *O, const double *v, double *y, double eps, const double *mean, const Plan &pl,
                     void *base, hipStream_t stream) {
  const int64_t ypd = (int64_t)pl.pg.RG * pl.pg.n_v;
  Carve cv(base);
  ProdWs w;
  carve_prod(cv, pl, ypd, &w);
  SvArgs a{};
  a.pg = pl.pg;
  a.pb = w.pb;
  a.sb = w.sb;
  a.op = make_operand(O);
  a.mean = mean;
  a.v = v;
  a.y = y;
  a.eps = eps;
  int rc = zero_sync(w, stream);
  if (rc) return rc;
  if (two_planes(O)) {
    if (pl.ke->sv2 == nullptr) return fail(SR_ERR_INVALID, "sr_sv_product: no two-plane kernel for this configuration");
    return launch_coop(pl.ke->sv2, pl.pg.G, &a, stream, pl.ke->nt, 0);
  }
  return launch_coop(pl.ke->sv, pl.pg.G, &a, stream, pl.ke->nt, pl.ke->ring_bytes);
}

int sr_sv_product(const sr_matrix *O, const double *v, double *y, double eps, hipStream_t stream) {
  int rc = check_sv_args(O, v, y, eps, "sr_sv_product");
  if (rc) return rc;
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  const double *mean = nullptr;
  double *mscr = nullptr;
  if (!O->col_mean) {
    rc = get_mean_scratch(dev, stream, O->n_p, &mscr);
    if (rc) return rc;
  }
  rc = ensure_mean(O, mscr, &mean, dev, di, stream);
  if (rc) return rc;
  Plan pl;
  rc = make_plan(O->dtype, di.grid, O->n_s, O->n_p, 1, &pl, streamed_cols(O));
  if (rc) return rc;
  void *base = nullptr;
  rc = get_workspace(dev, stream, prod_ws_bytes(pl, (int64_t)pl.pg.RG * pl.pg.n_v), &base);
  if (rc) return rc;
  return launch_sv(O, v, y, eps, mean, pl, base, stream);
}

int sr_sv_product_noalloc(const sr_matrix *O, const double *v, double *y, double eps, hipStream_t stream) {
  int rc = check_sv_args(O, v, y, eps, "sr_sv_product_noalloc");
  if (rc) return rc;
  if (O->col_mean == nullptr)
    return fail(SR_ERR_INVALID, "sr_sv_product_noalloc: col_mean is required (no pass computes it here)");
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  Plan pl;
  rc = make_plan(O->dtype, di.grid, O->n_s, O->n_p, 1, &pl, streamed_cols(O));
  if (rc) return rc;
  const size_t need = prod_ws_bytes(pl, (int64_t)pl.pg.RG * pl.pg.n_v);
  if (need > kNoAllocScratchBytes)
    return fail(SR_ERR_INVALID, "sr_sv_product_noalloc: this product needs %zu bytes of scratch, more than the %zu "
                                "the library holds", need, kNoAllocScratchBytes);
  void *base = nullptr;
  rc = scratch_address(dev, &base);
  if (rc) return rc;
  return launch_sv(O, v, y, eps, O->col_mean, pl, base, stream);
}

// ------------------------------------------------------------------------------------
// Several right-hand sides, batches of systems
// ------------------------------------------------------------------------------------
int check_batch_matrix(const sr_matrix *m, const char *where) {
  int rc = check_matrix(m, where);
  if (rc) return rc;
  if (m->dtype != SR_F64 && m->dtype != SR_F32)
    return fail(SR_ERR_INVALID, "%s: storage must be SR_F64 or SR_F32", where);
  if (m->O_lo != nullptr) return fail(SR_ERR_INVALID, "%s: a second code plane is not supported", where);
  return SR_OK;
}

int fill_zero(void *p, int64_t words, hipStream_t s) {
  uint32_t v = 0;
  uint32_t *q = (uint32_t *)p;
  void *args[] = {&q, &words, &v};
  const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(words, 256)));
  HIP_TRY(hipLaunchKernel(fill_kernel(), dim3(blocks), dim3(256), args, 0, s));
  return SR_OK;
}

// Geometry of one system's two-pass products (see BatchProduct): about two tasks per
// workgroup in each pass where the shape allows.  The update pass's splits hold at most
// kBatchSplitRows rows (their partials, SP x 8 x N_p float64, stay near 1.6 % of a
// float32 O); shorter splits cost more partial traffic than their balance gains.
BatchGeom batch_geometry(int G, int64_t n_s, int64_t n_p, int vec) {
  BatchGeom g{};
  g.n_s = n_s;
  g.n_p = n_p;
  const int nw = kBatchNT / 64;
  const int64_t cw = 64 * (int64_t)vec, bw = (int64_t)kBatchNT * vec;
  const int64_t target = (int64_t)g_batch_tasks * G;
  g.n_rb = cdiv(n_s, (int64_t)nw * kBatchRows);
  const int64_t max_parts = std::max<int64_t>(1, cdiv(n_p, 4 * cw));   // parts of >= 4 chunks
  const int64_t parts = std::min<int64_t>(max_parts, std::max<int64_t>(1, cdiv(target, g.n_rb)));
  g.pw = round_up(cdiv(n_p, parts), cw);
  g.P = (int)cdiv(n_p, g.pw);
  g.C = (int)cdiv(n_p, bw);
  const int64_t sp = std::max<int64_t>(cdiv(n_s, g_batch_split_rows),
                                       std::min<int64_t>(cdiv(target, g.C), cdiv(n_s, 64)));
  g.rs = cdiv(n_s, sp);
  g.SP = (int)cdiv(n_s, g.rs);
  return g;
}

// Buffer sizes of a batched launch (the largest system sets each).
struct BatchSizes {
  int64_t vstride = 0, wp = 0, yp = 0, swp = 0;
  void add(const BatchGeom &g) {
    vstride = std::max<int64_t>(vstride, g.n_p);
    wp = std::max<int64_t>(wp, (int64_t)g.P * g.n_s * kBatchK);
    yp = std::max<int64_t>(yp, (int64_t)g.SP * kBatchK * g.n_p);
    swp = std::max<int64_t>(swp, (int64_t)g.SP * kBatchK);
  }
};

// Carves the buffers every batched launch uses; the zeroed part (barrier flags, abort
// word) is cleared by a fill kernel.
struct BatchWs {
  BatchArgs a{};
  uint32_t *zero_base = nullptr;
  int64_t zero_words = 0;
};
size_t batch_ws_bytes(int G, const BatchSizes &z) {
  const int K = kBatchK;
  size_t b = 0;
  auto add = [&](size_t n) { b = (size_t)round_up((int64_t)b, 256) + n; };
  add(G * 4);
  add(64 * 4);
  add((size_t)4 * K * G * 8);
  add((size_t)K * z.vstride * 8);
  add((size_t)z.wp * 8);
  add((size_t)z.yp * 8);
  add((size_t)z.swp * 8);
  for (int i = 0; i < 4; ++i) add((size_t)K * z.vstride * 8);
  return b + 256;
}
void carve_batch(Carve &cv, int G, const BatchSizes &z, BatchWs *w) {
  const int K = kBatchK;
  const size_t start = (size_t)round_up((int64_t)cv.off, 256);
  w->a.sb.flags = cv.take<uint32_t>(G);
  w->a.sb.abort = cv.take<uint32_t>(64);
  const size_t end = cv.off;
  w->zero_base = (uint32_t *)(cv.base + start);
  w->zero_words = (int64_t)((end - start + 3) / 4);
  w->a.red = cv.take<double>((int64_t)4 * K * G);
  w->a.vs = cv.take<double>((int64_t)K * z.vstride);
  w->a.wp = cv.take<double>(z.wp);
  w->a.yp = cv.take<double>(z.yp);
  w->a.swp = cv.take<double>(z.swp);
  w->a.x = cv.take<double>((int64_t)K * z.vstride);
  w->a.r = cv.take<double>((int64_t)K * z.vstride);
  w->a.p = cv.take<double>((int64_t)K * z.vstride);
  w->a.q = cv.take<double>((int64_t)K * z.vstride);
  w->a.vstride = z.vstride;
}

int sr_svk_product(const sr_matrix *O, int32_t k, const double *V, const double *eps, double *Y, int32_t exact,
                   hipStream_t stream) {
  int rc = check_batch_matrix(O, "sr_svk_product");
  if (rc) return rc;
  if (k < 1 || k > kBatchK) return fail(SR_ERR_INVALID, "sr_svk_product: k must be in [1, %d]", kBatchK);
  if (V == nullptr || Y == nullptr || eps == nullptr) return fail(SR_ERR_INVALID, "sr_svk_product: null V, Y or eps");
  if (exact != 0 && exact != 1) return fail(SR_ERR_INVALID, "sr_svk_product: exact must be 0 or 1");
  const int64_t n_p = O->n_p;
  if (ranges_overlap(V, k * n_p * 8, Y, k * n_p * 8)) return fail(SR_ERR_INVALID, "sr_svk_product: V and Y overlap");
  for (int i = 0; i < k; ++i)
    if (!(eps[i] >= 0.0) || !std::isfinite(eps[i]))
      return fail(SR_ERR_INVALID, "sr_svk_product: eps must be finite and >= 0");
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  const double *mean = nullptr;
  double *mscr = nullptr;
  if (!O->col_mean) {
    rc = get_mean_scratch(dev, stream, n_p, &mscr);
    if (rc) return rc;
  }
  rc = ensure_mean(O, mscr, &mean, dev, di, stream);
  if (rc) return rc;
  const BatchEntry *be = batched_entry(O->dtype);
  BatchSys S{};
  S.bg = batch_geometry(di.grid, O->n_s, n_p, vec_of(O->dtype));
  BatchSizes z;
  z.add(S.bg);
  S.op = make_operand(O);
  S.mean = mean;
  S.k = k;
  for (int i = 0; i < kBatchK; ++i) S.eps[i] = i < k ? eps[i] : 0.0;
  void *base = nullptr;
  rc = get_workspace(dev, stream, batch_ws_bytes(di.grid, z) + 1024, &base, g_batch_ws);
  if (rc) return rc;
  Carve cv(base);
  BatchWs w;
  carve_batch(cv, di.grid, z, &w);
  BatchSys *table = cv.take<BatchSys>(1);
  // V padded to kBatchK columns in the p buffer, the result in q
  HIP_TRY(hipMemcpyAsync(w.a.p, V, (size_t)k * n_p * 8, hipMemcpyDeviceToDevice, stream));
  if (k < kBatchK) {
    rc = fill_zero(w.a.p + (int64_t)k * n_p, (int64_t)(kBatchK - k) * n_p * 2, stream);
    if (rc) return rc;
  }
  HIP_TRY(hipMemcpyAsync(table, &S, sizeof(S), hipMemcpyHostToDevice, stream));
  w.a.sys = table;
  w.a.n_sys = 1;
  rc = fill_zero(w.zero_base, w.zero_words, stream);
  if (rc) return rc;
  rc = launch_coop(be->sv, di.grid, &w.a, stream, be->nt, 0);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(Y, w.a.q, (size_t)k * n_p * 8, hipMemcpyDeviceToDevice, stream));
  // the host copy of the table must outlive the copy above: wait for it
  HIP_TRY(hipStreamSynchronize(stream));
  return SR_OK;
}

int sr_cg_solve_batched(int32_t n_sys, const sr_batch_system *sys, int32_t k, const sr_cg_opts *opt,
                        sr_cg_info *info, hipStream_t stream) {
  if (n_sys < 1 || sys == nullptr) return fail(SR_ERR_INVALID, "sr_cg_solve_batched: need n_sys >= 1 systems");
  if (k < 1 || k > kBatchK) return fail(SR_ERR_INVALID, "sr_cg_solve_batched: k must be in [1, %d]", kBatchK);
  int64_t max_np = 0;
  for (int s = 0; s < n_sys; ++s) {
    const sr_batch_system &b = sys[s];
    int rc = check_batch_matrix(&b.O, "sr_cg_solve_batched");
    if (rc) return rc;
    if (b.O.dtype != sys[0].O.dtype) return fail(SR_ERR_INVALID, "sr_cg_solve_batched: systems differ in dtype");
    if (b.g == nullptr || b.x == nullptr) return fail(SR_ERR_INVALID, "sr_cg_solve_batched: null g or x");
    if (ranges_overlap(b.g, k * b.O.n_p * 8, b.x, k * b.O.n_p * 8))
      return fail(SR_ERR_INVALID, "sr_cg_solve_batched: g and x overlap");
    for (int i = 0; i < k; ++i)
      if (!(b.eps[i] >= 0.0) || !std::isfinite(b.eps[i]))
        return fail(SR_ERR_INVALID, "sr_cg_solve_batched: eps must be finite and >= 0");
    max_np = std::max<int64_t>(max_np, b.O.n_p);
  }
  sr_cg_opts o{};
  o.rtol = 1e-10;
  if (opt) o = *opt;
  if (!(o.rtol > 0.0) || !std::isfinite(o.rtol)) return fail(SR_ERR_INVALID, "sr_cg_solve_batched: bad rtol");
  if (o.refresh_every < 0) return fail(SR_ERR_INVALID, "sr_cg_solve_batched: refresh_every must be >= 0");
  int64_t max_iter = o.max_iter > 0 ? o.max_iter : max_np + 100;
  if (max_iter > (1 << 30)) max_iter = 1 << 30;
  int dev;
  DeviceInfo di;
  int rc = device_check(&dev, &di);
  if (rc) return rc;
  const int dt = sys[0].O.dtype, vec = vec_of(dt);
  const BatchEntry *be = batched_entry(dt);
  std::vector<BatchSys> host(n_sys);
  BatchSizes z;
  int64_t mean_total = 0;
  for (int s = 0; s < n_sys; ++s) {
    host[s].bg = batch_geometry(di.grid, sys[s].O.n_s, sys[s].O.n_p, vec);
    z.add(host[s].bg);
    if (!sys[s].O.col_mean) mean_total += round_up(sys[s].O.n_p, 32);
  }
  const size_t info_n = (size_t)n_sys * kBatchK * 4 + 1;
  const size_t bytes = batch_ws_bytes(di.grid, z) + (size_t)mean_total * 8 + info_n * 8 +
                       (size_t)n_sys * sizeof(BatchSys) + 4096;
  void *base = nullptr;
  rc = get_workspace(dev, stream, bytes, &base, g_batch_ws);
  if (rc) return rc;
  Carve cv(base);
  double *means = cv.take<double>(std::max<int64_t>(mean_total, 1));
  BatchSys *table = cv.take<BatchSys>(n_sys);
  double *dinfo = cv.take<double>((int64_t)info_n);
  BatchWs w;
  carve_batch(cv, di.grid, z, &w);
  int64_t moff = 0;
  for (int s = 0; s < n_sys; ++s) {
    const sr_batch_system &b = sys[s];
    BatchSys &S = host[s];
    S.op = make_operand(&b.O);
    if (b.O.col_mean) {
      S.mean = b.O.col_mean;
    } else {
      double *m = means + moff;
      moff += round_up(b.O.n_p, 32);
      rc = run_grad(&b.O, nullptr, nullptr, nullptr, m, nullptr, dev, di, stream);
      if (rc) return rc;
      S.mean = m;
    }
    S.g = b.g;
    S.x = b.x;
    S.k = k;
    for (int i = 0; i < kBatchK; ++i) S.eps[i] = i < k ? b.eps[i] : 0.0;
  }
  HIP_TRY(hipMemcpyAsync(table, host.data(), (size_t)n_sys * sizeof(BatchSys), hipMemcpyHostToDevice, stream));
  w.a.sys = table;
  w.a.n_sys = n_sys;
  w.a.rtol = o.rtol;
  w.a.max_iter = (int)max_iter;
  w.a.refresh_every = o.refresh_every;
  // optional extra refreshes once the residual fell by refresh_drop since the last one
  if (!(o.refresh_drop >= 0.0 && o.refresh_drop < 1.0))
    return fail(SR_ERR_INVALID, "sr_cg_solve_batched: refresh_drop must be in [0, 1)");
  w.a.refresh_drop2 = o.refresh_drop * o.refresh_drop;
  w.a.info = dinfo;
  rc = fill_zero(w.zero_base, w.zero_words, stream);
  if (rc) return rc;
  rc = fill_zero(dinfo, (int64_t)info_n * 2, stream);
  if (rc) return rc;
  rc = launch_coop(be->cg, di.grid, &w.a, stream, be->nt, 0);
  if (rc) return rc;
  std::vector<double> hinfo(info_n);
  uint32_t habort = 0;
  HIP_TRY(hipMemcpyAsync(hinfo.data(), dinfo, info_n * 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&habort, w.a.sb.abort, sizeof(habort), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (habort != 0u || hinfo[info_n - 1] == 0.0)
    return fail(SR_ERR_TIMEOUT, "sr_cg_solve_batched: a cross-workgroup wait timed out");
  int status = SR_OK;
  for (int s = 0; s < n_sys; ++s)
    for (int i = 0; i < k; ++i) {
      const double *h = &hinfo[((size_t)s * kBatchK + i) * 4];
      const int st = (int)h[1];
      if (info) {
        sr_cg_info &ci = info[(size_t)s * k + i];
        ci.iters = (int32_t)h[0];
        ci.refreshes = 0;
        ci.status = st;
        ci.products = (int32_t)h[3];
        ci.rel_res_recur = h[2];
        ci.rel_res_true = h[2];
      }
      if (status == SR_OK && st != SR_OK) status = st;
    }
  if (status < 0) return fail(status, "sr_cg_solve_batched: a column reported %s", sr_status_string(status));
  return status;
}

int lm_davidson(const sr_matrix *O, const double *E, const sr_matrix *D, const lm_davidson_opts *opt, double *c,
                lm_davidson_info *info, hipStream_t stream) {
  int rc = check_matrix(O, "lm_davidson(O)");
  if (rc) return rc;
  rc = check_matrix(D, "lm_davidson(D)");
  if (rc) return rc;
  if (D->n_s != O->n_s || D->n_p != O->n_p || D->dtype != O->dtype)
    return fail(SR_ERR_INVALID, "lm_davidson: O and D must have the same n_s, n_p and dtype");
  if (O->O_lo != nullptr || D->O_lo != nullptr)
    return fail(SR_ERR_INVALID, "lm_davidson: a second code plane is not supported");
  if (E == nullptr || c == nullptr || info == nullptr) return fail(SR_ERR_INVALID, "lm_davidson: null E, c or info");
  lm_davidson_opts o{1e-8, 1000, 40, 0, 0};
  if (opt) o = *opt;
  if (o.precond < 0 || o.precond > 2) return fail(SR_ERR_INVALID, "lm_davidson: precond must be 0, 1 or 2");
  if (o.reserved != 0) return fail(SR_ERR_INVALID, "lm_davidson: reserved must be 0");
  if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return fail(SR_ERR_INVALID, "lm_davidson: tol must be finite and > 0");
  if (o.max_iter < 1) return fail(SR_ERR_INVALID, "lm_davidson: max_iter must be >= 1");
  if (o.max_sub < 2 || o.max_sub > kLmMaxSub)
    return fail(SR_ERR_INVALID, "lm_davidson: max_sub must be in [2, %d]", kLmMaxSub);
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  const int64_t n_p = O->n_p, n = n_p + 1, ld = round_up(n, 32);
  const int ms = o.max_sub;
  const int nb = std::min(di.grid, (int)std::max<int64_t>(1, cdiv(n, 4096)));
  // V, HV, SV [ms][ld]; r, c-temporaries [3][ld]; column means [ld]; reduction buffers
  const int sp_h = (int)std::min<int64_t>(64, std::max<int64_t>(1, cdiv(O->n_s, 128)));   // diag H splits
  const size_t bytes = ((size_t)3 * ms + 6) * ld * 8 + ((size_t)nb + 4) * kLmMaxSub * 8 +
                       (o.precond == 2 ? (size_t)sp_h * n_p * 8 : 0) + 4096;
  void *base = nullptr;
  rc = get_workspace(dev, stream, bytes, &base, g_lm_ws);
  if (rc) return rc;
  Carve cv(base);
  double *V = cv.take<double>((int64_t)ms * ld), *HV = cv.take<double>((int64_t)ms * ld);
  double *SV = cv.take<double>((int64_t)ms * ld);
  double *R = cv.take<double>(ld), *T1 = cv.take<double>(ld), *T2 = cv.take<double>(ld);
  double *mean = cv.take<double>(ld), *dvec = cv.take<double>(ld), *dhvec = cv.take<double>(ld);
  double *hpart = o.precond == 2 ? cv.take<double>((int64_t)sp_h * n_p) : nullptr;
  LmBufs lb{cv.take<double>((int64_t)nb * kLmMaxSub), cv.take<double>(4 * kLmMaxSub), nb};
  // device results read back together once per new direction: its column and row of the
  // projected matrix and its S-norm before scaling (the Gram-Schmidt coefficients use
  // lb.dots[0, kLmMaxSub) and never leave the device)
  double *d_col = lb.dots + kLmMaxSub, *d_row = lb.dots + 2 * kLmMaxSub, *d_nrm = lb.dots + 3 * kLmMaxSub;
  // the column means once, so that the products do not recompute them; for the diagonal
  // correction dvec = (1, diag S) and, for the exact one, dhvec = (<E>, diag H)
  sr_matrix Om = *O, Dm = *D;
  if (!O->col_mean || o.precond) {
    rc = run_grad(O, o.precond == 2 ? E : nullptr, nullptr, o.precond == 2 ? dhvec : nullptr, mean,
                  o.precond ? dvec + 1 : nullptr, dev, di, stream);
    if (rc) return rc;
    if (!O->col_mean) Om.col_mean = mean;
  }
  if (o.precond) {
    const double one = 1.0;
    HIP_TRY(hipMemcpyAsync(dvec, &one, 8, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
  }
  if (o.precond == 2) {
    DiagHArgs ha{};
    ha.o = make_operand(O);
    ha.d = make_operand(D);
    ha.mean = Om.col_mean;
    ha.E = E;
    ha.n_s = O->n_s;
    ha.n_p = n_p;
    ha.rs = cdiv(O->n_s, sp_h);
    ha.SP = (int)cdiv(O->n_s, ha.rs);
    ha.part = hpart;
    ha.out = dhvec + 1;
    void *hargs[] = {&ha};
    const unsigned cb = (unsigned)cdiv(n_p, lm_threads());
    HIP_TRY(hipLaunchKernel(diagh_part_kernel(O->dtype), dim3(cb, (unsigned)ha.SP), dim3(lm_threads()), hargs, 0,
                            stream));
    HIP_TRY(hipLaunchKernel(diagh_final_kernel(), dim3(cb), dim3(lm_threads()), hargs, 0, stream));
  }
  // the next direction from a residual: itself, or its diagonal correction
  auto correction = [&](const double *r, double *t, double th) -> int {
    if (!o.precond) {
      if (r != t) HIP_TRY(hipMemcpyAsync(t, r, (size_t)n * 8, hipMemcpyDeviceToDevice, stream));
      return SR_OK;
    }
    DivArgs a{r, o.precond == 2 ? dhvec : nullptr, dvec, t, n, th};
    void *args[] = {&a};
    const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(n, lm_threads())));
    HIP_TRY(hipLaunchKernel(divide_kernel(), dim3(blocks), dim3(lm_threads()), args, 0, stream));
    return SR_OK;
  };
  auto row = [&](double *B, int i) { return B + (int64_t)i * ld; };
  // S t = (t_0, (S_c) t_1..n_p)
  auto s_product = [&](const double *t, double *st) -> int {
    HIP_TRY(hipMemcpyAsync(st, t, 8, hipMemcpyDeviceToDevice, stream));
    return sr_sv_product(&Om, t + 1, st + 1, 0.0, stream);
  };
  std::vector<double> A((size_t)ms * ms, 0.0), y, tmp(ms);
  int m = 0, iters = 0, restarts = 0, status = SR_NOT_CONVERGED;
  double theta = 0.0, rnorm = INFINITY, ref_norm = 1.0;
  // start vector: Psi, c = e_0 (S-norm 1)
  rc = fill_zero(row(V, 0), ld * 2, stream);
  if (rc) return rc;
  {
    const double one = 1.0;
    HIP_TRY(hipMemcpyAsync(row(V, 0), &one, 8, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
  }
  while (iters < o.max_iter) {
    // row(V, m) holds the new direction: S-orthonormalize it, then its H and S products
    double *t = row(V, m), *st = row(SV, m), *ht = row(HV, m);
    {
      rc = s_product(t, st);
      if (rc) return rc;
      iters++;
      // S-orthogonalize against the basis (classical Gram-Schmidt, twice); S t follows
      // by linearity.  The coefficients and the norm stay on the device: the host waits
      // once per direction, for the new row and column of the projected matrix.
      for (int pass = 0; pass < 2 && m > 0; ++pass) {
        rc = lm_mdot_dev(lb, SV, ld, m, t, n, lb.dots, stream);
        if (rc) return rc;
        rc = lm_lincomb_dev(V, lb.dots, -1.0, m, nullptr, ld, 1.0, t, n, stream);
        if (rc) return rc;
        rc = lm_lincomb_dev(SV, lb.dots, -1.0, m, nullptr, ld, 1.0, st, n, stream);
        if (rc) return rc;
      }
      rc = lm_mdot_dev(lb, t, ld, 1, st, n, d_nrm, stream);
      if (rc) return rc;
      rc = lm_lincomb_dev(nullptr, nullptr, 0.0, 0, d_nrm, ld, 0.0, t, n, stream);
      if (rc) return rc;
      rc = lm_lincomb_dev(nullptr, nullptr, 0.0, 0, d_nrm, ld, 0.0, st, n, stream);
      if (rc) return rc;
      rc = lm_hv_product(&Om, E, &Dm, t, ht, stream);
      if (rc) return rc;
      // the new row and column of the projected matrix A = V^T H V
      rc = lm_mdot_dev(lb, V, ld, m + 1, ht, n, d_col, stream);
      if (rc) return rc;
      rc = lm_mdot_dev(lb, HV, ld, m + 1, t, n, d_row, stream);
      if (rc) return rc;
      std::vector<double> back((size_t)3 * kLmMaxSub);
      HIP_TRY(hipMemcpyAsync(back.data(), d_col, back.size() * 8, hipMemcpyDeviceToHost, stream));
      HIP_TRY(hipStreamSynchronize(stream));
      const double nrm2 = back[2 * kLmMaxSub];
      if (m == 0) ref_norm = nrm2;
      // no new direction (converged or S singular there): its scaled copy and products are
      // dropped with it
      if (!(nrm2 > 1e-28 * ref_norm)) break;
      for (int i = 0; i <= m; ++i) {
        A[(size_t)i * ms + m] = back[i];
        A[(size_t)m * ms + i] = back[kLmMaxSub + i];
      }
      m++;
    }
    std::vector<double> Am((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) Am[(size_t)i * m + j] = A[(size_t)i * ms + j];
    if (!lowest_eigenpair(Am, m, &theta, y)) {
      status = SR_BREAKDOWN;                 // the projected eigenproblem's QR did not converge
      break;
    }
    // Ritz residual r = H c - theta S c
    for (int i = 0; i < m; ++i) tmp[i] = -theta * y[i];
    rc = lm_lincomb(HV, y.data(), m, SV, tmp.data(), m, ld, 0.0, R, n, stream);
    if (rc) return rc;
    double rr = 0.0;
    rc = lm_mdot(lb, R, ld, 1, R, n, &rr, stream);
    if (rc) return rc;
    rnorm = std::sqrt(rr);
    if (rnorm <= o.tol * std::abs(theta)) {
      status = SR_OK;
      break;
    }
    if (m == ms) {
      // restart from the Ritz vector: V = [c], HV = [H c], SV = [S c] (y has unit norm, so
      // c^T S c = 1)
      rc = lm_lincomb(V, y.data(), m, nullptr, nullptr, 0, ld, 0.0, T1, n, stream);
      if (rc) return rc;
      rc = lm_lincomb(HV, y.data(), m, nullptr, nullptr, 0, ld, 0.0, T2, n, stream);
      if (rc) return rc;
      rc = lm_lincomb(SV, y.data(), m, nullptr, nullptr, 0, ld, 0.0, R, n, stream);
      if (rc) return rc;
      HIP_TRY(hipMemcpyAsync(row(V, 0), T1, (size_t)n * 8, hipMemcpyDeviceToDevice, stream));
      HIP_TRY(hipMemcpyAsync(row(HV, 0), T2, (size_t)n * 8, hipMemcpyDeviceToDevice, stream));
      HIP_TRY(hipMemcpyAsync(row(SV, 0), R, (size_t)n * 8, hipMemcpyDeviceToDevice, stream));
      double a00 = 0.0;
      rc = lm_mdot(lb, V, ld, 1, row(HV, 0), n, &a00, stream);
      if (rc) return rc;
      A.assign((size_t)ms * ms, 0.0);
      A[0] = a00;
      m = 1;
      restarts++;
      // the new direction: the residual of the restarted Ritz pair, H c - a00 S c
      y.assign(1, 1.0);
      tmp[0] = -a00;
      rc = lm_lincomb(HV, y.data(), 1, SV, tmp.data(), 1, ld, 0.0, row(V, 1), n, stream);
      if (rc) return rc;
      rc = correction(row(V, 1), row(V, 1), a00);
      if (rc) return rc;
      continue;
    }
    // next direction: the residual or its correction
    rc = correction(R, row(V, m), theta);
    if (rc) return rc;
  }
  // c = V y (the last Ritz vector)
  if (y.empty()) {
    y.assign(1, 1.0);
    m = std::max(m, 1);
  }
  rc = lm_lincomb(V, y.data(), std::min<int>(m, (int)y.size()), nullptr, nullptr, 0, ld, 0.0, c, n, stream);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(stream));
  info->iters = iters;
  info->restarts = restarts;
  info->status = status;
  info->reserved = 0;
  info->theta = theta;
  info->res_norm = rnorm;
  return status;
}

// Checks of one multi-shift system; its shifts sorted by eps into order.
static int check_shift_system(const char *name, const sr_matrix *O, const double *g, int32_t k, const double *eps,
                              const double *X, std::vector<int> &order) {
  int rc = check_matrix(O, name);
  if (rc) return rc;
  if (O->O_lo != nullptr || (O->dtype != SR_F64 && O->dtype != SR_F32))
    return fail(SR_ERR_INVALID, "%s: storage must be SR_F64 or SR_F32, one plane", name);
  if (k < 1 || k > kMaxShifts) return fail(SR_ERR_INVALID, "%s: k must be in [1, %d]", name, kMaxShifts);
  if (g == nullptr || X == nullptr || eps == nullptr) return fail(SR_ERR_INVALID, "%s: null g, X or eps", name);
  if (ranges_overlap(g, O->n_p * 8, X, (int64_t)k * O->n_p * 8)) return fail(SR_ERR_INVALID, "%s: g and X overlap", name);
  for (int i = 0; i < k; ++i)
    if (!(eps[i] >= 0.0) || !std::isfinite(eps[i])) return fail(SR_ERR_INVALID, "%s: eps must be finite and >= 0", name);
  // shifts in increasing order: the smallest drives the Krylov sequence
  order.resize(k);
  for (int i = 0; i < k; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return eps[a] < eps[b]; });
  return SR_OK;
}

static int check_shift_opts(const char *name, const sr_cg_opts *opt, sr_cg_opts &o) {
  o = sr_cg_opts{};
  o.rtol = 1e-10;
  if (opt) o = *opt;
  if (!(o.rtol > 0.0) || !std::isfinite(o.rtol)) return fail(SR_ERR_INVALID, "%s: bad rtol", name);
  if (o.refresh_every < 0) return fail(SR_ERR_INVALID, "%s: refresh_every must be >= 0", name);
  return SR_OK;
}

// Outcome of the shifts of one system from its kernel info (hs: 2 k per-shift words, status,
// ok, products, then k true residuals); a shift that missed rtol continues with sr_cg_solve
// from its x (warm start).  Returns the first non-OK status or an error code.
static int finish_shifts(const char *name, const sr_matrix *Om, const double *g, int32_t k, const double *eps,
                         double *X, const std::vector<int> &order, const double *hs, const sr_cg_opts &o,
                         sr_cg_info *info, hipStream_t stream) {
  if (hs[2 * k + 1] == 0.0) return fail(SR_ERR_TIMEOUT, "%s: a cross-workgroup wait timed out", name);
  const int kstatus = (int)hs[2 * k];
  const int launch_products = (int)hs[2 * k + 2];
  int status = kstatus < 0 ? kstatus : SR_OK;
  for (int s = 0; s < k && status >= 0; ++s) {
    const int i = order[s];
    double *xi = X + (int64_t)i * Om->n_p;
    const double rel = hs[2 * k + 3 + s];
    sr_cg_info ci{};
    ci.iters = (int32_t)hs[2 * s];
    ci.products = launch_products;
    ci.rel_res_recur = hs[2 * s + 1];
    ci.rel_res_true = rel;
    ci.status = SR_OK;
    if (!(rel <= o.rtol)) {
      sr_cg_opts po = o;
      po.use_x0 = 1;
      po.precond = 0;
      po.search_f64 = 0;
      po.res_history = nullptr;
      if (po.refresh_every == 0) po.refresh_every = 20;
      sr_cg_info pi{};
      const int prc = sr_cg_solve(Om, g, eps[i], xi, &po, &pi, stream);
      if (prc < 0) return prc;
      ci.iters += pi.iters;
      ci.refreshes = pi.refreshes;
      ci.products += pi.products;
      ci.rel_res_recur = pi.rel_res_recur;
      ci.rel_res_true = pi.rel_res_true;
      ci.status = prc;
    }
    if (info) info[i] = ci;
    if (status == SR_OK && ci.status != SR_OK) status = ci.status;
  }
  return status;
}

constexpr int kShiftInfoWords = 3 * kMaxShifts + 4;

// Argument block of one multi-shift system over the shared product buffers.
static void shift_args(ShiftArgs &sa, const Plan &pl, const ProdWs &w, const sr_matrix &Om, const double *g,
                       int32_t k, const double *eps, double *X, const std::vector<int> &order, double *r,
                       double *p, double *q, double *ps, double *sinfo, const sr_cg_opts &o, int64_t max_iter) {
  sa = ShiftArgs{};
  CgArgs &a = sa.c;
  a.pg = pl.pg;
  a.pb = w.pb;
  a.sb = w.sb;
  a.op = make_operand(&Om);
  a.mean = Om.col_mean;
  a.g = g;
  a.x = nullptr;
  a.r = r;
  a.p = p;
  a.q = q;
  a.eps = eps[order[0]];
  a.rtol = o.rtol;
  a.max_iter = (int)max_iter;
  sa.n_shift = k;
  sa.check = 1;
  for (int s = 0; s < kMaxShifts; ++s) {
    sa.dshift[s] = s < k ? eps[order[s]] - eps[order[0]] : 0.0;
    sa.xrow[s] = s < k ? X + (int64_t)order[s] * Om.n_p : nullptr;
  }
  sa.ps = ps;
  sa.sinfo = sinfo;
}

int sr_cg_solve_shifts(const sr_matrix *O, const double *g, int32_t k, const double *eps, double *X,
                       const sr_cg_opts *opt, sr_cg_info *info, hipStream_t stream) {
  const char *name = "sr_cg_solve_shifts";
  std::vector<int> order;
  int rc = check_shift_system(name, O, g, k, eps, X, order);
  if (rc) return rc;
  sr_cg_opts o;
  rc = check_shift_opts(name, opt, o);
  if (rc) return rc;
  const int64_t n_p = O->n_p;
  int64_t max_iter = o.max_iter > 0 ? o.max_iter : n_p + 100;
  if (max_iter > (1 << 30)) max_iter = 1 << 30;
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  // own buffers: the directions of the shifts, the means, the kernel's info
  const int64_t ld = round_up(n_p, 32);
  const size_t own = ((size_t)k + 1) * ld * 8 + (size_t)kShiftInfoWords * 8 + 1024;
  void *obase = nullptr;
  rc = get_workspace(dev, stream, own, &obase, g_shift_ws);
  if (rc) return rc;
  Carve oc(obase);
  double *ps = oc.take<double>((int64_t)k * ld), *mbuf = oc.take<double>(ld);
  double *sinfo = oc.take<double>(kShiftInfoWords);
  sr_matrix Om = *O;
  if (!O->col_mean) {
    rc = run_grad(O, nullptr, nullptr, nullptr, mbuf, nullptr, dev, di, stream);
    if (rc) return rc;
    Om.col_mean = mbuf;
  }
  Plan pl;
  rc = make_plan(O->dtype, di.grid, O->n_s, n_p, 1, &pl);
  if (rc) return rc;
  const void *fn = shift_kernel(O->dtype, pl.ke->nv, pl.ke->r, pl.ke->look, pl.ke->poll, pl.ke->nt);
  if (fn == nullptr) return fail(SR_ERR_INVALID, "%s: no multi-shift kernel for this configuration", name);
  const int64_t ypd = (int64_t)pl.pg.RG * n_p;
  const size_t bytes = prod_ws_bytes(pl, ypd) + (size_t)3 * (n_p * 8 + 256) + 1024;
  void *base = nullptr;
  rc = get_workspace(dev, stream, bytes, &base);
  if (rc) return rc;
  Carve cv(base);
  ProdWs w;
  carve_prod(cv, pl, ypd, &w);
  double *r = cv.take<double>(n_p), *p = cv.take<double>(n_p), *q = cv.take<double>(n_p);
  ShiftArgs sa;
  shift_args(sa, pl, w, Om, g, k, eps, X, order, r, p, q, ps, sinfo, o, max_iter);
  rc = zero_sync(w, stream);
  if (rc) return rc;
  rc = launch_coop(fn, pl.pg.G, &sa, stream, pl.ke->nt, pl.ke->ring_bytes);
  if (rc) return rc;
  std::vector<double> hs(kShiftInfoWords);
  uint32_t habort = 0;
  HIP_TRY(hipMemcpyAsync(hs.data(), sinfo, hs.size() * 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&habort, w.sb.abort, sizeof(habort), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (habort != 0u) return fail(SR_ERR_TIMEOUT, "%s: a cross-workgroup wait timed out", name);
  const int status = finish_shifts(name, &Om, g, k, eps, X, order, hs.data(), o, info, stream);
  HIP_TRY(hipStreamSynchronize(stream));
  if (status < 0) return fail(status, "%s: %s", name, sr_status_string(status));
  return status;
}

int sr_cg_solve_shifts_batched(int32_t n_sys, const sr_shift_system *sys, int32_t k, const sr_cg_opts *opt,
                               sr_cg_info *info, hipStream_t stream) {
  const char *name = "sr_cg_solve_shifts_batched";
  if (n_sys < 1 || sys == nullptr) return fail(SR_ERR_INVALID, "%s: need n_sys >= 1 systems", name);
  std::vector<std::vector<int>> orders(n_sys);
  int64_t max_np = 0;
  for (int i = 0; i < n_sys; ++i) {
    int rc = check_shift_system(name, &sys[i].O, sys[i].g, k, sys[i].eps, sys[i].X, orders[i]);
    if (rc) return rc;
    if (sys[i].O.dtype != sys[0].O.dtype) return fail(SR_ERR_INVALID, "%s: every system needs the same dtype", name);
    max_np = std::max<int64_t>(max_np, sys[i].O.n_p);
  }
  sr_cg_opts o;
  int rc = check_shift_opts(name, opt, o);
  if (rc) return rc;
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  const int dt = sys[0].O.dtype;
  // plans: one tile configuration for all (the kernel is instantiated per configuration),
  // each system its own geometry
  std::vector<Plan> pls(n_sys);
  size_t prod_bytes = 0;
  for (int i = 0; i < n_sys; ++i) {
    rc = make_plan(dt, di.grid, sys[i].O.n_s, sys[i].O.n_p, 1, &pls[i]);
    if (rc) return rc;
    if (pls[i].ke != pls[0].ke) return fail(SR_ERR_HIP, "%s: inconsistent tile choice", name);
    prod_bytes = std::max(prod_bytes, prod_ws_bytes(pls[i], (int64_t)pls[i].pg.RG * sys[i].O.n_p));
  }
  const Plan &p0 = pls[0];
  const void *fn = shift_kernel(dt, p0.ke->nv, p0.ke->r, p0.ke->look, p0.ke->poll, p0.ke->nt, true);
  if (fn == nullptr) return fail(SR_ERR_INVALID, "%s: no multi-shift kernel for this configuration", name);
  // own buffers: means of the systems without them, infos, the argument table
  int64_t mean_total = 0;
  for (int i = 0; i < n_sys; ++i)
    if (!sys[i].O.col_mean) mean_total += round_up(sys[i].O.n_p, 32);
  const size_t own = (size_t)mean_total * 8 + (size_t)n_sys * kShiftInfoWords * 8 +
                     (size_t)n_sys * (sizeof(ShiftArgs) + 256) + 4096;
  void *obase = nullptr;
  rc = get_workspace(dev, stream, own, &obase, g_shift_ws);
  if (rc) return rc;
  Carve oc(obase);
  double *means = oc.take<double>(std::max<int64_t>(mean_total, 1));
  double *sinfo = oc.take<double>((int64_t)n_sys * kShiftInfoWords);
  ShiftArgs *table = oc.take<ShiftArgs>(n_sys);
  std::vector<sr_matrix> Oms(n_sys);
  int64_t moff = 0;
  for (int i = 0; i < n_sys; ++i) {
    Oms[i] = sys[i].O;
    if (!sys[i].O.col_mean) {
      rc = run_grad(&sys[i].O, nullptr, nullptr, nullptr, means + moff, nullptr, dev, di, stream);
      if (rc) return rc;
      Oms[i].col_mean = means + moff;
      moff += round_up(sys[i].O.n_p, 32);
    }
  }
  // product buffers shared by the systems (one after another): the zeroed region (flags,
  // abort, exchange ring), reductions and sink sit at the same place for every geometry;
  // the vectors r, p, q and the shifts' directions are each system's own (chunked per
  // system, so a shared vector would be written by different XCDs with plain stores)
  int64_t vec_total = 0;
  for (int i = 0; i < n_sys; ++i) vec_total += (int64_t)(3 + k) * round_up(sys[i].O.n_p, 32) + 64;
  void *base = nullptr;
  rc = get_workspace(dev, stream, round_up((int64_t)prod_bytes, 256) + (size_t)vec_total * 8 + 4096, &base);
  if (rc) return rc;
  std::vector<ShiftArgs> hsa(n_sys);
  ProdWs w0;
  Carve vc((char *)base + round_up((int64_t)prod_bytes, 256));
  for (int i = 0; i < n_sys; ++i) {
    Carve cv(base);
    ProdWs w;
    carve_prod(cv, pls[i], (int64_t)pls[i].pg.RG * sys[i].O.n_p, &w);
    if (i == 0) w0 = w;
    if (w.sb.flags != w0.sb.flags || w.pb.xchg != w0.pb.xchg || w.sb.red != w0.sb.red)
      return fail(SR_ERR_HIP, "%s: inconsistent buffer layout", name);
    const int64_t ld = round_up(sys[i].O.n_p, 32);
    double *r = vc.take<double>(ld), *p = vc.take<double>(ld), *q = vc.take<double>(ld);
    double *ps = vc.take<double>((int64_t)k * ld);
    int64_t max_iter = o.max_iter > 0 ? o.max_iter : sys[i].O.n_p + 100;
    if (max_iter > (1 << 30)) max_iter = 1 << 30;
    shift_args(hsa[i], pls[i], w, Oms[i], sys[i].g, k, sys[i].eps, sys[i].X, orders[i], r, p, q, ps,
               sinfo + (int64_t)i * kShiftInfoWords, o, max_iter);
  }
  rc = zero_sync(w0, stream);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(table, hsa.data(), (size_t)n_sys * sizeof(ShiftArgs), hipMemcpyHostToDevice, stream));
  {
    const ShiftArgs *tp = table;
    int32_t n = n_sys;
    void *args[] = {(void *)&tp, (void *)&n};
    if (p0.ke->ring_bytes > 0)
      HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, p0.ke->ring_bytes));
    TimedLaunch tl(stream);
    HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(p0.pg.G), dim3(p0.ke->nt), args, (unsigned)p0.ke->ring_bytes, stream));
    tl.stop();
    tl.record(kTimeSolveLaunch);
  }
  std::vector<double> hs((size_t)n_sys * kShiftInfoWords);
  uint32_t habort = 0;
  HIP_TRY(hipMemcpyAsync(hs.data(), sinfo, hs.size() * 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&habort, w0.sb.abort, sizeof(habort), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (habort != 0u) return fail(SR_ERR_TIMEOUT, "%s: a cross-workgroup wait timed out", name);
  int status = SR_OK;
  for (int i = 0; i < n_sys; ++i) {
    const int st = finish_shifts(name, &Oms[i], sys[i].g, k, sys[i].eps, sys[i].X, orders[i],
                                 hs.data() + (size_t)i * kShiftInfoWords, o, info ? info + (int64_t)i * k : nullptr,
                                 stream);
    if (st < 0) return fail(st, "%s: system %d: %s", name, i, sr_status_string(st));
    if (status == SR_OK && st != SR_OK) status = st;
  }
  HIP_TRY(hipStreamSynchronize(stream));
  return status;
}

int sr_adjoint(const sr_matrix *O, const double *E, const double *x, const double *lam, double *dE, void *dO,
               int32_t dO_dtype, int64_t ld_dO, double *p12, double *deps, hipStream_t stream) {
  int rc = check_matrix(O, "sr_adjoint");
  if (rc) return rc;
  if (deps != nullptr && (ranges_overlap(deps, 8, x, O->n_p * 8) || ranges_overlap(deps, 8, lam, O->n_p * 8)))
    return fail(SR_ERR_INVALID, "sr_adjoint: deps overlaps x or lam");
  if (dO == nullptr && dE == nullptr && p12 == nullptr) {
    // dL/deps alone: no pass over O
    if (x == nullptr || lam == nullptr) return fail(SR_ERR_INVALID, "sr_adjoint: null x or lam");
    if (deps == nullptr) return fail(SR_ERR_INVALID, "sr_adjoint: no output requested");
    int dev;
    DeviceInfo di;
    rc = device_check(&dev, &di);
    if (rc) return rc;
    AdjFinishArgs fa{};
    fa.x = x;
    fa.lam = lam;
    fa.n_p = O->n_p;
    fa.deps = deps;
    void *args[] = {&fa};
    HIP_TRY(hipLaunchKernel(adjoint_finish_kernel(), dim3(1), dim3(1024), args, 0, stream));
    return SR_OK;
  }
  if (O->O_lo != nullptr) return fail(SR_ERR_INVALID, "sr_adjoint: a second code plane is not supported");
  if (E == nullptr || x == nullptr || lam == nullptr) return fail(SR_ERR_INVALID, "sr_adjoint: null E, x or lam");
  const int64_t n_s = O->n_s, n_p = O->n_p;
  if (dO != nullptr) {
    if (dO_dtype != SR_F64 && dO_dtype != SR_F32)
      return fail(SR_ERR_INVALID, "sr_adjoint: dO_dtype must be SR_F64 or SR_F32");
    const int64_t eb = dO_dtype == SR_F64 ? 8 : 4;
    if (ld_dO < n_p || ((uintptr_t)dO % 16) != 0 || (ld_dO * eb) % 16 != 0)
      return fail(SR_ERR_INVALID, "sr_adjoint: dO needs ld_dO >= n_p and 16-byte aligned rows");
    const int64_t nb = ((n_s - 1) * ld_dO + n_p) * eb;
    if (ranges_overlap(dO, nb, O->O, n_s * O->ld * elem_bytes(O->dtype)) || ranges_overlap(dO, nb, x, n_p * 8) ||
        ranges_overlap(dO, nb, lam, n_p * 8) || ranges_overlap(dO, nb, E, n_s * 8) ||
        (dE != nullptr && ranges_overlap(dO, nb, dE, n_s * 8)))
      return fail(SR_ERR_INVALID, "sr_adjoint: dO overlaps another argument");
  }
  if (dE != nullptr && (ranges_overlap(dE, n_s * 8, E, n_s * 8) || ranges_overlap(dE, n_s * 8, x, n_p * 8) ||
                        ranges_overlap(dE, n_s * 8, lam, n_p * 8)))
    return fail(SR_ERR_INVALID, "sr_adjoint: dE overlaps another argument");
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  const double *mean = nullptr;
  double *mscr = nullptr;
  if (!O->col_mean) {
    rc = get_mean_scratch(dev, stream, n_p, &mscr);
    if (rc) return rc;
  }
  rc = ensure_mean(O, mscr, &mean, dev, di, stream);
  if (rc) return rc;
  // row dots: column groups of NV 16-byte vectors per thread, about 2048 workgroups
  const int vec = vec_of(O->dtype), nt = adjoint_threads(), rr = adjoint_rows_per_block();
  const int nv = adjoint_nv(O);
  const int C = (int)adjoint_column_groups(O);
  const int RG = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(n_s, rr), std::max<int64_t>(1, 2048 / C)));
  void *base = nullptr;
  rc = get_workspace(dev, stream, (size_t)C * n_s * 16 + (size_t)n_s * 16 + 1024, &base);
  if (rc) return rc;
  Carve cv(base);
  RowDotsArgs ra{};
  ra.O = (const unsigned char *)O->O;
  ra.ldb = O->ld * elem_bytes(O->dtype);
  ra.scale = O->col_scale;
  ra.mean = mean;
  ra.x = x;
  ra.lam = lam;
  ra.n_s = n_s;
  ra.n_p = n_p;
  ra.wslice = round_up(cdiv(n_p, C), vec);
  ra.C = C;
  ra.RG = RG;
  ra.part = cv.take<double>((int64_t)C * n_s * 2);
  {
    void *args[] = {&ra};
    HIP_TRY(hipLaunchKernel(rowdots_kernel(O->dtype, nv), dim3((unsigned)((int64_t)C * RG)), dim3(nt), args, 0,
                            stream));
  }
  AdjFinishArgs fa{};
  fa.E = E;
  fa.part = ra.part;
  fa.n_s = n_s;
  fa.C = C;
  fa.coef = cv.take<double>(2 * n_s);
  fa.dE = dE;
  fa.p12 = p12;
  fa.x = x;
  fa.lam = lam;
  fa.n_p = n_p;
  fa.deps = deps;
  {
    void *args[] = {&fa};
    HIP_TRY(hipLaunchKernel(adjoint_finish_kernel(), dim3(1), dim3(1024), args, 0, stream));
  }
  if (dO != nullptr) {
    Rank2Args wa{};
    wa.coef = fa.coef;
    wa.lam = lam;
    wa.x = x;
    wa.n_s = n_s;
    wa.n_p = n_p;
    wa.ld = ld_dO;
    wa.dO = dO;
    const int W = dO_dtype == SR_F64 ? 2 : 4;
    const unsigned bx = (unsigned)cdiv(n_p, (int64_t)nt * W);
    const unsigned by = (unsigned)std::min<int64_t>(n_s, std::max<int64_t>(1, 16384 / (int64_t)bx));
    void *args[] = {&wa};
    HIP_TRY(hipLaunchKernel(rank2_kernel(dO_dtype), dim3(bx, by), dim3(nt), args, 0, stream));
  }
  return SR_OK;
}

int lm_hv_product(const sr_matrix *O, const double *E, const sr_matrix *D, const double *v, double *y,
                  hipStream_t stream) {
  int rc = check_matrix(O, "lm_hv_product(O)");
  if (rc) return rc;
  rc = check_matrix(D, "lm_hv_product(D)");
  if (rc) return rc;
  if (D->n_s != O->n_s || D->n_p != O->n_p || D->dtype != O->dtype)
    return fail(SR_ERR_INVALID, "lm_hv_product: O and D must have the same n_s, n_p and dtype");
  if (O->O_lo != nullptr || D->O_lo != nullptr)
    return fail(SR_ERR_INVALID, "lm_hv_product: a second code plane is not supported");
  if (E == nullptr || v == nullptr || y == nullptr) return fail(SR_ERR_INVALID, "lm_hv_product: null E, v or y");
  if (ranges_overlap(v, (O->n_p + 1) * 8, y, (O->n_p + 1) * 8))
    return fail(SR_ERR_INVALID, "lm_hv_product: v and y overlap");
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  const double *mean = nullptr;
  double *mscr = nullptr;
  if (!O->col_mean) {
    rc = get_mean_scratch(dev, stream, O->n_p, &mscr);
    if (rc) return rc;
  }
  rc = ensure_mean(O, mscr, &mean, dev, di, stream);
  if (rc) return rc;
  Plan pl;
  rc = make_plan(O->dtype, di.grid, O->n_s, O->n_p, 2, &pl);
  if (rc) return rc;
  const int64_t ypd = (int64_t)pl.pg.RG * O->n_p;
  void *base = nullptr;
  rc = get_workspace(dev, stream, prod_ws_bytes(pl, ypd), &base);
  if (rc) return rc;
  Carve cv(base);
  ProdWs w;
  carve_prod(cv, pl, ypd, &w);
  LmArgs a{};
  a.pg = pl.pg;
  a.pb = w.pb;
  a.sb = w.sb;
  a.ops[0] = make_operand(O);
  a.ops[1] = make_operand(D);
  a.mean = mean;
  a.E = E;
  a.v = v;
  a.y = y;
  rc = zero_sync(w, stream);
  if (rc) return rc;
  return launch_coop(pl.ke->lm, pl.pg.G, &a, stream, pl.ke->nt, pl.ke->ring_bytes);
}

// Checks, prepare pass (Jacobi), plan and workspace of a CG solve; fills `a` (its info
// array in the workspace) and zeroes the synchronisation words.
// Options of a CG solve over n_p parameters, with the defaults of a null opt, checked.
static int check_cg_opts(const char *name, const sr_cg_opts *opt, sr_cg_opts &o) {
  o = sr_cg_opts{};
  o.rtol = 1e-10;
  if (opt) o = *opt;
  if (!(o.rtol > 0.0) || !std::isfinite(o.rtol)) return fail(SR_ERR_INVALID, "%s: rtol must be finite and > 0", name);
  if (o.refresh_every < 0) return fail(SR_ERR_INVALID, "%s: refresh_every must be >= 0", name);
  if (o.restart_on_refresh != 0 && o.restart_on_refresh != 1)
    return fail(SR_ERR_INVALID, "%s: restart_on_refresh must be 0 or 1", name);
  if (!(o.refresh_drop >= 0.0 && o.refresh_drop < 1.0))
    return fail(SR_ERR_INVALID, "%s: refresh_drop must be in [0, 1)", name);
  if (o.use_x0 != 0 && o.use_x0 != 1) return fail(SR_ERR_INVALID, "%s: use_x0 must be 0 or 1", name);
  if (o.precond != 0 && o.precond != 1) return fail(SR_ERR_INVALID, "%s: precond must be 0 or 1", name);
  if (o.search_f64 != 0 && o.search_f64 != 1) return fail(SR_ERR_INVALID, "%s: search_f64 must be 0 or 1", name);
  if (o.reserved != 0) return fail(SR_ERR_INVALID, "%s: reserved must be 0", name);
  return SR_OK;
}

static int cg_setup(const char *name, const sr_matrix *O, const double *g, double eps, double *x,
                    const sr_cg_opts *opt, hipStream_t stream, CgArgs &a, Plan &pl, ProdWs &w, sr_cg_opts &o,
                    int64_t &max_iter) {
  int rc = check_matrix(O, name);
  if (rc) return rc;
  if (g == nullptr || x == nullptr) return fail(SR_ERR_INVALID, "%s: null g or x", name);
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(SR_ERR_INVALID, "%s: eps must be finite and >= 0", name);
  if (ranges_overlap(g, O->n_p * 8, x, O->n_p * 8)) return fail(SR_ERR_INVALID, "%s: g and x overlap", name);
  rc = check_cg_opts(name, opt, o);
  if (rc) return rc;
  if (o.precond && (O->O_lo != nullptr || (O->dtype != SR_F64 && O->dtype != SR_F32)))
    return fail(SR_ERR_INVALID, "%s: the Jacobi preconditioner needs SR_F64 or SR_F32 storage, one plane", name);
  max_iter = o.max_iter > 0 ? o.max_iter : O->n_p + 100;
  if (max_iter > (1 << 30)) max_iter = 1 << 30;
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  const double *mean = nullptr;
  double *mscr = nullptr, *diag = nullptr;
  if (o.precond) {
    // one prepare pass gives diag S (and the column means, used unless the caller gave them)
    rc = get_mean_scratch(dev, stream, 2 * round_up(O->n_p, 32), &mscr);
    if (rc) return rc;
    diag = mscr + round_up(O->n_p, 32);
    rc = run_grad(O, nullptr, nullptr, nullptr, mscr, diag, dev, di, stream);
    if (rc) return rc;
    mean = O->col_mean ? O->col_mean : mscr;
  } else {
    if (!O->col_mean) {
      rc = get_mean_scratch(dev, stream, O->n_p, &mscr);
      if (rc) return rc;
    }
    rc = ensure_mean(O, mscr, &mean, dev, di, stream);
    if (rc) return rc;
  }
  rc = make_plan(O->dtype, di.grid, O->n_s, O->n_p, 1, &pl, streamed_cols(O));
  if (rc) return rc;
  const int64_t ypd = (int64_t)pl.pg.RG * pl.pg.n_v;
  const size_t bytes = prod_ws_bytes(pl, ypd) + (size_t)3 * (O->n_p * 8 + 256) + 2048;
  void *base = nullptr;
  rc = get_workspace(dev, stream, bytes, &base);
  if (rc) return rc;
  Carve cv(base);
  carve_prod(cv, pl, ypd, &w);
  a = CgArgs{};
  a.pg = pl.pg;
  a.pb = w.pb;
  a.sb = w.sb;
  a.op = make_operand(O);
  a.mean = mean;
  a.g = g;
  a.x = x;
  a.r = cv.take<double>(O->n_p);
  a.p = cv.take<double>(O->n_p);
  a.q = cv.take<double>(O->n_p);
  a.info = cv.take<double>(kInfoWords);
  a.eps = eps;
  a.rtol = o.rtol;
  a.max_iter = (int)max_iter;
  a.refresh_every = o.refresh_every;
  a.use_x0 = o.use_x0;
  a.restart_on_refresh = o.restart_on_refresh;
  a.refresh_drop2 = o.refresh_drop * o.refresh_drop;
  a.hist = o.res_history;
  a.diag = diag;
  return zero_sync(w, stream);
}

// Kernels of a split CG solve (first launch, search step, residual phase) and their launch
// shape.
struct SplitKernels {
  const void *init, *step, *resid;
  int G, nt, shmem;
};

// Runs a split solve to its end: the first launch, then search steps and residual phases.
// Long products (>= kStepSyncBytes streamed) and solves whose rounds stopped advancing
// (below: fewer products than half a round's launches, as when every search step ends in
// an exit check near the attainable accuracy): the host reads the state after every
// launch and launches exactly the phase it asks for (a synchronisation costs tens of
// microseconds against a product of a fifth of a millisecond or more).  Otherwise rounds
// of search steps up to the next periodic refresh and one residual phase are queued
// without waiting; launches in a state that is not theirs return at once, and the host
// reads the state after each batch of rounds.  Leaves the final state in hinfo / habort.
// Every round and every per-launch step advances the solve by at least one product until
// it is done, and a solve makes at most 2 max_iter + 64 products, which bounds the loops.
static int run_split_cg(const SplitKernels &k, CgArgs &a, const uint32_t *abort_dev, int64_t product_bytes,
                        int refresh_every, int64_t max_iter, hipStream_t stream, double *hinfo, uint32_t *habort) {
  int rc = fill_zero(a.info, 2 * kInfoWords, stream);      // state: initial mode, counters 0
  if (rc) return rc;
  rc = launch_coop(k.init, k.G, &a, stream, k.nt, k.shmem);
  if (rc) return rc;
  *habort = 0;
  auto read_state = [&]() -> int {
    HIP_TRY(hipMemcpyAsync(hinfo, a.info, kInfoWords * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(habort, abort_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return SR_OK;
  };
  auto done = [&]() { return *habort != 0u || hinfo[kInfoOk] == 0.0 || (int)hinfo[kInfoMode] == kCgModeDone; };
  const int64_t max_products = 2 * max_iter + 64;
  const int steps = (refresh_every > 0 ? refresh_every : 16) + 1;
  bool per_launch = product_bytes >= kStepSyncBytes;
  int64_t rounds = 0, launches = 0;
  if (!per_launch) {
    for (int batch = 1;; batch = batch < 16 ? 2 * batch : 16) {
      const int64_t before = (int64_t)hinfo[kInfoProducts];
      for (int b = 0; b < batch; ++b) {
        for (int sidx = 0; sidx < steps; ++sidx) {
          rc = launch_coop(k.step, k.G, &a, stream, k.nt, k.shmem);
          if (rc) return rc;
        }
        rc = launch_coop(k.resid, k.G, &a, stream, k.nt, k.shmem);
        if (rc) return rc;
      }
      rounds += batch;
      rc = read_state();
      if (rc) return rc;
      if (done()) return SR_OK;
      if (rounds > max_products) return fail(SR_ERR_HIP, "split CG solve did not finish");
      if (2 * ((int64_t)hinfo[kInfoProducts] - before) < (int64_t)batch * steps) {
        per_launch = true;
        break;
      }
    }
  } else {
    rc = read_state();
    if (rc) return rc;
  }
  int64_t products = (int64_t)hinfo[kInfoProducts];
  while (!done()) {
    const bool search = (int)hinfo[kInfoMode] == kCgModeP;
    TimedLaunch tl(stream);
    rc = launch_coop(search ? k.step : k.resid, k.G, &a, stream, k.nt, k.shmem);
    if (rc) return rc;
    tl.stop();
    rc = read_state();
    if (rc) return rc;
    const int64_t now = (int64_t)hinfo[kInfoProducts];
    if (now > products) tl.record(search ? kTimeSearchStep : kTimeResidualPhase);
    products = now;
    if (++launches > max_products) return fail(SR_ERR_HIP, "split CG solve did not finish");
  }
  return SR_OK;
}

// Status and host outcome of a finished solve from its final state.
static int cg_outcome(const char *name, const double *hinfo, uint32_t habort, sr_cg_info *info) {
  int status = (int)hinfo[kInfoStatus];
  if (habort != 0u || hinfo[kInfoOk] == 0.0) status = fail(SR_ERR_TIMEOUT, "%s: a cross-workgroup wait timed out", name);
  else if (status == SR_ERR_NONFINITE) fail(SR_ERR_NONFINITE, "%s: non-finite scalar in CG", name);
  else if (status == SR_BREAKDOWN) fail(SR_BREAKDOWN, "%s: p.(S+eps I)p <= 0", name);
  else if (status == SR_NOT_CONVERGED) fail(SR_NOT_CONVERGED, "%s: max_iter reached", name);
  if (info) {
    info->iters = (int32_t)hinfo[kInfoIters];
    info->refreshes = (int32_t)hinfo[kInfoRefreshes];
    info->status = status;
    info->products = (int32_t)hinfo[kInfoProducts];
    info->rel_res_recur = hinfo[kInfoRelRecur];
    info->rel_res_true = hinfo[kInfoRelTrue];
  }
  return status;
}

int sr_cg_solve(const sr_matrix *O, const double *g, double eps, double *x, const sr_cg_opts *opt, sr_cg_info *info,
                hipStream_t stream) {
  CgArgs a;
  Plan pl;
  ProdWs w;
  sr_cg_opts o;
  int64_t max_iter = 0;
  int rc = cg_setup("sr_cg_solve", O, g, eps, x, opt, stream, a, pl, w, o, max_iter);
  if (rc) return rc;
  const bool exact_search = o.search_f64 != 0 && scaled(O->dtype) && !two_planes(O);
  // one stored plane without a preconditioner: one kernel per search iteration (only the
  // product is live during its streaming loop, which keeps the registers free of spills)
  // and a resumable residual phase (for scaled storage the float64 residual products);
  // small float64 / float32 products keep the one-launch solve
  const int64_t product_bytes = O->n_s * streamed_cols(O) * elem_bytes(O->dtype);
  const bool split = !two_planes(O) && !exact_search && !o.precond &&
                     (scaled(O->dtype) || product_bytes >= kSplitMinBytes);
  double hinfo[kInfoWords] = {};
  uint32_t habort = 0;
  if (split) {
    if (pl.ke->cgs == nullptr || pl.ke->cgr == nullptr || pl.ke->cgi == nullptr)
      return fail(SR_ERR_INVALID, "sr_cg_solve: no split CG kernels for this configuration");
    const SplitKernels k{pl.ke->cgi, pl.ke->cgs, pl.ke->cgr, pl.pg.G, pl.ke->nt, pl.ke->ring_bytes};
    rc = run_split_cg(k, a, w.sb.abort, product_bytes, o.refresh_every, max_iter, stream, hinfo, &habort);
    if (rc) return rc;
  } else {
    const void *cg_fn = two_planes(O) ? pl.ke->cg2 : (o.precond ? pl.ke->cgj : (exact_search ? pl.ke->cgx : pl.ke->cg));
    if (cg_fn == nullptr) return fail(SR_ERR_INVALID, "sr_cg_solve: no CG kernel of this kind for this configuration");
    TimedLaunch tl(stream);
    rc = launch_coop(cg_fn, pl.pg.G, &a, stream, pl.ke->nt, pl.ke->ring_bytes);
    if (rc) return rc;
    tl.stop();
    HIP_TRY(hipMemcpyAsync(hinfo, a.info, sizeof(hinfo), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(&habort, w.sb.abort, sizeof(habort), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    tl.record(kTimeSolveLaunch);
  }
  return cg_outcome("sr_cg_solve", hinfo, habort, info);
}

int sr_cg_solve_async(const sr_matrix *O, const double *g, double eps, double *x, const sr_cg_opts *opt,
                      double *info_dev, hipStream_t stream) {
  if (info_dev == nullptr) return fail(SR_ERR_INVALID, "sr_cg_solve_async: null info_dev");
  if (O != nullptr && (ranges_overlap(info_dev, kInfoWords * 8, x, O->n_p * 8) ||
                       ranges_overlap(info_dev, kInfoWords * 8, g, O->n_p * 8)))
    return fail(SR_ERR_INVALID, "sr_cg_solve_async: info_dev overlaps g or x");
  CgArgs a;
  Plan pl;
  ProdWs w;
  sr_cg_opts o;
  int64_t max_iter = 0;
  int rc = cg_setup("sr_cg_solve_async", O, g, eps, x, opt, stream, a, pl, w, o, max_iter);
  if (rc) return rc;
  a.info = info_dev;
  const bool exact_search = o.search_f64 != 0 && scaled(O->dtype) && !two_planes(O);
  const void *cg_fn = two_planes(O) ? pl.ke->cg2 : (o.precond ? pl.ke->cgj : (exact_search ? pl.ke->cgx : pl.ke->cg));
  if (cg_fn == nullptr) return fail(SR_ERR_INVALID, "sr_cg_solve_async: no CG kernel of this kind for this configuration");
  return launch_coop(cg_fn, pl.pg.G, &a, stream, pl.ke->nt, pl.ke->ring_bytes);
}

// ------------------------------------------------------------------------------------
// Index-coded CPS storage
// ------------------------------------------------------------------------------------
static int64_t cps_n_p(const sr_cps_matrix *M) { return M->n_corr * (int64_t)M->n_states + M->dense.n_p; }

static int check_cps(const sr_cps_matrix *M, const char *name) {
  if (M == nullptr) return fail(SR_ERR_INVALID, "%s: null matrix", name);
  if (M->reserved != 0) return fail(SR_ERR_INVALID, "%s: reserved must be 0", name);
  if (M->n_s < 1) return fail(SR_ERR_INVALID, "%s: n_s must be >= 1", name);
  if (M->n_corr < 0 || M->dense.n_p < 0) return fail(SR_ERR_INVALID, "%s: n_corr and dense.n_p must be >= 0", name);
  if (M->n_states < 1 || M->n_states > 256) return fail(SR_ERR_INVALID, "%s: n_states must be in [1, 256]", name);
  if (cps_n_p(M) < 1) return fail(SR_ERR_INVALID, "%s: no parameters", name);
  if (M->n_corr > ((int64_t)1 << 31) / M->n_states) return fail(SR_ERR_INVALID, "%s: too many correlator columns", name);
  if (M->n_corr > 0) {
    if (M->idx == nullptr || M->val == nullptr) return fail(SR_ERR_INVALID, "%s: null idx or val", name);
    if (M->ld_idx < M->n_s || M->ld_idx % 16 != 0 || ((uintptr_t)M->idx) % 16)
      return fail(SR_ERR_INVALID, "%s: idx must be 16-byte aligned with ld_idx >= n_s a multiple of 16", name);
  }
  if (M->dense.n_p > 0) {
    const sr_matrix &d = M->dense;
    if (d.n_s != M->n_s) return fail(SR_ERR_INVALID, "%s: dense.n_s must equal n_s", name);
    if (d.dtype != SR_F64 && d.dtype != SR_F32 && d.dtype != SR_BF16)
      return fail(SR_ERR_INVALID, "%s: the dense block must be SR_F64, SR_F32 or SR_BF16", name);
    if (d.O_lo != nullptr || d.lo_cols != nullptr || d.n_lo != 0)
      return fail(SR_ERR_INVALID, "%s: the dense block must have one plane", name);
    int rc = check_matrix(&d, name);
    if (rc) return rc;
  }
  return SR_OK;
}

// The dense block as its own matrix (no means: the caller's col_mean covers all columns).
static sr_matrix cps_dense(const sr_cps_matrix *M) {
  sr_matrix d = M->dense;
  d.col_mean = nullptr;
  return d;
}

// Kernels for the dense block's width (the narrowest register tile that holds a row).
static int cps_pick(const sr_cps_matrix *M, bool exact_search, const char *name, const CpsEntry **out) {
  const int dt = M->dense.n_p > 0 ? M->dense.dtype : SR_F64;
  int count = 0;
  const CpsEntry *tab = cps_table(dt, &count);
  const int64_t nvec = cdiv(M->dense.n_p, vec_of(dt));
  const int64_t need = std::max<int64_t>(1, cdiv(nvec, 512));
  const CpsEntry *pick = nullptr;
  for (int i = 0; i < count; ++i) {
    if (tab[i].nvt < need || (exact_search && tab[i].stepx == nullptr)) continue;
    if (pick == nullptr || tab[i].nvt < pick->nvt) pick = &tab[i];
  }
  if (pick == nullptr)
    return fail(SR_ERR_INVALID, "%s: a dense block of %lld columns is wider than the register tiles hold", name,
                (long long)M->dense.n_p);
  *out = pick;
  return SR_OK;
}

// Column means of the dense block into scratch[n_sp..n_p) when the matrix has none.
static int cps_mean(const sr_cps_matrix *M, int dev, const DeviceInfo &di, hipStream_t s, const double **mean) {
  if (M->col_mean != nullptr || M->dense.n_p == 0) {
    *mean = M->col_mean;
    return SR_OK;
  }
  double *scr = nullptr;
  int rc = get_mean_scratch(dev, s, cps_n_p(M), &scr);
  if (rc) return rc;
  const sr_matrix d = cps_dense(M);
  rc = run_grad(&d, nullptr, nullptr, nullptr, scr + M->n_corr * (int64_t)M->n_states, nullptr, dev, di, s);
  if (rc) return rc;
  *mean = scr;
  return SR_OK;
}

// Workspace and argument block of a CPS product or solve (cg: also the CG vectors).
static int cps_args(const sr_cps_matrix *M, const double *mean, double eps, bool cg, int dev, const DeviceInfo &di,
                    hipStream_t s, CgArgs &a) {
  const int G = di.grid;
  const int64_t n_p = cps_n_p(M), n_sp = M->n_corr * (int64_t)M->n_states, n_d = M->dense.n_p;
  const int64_t n_dp = n_d > 0 ? round_up(n_d, vec_of(M->dense.dtype)) : 0;
  size_t bytes = 0;
  auto add = [&](size_t n) { bytes = (size_t)round_up((int64_t)bytes, 256) + n; };
  add((size_t)G * 4);
  add(64 * 4);
  add((size_t)8 * G * 8);
  add((size_t)8 * G * 8);
  // correlator groups: the largest group whose float64 table fits the LDS table, then
  // (group, row range) items that cover the grid at least once
  const int64_t cpg_max = std::max<int64_t>(1, kCpsTableBytes / (8 * (int64_t)M->n_states));
  const int64_t n_grp = std::max<int64_t>(1, cdiv(M->n_corr, cpg_max));
  const int64_t cpg = M->n_corr > 0 ? cdiv(M->n_corr, n_grp) : 0;
  const int64_t ranges = std::max<int64_t>(1, G / n_grp);
  const int64_t rpr = round_up(cdiv(M->n_s, ranges), kCpsTileRows);
  add((size_t)M->n_s * 8);
  add((size_t)n_grp * M->n_s * 8);
  add((size_t)G * std::max<int64_t>(n_dp, 1) * 8);
  if (cg) {
    add((size_t)3 * n_p * 8);
    add(2 * kInfoWords * 8);
  }
  void *base = nullptr;
  int rc = get_workspace(dev, s, bytes + 512, &base);
  if (rc) return rc;
  Carve cv(base);
  a = CgArgs{};
  a.sb.flags = cv.take<uint32_t>(G);
  a.sb.abort = cv.take<uint32_t>(64);
  a.sb.red = cv.take<double>(8 * G);
  CpsOp &c = a.cps;
  c.red = cv.take<double>(8 * G);
  c.w = cv.take<double>(M->n_s);
  c.part_sp = cv.take<double>(n_grp * M->n_s);
  c.n_grp = (int32_t)n_grp;
  c.cpg = (int32_t)cpg;
  c.n_items = (int32_t)(n_grp * ranges);
  c.rpr = (int32_t)rpr;
  c.part = cv.take<double>((int64_t)G * std::max<int64_t>(n_dp, 1));
  c.n_dp = n_dp;
  c.idx = (const unsigned char *)M->idx;
  c.ld_idx = M->ld_idx;
  c.val = M->val;
  c.n_corr = M->n_corr;
  c.n_states = M->n_states;
  int tr = kCpsTileRows;
  while (tr > kCpsMinTileRows && cdiv(M->n_s, tr) < G) tr /= 2;
  c.tile_rows = tr;
  c.tiles = (int32_t)cdiv(M->n_s, tr);
  c.n_sp = n_sp;
  c.n_d = n_d;
  c.dO = (const unsigned char *)M->dense.O;
  c.dscale = n_d > 0 ? M->dense.col_scale : nullptr;
  c.ldb_d = n_d > 0 ? M->dense.ld * elem_bytes(M->dense.dtype) : 0;
  a.pg.G = G;
  a.pg.C = 1;
  a.pg.RG = G;
  a.pg.n_s = M->n_s;
  a.pg.n_p = n_p;
  a.pg.n_v = n_p;
  a.pg.wslice = n_p;
  a.pg.n_tiles = c.tiles;
  a.mean = mean;
  a.eps = eps;
  if (cg) {
    a.r = cv.take<double>(n_p);
    a.p = cv.take<double>(n_p);
    a.q = cv.take<double>(n_p);
    a.info = cv.take<double>(2 * kInfoWords);
  }
  return fill_zero(a.sb.flags, (int64_t)((char *)(a.sb.abort + 64) - (char *)a.sb.flags) / 4, s);
}

int sr_cps_grad(const sr_cps_matrix *M, const double *E, double *g, double *E_mean, double *col_mean_out,
                double *diagS_out, hipStream_t stream) {
  int rc = check_cps(M, "sr_cps_grad");
  if (rc) return rc;
  if (g != nullptr && E == nullptr) return fail(SR_ERR_INVALID, "sr_cps_grad: g needs E");
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  const int64_t n_sp = M->n_corr * (int64_t)M->n_states;
  if (M->dense.n_p > 0) {
    const sr_matrix d = cps_dense(M);
    rc = run_grad(&d, E, g ? g + n_sp : nullptr, E_mean, col_mean_out ? col_mean_out + n_sp : nullptr,
                  diagS_out ? diagS_out + n_sp : nullptr, dev, di, stream);
    if (rc) return rc;
  }
  if (M->n_corr > 0 || (E_mean != nullptr && M->dense.n_p == 0)) {
    CpsStatsArgs a{};
    a.idx = (const unsigned char *)M->idx;
    a.ld_idx = M->ld_idx;
    a.n_corr = M->n_corr;
    a.n_s = M->n_s;
    a.val = M->val;
    a.E = E;
    a.mean = col_mean_out;
    a.diag = diagS_out;
    a.g = g;
    a.Emean = M->dense.n_p == 0 ? E_mean : nullptr;
    a.n_states = M->n_states;
    void *args[] = {&a};
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(M->n_corr, 4 * (int64_t)di.cus));
    HIP_TRY(hipLaunchKernel(cps_stats_kernel(), dim3(blocks), dim3(512), args, 0, stream));
  }
  return SR_OK;
}

// y = (S + eps I) v over CPS storage; raw: the uncentred O^T (O v) / n_s (zero_mean, the
// dense block's means taken as 0).
static int cps_product(const char *name, const sr_cps_matrix *M, const double *v, double *y, double eps,
                       const double *zero_mean, hipStream_t stream) {
  const CpsEntry *ent = nullptr;
  int rc = cps_pick(M, false, name, &ent);
  if (rc) return rc;
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  const double *mean = zero_mean;
  if (mean == nullptr) {
    rc = cps_mean(M, dev, di, stream, &mean);
    if (rc) return rc;
  }
  CgArgs a;
  rc = cps_args(M, mean, eps, false, dev, di, stream, a);
  if (rc) return rc;
  a.cps.raw = zero_mean != nullptr ? 1 : 0;
  a.p = const_cast<double *>(v);
  a.q = y;
  return launch_coop(ent->sv, di.grid, &a, stream, 512, 0);
}

int sr_cps_sv_product(const sr_cps_matrix *M, const double *v, double *y, double eps, hipStream_t stream) {
  int rc = check_cps(M, "sr_cps_sv_product");
  if (rc) return rc;
  const int64_t n_p = cps_n_p(M);
  if (v == nullptr || y == nullptr) return fail(SR_ERR_INVALID, "sr_cps_sv_product: null v or y");
  if (ranges_overlap(v, n_p * 8, y, n_p * 8)) return fail(SR_ERR_INVALID, "sr_cps_sv_product: v and y overlap");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(SR_ERR_INVALID, "sr_cps_sv_product: eps must be finite and >= 0");
  return cps_product("sr_cps_sv_product", M, v, y, eps, nullptr, stream);
}

// ------------------------------------------------------------------------------------
// Products during sampling
// ------------------------------------------------------------------------------------
constexpr int kStreamMaxVectors = 8;

static int check_stream_acc(const sr_stream_acc *acc, const char *name) {
  if (acc == nullptr) return fail(SR_ERR_INVALID, "%s: null accumulator", name);
  if (acc->reserved != 0) return fail(SR_ERR_INVALID, "%s: reserved must be 0", name);
  if (acc->n_p < 1) return fail(SR_ERR_INVALID, "%s: n_p must be >= 1", name);
  if (acc->m < 1 || acc->m > kStreamMaxVectors) return fail(SR_ERR_INVALID, "%s: m must be in [1, %d]", name, kStreamMaxVectors);
  if (acc->A == nullptr || acc->s1 == nullptr || acc->scal == nullptr)
    return fail(SR_ERR_INVALID, "%s: null A, s1 or scal", name);
  return SR_OK;
}

extern "C++" {
namespace sr {
int stream_dot_blocks();   // workgroups per vector of the partial-dot kernel (sr_kernels_common.hip)
}
}

// Stream scratch, one size for every call on an accumulator (so that the finish does not
// grow the workspace): batch means, batch gradient, one raw product, zero means, <E>_b,
// then the partial dots of the finish (m x stream_dot_blocks()).
static size_t stream_ws_bytes(int64_t n_p, int m) {
  return (size_t)(4 * round_up(n_p, 32) + 64 + (int64_t)m * sr::stream_dot_blocks()) * 8;
}

static int stream_launch(int which, const StreamArgs &a, int blocks, hipStream_t s) {
  StreamArgs b = a;
  void *args[] = {&b};
  HIP_TRY(hipLaunchKernel(stream_kernel(which), dim3(blocks), dim3(which == 2 ? 512 : 256), args, 0, s));
  return SR_OK;
}

int sr_stream_begin(const sr_stream_acc *acc, hipStream_t stream) {
  int rc = check_stream_acc(acc, "sr_stream_begin");
  if (rc) return rc;
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  const int64_t n = acc->n_p;
  if ((rc = fill_zero(acc->A, 2 * n * acc->m, stream))) return rc;
  if ((rc = fill_zero(acc->s1, 2 * n, stream))) return rc;
  if (acc->se && (rc = fill_zero(acc->se, 2 * n, stream))) return rc;
  return fill_zero(acc->scal, 2 * 4, stream);
}

int sr_stream_accumulate(const sr_stream_acc *acc, const sr_matrix *O, const sr_cps_matrix *C, const double *E,
                         const double *Z, hipStream_t stream) {
  const char *name = "sr_stream_accumulate";
  int rc = check_stream_acc(acc, name);
  if (rc) return rc;
  if ((O == nullptr) == (C == nullptr)) return fail(SR_ERR_INVALID, "%s: give exactly one of O and C", name);
  if (Z == nullptr) return fail(SR_ERR_INVALID, "%s: null Z", name);
  int64_t n_s, n_p;
  if (O) {
    if ((rc = check_matrix(O, name))) return rc;
    if (O->O_lo != nullptr || O->lo_cols != nullptr) return fail(SR_ERR_INVALID, "%s: one-plane batches only", name);
    n_s = O->n_s;
    n_p = O->n_p;
  } else {
    if ((rc = check_cps(C, name))) return rc;
    n_s = C->n_s;
    n_p = cps_n_p(C);
  }
  if (n_p != acc->n_p) return fail(SR_ERR_INVALID, "%s: the batch has %lld parameters, the accumulator %lld", name,
                                   (long long)n_p, (long long)acc->n_p);
  if (E != nullptr && acc->se == nullptr) return fail(SR_ERR_INVALID, "%s: energies need acc->se", name);
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  // scratch: batch means, batch gradient, one raw product, zero means, <E>_b
  double *scr = nullptr;
  rc = get_workspace(dev, stream, stream_ws_bytes(n_p, acc->m), (void **)&scr, g_stream_ws);
  if (rc) return rc;
  const int64_t np32 = round_up(n_p, 32);
  double *mean_b = scr, *g_b = scr + np32, *y_b = scr + 2 * np32, *zeros = scr + 3 * np32, *Eb = scr + 4 * np32;
  if ((rc = fill_zero(zeros, 2 * n_p, stream))) return rc;
  if (O) {
    rc = run_grad(O, E, E ? g_b : nullptr, E ? Eb : nullptr, mean_b, nullptr, dev, di, stream);
  } else {
    rc = sr_cps_grad(C, E, E ? g_b : nullptr, E ? Eb : nullptr, mean_b, nullptr, stream);
  }
  if (rc) return rc;
  StreamArgs a{};
  a.n_p = n_p;
  a.m = acc->m;
  a.B = (double)n_s;
  a.A = acc->A;
  a.s1 = acc->s1;
  a.se = acc->se;
  a.scal = acc->scal;
  a.mean_b = mean_b;
  a.g_b = E ? g_b : nullptr;
  a.Emean_b = E ? Eb : nullptr;
  a.y_b = y_b;
  const int blocks = (int)std::min<int64_t>(4 * (int64_t)di.cus, std::max<int64_t>(1, cdiv(n_p, 256)));
  if ((rc = stream_launch(0, a, blocks, stream))) return rc;
  for (int i = 0; i < acc->m; ++i) {
    const double *zi = Z + (int64_t)i * n_p;
    if (O) {
      sr_matrix Oz = *O;
      Oz.col_mean = zeros;            // uncentred: O^T (O z) / n_s
      rc = sr_sv_product(&Oz, zi, y_b, 0.0, stream);
    } else {
      rc = cps_product(name, C, zi, y_b, 0.0, zeros, stream);
    }
    if (rc) return rc;
    a.i = i;
    if ((rc = stream_launch(1, a, blocks, stream))) return rc;
  }
  return SR_OK;
}

int sr_stream_finish(const sr_stream_acc *acc, const double *Z, double eps, double *Y, double *g, double *col_mean,
                     double *E_mean, hipStream_t stream) {
  const char *name = "sr_stream_finish";
  int rc = check_stream_acc(acc, name);
  if (rc) return rc;
  if (Z == nullptr || Y == nullptr) return fail(SR_ERR_INVALID, "%s: null Z or Y", name);
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(SR_ERR_INVALID, "%s: eps must be finite and >= 0", name);
  if (g != nullptr && acc->se == nullptr) return fail(SR_ERR_INVALID, "%s: g needs acc->se", name);
  const int64_t n_p = acc->n_p;
  if (ranges_overlap(Y, n_p * acc->m * 8, Z, n_p * acc->m * 8) || ranges_overlap(Y, n_p * acc->m * 8, acc->A, n_p * acc->m * 8))
    return fail(SR_ERR_INVALID, "%s: Y overlaps Z or A", name);
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  // partial dots of s1 . z_i: stream_dot_blocks() per vector (summed by the finish kernel)
  const int dot_blocks = sr::stream_dot_blocks();
  double *scr = nullptr;
  rc = get_workspace(dev, stream, stream_ws_bytes(n_p, acc->m), (void **)&scr, g_stream_ws);
  if (rc) return rc;
  StreamArgs a{};
  a.n_p = n_p;
  a.m = acc->m;
  a.A = acc->A;
  a.s1 = acc->s1;
  a.se = acc->se;
  a.scal = acc->scal;
  a.Z = Z;
  a.eps = eps;
  a.Y = Y;
  a.g = g;
  a.col_mean = col_mean;
  a.E_mean = E_mean;
  a.dots = scr + 4 * round_up(n_p, 32) + 16;
  if ((rc = stream_launch(2, a, acc->m * dot_blocks, stream))) return rc;
  const int blocks = (int)std::min<int64_t>(4 * (int64_t)di.cus, std::max<int64_t>(1, cdiv(n_p, 256)));
  return stream_launch(3, a, blocks, stream);
}

int sr_cps_cg_solve(const sr_cps_matrix *M, const double *g, double eps, double *x, const sr_cg_opts *opt,
                    sr_cg_info *info, hipStream_t stream) {
  const char *name = "sr_cps_cg_solve";
  int rc = check_cps(M, name);
  if (rc) return rc;
  const int64_t n_p = cps_n_p(M);
  if (g == nullptr || x == nullptr) return fail(SR_ERR_INVALID, "%s: null g or x", name);
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(SR_ERR_INVALID, "%s: eps must be finite and >= 0", name);
  if (ranges_overlap(g, n_p * 8, x, n_p * 8)) return fail(SR_ERR_INVALID, "%s: g and x overlap", name);
  sr_cg_opts o;
  rc = check_cg_opts(name, opt, o);
  if (rc) return rc;
  if (o.precond) return fail(SR_ERR_INVALID, "%s: the Jacobi preconditioner is not available for CPS storage", name);
  const bool exact_search = o.search_f64 != 0 && M->dense.n_p > 0 && M->dense.dtype == SR_BF16;
  const CpsEntry *ent = nullptr;
  rc = cps_pick(M, exact_search, name, &ent);
  if (rc) return rc;
  int64_t max_iter = o.max_iter > 0 ? o.max_iter : n_p + 100;
  if (max_iter > (1 << 30)) max_iter = 1 << 30;
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  const double *mean = nullptr;
  rc = cps_mean(M, dev, di, stream, &mean);
  if (rc) return rc;
  CgArgs a;
  rc = cps_args(M, mean, eps, true, dev, di, stream, a);
  if (rc) return rc;
  a.g = g;
  a.x = x;
  a.rtol = o.rtol;
  a.max_iter = (int)max_iter;
  a.refresh_every = o.refresh_every;
  a.use_x0 = o.use_x0;
  a.restart_on_refresh = o.restart_on_refresh;
  a.refresh_drop2 = o.refresh_drop * o.refresh_drop;
  a.hist = o.res_history;
  double hinfo[kInfoWords] = {};
  uint32_t habort = 0;
  const SplitKernels k{ent->init, exact_search ? ent->stepx : ent->step, ent->resid, di.grid, 512, 0};
  const int64_t bytes = M->n_corr * M->ld_idx +
                        (M->dense.n_p > 0 ? M->n_s * M->dense.n_p * elem_bytes(M->dense.dtype) : 0);
  rc = run_split_cg(k, a, a.sb.abort, bytes, o.refresh_every, max_iter, stream, hinfo, &habort);
  if (rc) return rc;
  return cg_outcome(name, hinfo, habort, info);
}

int sr_quantize(int64_t n_s, int64_t n_p, const void *in, int64_t ld_in, int32_t in_dtype, void *q, void *q_lo,
                int64_t ld_out, int32_t out_dtype, float *scale, hipStream_t stream) {
  if (n_s < 1 || n_p < 1) return fail(SR_ERR_INVALID, "sr_quantize: n_s and n_p must be >= 1");
  if (in_dtype != SR_F64 && in_dtype != SR_F32) return fail(SR_ERR_INVALID, "sr_quantize: in_dtype must be f64 or f32");
  if (out_dtype != SR_BF16 && out_dtype != SR_F16) return fail(SR_ERR_INVALID, "sr_quantize: out_dtype must be bf16 or f16");
  if (in == nullptr || q == nullptr || scale == nullptr) return fail(SR_ERR_INVALID, "sr_quantize: null pointer");
  if (ld_in < n_p || ld_out < n_p) return fail(SR_ERR_INVALID, "sr_quantize: ld < n_p");
  if (((uintptr_t)in) % 16 || ((uintptr_t)q) % 16 || ((uintptr_t)q_lo) % 16)
    return fail(SR_ERR_INVALID, "sr_quantize: pointers must be 16-byte aligned");
  if (q_lo != nullptr && (ranges_overlap(q, n_s * ld_out * 2, q_lo, n_s * ld_out * 2)))
    return fail(SR_ERR_INVALID, "sr_quantize: q and q_lo overlap");
  if ((ld_in * elem_bytes(in_dtype)) % 16 || (ld_out * 2) % 16)
    return fail(SR_ERR_INVALID, "sr_quantize: ld * element size must be a multiple of 16 bytes");
  int dev;
  DeviceInfo di;
  int rc = device_check(&dev, &di);
  if (rc) return rc;
  Plan pl;
  pl.words = 0;
  rc = geometry(di.grid, n_s, n_p, kNT * 8, 1, 1, 0, &pl.pg);
  if (rc) return rc;
  const int64_t ypd = (int64_t)pl.pg.RG * n_p;
  void *base = nullptr;
  rc = get_workspace(dev, stream, prod_ws_bytes(pl, ypd), &base);
  if (rc) return rc;
  Carve cv(base);
  ProdWs w;
  carve_prod(cv, pl, ypd, &w);
  QuantArgs a{};
  a.pg = pl.pg;
  a.pb = w.pb;
  a.sb = w.sb;
  a.in = (const unsigned char *)in;
  a.ldb_in = ld_in * elem_bytes(in_dtype);
  a.out = (unsigned char *)q;
  a.out_lo = (unsigned char *)q_lo;
  a.ld_out = ld_out;
  a.scale = scale;
  rc = zero_sync(w, stream);
  if (rc) return rc;
  rc = launch_coop(absmax_kernel(in_dtype), pl.pg.G, &a, stream);
  if (rc) return rc;
  void *args[] = {&a};
  HIP_TRY(hipLaunchKernel(quantize_kernel(in_dtype, out_dtype), dim3(di.grid * 8), dim3(kNT), args, 0, stream));
  return SR_OK;
}

static int check_quant_input(const char *where, int64_t n_s, int64_t n_p, const void *in, int64_t ld_in, int32_t in_dtype,
                      int32_t out_dtype, const float *scale) {
  if (n_s < 1 || n_p < 1) return fail(SR_ERR_INVALID, "%s: n_s and n_p must be >= 1", where);
  if (n_s > (int64_t)1 << 40 || n_p > (int64_t)1 << 31) return fail(SR_ERR_INVALID, "%s: dimensions out of range", where);
  if (in_dtype != SR_F64 && in_dtype != SR_F32) return fail(SR_ERR_INVALID, "%s: in_dtype must be f64 or f32", where);
  if (out_dtype != SR_BF16 && out_dtype != SR_F16) return fail(SR_ERR_INVALID, "%s: out_dtype must be bf16 or f16", where);
  if (in == nullptr || scale == nullptr) return fail(SR_ERR_INVALID, "%s: null pointer", where);
  if (ld_in < n_p) return fail(SR_ERR_INVALID, "%s: ld_in < n_p", where);
  if (((uintptr_t)in) % 16 || (ld_in * elem_bytes(in_dtype)) % 16)
    return fail(SR_ERR_INVALID, "%s: the input must be 16-byte aligned with rows of whole 16-byte vectors", where);
  return SR_OK;
}

int sr_remainder_columns(int64_t n_s, int64_t n_p, const void *in, int64_t ld_in, int32_t in_dtype, int32_t out_dtype,
                         const float *scale, double tol, int32_t *lo_cols, int64_t *n_lo, hipStream_t stream) {
  int rc = check_quant_input("sr_remainder_columns", n_s, n_p, in, ld_in, in_dtype, out_dtype, scale);
  if (rc) return rc;
  if (lo_cols == nullptr || n_lo == nullptr) return fail(SR_ERR_INVALID, "sr_remainder_columns: null output");
  if (std::isnan(tol)) return fail(SR_ERR_INVALID, "sr_remainder_columns: tol is NaN");
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  Plan pl;
  pl.words = 0;
  rc = geometry(di.grid, n_s, n_p, kNT * 8, 1, 1, 0, &pl.pg);
  if (rc) return rc;
  const int64_t ypd = (int64_t)pl.pg.RG * n_p;
  void *base = nullptr;
  rc = get_workspace(dev, stream, prod_ws_bytes(pl, ypd) + (size_t)n_p * 8 + 1024, &base);
  if (rc) return rc;
  Carve cv(base);
  ProdWs w;
  carve_prod(cv, pl, ypd, &w);
  RemArgs a{};
  a.pg = pl.pg;
  a.pb = w.pb;
  a.sb = w.sb;
  a.in = (const unsigned char *)in;
  a.ldb_in = ld_in * elem_bytes(in_dtype);
  a.scale = scale;
  a.err = cv.take<double>(n_p);
  int64_t *count = cv.take<int64_t>(1);
  rc = zero_sync(w, stream);
  if (rc) return rc;
  rc = launch_coop(remmax_kernel(in_dtype, out_dtype), pl.pg.G, &a, stream);
  if (rc) return rc;
  SelectArgs b{a.err, n_p, tol, lo_cols, count};
  void *args[] = {&b};
  HIP_TRY(hipLaunchKernel(select_kernel(), dim3(1), dim3(1024), args, 0, stream));
  int64_t h = 0;
  HIP_TRY(hipMemcpyAsync(&h, count, sizeof(h), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  *n_lo = h;
  return SR_OK;
}

int sr_quantize_remainder(int64_t n_s, int64_t n_p, const void *in, int64_t ld_in, int32_t in_dtype,
                          int32_t out_dtype, const float *scale, const int32_t *lo_cols, int64_t n_lo, void *q_lo,
                          int64_t ld_lo, hipStream_t stream) {
  int rc = check_quant_input("sr_quantize_remainder", n_s, n_p, in, ld_in, in_dtype, out_dtype, scale);
  if (rc) return rc;
  if (n_lo < 0 || n_lo > n_p) return fail(SR_ERR_INVALID, "sr_quantize_remainder: n_lo must be in [0, n_p]");
  if (n_lo == 0) return SR_OK;
  if (lo_cols == nullptr || q_lo == nullptr) return fail(SR_ERR_INVALID, "sr_quantize_remainder: null pointer");
  if (ld_lo < n_lo || (ld_lo * 2) % 16 || ((uintptr_t)q_lo) % 16)
    return fail(SR_ERR_INVALID, "sr_quantize_remainder: q_lo must be 16-byte aligned, ld_lo >= n_lo, ld_lo * 2 a "
                                "multiple of 16 bytes");
  int dev;
  DeviceInfo di;
  rc = device_check(&dev, &di);
  if (rc) return rc;
  QuantLoArgs a{};
  a.in = (const unsigned char *)in;
  a.ldb_in = ld_in * elem_bytes(in_dtype);
  a.n_s = n_s;
  a.n_p = n_p;
  a.n_lo = n_lo;
  a.ld_lo = ld_lo;
  a.scale = scale;
  a.cols = lo_cols;
  a.out = (unsigned char *)q_lo;
  void *args[] = {&a};
  HIP_TRY(hipLaunchKernel(quantize_lo_kernel(in_dtype, out_dtype), dim3(di.grid * 8), dim3(kNT), args, 0, stream));
  return SR_OK;
}

}  // extern "C"
