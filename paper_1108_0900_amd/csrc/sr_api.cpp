// libsr C-ABI: argument validation, launch planning, per-(device, stream) workspace and
// cooperative launches of the kernels.  Declarations and the contract are in sr.h.
#include "sr.h"

#include <hip/hip_runtime.h>

#include <cmath>
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
  return SR_OK;
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

int geometry(int G, int64_t n_s, int64_t n_p, int cols_per_wg, int vec, int r, int force_c, ProdGeom *pg) {
  int64_t C = pow2_ceil(cdiv(n_p, cols_per_wg));
  if (force_c > 0 && force_c >= C) C = force_c;
  if (C > G) return fail(SR_ERR_INVALID, "n_p = %lld exceeds the column capacity of this build (%lld)",
                         (long long)n_p, (long long)G * cols_per_wg);
  pg->G = G;
  pg->C = (int)C;
  pg->RG = G / (int)C;
  pg->n_s = n_s;
  pg->n_p = n_p;
  pg->wslice = round_up(cdiv(n_p, C), vec);
  pg->n_tiles = (int)cdiv(n_s, r);
  return SR_OK;
}

int make_plan(int dt, int G, int64_t n_s, int64_t n_p, int ndot, Plan *plan) {
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
  int rc = geometry(G, n_s, n_p, cols, vec, pick->r, f.nv > 0 && pick->nv == f.nv ? f.c : 0, &plan->pg);
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
  w->pb.xchg = cv.take<u64>((int64_t)pg.RG * kRing * pg.C * (pl.words > 0 ? pl.words : 1));
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
  add((size_t)pg.RG * kRing * pg.C * (pl.words > 0 ? pl.words : 1) * 8);
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
  int rc = geometry(di.grid, m->n_s, m->n_p, grad_nv(dt) * vec * kNT, vec, grad_rows(dt), 0, &pl.pg);
  if (rc) return rc;
  const int64_t ypd = (int64_t)pl.pg.RG * 3 * m->n_p;
  void *base = nullptr;
  rc = get_workspace(dev, s, prod_ws_bytes(pl, ypd), &base);
  if (rc) return rc;
  Carve cv(base);
  ProdWs w;
  carve_prod(cv, pl, ypd, &w);
  GradArgs a{};
  a.pg = pl.pg;
  a.pb = w.pb;
  a.sb = w.sb;
  a.op = make_operand(m);
  a.E = E;
  a.g_out = g;
  a.mean_out = mean;
  a.diag_out = diag;
  a.Emean_out = Emean;
  rc = zero_sync(w, s);
  if (rc) return rc;
  return launch_coop(grad_kernel(dt), pl.pg.G, &a, s);
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

int sr_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = SR_OK;
  for (auto *mp : {&g_ws, &g_mean_ws, &g_batch_ws}) {
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

int sr_sv_product(const sr_matrix *O, const double *v, double *y, double eps, hipStream_t stream) {
  int rc = check_matrix(O, "sr_sv_product");
  if (rc) return rc;
  if (v == nullptr || y == nullptr) return fail(SR_ERR_INVALID, "sr_sv_product: null v or y");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(SR_ERR_INVALID, "sr_sv_product: eps must be finite and >= 0");
  if (ranges_overlap(v, O->n_p * 8, y, O->n_p * 8)) return fail(SR_ERR_INVALID, "sr_sv_product: v and y overlap");
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
  rc = make_plan(O->dtype, di.grid, O->n_s, O->n_p, 1, &pl);
  if (rc) return rc;
  const int64_t ypd = (int64_t)pl.pg.RG * O->n_p;
  void *base = nullptr;
  rc = get_workspace(dev, stream, prod_ws_bytes(pl, ypd), &base);
  if (rc) return rc;
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
  rc = zero_sync(w, stream);
  if (rc) return rc;
  if (O->O_lo != nullptr) {
    if (pl.ke->sv2 == nullptr) return fail(SR_ERR_INVALID, "sr_sv_product: no two-plane kernel for this configuration");
    return launch_coop(pl.ke->sv2, pl.pg.G, &a, stream, pl.ke->nt, 0);
  }
  return launch_coop(pl.ke->sv, pl.pg.G, &a, stream, pl.ke->nt, pl.ke->ring_bytes);
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
  g.n_rb = cdiv(n_s, (int64_t)nw * kBatchRows);
  const int64_t max_parts = std::max<int64_t>(1, cdiv(n_p, 4 * cw));   // parts of >= 4 chunks
  const int64_t parts = std::min<int64_t>(max_parts, std::max<int64_t>(1, cdiv(2 * (int64_t)G, g.n_rb)));
  g.pw = round_up(cdiv(n_p, parts), cw);
  g.P = (int)cdiv(n_p, g.pw);
  g.C = (int)cdiv(n_p, bw);
  const int64_t sp = std::max<int64_t>(cdiv(n_s, kBatchSplitRows),
                                       std::min<int64_t>(cdiv(2 * (int64_t)G, g.C), cdiv(n_s, 64)));
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

int sr_adjoint(const sr_matrix *O, const double *E, const double *x, const double *lam, double *dE, void *dO,
               int32_t dO_dtype, int64_t ld_dO, double *p12, hipStream_t stream) {
  int rc = check_matrix(O, "sr_adjoint");
  if (rc) return rc;
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
  const int nv = n_p >= (int64_t)4 * vec * nt * 8 ? 4 : (n_p >= (int64_t)2 * vec * nt * 8 ? 2 : 1);
  const int64_t cols = (int64_t)nv * vec * nt;
  const int C = (int)std::min<int64_t>(cdiv(n_p, cols), 1 << 20);
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

int sr_cg_solve(const sr_matrix *O, const double *g, double eps, double *x, const sr_cg_opts *opt, sr_cg_info *info,
                hipStream_t stream) {
  int rc = check_matrix(O, "sr_cg_solve");
  if (rc) return rc;
  if (g == nullptr || x == nullptr) return fail(SR_ERR_INVALID, "sr_cg_solve: null g or x");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(SR_ERR_INVALID, "sr_cg_solve: eps must be finite and >= 0");
  if (ranges_overlap(g, O->n_p * 8, x, O->n_p * 8)) return fail(SR_ERR_INVALID, "sr_cg_solve: g and x overlap");
  sr_cg_opts o{};
  o.rtol = 1e-10;
  if (opt) o = *opt;
  if (!(o.rtol > 0.0) || !std::isfinite(o.rtol)) return fail(SR_ERR_INVALID, "sr_cg_solve: rtol must be finite and > 0");
  if (o.refresh_every < 0) return fail(SR_ERR_INVALID, "sr_cg_solve: refresh_every must be >= 0");
  if (o.restart_on_refresh != 0 && o.restart_on_refresh != 1)
    return fail(SR_ERR_INVALID, "sr_cg_solve: restart_on_refresh must be 0 or 1");
  if (!(o.refresh_drop >= 0.0 && o.refresh_drop < 1.0))
    return fail(SR_ERR_INVALID, "sr_cg_solve: refresh_drop must be in [0, 1)");
  if (o.refine != 0 && o.refine != 1) return fail(SR_ERR_INVALID, "sr_cg_solve: refine must be 0 or 1");
  if (o.use_x0 != 0 && o.use_x0 != 1) return fail(SR_ERR_INVALID, "sr_cg_solve: use_x0 must be 0 or 1");
  if (o.precond != 0 && o.precond != 1) return fail(SR_ERR_INVALID, "sr_cg_solve: precond must be 0 or 1");
  if (o.precond && (O->O_lo != nullptr || (O->dtype != SR_F64 && O->dtype != SR_F32)))
    return fail(SR_ERR_INVALID, "sr_cg_solve: the Jacobi preconditioner needs SR_F64 or SR_F32 storage, one plane");
  int64_t max_iter = o.max_iter > 0 ? o.max_iter : O->n_p + 100;
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
  Plan pl;
  rc = make_plan(O->dtype, di.grid, O->n_s, O->n_p, 1, &pl);
  if (rc) return rc;
  const int64_t ypd = (int64_t)pl.pg.RG * O->n_p;
  const size_t bytes = prod_ws_bytes(pl, ypd) + (size_t)3 * (O->n_p * 8 + 256) + 1024;
  void *base = nullptr;
  rc = get_workspace(dev, stream, bytes, &base);
  if (rc) return rc;
  Carve cv(base);
  ProdWs w;
  carve_prod(cv, pl, ypd, &w);
  CgArgs a{};
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
  a.info = cv.take<double>(8);
  a.eps = eps;
  a.rtol = o.rtol;
  a.max_iter = (int)max_iter;
  a.refresh_every = o.refresh_every;
  a.use_x0 = o.use_x0;
  // refinement over two code planes: search directions and residuals use different
  // operators, so a refresh must restart the direction
  a.refine = (O->O_lo != nullptr && o.refine != 0) ? 1 : 0;
  a.restart_on_refresh = (o.restart_on_refresh != 0 || a.refine) ? 1 : 0;
  a.refresh_drop2 = o.refresh_drop * o.refresh_drop;
  a.hist = o.res_history;
  a.diag = diag;
  rc = zero_sync(w, stream);
  if (rc) return rc;
  const void *cg_fn =
      O->O_lo == nullptr ? (o.precond ? pl.ke->cgj : pl.ke->cg) : (a.refine ? pl.ke->cgr : pl.ke->cg2);
  if (cg_fn == nullptr) return fail(SR_ERR_INVALID, "sr_cg_solve: no two-plane CG kernel for this configuration");
  rc = launch_coop(cg_fn, pl.pg.G, &a, stream, pl.ke->nt, pl.ke->ring_bytes);
  if (rc) return rc;
  double hinfo[8];
  uint32_t habort = 0;
  HIP_TRY(hipMemcpyAsync(hinfo, a.info, sizeof(hinfo), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&habort, w.sb.abort, sizeof(habort), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  int status = (int)hinfo[2];
  if (habort != 0u || hinfo[6] == 0.0) status = fail(SR_ERR_TIMEOUT, "sr_cg_solve: a cross-workgroup wait timed out");
  else if (status == SR_ERR_NONFINITE) fail(SR_ERR_NONFINITE, "sr_cg_solve: non-finite scalar in CG");
  else if (status == SR_BREAKDOWN) fail(SR_BREAKDOWN, "sr_cg_solve: p.(S+eps I)p <= 0");
  else if (status == SR_NOT_CONVERGED) fail(SR_NOT_CONVERGED, "sr_cg_solve: max_iter reached");
  if (info) {
    info->iters = (int32_t)hinfo[0];
    info->refreshes = (int32_t)hinfo[1];
    info->status = status;
    info->products = (int32_t)hinfo[3];
    info->rel_res_recur = hinfo[4];
    info->rel_res_true = hinfo[5];
  }
  return status;
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

}  // extern "C"
