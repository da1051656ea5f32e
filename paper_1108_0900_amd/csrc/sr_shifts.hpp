// Multi-shift CG: one right-hand side g and up to kMaxShifts shifts eps_s, all solved from
// the Krylov sequence of the smallest shift (Krylov spaces do not depend on the shift).
// Per iteration one fused product with (S + eps_0 I) serves every shift; the shifted
// systems follow by scalar recurrences (the collinear-residual form of shifted CG):
//   zeta_s' = zeta_s zeta_s^- alpha^- / (alpha beta^- (zeta_s^- - zeta_s)
//                                        + zeta_s^- alpha^- (1 + (eps_s - eps_0) alpha))
//   alpha_s = alpha zeta_s' / zeta_s,  x_s += alpha_s p_s,
//   beta_s = beta (zeta_s' / zeta_s)^2,  p_s = zeta_s' r + beta_s p_s,  r_s = zeta_s' r,
// with zeta = zeta^- = 1, alpha^- = 1, beta^- = 0 at the start (the base shift keeps
// zeta = 1).  A shift stops moving once |zeta_s| ||r|| <= rtol ||g||.  Residual
// replacement would break the collinearity, so there are no refreshes; the host checks
// every shift's true residual afterwards.
#pragma once
#include "sr_kernels.hpp"

namespace sr {

constexpr int kMaxShifts = 8;

struct ShiftArgs {
  CgArgs c;                          // g, x (unused), r, p (base direction), q, eps = eps_0, rtol, max_iter
  int n_shift;
  int check;                         // 1: true residual of every shift at the end (in the launch)
  double dshift[kMaxShifts];         // eps_s - eps_0 (>= 0)
  double *xrow[kMaxShifts];          // [n_p] solution of each shift (increasing eps)
  double *ps;                        // [n_shift][n_p] directions (row 0 unused: p holds it)
  double *sinfo;                     // [n_shift][2]: iterations, |zeta_s| ||r|| / ||g||; then status,
                                     // ok, products; then (check) [n_shift] true ||r_s|| / ||g||
};

// Multi-shift CG of one system (see above); returns false if the launch aborted.  ctx
// carries the barrier epochs and exchange steps in and out, nred the rotation of the grid
// reduction slots (several systems per launch: a system's first reduction must not reuse
// the slots of the previous system's last one, which no barrier separates from it).
template <int DT, int NV, int R, int L, int P_, int NT>
__device__ __forceinline__ bool shifts_body(const ShiftArgs &a, WgCtx &ctx, int &nred) {
  typedef CgKernel<DT, NV, R, L, P_, NT> K;
  const CgArgs &c = a.c;
  // Per-shift scalars are the same in every thread: thread 0 updates them in LDS and a
  // barrier publishes them, so that no register array holds them across the products.
  __shared__ double s_zeta[kMaxShifts], s_zold[kMaxShifts], s_as[kMaxShifts], s_zn[kMaxShifts], s_bs[kMaxShifts];
  __shared__ int s_done[kMaxShifts];       // iteration at which the shift stopped (-1: moving)
  __shared__ int s_any;
  const int G = (int)gridDim.x, tid = (int)threadIdx.x, ns = a.n_shift;
  const int64_t n = c.pg.n_p;
  const int64_t ch = (n + G - 1) / G;
  const int64_t j0 = min(n, (int64_t)blockIdx.x * ch), j1 = min(n, j0 + ch);
  int products = 0, status = 0, it = 0;
  double rr, gg, dummy;
  bool ok = true;
  {
    double prr = 0.0;
    for (int64_t j = j0 + tid; j < j1; j += NT) {
      const double gj = c.g[j];
      c.r[j] = gj;
      st_coh(&c.p[j], gj);
      for (int s = 0; s < ns; ++s) {
        a.xrow[s][j] = 0.0;
        if (s > 0) a.ps[s * n + j] = gj;
      }
      prr += gj * gj;
    }
    ok = grid_allreduce2(prr, 0.0, c.sb.red, nred, ctx.gs, rr, dummy);
  }
  gg = rr;
  if (tid == 0) {
    for (int s = 0; s < kMaxShifts; ++s) {
      s_zeta[s] = 1.0;
      s_zold[s] = 1.0;
      s_done[s] = (s >= ns || gg == 0.0) ? 0 : -1;
    }
  }
  __syncthreads();
  double alpha_old = 1.0, beta_old = 0.0;
  const double stop2 = c.rtol * c.rtol * gg;
  while (ok) {
    if (tid == 0) {
      int any = 0;
      for (int s = 0; s < ns; ++s) any |= s_done[s] < 0 ? 1 : 0;
      s_any = any;
    }
    __syncthreads();
    if (!s_any) break;
    if (it >= c.max_iter) {
      status = 1;
      break;
    }
    // q = (S + eps_0 I) p
    if (!(ok = K::template apply<false>(c, ctx, c.p, c.q, j0, j1, products))) break;
    double ppq = 0.0, pq;
    for (int64_t j = j0 + tid; j < j1; j += NT) ppq += ld_coh(&c.p[j]) * c.q[j];
    if (!(ok = grid_allreduce2(ppq, 0.0, c.sb.red, nred, ctx.gs, pq, dummy))) break;
    if (!isfinite(pq)) {
      status = -4;
      break;
    }
    if (!(pq > 0.0)) {
      status = 2;
      break;
    }
    const double alpha = rr / pq;
    if (tid == 0) {
      for (int s = 0; s < ns; ++s) {
        s_zn[s] = s_zeta[s];
        s_as[s] = 0.0;
        if (s_done[s] < 0) {
          const double den = alpha * beta_old * (s_zold[s] - s_zeta[s]) +
                             s_zold[s] * alpha_old * (1.0 + a.dshift[s] * alpha);
          s_zn[s] = s_zeta[s] * s_zold[s] * alpha_old / den;
          s_as[s] = alpha * s_zn[s] / s_zeta[s];
        }
      }
    }
    __syncthreads();
    double prr = 0.0;
    for (int64_t j = j0 + tid; j < j1; j += NT) {
      const double p0 = ld_coh(&c.p[j]);
      for (int s = 0; s < ns; ++s) {
        const double as = s_as[s];
        if (as != 0.0) a.xrow[s][j] += as * (s == 0 ? p0 : a.ps[s * n + j]);
      }
      const double rj = c.r[j] - alpha * c.q[j];
      c.r[j] = rj;
      prr += rj * rj;
    }
    double rr_new;
    if (!(ok = grid_allreduce2(prr, 0.0, c.sb.red, nred, ctx.gs, rr_new, dummy))) break;
    if (!isfinite(rr_new)) {
      status = -4;
      break;
    }
    const double beta = rr_new / rr;
    if (tid == 0) {
      for (int s = 0; s < ns; ++s) {
        const double t = s_zn[s] / s_zeta[s];
        s_bs[s] = beta * t * t;
      }
    }
    __syncthreads();
    for (int64_t j = j0 + tid; j < j1; j += NT) {
      const double rj = c.r[j];
      for (int s = 1; s < ns; ++s) {
        if (s_done[s] < 0) a.ps[s * n + j] = s_zn[s] * rj + s_bs[s] * a.ps[s * n + j];
      }
      st_coh(&c.p[j], rj + beta * ld_coh(&c.p[j]));    // the base sequence runs while any shift moves
    }
    it++;
    __syncthreads();                           // every thread has read s_done / s_zn
    if (tid == 0) {
      for (int s = 0; s < ns; ++s) {
        if (s_done[s] < 0 && s_zn[s] * s_zn[s] * rr_new <= stop2) s_done[s] = it;
        s_zold[s] = s_zeta[s];
        s_zeta[s] = s_zn[s];
      }
    }
    alpha_old = alpha;
    beta_old = beta;
    rr = rr_new;
    if (!(ok = grid_sync(ctx.gs))) break;      // p visible to every workgroup (and the LDS scalars)
  }
  if (blockIdx.x == 0 && tid == 0) {
    for (int s = 0; s < ns; ++s) {
      a.sinfo[s * 2 + 0] = (double)(s_done[s] < 0 ? it : s_done[s]);
      a.sinfo[s * 2 + 1] = sqrt(s_zeta[s] * s_zeta[s] * rr / (gg > 0.0 ? gg : 1.0));
    }
    a.sinfo[ns * 2] = (double)status;
    a.sinfo[ns * 2 + 1] = ok ? 1.0 : 0.0;
    a.sinfo[ns * 2 + 2] = (double)(products + (a.check ? ns : 0));
  }
  if (!ok || !a.check) return ok;
  // true residual of every shift, g - (S + eps_s I) x_s = g - (S + eps_0 I) x_s - dshift_s x_s:
  // the solutions go out with device-scope stores (the product reads other workgroups'
  // chunks), then one float64-accumulated product per shift
  for (int64_t j = j0 + tid; j < j1; j += NT)
    for (int sh = 0; sh < ns; ++sh) st_coh(&a.xrow[sh][j], a.xrow[sh][j]);
  if (!grid_sync(ctx.gs)) return false;
  for (int sh = 0; sh < ns; ++sh) {
    if (!K::template apply<K::kExactResidual>(c, ctx, a.xrow[sh], c.q, j0, j1, products)) return false;
    double prr = 0.0, tr;
    for (int64_t j = j0 + tid; j < j1; j += NT) {
      const double t = c.g[j] - K::ldq(&c.q[j]) - a.dshift[sh] * ld_coh(&a.xrow[sh][j]);
      prr += t * t;
    }
    if (!grid_allreduce2(prr, 0.0, c.sb.red, nred, ctx.gs, tr, dummy)) return false;
    if (blockIdx.x == 0 && tid == 0) a.sinfo[ns * 2 + 3 + sh] = gg > 0.0 ? sqrt(tr / gg) : 0.0;
  }
  return true;
}

template <int DT, int NV, int R, int L, int P_, int NT>
__global__ __launch_bounds__(NT) void k_cg_shifts(ShiftArgs a) {
  WgCtx ctx;
  init_ctx(ctx, a.c.pg, a.c.sb.flags, a.c.sb.abort, Storage<DT>::VEC);
  int nred = 0;
  shifts_body<DT, NV, R, L, P_, NT>(a, ctx, nred);
}

// Many systems in one persistent launch, one after another (each its own matrix geometry,
// one right-hand side, up to kMaxShifts shifts): the argument blocks sit in device memory
// and each is copied to LDS for its system (read through a global pointer they would be
// reloaded after every store); the barrier epochs, exchange steps and reduction slots
// continue from system to system.  Every system has its own vectors (a vector reused with
// another chunking would take plain stores of the same address from several XCDs).
template <int DT, int NV, int R, int L, int P_, int NT>
__global__ __launch_bounds__(NT) void k_cg_shifts_batched(const ShiftArgs *sys, int n_sys) {
  static_assert(sizeof(ShiftArgs) % 8 == 0, "the argument block is copied in 8-byte words");
  __shared__ ShiftArgs s_args;
  WgCtx ctx;
  uint32_t epoch = 0, xstep = 0;
  int nred = 0;
  for (int i = 0; i < n_sys; ++i) {
    __syncthreads();                     // the previous system no longer reads s_args
    for (int w = (int)threadIdx.x; w < (int)(sizeof(ShiftArgs) / 8); w += NT)
      ((u64 *)&s_args)[w] = ((const u64 *)&sys[i])[w];
    __syncthreads();
    const ShiftArgs &a = s_args;
    init_ctx(ctx, a.c.pg, a.c.sb.flags, a.c.sb.abort, Storage<DT>::VEC);
    ctx.gs.epoch = epoch;
    ctx.xstep = xstep;
    if (!shifts_body<DT, NV, R, L, P_, NT>(a, ctx, nred)) return;
    epoch = ctx.gs.epoch;
    xstep = ctx.xstep;
  }
}

// Multi-shift kernels of float64 and float32 storage, one per SR tile configuration.
struct ShiftEntry {
  int nv, r, look, poll, nt;
  const void *fn, *batched;
};
// The kernel for a tile configuration, or nullptr (other storage types).
const void *shift_kernel(int dt, int nv, int r, int look, int poll, int nt, bool batched = false);

}  // namespace sr
