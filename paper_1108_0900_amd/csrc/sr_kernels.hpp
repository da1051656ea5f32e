// libsr kernel templates for gfx950: prepare/gradient pass, bf16/f16 quantizer, fused
// overlap product, persistent conjugate gradient, and the linear-method Hamiltonian
// product.  Instantiated per storage type in sr_kernels_<type>.hip.
#pragma once
#include "sr_product.hpp"
#include "sr_launch.hpp"

namespace sr {

// ======================================================================================
// Shared helpers
// ======================================================================================

// Sum of one float64 per workgroup over the grid, visible to all workgroups.  `red` is
// [4 sets][2 values][G]; consecutive calls rotate the set, which is safe because at least
// one grid barrier separates a set's reads from its next writes.
__device__ __forceinline__ bool grid_allreduce2(double a, double b, double *red, int &nred, GridSync &gs,
                                                double &A, double &B) {
  const int G = (int)gridDim.x;
  const int set = nred & 3;
  nred++;
  a = block_sum(a);
  b = block_sum(b);
  if (threadIdx.x == 0) {
    st_coh(&red[(set * 2 + 0) * G + blockIdx.x], a);
    st_coh(&red[(set * 2 + 1) * G + blockIdx.x], b);
  }
  if (!grid_sync(gs)) return false;
  A = grid_sum_read(&red[(set * 2 + 0) * G]);
  B = grid_sum_read(&red[(set * 2 + 1) * G]);
  return true;
}

__device__ __forceinline__ double code_value(const unsigned char *rowp, int64_t col, int dt) {
  if (dt == DT_BF16) return (double)__uint_as_float((uint32_t)((const uint16_t *)rowp)[col] << 16);
  return (double)(float)__builtin_bit_cast(_Float16, ((const uint16_t *)rowp)[col]);
}

// Stored value of element `col` of a row (both code planes when `lorow` is given).
__device__ __forceinline__ double load_decoded(const unsigned char *rowp, const unsigned char *lorow, int64_t col,
                                               int dt, const float *scale) {
  switch (dt) {
    case DT_F64: return ((const double *)rowp)[col];
    case DT_F32: return (double)((const float *)rowp)[col];
    default: {
      double q = code_value(rowp, col, dt);
      if (lorow != nullptr) q += code_value(lorow, col, dt);
      return q * (double)scale[col];
    }
  }
}

// ======================================================================================
// Prepare / gradient pass (one read of O):  column means, diag S, g, E mean.
// Shifted sums about K_j = O_0j avoid the cancellation of sum(O^2) - N mean^2.
// ======================================================================================
template <int DT, int NV, int RT>
__global__ __launch_bounds__(kNT) void k_grad(GradArgs a) {
  typedef Storage<DT> St;
  constexpr int VEC = St::VEC;
  WgCtx ctx;
  init_ctx(ctx, a.pg, a.sb.flags, a.sb.abort, VEC);
  const int G = (int)gridDim.x, tid = (int)threadIdx.x;
  int nred = 0;
  const double inv_n = 1.0 / (double)a.pg.n_s;

  // --- energies: mean and the residual sum of (E - mean) ---
  double Emean = 0.0, sum_e = 0.0;
  if (a.E != nullptr) {
    const int64_t ch = (a.pg.n_s + G - 1) / G;
    const int64_t k0 = min(a.pg.n_s, (int64_t)blockIdx.x * ch), k1 = min(a.pg.n_s, k0 + ch);
    double s = 0.0;
    for (int64_t k = k0 + tid; k < k1; k += kNT) s += a.E[k];
    double dummy;
    if (!grid_allreduce2(s, 0.0, a.sb.red, nred, ctx.gs, Emean, dummy)) return;
    Emean *= inv_n;
    double se = 0.0;
    for (int64_t k = k0 + tid; k < k1; k += kNT) se += a.E[k] - Emean;
    if (!grid_allreduce2(se, 0.0, a.sb.red, nred, ctx.gs, sum_e, dummy)) return;
  }

  // --- column sums over this row group's rows, for the owned columns ---
  int64_t colv[NV];
  double K[NV][VEC], sA[NV][VEC], sB[NV][VEC], sC[NV][VEC];
  const unsigned char *O = a.op.O;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int64_t col = ctx.c0 + ((int64_t)i * kNT + tid) * VEC;
    colv[i] = (col < ctx.c1) ? col : -1;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      K[i][e] = 0.0;
      if (colv[i] >= 0 && col + e < a.pg.n_p) K[i][e] = load_decoded(O, a.op.lo, col + e, DT, a.op.scale);
      sA[i][e] = sB[i][e] = sC[i][e] = 0.0;
    }
  }
  double sc[NV][VEC];
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int64_t col = colv[i] + e;
      sc[i][e] = (a.op.scale != nullptr && colv[i] >= 0 && col < a.pg.n_p) ? (double)a.op.scale[col] : 1.0;
    }
  const int64_t n_tiles = (a.pg.n_s + RT - 1) / RT;
  const unsigned char *LO = a.op.lo;
  for (int64_t t = ctx.rg; t < n_tiles; t += a.pg.RG) {
    u32x4 buf[RT][NV], bufl[RT][NV];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const int64_t row = t * RT + r;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        if (row < a.pg.n_s && colv[i] >= 0) buf[r][i] = load_stream(O + row * a.op.ldb + colv[i] * St::BYTES);
        else buf[r][i] = u32x4{0u, 0u, 0u, 0u};
        if (LO != nullptr && row < a.pg.n_s && colv[i] >= 0)
          bufl[r][i] = load_stream(LO + row * a.op.ldb + colv[i] * St::BYTES);
        else bufl[r][i] = u32x4{0u, 0u, 0u, 0u};
      }
    }
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const int64_t row = t * RT + r;
      if (row >= a.pg.n_s) continue;
      const double e_k = (a.E != nullptr) ? a.E[row] - Emean : 0.0;
#pragma unroll
      for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const double q = (double)St::get(buf[r][i], e) + (double)St::get(bufl[r][i], e);
          const double x = q * sc[i][e] - K[i][e];
          sA[i][e] += x;
          sB[i][e] = fma(x, x, sB[i][e]);
          sC[i][e] = fma(e_k, x, sC[i][e]);
        }
    }
  }
  // partials: ypart holds [RG][3][n_p]
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (colv[i] < 0) continue;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int64_t col = colv[i] + e;
      if (col >= a.pg.n_p) continue;
      double *base = a.pb.ypart + (int64_t)ctx.rg * 3 * a.pg.n_p;
      st_coh(&base[col], sA[i][e]);
      st_coh(&base[a.pg.n_p + col], sB[i][e]);
      st_coh(&base[2 * a.pg.n_p + col], sC[i][e]);
    }
  }
  if (!grid_sync(ctx.gs)) return;

  // --- finish owned column chunk ---
  const int64_t ch = (a.pg.n_p + G - 1) / G;
  const int64_t j0 = min(a.pg.n_p, (int64_t)blockIdx.x * ch), j1 = min(a.pg.n_p, j0 + ch);
  for (int64_t j = j0 + tid; j < j1; j += kNT) {
    double A = 0.0, B = 0.0, Cg = 0.0;
    for (int rg = 0; rg < a.pg.RG; ++rg) {
      const double *base = a.pb.ypart + (int64_t)rg * 3 * a.pg.n_p;
      A += ld_coh(&base[j]);
      B += ld_coh(&base[a.pg.n_p + j]);
      Cg += ld_coh(&base[2 * a.pg.n_p + j]);
    }
    const double Kj = load_decoded(O, a.op.lo, j, DT, a.op.scale);
    const double dmean = A * inv_n;
    if (a.mean_out) a.mean_out[j] = Kj + dmean;
    if (a.diag_out) {
      double var = B * inv_n - dmean * dmean;
      a.diag_out[j] = var > 0.0 ? var : 0.0;
    }
    if (a.g_out) a.g_out[j] = 2.0 * inv_n * (Cg - dmean * sum_e);
  }
  if (blockIdx.x == 0 && tid == 0 && a.Emean_out) *a.Emean_out = Emean;
}

// ======================================================================================
// Quantizer: per-column absmax scale, then round-to-nearest-even codes.
// ======================================================================================
template <int IN_DT>
__global__ __launch_bounds__(kNT) void k_absmax(QuantArgs a) {
  WgCtx ctx;
  init_ctx(ctx, a.pg, a.sb.flags, a.sb.abort, 1);
  const int G = (int)gridDim.x, tid = (int)threadIdx.x;
  // slice of columns per column group, one column per thread per pass
  for (int64_t col = ctx.c0 + tid; col < ctx.c1; col += kNT) {
    double m = 0.0;
    for (int64_t row = ctx.rg; row < a.pg.n_s; row += a.pg.RG) {
      const double x = (IN_DT == DT_F64) ? ((const double *)(a.in + row * a.ldb_in))[col]
                                         : (double)((const float *)(a.in + row * a.ldb_in))[col];
      m = fmax(m, fabs(x));
    }
    st_coh(&a.pb.ypart[(int64_t)ctx.rg * a.pg.n_p + col], m);
  }
  if (!grid_sync(ctx.gs)) return;
  const int64_t ch = (a.pg.n_p + G - 1) / G;
  const int64_t j0 = min(a.pg.n_p, (int64_t)blockIdx.x * ch), j1 = min(a.pg.n_p, j0 + ch);
  for (int64_t j = j0 + tid; j < j1; j += kNT) {
    double m = 0.0;
    for (int rg = 0; rg < a.pg.RG; ++rg) m = fmax(m, ld_coh(&a.pb.ypart[(int64_t)rg * a.pg.n_p + j]));
    float s = (float)m;
    if (s == 0.0f) s = 1.0f;
    a.scale[j] = s;
  }
}

// Round a float64 to bf16 / f16 (nearest, ties to even) via float32 rounded to odd.
__device__ __forceinline__ uint32_t f64_to_f32_odd_bits(double t) {
  const float f = __double2float_rz(t);
  uint32_t b = __float_as_uint(f);
  if ((double)f != t) b |= 1u;
  return b;
}
__device__ __forceinline__ uint16_t rne_bf16(double t) {
  const uint32_t b = f64_to_f32_odd_bits(t);
  return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ uint16_t rne_f16(double t) {
  const float f = __uint_as_float(f64_to_f32_odd_bits(t));
  return __builtin_bit_cast(uint16_t, (_Float16)f);
}

template <int IN_DT, int OUT_DT>
__global__ __launch_bounds__(kNT) void k_quantize(QuantArgs a) {
  const int64_t nvec_row = a.ld_out / 8;      // 8 codes per 16-byte output vector
  const int64_t total = a.pg.n_s * nvec_row;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = idx / nvec_row, c0 = (idx % nvec_row) * 8;
    const unsigned char *rin = a.in + row * a.ldb_in;
    uint32_t w[4], wl[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      uint32_t pair = 0, lpair = 0;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int64_t col = c0 + 2 * h + e;
        uint16_t code = 0, lcode = 0;
        if (col < a.pg.n_p) {
          const double x = (IN_DT == DT_F64) ? ((const double *)rin)[col] : (double)((const float *)rin)[col];
          const double t = x / (double)a.scale[col];
          code = (OUT_DT == DT_BF16) ? rne_bf16(t) : rne_f16(t);
          if (a.out_lo != nullptr) {
            const double hv = (OUT_DT == DT_BF16) ? (double)__uint_as_float((uint32_t)code << 16)
                                                  : (double)(float)__builtin_bit_cast(_Float16, code);
            lcode = (OUT_DT == DT_BF16) ? rne_bf16(t - hv) : rne_f16(t - hv);
          }
        }
        pair |= (uint32_t)code << (16 * e);
        lpair |= (uint32_t)lcode << (16 * e);
      }
      w[h] = pair;
      wl[h] = lpair;
    }
    *(u32x4 *)(a.out + row * a.ld_out * 2 + c0 * 2) = u32x4{w[0], w[1], w[2], w[3]};
    if (a.out_lo != nullptr) *(u32x4 *)(a.out_lo + row * a.ld_out * 2 + c0 * 2) = u32x4{wl[0], wl[1], wl[2], wl[3]};
  }
}

// ======================================================================================
// (S + eps I) v
// ======================================================================================
template <int DT, int NV, int R, int L, int P_, int NT>
__global__ __launch_bounds__(NT) void k_sv(SvArgs a) {
  WgCtx ctx;
  init_ctx(ctx, a.pg, a.sb.flags, a.sb.abort, Storage<DT>::VEC);
  Product<DT, NV, R, 1, false, L, P_, NT> P;
  const double cshare = P.setup(ctx, a.pg, &a.op, a.mean, a.v);
  bool ok = P.accumulate(a.pg, a.pb, ctx, &a.op, cshare, nullptr, 0.0);
  if (ok) {
    P.store_partials(a.pg, a.pb, ctx);
    ok = grid_sync(ctx.gs);
  }
  const int G = (int)gridDim.x;
  const int64_t ch = (a.pg.n_p + G - 1) / G;
  const int64_t j0 = min(a.pg.n_p, (int64_t)blockIdx.x * ch), j1 = min(a.pg.n_p, j0 + ch);
  if (!ok) {   // a wait gave up: the result is NaN, never stale data
    for (int64_t j = j0 + threadIdx.x; j < j1; j += NT) a.y[j] = __builtin_nan("");
    return;
  }
  double S1, S2;
  sum_row_scalars(a.pb, a.pg, S1, S2);
  const double inv_n = 1.0 / (double)a.pg.n_s;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += NT) {
    const double acc = finish_column(a.pb, a.pg, j);
    const double s = a.op.scale ? (double)a.op.scale[j] : 1.0;
    a.y[j] = (s * acc - a.mean[j] * S1) * inv_n + a.eps * a.v[j];
  }
}

// (S + eps I) v for two code planes (stored value s_j (q + lo)), float64 accumulation.
template <int DT, int NV, int NT>
__global__ __launch_bounds__(NT) void k_sv2(SvArgs a) {
  WgCtx ctx;
  init_ctx(ctx, a.pg, a.sb.flags, a.sb.abort, Storage<DT>::VEC);
  Product<DT, NV, 1, 1, true, 1, 1, NT, 2> P;
  const double cshare = P.setup(ctx, a.pg, &a.op, a.mean, a.v);
  bool ok = P.accumulate(a.pg, a.pb, ctx, &a.op, cshare, nullptr, 0.0);
  if (ok) {
    P.store_partials(a.pg, a.pb, ctx);
    ok = grid_sync(ctx.gs);
  }
  const int G = (int)gridDim.x;
  const int64_t ch = (a.pg.n_p + G - 1) / G;
  const int64_t j0 = min(a.pg.n_p, (int64_t)blockIdx.x * ch), j1 = min(a.pg.n_p, j0 + ch);
  if (!ok) {   // a wait gave up: the result is NaN, never stale data
    for (int64_t j = j0 + threadIdx.x; j < j1; j += NT) a.y[j] = __builtin_nan("");
    return;
  }
  double S1, S2;
  sum_row_scalars(a.pb, a.pg, S1, S2);
  const double inv_n = 1.0 / (double)a.pg.n_s;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += NT) {
    const double acc = finish_column(a.pb, a.pg, j);
    a.y[j] = ((double)a.op.scale[j] * acc - a.mean[j] * S1) * inv_n + a.eps * a.v[j];
  }
}

// ======================================================================================
// Linear-method product  y = H v  (length n_p + 1)
// ======================================================================================
template <int DT, int NV, int R, int L, int P_, int NT>
__global__ __launch_bounds__(NT) void k_lm(LmArgs a) {
  WgCtx ctx;
  init_ctx(ctx, a.pg, a.sb.flags, a.sb.abort, Storage<DT>::VEC);
  Product<DT, NV, R, 2, false, L, P_, NT> P;
  const double v0 = a.v[0];
  const double cshare = P.setup(ctx, a.pg, a.ops, a.mean, a.v + 1);
  bool ok = P.accumulate(a.pg, a.pb, ctx, a.ops, cshare, a.E, v0);
  if (ok) {
    P.store_partials(a.pg, a.pb, ctx);
    ok = grid_sync(ctx.gs);
  }
  const int G = (int)gridDim.x;
  const int64_t ch = (a.pg.n_p + G - 1) / G;
  const int64_t j0 = min(a.pg.n_p, (int64_t)blockIdx.x * ch), j1 = min(a.pg.n_p, j0 + ch);
  if (!ok) {   // a wait gave up: the result is NaN, never stale data
    for (int64_t j = j0 + threadIdx.x; j < j1; j += NT) a.y[1 + j] = __builtin_nan("");
    if (blockIdx.x == 0 && threadIdx.x == 0) a.y[0] = __builtin_nan("");
    return;
  }
  double S1, S2;
  sum_row_scalars(a.pb, a.pg, S1, S2);
  const double inv_n = 1.0 / (double)a.pg.n_s;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += NT) {
    const double acc = finish_column(a.pb, a.pg, j);
    const double s = a.ops[0].scale ? (double)a.ops[0].scale[j] : 1.0;
    a.y[1 + j] = (s * acc - a.mean[j] * S1) * inv_n;
  }
  if (blockIdx.x == 0) {
    double se = 0.0;
    for (int64_t k = threadIdx.x; k < a.pg.n_s; k += NT) se += a.E[k];
    se = block_sum(se);
    if (threadIdx.x == 0) a.y[0] = se * inv_n * v0 + S2 * inv_n;
  }
}

// ======================================================================================
// Persistent conjugate gradient on (S + eps I) x = g
// ======================================================================================
template <int DT, int NV, int R, int L, int P_, int NT>
struct CgKernel {
  // q[j] = ((S + eps I) vin)_j for this workgroup's vector chunk [j0, j1).  EXACT selects
  // float64 accumulation (residual products of scaled storage).
  template <bool EXACT, int PLANES = 1>
  __device__ __forceinline__ static bool apply(const CgArgs &a, WgCtx &ctx, const double *vin, double *q,
                                               int64_t j0, int64_t j1, int &products) {
    // the float64-accumulated and the two-plane products use one-row tiles, one tile of
    // lookahead and the shortest poll depth (same column geometry, fewer registers)
    constexpr bool kSmall = EXACT || PLANES == 2;
    Product<DT, NV, (kSmall ? 1 : R), 1, EXACT, (kSmall ? 1 : L), (kSmall ? 1 : P_), NT, PLANES> P;
    const double cshare = P.setup(ctx, a.pg, &a.op, a.mean, vin);
    if (!P.accumulate(a.pg, a.pb, ctx, &a.op, cshare, nullptr, 0.0)) return false;
    P.store_partials(a.pg, a.pb, ctx);
    if (!grid_sync(ctx.gs)) return false;
    double S1, S2;
    sum_row_scalars(a.pb, a.pg, S1, S2);
    const double inv_n = 1.0 / (double)a.pg.n_s;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += NT) {
      const double acc = finish_column(a.pb, a.pg, j);
      const double s = a.op.scale ? (double)a.op.scale[j] : 1.0;
      q[j] = (s * acc - a.mean[j] * S1) * inv_n + a.eps * ld_coh(&vin[j]);
    }
    products++;
    return true;
  }
  // Residual products: float64 accumulation for scaled storage (the search-direction
  // products keep the storage type's own accumulation).
  static constexpr bool kExactResidual = (DT == DT_BF16 || DT == DT_F16);
};

// CGM selects the products of the solve, so that each kernel holds only the two it uses:
//   kCgOnePlane   one code plane: search directions in the storage type's accumulation,
//                 residuals float64-accumulated for scaled storage
//   kCgTwoPlanes  two code planes everywhere, float64 accumulation
//   kCgRefine     search directions on the first plane, residuals on both (refinement)
enum { kCgOnePlane = 0, kCgTwoPlanes = 1, kCgRefine = 2 };

template <int DT, int NV, int R, int L, int P_, int NT, int CGM = kCgOnePlane>
__global__ __launch_bounds__(NT) void k_cg(CgArgs a) {
  // Conjugate gradient (Hestenes-Stiefel) as a state machine with one product per pass
  // through the loop, so the product code is instantiated once per accumulation type.
  //   MODE_P        q = A p, then alpha, x += alpha p, r -= alpha q
  //   MODE_REFRESH  q = A x, r = g - q (every refresh_every iterations, or once the
  //                 recurrence residual fell by refresh_drop since the last refresh)
  //   MODE_CONFIRM  q = A x when the recurrence residual meets rtol; accept or replace r
  //   MODE_FINAL    q = A x to report the true residual of an unconverged exit
  //   MODE_X0       q = A x0 for a warm start
  typedef CgKernel<DT, NV, R, L, P_, NT> K;
  enum { MODE_P, MODE_REFRESH, MODE_CONFIRM, MODE_FINAL, MODE_X0, MODE_DONE };
  WgCtx ctx;
  init_ctx(ctx, a.pg, a.sb.flags, a.sb.abort, Storage<DT>::VEC);
  const int G = (int)gridDim.x, tid = (int)threadIdx.x;
  const int64_t n = a.pg.n_p;
  const int64_t ch = (n + G - 1) / G;
  const int64_t j0 = min(n, (int64_t)blockIdx.x * ch), j1 = min(n, j0 + ch);
  int nred = 0, products = 0, refreshes = 0, it = 0;
  int status = 0;       // SR_OK
  double rel_true = -1.0, rho = 0.0, gg = 1.0, dummy = 0.0;
  double rho_ref = 0.0;  // rho at the start or the last refresh (drop-triggered refreshes)
  bool ok = true, restart = false;
  int mode;

  // choose the next product from the recurrence residual
  auto decide = [&]() -> int {
    const double rel = sqrt(rho / gg);
    if (a.hist != nullptr && blockIdx.x == 0 && tid == 0 && it <= a.max_iter) a.hist[it] = rel;
    if (!isfinite(rho)) { status = -4; return MODE_DONE; }
    if (rel <= a.rtol) return MODE_CONFIRM;
    if (it >= a.max_iter) { status = 1; return MODE_FINAL; }
    return MODE_P;
  };
  // p <- r + beta p for the own chunk, then a barrier so every workgroup sees p
  auto update_p = [&](double beta) -> bool {
    for (int64_t j = j0 + tid; j < j1; j += NT) st_coh(&a.p[j], a.r[j] + beta * ld_coh(&a.p[j]));
    return grid_sync(ctx.gs);
  };

  if (a.use_x0) {
    mode = MODE_X0;
  } else {
    double prr = 0.0, pgg = 0.0;
    for (int64_t j = j0 + tid; j < j1; j += NT) {
      st_coh(&a.x[j], 0.0);
      const double gj = a.g[j];
      a.r[j] = gj;
      st_coh(&a.p[j], gj);
      prr += gj * gj;
      pgg += gj * gj;
    }
    ok = grid_allreduce2(prr, pgg, a.sb.red, nred, ctx.gs, rho, gg);
    rho_ref = rho;
    if (gg == 0.0) {
      gg = 1.0;
      rel_true = 0.0;
      mode = MODE_DONE;
    } else {
      mode = decide();
    }
  }

  while (ok && mode != MODE_DONE) {
    const bool on_p = (mode == MODE_P);
    if constexpr (CGM == kCgTwoPlanes) {
      // one product code for search directions and residuals: float64 accumulation
      // (measured faster here than float32 with the two planes in one kernel)
      ok = K::template apply<true, 2>(a, ctx, on_p ? a.p : a.x, a.q, j0, j1, products);
    } else if constexpr (CGM == kCgRefine) {
      if (on_p) ok = K::template apply<false>(a, ctx, a.p, a.q, j0, j1, products);
      else ok = K::template apply<true, 2>(a, ctx, a.x, a.q, j0, j1, products);
    } else if constexpr (K::kExactResidual) {
      if (on_p) ok = K::template apply<false>(a, ctx, a.p, a.q, j0, j1, products);
      else ok = K::template apply<true>(a, ctx, a.x, a.q, j0, j1, products);
    } else {
      ok = K::template apply<false>(a, ctx, on_p ? a.p : a.x, a.q, j0, j1, products);
    }
    if (!ok) break;
    if (mode == MODE_P) {
      double ppq = 0.0, pq;
      for (int64_t j = j0 + tid; j < j1; j += NT) ppq += ld_coh(&a.p[j]) * a.q[j];
      if (!(ok = grid_allreduce2(ppq, 0.0, a.sb.red, nred, ctx.gs, pq, dummy))) break;
      if (!isfinite(pq)) { status = -4; break; }
      if (!(pq > 0.0)) { status = 2; mode = MODE_FINAL; continue; }
      const double alpha = rho / pq;
      double prr = 0.0;
      for (int64_t j = j0 + tid; j < j1; j += NT) {
        st_coh(&a.x[j], ld_coh(&a.x[j]) + alpha * ld_coh(&a.p[j]));
        const double rj = a.r[j] - alpha * a.q[j];
        a.r[j] = rj;
        prr += rj * rj;
      }
      it++;
      if (a.refresh_every > 0 && it % a.refresh_every == 0) {
        if (!(ok = grid_sync(ctx.gs))) break;      // x visible to the refresh product
        mode = MODE_REFRESH;
        continue;
      }
      double rho_new;
      if (!(ok = grid_allreduce2(prr, 0.0, a.sb.red, nred, ctx.gs, rho_new, dummy))) break;
      if (rho_new <= a.refresh_drop2 * rho_ref && sqrt(rho_new / gg) > a.rtol) {
        // the recurrence residual fell by the requested factor: refresh now (x is
        // visible to every workgroup after the reduction's grid barrier)
        mode = MODE_REFRESH;
        continue;
      }
      const double beta = rho_new / rho;
      rho = rho_new;
      if (!(ok = update_p(beta))) break;
      mode = decide();
    } else if (mode == MODE_REFRESH) {
      double prr = 0.0, rho_new;
      for (int64_t j = j0 + tid; j < j1; j += NT) {
        const double rj = a.g[j] - a.q[j];
        a.r[j] = rj;
        prr += rj * rj;
      }
      refreshes++;
      if (!(ok = grid_allreduce2(prr, 0.0, a.sb.red, nred, ctx.gs, rho_new, dummy))) break;
      const double beta = a.restart_on_refresh ? 0.0 : rho_new / rho;
      rho = rho_new;
      rho_ref = rho_new;
      if (!(ok = update_p(beta))) break;
      mode = decide();
    } else if (mode == MODE_X0) {
      double prr = 0.0, pgg = 0.0;
      for (int64_t j = j0 + tid; j < j1; j += NT) {
        const double gj = a.g[j], rj = gj - a.q[j];
        a.r[j] = rj;
        st_coh(&a.p[j], rj);
        prr += rj * rj;
        pgg += gj * gj;
      }
      if (!(ok = grid_allreduce2(prr, pgg, a.sb.red, nred, ctx.gs, rho, gg))) break;
      rho_ref = rho;
      if (gg == 0.0) {
        for (int64_t j = j0 + tid; j < j1; j += NT) st_coh(&a.x[j], 0.0);
        gg = 1.0;
        rho = 0.0;
        rel_true = 0.0;
        mode = MODE_DONE;
      } else {
        mode = decide();
      }
    } else {   // MODE_CONFIRM or MODE_FINAL: true residual g - A x
      double prr = 0.0, tr;
      for (int64_t j = j0 + tid; j < j1; j += NT) {
        const double t = a.g[j] - a.q[j];
        if (mode == MODE_CONFIRM) a.r[j] = t;
        prr += t * t;
      }
      if (!(ok = grid_allreduce2(prr, 0.0, a.sb.red, nred, ctx.gs, tr, dummy))) break;
      rel_true = sqrt(tr / gg);
      if (mode == MODE_FINAL || rel_true <= a.rtol) {
        mode = MODE_DONE;
      } else if (it >= a.max_iter) {
        status = 1;
        mode = MODE_DONE;
      } else {
        // the recurrence residual drifted from the true one: continue from the true one
        rho = tr;
        rho_ref = tr;
        refreshes++;
        rel_true = -1.0;
        if (a.restart_on_refresh && !(ok = update_p(0.0))) break;
        mode = MODE_P;
      }
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    a.info[0] = (double)it;
    a.info[1] = (double)refreshes;
    a.info[2] = (double)status;
    a.info[3] = (double)products;
    a.info[4] = sqrt(rho / gg);
    a.info[5] = rel_true;
    a.info[6] = ok ? 1.0 : 0.0;
  }
}

// ======================================================================================
// Several right-hand sides: Y = (S + diag(eps)) V for the K columns of V
// ======================================================================================
// Sum of N values per workgroup over the grid, the same in every workgroup (fixed order).
// red: [4][N][G] slots used round-robin (a set is reused only after three more
// reductions, each of which contains a grid barrier).
template <int N>
__device__ __forceinline__ bool grid_allreduce_n(const double (&in)[N], double *red, int &nred, GridSync &gs,
                                                 double (&out)[N]) {
  __shared__ double s_w[16][N];
  __shared__ double s_o[N];
  const int G = (int)gridDim.x, set = nred & 3;
  const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
  nred++;
#pragma unroll
  for (int n = 0; n < N; ++n) {
    const double w = wave_sum(in[n]);
    if (lane == 0) s_w[wave][n] = w;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += s_w[w][threadIdx.x];
    st_coh(&red[((int64_t)set * N + threadIdx.x) * G + blockIdx.x], t);
  }
  if (!grid_sync(gs)) return false;
  if (wave < N) {      // wave n sums value n over the grid
    double acc = 0.0;
    for (int i = lane; i < G; i += 64) acc += ld_coh(&red[((int64_t)set * N + wave) * G + i]);
    acc = wave_sum(acc);
    if (lane == 0) s_o[wave] = acc;
  }
  if (N > 16) {        // more values than waves: the remaining ones by wave 0
    for (int n = 16; n < N; ++n) {
      if (wave == 0) {
        double acc = 0.0;
        for (int i = lane; i < G; i += 64) acc += ld_coh(&red[((int64_t)set * N + n) * G + i]);
        acc = wave_sum(acc);
        if (lane == 0) s_o[n] = acc;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int n = 0; n < N; ++n) out[n] = s_o[n];
  __syncthreads();
  return true;
}

// Y = (S + diag(eps)) V for the K columns of V in two passes over O, float64-accumulated.
// Eight columns at once make a one-pass product arithmetic-bound (each element of O
// takes part in K dots and K updates); split into passes, each does K multiply-adds per
// element and stays bound by the stream of O.
//   0. vs_k = s_j v_kj (scaled operand) and c_k = obar . v_k (grid sum).
//   1. Row dots: a workgroup takes a block of NW * kBatchRows rows (kBatchRows per wave)
//      and one column part; it walks the part in chunks of 64 * VEC columns, the chunk of
//      vs staged in LDS (double-buffered, next chunk's vs and tiles loaded during the
//      current one), and writes wp[part][row][k] (c_k taken off in part 0).
//   2. Updates: a workgroup takes threads * VEC columns and one split of the rows; the
//      split's centred row dots (summed over parts) sit in LDS, each thread accumulates
//      sum_rows O_rj w[row][k] for its VEC columns and all k, rows kBatchU at a time.
//   3. Finish: y_kj = (s_j sum_sp yp - obar_j sum_rows w_k) / N + eps_k v_kj.
// Buffers written in one pass and read by other workgroups in the next are accessed
// coherently; a grid barrier separates the passes.
constexpr int kBatchU = 8;   // rows in flight per thread in the update pass

template <int DT, int NT>
struct BatchProduct {
  typedef Storage<DT> St;
  static constexpr int K = kBatchK, VEC = St::VEC, NW = NT / 64, RB = kBatchRows;
  static constexpr int CW = 64 * VEC;            // columns per chunk of the row-dot pass
  static constexpr int BW = NT * VEC;            // columns per block of the update pass
  static constexpr int KPT = K * CW / NT;        // staged vs values per thread and chunk
  static constexpr int kLds = (2 * K * CW > K * kBatchSplitRows) ? 2 * K * CW : K * kBatchSplitRows;
  static_assert(K * CW % NT == 0, "chunk staging must divide evenly");
  static_assert(RB * K == 32, "the row-dot reduction takes 32 values per wave");

  __device__ __forceinline__ static double *lds() {
    __shared__ double s_buf[kLds];
    return s_buf;
  }

  // element e of a 16-byte vector, zero where masked (padding past n_p may hold NaN)
  __device__ __forceinline__ static double elem(const u32x4 &t, int e, bool in) {
    return in ? (double)St::get(t, e) : 0.0;
  }

  __device__ __forceinline__ static void stage_load(const BatchArgs &a, double (&vr)[KPT], int64_t c0, int64_t ce) {
#pragma unroll
    for (int m = 0; m < KPT; ++m) {
      const int idx = (int)threadIdx.x + m * NT;
      const int k = idx / CW, jj = idx % CW;
      const int64_t col = c0 + jj;
      vr[m] = col < ce ? ld_coh(&a.vs[k * a.vstride + col]) : 0.0;
    }
  }
  __device__ __forceinline__ static void stage_store(double *buf, const double (&vr)[KPT]) {
#pragma unroll
    for (int m = 0; m < KPT; ++m) buf[(int)threadIdx.x + m * NT] = vr[m];
  }
  __device__ __forceinline__ static void tiles_load(u32x4 (&t)[RB], const unsigned char *const (&rowp)[RB],
                                                    int64_t col) {
#pragma unroll
    for (int r = 0; r < RB; ++r) t[r] = load_stream(rowp[r] + col * St::BYTES);
  }

  // Pass 1 over this workgroup's tasks.
  __device__ static void row_dots(const BatchArgs &a, const BatchSys &S, const double (&c)[K]) {
    const BatchGeom &g = S.bg;
    double *const sv = lds();
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const int64_t ntask = g.n_rb * g.P;
    for (int64_t task = blockIdx.x; task < ntask; task += gridDim.x) {
      const int64_t rb = task / g.P;
      const int part = (int)(task % g.P);
      const int64_t cs = (int64_t)part * g.pw, ce = min(g.n_p, cs + g.pw);
      const int64_t r0 = rb * (NW * RB) + wave * RB;
      const unsigned char *rowp[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) rowp[r] = S.op.O + min(r0 + r, g.n_s - 1) * S.op.ldb;
      double acc[RB][K];
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[r][k] = 0.0;
      const int nch = (int)((ce - cs + CW - 1) / CW);
      double vr[KPT];
      u32x4 cur[RB], nxt[RB];
      // a lane past the part's end reads the part's first vector (masked below)
      auto lane_col = [&](int64_t c0) { return c0 + lane * VEC < ce ? c0 + lane * VEC : cs; };
      stage_load(a, vr, cs, ce);
      tiles_load(cur, rowp, lane_col(cs));
      __syncthreads();                       // the previous task's readers of sv are done
      stage_store(sv, vr);
      __syncthreads();
      for (int i = 0; i < nch; ++i) {
        const int64_t c0 = cs + (int64_t)i * CW;
        const bool more = i + 1 < nch;
        if (more) {
          stage_load(a, vr, c0 + CW, ce);
          tiles_load(nxt, rowp, lane_col(c0 + CW));
        }
        const double *vb = sv + (i & 1) * (K * CW) + lane * VEC;
        const int64_t col = c0 + lane * VEC;
        double o[RB][VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const bool in = col + e < ce;
#pragma unroll
          for (int r = 0; r < RB; ++r) o[r][e] = elem(cur[r], e, in);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
          double v[VEC];
#pragma unroll
          for (int e = 0; e < VEC; ++e) v[e] = vb[k * CW + e];
#pragma unroll
          for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[r][k] += o[r][e] * v[e];
        }
        if (more) stage_store(sv + ((i + 1) & 1) * (K * CW), vr);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RB; ++r) cur[r] = nxt[r];
      }
      double flat[RB * K];
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int k = 0; k < K; ++k) flat[r * K + k] = acc[r][k];
      const double sum = multi_wave_sum<RB * K>(flat, lane);   // lanes 2i, 2i + 1: value i
      const int vi = lane >> 1, r = vi / K, k = vi % K;
      const int64_t row = r0 + r;
      double ck = 0.0;
#pragma unroll
      for (int kk = 0; kk < K; ++kk) ck = kk == k ? c[kk] : ck;
      if ((lane & 1) == 0 && row < g.n_s)
        st_coh(&a.wp[((int64_t)part * g.n_s + row) * K + k], part == 0 ? sum - ck : sum);
    }
  }

  // Pass 2 over this workgroup's tasks.
  __device__ static void col_updates(const BatchArgs &a, const BatchSys &S) {
    const BatchGeom &g = S.bg;
    double *const sw = lds();
    const int tid = (int)threadIdx.x;
    const int64_t ntask = (int64_t)g.C * g.SP;
    for (int64_t task = blockIdx.x; task < ntask; task += gridDim.x) {
      const int cb = (int)(task % g.C), sp = (int)(task / g.C);
      const int64_t rs0 = (int64_t)sp * g.rs, rs1 = min(g.n_s, rs0 + g.rs);
      const int nrow = (int)(rs1 - rs0);
      __syncthreads();                       // the previous task's readers of sw are done
      for (int idx = tid; idx < nrow * K; idx += NT) {
        const int64_t row = rs0 + idx / K;
        const int k = idx % K;
        double t = 0.0;
        for (int p = 0; p < g.P; ++p) t += ld_coh(&a.wp[((int64_t)p * g.n_s + row) * K + k]);
        sw[idx] = t;
      }
      __syncthreads();
      if (cb == 0 && tid < 64) {             // this split's sums of the centred row dots
        double ps[K];
#pragma unroll
        for (int k = 0; k < K; ++k) ps[k] = 0.0;
        for (int r = tid; r < nrow; r += 64)
#pragma unroll
          for (int k = 0; k < K; ++k) ps[k] += sw[r * K + k];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double t = wave_sum(ps[k]);
          if (tid == 0) st_coh(&a.swp[(int64_t)sp * K + k], t);
        }
      }
      const int64_t col = (int64_t)cb * BW + (int64_t)tid * VEC;
      const bool live = col < g.n_p;
      const int64_t colc = live ? col : 0;
      bool in[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) in[e] = live && col + e < g.n_p;
      const unsigned char *base = S.op.O + colc * St::BYTES;
      double y[K][VEC];
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int e = 0; e < VEC; ++e) y[k][e] = 0.0;
      u32x4 cur[kBatchU], nxt[kBatchU];
#pragma unroll
      for (int u = 0; u < kBatchU; ++u) cur[u] = load_stream(base + min(rs0 + u, rs1 - 1) * S.op.ldb);
      for (int64_t r = rs0; r < rs1; r += kBatchU) {
        const bool more = r + kBatchU < rs1;
        if (more) {
#pragma unroll
          for (int u = 0; u < kBatchU; ++u) nxt[u] = load_stream(base + min(r + kBatchU + u, rs1 - 1) * S.op.ldb);
        }
#pragma unroll
        for (int u = 0; u < kBatchU; ++u) {
          if (r + u < rs1) {
            const double *wr = sw + (r + u - rs0) * K;
            double w[K];
#pragma unroll
            for (int k = 0; k < K; ++k) w[k] = wr[k];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
              const double o = elem(cur[u], e, in[e]);
#pragma unroll
              for (int k = 0; k < K; ++k) y[k][e] += o * w[k];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kBatchU; ++u) cur[u] = nxt[u];
      }
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          if (in[e]) st_coh(&a.yp[((int64_t)sp * K + k) * g.n_p + col + e], y[k][e]);
    }
  }

  // q_k = (S + eps_k I) v_k for the K columns of vin ([K][vstride]); this workgroup writes
  // columns [j0, j1) of q and reads only those of vin.
  __device__ static bool apply(const BatchArgs &a, const BatchSys &S, GridSync &gs, int &nred, const double *vin,
                               double *q, int64_t j0, int64_t j1) {
    const BatchGeom &g = S.bg;
    const int tid = (int)threadIdx.x;
    const int64_t vs = a.vstride;
    double part[K], c[K];
#pragma unroll
    for (int k = 0; k < K; ++k) part[k] = 0.0;
    for (int64_t j = j0 + tid; j < j1; j += NT) {
      const double s = S.op.scale ? (double)S.op.scale[j] : 1.0;
      const double m = S.mean[j];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double v = ld_coh(&vin[k * vs + j]);
        st_coh(&a.vs[k * vs + j], v * s);
        part[k] += m * v;
      }
    }
    if (!grid_allreduce_n<K>(part, a.red, nred, gs, c)) return false;   // (vs visible after it)
    row_dots(a, S, c);
    if (!grid_sync(gs)) return false;
    col_updates(a, S);
    if (!grid_sync(gs)) return false;
    __shared__ double s_s1[K];
    if (tid < 64) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        double t = 0.0;
        for (int sp = tid; sp < g.SP; sp += 64) t += ld_coh(&a.swp[(int64_t)sp * K + k]);
        t = wave_sum(t);
        if (tid == 0) s_s1[k] = t;
      }
    }
    __syncthreads();
    const double inv_n = 1.0 / (double)g.n_s;
    for (int64_t j = j0 + tid; j < j1; j += NT) {
      const double s = S.op.scale ? (double)S.op.scale[j] : 1.0;
      const double m = S.mean[j];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        double acc = 0.0;
        for (int sp = 0; sp < g.SP; ++sp) acc += ld_coh(&a.yp[((int64_t)sp * K + k) * g.n_p + j]);
        st_coh(&q[k * vs + j], (s * acc - m * s_s1[k]) * inv_n + S.eps[k] * ld_coh(&vin[k * vs + j]));
      }
    }
    __syncthreads();                         // s_s1 is read before the next product writes it
    return true;
  }
};

// Batched CG: for each system in turn, K independent CG iterations (one per right-hand
// side and shift) whose products share every read of O.  A column that has converged
// stops moving (step length zero) while the others continue.  Every product is
// float64-accumulated; all residuals are recomputed from x every refresh_every iterations,
// whenever a column's recurrence residual reaches rtol (its convergence is confirmed by
// the true residual, or it continues from it) and at max_iter.  Scalars are float64 and
// the same in every workgroup (fixed-order reductions), so all take the same branches.
template <int DT, int NT>
__global__ __launch_bounds__(NT) void k_cg_batched(BatchArgs a) {
  typedef BatchProduct<DT, NT> BP;
  constexpr int K = kBatchK;
  // The vectors x, r, p, q are split over the workgroups by each system's n_p, so a
  // workgroup's share moves between systems: every access to them is coherent (a plain
  // load could hit a line another workgroup's share left in this CU's cache).
  // Per-column CG state is the same in every thread of the workgroup: it lives in LDS
  // (thread 0 writes it, a barrier publishes it) so that no register holds it across
  // the products.
  __shared__ double s_rho[K], s_gg[K], s_rel[K], s_ref[K];
  __shared__ int s_status[K], s_iters[K], s_done[K];
  GridSync gs{a.sb.flags, a.sb.abort, 0u};
  const int G = (int)gridDim.x, tid = (int)threadIdx.x;
  const int64_t vs = a.vstride;
  double *const X = a.x;
  int nred = 0;
  bool ok = true;
  for (int sidx = 0; sidx < a.n_sys && ok; ++sidx) {
    const BatchSys &S = a.sys[sidx];
    // every workgroup has finished the previous system (its results are copied out of the
    // shared vectors) before this one overwrites them
    if (sidx > 0 && !(ok = grid_sync(gs))) break;
    const int64_t n = S.bg.n_p;
    const int64_t ch = (n + G - 1) / G;
    const int64_t j0 = min(n, (int64_t)blockIdx.x * ch), j1 = min(n, j0 + ch);
    const int kuse = S.k;
    {
      // x = 0, r = p = g; columns >= k are zero and done from the start
      double part[K], gg[K];
#pragma unroll
      for (int k = 0; k < K; ++k) part[k] = 0.0;
      for (int64_t j = j0 + tid; j < j1; j += NT) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double gj = k < kuse ? S.g[k * n + j] : 0.0;
          st_coh(&X[k * vs + j], 0.0);
          st_coh(&a.r[k * vs + j], gj);
          st_coh(&a.p[k * vs + j], gj);
          part[k] += gj * gj;
        }
      }
      if (!(ok = grid_allreduce_n<K>(part, a.red, nred, gs, gg))) break;
      if (tid == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          s_rho[k] = gg[k];
          s_ref[k] = gg[k];
          s_gg[k] = gg[k] == 0.0 ? 1.0 : gg[k];
          s_status[k] = 0;
          s_iters[k] = 0;
          s_done[k] = (k >= kuse || gg[k] == 0.0) ? 1 : 0;
          s_rel[k] = s_done[k] ? 0.0 : -1.0;
        }
      }
      __syncthreads();
    }
    int it = 0, products = 0;
    bool refreshed = false;
    while (true) {
      bool any = false, check = false;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (s_done[k]) continue;
        any = true;
        check |= !isfinite(s_rho[k]) || sqrt(s_rho[k] / s_gg[k]) <= a.rtol || s_rho[k] <= a.refresh_drop2 * s_ref[k];
      }
      if (!any) break;
      const bool at_limit = it >= a.max_iter;
      const bool periodic = a.refresh_every > 0 && it > 0 && it % a.refresh_every == 0 && !refreshed;
      if (check || at_limit || periodic) {
        // true residuals of every column: r = g - (S + eps) x, float64 accumulation
        if (!(ok = grid_sync(gs))) break;                     // x visible to all
        if (!(ok = BP::apply(a, S, gs, nred, X, a.q, j0, j1))) break;
        products++;
        double part[K], red[K];
        int done_mask = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          part[k] = 0.0;
          done_mask |= s_done[k] ? (1 << k) : 0;
        }
        for (int64_t j = j0 + tid; j < j1; j += NT) {
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const double t = (k < kuse ? S.g[k * n + j] : 0.0) - ld_coh(&a.q[k * vs + j]);
            if (!((done_mask >> k) & 1)) st_coh(&a.r[k * vs + j], t);
            part[k] += t * t;
          }
        }
        if (!(ok = grid_allreduce_n<K>(part, a.red, nred, gs, red))) break;
        if (tid == 0) {
#pragma unroll
          for (int k = 0; k < K; ++k) {
            if (s_done[k]) continue;
            const double rt = sqrt(red[k] / s_gg[k]);
            if (rt <= a.rtol || at_limit || !isfinite(rt)) {
              s_rel[k] = rt;
              s_status[k] = !isfinite(rt) ? -4 : (rt <= a.rtol ? 0 : 1);
              s_done[k] = 1;
              s_iters[k] = it;
            } else {
              s_rho[k] = red[k];       // continue from the true residual
              s_ref[k] = red[k];
            }
          }
        }
        __syncthreads();
        refreshed = true;
        continue;
      }
      // search step for every column (done ones do not move)
      if (!(ok = BP::apply(a, S, gs, nred, a.p, a.q, j0, j1))) break;
      products++;
      {
        double part[K], red[K], alpha[K];
#pragma unroll
        for (int k = 0; k < K; ++k) part[k] = 0.0;
        for (int64_t j = j0 + tid; j < j1; j += NT) {
#pragma unroll
          for (int k = 0; k < K; ++k) part[k] += ld_coh(&a.p[k * vs + j]) * ld_coh(&a.q[k * vs + j]);
        }
        if (!(ok = grid_allreduce_n<K>(part, a.red, nred, gs, red))) break;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const bool live = !s_done[k] && isfinite(red[k]) && red[k] > 0.0;
          alpha[k] = live ? s_rho[k] / red[k] : 0.0;
        }
        __syncthreads();        // every thread has read s_done / s_rho before thread 0 writes
        if (tid == 0) {
#pragma unroll
          for (int k = 0; k < K; ++k) {
            if (s_done[k]) continue;
            if (!isfinite(red[k])) {
              s_status[k] = -4;
              s_done[k] = 1;
              s_iters[k] = it;
            } else if (!(red[k] > 0.0)) {
              s_status[k] = 2;           // breakdown: p . A p <= 0
              s_done[k] = 1;
              s_iters[k] = it;
            }
          }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) part[k] = 0.0;
        for (int64_t j = j0 + tid; j < j1; j += NT) {
#pragma unroll
          for (int k = 0; k < K; ++k) {
            double rj = ld_coh(&a.r[k * vs + j]);
            if (alpha[k] != 0.0) {
              st_coh(&X[k * vs + j], ld_coh(&X[k * vs + j]) + alpha[k] * ld_coh(&a.p[k * vs + j]));
              rj -= alpha[k] * ld_coh(&a.q[k * vs + j]);
              st_coh(&a.r[k * vs + j], rj);
            }
            part[k] += rj * rj;
          }
        }
        if (!(ok = grid_allreduce_n<K>(part, a.red, nred, gs, red))) break;
        // (the reduction's barriers published thread 0's writes above)
        double beta[K];
#pragma unroll
        for (int k = 0; k < K; ++k) beta[k] = (!s_done[k] && s_rho[k] > 0.0) ? red[k] / s_rho[k] : 0.0;
        __syncthreads();
        if (tid == 0) {
#pragma unroll
          for (int k = 0; k < K; ++k)
            if (!s_done[k]) s_rho[k] = red[k];
        }
        for (int64_t j = j0 + tid; j < j1; j += NT) {
#pragma unroll
          for (int k = 0; k < K; ++k)
            st_coh(&a.p[k * vs + j], ld_coh(&a.r[k * vs + j]) + beta[k] * ld_coh(&a.p[k * vs + j]));
        }
      }
      if (!(ok = grid_sync(gs))) break;                       // p visible to all (and s_rho)
      it++;
      refreshed = false;
    }
    if (!ok) break;
    // results of this system
    for (int64_t j = j0 + tid; j < j1; j += NT) {
      for (int k = 0; k < kuse; ++k) S.x[k * n + j] = ld_coh(&X[k * vs + j]);
    }
    if (blockIdx.x == 0 && tid == 0) {
      for (int k = 0; k < K; ++k) {
        double *inf = a.info + ((int64_t)sidx * K + k) * 4;
        inf[0] = (double)s_iters[k];
        inf[1] = (double)s_status[k];
        inf[2] = s_rel[k];
        inf[3] = (double)products;
      }
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && tid == 0) a.info[(int64_t)a.n_sys * K * 4] = ok ? 1.0 : 0.0;
}

// Standalone K-right-hand-side product (tests, timing): Y = (S + diag(eps)) V, V in p,
// Y in q.
template <int DT, int NT>
__global__ __launch_bounds__(NT) void k_svk(BatchArgs a) {
  const BatchSys &S = a.sys[0];
  GridSync gs{a.sb.flags, a.sb.abort, 0u};
  const int G = (int)gridDim.x;
  const int64_t n = S.bg.n_p, ch = (n + G - 1) / G;
  const int64_t j0 = min(n, (int64_t)blockIdx.x * ch), j1 = min(n, j0 + ch);
  int nred = 0;
  if (!BatchProduct<DT, NT>::apply(a, S, gs, nred, a.p, a.q, j0, j1)) {
    for (int64_t j = j0 + threadIdx.x; j < j1; j += NT)
      for (int k = 0; k < kBatchK; ++k) a.q[k * a.vstride + j] = __builtin_nan("");
  }
}

}  // namespace sr
