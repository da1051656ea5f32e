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
// NT threads per workgroup: 2-byte storage runs 512 (8 waves per CU keep enough tiles in
// flight for its short rows), 4- and 8-byte storage 256 (their accumulators need the
// registers of one wave per SIMD).
template <int DT, int NV, int RT, int NT>
__global__ __launch_bounds__(NT) void k_grad(GradArgs a) {
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
    for (int64_t k = k0 + tid; k < k1; k += NT) s += a.E[k];
    double dummy;
    if (!grid_allreduce2(s, 0.0, a.sb.red, nred, ctx.gs, Emean, dummy)) return;
    Emean *= inv_n;
    double se = 0.0;
    for (int64_t k = k0 + tid; k < k1; k += NT) se += a.E[k] - Emean;
    if (!grid_allreduce2(se, 0.0, a.sb.red, nred, ctx.gs, sum_e, dummy)) return;
  }

  // --- column sums over this row group's rows, for the owned columns ---
  int64_t colv[NV];
  double K[NV][VEC], sA[NV][VEC], sB[NV][VEC], sC[NV][VEC];
  const unsigned char *O = a.op.O;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int64_t col = ctx.c0 + ((int64_t)i * NT + tid) * VEC;
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
  // Two register buffers: the loads of the next tile are in flight while this one is
  // summed.  Loads are unconditional (rows past n_s read the last row, vectors past the
  // slice read column 0; neither is summed into a stored column), so the compiler's wait
  // for one tile leaves the other in flight.
  // the tile's energies come with it: lane l loads row l % RT with a vector load (kept in
  // order with the tile loads), broadcast per row when summed
  static_assert(RT <= 64, "one lane per tile row");
  const int lane = tid & 63;
  auto load_tile = [&](int64_t t, u32x4 (&b)[RT][NV], u32x4 (&bl)[RT][NV], double &ev) {
    {
      int64_t row = t * RT + lane % RT;
      row = row < a.pg.n_s ? row : a.pg.n_s - 1;
      ev = a.E != nullptr ? a.E[row] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      int64_t row = t * RT + r;
      row = row < a.pg.n_s ? row : a.pg.n_s - 1;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int64_t c = colv[i] >= 0 ? colv[i] : 0;
        b[r][i] = load_stream(O + row * a.op.ldb + c * St::BYTES);
        bl[r][i] = LO != nullptr ? load_stream(LO + row * a.op.ldb + c * St::BYTES) : u32x4{0u, 0u, 0u, 0u};
      }
    }
  };
  auto sum_tile = [&](int64_t t, const u32x4 (&b)[RT][NV], const u32x4 (&bl)[RT][NV], double ev) {
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const int64_t row = t * RT + r;
      if (row >= a.pg.n_s) continue;
      const double e_k = (a.E != nullptr) ? __shfl(ev, r, 64) - Emean : 0.0;
#pragma unroll
      for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const double q = (double)St::get(b[r][i], e) + (double)St::get(bl[r][i], e);
          const double x = q * sc[i][e] - K[i][e];
          sA[i][e] += x;
          sB[i][e] = fma(x, x, sB[i][e]);
          sC[i][e] = fma(e_k, x, sC[i][e]);
        }
    }
  };
  {
    u32x4 bA[RT][NV], lA[RT][NV], bB[RT][NV], lB[RT][NV];
    double eA = 0.0, eB = 0.0;
    const int64_t RG = a.pg.RG;
    int64_t t = ctx.rg;
    if (t < n_tiles) load_tile(t, bA, lA, eA);
    for (; t < n_tiles; t += 2 * RG) {
      load_tile(t + RG, bB, lB, eB);
      sum_tile(t, bA, lA, eA);
      if (t + RG >= n_tiles) break;
      load_tile(t + 2 * RG, bA, lA, eA);
      sum_tile(t + RG, bB, lB, eB);
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
  for (int64_t j = j0 + tid; j < j1; j += NT) {
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
// Compact remainder plane: column selection, codes, and the prepare pass of its columns
// ======================================================================================
template <int OUT_DT> __device__ __forceinline__ uint16_t rne_code(double t) {
  return OUT_DT == DT_BF16 ? rne_bf16(t) : rne_f16(t);
}
template <int OUT_DT> __device__ __forceinline__ double code_to_double(uint16_t c) {
  return OUT_DT == DT_BF16 ? (double)__uint_as_float((uint32_t)c << 16) : (double)(float)__builtin_bit_cast(_Float16, c);
}
template <int IN_DT> __device__ __forceinline__ double input_value(const unsigned char *rowp, int64_t col) {
  return IN_DT == DT_F64 ? ((const double *)rowp)[col] : (double)((const float *)rowp)[col];
}

// err_j = max_k |O_kj / s_j - q_kj| (the single-plane error relative to the column scale),
// a column reduction over row groups like k_absmax.
template <int IN_DT, int OUT_DT>
__global__ __launch_bounds__(kNT) void k_remmax(RemArgs a) {
  WgCtx ctx;
  init_ctx(ctx, a.pg, a.sb.flags, a.sb.abort, 1);
  const int G = (int)gridDim.x, tid = (int)threadIdx.x;
  for (int64_t col = ctx.c0 + tid; col < ctx.c1; col += kNT) {
    const double s = (double)a.scale[col];
    double m = 0.0;
    for (int64_t row = ctx.rg; row < a.pg.n_s; row += a.pg.RG) {
      const double t = input_value<IN_DT>(a.in + row * a.ldb_in, col) / s;
      m = fmax(m, fabs(t - code_to_double<OUT_DT>(rne_code<OUT_DT>(t))));
    }
    st_coh(&a.pb.ypart[(int64_t)ctx.rg * a.pg.n_p + col], m);
  }
  if (!grid_sync(ctx.gs)) return;
  const int64_t ch = (a.pg.n_p + G - 1) / G;
  const int64_t j0 = min(a.pg.n_p, (int64_t)blockIdx.x * ch), j1 = min(a.pg.n_p, j0 + ch);
  for (int64_t j = j0 + tid; j < j1; j += kNT) {
    double m = 0.0;
    for (int rg = 0; rg < a.pg.RG; ++rg) m = fmax(m, ld_coh(&a.pb.ypart[(int64_t)rg * a.pg.n_p + j]));
    a.err[j] = m;
  }
}

// Remainder codes of the selected columns: lo_ki = code(O_k,j / s_j - q_kj), j = cols[i];
// padding columns n_lo..ld_lo-1 are written as zero.
template <int IN_DT, int OUT_DT>
__global__ __launch_bounds__(kNT) void k_quantize_lo(QuantLoArgs a) {
  const int64_t nvec_row = a.ld_lo / 8;
  const int64_t total = a.n_s * nvec_row;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = idx / nvec_row, c0 = (idx % nvec_row) * 8;
    const unsigned char *rin = a.in + row * a.ldb_in;
    uint32_t w[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      uint32_t pair = 0;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int64_t c = c0 + 2 * h + e;
        uint16_t code = 0;
        if (c < a.n_lo) {
          const int64_t j = lo_param(a.cols, c, a.n_p);
          const double t = input_value<IN_DT>(rin, j) / (double)a.scale[j];
          code = rne_code<OUT_DT>(t - code_to_double<OUT_DT>(rne_code<OUT_DT>(t)));
        }
        pair |= (uint32_t)code << (16 * e);
      }
      w[h] = pair;
    }
    *(u32x4 *)(a.out + row * a.ld_lo * 2 + c0 * 2) = u32x4{w[0], w[1], w[2], w[3]};
  }
}

// Prepare pass of the remainder columns (their stored value is s_j (q_kj + lo_ki)): sums of
// x - K, (x - K)^2, e (x - K) and e over a block of rows per thread and column, with the
// shift K = the column's value in row 0 and e = E - <E>.
template <int DT>
__device__ __forceinline__ double two_plane_value(const GradLoArgs &a, int64_t k, int64_t i, int64_t j, double s) {
  return (code_value(a.Q + k * a.ldb, j, DT) + code_value(a.LO + k * a.ldb_lo, i, DT)) * s;
}

template <int DT>
__global__ __launch_bounds__(kNT) void k_gradlo_part(GradLoArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const int64_t rb = blockIdx.y;
  if (i >= a.n_lo) return;
  const int64_t j = lo_param(a.cols, i, a.n_p);
  const double s = (double)a.scale[j];
  const double K = two_plane_value<DT>(a, 0, i, j, s);
  const double Em = a.E != nullptr ? *a.Emean : 0.0;
  const int64_t k0 = rb * a.rows_per_block;
  const int64_t k1 = min(a.n_s, k0 + a.rows_per_block);
  double sA = 0.0, sB = 0.0, sC = 0.0, sE = 0.0;
  int64_t k = k0;
  for (; k + 8 <= k1; k += 8) {
    double x[8], e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x[u] = two_plane_value<DT>(a, k + u, i, j, s) - K;
      e[u] = a.E != nullptr ? a.E[k + u] - Em : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sA += x[u];
      sB = fma(x[u], x[u], sB);
      sC = fma(e[u], x[u], sC);
      sE += e[u];
    }
  }
  for (; k < k1; ++k) {
    const double x = two_plane_value<DT>(a, k, i, j, s) - K;
    const double e = a.E != nullptr ? a.E[k] - Em : 0.0;
    sA += x;
    sB = fma(x, x, sB);
    sC = fma(e, x, sC);
    sE += e;
  }
  double *p = a.part + rb * 4 * a.n_lo;
  p[i] = sA;
  p[a.n_lo + i] = sB;
  p[2 * a.n_lo + i] = sC;
  p[3 * a.n_lo + i] = sE;
}

template <int DT>
__global__ __launch_bounds__(kNT) void k_gradlo_finish(GradLoArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (i >= a.n_lo) return;
  double A = 0.0, B = 0.0, Cg = 0.0, Es = 0.0;
  for (int rb = 0; rb < a.n_rb; ++rb) {
    const double *p = a.part + (int64_t)rb * 4 * a.n_lo;
    A += p[i];
    B += p[a.n_lo + i];
    Cg += p[2 * a.n_lo + i];
    Es += p[3 * a.n_lo + i];
  }
  const int64_t j = lo_param(a.cols, i, a.n_p);
  const double inv_n = 1.0 / (double)a.n_s;
  const double K = two_plane_value<DT>(a, 0, i, j, (double)a.scale[j]);
  const double dmean = A * inv_n;
  if (a.mean_out) a.mean_out[j] = K + dmean;
  if (a.diag_out) {
    const double var = B * inv_n - dmean * dmean;
    a.diag_out[j] = var > 0.0 ? var : 0.0;
  }
  if (a.g_out) a.g_out[j] = 2.0 * inv_n * (Cg - dmean * Es);
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
  int64_t i0, i1;
  lo_range(a.op, j0, j1, i0, i1);
  finish_lo<NT>(a.pb, a.pg, a.op, i0, i1, inv_n, a.y);
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
  // q[j] of this workgroup's chunk was written by this workgroup
  __device__ __forceinline__ static double ldq(const double *p) { return *p; }
  // per-workgroup context of the product (column slice, barrier state)
  __device__ __forceinline__ static void init(WgCtx &ctx, const CgArgs &a) {
    init_ctx(ctx, a.pg, a.sb.flags, a.sb.abort, Storage<DT>::VEC);
  }
  // q[j] = ((S + eps I) vin)_j for this workgroup's vector chunk [j0, j1).  EXACT selects
  // float64 accumulation (residual products of scaled storage).  SMALL: one-row tiles, one
  // tile of lookahead and the shortest poll depth (same column geometry, fewer registers),
  // used where a kernel holds two product codes or reads two planes; a kernel with a
  // single product code keeps the tuned tile.
  template <bool EXACT, int PLANES = 1, bool SMALL = (EXACT || PLANES == 2)>
  __device__ __forceinline__ static bool apply(const CgArgs &a, WgCtx &ctx, const double *vin, double *q,
                                               int64_t j0, int64_t j1, int &products) {
    constexpr bool kSmall = SMALL;
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
    if (PLANES == 1 && a.op.lo_cols != nullptr) {
      int64_t i0, i1;
      lo_range(a.op, j0, j1, i0, i1);
      finish_lo<NT>(a.pb, a.pg, a.op, i0, i1, inv_n, q);
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
//   kCgJacobi     one plane, Jacobi-preconditioned: z = r / (diag S + eps), rho = r . z
//                 (the convergence test stays on ||r|| / ||g||)
//   kCgExact      one plane (or a compact remainder plane) of scaled storage, every product
//                 float64-accumulated
enum { kCgOnePlane = 0, kCgTwoPlanes = 1, kCgJacobi = 3, kCgExact = 4 };

template <class K, int NT, int CGM, int PH>
__device__ __forceinline__ void cg_body(CgArgs &a) {
  // Conjugate gradient (Hestenes-Stiefel) as a state machine with one product per pass
  // through the loop, so the product code is instantiated once per accumulation type.
  //   MODE_P        q = A p, then alpha, x += alpha p, r -= alpha q
  //   MODE_REFRESH  q = A x, r = g - q (every refresh_every iterations, or once the
  //                 recurrence residual fell by refresh_drop since the last refresh)
  //   MODE_CONFIRM  q = A x when the recurrence residual meets rtol; accept or replace r
  //   MODE_FINAL    q = A x to report the true residual of an unconverged exit
  //   MODE_X0       q = A x0 for a warm start
  //   MODE_INIT     (split solves) x = 0, r = p = g, first decision
  enum { MODE_P = kCgModeP, MODE_REFRESH = kCgModeRefresh, MODE_CONFIRM = kCgModeConfirm, MODE_FINAL = kCgModeFinal,
         MODE_X0 = kCgModeX0, MODE_DONE = kCgModeDone, MODE_INIT = kCgModeInit };
  constexpr bool kJac = CGM == kCgJacobi;
  static_assert(PH == kPhAll || CGM == kCgOnePlane, "split solves: one plane");
  WgCtx ctx;
  K::init(ctx, a);
  if constexpr (PH != kPhAll) {
    // resume: the barrier epochs and exchange steps continue from the previous launch
    // (every workgroup passed the same barriers and products there)
    if (ld_coh32(a.sb.abort) != 0u) return;
    ctx.gs.epoch = ld_coh32(&a.sb.flags[blockIdx.x]);
    ctx.xstep = (uint32_t)ld_coh(&a.info[kInfoXstep]);
  }
  const int G = (int)gridDim.x, tid = (int)threadIdx.x;
  const int64_t n = a.pg.n_p;
  const int64_t ch = (n + G - 1) / G;
  const int64_t j0 = min(n, (int64_t)blockIdx.x * ch), j1 = min(n, j0 + ch);
  int nred = 0, products = 0, refreshes = 0, it = 0;
  int status = 0;       // SR_OK
  double rel_true = -1.0, rho = 0.0, gg = 1.0, dummy = 0.0;
  double rho_ref = 0.0;  // rho at the start or the last refresh (drop-triggered refreshes)
  double rz = 0.0;       // r . z with z = r / (diag S + eps) (Jacobi; rho = r . r stays the test)
  double rel_best = 0.0; // smallest true relative residual seen at a refresh or exit check
  bool ok = true, restart = false;
  int mode;
  if constexpr (PH != kPhAll) {
    it = (int)ld_coh(&a.info[kInfoIters]);
    refreshes = (int)ld_coh(&a.info[kInfoRefreshes]);
    status = (int)ld_coh(&a.info[kInfoStatus]);
    products = (int)ld_coh(&a.info[kInfoProducts]);
    rel_true = ld_coh(&a.info[kInfoRelTrue]);
    mode = (int)ld_coh(&a.info[kInfoMode]);
    rho = ld_coh(&a.info[kInfoRho]);
    gg = ld_coh(&a.info[kInfoGg]);
    rho_ref = ld_coh(&a.info[kInfoRhoRef]);
    rz = ld_coh(&a.info[kInfoRz]);
    rel_best = ld_coh(&a.info[kInfoRelBest]);
    if (mode == MODE_DONE || mode == MODE_P || mode == MODE_INIT)
      return;     // nothing for the residual phase (uniform: every workgroup read the same state)
  }

  // choose the next product from the recurrence residual
  auto decide = [&]() -> int {
    const double rel = sqrt(rho / gg);
    if (a.hist != nullptr && blockIdx.x == 0 && tid == 0 && it <= a.max_iter) a.hist[it] = rel;
    if (!isfinite(rho)) { status = -4; return MODE_DONE; }
    if (rel <= a.rtol) return MODE_CONFIRM;
    if (it >= a.max_iter) { status = 1; return MODE_FINAL; }
    return MODE_P;
  };
  // preconditioned residual component (z = r without preconditioning)
  auto zof = [&](int64_t j, double rj) -> double {
    if constexpr (kJac) return rj / (a.diag[j] + a.eps);
    else return rj;
  };
  // p <- z + beta p for the own chunk, then a barrier so every workgroup sees p
  auto update_p = [&](double beta) -> bool {
    for (int64_t j = j0 + tid; j < j1; j += NT) st_coh(&a.p[j], zof(j, a.r[j]) + beta * ld_coh(&a.p[j]));
    return grid_sync(ctx.gs);
  };

  if (PH == kPhAll && a.use_x0) {
    mode = MODE_X0;
  } else if (PH == kPhAll) {
    double prr = 0.0, pgg = 0.0, prz = 0.0;
    for (int64_t j = j0 + tid; j < j1; j += NT) {
      st_coh(&a.x[j], 0.0);
      const double gj = a.g[j], zj = zof(j, gj);
      a.r[j] = gj;
      st_coh(&a.p[j], zj);
      prr += gj * gj;
      pgg += gj * gj;
      if constexpr (kJac) prz += gj * zj;
    }
    ok = grid_allreduce2(prr, pgg, a.sb.red, nred, ctx.gs, rho, gg);
    if constexpr (kJac) {
      if (ok) ok = grid_allreduce2(prz, 0.0, a.sb.red, nred, ctx.gs, rz, dummy);
    }
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
    if (PH == kPhResidual && on_p) break;      // hand over to the search phase
    if constexpr (PH == kPhResidual) {
      ok = K::template apply<true>(a, ctx, a.x, a.q, j0, j1, products);
    } else if constexpr (CGM == kCgTwoPlanes) {
      // one product code for search directions and residuals: float64 accumulation
      // (measured faster here than float32 with the two planes in one kernel)
      ok = K::template apply<true, 2>(a, ctx, on_p ? a.p : a.x, a.q, j0, j1, products);
    } else if constexpr (CGM == kCgExact) {
      // one product code, float64 accumulation (one-row tiles: the tuned float32 tile held
      // in float64 spills inside the streaming loop)
      ok = K::template apply<true>(a, ctx, on_p ? a.p : a.x, a.q, j0, j1, products);
    } else if constexpr (K::kExactResidual) {
      if (on_p) ok = K::template apply<false>(a, ctx, a.p, a.q, j0, j1, products);
      else ok = K::template apply<true>(a, ctx, a.x, a.q, j0, j1, products);
    } else {
      ok = K::template apply<false>(a, ctx, on_p ? a.p : a.x, a.q, j0, j1, products);
    }
    if (!ok) break;
    if (mode == MODE_P) {
      double ppq = 0.0, pq;
      for (int64_t j = j0 + tid; j < j1; j += NT) ppq += ld_coh(&a.p[j]) * K::ldq(&a.q[j]);
      if (!(ok = grid_allreduce2(ppq, 0.0, a.sb.red, nred, ctx.gs, pq, dummy))) break;
      if (!isfinite(pq)) {
        status = -4;
        mode = MODE_DONE;
        break;
      }
      if (!(pq > 0.0)) { status = 2; mode = MODE_FINAL; continue; }
      const double alpha = (kJac ? rz : rho) / pq;
      double prr = 0.0, prz = 0.0;
      for (int64_t j = j0 + tid; j < j1; j += NT) {
        st_coh(&a.x[j], ld_coh(&a.x[j]) + alpha * ld_coh(&a.p[j]));
        const double rj = a.r[j] - alpha * K::ldq(&a.q[j]);
        a.r[j] = rj;
        prr += rj * rj;
        if constexpr (kJac) prz += rj * zof(j, rj);
      }
      it++;
      if (a.refresh_every > 0 && it % a.refresh_every == 0) {
        if (!(ok = grid_sync(ctx.gs))) break;      // x visible to the refresh product
        mode = MODE_REFRESH;
        continue;
      }
      double rho_new, rz_new = 0.0;
      if (!(ok = grid_allreduce2(prr, kJac ? prz : 0.0, a.sb.red, nred, ctx.gs, rho_new, kJac ? rz_new : dummy)))
        break;
      if (rho_new <= a.refresh_drop2 * rho_ref && sqrt(rho_new / gg) > a.rtol) {
        // the recurrence residual fell by the requested factor: refresh now (x is
        // visible to every workgroup after the reduction's grid barrier)
        mode = MODE_REFRESH;
        continue;
      }
      const double beta = kJac ? rz_new / rz : rho_new / rho;
      rho = rho_new;
      if constexpr (kJac) rz = rz_new;
      if (!(ok = update_p(beta))) break;
      mode = decide();
    } else if (mode == MODE_REFRESH) {
      double prr = 0.0, prz = 0.0, rho_new, rz_new = 0.0;
      for (int64_t j = j0 + tid; j < j1; j += NT) {
        const double rj = a.g[j] - K::ldq(&a.q[j]);
        a.r[j] = rj;
        prr += rj * rj;
        if constexpr (kJac) prz += rj * zof(j, rj);
      }
      refreshes++;
      if (!(ok = grid_allreduce2(prr, kJac ? prz : 0.0, a.sb.red, nred, ctx.gs, rho_new, kJac ? rz_new : dummy)))
        break;
      {
        // below the accuracy float64 can attain the iteration drifts: a true residual far
        // above the best one seen ends the solve (not converged) before it grows further
        const double tr_rel = sqrt(rho_new / gg);
        if (rel_best > 0.0 && tr_rel > kCgDivergence * rel_best) {
          status = 1;
          rel_true = tr_rel;
          mode = MODE_DONE;
          continue;
        }
        rel_best = (rel_best > 0.0 && rel_best < tr_rel) ? rel_best : tr_rel;
      }
      const double beta = a.restart_on_refresh ? 0.0 : (kJac ? rz_new / rz : rho_new / rho);
      rho = rho_new;
      if constexpr (kJac) rz = rz_new;
      rho_ref = rho_new;
      if (!(ok = update_p(beta))) break;
      mode = decide();
    } else if (mode == MODE_X0) {
      double prr = 0.0, pgg = 0.0, prz = 0.0;
      for (int64_t j = j0 + tid; j < j1; j += NT) {
        const double gj = a.g[j], rj = gj - K::ldq(&a.q[j]), zj = zof(j, rj);
        a.r[j] = rj;
        st_coh(&a.p[j], zj);
        prr += rj * rj;
        pgg += gj * gj;
        if constexpr (kJac) prz += rj * zj;
      }
      if (!(ok = grid_allreduce2(prr, pgg, a.sb.red, nred, ctx.gs, rho, gg))) break;
      if constexpr (kJac) {
        if (!(ok = grid_allreduce2(prz, 0.0, a.sb.red, nred, ctx.gs, rz, dummy))) break;
      }
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
      double prr = 0.0, prz = 0.0, tr, trz = 0.0;
      for (int64_t j = j0 + tid; j < j1; j += NT) {
        const double t = a.g[j] - K::ldq(&a.q[j]);
        if (mode == MODE_CONFIRM) a.r[j] = t;
        prr += t * t;
        if constexpr (kJac) prz += t * zof(j, t);
      }
      if (!(ok = grid_allreduce2(prr, kJac ? prz : 0.0, a.sb.red, nred, ctx.gs, tr, kJac ? trz : dummy))) break;
      rel_true = sqrt(tr / gg);
      if (mode == MODE_FINAL || rel_true <= a.rtol) {
        mode = MODE_DONE;
      } else if (it >= a.max_iter || (rel_best > 0.0 && rel_true > kCgDivergence * rel_best)) {
        status = 1;
        mode = MODE_DONE;
      } else {
        // the recurrence residual drifted from the true one: continue from the true one
        rho = tr;
        rho_ref = tr;
        if constexpr (kJac) rz = trz;
        rel_best = (rel_best > 0.0 && rel_best < rel_true) ? rel_best : rel_true;
        refreshes++;
        rel_true = -1.0;
        if (a.restart_on_refresh && !(ok = update_p(0.0))) break;
        mode = MODE_P;
      }
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    a.info[kInfoIters] = (double)it;
    a.info[kInfoRefreshes] = (double)refreshes;
    a.info[kInfoStatus] = (double)(ok ? status : -6);   // SR_ERR_TIMEOUT when a wait gave up
    a.info[kInfoProducts] = (double)products;
    a.info[kInfoRelRecur] = sqrt(rho / gg);
    a.info[kInfoRelTrue] = rel_true;
    a.info[kInfoOk] = ok ? 1.0 : 0.0;
    a.info[kInfoMode] = (double)(ok ? mode : MODE_DONE);
    a.info[kInfoRho] = rho;
    a.info[kInfoGg] = gg;
    a.info[kInfoRhoRef] = rho_ref;
    a.info[kInfoRz] = rz;
    a.info[kInfoXstep] = (double)ctx.xstep;
    a.info[kInfoRelBest] = rel_best;
  }
}

// One search-direction iteration of a split CG solve (one stored plane, the storage type's
// own accumulation: float32 for bf16/f16 codes, float64 for float64/float32 storage):
// q = (S + eps I) p, alpha, x += alpha p, r -= alpha q, rho, beta, p = r + beta p and the
// next decision, with the state read from CgArgs::info after the product and written back
// at the end, so nothing but the product is live during its streaming loop.  INIT: the
// solve's first launch instead, x = 0, r = p = g and the first decision (or the hand-over
// of a warm start to the residual phase).  A launch in any other state returns at once.
template <class K, int NT, bool INIT>
__device__ __forceinline__ void cg_step_body(CgArgs &a) {
  WgCtx ctx;
  K::init(ctx, a);
  if (ld_coh32(a.sb.abort) != 0u) return;
  const int mode0 = (int)ld_coh(&a.info[kInfoMode]);
  if (mode0 != (INIT ? kCgModeInit : kCgModeP)) return;
  ctx.gs.epoch = ld_coh32(&a.sb.flags[blockIdx.x]);
  ctx.xstep = (uint32_t)ld_coh(&a.info[kInfoXstep]);
  const int G = (int)gridDim.x, tid = (int)threadIdx.x;
  const int64_t n = a.pg.n_p;
  const int64_t ch = (n + G - 1) / G;
  const int64_t j0 = min(n, (int64_t)blockIdx.x * ch), j1 = min(n, j0 + ch);
  int nred = 0;
  double dummy;
  auto save = [&](int mode, bool ok, int it, int products, int status, double rho, double gg, double rho_ref) {
    if (blockIdx.x == 0 && tid == 0) {
      a.info[kInfoIters] = (double)it;
      a.info[kInfoStatus] = (double)(ok ? status : -6);   // SR_ERR_TIMEOUT when a wait gave up
      a.info[kInfoProducts] = (double)products;
      a.info[kInfoRelRecur] = sqrt(rho / gg);
      a.info[kInfoOk] = ok ? 1.0 : 0.0;
      a.info[kInfoMode] = (double)(ok ? mode : kCgModeDone);
      a.info[kInfoRho] = rho;
      a.info[kInfoGg] = gg;
      a.info[kInfoRhoRef] = rho_ref;
      a.info[kInfoXstep] = (double)ctx.xstep;
    }
  };
  auto decide = [&](int it, double rho, double gg, int &status) -> int {
    const double rel = sqrt(rho / gg);
    if (a.hist != nullptr && blockIdx.x == 0 && tid == 0 && it <= a.max_iter) a.hist[it] = rel;
    if (!isfinite(rho)) { status = -4; return kCgModeDone; }
    if (rel <= a.rtol) return kCgModeConfirm;
    if (it >= a.max_iter) { status = 1; return kCgModeFinal; }
    return kCgModeP;
  };

  if constexpr (INIT) {
    if (a.use_x0) {                 // the warm start's product runs in the residual phase
      save(kCgModeX0, true, 0, 0, 0, 0.0, 1.0, 0.0);
      if (blockIdx.x == 0 && tid == 0) a.info[kInfoRelTrue] = -1.0;
      return;
    }
    double prr = 0.0;
    for (int64_t j = j0 + tid; j < j1; j += NT) {
      st_coh(&a.x[j], 0.0);
      const double gj = a.g[j];
      a.r[j] = gj;
      st_coh(&a.p[j], gj);
      prr += gj * gj;
    }
    double rho, gg;
    const bool ok = grid_allreduce2(prr, prr, a.sb.red, nred, ctx.gs, rho, gg);
    int status = 0, mode;
    if (blockIdx.x == 0 && tid == 0) a.info[kInfoRelTrue] = -1.0;
    if (gg == 0.0) {
      gg = 1.0;
      mode = kCgModeDone;
      if (blockIdx.x == 0 && tid == 0) a.info[kInfoRelTrue] = 0.0;
    } else {
      mode = decide(0, rho, gg, status);
    }
    save(mode, ok, 0, 0, status, rho, gg, rho);
    return;
  } else {

  int dummy_products = 0;
  bool ok = K::template apply<false>(a, ctx, a.p, a.q, j0, j1, dummy_products);
  // the state, read after the product
  int it = (int)ld_coh(&a.info[kInfoIters]);
  int products = (int)ld_coh(&a.info[kInfoProducts]) + 1;
  int status = (int)ld_coh(&a.info[kInfoStatus]);
  double rho = ld_coh(&a.info[kInfoRho]);
  const double gg = ld_coh(&a.info[kInfoGg]);
  const double rho_ref = ld_coh(&a.info[kInfoRhoRef]);
  int mode = kCgModeP;
  if (!ok) {
    save(kCgModeDone, false, it, products, status, rho, gg, rho_ref);
    return;
  }
  double ppq = 0.0, pq;
  for (int64_t j = j0 + tid; j < j1; j += NT) ppq += ld_coh(&a.p[j]) * K::ldq(&a.q[j]);
  ok = grid_allreduce2(ppq, 0.0, a.sb.red, nred, ctx.gs, pq, dummy);
  if (ok && !isfinite(pq)) {
    status = -4;
    mode = kCgModeDone;
  } else if (ok && !(pq > 0.0)) {
    status = 2;
    mode = kCgModeFinal;
  } else if (ok) {
    const double alpha = rho / pq;
    double prr = 0.0;
    for (int64_t j = j0 + tid; j < j1; j += NT) {
      st_coh(&a.x[j], ld_coh(&a.x[j]) + alpha * ld_coh(&a.p[j]));
      const double rj = a.r[j] - alpha * K::ldq(&a.q[j]);
      a.r[j] = rj;
      prr += rj * rj;
    }
    it++;
    if (a.refresh_every > 0 && it % a.refresh_every == 0) {
      mode = kCgModeRefresh;        // x is visible to the next launch
    } else {
      double rho_new;
      ok = grid_allreduce2(prr, 0.0, a.sb.red, nred, ctx.gs, rho_new, dummy);
      if (ok && rho_new <= a.refresh_drop2 * rho_ref && sqrt(rho_new / gg) > a.rtol) {
        mode = kCgModeRefresh;
      } else if (ok) {
        const double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t j = j0 + tid; j < j1; j += NT) st_coh(&a.p[j], a.r[j] + beta * ld_coh(&a.p[j]));
        mode = decide(it, rho, gg, status);
      }
    }
  }
  save(mode, ok, it, products, status, rho, gg, rho_ref);
  }
}

template <int DT, int NV, int R, int L, int P_, int NT, int CGM = kCgOnePlane, int PH = kPhAll>
__global__ __launch_bounds__(NT) void k_cg(CgArgs a) {
  cg_body<CgKernel<DT, NV, R, L, P_, NT>, NT, CGM, PH>(a);
}
template <int DT, int NV, int R, int L, int P_, int NT>
__global__ __launch_bounds__(NT) void k_cg_step(CgArgs a) {
  cg_step_body<CgKernel<DT, NV, R, L, P_, NT>, NT, false>(a);
}
template <int DT, int NV, int R, int L, int P_, int NT>
__global__ __launch_bounds__(NT) void k_cg_init(CgArgs a) {
  cg_step_body<CgKernel<DT, NV, R, L, P_, NT>, NT, true>(a);
}

}  // namespace sr
