// Products and solves over index-coded correlator-product-state (CPS) storage.
//
// In a CPS ansatz every sample occupies exactly one state of each correlator (Sec. II.C,
// Eq. ansatz), so the derivative ratio of correlator p's parameter C_{p,s} is
// delta(s, s_kp) / C_{p,s}: one nonzero per correlator per row, whose value depends only on
// the column.  The storage keeps the state s_kp (one byte, correlator-major), the value of
// each correlator column, and the remaining parameters (the pairing block, Sec. III.A) as
// a dense block in any storage type.  Columns are ordered [correlator 0's n_states states |
// correlator 1 | ... | dense block].
//
// The product y = (S + eps I) v (Sec. II.A, Eq. sr_multiply_2) runs in one cooperative
// launch with three grid barriers:
//   A. partial row sums over groups of correlators: a workgroup stages its group's table
//      u_j = val_j v_j in LDS and gathers u[p, s_kp] for a range of rows; its share of
//      c = obar_D . v_D over the dense columns is reduced at the barrier;
//   1. row pass over row tiles of 128 rows (fewer when there are few samples, so that
//      every workgroup has one): w_k = (sum of the groups' partials) +
//      D_k . (s v)_D - c (the dense rows read once into registers), then the dense
//      partial sums P_d += D_kd w_k from the same registers;
//   2. per correlator, the histogram T_{p,s} = sum_{k: s_kp = s} (w_k - wbar) in int64
//      fixed point (integer sums do not depend on their order, so the product is the
//      same bit for bit on every run), y = val T / n_s + eps v; the dense columns sum the
//      workgroups' partials in a fixed order, y = (s P - obar_D sum w) / n_s + eps v.
// Centring: sum_k (O_kj - obar_j) w_k = sum_k O_kj (w_k - wbar) for any w, so the
// correlator columns need no column means; the dense columns keep the folded form.
//
// Data one workgroup writes and others read inside the launch (the partial row sums, w,
// P, y, and the vectors the CG updates) is written and read with device-scope accesses
// (an agent-scope acquire fence, which invalidates the XCD's L2, measured about 20 us on
// every workgroup: far more than these few values cost to read through).
#pragma once
#include <type_traits>

#include "sr_kernels.hpp"

namespace sr {

__device__ __forceinline__ void st_acc(double *p, double v) { st_coh(p, v); }
__device__ __forceinline__ void st_acc(float *p, float v) { st_coh32((uint32_t *)p, __float_as_uint(v)); }
__device__ __forceinline__ double ld_acc(const double *p) { return ld_coh(p); }
__device__ __forceinline__ float ld_acc(const float *p) { return __uint_as_float(ld_coh32((const uint32_t *)p)); }

// Fixed-point scale of a histogram of values whose absolute sum is at most A: every bin
// sum, and every partial sum on the way, stays below 2^62 in magnitude.
__device__ __forceinline__ double fixed_scale(double A) {
  if (!(A > 0.0) || !isfinite(A)) return 1.0;
  int e;
  (void)frexp(A, &e);                 // A < 2^e
  return ldexp(1.0, 62 - e);
}

// DDT: storage type of the dense block.  NVT: 16-byte vectors of a dense row per thread
// (n_d <= NVT * NT * VEC).  X: float64 accumulation for every product (search_f64).
template <int DDT, int NVT, bool X, int NT = 512>
struct CpsKernel {
  static_assert(NT == 512, "the row pass maps 64 lanes x 2 rows to a 128-row tile and 8 waves to correlator parts");
  static constexpr int VEC = Storage<DDT>::VEC;
  // rows per batch (RB rows x NVT vectors in registers); a second buffer to load the next
  // batch while this one is reduced measured no faster (the row pass is bound by the
  // decode and FMA work of the dot and the update, about 4.3 TB/s here, not by latency)
  static constexpr int RB = NVT >= 12 ? 1 : (NVT >= 8 ? 2 : (NVT >= 3 ? 4 : 8));
  static constexpr int NWAVE = NT / 64;
  static constexpr int kSlices = NT / kCpsTileRows;   // thread slices summing the group partials
  static constexpr int kPass = 8;               // correlators per histogram pass
  static constexpr bool kExactResidual = (DDT == DT_BF16 || DDT == DT_F16);

  // q was written by other workgroups in this launch
  __device__ __forceinline__ static double ldq(const double *p) { return ld_coh(p); }

  __device__ __forceinline__ static void init(WgCtx &ctx, const CgArgs &a) {
    ctx.rg = (int)blockIdx.x;
    ctx.cg = 0;
    ctx.c0 = ctx.c1 = 0;
    ctx.xstep = 0;
    ctx.gs.flags = a.sb.flags;
    ctx.gs.abort = a.sb.abort;
    ctx.gs.epoch = 0;
  }

  // q = (S + eps I) vin over the whole vector (j0, j1 unused: every workgroup finishes its
  // own columns and a closing barrier publishes q).  Returns false if the launch aborted.
  template <bool EXACT, int PLANES = 1, bool SMALL = false>
  __device__ static bool apply(const CgArgs &a, WgCtx &ctx, const double *vin, double *q, int64_t j0,
                               int64_t j1, int &products) {
    static_assert(PLANES == 1, "one dense plane");
    (void)j0;
    (void)j1;
    (void)SMALL;
    typedef typename std::conditional<(EXACT || X), double, typename Storage<DDT>::acc_t>::type acc_t;
    const CpsOp &c = a.cps;
    const int G = (int)gridDim.x, b = (int)blockIdx.x, tid = (int)threadIdx.x;
    const int64_t n_s = a.pg.n_s, n_sp = c.n_sp, n_d = c.n_d;
    const int ns = c.n_states;
      acc_t *part = (acc_t *)c.part;
    int nred = 0;
    double dummy;

    // ---- A. correlator partial row sums ----
    // Work item (group g, row range rr): correlators [g cpg, (g+1) cpg) and rows
    // [rr rpr, (rr+1) rpr).  The group's table u = val * v goes to LDS; lanes take pairs of
    // rows (one 2-byte state load per correlator), waves share the group's correlators, and
    // the waves' sums of each row are combined in a fixed order into part_sp[g][k].
    {
      __shared__ acc_t s_u[kCpsTableBytes / sizeof(acc_t)];
      const int wave = tid >> 6, lane = tid & 63;
      acc_t *part_sp = (acc_t *)c.part_sp;
      for (int it = b; it < c.n_items; it += G) {
        const int g = it % c.n_grp, rr = it / c.n_grp;
        const int64_t p0 = min(c.n_corr, (int64_t)g * c.cpg), p1 = min(c.n_corr, p0 + c.cpg);
        const int np_ = (int)(p1 - p0);
        __syncthreads();                 // s_u of the previous item is no longer read
        for (int e = tid; e < np_ * ns; e += NT) {
          const int64_t j = p0 * ns + e;
          s_u[e] = (acc_t)(c.val[j] * ld_coh(&vin[j]));
        }
        __syncthreads();
        // each wave takes whole blocks of 128 rows (a pair per lane, one 2-byte state load per
        // correlator) through all the group's correlators, so no two waves share a row and
        // no barrier is needed (16 rows per lane with 16-byte loads measured slower)
        const int64_t r0 = min(n_s, (int64_t)rr * c.rpr), r1 = min(n_s, r0 + c.rpr);
        for (int64_t kb = r0 + (int64_t)wave * kCpsTileRows; kb < r1; kb += (int64_t)NWAVE * kCpsTileRows) {
          const int64_t kp = kb + 2 * lane;
          acc_t s0 = (acc_t)0, s1 = (acc_t)0;
          if (kp < r1) {
            const unsigned char *ip = c.idx + p0 * c.ld_idx + kp;
            const int64_t sti = c.ld_idx;
            int i = 0;
            for (; i + 7 < np_; i += 8) {
              uint32_t pr[8];
#pragma unroll
              for (int d = 0; d < 8; ++d) pr[d] = *(const uint16_t *)(ip + d * sti);
#pragma unroll
              for (int d = 0; d < 8; ++d) {
                const unsigned sa = pr[d] & 0xFFu, sb = pr[d] >> 8;
                const acc_t *ut = s_u + (i + d) * ns;
                if (sa < (unsigned)ns) s0 += ut[sa];
                if (sb < (unsigned)ns) s1 += ut[sb];
              }
              ip += 8 * sti;
            }
            for (; i < np_; ++i) {
              const unsigned pr = *(const uint16_t *)ip;
              const unsigned sa = pr & 0xFFu, sb = pr >> 8;
              const acc_t *ut = s_u + i * ns;
              if (sa < (unsigned)ns) s0 += ut[sa];
              if (sb < (unsigned)ns) s1 += ut[sb];
              ip += sti;
            }
            st_acc(&part_sp[(int64_t)g * n_s + kp], s0);
            if (kp + 1 < r1) st_acc(&part_sp[(int64_t)g * n_s + kp + 1], s1);
          }
        }
      }
      // the dense block's centring share c = obar_D . v_D, reduced at the barrier
      const int64_t cd = (n_d + G - 1) / G;
      const int64_t d0 = min(n_d, (int64_t)b * cd), d1 = min(n_d, d0 + cd);
      double pc = 0.0;
      for (int64_t d = d0 + tid; d < d1; d += NT) pc += a.mean[n_sp + d] * ld_coh(&vin[n_sp + d]);
      double cD;
      if (!grid_allreduce2(pc, 0.0, c.red, nred, ctx.gs, cD, dummy)) return false;

      // ---- 1. row pass ----
      const int64_t nvec = (n_d + VEC - 1) / VEC;
      acc_t vs[NVT][VEC], P[NVT][VEC];
#pragma unroll
      for (int m = 0; m < NVT; ++m) {
        const int64_t vi = tid + (int64_t)m * NT;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const int64_t col = vi * VEC + e;
          double sv = 0.0;
          if (vi < nvec && col < n_d) sv = (c.dscale ? (double)c.dscale[col] : 1.0) * ld_coh(&vin[n_sp + col]);
          vs[m][e] = (acc_t)sv;
          P[m][e] = (acc_t)0;
        }
      }
      // the correlator part of the tile's row sums: tile_rows rows x (NT / tile_rows) slices
      __shared__ acc_t s_sp[kSlices][kCpsTileRows];
      acc_t *s_spf = &s_sp[0][0];
      const int tr = c.tile_rows, nsl = NT / tr;
      __shared__ double s_red[2][NWAVE][RB];
      double wsum = 0.0, wabs = 0.0;
      int par = 0;
      // one batch of RB dense rows into registers (rows past n_s and vectors past the row
      // load nothing)
      auto load_batch = [&](u32x4 (&D)[RB][NVT], int64_t k0b) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const int64_t k = k0b + r;
          const unsigned char *rowp = c.dO + k * c.ldb_d;
#pragma unroll
          for (int m = 0; m < NVT; ++m) {
            const int64_t vi = tid + (int64_t)m * NT;
            if (k < n_s && vi < nvec) D[r][m] = load_stream(rowp + vi * 16);
            else D[r][m] = u32x4{0u, 0u, 0u, 0u};
          }
        }
      };
      // row dots of a batch, their workgroup sums, w_k, then P += D w from the same registers
      auto process = [&](u32x4 (&D)[RB][NVT], int64_t k0, int rb) __attribute__((always_inline)) {
        acc_t pd[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          acc_t acc = (acc_t)0;
#pragma unroll
          for (int m = 0; m < NVT; ++m)
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc += (acc_t)Storage<DDT>::get(D[r][m], e) * vs[m][e];
          pd[r] = wave_sum(acc);
        }
        if (lane == 0) {
#pragma unroll
          for (int r = 0; r < RB; ++r) s_red[par][wave][r] = (double)pd[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const int64_t k = k0 + rb + r;
          double wr = 0.0;
          if (k < n_s) {
            for (int wv = 0; wv < NWAVE; ++wv) wr += s_red[par][wv][r];
            for (int pi = 0; pi < nsl; ++pi) wr += (double)s_spf[pi * tr + rb + r];
            wr -= cD;
          }
          if (tid == r && k < n_s) st_coh(&c.w[k], wr);
          if (tid == 0) {
            wsum += wr;
            wabs += fabs(wr);
          }
          const acc_t wa = (acc_t)wr;
#pragma unroll
          for (int m = 0; m < NVT; ++m) {
            // decode again from the packed vector (keeping the decoded values of the
            // whole batch live between the dot and this update costs registers)
            asm volatile("" : "+v"(D[r][m]));
#pragma unroll
            for (int e = 0; e < VEC; ++e) P[m][e] += (acc_t)Storage<DDT>::get(D[r][m], e) * wa;
          }
        }
        par ^= 1;   // the next batch writes the other half of s_red; a barrier separates
                    // this batch's reads from the writes two batches on
      };
      for (int t = b; t < c.tiles; t += G) {
        const int64_t k0 = (int64_t)t * tr;
        // 1a. correlator part of w for the tile's rows: the groups' partial sums, each of the
        //     nsl slices of threads summing a fixed subset of the groups
        {
          const int row = tid & (tr - 1), sl = tid / tr;
          const int64_t k = k0 + row;
          acc_t t = (acc_t)0;
          if (k < n_s) {
            const acc_t *part_sp = (const acc_t *)c.part_sp;
            for (int g = sl; g < c.n_grp; g += nsl) t += ld_acc(&part_sp[(int64_t)g * n_s + k]);
          }
          s_spf[sl * tr + row] = t;
        }
        __syncthreads();
        // 1b. dense part in batches of RB rows
        for (int rb = 0; rb < tr; rb += RB) {
          u32x4 D[RB][NVT];
          load_batch(D, k0 + rb);
          process(D, k0, rb);
        }
        __syncthreads();   // s_sp is rewritten by the next tile
      }
      // dense partial sums of this workgroup (zeros when it had no tile)
#pragma unroll
      for (int m = 0; m < NVT; ++m) {
        const int64_t vi = tid + (int64_t)m * NT;
        if (vi < nvec) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) st_acc(&part[(int64_t)b * c.n_dp + vi * VEC + e], P[m][e]);
        }
      }
      double Sw, Sa;
      if (!grid_allreduce2(tid == 0 ? wsum : 0.0, tid == 0 ? wabs : 0.0, c.red, nred, ctx.gs, Sw, Sa)) return false;

      // ---- 2. correlator histograms and dense finish ----
      const double inv_n = 1.0 / (double)n_s;
      // the uncentred product (raw) sums w_k itself; otherwise w_k - wbar, whose absolute
      // sum is at most sum |w_k| + n_s |wbar|
      const double wbar = c.raw ? 0.0 : Sw * inv_n;
      const double sigma = fixed_scale(c.raw ? Sa : Sa + fabs(Sw));
      const double inv_sigma = 1.0 / sigma;
      __shared__ long long s_bin[kPass][256];
      for (int64_t p0 = b; p0 < c.n_corr; p0 += (int64_t)G * kPass) {
        int np = 0;
        for (int e = 0; e < kPass; ++e)
          if (p0 + (int64_t)e * G < c.n_corr) np = e + 1;
        for (int i = tid; i < kPass * 256; i += NT) (&s_bin[0][0])[i] = 0;
        __syncthreads();
        for (int64_t k4 = (int64_t)tid * 4; k4 < n_s; k4 += (int64_t)NT * 4) {
          long long qv[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) qv[e] = (k4 + e < n_s) ? __double2ll_rn((ld_coh(&c.w[k4 + e]) - wbar) * sigma) : 0ll;
          for (int e = 0; e < np; ++e) {
            const uint32_t word = *(const uint32_t *)(c.idx + (p0 + (int64_t)e * G) * c.ld_idx + k4);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const unsigned s_ = (word >> (8 * r)) & 0xFFu;
              if (k4 + r < n_s && s_ < (unsigned)ns) atomicAdd((unsigned long long *)&s_bin[e][s_], (unsigned long long)qv[r]);
            }
          }
        }
        __syncthreads();
        for (int e = 0; e < np; ++e) {
          const int64_t p = p0 + (int64_t)e * G;
          for (int s_ = tid; s_ < ns; s_ += NT) {
            const int64_t j = p * ns + s_;
            const double T = (double)s_bin[e][s_] * inv_sigma;
            st_coh(&q[j], c.val[j] * T * inv_n + a.eps * ld_coh(&vin[j]));
          }
        }
        __syncthreads();
      }
      // dense columns: workgroup b finishes columns [b*cd, ...) (64 per block), each wave
      // summing a fixed range of the workgroups' partials, combined in wave order
      {
        __shared__ double s_col[NWAVE][64];
        const int gpw = (G + NWAVE - 1) / NWAVE;
        for (int64_t cb = d0; cb < d1; cb += 64) {
          const int64_t d = cb + lane;
          double acc = 0.0;
          if (d < d1) {
            const int g0 = wave * gpw, g1 = min(G, g0 + gpw);
            for (int g = g0; g < g1; ++g) acc += (double)ld_acc(&part[(int64_t)g * c.n_dp + d]);
          }
          s_col[wave][lane] = acc;
          __syncthreads();
          if (wave == 0 && d < d1) {
            double tot = 0.0;
            for (int wv = 0; wv < NWAVE; ++wv) tot += s_col[wv][lane];
            const double sc = c.dscale ? (double)c.dscale[d] : 1.0;
            const int64_t j = n_sp + d;
            st_coh(&q[j], (sc * tot - a.mean[j] * Sw) * inv_n + a.eps * ld_coh(&vin[j]));
          }
          __syncthreads();
        }
      }
    }
    if (!grid_sync(ctx.gs)) return false;
    products++;
    return true;
  }
};

// Standalone product: y = (S + eps I) v with the CG argument block (p = v, q = y).
template <int DDT, int NVT>
__global__ __launch_bounds__(512) void k_cps_sv(CgArgs a) {
  typedef CpsKernel<DDT, NVT, false> K;
  WgCtx ctx;
  K::init(ctx, a);
  int products = 0;
  K::template apply<false>(a, ctx, a.p, a.q, 0, 0, products);
}

// Split CG over CPS storage: first launch, one search iteration per launch (X: float64
// accumulation of the search products), and the residual phase.
template <int DDT, int NVT>
__global__ __launch_bounds__(512) void k_cps_cg_init(CgArgs a) {
  cg_step_body<CpsKernel<DDT, NVT, false>, 512, true>(a);
}
template <int DDT, int NVT, bool X>
__global__ __launch_bounds__(512) void k_cps_cg_step(CgArgs a) {
  cg_step_body<CpsKernel<DDT, NVT, X>, 512, false>(a);
}
template <int DDT, int NVT>
__global__ __launch_bounds__(512) void k_cps_cg_resid(CgArgs a) {
  cg_body<CpsKernel<DDT, NVT, false>, 512, kCgOnePlane, kPhResidual>(a);
}

}  // namespace sr
