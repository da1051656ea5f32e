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
  // rows per batch (RB rows x NVT vectors in registers)
  static constexpr int RB = NVT >= 12 ? 1 : (NVT >= 8 ? 2 : (NVT >= 3 ? 4 : 8));
  // a second batch buffer (the next batch's loads in flight while this batch is reduced)
  // where the registers have room for it: float32-accumulated 2-byte storage with at most
  // 12 vectors per batch (larger batches, or float64 accumulation, spill)
  static constexpr bool kTwoBuf = !X && (DDT == DT_BF16 || DDT == DT_F16) && RB * NVT <= 12;
  static constexpr int NWAVE = NT / 64;
  static constexpr int kSlices = NT / kCpsTileRows;   // thread slices summing the group partials
  static constexpr int kPass = 8;               // correlators per histogram pass
  static constexpr int kRowsA = 256;            // rows of one wave's block in the correlator phase
  static constexpr int kBatchA = 16;            // correlators whose state words load together there
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
    // [rr rpr, (rr+1) rpr).  The group's table u = val * v goes to LDS; each wave takes
    // whole blocks of 256 rows (four per lane, one 4-byte state load per correlator) through
    // all the group's correlators, so no two waves share a row and no barrier is needed.
    // A row's sum runs over the group's correlators in order into part_sp[g][k].
    {
      // the group's table, then one zero entry (states outside a correlator read it)
      constexpr int kZeroSlot = kCpsTableBytes / sizeof(acc_t);
      __shared__ acc_t s_u[kZeroSlot + 1];
      if (tid == 0) s_u[kZeroSlot] = (acc_t)0;   // the fill below never writes it
      const int wave = tid >> 6, lane = tid & 63;
      acc_t *part_sp = (acc_t *)c.part_sp;
      for (int it = b; it < c.n_items; it += G) {
        const int g = it % c.n_grp, rr = it / c.n_grp;
        const int64_t p0 = min(c.n_corr, (int64_t)g * c.cpg), p1 = min(c.n_corr, p0 + c.cpg);
        const int np_ = (int)(p1 - p0);
        __syncthreads();                 // s_u of the previous item is no longer read
        // four entries per thread load together
        const int ne = np_ * ns;
        for (int e0 = tid; e0 < ne; e0 += 4 * NT) {
          double tv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * NT;
            tv[u] = e < ne ? c.val[p0 * ns + e] * ld_coh(&vin[p0 * ns + e]) : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (e0 + u * NT < ne) s_u[e0 + u * NT] = (acc_t)tv[u];
        }
        __syncthreads();
        // The (block, batch of kBatchA correlators) pairs of this wave form one stream; the
        // state words of the next pair load while the current pair's table entries are
        // summed.  Rows k0 .. k0+3 of a lane lie below ld_idx (a multiple of 16, >= n_s)
        // whenever k0 < n_s, so the 4-byte loads stay inside the row.
        const int64_t r0 = min(n_s, (int64_t)rr * c.rpr), r1 = min(n_s, r0 + c.rpr);
        const int64_t sti = c.ld_idx;
        const int64_t kfirst = r0 + (int64_t)wave * kRowsA, wstride = (int64_t)NWAVE * kRowsA;
        const int nbat = (np_ + kBatchA - 1) / kBatchA;
        const int nblk = kfirst < r1 ? (int)((r1 - kfirst + wstride - 1) / wstride) : 0;
        const int total = nblk * nbat;
        const unsigned char *ib = c.idx + p0 * sti;
        if (np_ == 0) {                  // no correlators in the group: zero row sums
          for (int64_t kb = kfirst; kb < r1; kb += wstride) {
            const int64_t kp = kb + 4 * lane;
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (kp + r < r1) st_acc(&part_sp[(int64_t)g * n_s + kp + r], (acc_t)0);
          }
          continue;
        }
        // No branch around a load or a table read (a branch makes the compiler wait for
        // every outstanding access at the join): lanes past the range read its last four
        // rows (kmax <= r1 - 1 < ld_idx - 3), batches past the group's correlators read its
        // last one, and states outside the correlator (s >= n_states) read the table's
        // zero entry (no select after the read, so the reads of a batch issue together).
        const int64_t kmax = (r1 - 1) & ~(int64_t)3;
        auto fetch = [&](uint32_t (&dst)[kBatchA], int blk, int bt) __attribute__((always_inline)) {
          const int64_t kp = min(kfirst + (int64_t)blk * wstride + 4 * lane, kmax);
          const int i0 = bt * kBatchA;
#pragma unroll
          for (int d = 0; d < kBatchA; ++d) dst[d] = *(const uint32_t *)(ib + (int64_t)min(i0 + d, np_ - 1) * sti + kp);
        };
        auto add_entry = [&](acc_t (&s4)[4], uint32_t word, int base) __attribute__((always_inline)) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const unsigned st = (word >> (8 * r)) & 0xFFu;
            s4[r] += s_u[st < (unsigned)ns ? base + (int)st : kZeroSlot];
          }
        };
        uint32_t cur[kBatchA], nxt[kBatchA];
        fetch(cur, 0, 0);
        acc_t s4[4] = {(acc_t)0, (acc_t)0, (acc_t)0, (acc_t)0};
        int blk = 0, bt = 0;
        for (int t = 0; t < total; ++t) {
          int nb = blk, nt = bt + 1;
          if (nt == nbat) {
            nt = 0;
            ++nb;
          }
          fetch(nxt, nb, nt);            // past the wave's last block: clamped, unused
          const int i0 = bt * kBatchA;
          if (i0 + kBatchA <= np_) {     // a full batch: straight-line table reads
#pragma unroll
            for (int d = 0; d < kBatchA; ++d) add_entry(s4, cur[d], (i0 + d) * ns);
          } else {
#pragma unroll
            for (int d = 0; d < kBatchA; ++d)
              if (i0 + d < np_) add_entry(s4, cur[d], (i0 + d) * ns);
          }
          if (nt == 0) {                 // the block's last batch: its rows' sums are complete
            const int64_t kp = kfirst + (int64_t)blk * wstride + 4 * lane;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              if (kp + r < r1) st_acc(&part_sp[(int64_t)g * n_s + kp + r], s4[r]);
              s4[r] = (acc_t)0;
            }
          }
          blk = nb;
          bt = nt;
#pragma unroll
          for (int d = 0; d < kBatchA; ++d) cur[d] = nxt[d];
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
      {
        // (s v) of the thread's columns with no branch around a load (columns past the
        // block read its last column and are zeroed), so the loads issue together
        const int64_t dmax = n_d > 0 ? n_d - 1 : 0;
        auto coef = [&](bool scaled) __attribute__((always_inline)) {
#pragma unroll
          for (int m = 0; m < NVT; ++m) {
            const int64_t vi = tid + (int64_t)m * NT;
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
              const int64_t col = vi * VEC + e, cc = min(col, dmax);
              double sv = ld_coh(&vin[n_sp + cc]);
              if (scaled) sv *= (double)c.dscale[cc];
              vs[m][e] = (vi < nvec && col < n_d) ? (acc_t)sv : (acc_t)0;
              P[m][e] = (acc_t)0;
            }
          }
        };
        if (EXACT || n_d == 0) {
          // (the float64-accumulated product, run inside the CG's residual logic, loads them
          // one after another: its registers are the scarcer)
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
        } else if (c.dscale) {
          coef(true);
        } else {
          coef(false);
        }
      }
      // bf16 block with float32 accumulation: the row dots take packed bf16 pair products,
      // (s v) split into a bf16 high part and the bf16 rounding of its remainder (about 16
      // significant bits), so the stored pairs need no decoding for the dot
      constexpr bool kDot2 = DDT == DT_BF16 && !(EXACT || X);
      uint32_t vp[kDot2 ? NVT : 1][VEC];
      if constexpr (kDot2) {
#pragma unroll
        for (int m = 0; m < NVT; ++m)
#pragma unroll
          for (int w = 0; w < VEC / 2; ++w) {
            uint32_t hi[2], lo[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const float f = (float)vs[m][2 * w + h];
              hi[h] = bf16_rne(f);
              lo[h] = bf16_rne(f - __uint_as_float(hi[h] << 16));   // f - hi is exact
            }
            vp[m][w] = hi[0] | (hi[1] << 16);
            vp[m][VEC / 2 + w] = lo[0] | (lo[1] << 16);
          }
      }
      // the correlator part of the tile's row sums: tile_rows rows x (NT / tile_rows) slices
      __shared__ acc_t s_sp[kSlices][kCpsTileRows];
      __shared__ double s_spr[kCpsTileRows];      // the correlator part of each tile row's w
      acc_t *s_spf = &s_sp[0][0];
      const int tr = c.tile_rows, nsl = NT / tr;
      __shared__ double s_red[2][NWAVE][RB];
      double wsum = 0.0, wabs = 0.0;
      int par = 0;
      // One batch of RB dense rows into registers.  Rows past n_s and vectors past the row
      // load the last row's or vector's data instead (no branch around a load: the
      // compiler's wait counting then keeps the other batch's loads in flight).  Such
      // values only ever meet a zero weight (w_k = 0 for k >= n_s, v = 0 past the row) and
      // are never stored.
      auto load_batch = [&](u32x4 (&D)[RB][NVT], int64_t k0b) __attribute__((always_inline)) {
        if (nvec == 0) {
#pragma unroll
          for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int m = 0; m < NVT; ++m) D[r][m] = u32x4{0u, 0u, 0u, 0u};
          return;
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const int64_t k = min(k0b + r, n_s - 1);
          const unsigned char *rowp = c.dO + k * c.ldb_d;
#pragma unroll
          for (int m = 0; m < NVT; ++m) {
            const int64_t vi = min(tid + (int64_t)m * NT, nvec - 1);
            D[r][m] = load_stream(rowp + vi * 16);
          }
        }
      };
      double my_w = 0.0;                 // w of the tile's row k0 + tid (threads below tile_rows)
      // row dots of a batch, their workgroup sums, w_k, then P += D w from the same registers
      auto process = [&](u32x4 (&D)[RB][NVT], int64_t k0, int rb) __attribute__((always_inline)) {
        acc_t pd[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          acc_t acc = (acc_t)0;
          if constexpr (kDot2) {
            float ah = 0.0f, al = 0.0f;
#pragma unroll
            for (int m = 0; m < NVT; ++m)
#pragma unroll
              for (int w = 0; w < VEC / 2; ++w) {
                ah = dot2_bf16(D[r][m][w], vp[m][w], ah);
                al = dot2_bf16(D[r][m][w], vp[m][VEC / 2 + w], al);
              }
            acc = (acc_t)(ah + al);
          } else {
#pragma unroll
            for (int m = 0; m < NVT; ++m)
#pragma unroll
              for (int e = 0; e < VEC; ++e) acc += (acc_t)Storage<DDT>::get(D[r][m], e) * vs[m][e];
          }
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
            wr += s_spr[rb + r];
            wr -= cD;
          }
          if (tid == rb + r) my_w = wr;   // stored after the tile (no store inside the batch loop)
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
      // 1a. correlator part of w for the tile's rows: the groups' partial sums, each of the
      //     nsl slices of threads summing a fixed subset of the groups
      auto tile_head = [&](int64_t k0) __attribute__((always_inline)) {
        const int row = tid & (tr - 1), sl = tid / tr;
        const int64_t k = k0 + row;
        acc_t t = (acc_t)0;
        if (k < n_s) {
          const acc_t *part_sp = (const acc_t *)c.part_sp;
          for (int g = sl; g < c.n_grp; g += nsl) t += ld_acc(&part_sp[(int64_t)g * n_s + k]);
        }
        s_spf[sl * tr + row] = t;
        __syncthreads();
        // each row's slices summed once for the tile (not once per row inside the batches)
        if (tid < tr) {
          double sp = 0.0;
          for (int pi = 0; pi < nsl; ++pi) sp += (double)s_spf[pi * tr + tid];
          s_spr[tid] = sp;
        }
        __syncthreads();
      };
      auto tile_tail = [&](int64_t k0) __attribute__((always_inline)) {
        if (tid < tr && k0 + tid < n_s) st_coh(&c.w[k0 + tid], my_w);
        __syncthreads();                 // s_sp is rewritten by the next tile
      };
      // 1b. dense part in batches of RB rows.  Where the registers allow, two buffers: the
      //     next batch loads while this one is reduced, with no branch around any load (a
      //     tile has an even number of batches; the last one of a tile loads the first batch
      //     of the workgroup's next tile, past the end a clamped row that is never used).
      bool piped = false;
      if constexpr (kTwoBuf && !EXACT) {
        static_assert(kCpsMinTileRows % (2 * RB) == 0, "an even number of batches per tile");
        if (nvec > 0) {
          piped = true;
          u32x4 D0[RB][NVT], D1[RB][NVT];
          load_batch(D0, (int64_t)b * tr);
          for (int t = b; t < c.tiles; t += G) {
            const int64_t k0 = (int64_t)t * tr, k0n = (int64_t)(t + G) * tr;
            tile_head(k0);
            for (int rb = 0; rb < tr; rb += 2 * RB) {
              load_batch(D1, k0 + rb + RB);
              process(D0, k0, rb);
              load_batch(D0, rb + 2 * RB < tr ? k0 + rb + 2 * RB : k0n);
              process(D1, k0, rb + RB);
            }
            tile_tail(k0);
          }
        }
      }
      if (!piped) {
        for (int t = b; t < c.tiles; t += G) {
          const int64_t k0 = (int64_t)t * tr;
          tile_head(k0);
          for (int rb = 0; rb < tr; rb += RB) {
            u32x4 D[RB][NVT];
            load_batch(D, k0 + rb);
            process(D, k0, rb);
          }
          tile_tail(k0);
        }
      }
      // dense partial sums of this workgroup (zeros when it had no tile)
#pragma unroll
      for (int m = 0; m < NVT; ++m) {
        const int64_t vi = tid + (int64_t)m * NT;
        if (vi < nvec) {
          acc_t *dst = &part[(int64_t)b * c.n_dp + vi * VEC];
          if constexpr (sizeof(acc_t) == 4) {
            // float partials in pairs (8-byte aligned: n_dp and the vector start are
            // multiples of VEC)
#pragma unroll
            for (int e = 0; e < VEC; e += 2)
              st_coh64((u64 *)(dst + e), (u64)__float_as_uint((float)P[m][e]) | ((u64)__float_as_uint((float)P[m][e + 1]) << 32));
          } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) st_acc(&dst[e], P[m][e]);
          }
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
        // rows k4 .. k4+3 of every pass correlator: w and the state words of the thread's next
        // rows load while this step's bins are added.  No branch around a load or an atomic
        // (a branch makes the compiler wait for every outstanding access at the join):
        // loads past the rows or the pass's correlators read clamped addresses (the last
        // rows, kmax4 + 3 < ld_idx; the pass's first correlator); rows past n_s add zero,
        // and a state outside the correlator adds to its own bin, which is never read.
        const int64_t kstep = (int64_t)NT * 4, kmax4 = (n_s - 1) & ~(int64_t)3;
        double wv[4], wn[4];
        uint32_t sw[kPass], sn[kPass];
        auto fetch = [&](double (&wo)[4], uint32_t (&so)[kPass], int64_t k4) __attribute__((always_inline)) {
          const int64_t kc = min(k4, kmax4);
#pragma unroll
          for (int e = 0; e < 4; ++e) wo[e] = ld_coh(&c.w[min(kc + e, n_s - 1)]);
#pragma unroll
          for (int e = 0; e < kPass; ++e)
            so[e] = *(const uint32_t *)(c.idx + (p0 + (int64_t)(e < np ? e : 0) * G) * c.ld_idx + kc);
        };
        fetch(wv, sw, (int64_t)tid * 4);
        for (int64_t k4 = (int64_t)tid * 4; k4 < n_s; k4 += kstep) {
          fetch(wn, sn, k4 + kstep);     // past the rows: clamped, unused
          long long qv[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) qv[e] = (k4 + e < n_s) ? __double2ll_rn((wv[e] - wbar) * sigma) : 0ll;
#pragma unroll
          for (int e = 0; e < kPass; ++e) {
            if (e < np) {
#pragma unroll
              for (int r = 0; r < 4; ++r)   // (a state s >= n_states adds to a bin never read)
                atomicAdd((unsigned long long *)&s_bin[e][(sw[e] >> (8 * r)) & 0xFFu], (unsigned long long)qv[r]);
            }
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) wv[e] = wn[e];
#pragma unroll
          for (int e = 0; e < kPass; ++e) sw[e] = sn[e];
        }
        __syncthreads();
        // the pass correlators' values and v load together (one after another in the
        // float64-accumulated product, whose registers are the scarcer)
        if constexpr (EXACT) {
          for (int e = 0; e < np; ++e) {
            const int64_t p = p0 + (int64_t)e * G;
            for (int s_ = tid; s_ < ns; s_ += NT) {
              const int64_t j = p * ns + s_;
              const double T = (double)s_bin[e][s_] * inv_sigma;
              st_coh(&q[j], c.val[j] * T * inv_n + a.eps * ld_coh(&vin[j]));
            }
          }
        } else
        for (int s_ = tid; s_ < ns; s_ += NT) {
          double vv[kPass], vl[kPass];
#pragma unroll
          for (int e = 0; e < kPass; ++e) {
            const int64_t j = (p0 + (int64_t)e * G) * ns + s_;
            vv[e] = e < np ? c.val[j] : 0.0;
            vl[e] = e < np ? ld_coh(&vin[j]) : 0.0;
          }
#pragma unroll
          for (int e = 0; e < kPass; ++e) {
            if (e < np) {
              const double T = (double)s_bin[e][s_] * inv_sigma;
              st_coh(&q[(p0 + (int64_t)e * G) * ns + s_], vv[e] * T * inv_n + a.eps * vl[e]);
            }
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
            // eight workgroups' partials load together, then add in workgroup order
            int g = g0;
            for (; g + 8 <= g1; g += 8) {
              acc_t t8[8];
#pragma unroll
              for (int u = 0; u < 8; ++u) t8[u] = ld_acc(&part[(int64_t)(g + u) * c.n_dp + d]);
#pragma unroll
              for (int u = 0; u < 8; ++u) acc += (double)t8[u];
            }
            for (; g < g1; ++g) acc += (double)ld_acc(&part[(int64_t)g * c.n_dp + d]);
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
