// Batched form: several right-hand sides per product and many independent systems in
// one persistent launch (float64 and float32 storage).
#pragma once
#include "sr_kernels.hpp"

namespace sr {

constexpr int pow2_at_least(int n) { return n <= 1 ? 1 : 2 * pow2_at_least((n + 1) / 2); }
constexpr int log2_exact(int n) { return n <= 1 ? 0 : 1 + log2_exact(n / 2); }

// Sums of N values (N a power of two <= 64) over the 64 lanes of a wave by recursive
// halving: at each of the first log2(N) exchange stages a lane keeps half of its values
// and adds its partner's copies of them, so N sums cost N - 1 + 6 - log2(N) exchanges
// instead of 6 N.  On return lane l holds the sum of value l >> (6 - log2(N)).
template <int N, int STAGE, typename T> __device__ __forceinline__ void multi_wave_stage(T (&v)[N], int lane) {
  if constexpr ((N >> STAGE) > 1) {
    constexpr int off = 32 >> STAGE, half = N >> (STAGE + 1);
    const bool upper = (lane & off) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const T send = upper ? v[i] : v[i + half];
      const T keep = upper ? v[i + half] : v[i];
      v[i] = keep + __shfl_xor(send, off, 64);
    }
    multi_wave_stage<N, STAGE + 1>(v, lane);   // (stages as template arguments: every index is static)
  }
}
template <int N, typename T> __device__ __forceinline__ T multi_wave_sum(T (&v)[N], int lane) {
  static_assert(N >= 1 && N <= 64 && (N & (N - 1)) == 0, "N must be a power of two <= 64");
  constexpr int L = log2_exact(N);
  multi_wave_stage<N, 0>(v, lane);
  T x = v[0];
#pragma unroll
  for (int off = 32 >> L; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
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
//   2. Updates: a workgroup takes threads * VEC columns and one split of at most
//      kBatchSplitRows rows; the split's centred row dots (summed over parts) sit in LDS,
//      each thread accumulates sum_rows O_rj w[row][k] for its VEC columns and all k,
//      rows kBatchU at a time.
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
