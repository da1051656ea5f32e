// Implicit-adjoint backward of the SR solve x = (S + eps I)^{-1} g (the differentiation
// form; the paper has no backward).  With lambda = (S + eps I)^{-1} dL/dx from a second
// CG solve, the gradients with respect to the sampled inputs are rank-2 outer products
// (closed form derived from Eq. sr_overlap and the gradient g = 2 cov(E, O)):
//   p1 = Oc x,  p2 = Oc lambda                      (one read of O, two dots per row)
//   dL/dO_kj = (1/N) [ (2 e_k - p1_k) lambda_j - p2_k x_j ],   e_k = E_k - <E>
//   dL/dE_k  = (2/N) p2_k
// Three launches: the two-vector row dots (partials per column group), a one-block
// finish (fixed-order sums over column groups, <E>, the row coefficients), and the
// rank-2 write of dL/dO.
#include "sr_launch.hpp"

namespace sr {

constexpr int kAdjNT = 256;   // threads per workgroup of the adjoint kernels
constexpr int kAdjRR = 4;     // rows reduced together in the row-dot kernel

// Workgroup (cg, rg) = (blockIdx.x % C, blockIdx.x / C) owns columns
// [cg*wslice, min(n_p, (cg+1)*wslice)) and rows rg*RR, (rg + RG)*RR, ...; for each row
// it writes its share of p1 and p2 (its centring share subtracted) to part[cg][row][2].
template <int DT, int NV>
__global__ __launch_bounds__(kAdjNT) void k_rowdots2(RowDotsArgs a) {
  typedef Storage<DT> St;
  constexpr int VEC = St::VEC;
  constexpr int NW = kAdjNT / 64;
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cg = (int)(blockIdx.x % (unsigned)a.C), rg = (int)(blockIdx.x / (unsigned)a.C);
  const int64_t c0 = (int64_t)cg * a.wslice;
  const int64_t c1 = min(a.n_p, c0 + a.wslice);
  double xs[NV][VEC], ls[NV][VEC];
  int64_t colv[NV];
  unsigned valid[NV];                  // bit e: element e of vector i is a column < n_p
  double cx = 0.0, cl = 0.0;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int64_t col = c0 + ((int64_t)i * kAdjNT + tid) * VEC;
    colv[i] = col < c1 ? col : c0;     // a valid address of the slice; its elements are masked
    valid[i] = 0u;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int64_t j = col + e;
      const bool in = col < c1 && j < a.n_p;
      valid[i] |= in ? (1u << e) : 0u;
      const double s = (in && a.scale != nullptr) ? (double)a.scale[j] : 1.0;
      xs[i][e] = in ? a.x[j] * s : 0.0;
      ls[i][e] = in ? a.lam[j] * s : 0.0;
      if (in) {
        cx += a.mean[j] * a.x[j];
        cl += a.mean[j] * a.lam[j];
      }
    }
  }
  __shared__ double s_red[2][NW][2 * kAdjRR];
  __shared__ double s_c[NW][2];
  cx = wave_sum(cx);
  cl = wave_sum(cl);
  if (lane == 0) {
    s_c[wave][0] = cx;
    s_c[wave][1] = cl;
  }
  __syncthreads();
  double shx = 0.0, shl = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    shx += s_c[w][0];
    shl += s_c[w][1];
  }
  int buf = 0;
  for (int64_t r0 = (int64_t)rg * kAdjRR; r0 < a.n_s; r0 += (int64_t)a.RG * kAdjRR) {
    double d[2 * kAdjRR];
#pragma unroll
    for (int rr = 0; rr < kAdjRR; ++rr) {
      const int64_t row = min(r0 + rr, a.n_s - 1);
      const unsigned char *rowp = a.O + row * a.ldb;
      double d1 = 0.0, d2 = 0.0;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const u32x4 q = load_stream(rowp + colv[i] * St::BYTES);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          // padding past n_p may hold anything (NaN): select, do not multiply by zero
          const double o = ((valid[i] >> e) & 1u) ? (double)St::get(q, e) : 0.0;
          d1 += o * xs[i][e];
          d2 += o * ls[i][e];
        }
      }
      d[2 * rr] = wave_sum(d1);
      d[2 * rr + 1] = wave_sum(d2);
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 2 * kAdjRR; ++k) s_red[buf][wave][k] = d[k];
    }
    __syncthreads();
    if (tid < 2 * kAdjRR) {
      const int64_t row = r0 + tid / 2;
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) t += s_red[buf][w][tid];
      if (row < a.n_s) a.part[((int64_t)cg * a.n_s + row) * 2 + (tid & 1)] = t - ((tid & 1) ? shl : shx);
    }
    buf ^= 1;   // the other buffer is written next: one barrier per row block suffices
  }
}

// One workgroup: <E>, then per row p1, p2 (fixed order over column groups), dE and the
// coefficients of the rank-2 update: coef[k] = (2 e_k - p1_k)/N, coef[n_s + k] = -p2_k/N;
// and dL/deps = -lambda . x when asked (n_s = 0: that alone).
__global__ __launch_bounds__(1024) void k_adjoint_finish(AdjFinishArgs a) {
  __shared__ double s_w[16];
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (a.deps != nullptr) {
    double d = 0.0;
    for (int64_t j = tid; j < a.n_p; j += 1024) d += a.lam[j] * a.x[j];
    d = wave_sum(d);
    if (lane == 0) s_w[wave] = d;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < 16; ++w) t += s_w[w];
      *a.deps = -t;
    }
    __syncthreads();
  }
  if (a.n_s == 0) return;
  double se = 0.0;
  for (int64_t k = tid; k < a.n_s; k += 1024) se += a.E[k];
  se = wave_sum(se);
  if (lane == 0) s_w[wave] = se;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < 16; ++w) tot += s_w[w];
  const double inv_n = 1.0 / (double)a.n_s;
  const double emean = tot * inv_n;
  for (int64_t k = tid; k < a.n_s; k += 1024) {
    double p1 = 0.0, p2 = 0.0;
    for (int c = 0; c < a.C; ++c) {
      p1 += a.part[((int64_t)c * a.n_s + k) * 2 + 0];
      p2 += a.part[((int64_t)c * a.n_s + k) * 2 + 1];
    }
    a.coef[k] = (2.0 * (a.E[k] - emean) - p1) * inv_n;
    a.coef[a.n_s + k] = -p2 * inv_n;
    if (a.dE != nullptr) a.dE[k] = 2.0 * p2 * inv_n;
    if (a.p12 != nullptr) {
      a.p12[k] = p1;
      a.p12[a.n_s + k] = p2;
    }
  }
}

// dO[k][j] = coef[k] lambda_j + coef[n_s + k] x_j.  Each thread owns one 16-byte output
// vector of columns and walks rows blockIdx.y, blockIdx.y + gridDim.y, ...
template <typename T>
__global__ __launch_bounds__(kAdjNT) void k_rank2(Rank2Args a) {
  constexpr int W = 16 / (int)sizeof(T);
  const int64_t col = ((int64_t)blockIdx.x * kAdjNT + threadIdx.x) * W;
  if (col >= a.n_p) return;
  double lv[W], xv[W];
#pragma unroll
  for (int e = 0; e < W; ++e) {
    const bool in = col + e < a.n_p;
    lv[e] = in ? a.lam[col + e] : 0.0;
    xv[e] = in ? a.x[col + e] : 0.0;
  }
  const bool full = col + W <= a.n_p;
  for (int64_t k = blockIdx.y; k < a.n_s; k += gridDim.y) {
    const double ca = a.coef[k], cb = a.coef[a.n_s + k];
    T *row = (T *)a.dO + k * a.ld;
    if (full) {
      if constexpr (W == 2) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        d2 v = {ca * lv[0] + cb * xv[0], ca * lv[1] + cb * xv[1]};
        __builtin_nontemporal_store(v, (d2 *)(row + col));
      } else {
        typedef float f4 __attribute__((ext_vector_type(4)));
        f4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (float)(ca * lv[e] + cb * xv[e]);
        __builtin_nontemporal_store(v, (f4 *)(row + col));
      }
    } else {
      for (int e = 0; e < W && col + e < a.n_p; ++e) row[col + e] = (T)(ca * lv[e] + cb * xv[e]);
    }
  }
}

template <int DT>
static const void *rowdots_for(int nv) {
  switch (nv) {
    case 1: return (const void *)&k_rowdots2<DT, 1>;
    case 2: return (const void *)&k_rowdots2<DT, 2>;
    default: return (const void *)&k_rowdots2<DT, 4>;
  }
}

const void *rowdots_kernel(int dt, int nv) {
  switch (dt) {
    case DT_F64: return rowdots_for<DT_F64>(nv);
    case DT_F32: return rowdots_for<DT_F32>(nv);
    case DT_BF16: return rowdots_for<DT_BF16>(nv);
    default: return rowdots_for<DT_F16>(nv);
  }
}
const void *adjoint_finish_kernel() { return (const void *)&k_adjoint_finish; }
const void *rank2_kernel(int out_dt) {
  return out_dt == DT_F64 ? (const void *)&k_rank2<double> : (const void *)&k_rank2<float>;
}
int adjoint_threads() { return kAdjNT; }
int adjoint_rows_per_block() { return kAdjRR; }

}  // namespace sr
