// Storage-independent kernels (fill, prepare/gradient pass, quantizer) and the registry.
#include "sr_kernels.hpp"

namespace sr {

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Columns with err_j > tol, in increasing order (one workgroup of 1024 threads, a chunk of
// 1024 columns per pass: wave ballots, then the waves' counts).
__global__ __launch_bounds__(1024) void k_select(SelectArgs a) {
  __shared__ int s_cnt[16];
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t base = 0;
  for (int64_t c0 = 0; c0 < a.n_p; c0 += 1024) {
    const int64_t j = c0 + tid;
    const bool f = j < a.n_p && a.err[j] > a.tol;
    const u64 b = __ballot(f);
    const int below = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) s_cnt[wave] = __popcll(b);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      off += (w < wave) ? s_cnt[w] : 0;
      tot += s_cnt[w];
    }
    if (f) a.cols[base + off + below] = (int32_t)j;
    base += tot;
    __syncthreads();
  }
  if (tid == 0) *a.count = base;
}

// Column statistics of the correlator columns of index-coded CPS storage (one state per
// correlator per sample, Sec. II.C): with f_j the fraction of samples in state s of
// correlator p (j = p * n_states + s) and value val_j,
//   mean_j = val_j f_j,  diag S_j = val_j^2 f_j (1 - f_j),
//   g_j = (2/n_s) val_j (B_j - f_j B),  B_j = sum_{k in state} e_k,  B = sum_k e_k,
// with e_k = E_k - <E> (the centred form: B vanishes in exact arithmetic, and subtracting
// f_j B cancels its rounding, so a column every sample occupies gets exactly 0).  One
// workgroup per correlator (round robin); B_j and B are int64 fixed point (integer sums do
// not depend on their order, so every run gives the same bits).  Every workgroup computes
// <E>, sum |e| and B itself, in the same order.
__global__ __launch_bounds__(512) void k_cps_stats(CpsStatsArgs a) {
  constexpr int NT = 512;
  __shared__ unsigned int s_cnt[256];
  __shared__ long long s_e[256];
  const int tid = (int)threadIdx.x;
  const int64_t n_s = a.n_s;
  const int ns = a.n_states;
  const double inv_n = 1.0 / (double)n_s;
  __shared__ long long s_ball[NT / 64];
  double Ebar = 0.0, sigma = 1.0, Ball = 0.0;
  if (a.E != nullptr) {
    double se = 0.0;
    for (int64_t k = tid; k < n_s; k += NT) se += a.E[k];
    Ebar = block_sum(se) * inv_n;
    double sa = 0.0;
    for (int64_t k = tid; k < n_s; k += NT) sa += fabs(a.E[k] - Ebar);
    const double A = block_sum(sa);
    if (A > 0.0 && isfinite(A)) {
      int e;
      (void)frexp(A, &e);
      sigma = ldexp(1.0, 62 - e);
    }
    long long bt = 0;
    for (int64_t k = tid; k < n_s; k += NT) bt += __double2ll_rn((a.E[k] - Ebar) * sigma);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) bt += __shfl_xor(bt, off, 64);
    if ((tid & 63) == 0) s_ball[tid >> 6] = bt;
    __syncthreads();
    long long tot = 0;
    for (int w = 0; w < NT / 64; ++w) tot += s_ball[w];
    Ball = (double)tot;
    if (blockIdx.x == 0 && tid == 0 && a.Emean != nullptr) *a.Emean = Ebar;
  }
  for (int64_t p = blockIdx.x; p < a.n_corr; p += gridDim.x) {
    for (int i = tid; i < 256; i += NT) {
      s_cnt[i] = 0u;
      s_e[i] = 0ll;
    }
    __syncthreads();
    const unsigned char *row = a.idx + p * a.ld_idx;
    for (int64_t k4 = (int64_t)tid * 4; k4 < n_s; k4 += (int64_t)NT * 4) {
      const uint32_t word = *(const uint32_t *)(row + k4);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t k = k4 + r;
        const unsigned s = (word >> (8 * r)) & 0xFFu;
        if (k < n_s && s < (unsigned)ns) {
          atomicAdd(&s_cnt[s], 1u);
          if (a.E != nullptr)
            atomicAdd((unsigned long long *)&s_e[s], (unsigned long long)__double2ll_rn((a.E[k] - Ebar) * sigma));
        }
      }
    }
    __syncthreads();
    for (int s = tid; s < ns; s += NT) {
      const int64_t j = p * ns + s;
      const double f = (double)s_cnt[s] * inv_n, v = a.val[j];
      if (a.mean) a.mean[j] = v * f;
      if (a.diag) a.diag[j] = v * v * f * (1.0 - f);
      if (a.g && a.E) a.g[j] = 2.0 * inv_n * v * (((double)s_e[s] - f * Ball) / sigma);
    }
    __syncthreads();
  }
}
const void *cps_stats_kernel() { return (const void *)&k_cps_stats; }

// Products during sampling (Sec. I: each sampled configuration adds an outer product).
// Accumulators over the batches seen so far, with n the samples, obar = s1 / n:
//   A_i = sum_k O_k (O_k . z_i),  s1 = sum_k O_k,  se = sum_k E_k O_k,  scal = (n, sum_k E_k)
// A batch of B samples with column means mean_b, <E>_b and gradient g_b adds
//   s1 += B mean_b,  se += B (g_b / 2 + <E>_b mean_b),  A_i += B y_b (y_b = O_b^T (O_b z_i) / B).
__global__ void k_stream_stats(StreamArgs a) {
  const double Eb = a.Emean_b ? *a.Emean_b : 0.0;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.n_p; j += (int64_t)gridDim.x * blockDim.x) {
    a.s1[j] += a.B * a.mean_b[j];
    if (a.se && a.g_b) a.se[j] += a.B * (0.5 * a.g_b[j] + Eb * a.mean_b[j]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.scal[0] += a.B;
    if (a.Emean_b) a.scal[1] += a.B * Eb;
  }
}
__global__ void k_stream_addy(StreamArgs a) {
  double *Ai = a.A + (int64_t)a.i * a.n_p;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.n_p; j += (int64_t)gridDim.x * blockDim.x)
    Ai[j] += a.B * a.y_b[j];
}
// Partial dots of s1 . z_i: kStreamDotBlocks workgroups per vector, each over a fixed chunk
// of the parameters, write dots[i * kStreamDotBlocks + b]; k_stream_finish sums them in
// block order (a fixed order: the result is the same on every run).
constexpr int kStreamDotBlocks = 64;
constexpr int kStreamDotVectors = 8;     // at most this many vectors (the host checks m)
int stream_dot_blocks() { return kStreamDotBlocks; }
__global__ __launch_bounds__(512) void k_stream_dots(StreamArgs a) {
  const int i = (int)blockIdx.x / kStreamDotBlocks, b = (int)blockIdx.x % kStreamDotBlocks;
  const int64_t ch = (a.n_p + kStreamDotBlocks - 1) / kStreamDotBlocks;
  const int64_t j0 = min(a.n_p, (int64_t)b * ch), j1 = min(a.n_p, j0 + ch);
  const double *z = a.Z + (int64_t)i * a.n_p;
  double acc = 0.0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 512) acc += a.s1[j] * z[j];
  acc = block_sum(acc);
  if (threadIdx.x == 0) a.dots[blockIdx.x] = acc;
}
// Y_i = A_i / n - obar (s1 . z_i) / n + eps z_i  (the centred product: sum_k (O_k - obar)(O_k . z_i) / n),
// g = 2 (se / n - <E> obar), col_mean = obar, E_mean = <E>
__global__ void k_stream_finish(StreamArgs a) {
  const double n = a.scal[0], inv_n = 1.0 / n, Ebar = a.scal[1] * inv_n;
  __shared__ double s_dots[kStreamDotVectors];
  if ((int)threadIdx.x < a.m && (int)threadIdx.x < kStreamDotVectors) {
    double t = 0.0;
    for (int b = 0; b < kStreamDotBlocks; ++b) t += a.dots[threadIdx.x * kStreamDotBlocks + b];
    s_dots[threadIdx.x] = t;
  }
  __syncthreads();
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.n_p; j += (int64_t)gridDim.x * blockDim.x) {
    const double ob = a.s1[j] * inv_n;
    for (int i = 0; i < a.m; ++i) {
      const int64_t ij = (int64_t)i * a.n_p + j;
      a.Y[ij] = a.A[ij] * inv_n - ob * (s_dots[i] * inv_n) + a.eps * a.Z[ij];
    }
    if (a.col_mean) a.col_mean[j] = ob;
    if (a.g && a.se) a.g[j] = 2.0 * (a.se[j] * inv_n - Ebar * ob);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && a.E_mean) *a.E_mean = Ebar;
}
const void *stream_kernel(int which) {
  switch (which) {
    case 0: return (const void *)&k_stream_stats;
    case 1: return (const void *)&k_stream_addy;
    case 2: return (const void *)&k_stream_dots;
    default: return (const void *)&k_stream_finish;
  }
}

// Streaming-read ceiling: every thread reads U 16-byte vectors per pass with the
// products' non-temporal loads, grid-stride over `bytes`, and folds them into one word so
// the loads are kept; the workgroup's words go to sink[blockIdx.x].
template <int U>
__global__ __launch_bounds__(512) void k_stream_read(const unsigned char *p, int64_t n_vec, uint32_t *sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (; i + (U - 1) * stride < n_vec; i += U * stride) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load_stream(p + (i + u * stride) * 16);
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u][0] ^ v[u][1] ^ v[u][2] ^ v[u][3];
  }
  for (; i < n_vec; i += stride) {
    const u32x4 v = load_stream(p + i * 16);
    acc ^= v[0] ^ v[1] ^ v[2] ^ v[3];
  }
  __shared__ uint32_t s_acc[8];
  for (int off = 32; off >= 1; off >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, off, 64);
  if ((threadIdx.x & 63) == 0) s_acc[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t ^= s_acc[w];
    sink[blockIdx.x] = t;
  }
}
const void *stream_read_kernel(int unroll) {
  switch (unroll) {
    case 2: return (const void *)&k_stream_read<2>;
    case 4: return (const void *)&k_stream_read<4>;
    case 8: return (const void *)&k_stream_read<8>;
    default: return nullptr;
  }
}

const KernelEntry *kernel_table_f64(int *count);
const KernelEntry *kernel_table_f32(int *count);
const KernelEntry *kernel_table_bf16(int *count);
const KernelEntry *kernel_table_f16(int *count);

const BatchEntry *batched_entry_f64();
const BatchEntry *batched_entry_f32();

const void *shift_kernel_f64(int nv, int r, int look, int poll, int nt, bool batched);
const void *shift_kernel_f32(int nv, int r, int look, int poll, int nt, bool batched);
const void *shift_kernel(int dt, int nv, int r, int look, int poll, int nt, bool batched) {
  switch (dt) {
    case DT_F64: return shift_kernel_f64(nv, r, look, poll, nt, batched);
    case DT_F32: return shift_kernel_f32(nv, r, look, poll, nt, batched);
    default: return nullptr;
  }
}

const BatchEntry *batched_entry(int dt) {
  switch (dt) {
    case DT_F64: return batched_entry_f64();
    case DT_F32: return batched_entry_f32();
    default: return nullptr;
  }
}

const CpsEntry *cps_table_f64(int *count);
const CpsEntry *cps_table_f32(int *count);
const CpsEntry *cps_table_bf16(int *count);
const CpsEntry *cps_table(int dt, int *count) {
  switch (dt) {
    case DT_F64: return cps_table_f64(count);
    case DT_F32: return cps_table_f32(count);
    case DT_BF16: return cps_table_bf16(count);
    default: *count = 0; return nullptr;
  }
}

const KernelEntry *kernel_table(int dt, int *count) {
  switch (dt) {
    case DT_F64: return kernel_table_f64(count);
    case DT_F32: return kernel_table_f32(count);
    case DT_BF16: return kernel_table_bf16(count);
    default: return kernel_table_f16(count);
  }
}

const void *grad_kernel(int dt) {
  switch (dt) {
    case DT_F64: return (const void *)&k_grad<DT_F64, 4, 4, 256>;
    case DT_F32: return (const void *)&k_grad<DT_F32, 2, 8, 256>;
    case DT_BF16: return (const void *)&k_grad<DT_BF16, 1, 8, 512>;
    default: return (const void *)&k_grad<DT_F16, 1, 8, 512>;
  }
}
int grad_nv(int dt) { return dt == DT_F64 ? 4 : dt == DT_F32 ? 2 : 1; }
int grad_threads(int dt) { return dt == DT_F64 || dt == DT_F32 ? 256 : 512; }
int grad_rows(int dt) { return dt == DT_F64 ? 4 : 8; }

const void *absmax_kernel(int in_dt) {
  return in_dt == DT_F64 ? (const void *)&k_absmax<DT_F64> : (const void *)&k_absmax<DT_F32>;
}
const void *quantize_kernel(int in_dt, int out_dt) {
  if (in_dt == DT_F64)
    return out_dt == DT_BF16 ? (const void *)&k_quantize<DT_F64, DT_BF16> : (const void *)&k_quantize<DT_F64, DT_F16>;
  return out_dt == DT_BF16 ? (const void *)&k_quantize<DT_F32, DT_BF16> : (const void *)&k_quantize<DT_F32, DT_F16>;
}
const void *fill_kernel() { return (const void *)&k_fill_u32; }

const void *gradlo_part_kernel(int dt) {
  return dt == DT_BF16 ? (const void *)&k_gradlo_part<DT_BF16> : (const void *)&k_gradlo_part<DT_F16>;
}
const void *gradlo_finish_kernel(int dt) {
  return dt == DT_BF16 ? (const void *)&k_gradlo_finish<DT_BF16> : (const void *)&k_gradlo_finish<DT_F16>;
}
const void *remmax_kernel(int in_dt, int out_dt) {
  if (in_dt == DT_F64)
    return out_dt == DT_BF16 ? (const void *)&k_remmax<DT_F64, DT_BF16> : (const void *)&k_remmax<DT_F64, DT_F16>;
  return out_dt == DT_BF16 ? (const void *)&k_remmax<DT_F32, DT_BF16> : (const void *)&k_remmax<DT_F32, DT_F16>;
}
const void *select_kernel() { return (const void *)&k_select; }
const void *quantize_lo_kernel(int in_dt, int out_dt) {
  if (in_dt == DT_F64)
    return out_dt == DT_BF16 ? (const void *)&k_quantize_lo<DT_F64, DT_BF16>
                             : (const void *)&k_quantize_lo<DT_F64, DT_F16>;
  return out_dt == DT_BF16 ? (const void *)&k_quantize_lo<DT_F32, DT_BF16> : (const void *)&k_quantize_lo<DT_F32, DT_F16>;
}

}  // namespace sr
