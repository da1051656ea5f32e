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

const void *shift_kernel_f64(int nv, int r, int look, int poll, int nt);
const void *shift_kernel_f32(int nv, int r, int look, int poll, int nt);
const void *shift_kernel(int dt, int nv, int r, int look, int poll, int nt) {
  switch (dt) {
    case DT_F64: return shift_kernel_f64(nv, r, look, poll, nt);
    case DT_F32: return shift_kernel_f32(nv, r, look, poll, nt);
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
    case DT_F64: return (const void *)&k_grad<DT_F64, 4, 4>;
    case DT_F32: return (const void *)&k_grad<DT_F32, 2, 8>;
    case DT_BF16: return (const void *)&k_grad<DT_BF16, 1, 8>;
    default: return (const void *)&k_grad<DT_F16, 1, 8>;
  }
}
int grad_nv(int dt) { return dt == DT_F64 ? 4 : dt == DT_F32 ? 2 : 1; }
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
