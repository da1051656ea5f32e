// Storage-independent kernels (fill, prepare/gradient pass, quantizer) and the registry.
#include "sr_kernels.hpp"

namespace sr {

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
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

}  // namespace sr
