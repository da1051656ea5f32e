// Vector kernels of the generalized Davidson solver of the linear method (Sec. II.B): the
// products H t and S t come from the fused product kernels; what remains per iteration
// are a few dot products against the subspace bases and linear combinations of them.
// Every reduction has a fixed order (partial sums per workgroup, then one workgroup).
#include "sr_lm.hpp"

namespace sr {

constexpr int kLmNT = 256;

// part[b][i] = sum over workgroup b's slice of j of X[i][j] * w[j], i < m.
__global__ __launch_bounds__(kLmNT) void k_mdot_part(MdotArgs a) {
  const int64_t ch = (a.n + gridDim.x - 1) / gridDim.x;
  const int64_t j0 = min(a.n, (int64_t)blockIdx.x * ch), j1 = min(a.n, j0 + ch);
  __shared__ double s_w[kLmNT / 64];
  for (int i = 0; i < a.m; ++i) {
    double acc = 0.0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kLmNT) acc += a.X[i * a.ld + j] * a.w[j];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int q = 0; q < kLmNT / 64; ++q) t += s_w[q];
      a.part[(int64_t)blockIdx.x * a.m + i] = t;
    }
    __syncthreads();
  }
}

// out[i] = sum over workgroups b (in order) of part[b][i].
__global__ __launch_bounds__(64) void k_mdot_final(MdotArgs a) {
  const int i = (int)threadIdx.x;
  if (i < a.m) {
    double t = 0.0;
    for (int b = 0; b < a.nb; ++b) t += a.part[(int64_t)b * a.m + i];
    a.out[i] = t;
  }
}

// out[j] = beta out[j] + sum_i ca[i] X[i][j] + sum_i cz[i] Z[i][j]  (out may be a row of X
// or Z only when that row's coefficient is zero).
__global__ __launch_bounds__(kLmNT) void k_lincomb(LincombArgs a) {
  for (int64_t j = (int64_t)blockIdx.x * kLmNT + threadIdx.x; j < a.n; j += (int64_t)gridDim.x * kLmNT) {
    double t = a.beta == 0.0 ? 0.0 : a.beta * a.out[j];
    for (int i = 0; i < a.mx; ++i) t += a.ca[i] * a.X[i * a.ld + j];
    for (int i = 0; i < a.mz; ++i) t += a.cz[i] * a.Z[i * a.ld + j];
    a.out[j] = t;
  }
}

// out[j] = in[j] / d[j] (the diagonal preconditioner of the Davidson correction); a
// non-positive d[j] (a constant column) leaves the component as it is.
__global__ __launch_bounds__(kLmNT) void k_divide(DivArgs a) {
  for (int64_t j = (int64_t)blockIdx.x * kLmNT + threadIdx.x; j < a.n; j += (int64_t)gridDim.x * kLmNT) {
    const double d = a.d[j];
    a.out[j] = d > 0.0 ? a.in[j] / d : a.in[j];
  }
}

const void *divide_kernel() { return (const void *)&k_divide; }
const void *mdot_part_kernel() { return (const void *)&k_mdot_part; }
const void *mdot_final_kernel() { return (const void *)&k_mdot_final; }
const void *lincomb_kernel() { return (const void *)&k_lincomb; }
int lm_threads() { return kLmNT; }

}  // namespace sr
