// Vector kernels of the generalized Davidson solver of the linear method (Sec. II.B): the
// products H t and S t come from the fused product kernels; what remains per iteration
// are a few dot products against the subspace bases and linear combinations of them.
// Every reduction has a fixed order (partial sums per workgroup, then one workgroup).
#include "sr_lm.hpp"

namespace sr {

constexpr int kLmNT = 256;

// part[b][i] = sum over workgroup (b, i)'s slice of j of X[i][j] * w[j]: one workgroup
// row per dot (grid nb x m), so the m reductions run side by side.
__global__ __launch_bounds__(kLmNT) void k_mdot_part(MdotArgs a) {
  const int64_t ch = (a.n + gridDim.x - 1) / gridDim.x;
  const int64_t j0 = min(a.n, (int64_t)blockIdx.x * ch), j1 = min(a.n, j0 + ch);
  const int i = (int)blockIdx.y;
  __shared__ double s_w[kLmNT / 64];
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
// or Z only when that row's coefficient is zero).  X's coefficients and beta may instead
// come from device memory (cdev, bdev), so that no host round trip sits between the dot
// products that produce them and this combination.
__global__ __launch_bounds__(kLmNT) void k_lincomb(LincombArgs a) {
  const double beta = a.bdev != nullptr ? 1.0 / sqrt(*a.bdev) : a.beta;
  for (int64_t j = (int64_t)blockIdx.x * kLmNT + threadIdx.x; j < a.n; j += (int64_t)gridDim.x * kLmNT) {
    double t = beta == 0.0 ? 0.0 : beta * a.out[j];
    for (int i = 0; i < a.mx; ++i) t += (a.cdev != nullptr ? a.cdev_sign * a.cdev[i] : a.ca[i]) * a.X[i * a.ld + j];
    for (int i = 0; i < a.mz; ++i) t += a.cz[i] * a.Z[i * a.ld + j];
    a.out[j] = t;
  }
}

// The diagonal preconditioner of the Davidson correction.  With diag H: out[j] =
// in[j] / (dh[j] - theta ds[j]), the denominator kept at least 1e-8 of its terms' size
// (sign kept) where it nearly vanishes; without: out[j] = in[j] / ds[j], a non-positive
// ds[j] (a constant column) leaving the component as it is.
__global__ __launch_bounds__(kLmNT) void k_divide(DivArgs a) {
  for (int64_t j = (int64_t)blockIdx.x * kLmNT + threadIdx.x; j < a.n; j += (int64_t)gridDim.x * kLmNT) {
    if (a.dh != nullptr) {
      const double h = a.dh[j], s = a.ds[j], den = h - a.theta * s;
      const double floor = 1e-8 * (fabs(h) + fabs(a.theta * s)) + 1e-300;
      a.out[j] = a.in[j] / (fabs(den) >= floor ? den : copysign(floor, den));
    } else {
      const double s = a.ds[j];
      a.out[j] = s > 0.0 ? a.in[j] / s : a.in[j];
    }
  }
}

// One stored element as float64 (column scale applied for scaled storage).
template <int DT>
__device__ __forceinline__ double stored_elem(const Operand &op, int64_t k, int64_t j) {
  const unsigned char *row = op.O + k * op.ldb;
  double v;
  if constexpr (DT == DT_F64) {
    v = ((const double *)row)[j];
  } else if constexpr (DT == DT_F32) {
    v = (double)((const float *)row)[j];
  } else if constexpr (DT == DT_BF16) {
    v = (double)__uint_as_float((uint32_t)((const uint16_t *)row)[j] << 16);
  } else {
    v = (double)__builtin_bit_cast(_Float16, ((const uint16_t *)row)[j]);
  }
  return op.scale != nullptr ? v * (double)op.scale[j] : v;
}

// part[sp][j] = sum over the rows k of split sp of Oc_kj (E_k Oc_kj + D_kj); thread = column.
template <int DT>
__global__ __launch_bounds__(kLmNT) void k_diagh_part(DiagHArgs a) {
  const int64_t j = (int64_t)blockIdx.x * kLmNT + threadIdx.x;
  const int sp = (int)blockIdx.y;
  if (j >= a.n_p) return;
  const int64_t k0 = (int64_t)sp * a.rs, k1 = min(a.n_s, k0 + a.rs);
  const double m = a.mean[j];
  double acc = 0.0;
  for (int64_t k = k0; k < k1; ++k) {
    const double oc = stored_elem<DT>(a.o, k, j) - m;
    acc += oc * (a.E[k] * oc + stored_elem<DT>(a.d, k, j));
  }
  a.part[(int64_t)sp * a.n_p + j] = acc;
}

// out[j] = (sum over splits in order of part[sp][j]) / n_s.
__global__ __launch_bounds__(kLmNT) void k_diagh_final(DiagHArgs a) {
  const int64_t j = (int64_t)blockIdx.x * kLmNT + threadIdx.x;
  if (j >= a.n_p) return;
  double t = 0.0;
  for (int sp = 0; sp < a.SP; ++sp) t += a.part[(int64_t)sp * a.n_p + j];
  a.out[j] = t / (double)a.n_s;
}

const void *divide_kernel() { return (const void *)&k_divide; }
const void *diagh_part_kernel(int dt) {
  switch (dt) {
    case DT_F64: return (const void *)&k_diagh_part<DT_F64>;
    case DT_F32: return (const void *)&k_diagh_part<DT_F32>;
    case DT_BF16: return (const void *)&k_diagh_part<DT_BF16>;
    default: return (const void *)&k_diagh_part<DT_F16>;
  }
}
const void *diagh_final_kernel() { return (const void *)&k_diagh_final; }
const void *mdot_part_kernel() { return (const void *)&k_mdot_part; }
const void *mdot_final_kernel() { return (const void *)&k_mdot_final; }
const void *lincomb_kernel() { return (const void *)&k_lincomb; }
int lm_threads() { return kLmNT; }

}  // namespace sr
