// Device-side building blocks shared by the libsr kernels (gfx950, wave64).
//
//  * Storage decoding: 16-byte vector loads of the stored derivative ratios and the
//    per-element decode for float64, float32, bfloat16 and float16 storage.
//  * Coherent accesses: data shared between workgroups inside one launch is written and
//    read with relaxed device-scope atomics, which gfx950 issues as write-through /
//    coherent-read accesses (no L2 writeback or invalidate is needed around them).
//  * Grid barrier: every workgroup publishes an epoch in its own flag word and polls the
//    flags of all others (no contended read-modify-write), with a bounded spin that turns
//    a lost workgroup into an abort flag instead of a hang.
//  * Partial-sum exchange: workgroups that split the columns of one row tile publish their
//    partial dot products as 64-bit words that carry a round tag in the upper half, so a
//    reader knows a word is current without any separate flag or fence.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sr {

typedef unsigned long long u64;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

enum { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_F16 = 3 };

// Upper bound of polls in one cross-workgroup wait (each poll is a round trip through
// the coherent memory level, about a microsecond); beyond it the wait gives up and the
// launch aborts, so every wave reaches the end of the kernel.
constexpr uint64_t kSpinLimit = 1ull << 23;

// ------------------------------------------------------------------------------------
// Storage decoding
// ------------------------------------------------------------------------------------
template <int DT> struct Storage;

template <> struct Storage<DT_F64> {
  static constexpr int VEC = 2;          // elements per 16-byte vector
  static constexpr int BYTES = 8;
  typedef double acc_t;                  // accumulation type of the products
  static constexpr int WPD = 2;          // exchange words per partial dot
  __device__ static __forceinline__ double get(const u32x4 &v, int e) {
    u64 b = ((u64)v[2 * e + 1] << 32) | (u64)v[2 * e];
    return __longlong_as_double((long long)b);
  }
};
template <> struct Storage<DT_F32> {
  static constexpr int VEC = 4;
  static constexpr int BYTES = 4;
  typedef double acc_t;
  static constexpr int WPD = 2;
  __device__ static __forceinline__ double get(const u32x4 &v, int e) {
    return (double)__uint_as_float(v[e]);
  }
};
template <> struct Storage<DT_BF16> {
  static constexpr int VEC = 8;
  static constexpr int BYTES = 2;
  typedef float acc_t;
  static constexpr int WPD = 1;
  __device__ static __forceinline__ float get(const u32x4 &v, int e) {
    uint32_t w = v[e >> 1];
    return __uint_as_float((e & 1) ? (w & 0xFFFF0000u) : (w << 16));
  }
};
template <> struct Storage<DT_F16> {
  static constexpr int VEC = 8;
  static constexpr int BYTES = 2;
  typedef float acc_t;
  static constexpr int WPD = 1;
  __device__ static __forceinline__ float get(const u32x4 &v, int e) {
    uint32_t w = v[e >> 1];
    uint16_t h = (uint16_t)((e & 1) ? (w >> 16) : (w & 0xFFFFu));
    return (float)__builtin_bit_cast(_Float16, h);
  }
};

// Streaming 16-byte load of stored ratios (read once per product: non-temporal).  The
// pointer is cast to the global address space: a pointer the kernel read from memory
// (a table of systems) would otherwise be generic, and generic (flat) loads also count
// against the LDS wait counter, so every LDS wait would drain the tile prefetch.
typedef __attribute__((address_space(1))) const u32x4 global_u32x4;
__device__ __forceinline__ u32x4 load_stream(const void *p) {
  return __builtin_nontemporal_load((global_u32x4 *)p);
}

// ------------------------------------------------------------------------------------
// Coherent (device-scope) accesses for data shared between workgroups of one launch
// ------------------------------------------------------------------------------------
// (all of them address global memory: the casts keep pointers read from memory from
// turning into generic accesses)
typedef __attribute__((address_space(1))) u64 global_u64;
typedef __attribute__((address_space(1))) uint32_t global_u32;
__device__ __forceinline__ void st_coh(double *p, double v) {
  __hip_atomic_store((global_u64 *)p, (u64)__double_as_longlong(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double *p) {
  return __longlong_as_double(
      (long long)__hip_atomic_load((global_u64 *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_coh64(u64 *p, u64 v) {
  __hip_atomic_store((global_u64 *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 ld_coh64(const u64 *p) {
  return __hip_atomic_load((global_u64 *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh32(uint32_t *p, uint32_t v) {
  __hip_atomic_store((global_u32 *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_coh32(const uint32_t *p) {
  return __hip_atomic_load((global_u32 *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until this wave's outstanding vector-memory operations (including coherent stores)
// have completed, so that a flag written afterwards is observed after them.
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// ------------------------------------------------------------------------------------
// Reductions
// ------------------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// ------------------------------------------------------------------------------------
// Grid barrier and abort flag
// ------------------------------------------------------------------------------------
struct GridSync {
  uint32_t *flags;   // [gridDim.x], zero at launch
  uint32_t *abort;   // [1], zero at launch
  uint32_t epoch;    // barriers passed by this workgroup
};

// All workgroups of the (co-resident) grid meet here.  Returns false if the launch was
// aborted (a wait exceeded its bound here or elsewhere).
__device__ __forceinline__ bool grid_sync(GridSync &gs) {
  __shared__ int s_ok;
  wait_vmem();
  __syncthreads();
  gs.epoch++;
  if (threadIdx.x < 64) {
    if (threadIdx.x == 0) st_coh32(&gs.flags[blockIdx.x], gs.epoch);
    const int G = (int)gridDim.x;
    int ok = 1;
    uint64_t spins = 0;
    while (true) {
      bool mine = true;
      for (int i = (int)threadIdx.x; i < G; i += 64) mine &= (ld_coh32(&gs.flags[i]) >= gs.epoch);
      if (__all(mine)) break;
      if (ld_coh32(gs.abort) != 0u) { ok = 0; break; }
      if (++spins > kSpinLimit) {
        if (threadIdx.x == 0) st_coh32(gs.abort, 1u);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (threadIdx.x == 0) s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Sum of one float64 value per workgroup over the whole grid, identical in every
// workgroup (fixed order).  `slots` is [gridDim.x]; a grid_sync separates the writes from
// the reads.  Call with the same `slots` only after another grid_sync.
__device__ __forceinline__ double grid_sum_read(const double *slots) {
  __shared__ double s_res;
  if (threadIdx.x < 64) {
    double acc = 0.0;
    for (int i = (int)threadIdx.x; i < (int)gridDim.x; i += 64) acc += ld_coh(&slots[i]);
    acc = wave_sum(acc);
    if (threadIdx.x == 0) s_res = acc;
  }
  __syncthreads();
  double r = s_res;
  __syncthreads();
  return r;
}

// Workgroup-wide sum of one float64 per thread (blockDim.x a multiple of 64, <= 1024).
__device__ __forceinline__ double block_sum(double x) {
  __shared__ double s_part[16];
  __shared__ double s_tot;
  x = wave_sum(x);
  const int wave = (int)threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) s_part[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s_part[w];
    s_tot = t;
  }
  __syncthreads();
  double r = s_tot;
  __syncthreads();
  return r;
}

}  // namespace sr
