// Fused one-read product with the centred sampled overlap (and the linear-method
// Hamiltonian), Sec. II.A Eq. sr_multiply_2 and Sec. II.B Eq. linear_eigen.
//
// For each sample row k the method needs the scalar w_k = Oc_k . v before the row can be
// accumulated into y = sum_k w_k Oc_k.  A row is kept in registers between the two uses,
// so O is read from HBM exactly once per product:
//
//   * The grid (one workgroup of 256 threads per CU, all co-resident) is split into
//     RG row groups x C column groups.  Column group cg owns a slice of `wslice` columns;
//     row group rg owns row tiles rg, rg+RG, rg+2RG, ... of R rows each.
//   * Each thread owns NV 16-byte vectors of its slice (coalesced across the workgroup)
//     and keeps v (times the column scale) and its y accumulators in registers.
//   * Tile j: load -> partial dots (wave shuffles, then LDS across waves) -> if C > 1,
//     publish the partial dots as tagged 64-bit words and read the other C-1 column
//     groups' words one pipeline step later -> w -> y += w * tile.  NB tile buffers are
//     in flight so HBM streaming continues while the exchange completes.
//   * Centering is folded in: each column group subtracts its share of obar . v from its
//     partial dot, and the final y uses y_i = s_i (O^T w)_i - obar_i sum_k w_k.
//   * Row-group partial y vectors (float64) go to a workspace; a grid barrier later lets
//     any workgroup finish a column range with a fixed-order sum over row groups.
#pragma once
#include "sr_device.hpp"

namespace sr {

constexpr int kNT = 256;            // threads per workgroup (4 waves)
constexpr int kNW = kNT / 64;       // waves per workgroup
constexpr int kRing = 4;            // exchange slots per row group (>= 3 needed)

struct ProdGeom {
  int G, C, RG;                     // grid size, column groups, row groups (G = C*RG)
  int n_tiles;                      // ceil(n_s / R)
  int64_t n_s, n_p, wslice;         // wslice: columns per column group, multiple of VEC
};

struct ProdBufs {
  double *ypart;                    // [RG][n_p]   row-group partial O^T w
  double *spart;                    // [RG][2]     row-group scalars
  u64 *xchg;                        // [RG][kRing][C][words]
};

struct WgCtx {
  int rg, cg;
  int64_t c0, c1;                   // owned column slice [c0, c1)
  uint32_t xstep;                   // exchange steps performed in this launch
  GridSync gs;
};

// Workgroup -> (row group, column group).  Workgroup b runs on XCD b % 8 (round-robin
// dispatch); the column groups of one row group are placed on as few XCDs as possible so
// their exchanges stay local when they can.  Requires G % 8 == 0 and C | G/8 or G/8 | C.
__device__ __forceinline__ void map_workgroup(int b, int G, int C, int &rg, int &cg) {
  const int L = G / 8;
  const int xcd = b % 8, local = b / 8;
  if (C <= L) {
    rg = xcd * (L / C) + local / C;
    cg = local % C;
  } else {
    const int xpg = C / L;
    rg = xcd / xpg;
    cg = (xcd % xpg) * L + local;
  }
}

__device__ __forceinline__ void init_ctx(WgCtx &ctx, const ProdGeom &pg, uint32_t *flags, uint32_t *abort,
                                         int vec) {
  map_workgroup((int)blockIdx.x, pg.G, pg.C, ctx.rg, ctx.cg);
  ctx.c0 = (int64_t)ctx.cg * pg.wslice;
  ctx.c1 = ctx.c0 + pg.wslice;
  if (ctx.c1 > pg.n_p) ctx.c1 = pg.n_p;
  if (ctx.c0 > pg.n_p) ctx.c0 = pg.n_p;
  ctx.xstep = 0;
  ctx.gs.flags = flags;
  ctx.gs.abort = abort;
  ctx.gs.epoch = 0;
  (void)vec;
}

// One matrix operand of the product.
struct Operand {
  const unsigned char *O;           // base pointer
  int64_t ldb;                      // row stride in bytes
  const float *scale;               // per-column scale (scaled storage) or nullptr
};

// Accumulation type of a product: the storage type's own, or float64 when EXACT (used
// for the residual products of scaled storage, so that the residual is that of the
// stored matrix to float64 accuracy).
template <int DT, bool EXACT> struct AccOf { typedef typename Storage<DT>::acc_t type; };
template <int DT> struct AccOf<DT, true> { typedef double type; };

// NDOT = 1: SR overlap product.  NDOT = 2: linear-method product (second operand D is
// only dotted, never accumulated).
template <int DT, int NV, int R, int NB, int NDOT, bool EXACT = false>
struct Product {
  typedef Storage<DT> St;
  typedef typename AccOf<DT, EXACT>::type acc_t;
  static constexpr int VEC = St::VEC;
  static constexpr int WPD = sizeof(acc_t) == 8 ? 2 : 1;   // exchange words per partial dot
  // exchange words per column group per tile; the ring is laid out for float64 partials
  // so that float32 and float64 products of the same launch can share it
  static constexpr int WORDS = NDOT * R * 2;

  // --- per-thread state ---
  int64_t colv[NV];                 // first column of each owned vector, or -1
  u32x4 msk[NV];                    // element mask (vector straddling n_p)
  acc_t vc[NDOT][NV][VEC];          // v_j * s_j per operand (0 outside the slice)
  acc_t yacc[NV][VEC];              // partial (O^T w)_j
  u32x4 buf[NB][NDOT][R][NV];       // row-tile buffers
  double s1, s2;                    // row-group scalars (SR: sum w; LM: sum z, sum(E t + u))
  bool need_mask;

  __device__ __forceinline__ static u32x4 elem_mask(int nvalid) {
    // keep the bytes of the first nvalid elements of a 16-byte vector
    u32x4 m;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int first_byte = w * 4;
      const int valid_bytes = nvalid * St::BYTES;
      uint32_t mw;
      if (valid_bytes >= first_byte + 4) mw = 0xFFFFFFFFu;
      else if (valid_bytes <= first_byte) mw = 0u;
      else mw = 0xFFFFFFFFu >> (8 * (first_byte + 4 - valid_bytes));
      m[w] = mw;
    }
    return m;
  }

  // Load the owned coefficients; returns this workgroup's share of obar . v (operand 0).
  __device__ __forceinline__ double setup(const WgCtx &ctx, const ProdGeom &pg, const Operand *ops,
                                          const double *__restrict__ mean, const double *v) {
    const int tid = (int)threadIdx.x;
    double cpart = 0.0;
    need_mask = false;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int64_t col = ctx.c0 + ((int64_t)i * kNT + tid) * VEC;
      colv[i] = (col < ctx.c1) ? col : -1;
      int nvalid = 0;
      if (colv[i] >= 0) {
        const int64_t rem = pg.n_p - col;
        nvalid = rem >= VEC ? VEC : (int)rem;
      }
      msk[i] = elem_mask(nvalid);
      if (colv[i] >= 0 && nvalid < VEC) need_mask = true;
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        double vj = 0.0;
        if (e < nvalid) {
          vj = ld_coh(&v[col + e]);
          cpart += mean[col + e] * vj;
        }
#pragma unroll
        for (int d = 0; d < NDOT; ++d) {
          double s = 1.0;
          if (ops[d].scale != nullptr && e < nvalid) s = (double)ops[d].scale[col + e];
          vc[d][i][e] = (acc_t)(vj * s);
        }
        yacc[i][e] = (acc_t)0;
      }
    }
    s1 = 0.0;
    s2 = 0.0;
    // need_mask is per thread; make it uniform (any thread) so branches stay uniform
    need_mask = __syncthreads_or(need_mask ? 1 : 0) != 0;
    return block_sum(cpart);
  }

  template <int B>
  __device__ __forceinline__ void issue(const WgCtx &ctx, const ProdGeom &pg, const Operand *ops, int j) {
    const int64_t row0 = ((int64_t)j * pg.RG + ctx.rg) * R;
#pragma unroll
    for (int d = 0; d < NDOT; ++d)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t row = row0 + r;
        const unsigned char *rowp = ops[d].O + row * ops[d].ldb;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          if (row < pg.n_s && colv[i] >= 0) buf[B][d][r][i] = load_stream(rowp + colv[i] * St::BYTES);
          else buf[B][d][r][i] = u32x4{0u, 0u, 0u, 0u};
        }
      }
  }

  template <int B>
  __device__ __forceinline__ void dots(acc_t (&part)[NDOT][R]) {
#pragma unroll
    for (int d = 0; d < NDOT; ++d)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc_t acc = (acc_t)0;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          u32x4 x = buf[B][d][r][i];
          if (need_mask) x &= msk[i];
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc += (acc_t)St::get(x, e) * vc[d][i][e];
        }
        part[d][r] = acc;
      }
  }

  // Workgroup reduction of the per-thread partial dots; result (minus the centering share
  // for operand 0) in s_red[d][r] (float64, LDS) for every thread.
  __device__ __forceinline__ void reduce(acc_t (&part)[NDOT][R], double cshare, double (&s_red)[NDOT][R],
                                         double (&s_wave)[kNW][NDOT][R]) {
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
#pragma unroll
    for (int d = 0; d < NDOT; ++d)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc_t s = wave_sum(part[d][r]);
        if (lane == 0) s_wave[wave][d][r] = (double)s;
      }
    __syncthreads();
    if (threadIdx.x < NDOT * R) {
      const int d = (int)threadIdx.x / R, r = (int)threadIdx.x % R;
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kNW; ++w) t += s_wave[w][d][r];
      if (d == 0) t -= cshare;
      s_red[d][r] = t;
    }
    __syncthreads();
  }

  __device__ __forceinline__ u64 *slot_base(const ProdBufs &pb, const ProdGeom &pg, const WgCtx &ctx,
                                             uint32_t step) const {
    const int slot = (int)(step % kRing);
    return pb.xchg + (((int64_t)ctx.rg * kRing + slot) * pg.C) * WORDS;
  }

  __device__ __forceinline__ void publish(const ProdBufs &pb, const ProdGeom &pg, const WgCtx &ctx, uint32_t step,
                                          const double (&s_red)[NDOT][R]) {
    u64 *base = slot_base(pb, pg, ctx, step) + (int64_t)ctx.cg * WORDS;
    const u64 tag = (u64)(step / kRing + 1) << 32;
    if (threadIdx.x < NDOT * R) {
      const int d = (int)threadIdx.x / R, r = (int)threadIdx.x % R;
      const double val = s_red[d][r];
      if (WPD == 1) {
        const float f = (float)val;
        st_coh64(&base[d * R + r], tag | (u64)__float_as_uint(f));
      } else {
        const u64 b = (u64)__double_as_longlong(val);
        st_coh64(&base[(d * R + r) * 2 + 0], tag | (b & 0xFFFFFFFFull));
        st_coh64(&base[(d * R + r) * 2 + 1], tag | (b >> 32));
      }
    }
  }

  // Wait for all C column groups' words of `step` and sum them (fixed order, identical in
  // every column group).  Result in s_tot[d][r].  Returns false on abort.
  __device__ __forceinline__ bool collect(const ProdBufs &pb, const ProdGeom &pg, const WgCtx &ctx, uint32_t step,
                                          double (&s_tot)[NDOT][R]) {
    __shared__ int s_ok;
    if (threadIdx.x < 64) {
      const u64 *base = slot_base(pb, pg, ctx, step);
      const uint32_t tag = step / kRing + 1;
      const int lane = (int)threadIdx.x;
      double acc[NDOT][R];
      int ok = 1;
      uint64_t spins = 0;
      while (true) {
        bool mine = true;
#pragma unroll
        for (int d = 0; d < NDOT; ++d)
#pragma unroll
          for (int r = 0; r < R; ++r) acc[d][r] = 0.0;
        for (int c = lane; c < pg.C; c += 64) {
          const u64 *wp = base + (int64_t)c * WORDS;
#pragma unroll
          for (int d = 0; d < NDOT; ++d)
#pragma unroll
            for (int r = 0; r < R; ++r) {
              if (WPD == 1) {
                const u64 w = ld_coh64(&wp[d * R + r]);
                mine &= ((uint32_t)(w >> 32) == tag);
                acc[d][r] += (double)__uint_as_float((uint32_t)w);
              } else {
                const u64 lo = ld_coh64(&wp[(d * R + r) * 2 + 0]);
                const u64 hi = ld_coh64(&wp[(d * R + r) * 2 + 1]);
                mine &= ((uint32_t)(lo >> 32) == tag) && ((uint32_t)(hi >> 32) == tag);
                acc[d][r] += __longlong_as_double((long long)((hi << 32) | (lo & 0xFFFFFFFFull)));
              }
            }
        }
        if (__all(mine)) break;
        if (++spins > kSpinLimit || ((spins & 255) == 0 && ld_coh32(ctx.gs.abort) != 0u)) {
          if (lane == 0) st_coh32(ctx.gs.abort, 1u);
          ok = 0;
          break;
        }
      }
#pragma unroll
      for (int d = 0; d < NDOT; ++d)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double t = wave_sum(acc[d][r]);
          if (lane == 0) s_tot[d][r] = t;
        }
      if (lane == 0) s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
  }

  // y += w * tile for tile j held in buffer B.
  template <int B>
  __device__ __forceinline__ void update(const ProdGeom &pg, const WgCtx &ctx, int j, const double (&tot)[NDOT][R],
                                         const double *__restrict__ E, double v0) {
    const int64_t row0 = ((int64_t)j * pg.RG + ctx.rg) * R;
    acc_t w[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = row0 + r;
      double wr = 0.0;
      if (row < pg.n_s) {
        if (NDOT == 1) {
          wr = tot[0][r];
          s1 += wr;
        } else {
          const double t = tot[0][r], u = tot[1][r];
          const double e = E[row];
          wr = e * (v0 + t) + u;
          s1 += wr;
          s2 += e * t + u;
        }
      }
      w[r] = (acc_t)wr;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        u32x4 x = buf[B][0][r][i];
        if (need_mask) x &= msk[i];
#pragma unroll
        for (int e = 0; e < VEC; ++e) yacc[i][e] += (acc_t)St::get(x, e) * w[r];
      }
    }
  }

  // One pipeline step for local tile j (buffer B = j % NB).
  template <int B>
  __device__ __forceinline__ bool step(const ProdGeom &pg, const ProdBufs &pb, WgCtx &ctx, const Operand *ops,
                                       int j, int n_my, double cshare, const double *__restrict__ E, double v0,
                                       double (&s_red)[NDOT][R], double (&s_wave)[kNW][NDOT][R],
                                       double (&s_tot)[NDOT][R]) {
    constexpr int BP = (B + NB - 1) % NB;   // buffer of tile j-1
    if (pg.C == 1) {
      if (j < n_my) {
        acc_t part[NDOT][R];
        dots<B>(part);
        reduce(part, cshare, s_red, s_wave);
        update<B>(pg, ctx, j, s_red, E, v0);
        if (j + NB < n_my) issue<B>(ctx, pg, ops, j + NB);
      }
      return true;
    }
    if (j < n_my) {
      acc_t part[NDOT][R];
      dots<B>(part);
      reduce(part, cshare, s_red, s_wave);
      publish(pb, pg, ctx, ctx.xstep + (uint32_t)j, s_red);
    }
    if (j >= 1 && j - 1 < n_my) {
      if (!collect(pb, pg, ctx, ctx.xstep + (uint32_t)(j - 1), s_tot)) return false;
      update<BP>(pg, ctx, j - 1, s_tot, E, v0);
      __syncthreads();   // s_tot is rewritten by the next collect
    }
    if (j - 1 + NB < n_my) issue<BP>(ctx, pg, ops, j - 1 + NB);
    return true;
  }

  // Accumulate this workgroup's share of O^T w over its row group's tiles.
  __device__ __forceinline__ bool accumulate(const ProdGeom &pg, const ProdBufs &pb, WgCtx &ctx, const Operand *ops,
                                             double cshare, const double *__restrict__ E, double v0) {
    __shared__ double s_red[NDOT][R];
    __shared__ double s_wave[kNW][NDOT][R];
    __shared__ double s_tot[NDOT][R];
    const int n_my = (ctx.rg < pg.n_tiles) ? (pg.n_tiles - ctx.rg + pg.RG - 1) / pg.RG : 0;
    const int pre = (pg.C == 1) ? NB : NB - 1;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b < pre && b < n_my) {
        if (b == 0) issue<0>(ctx, pg, ops, 0);
        if (NB > 1 && b == 1) issue<(1 % NB)>(ctx, pg, ops, 1);
        if (NB > 2 && b == 2) issue<(2 % NB)>(ctx, pg, ops, 2);
        if (NB > 3 && b == 3) issue<(3 % NB)>(ctx, pg, ops, 3);
      }
    }
    const int last = (pg.C == 1) ? n_my : n_my + 1;   // exclusive bound of steps
    bool ok = true;
    for (int j0 = 0; j0 < last && ok; j0 += NB) {
      ok = step<0>(pg, pb, ctx, ops, j0, n_my, cshare, E, v0, s_red, s_wave, s_tot);
      if (NB > 1 && ok && j0 + 1 < last)
        ok = step<(1 % NB)>(pg, pb, ctx, ops, j0 + 1, n_my, cshare, E, v0, s_red, s_wave, s_tot);
      if (NB > 2 && ok && j0 + 2 < last)
        ok = step<(2 % NB)>(pg, pb, ctx, ops, j0 + 2, n_my, cshare, E, v0, s_red, s_wave, s_tot);
      if (NB > 3 && ok && j0 + 3 < last)
        ok = step<(3 % NB)>(pg, pb, ctx, ops, j0 + 3, n_my, cshare, E, v0, s_red, s_wave, s_tot);
    }
    ctx.xstep += (uint32_t)n_my;
    return ok;
  }

  // Store the row group's partial y (float64) and scalars, coherently.
  __device__ __forceinline__ void store_partials(const ProdGeom &pg, const ProdBufs &pb, const WgCtx &ctx) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      if (colv[i] < 0) continue;
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int64_t col = colv[i] + e;
        if (col < pg.n_p) st_coh(&pb.ypart[(int64_t)ctx.rg * pg.n_p + col], (double)yacc[i][e]);
      }
    }
    if (ctx.cg == 0 && threadIdx.x == 0) {
      st_coh(&pb.spart[ctx.rg * 2 + 0], s1);
      st_coh(&pb.spart[ctx.rg * 2 + 1], s2);
    }
  }
};

// Column j of the finished product: (s_j * sum_rg ypart[rg][j] - mean_j * S1) with
// S1 = sum_rg spart[rg][0]; a fixed summation order over row groups.
__device__ __forceinline__ double finish_column(const ProdBufs &pb, const ProdGeom &pg, int64_t j) {
  double acc = 0.0;
  for (int rg = 0; rg < pg.RG; ++rg) acc += ld_coh(&pb.ypart[(int64_t)rg * pg.n_p + j]);
  return acc;
}

__device__ __forceinline__ void sum_row_scalars(const ProdBufs &pb, const ProdGeom &pg, double &S1, double &S2) {
  __shared__ double s_s[2];
  if (threadIdx.x < 64) {
    double a = 0.0, b = 0.0;
    for (int rg = (int)threadIdx.x; rg < pg.RG; rg += 64) {
      a += ld_coh(&pb.spart[rg * 2 + 0]);
      b += ld_coh(&pb.spart[rg * 2 + 1]);
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (threadIdx.x == 0) { s_s[0] = a; s_s[1] = b; }
  }
  __syncthreads();
  S1 = s_s[0];
  S2 = s_s[1];
  __syncthreads();
}

}  // namespace sr
