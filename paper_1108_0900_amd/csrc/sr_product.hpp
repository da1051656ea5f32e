// Fused one-read product with the centred sampled overlap (and the linear-method
// Hamiltonian), Sec. II.A Eq. sr_multiply_2 and Sec. II.B Eq. linear_eigen.
//
// For each sample row k the method needs the scalar w_k = Oc_k . v before the row can be
// accumulated into y = sum_k w_k Oc_k.  A row tile stays on chip between the two uses, so
// O is read from HBM exactly once per product:
//
//   * The grid (one workgroup per CU, all co-resident; NT = 256 or 512 threads, i.e. one
//     or two waves per SIMD) is split into RG row groups x C column groups.  Column group cg owns a slice of `wslice` columns; row group rg owns
//     row tiles rg, rg+RG, rg+2RG, ... of R rows each.
//   * Each thread of the workgroup (NT threads) owns NV 16-byte vectors of the slice
//     (coalesced across the workgroup) and keeps v (times the column scale) and its y accumulators
//     in registers.
//   * Row tiles stay in a ring of registers from their load (LOOK steps ahead) until they
//     are accumulated LAG steps after their dots, so each tile is read from HBM once.
//     Step t: issue the loads of tile t+LOOK; partial dots of tile t (wave shuffles, then
//     LDS); accumulate tile t-LAG with the row weights w delivered by the exchange.  One
//     barrier per step.  Every load is unconditional, so the compiler waits for exactly
//     the tile a step consumes and leaves the later ones in flight.
//   * Wave 0 also runs the exchange: after barrier t it combines the waves' partials and,
//     with C > 1, publishes them as tagged 64-bit words.  The other column groups' words
//     of step e are loaded at the start of step e+ADV (before that step's tile loads, so
//     the in-order completion counter never makes the poll wait for newer tiles) and
//     checked at the end of step e+ADV+1: the round trip through the coherent memory
//     level overlaps more than a step of streaming.
//   * Centering is folded in: each column group subtracts its share of obar . v from its
//     partial dot, and the final y uses y_i = s_i (O^T w)_i - obar_i sum_k w_k.
//   * Row-group partial y vectors (float64) go to a workspace; a grid barrier later lets
//     any workgroup finish a column range with a fixed-order sum over row groups.
#pragma once
#include <utility>
#include "sr_device.hpp"

namespace sr {

constexpr int kNT = 256;            // workgroup size of the column-statistics kernels
constexpr int kRing = 16;           // exchange slots per row group (> 2 * poll delay + 1)

struct ProdGeom {
  int G, C, RG;                     // grid size, column groups, row groups (C*RG <= G: the
                                    // workgroups past them, if any, are idle in products)
  int n_tiles;                      // ceil(n_s / R)
  int64_t n_s, n_p, wslice;         // wslice: columns per column group, multiple of VEC
  int64_t n_v;                      // streamed columns: n_p, or with a compact remainder
                                    // plane n_q + n_lo (see Operand)
};

struct ProdBufs {
  double *ypart;                    // [RG][n_v]   row-group partial O^T w
  double *spart;                    // [RG][2]     row-group scalars
  u64 *xchg;                        // [RG][kRing][C][words]
  u64 *sink;                        // [G][words]  target of the tail steps' publishes
};

struct WgCtx {
  int rg, cg;
  int64_t c0, c1;                   // owned column slice [c0, c1)
  uint32_t xstep;                   // exchange steps performed in this launch
  GridSync gs;
};

// Workgroup -> (row group, column group).  Workgroup b runs on XCD b % 8 (round-robin
// dispatch); the column groups of one row group are placed on as few XCDs as possible so
// their exchanges stay local when they can.  Requires G % 8 == 0 and C <= G/8 (then each
// XCD holds (G/8)/C row groups, RG = 8 (G/8)/C, and an XCD's workgroups past them get
// rg = G: idle) or G/8 | C (RG = G/C).
__device__ __forceinline__ void map_workgroup(int b, int G, int C, int &rg, int &cg) {
  const int L = G / 8;
  const int xcd = b % 8, local = b / 8;
  if (C <= L) {
    const int per = L / C;
    if (local < per * C) {
      rg = xcd * per + local / C;
      cg = local % C;
    } else {
      rg = G;
      cg = 0;
    }
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
  if (ctx.c1 > pg.n_v) ctx.c1 = pg.n_v;
  if (ctx.c0 > pg.n_v) ctx.c0 = pg.n_v;
  ctx.xstep = 0;
  ctx.gs.flags = flags;
  ctx.gs.abort = abort;
  ctx.gs.epoch = 0;
  (void)vec;
}

// One matrix operand of the product.
//
// Compact remainder plane (scaled storage, lo_cols != nullptr): only the columns
// lo_cols[0..n_lo) (strictly increasing parameter indices) carry a second code, stored as
// their own matrix `lo` with row stride ldb_lo.  The single-plane product streams it as n_lo
// extra columns after the first plane: streamed column c < n_q is parameter c of the first
// plane (n_q = n_p rounded up to whole 16-byte vectors, so no vector spans both), column
// n_q + i is remainder column i, whose coefficient is that of parameter lo_cols[i] and whose
// partial (O^T w) is added to that parameter's when the product is finished.
struct Operand {
  const unsigned char *O;           // base pointer
  const unsigned char *lo;          // second code plane (same layout, PLANES = 2), the
                                    // compact remainder plane (lo_cols given), or nullptr
  int64_t ldb;                      // row stride in bytes
  const float *scale;               // per-column scale (scaled storage) or nullptr
  const int32_t *lo_cols;           // compact remainder plane: parameter of each column
  int64_t n_lo, ldb_lo;             // its columns and row stride in bytes
  int64_t n_q;                      // first streamed column of the compact plane; with no
                                    // compact plane larger than any column
};

// Parameter of compact remainder column i, kept inside [0, n_p) whatever the list holds.
__device__ __forceinline__ int64_t lo_param(const int32_t *L, int64_t i, int64_t n_p) {
  const int64_t j = L[i];
  return j < 0 ? 0 : (j >= n_p ? n_p - 1 : j);
}

// First index i in [0, n) with L[i] >= key (L increasing), or n; every lane of the calling
// wave gets the result.  64-way search: a few rounds of one load per lane.
__device__ __forceinline__ int64_t lower_bound_wave(const int32_t *L, int64_t n, int64_t key) {
  const int lane = (int)threadIdx.x & 63;
  int64_t lo = 0, hi = n;           // every index < lo has L < key, every index >= hi has L >= key
  while (hi - lo > 64) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t pos = lo + (int64_t)lane * step;
    const bool less = pos < hi && (int64_t)L[pos] < key;
    const int c = __popcll(__ballot(less));
    if (c == 0) return lo;
    const int64_t nhi = lo + (int64_t)c * step;
    lo = lo + (int64_t)(c - 1) * step + 1;
    hi = nhi < hi ? nhi : hi;
  }
  const int64_t pos = lo + lane;
  const bool less = pos < hi && (int64_t)L[pos] < key;
  return lo + __popcll(__ballot(less));
}

// Accumulation type of a product: the storage type's own, or float64 when EXACT (used
// for the residual products of scaled storage, so that the residual is that of the
// stored matrix to float64 accuracy).
template <int DT, bool EXACT> struct AccOf { typedef typename Storage<DT>::acc_t type; };
template <int DT> struct AccOf<DT, true> { typedef double type; };

// bf16 bits of a float, rounded to nearest even (finite inputs).
__device__ __forceinline__ uint32_t bf16_rne(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}
// c + a.lo * b.lo + a.hi * b.hi for two packed bf16 pairs, float32 accumulation.
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2_t;
__device__ __forceinline__ float dot2_bf16(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a), __builtin_bit_cast(bf16x2_t, b), c, false);
}

// NDOT = 1: SR overlap product.  NDOT = 2: linear-method product (second operand D is
// only dotted, never accumulated).
//   NV    16-byte vectors per thread and row (slice width NV*VEC*NT columns)
//   R     rows per tile
//   LOOK  tiles whose loads are in flight ahead of the one being consumed
//   PD    poll depth: the other column groups' partial dots of tile t are loaded at the
//         start of step t + kAdv and used at the end of step t + kAdv + PD, so PD steps of
//         streaming cover the latency of those coherent loads
//   NT    threads per workgroup
//   PLANES 2: the operand is s_j (q + lo) read from two code planes (NDOT = 1 only)
template <int DT, int NV, int R, int NDOT, bool EXACT = false, int LOOK = 2, int PD = 1, int NT = 256,
          int PLANES = 1>
struct Product {
  static_assert(PLANES == 1 || NDOT == 1, "two code planes only for the SR product");
  static constexpr int NOPS = NDOT + PLANES - 1;   // loaded tiles per row (operands, planes)
  // the single-plane SR product of scaled storage can stream a compact remainder plane
  static constexpr bool kCompact = PLANES == 1 && NDOT == 1 && Storage<DT>::BYTES == 2;
  static constexpr int NW = NT / 64;          // waves per workgroup
  static constexpr int kLook = LOOK;
  // the poll of tile t starts at step t + kAdv (PD = 0: one step later, finished in the
  // same step; the tile is accumulated at the same step either way)
  static constexpr int kAdv = PD == 0 ? 3 : 2;
  static constexpr int kPD = PD;
  static constexpr int kNPoll = PD + 1;       // poll buffers in flight
  static constexpr int kLag = kAdv + PD + 1;  // tile t is accumulated at step t + kLag
  // register ring: a tile lives from step t-LOOK to t+kLag; its size is a multiple of the
  // number of poll buffers so that both rings are indexed at compile time
  static constexpr int kNBuf = ((LOOK + kLag + 1) + kNPoll - 1) / kNPoll * kNPoll;
  static_assert(PD >= 0, "poll depth");
  // A workgroup at step t has seen every member of its row group publish step
  // t - 1 - kAdv - PD, so each member is at step >= t - kAdv - PD and may still be
  // (re)reading step t - 2 (kAdv + PD).  Those slots must stay distinct from the one
  // step t publishes to.
  static_assert(kRing > 2 * (kAdv + PD), "exchange ring too small for the poll depth");
  typedef Storage<DT> St;
  typedef typename AccOf<DT, EXACT>::type acc_t;
  static constexpr int VEC = St::VEC;
  static constexpr int WPD = sizeof(acc_t) == 8 ? 2 : 1;   // exchange words per partial dot
  // exchange words per column group per tile; the ring is laid out for float64 partials
  // so that float32 and float64 products of the same launch can share it
  static constexpr int WORDS = NDOT * R * 2;
  static constexpr int PW = NDOT * R * WPD;                  // polled words per column group

  // --- per-thread state (data threads) ---
  int col0;                         // first streamed column of vector 0; vector i starts at col0 + i*NT*VEC
  int nvec;                         // owned vectors that start inside the slice (0..NV)
  int n_p;                          // parameters (for the mask of a vector straddling n_p)
  int n_q, n_qe;                    // streamed columns [n_q, n_qe) are the compact remainder
                                    // plane's (n_q = n_qe = 2^31 - 1 without one)
  acc_t vc[NDOT][NV][VEC];          // v_j * s_j per operand (0 outside the slice)
  // bf16 codes, float32 accumulation: the row dots run as packed bf16 pair products
  // (v_dot2 with float32 accumulation), v_j s_j split into a bf16 high part and a bf16
  // remainder (words 0-3: the high parts of element pairs 2w, 2w+1; words 4-7: the
  // remainders), which keeps about 16 significant bits of each coefficient
  static constexpr bool kDot2 = DT == DT_BF16 && !EXACT && PLANES == 1;
  uint32_t vp[NDOT][NV][VEC];
  acc_t yacc[NV][VEC];              // partial (O^T w)_j
  u32x4 buf[kNBuf][NOPS][R][NV];    // register ring of row tiles
  double s1, s2;                    // row-group scalars (SR: sum w; LM: sum z, sum(E t + u))
  bool need_mask;
  int mcode;                        // straddling vectors, one byte each: index * 8 + valid elements
                                    // (NV * 8: none); at most two (the ends of the two planes)
  // --- exchange state (wave 0) ---
  static constexpr int kCh = 2;     // column groups per lane read ahead (C <= 128 asynchronously)
  u64 pw[kNPoll][kCh][PW];          // words of column groups lane, lane + 64 for the pending polls
  double cshare;

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

  __device__ __forceinline__ int64_t colv(int i) const { return (int64_t)col0 + (int64_t)i * (NT * VEC); }

  // Valid elements of the 16-byte vector starting at streamed column c (0..VEC).
  __device__ __forceinline__ int valid_of(int64_t c) const {
    const int64_t end = c < n_q ? (int64_t)n_p : (int64_t)n_qe;
    const int64_t nv = end - c;
    return nv < 0 ? 0 : (nv > VEC ? VEC : (int)nv);
  }

  // Load the owned coefficients; returns this workgroup's share of obar . v (operand 0).
  __device__ __forceinline__ double setup(const WgCtx &ctx, const ProdGeom &pg, const Operand *ops,
                                          const double *__restrict__ mean, const double *v) {
    const int tid = (int)threadIdx.x;
    const bool data = true;
    double cpart = 0.0;
    col0 = (int)(ctx.c0 + (int64_t)tid * VEC);
    nvec = 0;
    n_p = (int)pg.n_p;
    const bool compact = kCompact && ops[0].lo_cols != nullptr;
    n_q = compact ? (int)ops[0].n_q : 0x7fffffff;
    n_qe = compact ? (int)(ops[0].n_q + ops[0].n_lo) : 0x7fffffff;
    bool straddles = false;
    mcode = NV * 8 * 0x101;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int64_t col = colv(i);
      const bool in = data && col < ctx.c1;
      int nvalid = 0;
      if (in) {
        nvec = i + 1;
        nvalid = valid_of(col);
        if (nvalid < VEC) {
          // the first straddling vector goes to byte 0, a second one (past n_q) to byte 1
          mcode = straddles ? (mcode & 0xFF) | ((i * 8 + nvalid) << 8) : (mcode & 0xFF00) | (i * 8 + nvalid);
          straddles = true;
        }
      }
      const bool lo = col >= n_q;     // a vector of the compact remainder plane
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        // parameter of streamed column col + e
        int64_t j = col + e;
        if (lo && e < nvalid) j = lo_param(ops[0].lo_cols, col - n_q + e, pg.n_p);
        double vj = 0.0;
        if (e < nvalid) {
          vj = ld_coh(&v[j]);
          if (!lo) cpart += mean[j] * vj;
        }
#pragma unroll
        for (int d = 0; d < NDOT; ++d) {
          double s = 1.0;
          if (ops[d].scale != nullptr && e < nvalid) s = (double)ops[d].scale[j];
          vc[d][i][e] = (acc_t)(vj * s);
        }
        yacc[i][e] = (acc_t)0;
      }
      if constexpr (kDot2) {
#pragma unroll
        for (int d = 0; d < NDOT; ++d)
#pragma unroll
          for (int w = 0; w < VEC / 2; ++w) {
            uint32_t hi[2], lo[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const float f = (float)vc[d][i][2 * w + h];
              hi[h] = bf16_rne(f);
              lo[h] = bf16_rne(f - __uint_as_float(hi[h] << 16));   // f - hi is exact
            }
            vp[d][i][w] = hi[0] | (hi[1] << 16);
            vp[d][i][VEC / 2 + w] = lo[0] | (lo[1] << 16);
          }
      }
    }
    s1 = 0.0;
    s2 = 0.0;
    // uniform flag: does any thread own a straddling vector?
    need_mask = __syncthreads_or(straddles ? 1 : 0) != 0;
    cshare = block_sum(cpart);
    return cshare;
  }

  // Loads of tile j into buffer B.  Every load is issued unconditionally (rows past n_s
  // and vectors past the slice read a valid address of the same matrix instead, and
  // their row weights / coefficients are zero), so the compiler can wait for exactly the
  // loads a step needs and leave the later tiles in flight.
  template <int B>
  __device__ __forceinline__ void issue(const WgCtx &ctx, const ProdGeom &pg, const Operand *ops, int j) {
    const int64_t row0 = ((int64_t)j * pg.RG + ctx.rg) * R;
#pragma unroll
    for (int d = 0; d < NOPS; ++d)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int64_t row = row0 + r;
        row = row < pg.n_s ? row : pg.n_s - 1;
        const Operand &op = ops[PLANES == 2 ? 0 : d];
        const unsigned char *base = (PLANES == 2 && d == 1) ? op.lo : op.O;
        const unsigned char *rowp = base + row * op.ldb;
        // the compact remainder plane's row (its vectors are selected per thread)
        const unsigned char *rowl = kCompact ? op.lo + row * op.ldb_lo : rowp;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          const int64_t col = i < nvec ? colv(i) : 0;
          // one load either way (the address is selected), so no load sits in a branch
          const bool lo = kCompact && col >= n_q;
          buf[B][d][r][i] = load_stream(lo ? rowl + (col - n_q) * St::BYTES : rowp + col * St::BYTES);
        }
      }
  }

  template <int B>
  __device__ __forceinline__ void dots(acc_t (&part)[NDOT][R]) {
    if (need_mask) {
      // zero the bytes past the end of a plane's columns (row padding may hold anything)
      // before any use.  A thread has at most two straddling vectors, one at the end of
      // each plane (vectors outside the slice read valid columns with zero coefficients);
      // their masks are rebuilt per tile from one packed code, kept opaque so that the
      // compiler does not hoist NV masks out of the streaming loop
      int code = mcode;
      asm volatile("" : "+v"(code));
      const u32x4 ma = elem_mask(code & 7), mb = elem_mask((code >> 8) & 7);
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const bool ha = ((code >> 3) & 31) == i, hb = ((code >> 11) & 31) == i;
        u32x4 mi;
#pragma unroll
        for (int w = 0; w < 4; ++w) mi[w] = ha ? ma[w] : (hb ? mb[w] : 0xFFFFFFFFu);
#pragma unroll
        for (int d = 0; d < NOPS; ++d)
#pragma unroll
          for (int r = 0; r < R; ++r) buf[B][d][r][i] &= mi;
      }
    }
    if constexpr (kDot2) {
#pragma unroll
      for (int d = 0; d < NDOT; ++d)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float ah = 0.0f, al = 0.0f;
#pragma unroll
          for (int i = 0; i < NV; ++i) {
            const u32x4 x = buf[B][d][r][i];
#pragma unroll
            for (int w = 0; w < VEC / 2; ++w) {
              ah = dot2_bf16(x[w], vp[d][i][w], ah);
              al = dot2_bf16(x[w], vp[d][i][VEC / 2 + w], al);
            }
          }
          part[d][r] = (acc_t)(ah + al);
        }
      return;
    }
#pragma unroll
    for (int d = 0; d < NDOT; ++d)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc_t acc = (acc_t)0;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          const u32x4 x = buf[B][d][r][i];
          if (PLANES == 2) {
            const u32x4 xl = buf[B][1][r][i];
#pragma unroll
            for (int e = 0; e < VEC; ++e)
              acc += ((acc_t)St::get(x, e) + (acc_t)St::get(xl, e)) * vc[d][i][e];
          } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc += (acc_t)St::get(x, e) * vc[d][i][e];
          }
        }
        part[d][r] = acc;
      }
  }

  __device__ __forceinline__ u64 *slot_base(const ProdBufs &pb, const ProdGeom &pg, const WgCtx &ctx,
                                             uint32_t step) const {
    const int slot = (int)(step % kRing);
    // an idle workgroup (rg >= RG) only issues the unconditional poll loads, whose words
    // it never uses: it reads the last row group's slots
    const int rg = ctx.rg < pg.RG ? ctx.rg : pg.RG - 1;
    return pb.xchg + (((int64_t)rg * kRing + slot) * pg.C) * WORDS;
  }

  // Exchange wave: publish this column group's partial dots of exchange step `step`.
  // Every lane stores (lane l writes word l mod PW, the same value as the lanes it
  // shares the word with), so the store is issued unconditionally and the compiler's
  // count of outstanding memory operations stays exact.
  // Tail steps (tile >= n_my) publish to this workgroup's sink words instead: after its
  // last poll a workgroup runs its tail steps without waiting for the others, and a
  // publish into the ring could then overwrite a slot a slower member still reads.
  __device__ __forceinline__ void publish(const ProdBufs &pb, const ProdGeom &pg, const WgCtx &ctx, uint32_t step,
                                          bool tail, const double (&red)[NDOT][R]) {
    u64 *base = tail ? pb.sink + (int64_t)blockIdx.x * WORDS
                     : slot_base(pb, pg, ctx, step) + (int64_t)ctx.cg * WORDS;
    const u64 tag = (u64)(step / kRing + 1) << 32;
    const int k = ((int)threadIdx.x & 63) % PW;     // word written by this lane
    const int dr = k / WPD;                          // which partial dot
    double val = red[0][0];
#pragma unroll
    for (int d = 0; d < NDOT; ++d)
#pragma unroll
      for (int r = 0; r < R; ++r) val = (dr == d * R + r) ? red[d][r] : val;
    u64 word;
    if (WPD == 1) {
      word = tag | (u64)__float_as_uint((float)val);
    } else {
      const u64 b = (u64)__double_as_longlong(val);
      word = tag | ((k % 2) == 0 ? (b & 0xFFFFFFFFull) : (b >> 32));
    }
    st_coh64(&base[k], word);
  }

  // Exchange wave: issue the loads of column groups lane and lane + 64 into poll buffer Q
  // (no wait).  Issued unconditionally: column groups past C read group 0's words and
  // steps outside the product read a valid slot; neither result is used.
  template <int Q>
  __device__ __forceinline__ void poll_issue(const ProdBufs &pb, const ProdGeom &pg, const WgCtx &ctx,
                                             uint32_t step) {
    const int lane = (int)threadIdx.x & 63;
    const u64 *base = slot_base(pb, pg, ctx, step);
#pragma unroll
    for (int h = 0; h < kCh; ++h) {
      const int c = lane + 64 * h < pg.C ? lane + 64 * h : 0;
#pragma unroll
      for (int k = 0; k < PW; ++k) pw[Q][h][k] = ld_coh64(&base[(int64_t)c * WORDS + k]);
    }
  }

  __device__ __forceinline__ static bool words_ok(const u64 *w, uint32_t tag) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < PW; ++k) ok &= ((uint32_t)(w[k] >> 32) == tag);
    return ok;
  }
  __device__ __forceinline__ static void words_add(const u64 *w, double (&acc)[NDOT][R]) {
#pragma unroll
    for (int d = 0; d < NDOT; ++d)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (WPD == 1) {
          acc[d][r] += (double)__uint_as_float((uint32_t)w[d * R + r]);
        } else {
          const u64 lo = w[(d * R + r) * 2 + 0], hi = w[(d * R + r) * 2 + 1];
          acc[d][r] += __longlong_as_double((long long)((hi << 32) | (lo & 0xFFFFFFFFull)));
        }
      }
  }

  // Exchange wave: finish the poll of `step` (words of the first 128 column groups
  // already issued by poll_issue), re-reading until every column group's words carry the
  // step's tag; sum in a fixed order (lane's groups in order, then butterfly) and store
  // the row weights in tot[d][r].  Returns false if the wait gave up (abort).
  template <int Q>
  __device__ __forceinline__ bool poll_finish(const ProdBufs &pb, const ProdGeom &pg, const WgCtx &ctx,
                                              uint32_t step, double (*tot)[R]) {
    const int lane = (int)threadIdx.x & 63;
    const uint32_t tag = step / kRing + 1;
    const u64 *base = slot_base(pb, pg, ctx, step);
    uint64_t spins = 0;
    bool ok = true;
    auto lane_ok = [&](const u64 (&w)[kCh][PW]) {
      bool good = true;
#pragma unroll
      for (int h = 0; h < kCh; ++h) good &= (lane + 64 * h >= pg.C) || words_ok(w[h], tag);
      return good;
    };
    // the words issued ahead.  The first check is kept out of the retry loop so that it
    // waits only for those words, not for the tile loads issued after them.
    if (!__all(lane_ok(pw[Q]))) {
      u64 w[kCh][PW];
      while (true) {
#pragma unroll
        for (int h = 0; h < kCh; ++h) {
          const int c = lane + 64 * h < pg.C ? lane + 64 * h : 0;
#pragma unroll
          for (int k = 0; k < PW; ++k) w[h][k] = ld_coh64(&base[(int64_t)c * WORDS + k]);
        }
        if (__all(lane_ok(w))) break;
        if (++spins > kSpinLimit || ((spins & 255) == 0 && ld_coh32(ctx.gs.abort) != 0u)) {
          ok = false;
          break;
        }
      }
#pragma unroll
      for (int h = 0; h < kCh; ++h)
#pragma unroll
        for (int k = 0; k < PW; ++k) pw[Q][h][k] = w[h][k];
    }
    double acc[NDOT][R];
#pragma unroll
    for (int d = 0; d < NDOT; ++d)
#pragma unroll
      for (int r = 0; r < R; ++r) acc[d][r] = 0.0;
#pragma unroll
    for (int h = 0; h < kCh; ++h)
      if (lane + 64 * h < pg.C) words_add(pw[Q][h], acc);
    // further column groups (C > 128): read synchronously
    for (int c0 = 64 * kCh; ok && c0 < pg.C; c0 += 64) {
      const int c = c0 + lane;
      u64 w[PW];
      while (true) {
        if (c < pg.C) {
          const u64 *wp = base + (int64_t)c * WORDS;
#pragma unroll
          for (int k = 0; k < PW; ++k) w[k] = ld_coh64(&wp[k]);
        }
        if (__all(c >= pg.C || words_ok(w, tag))) break;
        if (++spins > kSpinLimit || ((spins & 255) == 0 && ld_coh32(ctx.gs.abort) != 0u)) {
          ok = false;
          break;
        }
      }
      if (c < pg.C) words_add(w, acc);
    }
    if (!ok && lane == 0) st_coh32(ctx.gs.abort, 1u);
#pragma unroll
    for (int d = 0; d < NDOT; ++d)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double t = wave_sum(acc[d][r]);
        if (lane == 0) tot[d][r] = t;
      }
    return ok;
  }

  // y += w * tile for tile j, held in register buffer B.
  template <int B>
  __device__ __forceinline__ void update(const ProdGeom &pg, const WgCtx &ctx, int j, const double (*tot)[R],
                                         const double *__restrict__ E, double v0) {
    const int64_t row0 = ((int64_t)j * pg.RG + ctx.rg) * R;
    acc_t w[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = row0 + r;
      const bool valid = row < pg.n_s;
      double wr;
      if (NDOT == 1) {
        wr = valid ? tot[0][r] : 0.0;
        s1 += wr;
      } else {
        // the load is unconditional (clamped row) so that no memory operation sits in a
        // branch; the row's weight is zero past n_s
        const double e = E[valid ? row : pg.n_s - 1];
        const double t = tot[0][r], u = tot[1][r];
        wr = valid ? e * (v0 + t) + u : 0.0;
        s1 += wr;
        s2 += valid ? e * t + u : 0.0;
      }
      w[r] = (acc_t)wr;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const u32x4 x = buf[B][0][r][i];
        if (PLANES == 2) {
          const u32x4 xl = buf[B][NOPS - 1][r][i];
#pragma unroll
          for (int e = 0; e < VEC; ++e) yacc[i][e] += ((acc_t)St::get(x, e) + (acc_t)St::get(xl, e)) * w[r];
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) yacc[i][e] += (acc_t)St::get(x, e) * w[r];
        }
      }
    }
  }

  // Roles of the waves when there are several column groups: wave 0 polls the other
  // groups' partial dots (kPoll), wave 1 combines the waves' partial dots and publishes
  // them (kPublish), the others only stream (kPlain).  Splitting the two halves the
  // serial work any one wave adds between barriers; for 2-byte storage (short steps)
  // that pays, for 4- and 8-byte storage wave 0 does both (kBoth) (measured on MI355X).
  enum { kPlain = 0, kPoll = 1, kPublish = 2, kBoth = 3 };
  static constexpr bool kSplit = St::BYTES == 2;

  // One pipeline step t (register buffer B = t % kNBuf) of a wave with role X.  Inside a
  // step no memory operation is conditional, so the compiler waits for exactly the loads
  // each use needs.
  template <int B, int X>
  __device__ __forceinline__ void step(const ProdGeom &pg, const ProdBufs &pb, WgCtx &ctx, const Operand *ops, int t,
                                       int n_my, const double *__restrict__ E, double v0,
                                       double (*s_part)[NW][NDOT][R], double (*s_tot)[NDOT][R], bool &ok) {
    constexpr int QI = ((B - kAdv) % kNPoll + kNPoll) % kNPoll;        // exchange t - kAdv
    constexpr int QF = ((B - kAdv - PD) % kNPoll + kNPoll) % kNPoll;   // exchange t - kAdv - PD
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    // polling wave: start loading the words of step t - kAdv (before this step's tile
    // loads, so waiting for them later never waits for this step's tiles)
    if constexpr ((X & kPoll) != 0) poll_issue<QI>(pb, pg, ctx, ctx.xstep + (uint32_t)(t - kAdv));
    // streaming: unconditional in every step (tiles past n_my read clamped rows with zero
    // weight), so the wait for tile t leaves tiles t+1..t+kLook in flight
    issue<(B + kLook) % kNBuf>(ctx, pg, ops, t + kLook);
    {
      acc_t part[NDOT][R];
      dots<B>(part);
#pragma unroll
      for (int d = 0; d < NDOT; ++d)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const acc_t sw = wave_sum(part[d][r]);
          if (lane == 0) s_part[t & 1][wave][d][r] = (double)sw;
        }
    }
    const int u = t - kLag;
    if (u >= 0 && u < n_my) update<(B + kNBuf - kLag) % kNBuf>(pg, ctx, u, s_tot[u % kNBuf], E, v0);
    if constexpr ((X & kPoll) != 0) {
      // finish the poll started at the beginning of step t - PD
      const int e = t - kAdv - PD;
      if (e >= 0 && e < n_my && ok) ok = poll_finish<QF>(pb, pg, ctx, ctx.xstep + (uint32_t)e, s_tot[e % kNBuf]);
    }
    __syncthreads();
    if ((X & kPublish) != 0 || (X == kPlain && pg.C == 1 && wave == 0 && t < n_my)) {
      double red[NDOT][R];
#pragma unroll
      for (int d = 0; d < NDOT; ++d)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          double sm = 0.0;
#pragma unroll
          for (int w = 0; w < NW; ++w) sm += s_part[t & 1][w][d][r];
          red[d][r] = (d == 0) ? sm - cshare : sm;
        }
      if constexpr ((X & kPublish) != 0) {
        // every step publishes (the tail steps past n_my into the sink), so the store is
        // not conditional
        publish(pb, pg, ctx, ctx.xstep + (uint32_t)t, t >= n_my, red);
      } else {
        if (lane == 0) {
#pragma unroll
          for (int d = 0; d < NDOT; ++d)
#pragma unroll
            for (int r = 0; r < R; ++r) s_tot[t % kNBuf][d][r] = red[d][r];
        }
      }
    }
  }

  // Steps t0 .. t0 + kNBuf - 1, one per register buffer, fully unrolled.
  template <int X, int... Bs>
  __device__ __forceinline__ void round_of_steps(std::integer_sequence<int, Bs...>, const ProdGeom &pg,
                                                 const ProdBufs &pb, WgCtx &ctx, const Operand *ops, int t0, int n_my,
                                                 const double *__restrict__ E, double v0,
                                                 double (*s_part)[NW][NDOT][R], double (*s_tot)[NDOT][R], bool &ok) {
    (step<Bs, X>(pg, pb, ctx, ops, t0 + Bs, n_my, E, v0, s_part, s_tot, ok), ...);
  }

  // The whole streaming loop of one wave with role X.  Every role executes the same
  // number of barriers.
  template <int X>
  __device__ __forceinline__ bool stream_rows(const ProdGeom &pg, const ProdBufs &pb, WgCtx &ctx, const Operand *ops,
                                              int n_my, int rounds, const double *__restrict__ E, double v0,
                                              double (*s_part)[NW][NDOT][R], double (*s_tot)[NDOT][R]) {
    issue<0>(ctx, pg, ops, 0);
    if (kLook > 1) issue<(1 % kNBuf)>(ctx, pg, ops, 1);
    if (kLook > 2) issue<(2 % kNBuf)>(ctx, pg, ops, 2);
    if (kLook > 3) issue<(3 % kNBuf)>(ctx, pg, ops, 3);
    bool ok = true;
    for (int q = 0; q < rounds; ++q)
      round_of_steps<X>(std::make_integer_sequence<int, kNBuf>{}, pg, pb, ctx, ops, q * kNBuf, n_my, E, v0, s_part,
                        s_tot, ok);
    return ok;
  }

  // Accumulate this workgroup's share of O^T w over its row group's tiles.
  __device__ __forceinline__ bool accumulate(const ProdGeom &pg, const ProdBufs &pb, WgCtx &ctx, const Operand *ops,
                                             double /*cshare*/, const double *__restrict__ E, double v0) {
    __shared__ double s_part[2][NW][NDOT][R];
    __shared__ double s_tot[kNBuf][NDOT][R];
    __shared__ int s_ok;
    const int n_tiles = (int)((pg.n_s + R - 1) / R);
    // an idle workgroup (rg >= RG) has no tiles: it runs the tail steps only (clamped rows,
    // publishes to its sink) and every barrier
    const int n_my = (ctx.rg < pg.RG && ctx.rg < n_tiles) ? (n_tiles - ctx.rg + pg.RG - 1) / pg.RG : 0;
    static_assert(kLook <= 4, "prologue issues at most 4 tiles");
    // whole rounds of kNBuf steps: no step is skipped, so the loop body has no branch
    // around loads (steps past n_my + kLag only stream clamped rows)
    const int rounds = (n_my + kLag + kNBuf - 1) / kNBuf;
    static_assert(NW >= 2, "the exchange roles need two waves");
    const int wave = (int)(threadIdx.x >> 6);
    bool ok;
    if (pg.C > 1 && wave == 0)
      ok = stream_rows<(kSplit ? kPoll : kBoth)>(pg, pb, ctx, ops, n_my, rounds, E, v0, s_part, s_tot);
    else if (kSplit && pg.C > 1 && wave == 1)
      ok = stream_rows<kPublish>(pg, pb, ctx, ops, n_my, rounds, E, v0, s_part, s_tot);
    else
      ok = stream_rows<kPlain>(pg, pb, ctx, ops, n_my, rounds, E, v0, s_part, s_tot);
    // the next product starts on a fresh block of kRing steps, so no word this product
    // left in the ring carries one of its tags (products may differ in words per slot);
    // every workgroup advances by the same amount (the most tiles of any row group), so
    // the step count is the same in all of them, also when the next product has another
    // geometry (several systems in one launch regroup the workgroups)
    const uint32_t most = (uint32_t)((n_tiles + pg.RG - 1) / pg.RG);
    ctx.xstep += (most + kRing - 1) / kRing * kRing;
    if (threadIdx.x == 0) s_ok = ok ? 1 : 0;
    __syncthreads();
    return s_ok != 0;
  }

  // Dynamic LDS of the launch (the tile ring lives in registers).
  static constexpr int ring_bytes() { return 0; }

  // Store the row group's partial y (float64) and scalars, coherently.
  __device__ __forceinline__ void store_partials(const ProdGeom &pg, const ProdBufs &pb, const WgCtx &ctx) {
    if (ctx.rg >= pg.RG) return;     // idle workgroup
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      if (i >= nvec) continue;
      const int nvalid = valid_of(colv(i));
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int64_t col = colv(i) + e;
        if (e < nvalid) st_coh(&pb.ypart[(int64_t)ctx.rg * pg.n_v + col], (double)yacc[i][e]);
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
  for (int rg = 0; rg < pg.RG; ++rg) acc += ld_coh(&pb.ypart[(int64_t)rg * pg.n_v + j]);
  return acc;
}

// Remainder columns [i0, i1) of a compact plane whose parameters lie in [j0, j1).
__device__ __forceinline__ void lo_range(const Operand &op, int64_t j0, int64_t j1, int64_t &i0, int64_t &i1) {
  if (op.lo_cols == nullptr) {
    i0 = i1 = 0;
    return;
  }
  i0 = lower_bound_wave(op.lo_cols, op.n_lo, j0);
  i1 = lower_bound_wave(op.lo_cols, op.n_lo, j1);
}

// Add the compact remainder plane's share to the finished columns of this workgroup:
// y_j += s_j (sum_rg ypart[rg][n_q + i]) / n_s for the remainder columns i in [i0, i1)
// (parameters j = lo_cols[i] inside the workgroup's finished range).  The callers wrote
// y_j in the same workgroup; barriers before and after order the accesses.
template <int NT>
__device__ __forceinline__ void finish_lo(const ProdBufs &pb, const ProdGeom &pg, const Operand &op, int64_t i0,
                                          int64_t i1, double inv_n, double *y) {
  if (i1 <= i0) return;
  __syncthreads();
  for (int64_t i = i0 + threadIdx.x; i < i1; i += NT) {
    const int64_t j = lo_param(op.lo_cols, i, pg.n_p);
    const double acc = finish_column(pb, pg, op.n_q + i);
    y[j] += (double)op.scale[j] * acc * inv_n;
  }
  __syncthreads();
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
