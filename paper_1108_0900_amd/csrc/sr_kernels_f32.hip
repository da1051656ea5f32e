// Product, CG and linear-method kernels for DT_F32 storage.
#include "sr_batch.hpp"
#include "sr_shifts.hpp"

namespace sr {

#define SR_REG_SR(NV, R, L, P, NT)                                                                   \
  {DT_F32, NV, R, L, P, NT, 0, (const void *)&k_sv<DT_F32, NV, R, L, P, NT>,                        \
   (const void *)&k_cg<DT_F32, NV, R, L, P, NT>, nullptr,                                            \
   nullptr, nullptr, (const void *)&k_cg<DT_F32, NV, R, L, P, NT, kCgJacobi>, nullptr,               \
   (const void *)&k_cg_step<DT_F32, NV, R, L, P, NT>,                                                 \
   (const void *)&k_cg<DT_F32, NV, R, L, P, NT, kCgOnePlane, kPhResidual>,                            \
   (const void *)&k_cg_init<DT_F32, NV, R, L, P, NT>, Product<DT_F32, NV, R, 1, false, L, P, NT>::ring_bytes()},
#define SR_REG_LM(NV, R, L, P, NT)                                                                   \
  {DT_F32, NV, R, L, P, NT, 1, nullptr, nullptr, (const void *)&k_lm<DT_F32, NV, R, L, P, NT>, nullptr, \
   nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, Product<DT_F32, NV, R, 2, false, L, P, NT>::ring_bytes()},

static const KernelEntry g_entries_f32[] = {SR_SR_CONFIGS_F32(SR_REG_SR) SR_LM_CONFIGS(SR_REG_LM)};

// Batched solves: one tile configuration (K = 8 right-hand sides need the registers of
// one 16-byte vector per thread).
static const BatchEntry g_batch_f32 = {(const void *)&k_cg_batched<DT_F32, kBatchNT>,
                                           (const void *)&k_svk<DT_F32, kBatchNT>, kBatchNT};
const BatchEntry *batched_entry_f32() { return &g_batch_f32; }

// Multi-shift CG, one kernel per SR tile configuration.
#define SR_REG_SHIFT(NV, R, L, P, NT)                                                                \
  {NV, R, L, P, NT, (const void *)&k_cg_shifts<DT_F32, NV, R, L, P, NT>,                              \
   (const void *)&k_cg_shifts_batched<DT_F32, NV, R, L, P, NT>},
static const ShiftEntry g_shift_f32[] = {SR_SR_CONFIGS_F32(SR_REG_SHIFT)};
const void *shift_kernel_f32(int nv, int r, int look, int poll, int nt, bool batched) {
  for (const ShiftEntry &e : g_shift_f32)
    if (e.nv == nv && e.r == r && e.look == look && e.poll == poll && e.nt == nt) return batched ? e.batched : e.fn;
  return nullptr;
}

const KernelEntry *kernel_table_f32(int *count) {
  *count = (int)(sizeof(g_entries_f32) / sizeof(g_entries_f32[0]));
  return g_entries_f32;
}

}  // namespace sr
