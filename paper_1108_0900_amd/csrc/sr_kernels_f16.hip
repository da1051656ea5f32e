// Product, CG and linear-method kernels for DT_F16 storage.
#include "sr_kernels.hpp"

namespace sr {

#define SR_REG_SR(NV, R, L, P, NT)                                                                   \
  {DT_F16, NV, R, L, P, NT, 0, (const void *)&k_sv<DT_F16, NV, R, L, P, NT>,                        \
   (const void *)&k_cg<DT_F16, NV, R, L, P, NT>, nullptr,                                            \
   (const void *)&k_sv2<DT_F16, NV, NT>, (const void *)&k_cg<DT_F16, NV, 1, 1, 1, NT, kCgTwoPlanes>,             \
   nullptr,                                                                                          \
   (const void *)&k_cg<DT_F16, NV, R, L, P, NT, kCgExact>,                                             \
   (const void *)&k_cg_step<DT_F16, NV, R, L, P, NT>,                                                     \
   (const void *)&k_cg<DT_F16, NV, R, L, P, NT, kCgOnePlane, kPhResidual>,                               \
   (const void *)&k_cg_init<DT_F16, NV, R, L, P, NT>,                                                     \
   Product<DT_F16, NV, R, 1, false, L, P, NT>::ring_bytes()},
#define SR_REG_LM(NV, R, L, P, NT)                                                                   \
  {DT_F16, NV, R, L, P, NT, 1, nullptr, nullptr, (const void *)&k_lm<DT_F16, NV, R, L, P, NT>, nullptr, \
   nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, Product<DT_F16, NV, R, 2, false, L, P, NT>::ring_bytes()},

static const KernelEntry g_entries_f16[] = {SR_SR_CONFIGS_F16(SR_REG_SR) SR_LM_CONFIGS(SR_REG_LM)};

const KernelEntry *kernel_table_f16(int *count) {
  *count = (int)(sizeof(g_entries_f16) / sizeof(g_entries_f16[0]));
  return g_entries_f16;
}

}  // namespace sr
