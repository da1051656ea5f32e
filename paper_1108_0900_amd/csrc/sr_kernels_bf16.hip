// Product, CG and linear-method kernels for DT_BF16 storage.
#include "sr_kernels.hpp"

namespace sr {

#define SR_REG_SR(NV, R, L, P, NT)                                                                   \
  {DT_BF16, NV, R, L, P, NT, 0, (const void *)&k_sv<DT_BF16, NV, R, L, P, NT>,                        \
   (const void *)&k_cg<DT_BF16, NV, R, L, P, NT>, nullptr,                                            \
   (const void *)&k_sv2<DT_BF16, NV, NT>, (const void *)&k_cg<DT_BF16, NV, 1, 1, 1, NT, kCgTwoPlanes>,             \
   nullptr,                                                                                          \
   (const void *)&k_cg<DT_BF16, NV, R, L, P, NT, kCgExact>,                                             \
   (const void *)&k_cg_step<DT_BF16, NV, R, L, P, NT>,                                                     \
   (const void *)&k_cg<DT_BF16, NV, R, L, P, NT, kCgOnePlane, kPhResidual>,                               \
   (const void *)&k_cg_init<DT_BF16, NV, R, L, P, NT>,                                                     \
   Product<DT_BF16, NV, R, 1, false, L, P, NT>::ring_bytes()},
#define SR_REG_LM(NV, R, L, P, NT)                                                                   \
  {DT_BF16, NV, R, L, P, NT, 1, nullptr, nullptr, (const void *)&k_lm<DT_BF16, NV, R, L, P, NT>, nullptr, \
   nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, Product<DT_BF16, NV, R, 2, false, L, P, NT>::ring_bytes()},

static const KernelEntry g_entries_bf16[] = {SR_SR_CONFIGS_BF16(SR_REG_SR) SR_LM_CONFIGS(SR_REG_LM)};

const KernelEntry *kernel_table_bf16(int *count) {
  *count = (int)(sizeof(g_entries_bf16) / sizeof(g_entries_bf16[0]));
  return g_entries_bf16;
}

}  // namespace sr
