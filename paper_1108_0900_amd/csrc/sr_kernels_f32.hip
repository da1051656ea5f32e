// Product, CG and linear-method kernels for DT_F32 storage.
#include "sr_kernels.hpp"

namespace sr {

#define SR_REGISTER(NV, R, NB) \
  {DT_F32, NV, R, NB, (const void *)&k_sv<DT_F32, NV, R, NB>, (const void *)&k_cg<DT_F32, NV, R, NB>, \
   (const void *)&k_lm<DT_F32, NV, R, NB>},

static const KernelEntry g_entries_f32[] = {SR_PRODUCT_CONFIGS_F32(SR_REGISTER)};

const KernelEntry *kernel_table_f32(int *count) {
  *count = (int)(sizeof(g_entries_f32) / sizeof(g_entries_f32[0]));
  return g_entries_f32;
}

}  // namespace sr
