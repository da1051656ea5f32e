// Product, CG and linear-method kernels for DT_F16 storage.
#include "sr_kernels.hpp"

namespace sr {

#define SR_REGISTER(NV, R, NB) \
  {DT_F16, NV, R, NB, (const void *)&k_sv<DT_F16, NV, R, NB>, (const void *)&k_cg<DT_F16, NV, R, NB>, \
   (const void *)&k_lm<DT_F16, NV, R, NB>},

static const KernelEntry g_entries_f16[] = {SR_PRODUCT_CONFIGS_F16(SR_REGISTER)};

const KernelEntry *kernel_table_f16(int *count) {
  *count = (int)(sizeof(g_entries_f16) / sizeof(g_entries_f16[0]));
  return g_entries_f16;
}

}  // namespace sr
