// Product, CG and linear-method kernels for DT_BF16 storage.
#include "sr_kernels.hpp"

namespace sr {

#define SR_REGISTER(NV, R, NB) \
  {DT_BF16, NV, R, NB, (const void *)&k_sv<DT_BF16, NV, R, NB>, (const void *)&k_cg<DT_BF16, NV, R, NB>, \
   (const void *)&k_lm<DT_BF16, NV, R, NB>},

static const KernelEntry g_entries_bf16[] = {SR_PRODUCT_CONFIGS_BF16(SR_REGISTER)};

const KernelEntry *kernel_table_bf16(int *count) {
  *count = (int)(sizeof(g_entries_bf16) / sizeof(g_entries_bf16[0]));
  return g_entries_bf16;
}

}  // namespace sr
