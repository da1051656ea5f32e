// Product, CG and linear-method kernels for DT_F64 storage.
#include "sr_kernels.hpp"

namespace sr {

#define SR_REGISTER(NV, R, NB) \
  {DT_F64, NV, R, NB, (const void *)&k_sv<DT_F64, NV, R, NB>, (const void *)&k_cg<DT_F64, NV, R, NB>, \
   (const void *)&k_lm<DT_F64, NV, R, NB>},

static const KernelEntry g_entries_f64[] = {SR_PRODUCT_CONFIGS_F64(SR_REGISTER)};

const KernelEntry *kernel_table_f64(int *count) {
  *count = (int)(sizeof(g_entries_f64) / sizeof(g_entries_f64[0]));
  return g_entries_f64;
}

}  // namespace sr
