// Index-coded CPS storage kernels with a DT_BF16 dense block.
#include "sr_cps.hpp"

namespace sr {

// float64-accumulated search products hold twice the registers: narrow tiles only
#define STEPX(NVT) ((NVT) <= 4 ? (const void *)&k_cps_cg_step<DT_BF16, ((NVT) <= 4 ? (NVT) : 4), true> : nullptr)
#define SR_REG_CPS(NVT)                                                                              \
  {DT_BF16, NVT, (const void *)&k_cps_sv<DT_BF16, NVT>, (const void *)&k_cps_cg_init<DT_BF16, NVT>,       \
   (const void *)&k_cps_cg_step<DT_BF16, NVT, false>, STEPX(NVT), \
   (const void *)&k_cps_cg_resid<DT_BF16, NVT>},

static const CpsEntry g_cps_bf16[] = {SR_REG_CPS(2) SR_REG_CPS(3) SR_REG_CPS(4) SR_REG_CPS(8)};

const CpsEntry *cps_table_bf16(int *count) {
  *count = (int)(sizeof(g_cps_bf16) / sizeof(g_cps_bf16[0]));
  return g_cps_bf16;
}

}  // namespace sr
