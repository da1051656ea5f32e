// Index-coded CPS storage kernels with a DT_F64 dense block.
#include "sr_cps.hpp"

namespace sr {

#define SR_REG_CPS(NVT)                                                                              \
  {DT_F64, NVT, (const void *)&k_cps_sv<DT_F64, NVT>, (const void *)&k_cps_cg_init<DT_F64, NVT>,       \
   (const void *)&k_cps_cg_step<DT_F64, NVT, false>, nullptr, \
   (const void *)&k_cps_cg_resid<DT_F64, NVT>},

static const CpsEntry g_cps_f64[] = {SR_REG_CPS(2) SR_REG_CPS(4) SR_REG_CPS(8) SR_REG_CPS(12) SR_REG_CPS(16)};

const CpsEntry *cps_table_f64(int *count) {
  *count = (int)(sizeof(g_cps_f64) / sizeof(g_cps_f64[0]));
  return g_cps_f64;
}

}  // namespace sr
