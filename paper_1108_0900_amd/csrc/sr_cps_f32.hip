// Index-coded CPS storage kernels with a DT_F32 dense block.
#include "sr_cps.hpp"

namespace sr {

#define SR_REG_CPS(NVT)                                                                              \
  {DT_F32, NVT, (const void *)&k_cps_sv<DT_F32, NVT>, (const void *)&k_cps_cg_init<DT_F32, NVT>,       \
   (const void *)&k_cps_cg_step<DT_F32, NVT, false>, nullptr, \
   (const void *)&k_cps_cg_resid<DT_F32, NVT>},

static const CpsEntry g_cps_f32[] = {SR_REG_CPS(2) SR_REG_CPS(3) SR_REG_CPS(4) SR_REG_CPS(6) SR_REG_CPS(8)};

const CpsEntry *cps_table_f32(int *count) {
  *count = (int)(sizeof(g_cps_f32) / sizeof(g_cps_f32[0]));
  return g_cps_f32;
}

}  // namespace sr
