// FP64 MFMA GEMM instantiations (v_mfma_f64_16x16x4f64), single and grouped launches.
#include "omm_gemm_impl.h"

namespace omm {
namespace gemm_detail {

grouped_fn pick_grouped_f64(const GemmDesc& d) {
  if (d.ta != T_F64 || d.tb != T_F64 || d.tc != T_F64 || d.tx != T_F64) return nullptr;
  if (d.la == KC && d.lb == KC)
    return pick_grouped_tile<CF64, double, double, double, double, KC, KC>(d.tile);
  if (d.la == KC && d.lb == RC)
    return pick_grouped_tile<CF64, double, double, double, double, KC, RC>(d.tile);
  return nullptr;
}

gemm_fn pick_f64(const GemmDesc& d) {
  if (d.ta == T_F64 && d.tb == T_F64 && d.tc == T_F64 && d.tx == T_F64)
    return pick_layout<CF64, double, double, double, double>(d.la, d.lb, d.tile);
  return nullptr;
}

}  // namespace gemm_detail
}  // namespace omm
