// FP32 MFMA GEMM instantiations (v_mfma_f32_16x16x4f32).
#include "omm_gemm_impl.h"

namespace omm {
namespace gemm_detail {

namespace {
template <typename TA, typename TB, typename TC, typename TX>
gemm_fn pick2(const GemmDesc& d) {
  if (d.la == KC && d.lb == KC) return pick_tile<CF32, TA, TB, TC, TX, KC, KC>(d.tile);
  if (d.la == KC && d.lb == RC) return pick_tile<CF32, TA, TB, TC, TX, KC, RC>(d.tile);
  return nullptr;
}
}  // namespace

namespace {
template <typename TA, typename TB, typename TC, typename TX>
grouped_fn pickg2(const GemmDesc& d) {
  if (d.la == KC && d.lb == KC) return pick_grouped_tile<CF32, TA, TB, TC, TX, KC, KC>(d.tile);
  if (d.la == KC && d.lb == RC) return pick_grouped_tile<CF32, TA, TB, TC, TX, KC, RC>(d.tile);
  return nullptr;
}
}  // namespace

grouped_fn pick_grouped_f32(const GemmDesc& d) {
  if (d.ta == T_F32 && d.tb == T_F32 && d.tc == T_F32 && d.tx == T_F32)
    return pickg2<float, float, float, float>(d);
  if (d.ta == T_F32 && d.tb == T_F32 && d.tc == T_F64 && d.tx == T_F64)
    return pickg2<float, float, double, double>(d);
  if (d.ta == T_F64 && d.tb == T_F32 && d.tc == T_F32 && d.tx == T_F32)
    return pickg2<double, float, float, float>(d);
  return nullptr;
}

gemm_fn pick_f32(const GemmDesc& d) {
  if (d.ta == T_F32 && d.tb == T_F32 && d.tc == T_F32 && d.tx == T_F32)
    return pick2<float, float, float, float>(d);
  if (d.ta == T_F32 && d.tb == T_F32 && d.tc == T_F64 && d.tx == T_F64)
    return pick2<float, float, double, double>(d);
  if (d.ta == T_F64 && d.tb == T_F32 && d.tc == T_F32 && d.tx == T_F32)
    return pick2<double, float, float, float>(d);
  return nullptr;
}

}  // namespace gemm_detail
}  // namespace omm
