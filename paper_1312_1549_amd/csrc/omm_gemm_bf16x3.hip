// BF16x3 split MFMA GEMM instantiations (v_mfma_f32_16x16x32_bf16) on pre-split bf16 planes.
#include "omm_gemm_impl.h"

namespace omm {
namespace gemm_detail {

namespace {
template <typename TA, typename TB, typename TC, typename TX>
gemm_fn pick2(const GemmDesc& d) {
  if (d.la == KC && d.lb == KC) return pick_tile<CBF16X3, TA, TB, TC, TX, KC, KC>(d.tile);
  if (d.la == KC && d.lb == RC) return pick_tile<CBF16X3, TA, TB, TC, TX, KC, RC>(d.tile);
  return nullptr;
}
}  // namespace

gemm_fn pick_bf16x3(const GemmDesc& d) {
  typedef unsigned short P;  // pre-split bf16 (hi, lo) planes
  if (d.ta == T_BF16P && d.tb == T_BF16P && d.tc == T_F32 && d.tx == T_F32)
    return pick2<P, P, float, float>(d);
  if (d.ta == T_BF16P && d.tb == T_BF16P && d.tc == T_F64 && d.tx == T_F64)
    return pick2<P, P, double, double>(d);
  // FP32 output with an FP64 addend (the gradient over the FP64 state)
  if (d.ta == T_BF16P && d.tb == T_BF16P && d.tc == T_F32 && d.tx == T_F64 && d.la == KC &&
      d.lb == KC)
    return pick_tile<CBF16X3, P, P, float, double, KC, KC>(d.tile);
  return nullptr;
}

sk_fn pick_sk_bf16x3(const GemmDesc& d) {
  if (d.la != KC || d.lb != KC || d.ta != T_BF16P || d.tb != T_BF16P) return nullptr;
  if (d.tc == T_F32 && d.tx == T_F32) return pick_sk_kernel<CBF16X3, float, float>();
  if (d.tc == T_F64 && d.tx == T_F64) return pick_sk_kernel<CBF16X3, double, double>();
  // the gradient: FP32 output, FP64 addend
  if (d.tc == T_F32 && d.tx == T_F64) return pick_sk_kernel<CBF16X3, float, double>();
  return nullptr;
}

}  // namespace gemm_detail
}  // namespace omm
