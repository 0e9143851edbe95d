// Two-product BF16 MFMA GEMM instantiations on pre-split bf16 planes: one operand holds exact
// bf16 values (its hi plane alone), the other a hi/lo pair. Used for products with the search
// direction (A) in the BF16x3 scheme. The one-product mode (both operands single planes, FP32
// output) applies the preconditioner's bf16 rounding to the gradient's.
#include "omm_gemm_impl.h"

namespace omm {
namespace gemm_detail {

namespace {
template <int MODE>
gemm_fn pick_mode(const GemmDesc& d) {
  typedef unsigned short P;
  if (d.la != KC || d.lb != KC || d.ta != T_BF16P || d.tb != T_BF16P) return nullptr;
  if (d.tc == T_F32 && d.tx == T_F32) return pick_tile<MODE, P, P, float, float, KC, KC>(d.tile);
  if (d.tc == T_F64 && d.tx == T_F64) return pick_tile<MODE, P, P, double, double, KC, KC>(d.tile);
  return nullptr;
}
}  // namespace

gemm_fn pick_bf16x2(const GemmDesc& d) {
  if (d.compute == CBF16X2A) return pick_mode<CBF16X2A>(d);
  if (d.compute == CBF16X2B) return pick_mode<CBF16X2B>(d);
  if (d.compute == CBF16X1 && d.la == KC && d.lb == KC && d.ta == T_BF16P && d.tb == T_BF16P &&
      d.tc == T_F32 && d.tx == T_F32)
    return pick_tile<CBF16X1, unsigned short, unsigned short, float, float, KC, KC>(d.tile);
  return nullptr;
}

namespace {
template <int MODE>
sk_fn pick_sk_mode(const GemmDesc& d) {
  if (d.la != KC || d.lb != KC || d.ta != T_BF16P || d.tb != T_BF16P) return nullptr;
  if (d.tc == T_F32 && d.tx == T_F32) return pick_sk_kernel<MODE, float, float>();
  if (d.tc == T_F64 && d.tx == T_F64) return pick_sk_kernel<MODE, double, double>();
  return nullptr;
}
}  // namespace

sk_fn pick_sk_bf16x2(const GemmDesc& d) {
  if (d.compute == CBF16X2A) return pick_sk_mode<CBF16X2A>(d);
  if (d.compute == CBF16X2B) return pick_sk_mode<CBF16X2B>(d);
  // (its instantiation spills a few per-work-item values to scratch memory, outside the K loop)
  if (d.compute == CBF16X1 && d.la == KC && d.lb == KC && d.ta == T_BF16P && d.tb == T_BF16P &&
      d.tc == T_F32 && d.tx == T_F32)
    return pick_sk_kernel<CBF16X1, float, float>();
  return nullptr;
}

}  // namespace gemm_detail
}  // namespace omm
