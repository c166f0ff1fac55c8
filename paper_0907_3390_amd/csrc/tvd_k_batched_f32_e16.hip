// Batched advance, FP32, block edge 16: the compiled launch variants.
#include "tvd_batched_launch.hpp"

namespace tvd {

hipError_t launch_batched_f32_e16(int order, const Variant& v, bool gather, const KParams& kp,
                                  hipStream_t s) {
#define TVD_VARIANT(E, TH, P, SP)                                    \
  if (v.edge == E && v.threads == TH && v.pad == P && v.split == SP) \
    return launch_b<float, E, TH, P, SP>(order, gather, kp, s);
  TVD_VARIANT(16, 512, 0, 1)
  TVD_VARIANT(16, 512, 0, 3)
  TVD_VARIANT(16, 512, 0, 2)
  TVD_VARIANT(16, 512, 0, 0)
  TVD_VARIANT(16, 512, 16, 1)
  TVD_VARIANT(16, 512, 16, 3)
#undef TVD_VARIANT
  return hipErrorInvalidValue;
}

}  // namespace tvd
