// Batched advance, FP64, block edge 8: the compiled launch variants.
#include "tvd_batched_launch.hpp"

namespace tvd {

hipError_t launch_batched_f64_e8(int order, const Variant& v, bool gather, const KParams& kp,
                                 hipStream_t s) {
#define TVD_VARIANT(E, TH, P, SP)                                    \
  if (v.edge == E && v.threads == TH && v.pad == P && v.split == SP) \
    return launch_b<double, E, TH, P, SP>(order, gather, kp, s);
  TVD_VARIANT(8, 128, 8, 0)
  TVD_VARIANT(8, 128, 8, 2)
  TVD_VARIANT(8, 256, 8, 0)
  TVD_VARIANT(8, 64, 8, 0)
#undef TVD_VARIANT
  return hipErrorInvalidValue;
}

}  // namespace tvd
