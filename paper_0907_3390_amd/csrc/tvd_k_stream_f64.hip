// Streamed advance, FP64: the compiled instantiations (block edges 16 and 32,
// both sweep orders, slabs of 8 planes, half or whole second-sweep pencils).
#include "tvd_stream.hpp"

namespace tvd {

template <int E, int ORDER, bool SPLITB>
static hipError_t launch_one(const KParams& kp, const StreamParams& sp, hipStream_t s) {
  const dim3 grid((unsigned)sp.n_chains * (unsigned)sp.quads), block(kStreamNT);
  hipLaunchKernelGGL((k_stream<double, E, ORDER, 8, SPLITB>), grid, block, 0, s, kp, sp);
  return hipGetLastError();
}

hipError_t launch_stream_f64(int order, int edge, bool splitb, const KParams& kp,
                             const StreamParams& sp, hipStream_t s) {
  if (edge == 16) {
    if (splitb) return order == 0 ? launch_one<16, 0, true>(kp, sp, s) : launch_one<16, 1, true>(kp, sp, s);
    return order == 0 ? launch_one<16, 0, false>(kp, sp, s) : launch_one<16, 1, false>(kp, sp, s);
  }
  if (edge == 32) {
    if (splitb) return order == 0 ? launch_one<32, 0, true>(kp, sp, s) : launch_one<32, 1, true>(kp, sp, s);
    return order == 0 ? launch_one<32, 0, false>(kp, sp, s) : launch_one<32, 1, false>(kp, sp, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace tvd
