// Streamed advance, FP32: the compiled instantiations (block edges 16 and 32,
// both sweep orders, slabs of 8 planes; with flux records, edge 16 and the
// half-pencil second sweep).
#include "tvd_stream.hpp"

namespace tvd {

template <int E, int ORDER, bool SPLITB>
static hipError_t launch_one(const KParams& kp, const StreamParams& sp, hipStream_t s) {
  const dim3 grid((unsigned)sp.n_chains * (unsigned)sp.quads), block(kStreamNT);
  hipLaunchKernelGGL((k_stream<float, E, ORDER, 8, SPLITB>), grid, block, 0, s, kp, sp);
  return hipGetLastError();
}

hipError_t launch_stream_f32(int order, int edge, bool splitb, const KParams& kp,
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

// With flux records the second sweep runs in whole pencils: the records'
// pointers and the halves' held results together exceed the register file
// (300-430 registers spilled per lane), whole pencils fit (about 248).
template <int ORDER, int FLUX>
static hipError_t launch_flux(const KParams& kp, const StreamParams& sp, hipStream_t s) {
  const dim3 grid((unsigned)sp.n_chains * (unsigned)sp.quads), block(kStreamNT);
  hipLaunchKernelGGL((k_stream<float, 16, ORDER, 8, false, FLUX>), grid, block, 0, s, kp, sp);
  return hipGetLastError();
}

hipError_t launch_stream_flux_f32(int order, bool accumulate, const KParams& kp,
                                  const StreamParams& sp, hipStream_t s) {
  if (accumulate) return order == 0 ? launch_flux<0, 2>(kp, sp, s) : launch_flux<1, 2>(kp, sp, s);
  return order == 0 ? launch_flux<0, 1>(kp, sp, s) : launch_flux<1, 1>(kp, sp, s);
}

}  // namespace tvd
