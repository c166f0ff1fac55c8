// The batched launch of one compiled variant (shared by the translation units
// that instantiate the variants of one element type and block edge).
#pragma once

#include "tvd_block.hpp"

namespace tvd {

// The flux-recording advance exists for one variant per (type, edge): the
// default ones (edge 16: 512 threads, pad 16, split 3; edge 8: 128 threads
// FP32 or 256 threads FP64, pad 8, split 0).
template <typename T, int N, int NT, int PAD, int SPLIT>
constexpr bool kFluxVariant =
    N == 16 ? (NT == 512 && PAD == 16 && SPLIT == 3)
            : (NT == (sizeof(T) == 4 ? 128 : 256) && PAD == 8 && SPLIT == 0);

template <typename T, int N, int NT, int PAD, int SPLIT>
inline hipError_t launch_b(int order, bool gather, const KParams& kp, hipStream_t s) {
  const dim3 grid(kp.nblocks), block(NT);
  if (kp.flux) {
    if constexpr (kFluxVariant<T, N, NT, PAD, SPLIT>) {
      if (gather) {
        if (kp.flux_acc) {
          if (order == 0) hipLaunchKernelGGL((k_batched<T, N, 0, NT, PAD, SPLIT, true, 2>), grid, block, 0, s, kp);
          else hipLaunchKernelGGL((k_batched<T, N, 1, NT, PAD, SPLIT, true, 2>), grid, block, 0, s, kp);
        } else {
          if (order == 0) hipLaunchKernelGGL((k_batched<T, N, 0, NT, PAD, SPLIT, true, 1>), grid, block, 0, s, kp);
          else hipLaunchKernelGGL((k_batched<T, N, 1, NT, PAD, SPLIT, true, 1>), grid, block, 0, s, kp);
        }
        return hipGetLastError();
      }
      if (kp.flux_acc) {
        if (order == 0) hipLaunchKernelGGL((k_batched<T, N, 0, NT, PAD, SPLIT, false, 2>), grid, block, 0, s, kp);
        else hipLaunchKernelGGL((k_batched<T, N, 1, NT, PAD, SPLIT, false, 2>), grid, block, 0, s, kp);
      } else {
        if (order == 0) hipLaunchKernelGGL((k_batched<T, N, 0, NT, PAD, SPLIT, false, 1>), grid, block, 0, s, kp);
        else hipLaunchKernelGGL((k_batched<T, N, 1, NT, PAD, SPLIT, false, 1>), grid, block, 0, s, kp);
      }
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (gather) {
    if (order == 0) hipLaunchKernelGGL((k_batched<T, N, 0, NT, PAD, SPLIT, true>), grid, block, 0, s, kp);
    else hipLaunchKernelGGL((k_batched<T, N, 1, NT, PAD, SPLIT, true>), grid, block, 0, s, kp);
  } else {
    if (order == 0) hipLaunchKernelGGL((k_batched<T, N, 0, NT, PAD, SPLIT, false>), grid, block, 0, s, kp);
    else hipLaunchKernelGGL((k_batched<T, N, 1, NT, PAD, SPLIT, false>), grid, block, 0, s, kp);
  }
  return hipGetLastError();
}

}  // namespace tvd
