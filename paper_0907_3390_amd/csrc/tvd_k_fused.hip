// The persistent launch over a batch of mixed block edges (FP32): a planning
// kernel and per-XCD work queues.
#include "tvd_block.hpp"

namespace tvd {

// ---------------------------------------------------------------------------
// persistent launch over a batch of mixed edges
// ---------------------------------------------------------------------------
//
// The plan kernel partitions the blocks by edge (kp.d_edge, or the uniform
// kp.edge for all), stably: edge-16 blocks first,
// then edge-8 blocks, in block order (list), with their counts (count[0],
// count[1]), and clears the work counters (next).  A block of any other edge
// is skipped and counted once in the non-physical counter.
//
// Work items: item w < n16 is edge-16 block list[w], advanced by the whole
// workgroup; item w >= n16 is the quad of edge-8 blocks
// list[n16 + 4(w - n16) + q], q = 0..3, one per quarter of the workgroup,
// each quarter with its own LDS.  The items are cut into one queue per XCD
// (contiguous ranges, so neighbouring blocks meet in one L2, each range
// edge-16 blocks first); a workgroup drains its XCD's queue and then helps
// the others.

constexpr int kPlanNT = 1024;
constexpr int kXcds = 8;
// the variants the persistent kernel runs (edge 16 on the whole workgroup,
// edge 8 on each quarter)
constexpr int kFusedPad16 = 16, kFusedSplit16 = 3;
constexpr int kFusedPad8 = 8, kFusedSplit8 = 2;

__global__ __launch_bounds__(kPlanNT) void k_plan(const int32_t* __restrict__ edge, int uniform,
                                                  int n, FusedPlan pl,
                                                  unsigned long long* counters) {
  __shared__ int w16[kPlanNT / 64], w8[kPlanNT / 64];
  __shared__ int tot16, tot8;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  int c16 = 0, c8 = 0;
  for (int i = t; i < n; i += kPlanNT) {
    const int e = edge ? edge[i] : uniform;
    c16 += e == 16;
    c8 += e == 8;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    c16 += __shfl_xor(c16, off);
    c8 += __shfl_xor(c8, off);
  }
  if (l == 0) {
    w16[w] = c16;
    w8[w] = c8;
  }
  __syncthreads();
  if (t == 0) {
    int a = 0, c = 0;
    for (int k = 0; k < kPlanNT / 64; ++k) {
      a += w16[k];
      c += w8[k];
    }
    tot16 = a;
    tot8 = c;
    pl.count[0] = a;
    pl.count[1] = c;
    if (n - a - c > 0) atomicAdd(&counters[1], (unsigned long long)(n - a - c));
  }
  if (t < kXcds) pl.next[t] = 0u;
  __syncthreads();
  const int n16 = tot16;
  int run16 = 0, run8 = 0;
  const unsigned long long below = l == 0 ? 0ull : (~0ull >> (64 - l));
  for (int base = 0; base < n; base += kPlanNT) {
    const int i = base + t;
    const int e = i < n ? (edge ? edge[i] : uniform) : 0;
    const unsigned long long m16 = __ballot(e == 16), m8 = __ballot(e == 8);
    __syncthreads();  // the previous chunk's totals have been read
    if (l == 0) {
      w16[w] = __popcll(m16);
      w8[w] = __popcll(m8);
    }
    __syncthreads();
    int o16 = 0, o8 = 0, a16 = 0, a8 = 0;
    for (int k = 0; k < kPlanNT / 64; ++k) {
      if (k < w) {
        o16 += w16[k];
        o8 += w8[k];
      }
      a16 += w16[k];
      a8 += w8[k];
    }
    if (e == 16) pl.list[run16 + o16 + __popcll(m16 & below)] = i;
    if (e == 8) pl.list[n16 + run8 + o8 + __popcll(m8 & below)] = i;
    run16 += a16;
    run8 += a8;
  }
}

// [lo, hi) of part k when n items are cut into kXcds contiguous parts
__device__ __forceinline__ int part_lo(int n, int k) {
  const int q = n / kXcds, r = n % kXcds;
  return k * q + (k < r ? k : r);
}

template <typename T, int ORDER, bool GATHER, int FLUX = 0>
__global__ __launch_bounds__(512) void k_fused(KParams kp, FusedPlan pl) {
  using B16 = BlockLds<T, 16, kFusedPad16>;
  using B8 = BlockLds<T, 8, kFusedPad8>;
  static_assert(4 * sizeof(B8) <= sizeof(B16), "four edge-8 blocks share the edge-16 LDS");
  __shared__ B16 sm;
  __shared__ int item;
  const int xcd = blockIdx.x % kXcds;
  const int n16 = pl.count[0], n8 = pl.count[1];
  const int nq = (n8 + 3) / 4;
  // thread 0 only: queues drained so far, and the ticket drawn during the
  // previous item from queue (xcd + qi) % kXcds (-1: none)
  int qi = 0;
  int ticket = -1;
  for (;;) {
    if (threadIdx.x == 0) {
      int wi = -1;
      for (; qi < kXcds; ++qi) {
        const int x = (xcd + qi) % kXcds;
        const int lo16 = part_lo(n16, x), hi16 = part_lo(n16, x + 1);
        const int loq = part_lo(nq, x), hiq = part_lo(nq, x + 1);
        const int k = ticket >= 0 ? ticket : (int)atomicAdd(&pl.next[x], 1u);
        ticket = -1;
        if (k < hi16 - lo16) {
          wi = lo16 + k;
          break;
        }
        if (k < hi16 - lo16 + hiq - loq) {
          wi = n16 + loq + k - (hi16 - lo16);
          break;
        }
      }
      item = wi;
    }
    __syncthreads();
    const int wi = item;
    __syncthreads();
    if (wi < 0) break;  // uniform over the workgroup
    // thread 0 draws the next ticket from its current queue late in this item
    unsigned* const ahead = threadIdx.x == 0 ? &pl.next[(xcd + qi) % kXcds] : nullptr;
    // The thread index is passed through an empty asm statement (no
    // instruction) so that the per-thread pencil indexing of every sweep is
    // recomputed per item: hoisted out of the loop it stays live across all
    // three sweeps and makes the register allocator spill.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (wi < n16) {
      advance_block<T, 16, ORDER, 512, kFusedPad16, kFusedSplit16, GATHER, FLUX>(
          kp, pl.list[wi], tid, sm, ahead, &ticket);
    } else {
      const int q = tid >> 7;
      const int i = 4 * (wi - n16) + q;
      const int b = i < n8 ? pl.list[n16 + i] : -1;
      B8* quarter = reinterpret_cast<B8*>(&sm) + q;
      advance_block<T, 8, ORDER, 128, kFusedPad8, kFusedSplit8, GATHER, FLUX>(
          kp, b, tid & 127, *quarter, ahead, &ticket);
    }
  }
}


hipError_t launch_fused(int dtype, int order, bool gather, const KParams& kp, const FusedPlan& pl,
                        int workgroups, hipStream_t s) {
  if (dtype != 1) return hipErrorInvalidValue;  // FP64 edge 16 does not fit in LDS
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanNT), 0, s, kp.d_edge, kp.edge, kp.nblocks, pl,
                     kp.counters);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid(workgroups), block(512);
  if (kp.flux) {
    if (gather) return hipErrorInvalidValue;
    if (kp.flux_acc) {
      if (order == 0) hipLaunchKernelGGL((k_fused<float, 0, false, 2>), grid, block, 0, s, kp, pl);
      else hipLaunchKernelGGL((k_fused<float, 1, false, 2>), grid, block, 0, s, kp, pl);
    } else {
      if (order == 0) hipLaunchKernelGGL((k_fused<float, 0, false, 1>), grid, block, 0, s, kp, pl);
      else hipLaunchKernelGGL((k_fused<float, 1, false, 1>), grid, block, 0, s, kp, pl);
    }
  } else if (gather) {
    if (order == 0) hipLaunchKernelGGL((k_fused<float, 0, true>), grid, block, 0, s, kp, pl);
    else hipLaunchKernelGGL((k_fused<float, 1, true>), grid, block, 0, s, kp, pl);
  } else {
    if (order == 0) hipLaunchKernelGGL((k_fused<float, 0, false>), grid, block, 0, s, kp, pl);
    else hipLaunchKernelGGL((k_fused<float, 1, false>), grid, block, 0, s, kp, pl);
  }
  return hipGetLastError();
}


}  // namespace tvd
