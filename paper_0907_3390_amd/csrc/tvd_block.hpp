// Device code shared by the advance kernels (one translation unit per group
// of instantiations, so that the library builds in parallel): fixed-order
// block reductions, the per-cell diagnostics of an output state, the
// coefficients of a sweep, the pencil sources and sinks of the three sweeps,
// patch-boundary flux records and advance_block, one step of one block by a
// thread group.
//
// Scheme: Schive, Tsai & Chiueh, GAMER, Sec. 2.2 (equations cited in
// tvd_device.hpp); signal speed Eq. (CFL), Sec. 3.4; patch-boundary fluxes
// for the closing step, Sec. 3.1.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "tvd_device.hpp"
#include "tvd_internal.hpp"

namespace tvd {

// ---------------------------------------------------------------------------
// block-level reductions (fixed order, hence deterministic)
// ---------------------------------------------------------------------------

// NT threads with indices tid in [0, NT) reduce; when several groups share a
// workgroup (each with its own `red`), every thread of the workgroup calls.
template <int NT>
__device__ double block_max(double v, double* red, int tid) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  const int w = tid >> 6, l = tid & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (tid == 0) {
    r = red[0];
    for (int i = 1; i < NT / 64; ++i) r = fmax(r, red[i]);
  }
  __syncthreads();
  return r;  // valid in thread 0
}

template <int NT>
__device__ void block_csum(CSum a[kNV], CSum* red, int tid) {
#pragma unroll
  for (int k = 0; k < kNV; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      CSum o{__shfl_xor(a[k].s, off), __shfl_xor(a[k].c, off)};
      a[k] = csum_merge(a[k], o);
    }
  }
  const int w = tid >> 6, l = tid & 63;
  if (l == 0)
    for (int k = 0; k < kNV; ++k) red[w * kNV + k] = a[k];
  __syncthreads();
  if (tid == 0) {
    for (int k = 0; k < kNV; ++k) {
      CSum r = red[k];
      for (int i = 1; i < NT / 64; ++i) r = csum_merge(r, red[i * kNV + k]);
      a[k] = r;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// per-cell diagnostics on an output state (FP64): Eq. (CFL) speed, health
// ---------------------------------------------------------------------------

struct CellDiag {
  double smax;
  unsigned floored, bad;
  CSum sum[kNV];
};

__device__ __forceinline__ void diag_init(CellDiag& d) {
  d.smax = 0.0;
  d.floored = d.bad = 0;
  for (int k = 0; k < kNV; ++k) d.sum[k] = CSum{0.0, 0.0};
}

// Eq. (CFL) signal speed c_s + max |v| of an FP32 state, in FP64.  The
// division and the square root are the hardware reciprocal and reciprocal
// square root estimates (about 2^-23 relative) refined by Newton steps on
// FMAs (two for 1/rho; for the square root one Goldschmidt step and two
// corrections), which lands within a few FP64 ulp of the correctly rounded
// evaluation, far below the FP32 state's own rounding, in about half the
// instructions of IEEE division and square root.  Square roots of values
// below 2^-1000 are taken as 0 (the estimate does not cover denormals).
__device__ __forceinline__ double speed_of_f32_state(const float u[kNV], double gamma,
                                                     double pfloor) {
  const double rho = u[0], mx = u[1], my = u[2], mz = u[3], e = u[4];
  double r = __builtin_amdgcn_rcp(rho);
  double t = __builtin_fma(-rho, r, 1.0);
  r = __builtin_fma(r, t, r);
  t = __builtin_fma(-rho, r, 1.0);
  r = __builtin_fma(r, t, r);
  const double m2 = __builtin_fma(mz, mz, __builtin_fma(my, my, mx * mx));
  const double P = __builtin_fmax((gamma - 1.0) * __builtin_fma(-0.5 * m2, r, e), pfloor);
  const double x = (gamma * P) * r;
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double q = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, q, g);
  h = __builtin_fma(h, q, h);
  double dd = __builtin_fma(-g, g, x);
  g = __builtin_fma(dd, h, g);
  dd = __builtin_fma(-g, g, x);
  g = __builtin_fma(dd, h, g);
  const double cs = x >= 0x1p-1000 ? g : 0.0;
  const double mm = __builtin_fmax(__builtin_fabs(mx), __builtin_fmax(__builtin_fabs(my), __builtin_fabs(mz)));
  return __builtin_fma(mm, r, cs);
}

// Health check of one output cell (in the bulk precision) and, as the
// flags ask, its Eq. (CFL) signal speed (FP64: IEEE division and square
// root for an FP64 state, refined estimates for an FP32 one) and its share
// of the compensated conservation sums.
template <typename T>
__device__ __forceinline__ void diag_cell(CellDiag& d, const T u[kNV], int flags, double gamma,
                                          double pfloor) {
  {
    const T inv = Num<T>::rcp(u[0]);
    const T m2 = Num<T>::fma(u[1], u[1], u[2] * u[2] + u[3] * u[3]);
    const T P = T(gamma - 1.0) * Num<T>::fma(T(-0.5) * m2, inv, u[4]);
    d.floored += P < T(pfloor);
    d.bad += !(u[0] > T(0)) || !__builtin_isfinite(P);
  }
  if constexpr (sizeof(T) == 4) {
    if (flags & kDiagSpeed) d.smax = __builtin_fmax(d.smax, speed_of_f32_state(u, gamma, pfloor));
  } else if (flags & kDiagSpeed) {
    const double rho = u[0], mx = u[1], my = u[2], mz = u[3], e = u[4];
    const double inv = 1.0 / rho;
    const double vx = mx * inv, vy = my * inv, vz = mz * inv;
    const double kin = 0.5 * (mx * vx + my * vy + mz * vz);
    double P = (gamma - 1.0) * (e - kin);
    P = P < pfloor ? pfloor : P;
    const double cs = __builtin_sqrt(gamma * P * inv);
    const double s = cs + fmax(fabs(vx), fmax(fabs(vy), fabs(vz)));
    d.smax = s > d.smax ? s : d.smax;
  }
  if (flags & kDiagSums) {
#pragma unroll
    for (int k = 0; k < kNV; ++k) csum_add(d.sum[k], (double)u[k]);
  }
}

// Reduce the diagnostics of the NT threads working on block b (b < 0: no
// block, the thread group only takes part in the barriers) and publish them.
template <int NT>
__device__ void diag_publish(CellDiag& d, int b, double dh, const KParams& kp, void* scratch,
                             int tid) {
  unsigned fl = d.floored, bad = d.bad;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    fl += __shfl_xor(fl, off);
    bad += __shfl_xor(bad, off);
  }
  if ((tid & 63) == 0 && (fl | bad)) {
    if (fl) atomicAdd(&kp.counters[0], (unsigned long long)fl);
    if (bad) atomicAdd(&kp.counters[1], (unsigned long long)bad);
  }
  if (kp.diag & kDiagSpeed) {
    const double sm = block_max<NT>(d.smax, reinterpret_cast<double*>(scratch), tid);
    if (tid == 0 && b >= 0) kp.ws_smax[b] = sm;
  }
  if (kp.diag & kDiagSums) {
    block_csum<NT>(d.sum, reinterpret_cast<CSum*>(scratch), tid);
    if (tid == 0 && b >= 0) {
      const double w = dh * dh * dh;
      for (int k = 0; k < kNV; ++k) {
        // the block's compensated sum times dh^3 (exact for dyadic dh)
        kp.ws_sums[(size_t)b * 2 * kNV + 2 * k] = d.sum[k].s * w;
        kp.ws_sums[(size_t)b * 2 * kNV + 2 * k + 1] = d.sum[k].c * w;
      }
    }
  }
}

// Workgroups are handed to the 8 XCDs round robin (workgroup i to XCD i % 8).
// Give each XCD a contiguous range of blocks instead, so that neighbouring
// blocks, which share ghost-zone data, meet in the same L2.
__device__ __forceinline__ int xcd_block(int i, int n) {
  constexpr int kXcd = 8;
  const int q = n / kXcd, r = n % kXcd;
  const int k = i % kXcd, t = i / kXcd;
  return k * q + (k < r ? k : r) + t;
}

__device__ __forceinline__ int block_edge(const KParams& kp, int b) {
  return kp.d_edge ? kp.d_edge[b] : kp.edge;
}

template <typename T>
__device__ __forceinline__ Coef<T> make_coef(const KParams& kp, int b, double& dh_out) {
  const double dt = kp.d_dt ? kp.d_dt[b] : kp.dt;
  const double dh = kp.d_dh ? kp.d_dh[b] : kp.dh;
  dh_out = dh;
  const double lam = dt / dh;  // FP64, rounded once to T
  Coef<T> cf;
  // halves of the rounded gamma - 1 and floor: exact, so P*/2 is exactly half
  // of max((gamma - 1)(e - K), p_floor) evaluated in T
  cf.hgamma = T(0.5 * kp.gamma);
  cf.hgm1 = T(0.5) * T(kp.gamma - 1.0);
  cf.hpfloor = T(0.5) * T(kp.pfloor);
  cf.lam = T(lam);
  cf.hlam = T(0.5 * lam);
  return cf;
}

// ---------------------------------------------------------------------------
// batched kernel: sweep 0 streams pencils from HBM, sweeps 1-2 in LDS
// ---------------------------------------------------------------------------
//
// LDS holds the block after sweep 0: only the n interior cells along the
// first sweep axis are kept (n x (n+6) x (n+6) cells per variable), indexed
// by (c0, c1, c2) = coordinates along the first, second and third sweep axes.
// Rows along c0 are XOR-swizzled by (c1 + c2) and rows along c2 padded so
// that the strided accesses of every sweep spread over the LDS banks.

template <int N, int PAD>
struct LdsLayout {
  static constexpr int M = N + 2 * kG;
  static constexpr int P1 = N;              // c1 pitch
  static constexpr int P2 = N * M + PAD;    // c2 pitch
  static constexpr int PLANE = P2 * M;      // one variable
  __device__ static inline int idx(int c0, int c1, int c2) {
    return (c0 ^ ((c1 + c2) & (N - 1))) + P1 * c1 + P2 * c2;
  }
};

// Sweep 0 source: a pencil of the ghosted block in HBM.
template <typename T, int M, int D>
struct GlobalPencil {
  const T* __restrict__ p;  // cell j = 0 of the pencil, variable 0
  __device__ inline void load(int j, T u[kNV]) const {
    constexpr int S = D == 0 ? 1 : D == 1 ? M : M * M;
    constexpr int M3 = M * M * M;
    const T* c = p + j * S;
#pragma unroll
    for (int k = 0; k < kNV; ++k) u[k] = c[gcomp<D>(k) * M3];
  }
};

// Sweep 0 source in gather mode: the pencil crosses three blocks along its
// axis D (0: x or 2: z); p[r] points at the pencil's row in the block at
// offset r-1 along D (the west / own / east interior, or below / own / above).
// Cells j < 3 come from the lower neighbour, j >= N+3 from the upper one.
template <typename T, int N, int D>
struct GatherPencil {
  const T* p[3];
  __device__ inline void load(int j, T u[kNV]) const {
    constexpr int N3 = N * N * N;
    constexpr int S = D == 0 ? 1 : N * N;
    const int r = j < kG ? 0 : (j >= N + kG ? 2 : 1);
    const int jl = j - kG - (r - 1) * N;
    const T* c = p[r] + jl * S;
#pragma unroll
    for (int k = 0; k < kNV; ++k) u[k] = c[gcomp<D>(k) * N3];
  }
};

__device__ __forceinline__ int ghost_region(int c, int n) { return c < kG ? -1 : (c >= n + kG ? 1 : 0); }

// Sweep 0 sink: interior cells along c0 into LDS.
template <typename T, class L, int D>
struct LdsSink0 {
  T* s;
  int c1, c2;
  __device__ inline void store(int i, const T u[kNV]) const {
    const int o = L::idx(i, c1, c2);
#pragma unroll
    for (int k = 0; k < kNV; ++k) s[gcomp<D>(k) * L::PLANE + o] = u[k];
  }
};

// Sweep 1: in-place pencil along c1 at (c0, c2).
template <typename T, class L, int D>
struct LdsPencil1 {
  T* s;
  int c0, c2;
  __device__ inline void load(int j, T u[kNV]) const {
    const int o = L::idx(c0, j, c2);
#pragma unroll
    for (int k = 0; k < kNV; ++k) u[k] = s[gcomp<D>(k) * L::PLANE + o];
  }
  __device__ inline void store(int i, const T u[kNV]) const {
    const int o = L::idx(c0, i + kG, c2);
#pragma unroll
    for (int k = 0; k < kNV; ++k) s[gcomp<D>(k) * L::PLANE + o] = u[k];
  }
};

// Sweep 2: in-place pencil along c2 at (c0, c1).
template <typename T, class L, int D>
struct LdsPencil2 {
  T* s;
  int c0, c1;
  __device__ inline void load(int j, T u[kNV]) const {
    const int o = L::idx(c0, c1, j);
#pragma unroll
    for (int k = 0; k < kNV; ++k) u[k] = s[gcomp<D>(k) * L::PLANE + o];
  }
  __device__ inline void store(int i, const T u[kNV]) const {
    const int o = L::idx(c0, c1, i + kG);
#pragma unroll
    for (int k = 0; k < kNV; ++k) s[gcomp<D>(k) * L::PLANE + o] = u[k];
  }
};

// Sweep 2 sink: finished cells go straight to the block's interior in HBM
// (axis D stride), in global component order, and feed the per-cell
// diagnostics; no copy-out pass through LDS is needed.
template <typename T, int N, int D>
struct GlobalOut {
  T* p;          // cell 0 of the output pencil, variable 0
  CellDiag* dg;
  int diag;
  double gamma, pfloor;
  __device__ inline void store(int i, const T u[kNV]) const {
    constexpr int S = D == 0 ? 1 : D == 1 ? N : N * N;
    constexpr int N3 = N * N * N;
    T ug[kNV];
#pragma unroll
    for (int k = 0; k < kNV; ++k) ug[gcomp<D>(k)] = u[k];
    T* c = p + i * S;
#pragma unroll
    for (int k = 0; k < kNV; ++k) c[k * N3] = ug[k];
    diag_cell<T>(*dg, ug, diag, gamma, pfloor);
  }
  // K consecutive cells i0 .. i0+K-1 of an x pencil (D == 0, stride 1) at
  // once: each variable's run goes out in 16-byte stores, so that a wave
  // writes whole row segments instead of one scattered element per lane.
  // p + i0 must be 16-byte aligned.
  template <int K>
  __device__ inline void store_run(int i0, const T v[K][kNV]) const {
    static_assert(D == 0 && (K * sizeof(T)) % 16 == 0, "runs along x of 16-byte multiples");
    constexpr int N3 = N * N * N;
    constexpr int W = 16 / sizeof(T);  // elements per 16-byte store
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
      T* c = p + i0 + k * N3;
#pragma unroll
      for (int i = 0; i < K; i += W) {
        if constexpr (W == 4) {
          *reinterpret_cast<float4*>(c + i) =
              make_float4(v[i][k], v[i + 1][k], v[i + 2][k], v[i + 3][k]);
        } else {
          *reinterpret_cast<double2*>(c + i) = make_double2(v[i][k], v[i + 1][k]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < K; ++i) diag_cell<T>(*dg, v[i], diag, gamma, pfloor);
  }
};

// Half of a pencil: the interior cells [off, off + N/2) of an LDS pencil,
// computed from its cells [off, off + N/2 + 6).  Two threads sharing a
// pencil this way repeat the flux work of the six cells their halves overlap,
// in exchange for twice the parallelism.  Each half reads cells the other
// half updates, so the halves cannot update in place while they compute:
// their results wait in registers (Held) until the whole workgroup has
// passed a barrier.
template <class A>
struct Shifted {
  A a;
  int off;
  template <typename T>
  __device__ inline void load(int j, T u[kNV]) const { a.load(j + off, u); }
  template <typename T>
  __device__ inline void store(int i, const T u[kNV]) const { a.store(i + off, u); }
};

template <typename T, int NH>
struct Held {
  mutable T v[NH][kNV];
  __device__ inline void store(int i, const T u[kNV]) const {
#pragma unroll
    for (int k = 0; k < kNV; ++k) v[i][k] = u[k];
  }
  template <class A>
  __device__ inline void flush(const A& a) const {
#pragma unroll
    for (int i = 0; i < NH; ++i) a.store(i, v[i]);
  }
};

// A sweep destination that also records the patch-boundary fluxes of its
// pencil: the flux through every interface on a multiple of the patch edge
// goes to the block's flux record (the closing step's input, Sec. 3.1), as
// w H, replacing the record's value or (ACC) added to it, so that the
// records of several sub-steps can be summed with time weights.  fp is the
// record entry of this pencil's face cell on plane 0, variable 0 (null for a
// pencil outside the interior, which records nothing); planes are 5 N^2
// apart, variables N^2, in global component order.  off is the first cell
// of a half pencil: the interface the two halves share is recorded by the
// first half only.
template <typename T, int N, int D, bool ACC, class Dst>
struct FluxTap {
  const Dst& dst;
  T* fp;
  int off;
  T w;
  static constexpr bool kFlux = true;
  __device__ inline void store(int i, const T u[kNV]) const { dst.store(i, u); }
  __device__ inline void flux(int f, const T H[kNV]) const {
    const int g = f + off;
    if (fp != nullptr && g % kPatch == 0 && (f > 0 || off == 0)) {
      T* p = fp + (g / kPatch) * (kNV * N * N);
#pragma unroll
      for (int k = 0; k < kNV; ++k) {
        T* q = p + gcomp<D>(k) * (N * N);
        if constexpr (ACC) *q = *q + w * H[k];
        else *q = w * H[k];
      }
    }
  }
};

// dst itself (FLUX = 0), or dst recording fluxes: writing them (1) or adding
// them to the records (2).
template <int FLUX, typename T, int N, int D, class Dst>
__device__ __forceinline__ decltype(auto) tap(const Dst& dst, T* fp, int off, const KParams& kp) {
  if constexpr (FLUX != 0) {
    return FluxTap<T, N, D, FLUX == 2, Dst>{dst, fp, off, (T)kp.flux_w};
  } else {
    (void)fp;
    (void)off;
    (void)kp;
    return (dst);
  }
}

// Record entry of face cell (a, b) on plane 0 of axis d (null if no record).
template <typename T, int N>
__device__ __forceinline__ T* flux_entry(T* rec, int d, int a, int b) {
  return rec ? rec + d * ((N / kPatch + 1) * kNV * N * N) + a * N + b : nullptr;
}

// LDS a thread group needs for one block: the block after sweep 0, the 27
// neighbour offsets of gather mode and a flag word.
template <typename T, int N, int PAD>
struct BlockLds {
  T s[kNV * LdsLayout<N, PAD>::PLANE];
  int64_t nboff[27];
  int nbad;
};

// One step (one sweep triple) of block b by the NT threads tid = 0..NT-1 of
// a thread group, which may be the whole workgroup or a slice of it; every
// thread of the workgroup calls with the same template arguments, so that
// all of them meet the same barriers.  b < 0 means no block: the group only
// takes part in the barriers.
//
// Sweep 1 (SPLIT bit 0): the first NT/2 threads take whole pencils, the
// remaining pencils are split in halves over the other threads, so that all
// four SIMDs carry about the same number of wave-pencils.
// Sweep 2 (SPLIT bit 1): every pencil is split in halves over all threads.
//
// lookahead (persistent launch, one thread of the workgroup): a work counter
// to draw the next ticket from once the second sweep is done, so that the
// atomic's latency hides behind the third sweep; the ticket goes to *ticket.
template <typename T, int N, int ORDER, int NT, int PAD, int SPLIT, bool GATHER,
          int FLUX = 0>
__device__ __forceinline__ void advance_block(const KParams& kp, int b, int tid,
                                              BlockLds<T, N, PAD>& sm,
                                              unsigned* lookahead = nullptr,
                                              int* ticket = nullptr) {
  using L = LdsLayout<N, PAD>;
  constexpr int M = N + 2 * kG;
  constexpr int M3 = M * M * M;
  constexpr int N3 = N * N * N;
  constexpr int D0 = ORDER == 0 ? 0 : 2;
  constexpr int D1 = 1;
  constexpr int D2 = ORDER == 0 ? 2 : 0;
  T* const S = sm.s;

  bool active = b >= 0;
  T* __restrict__ bout = nullptr;
  double dh = 1.0;
  Coef<T> cf{};
  // FLUX: this block's patch-boundary flux record; face cells (a, b) of an
  // axis are its two other axes, the higher-numbered first
  T* frec = nullptr;
  if (active) {
    bout = reinterpret_cast<T*>(kp.uout) + (kp.out_off ? kp.out_off[b] : (int64_t)b * kNV * N3);
    cf = make_coef<T>(kp, b, dh);
    if constexpr (FLUX)
      frec = reinterpret_cast<T*>(kp.flux) +
             (kp.flux_off ? kp.flux_off[b] : (int64_t)b * flux_record_size(N));
  }

  if constexpr (GATHER) {
    // offsets of the 27 blocks around b; a missing or mismatched neighbour
    // makes the block unadvanceable here (counted, output left untouched)
    if (tid == 0) sm.nbad = 0;
    __syncthreads();
    if (active && tid < 27) {
      const int nb = kp.nbr[27 * (int64_t)b + tid];
      const bool ok = nb >= 0 && nb < kp.nsrc && block_edge(kp, nb) == N;
      if (!ok) atomicAdd(&sm.nbad, 1);
      sm.nboff[tid] = ok ? (kp.out_off ? kp.out_off[nb] : (int64_t)nb * kNV * N3) : 0;
    }
    __syncthreads();
    if (active && sm.nbad) {
      if (tid == 0) atomicAdd(&kp.counters[1], (unsigned long long)N3);
      active = false;
    }
    const T* __restrict__ uin = reinterpret_cast<const T*>(kp.uin);
    // sweep 0 straight from the neighbours' interiors
    for (int p = tid; active && p < M * M; p += NT) {
      int c1, c2;
      if (ORDER == 0) {
        c1 = p % M;
        c2 = p / M;
      } else {
        c2 = p % M;
        c1 = p / M;
      }
      GatherPencil<T, N, D0> src;
      if (ORDER == 0) {  // x pencil at (y, z) = (c1, c2)
        const int ry = ghost_region(c1, N), rz = ghost_region(c2, N);
        const int t = N * (c1 - kG - ry * N) + N * N * (c2 - kG - rz * N);
#pragma unroll
        for (int r = 0; r < 3; ++r) src.p[r] = uin + sm.nboff[r + 3 * (ry + 1) + 9 * (rz + 1)] + t;
      } else {           // z pencil at (x, y) = (c2, c1)
        const int rx = ghost_region(c2, N), ry = ghost_region(c1, N);
        const int t = (c2 - kG - rx * N) + N * (c1 - kG - ry * N);
#pragma unroll
        for (int r = 0; r < 3; ++r) src.p[r] = uin + sm.nboff[(rx + 1) + 3 * (ry + 1) + 9 * r] + t;
      }
      const LdsSink0<T, L, D0> dst{S, c1, c2};
      T* fp = nullptr;
      if constexpr (FLUX) {
        // as for the ghosted source below: x pencils face (z, y) = (c2, c1),
        // z pencils face (y, x) = (c1, c2)
        const bool in = c1 >= kG && c1 < N + kG && c2 >= kG && c2 < N + kG;
        fp = in ? flux_entry<T, N>(frec, D0, (ORDER == 0 ? c2 : c1) - kG,
                                   (ORDER == 0 ? c1 : c2) - kG)
                : nullptr;
      }
      pencil_sweep<T, N>(src, tap<FLUX, T, N, D0>(dst, fp, 0, kp), cf);
    }
  } else {
    const T* __restrict__ bin =
        active ? reinterpret_cast<const T*>(kp.uin) +
                     (kp.in_off ? kp.in_off[b] : (int64_t)b * kNV * M3)
               : nullptr;
    // sweep 0: every (c1, c2) pencil, ghosts of the later axes included
    for (int p = tid; active && p < M * M; p += NT) {
      int c1, c2, start;
      if (ORDER == 0) {  // x pencils; consecutive threads step in y
        c1 = p % M;
        c2 = p / M;
        start = c1 * M + c2 * M * M;
      } else {           // z pencils; consecutive threads step in x
        c2 = p % M;
        c1 = p / M;
        start = c2 + c1 * M;
      }
      const GlobalPencil<T, M, D0> src{bin + start};
      const LdsSink0<T, L, D0> dst{S, c1, c2};
      T* fp = nullptr;
      if constexpr (FLUX) {
        // x pencils: face (z, y) = (c2, c1); z pencils: face (y, x) = (c1, c2)
        const bool in = c1 >= kG && c1 < N + kG && c2 >= kG && c2 < N + kG;
        fp = in ? flux_entry<T, N>(frec, D0, (ORDER == 0 ? c2 : c1) - kG,
                                   (ORDER == 0 ? c1 : c2) - kG)
                : nullptr;
      }
      pencil_sweep<T, N>(src, tap<FLUX, T, N, D0>(dst, fp, 0, kp), cf);
    }
  }
  __syncthreads();
  // sweep 1: interior along c0, all of c2 (y pencils; face (z, x) is
  // (c2, c0) for xyz and (c0, c2) for zyx)
  auto sweep1_flux = [&](int c0, int c2) -> T* {
    if (c2 < kG || c2 >= N + kG) return nullptr;
    return ORDER == 0 ? flux_entry<T, N>(frec, 1, c2 - kG, c0)
                      : flux_entry<T, N>(frec, 1, c0, c2 - kG);
  };
  if constexpr ((SPLIT & 1) != 0) {
    constexpr int F = NT / 2;          // whole pencils
    constexpr int R = N * M - F;       // pencils done in halves
    static_assert(R > 0 && 2 * R <= NT - F, "split layout does not fit the thread group");
    const int t = tid;
    const bool half = active && t >= F && t - F < 2 * R;
    const int p = t < F ? t : F + (t - F) / 2;
    const Shifted<LdsPencil1<T, L, D1>> acc{{S, p % N, p / N}, ((t - F) & 1) * (N / 2)};
    Held<T, N / 2> held;
    T* fp = nullptr;
    if constexpr (FLUX) fp = sweep1_flux(acc.a.c0, acc.a.c2);
    if (active && t < F) {
      pencil_sweep<T, N>(acc.a, tap<FLUX, T, N, D1>(acc.a, fp, 0, kp), cf);
    } else if (half) {
      pencil_sweep<T, N / 2>(acc, tap<FLUX, T, N, D1>(held, fp, acc.off, kp), cf);
    }
    __syncthreads();
    if (half) held.flush(acc);
  } else {
    for (int p = tid; active && p < N * M; p += NT) {
      const LdsPencil1<T, L, D1> acc{S, p % N, p / N};
      T* fp = nullptr;
      if constexpr (FLUX) fp = sweep1_flux(acc.c0, acc.c2);
      pencil_sweep<T, N>(acc, tap<FLUX, T, N, D1>(acc, fp, 0, kp), cf);
    }
  }
  __syncthreads();
  if (lookahead) *ticket = (int)atomicAdd(lookahead, 1u);
  // sweep 2: interior along c0 and c1, results straight to HBM with the
  // per-cell diagnostics (a pencil at (c0, c1) is the column x = c0,
  // y = c1 - 3 along z for xyz, or z = c0, y = c1 - 3 along x for zyx)
  CellDiag dg;
  diag_init(dg);
  auto out_pencil = [&](int c0, int c1) {
    const int y = c1 - kG;
    T* base = ORDER == 0 ? bout + c0 + N * y : bout + N * y + N * N * c0;
    return GlobalOut<T, N, D2>{base, &dg, kp.diag, kp.gamma, kp.pfloor};
  };
  // face of a sweep-2 pencil: (y, x) = (c1, c0) for z pencils, (z, y) =
  // (c0, c1) for x pencils
  auto sweep2_flux = [&](int c0, int c1) -> T* {
    return ORDER == 0 ? flux_entry<T, N>(frec, 2, c1 - kG, c0)
                      : flux_entry<T, N>(frec, 0, c0, c1 - kG);
  };
  if constexpr ((SPLIT & 2) != 0) {
    static_assert(2 * N * N == NT, "sweep-2 halves need one thread each");
    if (active) {
      const int p = tid / 2, off = (tid & 1) * (N / 2);
      const int c0 = p % N, c1 = p / N + kG;
      const Shifted<LdsPencil2<T, L, D2>> src{{S, c0, c1}, off};
      T* fp = nullptr;
      if constexpr (FLUX) fp = sweep2_flux(c0, c1);
      if constexpr (ORDER == 1 && sizeof(T) == 4) {
        // x pencils: the half pencil's cells wait in registers and leave as
        // 16-byte runs along x (along z the lanes' stores already coalesce;
        // FP64 keeps the direct stores, its registers are already full)
        Held<T, N / 2> held;
        pencil_sweep<T, N / 2>(src, tap<FLUX, T, N, D2>(held, fp, off, kp), cf);
        out_pencil(c0, c1).template store_run<N / 2>(off, held.v);
      } else {
        const Shifted<GlobalOut<T, N, D2>> dst{out_pencil(c0, c1), off};
        pencil_sweep<T, N / 2>(src, tap<FLUX, T, N, D2>(dst, fp, off, kp), cf);
      }
    }
  } else {
    for (int p = tid; active && p < N * N; p += NT) {
      const int c0 = p % N, c1 = p / N + kG;
      const LdsPencil2<T, L, D2> src{S, c0, c1};
      T* fp = nullptr;
      if constexpr (FLUX) fp = sweep2_flux(c0, c1);
      const auto dst = out_pencil(c0, c1);
      pencil_sweep<T, N>(src, tap<FLUX, T, N, D2>(dst, fp, 0, kp), cf);
    }
  }
  __syncthreads();
  diag_publish<NT>(dg, active ? b : -1, dh, kp, S, tid);
}

// One workgroup per block, blocks spread over the XCDs in contiguous ranges.
// With mixed edges each edge has its own launch and a workgroup whose block
// has the other edge exits at once.
template <typename T, int N, int ORDER, int NT, int PAD, int SPLIT, bool GATHER,
          int FLUX = 0>
__global__ __launch_bounds__(NT) void k_batched(KParams kp) {
  __shared__ BlockLds<T, N, PAD> sm;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  if (block_edge(kp, b) != N) return;  // uniform over the workgroup
  advance_block<T, N, ORDER, NT, PAD, SPLIT, GATHER, FLUX>(kp, b, threadIdx.x, sm);
}


}  // namespace tvd
