// HIP kernels for gfx950: the batched, persistent and plain relaxing-TVD
// advance (optionally writing patch-boundary flux records), the CFL signal
// speed, compensated conservation sums, their finalisation, the device time
// step, the sibling and coarse-fine ghost-zone fills, and the closing step of
// a level pair (restriction and coarse-fine flux correction).
//
// Scheme: Schive, Tsai & Chiueh, GAMER, Sec. 2.2 (equations cited in
// tvd_device.hpp); signal speed Eq. (CFL), Sec. 3.4; AMR ghost zones and the
// closing step, Secs. 2.1, 2.2 and 3.1.
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

// Health check of one output cell (in the bulk precision) and, as the
// flags ask, its Eq. (CFL) signal speed (FP64, one division) and its share
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
  if (flags & kDiagSpeed) {
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
      const bool ok = nb >= 0 && nb < kp.nblocks && block_edge(kp, nb) == N;
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
      pencil_sweep<T, N>(src, dst, cf);
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

// ---------------------------------------------------------------------------
// plain FP64 kernel: one workgroup per 8^3 block, whole ghosted block in LDS,
// the three sweeps in place with the region rule
// ---------------------------------------------------------------------------

constexpr int kPlainN = 8;
constexpr int kPlainM = kPlainN + 2 * kG;
constexpr int kPlainM3 = kPlainM * kPlainM * kPlainM;
constexpr int kPlainNT = 256;

template <int D>
struct PlainPencil {
  double* s;
  int base;  // cell j = 0 of the pencil
  static constexpr int S = D == 0 ? 1 : D == 1 ? kPlainM : kPlainM * kPlainM;
  __device__ inline void load(int j, double u[kNV]) const {
#pragma unroll
    for (int k = 0; k < kNV; ++k) u[k] = s[gcomp<D>(k) * kPlainM3 + base + j * S];
  }
  __device__ inline void store(int i, const double u[kNV]) const {
#pragma unroll
    for (int k = 0; k < kNV; ++k) s[gcomp<D>(k) * kPlainM3 + base + (i + kG) * S] = u[k];
  }
};

// Sweep along D; the transverse axis A is kept whole (ghosts included) when
// LATER_A is set, i.e. when A is swept later in this step, else restricted
// to the interior.  The two transverse axes are (D+1)%3 and (D+2)%3.
template <int D, bool LATER1, bool LATER2>
__device__ void plain_sweep(double* s, const Coef<double>& cf) {
  constexpr int A1 = (D + 1) % 3, A2 = (D + 2) % 3;
  constexpr int lo1 = LATER1 ? 0 : kG, n1 = LATER1 ? kPlainM : kPlainN;
  constexpr int lo2 = LATER2 ? 0 : kG, n2 = LATER2 ? kPlainM : kPlainN;
  constexpr int st[3] = {1, kPlainM, kPlainM * kPlainM};
  for (int p = threadIdx.x; p < n1 * n2; p += kPlainNT) {
    const int a1 = lo1 + p % n1, a2 = lo2 + p / n1;
    const PlainPencil<D> acc{s, a1 * st[A1] + a2 * st[A2]};
    pencil_sweep<double, kPlainN>(acc, acc, cf);
  }
}

template <int ORDER>
__global__ __launch_bounds__(kPlainNT) void k_plain_f64(KParams kp) {
  constexpr int N3 = kPlainN * kPlainN * kPlainN;
  __shared__ double S[kNV * kPlainM3];
  const int b = blockIdx.x;
  const double* __restrict__ bin = reinterpret_cast<const double*>(kp.uin) +
                                   (kp.in_off ? kp.in_off[b] : (int64_t)b * kNV * kPlainM3);
  double* __restrict__ bout = reinterpret_cast<double*>(kp.uout) +
                              (kp.out_off ? kp.out_off[b] : (int64_t)b * kNV * N3);
  double dh;
  const Coef<double> cf = make_coef<double>(kp, b, dh);
  for (int i = threadIdx.x; i < kNV * kPlainM3; i += kPlainNT) S[i] = bin[i];
  __syncthreads();
  if (ORDER == 0) {
    plain_sweep<0, true, true>(S, cf);    // x: y, z later
    __syncthreads();
    plain_sweep<1, true, false>(S, cf);   // y: z later, x earlier
    __syncthreads();
    plain_sweep<2, false, false>(S, cf);  // z: x, y earlier
  } else {
    plain_sweep<2, true, true>(S, cf);    // z: x, y later
    __syncthreads();
    plain_sweep<1, false, true>(S, cf);   // y: z earlier, x later
    __syncthreads();
    plain_sweep<0, false, false>(S, cf);  // x: y, z earlier
  }
  __syncthreads();
  CellDiag dg;
  diag_init(dg);
  for (int i = threadIdx.x; i < N3; i += kPlainNT) {
    const int x = i % kPlainN, y = (i / kPlainN) % kPlainN, z = i / (kPlainN * kPlainN);
    const int o = (x + kG) + kPlainM * ((y + kG) + kPlainM * (z + kG));
    double u[kNV];
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
      u[k] = S[k * kPlainM3 + o];
      bout[k * N3 + i] = u[k];
    }
    diag_cell<double>(dg, u, kp.diag, kp.gamma, kp.pfloor);
  }
  __syncthreads();
  diag_publish<kPlainNT>(dg, b, dh, kp, S, threadIdx.x);
}

// ---------------------------------------------------------------------------
// standalone signal speed and conservation sums (one workgroup per block)
// ---------------------------------------------------------------------------

constexpr int kRedNT = 256;

template <typename T>
__global__ __launch_bounds__(kRedNT) void k_block_diag(KParams kp, int layout) {
  __shared__ CSum red[kRedNT / 64 * kNV];
  const int b = blockIdx.x;
  const int n = block_edge(kp, b);
  const int m = layout == 0 ? n + 2 * kG : n;
  const int g = layout == 0 ? kG : 0;
  const int64_t m3 = (int64_t)m * m * m;
  const T* base = reinterpret_cast<const T*>(kp.uin) +
                  (layout == 0 ? (kp.in_off ? kp.in_off[b] : (int64_t)b * kNV * m3)
                               : (kp.out_off ? kp.out_off[b] : (int64_t)b * kNV * m3));
  const double dh = kp.d_dh ? kp.d_dh[b] : kp.dh;
  CellDiag dg;
  diag_init(dg);
  const int n3 = n * n * n;
  for (int i = threadIdx.x; i < n3; i += kRedNT) {
    const int x = i % n, y = (i / n) % n, z = i / (n * n);
    const int64_t o = (x + g) + (int64_t)m * ((y + g) + (int64_t)m * (z + g));
    T u[kNV];
#pragma unroll
    for (int k = 0; k < kNV; ++k) u[k] = base[k * m3 + o];
    diag_cell<T>(dg, u, kp.diag, kp.gamma, kp.pfloor);
  }
  if (kp.diag & kDiagSpeed) {
    const double sm = block_max<kRedNT>(dg.smax, reinterpret_cast<double*>(red), threadIdx.x);
    if (threadIdx.x == 0) kp.ws_smax[b] = sm;
  } else {
    block_csum<kRedNT>(dg.sum, red, threadIdx.x);
    if (threadIdx.x == 0) {
      const double w = dh * dh * dh;
      for (int k = 0; k < kNV; ++k) {
        kp.ws_sums[(size_t)b * 2 * kNV + 2 * k] = dg.sum[k].s * w;
        kp.ws_sums[(size_t)b * 2 * kNV + 2 * k + 1] = dg.sum[k].c * w;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// finalisation: one workgroup, fixed partition and fixed tree
// ---------------------------------------------------------------------------

constexpr int kFinNT = 1024;

__global__ __launch_bounds__(kFinNT) void k_finalize_max(const double* ws, int n, double* out) {
  __shared__ double red[kFinNT / 64];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += kFinNT) m = fmax(m, ws[i]);
  const double r = block_max<kFinNT>(m, red, threadIdx.x);
  if (threadIdx.x == 0) out[0] = r;
}

__global__ __launch_bounds__(kFinNT) void k_finalize_sums(const double* ws, int n, double* out) {
  __shared__ CSum red[kFinNT / 64 * kNV];
  CSum a[kNV];
  for (int k = 0; k < kNV; ++k) a[k] = CSum{0.0, 0.0};
  // contiguous chunk per thread, in block order
  const int per = (n + kFinNT - 1) / kFinNT;
  const int lo = threadIdx.x * per;
  const int hi = min(n, lo + per);
  for (int b = lo; b < hi; ++b)
    for (int k = 0; k < kNV; ++k)
      a[k] = csum_merge(a[k], CSum{ws[(size_t)b * 2 * kNV + 2 * k], ws[(size_t)b * 2 * kNV + 2 * k + 1]});
  block_csum<kFinNT>(a, red, threadIdx.x);
  if (threadIdx.x == 0)
    for (int k = 0; k < kNV; ++k) out[k] = a[k].s + a[k].c;
}

__global__ void k_dt_from_speed(KParams kp, const double* smax, double cfl, double* dt_out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= kp.nblocks) return;
  const double dh = kp.d_dh ? kp.d_dh[b] : kp.dh;
  dt_out[b] = cfl * dh / smax[0];
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// sibling ghost fill
// ---------------------------------------------------------------------------

constexpr int kFillNT = 256;

template <typename T>
__global__ __launch_bounds__(kFillNT) void k_fill_ghosts(KParams kp, const int32_t* nbr,
                                                        int chunks) {
  const int b = blockIdx.x / chunks;
  const int chunk = blockIdx.x % chunks;
  const int n = block_edge(kp, b);
  const int m = n + 2 * kG;
  const int m3 = m * m * m;
  const int n3 = n * n * n;
  const int cell = chunk * kFillNT + threadIdx.x;
  if (cell >= m3) return;
  const int x = cell % m, y = (cell / m) % m, z = cell / (m * m);
  const int rx = x < kG ? -1 : (x >= n + kG ? 1 : 0);
  const int ry = y < kG ? -1 : (y >= n + kG ? 1 : 0);
  const int rz = z < kG ? -1 : (z >= n + kG ? 1 : 0);
  const int src = nbr[27 * b + (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)];
  if (src < 0) return;
  if (src >= kp.nblocks || block_edge(kp, src) != n) {
    atomicAdd(&kp.counters[1], 1ull);
    return;
  }
  const int sx = x - kG - rx * n, sy = y - kG - ry * n, sz = z - kG - rz * n;
  const int so = sx + n * (sy + n * sz);
  const T* s = reinterpret_cast<const T*>(kp.uout) +
               (kp.out_off ? kp.out_off[src] : (int64_t)src * kNV * n3);
  T* d = reinterpret_cast<T*>(const_cast<void*>(kp.uin)) +
         (kp.in_off ? kp.in_off[b] : (int64_t)b * kNV * m3);
#pragma unroll
  for (int k = 0; k < kNV; ++k) d[(int64_t)k * m3 + cell] = s[(int64_t)k * n3 + so];
}

// ---------------------------------------------------------------------------
// coarse-fine ghost fill: sibling copy, else Min-Mod limited linear
// interpolation from the level one coarser (Sec. 2.2)
// ---------------------------------------------------------------------------

// Min-Mod limiter: 0 unless a and b are both positive or both negative, then
// the one of smaller magnitude (b on a tie).
template <typename T>
__device__ __forceinline__ T minmod(T a, T b) {
  const bool same = (a > T(0) && b > T(0)) || (a < T(0) && b < T(0));
  return same ? (Num<T>::abs(a) < Num<T>::abs(b) ? a : b) : T(0);
}

// Coarse blocks are 8^3 patches; cin points at the coarse interiors, cnbr at
// the 27 coarse patches around the fine block's parent.  Coarse index i
// (per axis, relative to the parent's corner) lies in region i >> 3.
template <typename T>
struct CoarseNbhd {
  const T* cin;
  const int64_t* coff;  // coarse out offsets (or null: dense)
  const int32_t* cnbr;  // 27 entries of this fine block
  int ncoarse;
  // Branch-free, so that the seven reads of a cell's stencil issue together:
  // a cell outside the 27 patches or a missing patch reads block 0 instead
  // (ncoarse >= 1 is checked by the caller) and reports false.
  __device__ inline bool get(int ix, int iy, int iz, T u[kNV]) const {
    const int qx = ix >> 3, qy = iy >> 3, qz = iz >> 3;
    const bool in = qx >= -1 && qx <= 1 && qy >= -1 && qy <= 1 && qz >= -1 && qz <= 1;
    const int cb = cnbr[in ? (qx + 1) + 3 * (qy + 1) + 9 * (qz + 1) : 13];
    const bool ok = in && cb >= 0 && cb < ncoarse;
    const int cs = ok ? cb : 0;
    const T* c = cin + (coff ? coff[cs] : (int64_t)cs * kNV * 512) + (ix & 7) + 8 * (iy & 7) +
                 64 * (iz & 7);
#pragma unroll
    for (int k = 0; k < kNV; ++k) u[k] = c[k * 512];
    return ok;
  }
};

// Ghosted cells per thread in the coarse-fine fill: a thread resolves the
// source of each of its cells first and then issues all their sibling reads
// together, so the chain of table lookups before a copy is paid once per
// kFillCPT cells.
constexpr int kFillCPT = 4;

// Interpolated ghost cell (x, y, z) of fine block b: Min-Mod limited linear
// interpolation from the coarse level.
template <typename T>
__device__ __forceinline__ void fill_interp(const KParams& kp, int b, int x, int y, int z,
                                            T* d, int64_t m3, int cell, const T* cin,
                                            const int64_t* coff, int ncoarse,
                                            const int32_t* cnbr, const int32_t* corigin) {
  if (ncoarse <= 0) {
    atomicAdd(&kp.counters[1], 1ull);
    return;
  }
  // fine index relative to the parent's corner, in fine cells
  const int fx = 2 * corigin[3 * b + 0] + x - kG;
  const int fy = 2 * corigin[3 * b + 1] + y - kG;
  const int fz = 2 * corigin[3 * b + 2] + z - kG;
  const int cx = fx >> 1, cy = fy >> 1, cz = fz >> 1;  // floor
  const T q = T(0.25);
  const T dx = (fx & 1) ? q : -q, dy = (fy & 1) ? q : -q, dz = (fz & 1) ? q : -q;
  const CoarseNbhd<T> cn{cin, coff, cnbr + 27 * (int64_t)b, ncoarse};
  // all seven stencil reads first (no short-circuit between them)
  T u[kNV], xp[kNV], xm[kNV], yp[kNV], ym[kNV], zp[kNV], zm[kNV], out[kNV];
  bool ok = cn.get(cx, cy, cz, u);
  ok = cn.get(cx + 1, cy, cz, xp) & ok;
  ok = cn.get(cx - 1, cy, cz, xm) & ok;
  ok = cn.get(cx, cy + 1, cz, yp) & ok;
  ok = cn.get(cx, cy - 1, cz, ym) & ok;
  ok = cn.get(cx, cy, cz + 1, zp) & ok;
  ok = cn.get(cx, cy, cz - 1, zm) & ok;
  // x, then y, then z (the order of the sum)
#pragma unroll
  for (int k = 0; k < kNV; ++k) {
    out[k] = u[k];
    out[k] = out[k] + dx * minmod(xp[k] - u[k], u[k] - xm[k]);
    out[k] = out[k] + dy * minmod(yp[k] - u[k], u[k] - ym[k]);
    out[k] = out[k] + dz * minmod(zp[k] - u[k], u[k] - zm[k]);
  }
  if (!ok) {
    atomicAdd(&kp.counters[1], 1ull);
    return;
  }
#pragma unroll
  for (int k = 0; k < kNV; ++k) d[(int64_t)k * m3 + cell] = out[k];
}

// One workgroup per kFillNT * kFillCPT ghosted cells of a fine block; chunks
// workgroups per block.  A cell is a sibling copy when the block's neighbour
// table names a block for its region, else interpolated from the coarse
// level.
template <typename T>
__global__ __launch_bounds__(kFillNT) void k_fill_ghosts_amr(KParams kp, const int32_t* nbr,
                                                            int chunks, const T* cin,
                                                            const int64_t* coff, int ncoarse,
                                                            const int32_t* cnbr,
                                                            const int32_t* corigin) {
  const int b = blockIdx.x / chunks;
  const int chunk = blockIdx.x % chunks;
  const int n = block_edge(kp, b);
  const int m = n + 2 * kG;
  const int m3 = m * m * m;
  const int n3 = n * n * n;
  T* d = reinterpret_cast<T*>(const_cast<void*>(kp.uin)) +
         (kp.in_off ? kp.in_off[b] : (int64_t)b * kNV * m3);
  const T* own = reinterpret_cast<const T*>(kp.uout) +
                 (kp.out_off ? kp.out_off[b] : (int64_t)b * kNV * n3);
  // 0: no cell, 1: sibling copy from sp[i], 2: interpolated
  int kind[kFillCPT];
  const T* sp[kFillCPT];
#pragma unroll
  for (int i = 0; i < kFillCPT; ++i) {
    const int cell = (chunk * kFillCPT + i) * kFillNT + threadIdx.x;
    kind[i] = 0;
    sp[i] = own;  // a valid address for the unconditional reads below
    if (cell < m3) {
      const int x = cell % m, y = (cell / m) % m, z = cell / (m * m);
      const int rx = x < kG ? -1 : (x >= n + kG ? 1 : 0);
      const int ry = y < kG ? -1 : (y >= n + kG ? 1 : 0);
      const int rz = z < kG ? -1 : (z >= n + kG ? 1 : 0);
      const int src = nbr[27 * b + (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)];
      if (src < 0) {
        kind[i] = 2;
      } else if (src >= kp.nblocks || block_edge(kp, src) != n) {
        atomicAdd(&kp.counters[1], 1ull);
      } else {
        const int sx = x - kG - rx * n, sy = y - kG - ry * n, sz = z - kG - rz * n;
        sp[i] = reinterpret_cast<const T*>(kp.uout) +
                (kp.out_off ? kp.out_off[src] : (int64_t)src * kNV * n3) +
                (sx + n * (sy + n * sz));
        kind[i] = 1;
      }
    }
  }
  T v[kFillCPT][kNV];
#pragma unroll
  for (int i = 0; i < kFillCPT; ++i)
#pragma unroll
    for (int k = 0; k < kNV; ++k) v[i][k] = sp[i][(int64_t)k * n3];
#pragma unroll
  for (int i = 0; i < kFillCPT; ++i) {
    const int cell = (chunk * kFillCPT + i) * kFillNT + threadIdx.x;
    if (kind[i] == 1) {
#pragma unroll
      for (int k = 0; k < kNV; ++k) d[(int64_t)k * m3 + cell] = v[i][k];
    }
  }
#pragma unroll 1
  for (int i = 0; i < kFillCPT; ++i) {
    if (kind[i] != 2) continue;
    const int cell = (chunk * kFillCPT + i) * kFillNT + threadIdx.x;
    const int x = cell % m, y = (cell / m) % m, z = cell / (m * m);
    fill_interp<T>(kp, b, x, y, z, d, m3, cell, cin, coff, ncoarse, cnbr, corigin);
  }
}

// ---------------------------------------------------------------------------
// closing step of a level pair (Sec. 2.1, step 3; Sec. 3.1)
// ---------------------------------------------------------------------------
//
// Both kernels take the coarse level as ck (its interior blocks, read and
// written, at ck.uout / ck.out_off; its flux records at ck.flux /
// ck.flux_off) and the fine level as fk (interior blocks read at fk.uin with
// the interior offsets fk.out_off; flux records at fk.flux / fk.flux_off).
// A row that names a block out of range, an edge other than 8 or 16, or a
// region outside its blocks is skipped and its cells are counted as
// non-physical.

constexpr int kCloseNT = 256;

template <typename T>
__device__ __forceinline__ const T* interior_of(const KParams& k, const void* base, int b, int e) {
  return static_cast<const T*>(base) + (k.out_off ? k.out_off[b] : (int64_t)b * kNV * e * e * e);
}

template <typename T>
__device__ __forceinline__ const T* record_of(const KParams& k, int b, int e) {
  return static_cast<const T*>(k.flux) + (k.flux_off ? k.flux_off[b] : (int64_t)b * flux_record_size(e));
}

__device__ __forceinline__ bool edge_ok(int e) { return e == 8 || e == 16; }

// Restriction of one row (f, c, ox, oy, oz) by the calling workgroup: the
// (e_f/2)^3 coarse cells of block c at offset (ox, oy, oz) become the mean of
// their eight children in fine block f, summed in the order (dz, dy, dx) =
// 000, 001, .., 111, then times 1/8.
template <typename T>
__device__ __forceinline__ void restrict_row(const KParams& ck, const KParams& fk, const int32_t* r) {
  const int f = r[0], c = r[1], ox = r[2], oy = r[3], oz = r[4];
  const bool fin = f >= 0 && f < fk.nblocks, cin = c >= 0 && c < ck.nblocks;
  const int ef = fin ? block_edge(fk, f) : 0, ec = cin ? block_edge(ck, c) : 0;
  const int h = ef / 2;
  const bool ok = fin && cin && edge_ok(ef) && edge_ok(ec) && ox >= 0 && oy >= 0 && oz >= 0 &&
                  ox + h <= ec && oy + h <= ec && oz + h <= ec;
  if (!ok) {
    if (threadIdx.x == 0) atomicAdd(&ck.counters[1], edge_ok(ef) ? (unsigned long long)h * h * h : 1ull);
    return;
  }
  const T* u = interior_of<T>(fk, fk.uin, f, ef);
  T* v = const_cast<T*>(interior_of<T>(ck, ck.uout, c, ec));
  const int h3 = h * h * h;
  const int64_t ef3 = (int64_t)ef * ef * ef, ec3 = (int64_t)ec * ec * ec;
  const T eighth = T(0.125);
  if ((reinterpret_cast<uintptr_t>(u) & 15) == 0) {
    // 16-byte loads along x: W = 16 / sizeof(T) children per row load,
    // W / 2 coarse cells per item; same sums in the same order
    constexpr int W = 16 / sizeof(T), O = W / 2;
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    const int hx = h / O;
    const int items = kNV * h * h * hx;
    for (int i = threadIdx.x; i < items; i += blockDim.x) {
      const int k = i / (h * h * hx), rem = i % (h * h * hx);
      const int xq = rem % hx, y = (rem / hx) % h, z = rem / (hx * h);
      const T* p = u + k * ef3 + W * xq + ef * (2 * y + ef * (2 * z));
      T a[W], b[W], cz[W], d[W];
      *reinterpret_cast<V*>(a) = *reinterpret_cast<const V*>(p);                // dz 0, dy 0
      *reinterpret_cast<V*>(b) = *reinterpret_cast<const V*>(p + ef);           // dz 0, dy 1
      *reinterpret_cast<V*>(cz) = *reinterpret_cast<const V*>(p + ef * ef);     // dz 1, dy 0
      *reinterpret_cast<V*>(d) = *reinterpret_cast<const V*>(p + ef * ef + ef); // dz 1, dy 1
      T* q = v + k * ec3 + (ox + O * xq) + ec * ((oy + y) + (int64_t)ec * (oz + z));
#pragma unroll
      for (int o = 0; o < O; ++o) {
        T sum = a[2 * o];
        sum = sum + a[2 * o + 1];
        sum = sum + b[2 * o];
        sum = sum + b[2 * o + 1];
        sum = sum + cz[2 * o];
        sum = sum + cz[2 * o + 1];
        sum = sum + d[2 * o];
        sum = sum + d[2 * o + 1];
        q[o] = sum * eighth;
      }
    }
    return;
  }
  for (int i = threadIdx.x; i < kNV * h3; i += blockDim.x) {
    const int k = i / h3, cell = i % h3;
    const int x = cell % h, y = (cell / h) % h, z = cell / (h * h);
    const T* p = u + k * ef3 + 2 * x + ef * (2 * y + ef * (2 * z));
    const int sy = ef, sz = ef * ef;
    T sum = p[0];
    sum = sum + p[1];
    sum = sum + p[sy];
    sum = sum + p[sy + 1];
    sum = sum + p[sz];
    sum = sum + p[sz + 1];
    sum = sum + p[sz + sy];
    sum = sum + p[sz + sy + 1];
    v[k * ec3 + (ox + x) + ec * ((oy + y) + (int64_t)ec * (oz + z))] = sum * eighth;
  }
}

// Flux correction of one row (c, d, s, qc, oa, ob, f, qf) by the calling
// workgroup.  Face cells (oa + a, ob + b), a, b < e_f/2, of plane qc along
// axis d of coarse block c are covered by the 2 x 2 fine face cells
// (2a.., 2b..) of plane qf of fine block f; the coarse cell on the s side of
// the plane (s = 1: below it, the interface is its + face) takes
// u + lam (H_c - H_f), or u - lam (H_c - H_f) for s = 0, with lam =
// dt_c / dh_c and H_f the mean of the four fine fluxes summed
// ((f00 + f01) + f10) + f11.
template <typename T>
__device__ __forceinline__ void correct_row(const KParams& ck, const KParams& fk, const int32_t* r) {
  const int c = r[0], d = r[1], s = r[2], qc = r[3], oa = r[4], ob = r[5], f = r[6], qf = r[7];
  const bool fin = f >= 0 && f < fk.nblocks, cin = c >= 0 && c < ck.nblocks;
  const int ef = fin ? block_edge(fk, f) : 0, ec = cin ? block_edge(ck, c) : 0;
  const int h = ef / 2;
  const bool ok = fin && cin && edge_ok(ef) && edge_ok(ec) && d >= 0 && d < 3 && (s == 0 || s == 1) &&
                  (s ? qc >= 1 && qc <= ec / kPatch : qc >= 0 && qc < ec / kPatch) && qf >= 0 &&
                  qf <= ef / kPatch && oa >= 0 && ob >= 0 && oa + h <= ec && ob + h <= ec;
  if (!ok) {
    if (threadIdx.x == 0) atomicAdd(&ck.counters[1], edge_ok(ef) ? (unsigned long long)h * h : 1ull);
    return;
  }
  T* u = const_cast<T*>(interior_of<T>(ck, ck.uout, c, ec));
  const T* Hc = record_of<T>(ck, c, ec) + (int64_t)(d * (ec / kPatch + 1) + qc) * kNV * ec * ec;
  const T* Hf = record_of<T>(fk, f, ef) + (int64_t)(d * (ef / kPatch + 1) + qf) * kNV * ef * ef;
  const double dt = ck.d_dt ? ck.d_dt[c] : ck.dt, dh = ck.d_dh ? ck.d_dh[c] : ck.dh;
  const T lam = (T)(dt / dh);
  const T quarter = T(0.25);
  // cell strides along d and along the face axes (the higher-numbered first)
  const int st[3] = {1, ec, ec * ec};
  const int dhi = d == 0 ? 2 : d == 1 ? 2 : 1, dlo = d == 0 ? 1 : 0;
  const int i_d = s ? kPatch * qc - 1 : kPatch * qc;
  const int64_t ec3 = (int64_t)ec * ec * ec;
  for (int i = threadIdx.x; i < kNV * h * h; i += blockDim.x) {
    const int k = i / (h * h), a = (i / h) % h, b = i % h;
    const T* F = Hf + k * ef * ef + (2 * a) * ef + 2 * b;
    const T hf = (((F[0] + F[1]) + F[ef]) + F[ef + 1]) * quarter;
    const T t = Hc[k * ec * ec + (oa + a) * ec + (ob + b)] - hf;
    T* p = u + k * ec3 + i_d * st[d] + (oa + a) * st[dhi] + (ob + b) * st[dlo];
    *p = s ? *p + lam * t : *p - lam * t;
  }
}

// One workgroup per restriction row.
template <typename T>
__global__ __launch_bounds__(kCloseNT) void k_restrict(KParams ck, KParams fk, const int32_t* rows) {
  restrict_row<T>(ck, fk, rows + 5 * (int64_t)blockIdx.x);
}

// One workgroup per face row of one pass (rows of one pass never share a
// cell).
template <typename T>
__global__ __launch_bounds__(kCloseNT) void k_flux_correct(KParams ck, KParams fk, const int32_t* rows) {
  correct_row<T>(ck, fk, rows + 8 * (int64_t)blockIdx.x);
}

// The closing of a level pair in one launch: workgroup g < ngroups applies
// the face rows [start[g], start[g+1]) of one coarse block in pass order,
// with a barrier wherever the pass changes, so that a cell on several
// interfaces takes its corrections in the order x-, x+, y-, y+, z-, z+; the
// workgroups after them restrict one row each.  The face groups come first
// so that their short dependent chains start early and overlap the
// bandwidth-bound restriction.  A group whose rows name different coarse
// blocks, or whose range leaves [0, nf), is skipped and counted as
// non-physical.
template <typename T>
__global__ __launch_bounds__(kCloseNT) void k_close_level(KParams ck, KParams fk,
                                                          const int32_t* rrows, int ngroups,
                                                          const int32_t* frows, int nf,
                                                          const int32_t* start) {
  if ((int)blockIdx.x >= ngroups) {
    restrict_row<T>(ck, fk, rrows + 5 * (int64_t)(blockIdx.x - ngroups));
    return;
  }
  const int g = blockIdx.x;
  const int lo = start[g], hi = start[g + 1];
  bool ok = lo >= 0 && lo <= hi && hi <= nf;
  for (int r = lo; ok && r < hi; ++r) ok = frows[8 * (int64_t)r] == frows[8 * (int64_t)lo];
  if (!ok) {
    if (threadIdx.x == 0) atomicAdd(&ck.counters[1], 1ull);
    return;
  }
  int prev = -1;
  for (int r = lo; r < hi; ++r) {
    const int32_t* row = frows + 8 * (int64_t)r;
    const int pass = 2 * row[1] + row[2];
    if (pass != prev) {
      __syncthreads();  // the previous pass's corrections are in place
      prev = pass;
    }
    correct_row<T>(ck, fk, row);
  }
}

// ---------------------------------------------------------------------------
// Poisson equation on patch groups: red-black SOR (Sec. 2.3; Sec. 3.2)
// ---------------------------------------------------------------------------
//
// One workgroup of 128 threads per patch group.  The whole 18^3 potential
// (16^3 cells and the Dirichlet ghost layer) lives in LDS; the paper's split
// of odd and even cells between shared memory and registers answered a
// 16 KB shared memory and is not needed in 160 KB.  Thread (xp, y) owns the
// x pair of columns 2xp, 2xp + 1 at row y and keeps both (ghost ends
// included) and their source terms in registers: in every z slice exactly
// one of the two cells has the parity being updated, so each thread updates
// one cell per slice and half-step, its z and in-pair x neighbours from
// registers, its y neighbours and outer x neighbour from LDS, and writes the
// new value to both.  Residual (Eq. Residual) and update (Eq. SOR) in the
// order x+1, y+1, z+1, x-1, y-1, z-1, minus 6 phi, minus the source; phi +
// (omega/6) R; no contraction.  The one-norms of the residuals and of phi
// are reduced in FP64 after every iteration for the stopping rule.

constexpr int kSorN = 16, kSorM = kSorN + 2, kSorNT = 128;

struct SorParams {
  const void* phi_in;   // [G][18^3]
  const void* rho;      // [G][16^3]
  void* phi_out;        // [G][16^3]
  const double* d_dh;   // [G] or null
  double dh, G, omega, tol;
  int ngroups, min_iter, max_iter;
  int32_t* iters;       // [G] or null
  double* resid;        // [G] or null
};

template <typename T>
__global__ __launch_bounds__(kSorNT) void k_sor(SorParams p) {
  constexpr int N = kSorN, M = kSorM, M3 = M * M * M, N3 = N * N * N;
  constexpr int CH = sizeof(T) == 4 ? 8 : 1;  // slices whose loads are issued together (FP64: registers are full)
  __shared__ T s[M3];
  __shared__ double red[2][kSorNT / 64];
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const T* in = static_cast<const T*>(p.phi_in) + (int64_t)g * M3;
  const T* rho = static_cast<const T*>(p.rho) + (int64_t)g * N3;
  for (int i = tid; i < M3; i += kSorNT) s[i] = in[i];
  const int xp = tid % (N / 2), y = tid / (N / 2);
  const int x0 = 2 * xp;  // interior x of column 0 (column 1 is x0 + 1)
  const double dh = p.d_dh ? p.d_dh[g] : p.dh;
  const T fac = (T)(4.0 * 3.141592653589793 * p.G * (dh * dh));
  const T w6 = (T)(p.omega / 6.0);
  const T six = T(6);
  T c0[M], c1[M], q0[N], q1[N];
#pragma unroll
  for (int z = 0; z < N; ++z) {
    const T* r = rho + x0 + N * (y + N * z);
    q0[z] = fac * r[0];
    q1[z] = fac * r[1];
  }
  double src_norm = 0.0;
#pragma unroll
  for (int z = 0; z < N; ++z) src_norm += (double)(q0[z] < T(0) ? -q0[z] : q0[z]) +
                                          (double)(q1[z] < T(0) ? -q1[z] : q1[z]);
  __syncthreads();
  // LDS index of ghosted cell (x, y, z), interior coordinates (-1 .. 16)
  auto at = [&](int x, int yy, int z) { return (x + 1) + M * ((yy + 1) + M * (z + 1)); };
#pragma unroll
  for (int z = 0; z < M; ++z) {
    c0[z] = s[at(x0, y, z - 1)];
    c1[z] = s[at(x0 + 1, y, z - 1)];
  }
  // reduce two doubles over the workgroup in one pass (every thread gets
  // both sums, in the same order)
  auto block_sum2 = [&](double& a, double& b) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_xor(a, off);
      b += __shfl_xor(b, off);
    }
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = a;
      red[1][tid >> 6] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
#pragma unroll
    for (int w = 0; w < kSorNT / 64; ++w) {
      a += red[0][w];
      b += red[1][w];
    }
    __syncthreads();  // read before the next reduction writes
  };
  double unused = 0.0;
  block_sum2(src_norm, unused);
  int it = 0;
  double rnorm = 0.0;
  for (;;) {
    double racc = 0.0;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      // slices in chunks of CH: the chunk's LDS neighbours (all of the other
      // parity, which this half-step never writes) are loaded first, so the
      // loads overlap instead of each waiting behind the previous slice's
      // store
#pragma unroll
      for (int z0 = 0; z0 < N; z0 += CH) {
        T xo[CH], yu[CH], yd[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int z = z0 + k;
          const bool one = ((x0 + y + z + half) & 1) != 0;
          const int x = x0 + (one ? 1 : 0);
          xo[k] = s[at(one ? x + 1 : x - 1, y, z)];
          yu[k] = s[at(x, y + 1, z)];
          yd[k] = s[at(x, y - 1, z)];
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int z = z0 + k;
          // the cell of this parity in slice z: column 0 if x0 + y + z has it
          const bool one = ((x0 + y + z + half) & 1) != 0;
          const int x = x0 + (one ? 1 : 0);
          const T c = one ? c1[z + 1] : c0[z + 1];
          // x neighbours: the pair partner from registers, the outer one from LDS
          const T xin = one ? c0[z + 1] : c1[z + 1];
          const T xp1 = one ? xo[k] : xin;
          const T xm1 = one ? xin : xo[k];
          const T zp1 = one ? c1[z + 2] : c0[z + 2];
          const T zm1 = one ? c1[z] : c0[z];
          T sum = xp1;
          sum = sum + yu[k];
          sum = sum + zp1;
          sum = sum + xm1;
          sum = sum + yd[k];
          sum = sum + zm1;
          const T R = (sum - six * c) - (one ? q1[z] : q0[z]);
          const T v = c + w6 * R;
          if (one) c1[z + 1] = v;
          else c0[z + 1] = v;
          s[at(x, y, z)] = v;
          racc += (double)(R < T(0) ? -R : R);
        }
      }
      __syncthreads();
    }
    ++it;
    double pacc = 0.0;
#pragma unroll
    for (int z = 1; z <= N; ++z)
      pacc += (double)(c0[z] < T(0) ? -c0[z] : c0[z]) + (double)(c1[z] < T(0) ? -c1[z] : c1[z]);
    block_sum2(racc, pacc);
    rnorm = racc;
    if (it >= p.max_iter || (it >= p.min_iter && rnorm <= p.tol * (src_norm + 6.0 * pacc))) break;
  }
  T* out = static_cast<T*>(p.phi_out) + (int64_t)g * N3;
#pragma unroll
  for (int z = 0; z < N; ++z) {
    out[x0 + N * (y + N * z)] = c0[z + 1];
    out[x0 + 1 + N * (y + N * z)] = c1[z + 1];
  }
  if (tid == 0) {
    if (p.iters) p.iters[g] = it;
    if (p.resid) p.resid[g] = rnorm;
  }
}

// ---------------------------------------------------------------------------
// self-gravity source operator G (Sec. 2.3)
// ---------------------------------------------------------------------------
//
// One thread per interior cell of a uniform-edge batch: accelerations from
// 3-point central differences of the potential (one ghost layer), momentum
// m_d + (a rho)(phi_-d - phi_+d) with a = dt/(2 dh), energy
// e + ((s_x + s_y) + s_z) b with s_d = (m_d + m_d')(phi_-d - phi_+d) and
// b = dt/(4 dh) (the work of the time-centred momentum, which leaves the
// internal energy unchanged), a and b rounded once from FP64.  The state is
// updated in place; density is not touched.  HBM-bound: per cell it reads
// four state values and the potential and writes four.

constexpr int kGravNT = 256;

template <typename T, int N>
__global__ __launch_bounds__(kGravNT) void k_gravity(KParams kp, const T* __restrict__ phi) {
  constexpr int M = N + 2, N3 = N * N * N, M3 = M * M * M;
  const int64_t i = (int64_t)blockIdx.x * kGravNT + threadIdx.x;
  if (i >= (int64_t)kp.nblocks * N3) return;
  const int b = (int)(i / N3), c = (int)(i % N3);
  const int x = c % N, y = (c / N) % N, z = c / (N * N);
  T* u = static_cast<T*>(kp.uout) + (kp.out_off ? kp.out_off[b] : (int64_t)b * kNV * N3) + c;
  const T* p = phi + (int64_t)b * M3 + (x + 1) + M * ((y + 1) + M * (z + 1));
  const double dt = kp.d_dt ? kp.d_dt[b] : kp.dt, dh = kp.d_dh ? kp.d_dh[b] : kp.dh;
  const T a = (T)(dt / (2.0 * dh)), bq = (T)(dt / (4.0 * dh));
  const T dpx = p[-1] - p[1], dpy = p[-M] - p[M], dpz = p[-M * M] - p[M * M];
  const T ar = a * u[0];
  const T mx = u[N3], my = u[2 * N3], mz = u[3 * N3];
  const T nx = mx + ar * dpx, ny = my + ar * dpy, nz = mz + ar * dpz;
  const T sx = (mx + nx) * dpx, sy = (my + ny) * dpy, sz = (mz + nz) * dpz;
  u[N3] = nx;
  u[2 * N3] = ny;
  u[3 * N3] = nz;
  u[4 * N3] = u[4 * N3] + ((sx + sy) + sz) * bq;
}

// ---------------------------------------------------------------------------
// launchers and the variant table
// ---------------------------------------------------------------------------

static const Variant kVariants[] = {
    {16, 512, 0, 1},  // FP32 edge 16: one workgroup per CU
    {16, 512, 0, 3},
    {16, 512, 0, 2},
    {16, 512, 0, 0},
    {16, 512, 16, 1},
    {16, 512, 16, 3},
    {8, 128, 8, 0},
    {8, 128, 8, 2},
    {8, 256, 8, 0},
    {8, 64, 8, 0},
};

int variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
Variant variant_at(int i) { return kVariants[i]; }

bool variant_supported(int dtype, const Variant& v) {
  // FP64 edge 16 does not fit the 160 KB LDS.
  return !(dtype == 2 && v.edge == 16);
}

// The flux-recording advance exists for one variant per (type, edge): the
// default ones (edge 16: 512 threads, pad 16, split 3; edge 8: 128 threads
// FP32 or 256 threads FP64, pad 8, split 0).
template <typename T, int N, int NT, int PAD, int SPLIT>
constexpr bool kFluxVariant =
    N == 16 ? (NT == 512 && PAD == 16 && SPLIT == 3)
            : (NT == (sizeof(T) == 4 ? 128 : 256) && PAD == 8 && SPLIT == 0);

template <typename T, int N, int NT, int PAD, int SPLIT>
static hipError_t launch_b(int order, bool gather, const KParams& kp, hipStream_t s) {
  const dim3 grid(kp.nblocks), block(NT);
  if (kp.flux) {
    if constexpr (kFluxVariant<T, N, NT, PAD, SPLIT>) {
      if (gather) return hipErrorInvalidValue;
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

template <typename T>
static hipError_t launch_typed(int order, const Variant& v, bool gather, const KParams& kp,
                               hipStream_t s) {
#define TVD_VARIANT(E, TH, P, SP)                                                   \
  if (v.edge == E && v.threads == TH && v.pad == P && v.split == SP)                \
    return launch_b<T, E, TH, P, SP>(order, gather, kp, s);
  if constexpr (sizeof(T) == 4) {  // FP64 edge 16 does not fit in LDS
    TVD_VARIANT(16, 512, 0, 1)
    TVD_VARIANT(16, 512, 0, 3)
    TVD_VARIANT(16, 512, 0, 2)
    TVD_VARIANT(16, 512, 0, 0)
    TVD_VARIANT(16, 512, 16, 1)
    TVD_VARIANT(16, 512, 16, 3)
  }
  TVD_VARIANT(8, 128, 8, 0)
  TVD_VARIANT(8, 128, 8, 2)
  TVD_VARIANT(8, 256, 8, 0)
  TVD_VARIANT(8, 64, 8, 0)
#undef TVD_VARIANT
  return hipErrorInvalidValue;
}

hipError_t launch_batched(int dtype, int order, const Variant& v, bool gather, const KParams& kp,
                          hipStream_t s) {
  if (dtype == 1) return launch_typed<float>(order, v, gather, kp, s);
  if (v.edge == 16) return hipErrorInvalidValue;
  return launch_typed<double>(order, v, gather, kp, s);
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

hipError_t launch_plain_f64(int order, const KParams& kp, hipStream_t s) {
  const dim3 grid(kp.nblocks), block(kPlainNT);
  if (order == 0) hipLaunchKernelGGL((k_plain_f64<0>), grid, block, 0, s, kp);
  else hipLaunchKernelGGL((k_plain_f64<1>), grid, block, 0, s, kp);
  return hipGetLastError();
}

static hipError_t launch_diag(int dtype, int layout, KParams kp, int flags, hipStream_t s) {
  kp.diag = flags;
  if (dtype == 1) hipLaunchKernelGGL((k_block_diag<float>), dim3(kp.nblocks), dim3(kRedNT), 0, s, kp, layout);
  else hipLaunchKernelGGL((k_block_diag<double>), dim3(kp.nblocks), dim3(kRedNT), 0, s, kp, layout);
  return hipGetLastError();
}

hipError_t launch_signal_speed(int dtype, int layout, const KParams& kp, hipStream_t s) {
  return launch_diag(dtype, layout, kp, kDiagSpeed, s);
}

hipError_t launch_cons_sums(int dtype, int layout, const KParams& kp, hipStream_t s) {
  return launch_diag(dtype, layout, kp, kDiagSums, s);
}

hipError_t launch_finalize_max(const double* ws, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_max, dim3(1), dim3(kFinNT), 0, s, ws, n, out);
  return hipGetLastError();
}

hipError_t launch_finalize_sums(const double* ws, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_sums, dim3(1), dim3(kFinNT), 0, s, ws, n, out);
  return hipGetLastError();
}

hipError_t launch_dt_from_speed(const KParams& kp, const double* smax, double cfl, double* dt_out,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_dt_from_speed, dim3((kp.nblocks + 255) / 256), dim3(256), 0, s, kp, smax,
                     cfl, dt_out);
  return hipGetLastError();
}

hipError_t launch_fill_ghosts(int dtype, const KParams& kp, const int32_t* nbr, int max_edge,
                              hipStream_t s) {
  const int m = max_edge + 2 * kG;
  const int chunks = (m * m * m + kFillNT - 1) / kFillNT;
  const dim3 grid((unsigned)kp.nblocks * chunks), block(kFillNT);
  if (dtype == 1) hipLaunchKernelGGL((k_fill_ghosts<float>), grid, block, 0, s, kp, nbr, chunks);
  else hipLaunchKernelGGL((k_fill_ghosts<double>), grid, block, 0, s, kp, nbr, chunks);
  return hipGetLastError();
}

hipError_t launch_fill_ghosts_amr(int dtype, const KParams& kp, const int32_t* nbr, int max_edge,
                                  const void* cin, const int64_t* coff, int ncoarse,
                                  const int32_t* cnbr, const int32_t* corigin, hipStream_t s) {
  const int m = max_edge + 2 * kG;
  const int chunks = (m * m * m + kFillNT * kFillCPT - 1) / (kFillNT * kFillCPT);
  const dim3 grid((unsigned)kp.nblocks * chunks), block(kFillNT);
  if (dtype == 1)
    hipLaunchKernelGGL((k_fill_ghosts_amr<float>), grid, block, 0, s, kp, nbr, chunks,
                       static_cast<const float*>(cin), coff, ncoarse, cnbr, corigin);
  else
    hipLaunchKernelGGL((k_fill_ghosts_amr<double>), grid, block, 0, s, kp, nbr, chunks,
                       static_cast<const double*>(cin), coff, ncoarse, cnbr, corigin);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_restrict(int dtype, const KParams& ck, const KParams& fk, const int32_t* rows,
                           int nrows, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  if (dtype == 1) hipLaunchKernelGGL((k_restrict<float>), dim3(nrows), dim3(kCloseNT), 0, s, ck, fk, rows);
  else hipLaunchKernelGGL((k_restrict<double>), dim3(nrows), dim3(kCloseNT), 0, s, ck, fk, rows);
  return hipGetLastError();
}

hipError_t launch_close_level(int dtype, const KParams& ck, const KParams& fk,
                              const int32_t* rrows, int nr, const int32_t* frows, int nf,
                              const int32_t* start, int ngroups, hipStream_t s) {
  const int grid = nr + ngroups;
  if (grid <= 0) return hipSuccess;
  if (dtype == 1)
    hipLaunchKernelGGL((k_close_level<float>), dim3(grid), dim3(kCloseNT), 0, s, ck, fk, rrows,
                       ngroups, frows, nf, start);
  else
    hipLaunchKernelGGL((k_close_level<double>), dim3(grid), dim3(kCloseNT), 0, s, ck, fk, rrows,
                       ngroups, frows, nf, start);
  return hipGetLastError();
}

hipError_t launch_flux_correct(int dtype, const KParams& ck, const KParams& fk, const int32_t* rows,
                               int nrows, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  if (dtype == 1)
    hipLaunchKernelGGL((k_flux_correct<float>), dim3(nrows), dim3(kCloseNT), 0, s, ck, fk, rows);
  else
    hipLaunchKernelGGL((k_flux_correct<double>), dim3(nrows), dim3(kCloseNT), 0, s, ck, fk, rows);
  return hipGetLastError();
}

__global__ void k_lerp_f32(int64_t n, const float* a, const float* b, float* out, float w) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = a[i] + w * (b[i] - a[i]);
}

__global__ void k_lerp_f64(int64_t n, const double* a, const double* b, double* out, double w) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = a[i] + w * (b[i] - a[i]);
}

hipError_t launch_lerp(int dtype, int64_t n, const void* a, const void* b, void* out, double w,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (dtype == 1)
    hipLaunchKernelGGL(k_lerp_f32, grid, block, 0, s, n, static_cast<const float*>(a),
                       static_cast<const float*>(b), static_cast<float*>(out), (float)w);
  else
    hipLaunchKernelGGL(k_lerp_f64, grid, block, 0, s, n, static_cast<const double*>(a),
                       static_cast<const double*>(b), static_cast<double*>(out), w);
  return hipGetLastError();
}

hipError_t launch_sor(int dtype, int ngroups, const void* phi_in, const void* rho, void* phi_out,
                      const double* d_dh, double dh, double G, double omega, double tol,
                      int min_iter, int max_iter, int32_t* iters, double* resid, hipStream_t s) {
  if (ngroups <= 0) return hipSuccess;
  SorParams p{phi_in, rho, phi_out, d_dh, dh, G, omega, tol, ngroups, min_iter, max_iter, iters,
              resid};
  if (dtype == 1) hipLaunchKernelGGL(k_sor<float>, dim3(ngroups), dim3(kSorNT), 0, s, p);
  else hipLaunchKernelGGL(k_sor<double>, dim3(ngroups), dim3(kSorNT), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_gravity(int dtype, const KParams& kp, const void* phi, hipStream_t s) {
  const int64_t cells = (int64_t)kp.nblocks * kp.edge * kp.edge * kp.edge;
  if (cells <= 0) return hipSuccess;
  const dim3 grid((unsigned)((cells + kGravNT - 1) / kGravNT)), block(kGravNT);
  if (dtype == 1) {
    if (kp.edge == 16) hipLaunchKernelGGL((k_gravity<float, 16>), grid, block, 0, s, kp, static_cast<const float*>(phi));
    else hipLaunchKernelGGL((k_gravity<float, 8>), grid, block, 0, s, kp, static_cast<const float*>(phi));
  } else {
    if (kp.edge == 16) hipLaunchKernelGGL((k_gravity<double, 16>), grid, block, 0, s, kp, static_cast<const double*>(phi));
    else hipLaunchKernelGGL((k_gravity<double, 8>), grid, block, 0, s, kp, static_cast<const double*>(phi));
  }
  return hipGetLastError();
}

}  // namespace tvd
