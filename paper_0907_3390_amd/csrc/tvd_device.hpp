// Device-side building blocks of the relaxing TVD patch advance for gfx950.
//
// One 1-D sweep of the scheme (Schive, Tsai & Chiueh, GAMER, Sec. 2.2) is
// applied to a pencil of n+6 cells by a single thread that walks the pencil
// once, keeping a rolling window of cell states and fluxes in registers: the
// split fluxes of Eq. (LRFlux), the first-order upwind half step of
// Eq. (MidpointValue), the recomputed midpoint fluxes with the van Leer
// limited correction of Eqs. (2ndTVDFluxCorr)-(2ndRFlux) (left-moving flux
// mirrored about the interface), and the full step of Eq. (FullstepValue).
// Fluxes never leave registers, so a sweep needs no LDS traffic beyond one
// read and one write of each cell state.  This replaces the paper's design of
// one thread per cell with fluxes exchanged through shared memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvd {

constexpr int kNV = 5;     // rho, m_x, m_y, m_z, e
constexpr int kG = 3;      // ghost zones per side (seven-point stencil)

// Arithmetic of the bulk type.  FP32 uses the hardware reciprocal and square
// root (about 1 ulp); FP64 keeps IEEE division and square root.
template <typename T> struct Num;
template <> struct Num<float> {
  __device__ static inline float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
  __device__ static inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  __device__ static inline float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
  __device__ static inline float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
  __device__ static inline float abs(float x) { return __builtin_fabsf(x); }
  __device__ static inline float max(float a, float b) { return __builtin_fmaxf(a, b); }
};
template <> struct Num<double> {
  __device__ static inline double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
  __device__ static inline double rcp(double x) { return 1.0 / x; }
  __device__ static inline double div(double a, double b) { return a / b; }
  __device__ static inline double sqrt(double x) { return __builtin_sqrt(x); }
  __device__ static inline double abs(double x) { return __builtin_fabs(x); }
  __device__ static inline double max(double a, double b) { return __builtin_fmax(a, b); }
};

// Per-block coefficients of one sweep.
template <typename T> struct Coef {
  T hgamma;   // gamma / 2
  T hgm1;     // (gamma - 1) / 2
  T hpfloor;  // pressure floor / 2
  T lam;      // dt / dh
  T hlam;     // dt / (2 dh)
};

// Freezing speed and split fluxes of one cell, Eq. (LRFlux) multiplied out:
// F^R = (c u + F)/2, F^L = (c u - F)/2 with c = |v_n| + c_s.  Components are
// in pencil order: 0 rho, 1 normal momentum, 2-3 transverse momenta, 4 e.
// The pressure entering F and c_s is max(P, p_floor) (the IEEE max, so a
// pressure that is not a number becomes p_floor; such states are reported by
// the health counters).
//
// The library is built without implicit FMA contraction; every fused
// multiply-add here is explicit, so identical inputs give identical results
// wherever the expression appears, and the two transverse momenta enter
// symmetrically (a uniform state stays bit-exact, axis permutations and
// reflections commute with the update bit for bit).
template <typename T>
__device__ __forceinline__ void split_flux(const T u[kNV], const Coef<T>& cf, T FR[kNV],
                                           T FL[kNV]) {
  using F = Num<T>;
  const T inv = F::rcp(u[0]);
  const T mt2 = u[2] * u[2] + u[3] * u[3];
  const T m2 = F::fma(u[1], u[1], mt2);
  // Everything is carried at half scale, which is exact (scaling by 2^-1
  // commutes with rounding): hP = P*/2 = max((gamma-1)/2 (e - m^2/2rho),
  // p_floor/2), v_n/2 = (m_n/2)/rho, c/2 = |v_n/2| + sqrt((gamma/2)(P*/2)/rho).
  const T hP = F::max(cf.hgm1 * F::fma(T(-0.5) * m2, inv, u[4]), cf.hpfloor);
  const T hcs = F::sqrt((cf.hgamma * hP) * inv);
  T hF[kNV];
  hF[0] = T(0.5) * u[1];
  const T hv = hF[0] * inv;
  const T hc = F::abs(hv) + hcs;
  hF[1] = F::fma(u[1], hv, hP);
  hF[2] = u[2] * hv;
  hF[3] = u[3] * hv;
  hF[4] = F::fma(T(2), hP, u[4]) * hv;  // (e + P*) v_n / 2
#pragma unroll
  for (int k = 0; k < kNV; ++k) {
    FR[k] = F::fma(hc, u[k], hF[k]);
    FL[k] = F::fma(hc, u[k], -hF[k]);
  }
}

// Eq. (vanLeer) on the halved corrections (a/2, b/2): 2 (a/2)(b/2) / ((a+b)/2)
// = ab / (a+b) when ab > 0, else 0.
template <typename T>
__device__ __forceinline__ T vanleer(T a, T b) {
  const T p = a * b;
  return p > T(0) ? Num<T>::div(p, a + b) : T(0);
}
// The multiply whose zero operand wins over an infinite or NaN one
// (v_mul_legacy_f32; an ordinary IEEE product otherwise).
extern "C" __device__ float tvd_fmul_zero_wins(float, float) __asm("llvm.amdgcn.fmul.legacy");

// FP32, without a compare and select: max(ab, 0) times the reciprocal of
// a+b.  a+b = 0 only happens with ab <= 0, where the result must be 0, not
// 0 * inf: the zero-wins product gives exactly that, and for ab > 0 it is
// ab * rcp(a+b) exactly.
template <>
__device__ __forceinline__ float vanleer<float>(float a, float b) {
  return tvd_fmul_zero_wins(Num<float>::max(a * b, 0.0f), Num<float>::rcp(a + b));
}

// Whether a sweep destination also takes the interface fluxes of the full
// step (a static member kFlux = true and a member flux(f, H)).
template <class D, class = void>
struct TakesFlux {
  static constexpr bool value = false;
};
template <class D>
struct TakesFlux<D, decltype((void)D::kFlux)> {
  static constexpr bool value = D::kFlux;
};

// One sweep over a pencil of M = N+6 cells.  Src::load(j, u) fetches cell j
// (0 .. M-1, ghosts included) in pencil component order; Dst::store(i, u)
// writes interior cell i (0 .. N-1).  The loop is fully unrolled, so the
// rolling windows (indexed modulo 4) live in registers.  A destination that
// takes fluxes gets dst.flux(f, H) for every interface f - 1/2, f = 0 .. N:
// the flux of Eq. (FullstepValue), u_i -= lam (H at i+1 - H at i).
template <typename T, int N, class Src, class Dst>
__device__ __forceinline__ void pencil_sweep(const Src& src, const Dst& dst, const Coef<T>& cf) {
  constexpr int M = N + 2 * kG;
  T q[4][kNV];     // cell states u^t, ring over j
  T FRh[4][kNV];   // midpoint right-moving fluxes, ring over j
  T FLh[4][kNV];   // midpoint left-moving fluxes, ring over j
  T FRp[kNV];      // F^R of the previous cell
  T Gp[kNV];       // first-order interface flux G_{j-3/2}
  T Hp[kNV];       // second-order interface flux of the previous interface
#pragma unroll
  for (int j = 0; j < M; ++j) {
    T* qj = q[j & 3];
    src.load(j, qj);
    T FR[kNV], FL[kNV];
    split_flux(qj, cf, FR, FL);
    if (j >= 1) {
      // first-order upwind flux at j-1/2: F^R_{j-1} - F^L_j
      T G[kNV];
#pragma unroll
      for (int k = 0; k < kNV; ++k) G[k] = FRp[k] - FL[k];
      if (j >= 2) {
        // Eq. (MidpointValue) for cell j-1, then its midpoint fluxes
        T h[kNV];
        const T* qm = q[(j - 1) & 3];
#pragma unroll
        for (int k = 0; k < kNV; ++k) h[k] = Num<T>::fma(-cf.hlam, G[k] - Gp[k], qm[k]);
        split_flux(h, cf, FRh[(j - 1) & 3], FLh[(j - 1) & 3]);
      }
#pragma unroll
      for (int k = 0; k < kNV; ++k) Gp[k] = G[k];
    }
#pragma unroll
    for (int k = 0; k < kNV; ++k) FRp[k] = FR[k];
    if (j >= 5) {
      // second-order flux at interface (j-3)+1/2 from midpoint fluxes of
      // cells j-4 .. j-1 (Eqs. 2ndFluxCorr, vanLeer, 2ndRFlux and mirror)
      const int a = (j - 4) & 3, b = (j - 3) & 3, c = (j - 2) & 3, d = (j - 1) & 3;
      T H[kNV];
#pragma unroll
      for (int k = 0; k < kNV; ++k) {
        const T R = FRh[b][k] + vanleer(FRh[b][k] - FRh[a][k], FRh[c][k] - FRh[b][k]);
        const T L = FLh[c][k] + vanleer(FLh[c][k] - FLh[d][k], FLh[b][k] - FLh[c][k]);
        H[k] = R - L;
      }
      if constexpr (TakesFlux<Dst>::value) dst.flux(j - 5, H);
      if (j >= 6) {
        // Eq. (FullstepValue) for cell j-3 (interior cell j-6), from u^t
        T out[kNV];
        const T* q0 = q[(j - 3) & 3];
#pragma unroll
        for (int k = 0; k < kNV; ++k) out[k] = Num<T>::fma(-cf.lam, H[k] - Hp[k], q0[k]);
        dst.store(j - 6, out);
      }
#pragma unroll
      for (int k = 0; k < kNV; ++k) Hp[k] = H[k];
    }
  }
}

// Global component index of pencil component k for a sweep along axis D.
template <int D>
__device__ __host__ constexpr int gcomp(int k) {
  return k == 0 ? 0 : k == 4 ? 4 : k == 1 ? 1 + D : k == 2 ? 1 + (D + 1) % 3 : 1 + (D + 2) % 3;
}

// ---- FP64 compensated accumulation (Neumaier) and exact pair merge --------

struct CSum {
  double s, c;
};

// Neumaier's compensated step: the rounding error of s + v, recovered
// exactly, goes to the compensation.  The error is taken by Knuth's
// branch-free TwoSum, which yields the same exact value as Neumaier's
// magnitude test with (s - t) + v or (v - t) + s, in fewer instructions.
__device__ __forceinline__ void csum_add(CSum& a, double v) {
  const double t = a.s + v;
  const double z = t - a.s;
  a.c += (a.s - (t - z)) + (v - z);
  a.s = t;
}

// Merge two compensated partial sums: the rounding error of s1 + s2 is
// recovered exactly (TwoSum) and added to the compensations.
__device__ __forceinline__ CSum csum_merge(CSum a, CSum b) {
  const double s = a.s + b.s;
  const double bb = s - a.s;
  const double err = (a.s - (s - bb)) + (b.s - bb);
  return CSum{s, (a.c + b.c) + err};
}

}  // namespace tvd
