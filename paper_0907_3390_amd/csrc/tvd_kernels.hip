// HIP kernels for gfx950 besides the batched and persistent advance: the
// plain FP64 advance, the standalone CFL signal speed and compensated
// conservation sums with their finalisation, the device time step, the
// sibling and coarse-fine ghost-zone fills, the closing step of a level pair
// (restriction and coarse-fine flux correction), red-black SOR for the
// Poisson equation, the self-gravity operator and the time interpolation of
// a level; the variant table and the dispatch of the batched advance.
//
// Scheme: Schive, Tsai & Chiueh, GAMER, Sec. 2.2 (equations cited in
// tvd_device.hpp); signal speed Eq. (CFL), Sec. 3.4; AMR ghost zones and the
// closing step, Secs. 2.1, 2.2 and 3.1; Poisson solver and gravity, Sec. 2.3.
#include "tvd_block.hpp"

namespace tvd {

hipError_t launch_batched_f32_e16(int order, const Variant& v, bool gather, const KParams& kp,
                                  hipStream_t s);
hipError_t launch_batched_f32_e8(int order, const Variant& v, bool gather, const KParams& kp,
                                 hipStream_t s);
hipError_t launch_batched_f64_e8(int order, const Variant& v, bool gather, const KParams& kp,
                                 hipStream_t s);

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

// The partials are n records of 10 doubles (sum, compensation of each
// variable).  Thread t merges the records t, t + 1024, t + 2048, ... in
// that order, so that the lanes of a wave read consecutive records
// (coalesced), then the fixed tree of block_csum: deterministic.
__global__ __launch_bounds__(kFinNT) void k_finalize_sums(const double* ws, int n, double* out) {
  __shared__ CSum red[kFinNT / 64 * kNV];
  CSum a[kNV];
  for (int k = 0; k < kNV; ++k) a[k] = CSum{0.0, 0.0};
  for (int b = threadIdx.x; b < n; b += kFinNT) {
    const double2* r = reinterpret_cast<const double2*>(ws + (size_t)b * 2 * kNV);
    double2 v[kNV];
#pragma unroll
    for (int k = 0; k < kNV; ++k) v[k] = r[k];
#pragma unroll
    for (int k = 0; k < kNV; ++k) a[k] = csum_merge(a[k], CSum{v[k].x, v[k].y});
  }
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

// floor(i / d) by a 24-bit multiply and a shift, m = ceil(2^K / d), for small
// numerators and divisors; checked exhaustively: K = 16 is exact for
// 0 <= i < 4096 and 1 <= d <= 26, K = 19 for 0 <= i < 16384 and 2 <= d <= 32
// (the product staying below 2^32).
template <int K>
struct SmallDiv {
  unsigned m;
  __device__ explicit SmallDiv(int d) : m(((1u << K) + (unsigned)d - 1u) / (unsigned)d) {}
  __device__ int operator()(int i) const { return (int)(__umul24((unsigned)i, m) >> K); }
};

// (x, y, z) of ghosted cell `cell` of an m^3 block (m = n + 6 <= 22, so
// cell < 10648); dm divides by m
__device__ __forceinline__ void ghosted_xyz(int cell, int m, const SmallDiv<19>& dm, int& x,
                                            int& y, int& z) {
  const int q = dm(cell), r = dm(q);
  x = cell - q * m;
  y = q - r * m;
  z = r;
}

// ---------------------------------------------------------------------------
// sibling ghost fill
// ---------------------------------------------------------------------------

constexpr int kFillNT = 256;

// The 27 region sources of block b, resolved once per workgroup by threads
// 0..26 into LDS: kind 1 (sibling copy, base = the source's interior), 2 (no
// sibling: base = own interior) or 0 (a source out of range or of another
// edge: its cells are counted as non-physical).  The caller synchronises.
template <typename T>
__device__ __forceinline__ void resolve_regions(const KParams& kp, const int32_t* nbr, int b,
                                                int n, const T* own, const T** s_base,
                                                int* s_kind) {
  const int r = threadIdx.x;
  if (r >= 27) return;
  const int src = nbr[27 * (int64_t)b + r];
  int kind = 2;
  const T* base = own;
  if (src >= 0) {
    if (src >= kp.nblocks || block_edge(kp, src) != n) {
      kind = 0;
    } else {
      kind = 1;
      base = reinterpret_cast<const T*>(kp.uout) +
             (kp.out_off ? kp.out_off[src] : (int64_t)src * kNV * n * n * n);
    }
  }
  s_kind[r] = kind;
  s_base[r] = base;
}

template <typename T>
__global__ __launch_bounds__(kFillNT) void k_fill_ghosts(KParams kp, const int32_t* nbr,
                                                        int chunks) {
  __shared__ const T* s_base[27];
  __shared__ int s_kind[27];
  // contiguous ranges of (block, chunk) items per XCD: a block's chunks, and
  // neighbouring blocks, which read the same sibling interiors, share an L2
  const int item = xcd_block(blockIdx.x, gridDim.x);
  const int b = item / chunks;
  const int chunk = item % chunks;
  const int n = block_edge(kp, b);
  const int m = n + 2 * kG;
  const int m3 = m * m * m;
  const SmallDiv<19> dm(m);
  const int n3 = n * n * n;
  const T* own = reinterpret_cast<const T*>(kp.uout) +
                 (kp.out_off ? kp.out_off[b] : (int64_t)b * kNV * n3);
  resolve_regions<T>(kp, nbr, b, n, own, s_base, s_kind);
  __syncthreads();
  const int cell = chunk * kFillNT + threadIdx.x;
  if (cell >= m3) return;
  int x, y, z;
  ghosted_xyz(cell, m, dm, x, y, z);
  const int rx = x < kG ? -1 : (x >= n + kG ? 1 : 0);
  const int ry = y < kG ? -1 : (y >= n + kG ? 1 : 0);
  const int rz = z < kG ? -1 : (z >= n + kG ? 1 : 0);
  const int r = (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1);
  const int kind = s_kind[r];
  if (kind == 2) return;  // no sibling: left to the caller
  if (kind == 0) {
    atomicAdd(&kp.counters[1], 1ull);
    return;
  }
  const int sx = x - kG - rx * n, sy = y - kG - ry * n, sz = z - kG - rz * n;
  const T* sp = s_base[r] + (sx + n * (sy + n * sz));
  T* d = reinterpret_cast<T*>(const_cast<void*>(kp.uin)) +
         (kp.in_off ? kp.in_off[b] : (int64_t)b * kNV * m3);
#pragma unroll
  for (int k = 0; k < kNV; ++k) d[(int64_t)k * m3 + cell] = sp[(int64_t)k * n3];
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
  int cs;               // log2 of the coarse block edge: 3 (8^3 patches) or 4 (16^3 groups)
  // Branch-free, so that the seven reads of a cell's stencil issue together:
  // a cell outside the 27 coarse blocks or a missing block reads block 0
  // instead (ncoarse >= 1 is checked by the caller) and reports false.
  // (ix, iy, iz): coarse cell relative to the corner of the central block.
  __device__ inline bool get(int ix, int iy, int iz, T u[kNV]) const {
    const int qx = ix >> cs, qy = iy >> cs, qz = iz >> cs;
    const bool in = qx >= -1 && qx <= 1 && qy >= -1 && qy <= 1 && qz >= -1 && qz <= 1;
    const int cb = cnbr[in ? (qx + 1) + 3 * (qy + 1) + 9 * (qz + 1) : 13];
    const bool ok = in && cb >= 0 && cb < ncoarse;
    const int cs_b = ok ? cb : 0;
    const int ce = 1 << cs, cm = ce - 1;
    const int64_t c3 = (int64_t)ce * ce * ce;
    const T* c = cin + (coff ? coff[cs_b] : (int64_t)cs_b * kNV * c3) + (ix & cm) +
                 ce * (iy & cm) + ce * ce * (iz & cm);
#pragma unroll
    for (int k = 0; k < kNV; ++k) u[k] = c[k * c3];
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
                                            const int64_t* coff, int ncoarse, int cshift,
                                            const int32_t* cnbr, const int32_t* corigin) {
  if (ncoarse <= 0) {
    atomicAdd(&kp.counters[1], 1ull);
    return;
  }
  // fine index relative to the central coarse block's corner, in fine cells
  const int fx = 2 * corigin[3 * b + 0] + x - kG;
  const int fy = 2 * corigin[3 * b + 1] + y - kG;
  const int fz = 2 * corigin[3 * b + 2] + z - kG;
  const int cx = fx >> 1, cy = fy >> 1, cz = fz >> 1;  // floor
  const T q = T(0.25);
  const T dx = (fx & 1) ? q : -q, dy = (fy & 1) ? q : -q, dz = (fz & 1) ? q : -q;
  const CoarseNbhd<T> cn{cin, coff, cnbr + 27 * (int64_t)b, ncoarse, cshift};
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
                                                            int cshift, const int32_t* cnbr,
                                                            const int32_t* corigin) {
  __shared__ const T* s_base[27];
  __shared__ int s_kind[27];
  // contiguous ranges of (block, chunk) items per XCD: a block's chunks, and
  // neighbouring blocks, which read the same sibling interiors, share an L2
  const int item = xcd_block(blockIdx.x, gridDim.x);
  const int b = item / chunks;
  const int chunk = item % chunks;
  const int n = block_edge(kp, b);
  const int m = n + 2 * kG;
  const int m3 = m * m * m;
  const SmallDiv<19> dm(m);
  const int n3 = n * n * n;
  T* d = reinterpret_cast<T*>(const_cast<void*>(kp.uin)) +
         (kp.in_off ? kp.in_off[b] : (int64_t)b * kNV * m3);
  const T* own = reinterpret_cast<const T*>(kp.uout) +
                 (kp.out_off ? kp.out_off[b] : (int64_t)b * kNV * n3);
  resolve_regions<T>(kp, nbr, b, n, own, s_base, s_kind);
  __syncthreads();
  // 0: no cell, 1: sibling copy from sp[i], 2: interpolated
  int kind[kFillCPT];
  const T* sp[kFillCPT];
#pragma unroll
  for (int i = 0; i < kFillCPT; ++i) {
    const int cell = (chunk * kFillCPT + i) * kFillNT + threadIdx.x;
    kind[i] = 0;
    sp[i] = own;  // a valid address for the unconditional reads below
    if (cell < m3) {
      int x, y, z;
      ghosted_xyz(cell, m, dm, x, y, z);
      const int rx = x < kG ? -1 : (x >= n + kG ? 1 : 0);
      const int ry = y < kG ? -1 : (y >= n + kG ? 1 : 0);
      const int rz = z < kG ? -1 : (z >= n + kG ? 1 : 0);
      const int r = (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1);
      kind[i] = s_kind[r];
      if (kind[i] == 0) {
        atomicAdd(&kp.counters[1], 1ull);
      } else if (kind[i] == 1) {
        const int sx = x - kG - rx * n, sy = y - kG - ry * n, sz = z - kG - rz * n;
        sp[i] = s_base[r] + (sx + n * (sy + n * sz));
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
    int x, y, z;
    ghosted_xyz(cell, m, dm, x, y, z);
    fill_interp<T>(kp, b, x, y, z, d, m3, cell, cin, coff, ncoarse, cshift, cnbr, corigin);
  }
}

// The coarse-fine ghost zones of a gathering advance: fine block b's ghost
// cells in every region whose neighbour entry names a source-only block
// (index >= kp.nblocks: a stand-in for the missing sibling) are
// interpolated from the coarse level (Min-Mod limited, as in fill_interp)
// and written into that block's interior, where the gathering advance
// reads them; regions with a real sibling are left to the advance.  The
// coarse level is taken at old + w (new - old) (w = 0: the old state
// alone), the same expression as tvd_lerp.
//
// One workgroup per (fine block, ghost region) pair; pairs with a real
// sibling return at once.  (A grid-stride loop of 8 workgroups per CU over
// the pairs ran 1.4 times longer: each wave then waits, at its first
// barrier of a pair, for the stores of the previous one.)  For each
// stand-in region, the coarse cells under the region's ghost slab (3 fine
// cells thick) and the ring of cells around them that their stencils reach
// are staged in LDS first, each read once (at old + w (new - old)) with all
// of a thread's reads in flight together; one thread per coarse cell under
// the slab then takes the cell's three limited slopes, which replace the
// staged values in LDS; last, one thread per fine cell of the slab (x
// fastest, so that neighbouring lanes write neighbouring addresses) writes
// u + dx s_x + dy s_y + dz s_z in that order, the same operations as for a
// single ghost cell in fill_interp.  Cells shared by the slabs of several
// fine blocks get the same value from each.
constexpr int kCfNT = 128;     // coarse cells under a face slab of a 16^3 block: 2 x 8 x 8
constexpr int kCfStage = 400;  // staged coarse cells of that slab: 4 x 10 x 10
constexpr int kCfPer = (kCfStage + kCfNT - 1) / kCfNT;
static_assert(4 * kCfNT >= kCfStage, "the slopes reuse the staging buffer");

// One (fine block b, ghost region) pair of k_fill_coarse_fine; every return
// is uniform over the workgroup.
template <typename T>
__device__ __forceinline__ void fill_cf_pair(const KParams& kp, int b, int rr, int t,
                                             const int32_t* nbr, const T* cold, const T* cnew,
                                             T w, const int64_t* coff, int ncoarse, int cshift,
                                             const int32_t* cnbr, const int32_t* corigin,
                                             T* sbuf, int* sgood, int* sok, int32_t* scb) {
  const int r = rr < 13 ? rr : rr + 1;
  const int ra[3] = {r % 3 - 1, (r / 3) % 3 - 1, r / 9 - 1};
  // the neighbour entry, b's corner and b's coarse table are read together,
  // before the pair is known to need them: one wait instead of three
  const int v = nbr[27 * (int64_t)b + r];
  int co[3] = {corigin[3 * b + 0], corigin[3 * b + 1], corigin[3 * b + 2]};
  int cbt = cnbr[27 * (int64_t)b + (t < 27 ? t : 0)];
  asm volatile("" : "+v"(cbt), "+s"(co[0]), "+s"(co[1]), "+s"(co[2]));
  if (v < kp.nblocks) return;  // a real sibling (uniform over the workgroup)
  const int n = kp.edge, h = n / 2;
  // per axis: the slab's ghosted fine coordinates [lo, hi) and the coarse
  // cells [c0, c0 + cnt) under it
  int lo[3], hi[3], c0[3], cnt[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = ra[a] < 0 ? 0 : (ra[a] == 0 ? kG : n + kG);
    hi[a] = ra[a] < 0 ? kG : (ra[a] == 0 ? n + kG : n + 2 * kG);
    c0[a] = ra[a] < 0 ? co[a] - 2 : (ra[a] == 0 ? co[a] : co[a] + h);
    cnt[a] = ra[a] == 0 ? h : 2;
  }
  const bool mine = t < cnt[0] * cnt[1] * cnt[2];
  // cnt is 2 or h (4 or 8): powers of two
  const int lg0 = __builtin_ctz(cnt[0]), lg1 = __builtin_ctz(cnt[1]);
  const int l[3] = {t & (cnt[0] - 1), (t >> lg0) & (cnt[1] - 1), t >> (lg0 + lg1)};
  int kids = 0;  // children of this thread's coarse cell inside the slab
#pragma unroll
  for (int pz = 0; pz < 2; ++pz)
#pragma unroll
    for (int py = 0; py < 2; ++py)
#pragma unroll
      for (int px = 0; px < 2; ++px) {
        const int g[3] = {2 * (c0[0] + l[0]) + px - 2 * co[0] + kG,
                          2 * (c0[1] + l[1]) + py - 2 * co[1] + kG,
                          2 * (c0[2] + l[2]) + pz - 2 * co[2] + kG};
        kids += g[0] >= lo[0] && g[0] < hi[0] && g[1] >= lo[1] && g[1] < hi[1] &&
                g[2] >= lo[2] && g[2] < hi[2];
      }
  if (v >= kp.nsrc || ncoarse <= 0) {
    if (mine) atomicAdd(&kp.counters[1], (unsigned long long)kids);
    return;
  }
  if (t < 27) scb[t] = cbt;
  __syncthreads();
  // stage the box [c0 - 1, c0 + cnt + 1) per axis
  const int s[3] = {cnt[0] + 2, cnt[1] + 2, cnt[2] + 2};
  const int ns = s[0] * s[1] * s[2];
  const SmallDiv<16> div0(s[0]), div1(s[1]);
  const CoarseNbhd<T> ca{cold, coff, scb, ncoarse, cshift}, cb{cnew, coff, scb, ncoarse, cshift};
  T a[kCfPer][kNV], e[kCfPer][kNV];
  bool okj[kCfPer];
#pragma unroll
  for (int j = 0; j < kCfPer; ++j) {
    const int i = min(t + j * kCfNT, ns - 1);  // past the box: a repeat of its last cell
    const int q0 = div0(i), q1 = div1(q0);
    const int ix = c0[0] - 1 + (i - q0 * s[0]), iy = c0[1] - 1 + (q0 - q1 * s[1]),
              iz = c0[2] - 1 + q1;
    okj[j] = ca.get(ix, iy, iz, a[j]);
    if (w != T(0)) cb.get(ix, iy, iz, e[j]);
  }
#pragma unroll
  for (int j = 0; j < kCfPer; ++j) {
    const int i = t + j * kCfNT;
    if (i >= ns) continue;
#pragma unroll
    for (int k = 0; k < kNV; ++k) sbuf[k * kCfStage + i] = w != T(0) ? a[j][k] + w * (e[j][k] - a[j][k]) : a[j][k];
    sok[i] = okj[j];
  }
  __syncthreads();
  T u[kNV], sx[kNV], sy[kNV], sz[kNV];
  if (mine) {
    const int sc = (l[0] + 1) + s[0] * ((l[1] + 1) + s[1] * (l[2] + 1));
    const int sx1 = 1, sy1 = s[0], sz1 = s[0] * s[1];
    const bool ok = sok[sc] & sok[sc + sx1] & sok[sc - sx1] & sok[sc + sy1] & sok[sc - sy1] &
                    sok[sc + sz1] & sok[sc - sz1];
    sgood[t] = ok;
    if (!ok) atomicAdd(&kp.counters[1], (unsigned long long)kids);
    const T* sv = sbuf;
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
      const T* c = sv + k * kCfStage + sc;
      u[k] = c[0];
      sx[k] = minmod(c[sx1] - u[k], u[k] - c[-sx1]);
      sy[k] = minmod(c[sy1] - u[k], u[k] - c[-sy1]);
      sz[k] = minmod(c[sz1] - u[k], u[k] - c[-sz1]);
    }
  }
  __syncthreads();
  if (mine) {
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
      sbuf[(0 * kNV + k) * kCfNT + t] = u[k];
      sbuf[(1 * kNV + k) * kCfNT + t] = sx[k];
      sbuf[(2 * kNV + k) * kCfNT + t] = sy[k];
      sbuf[(3 * kNV + k) * kCfNT + t] = sz[k];
    }
  }
  __syncthreads();
  const int ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
  const int nf = ex * ey * ez;
  const int64_t n3 = (int64_t)n * n * n;
  T* d = reinterpret_cast<T*>(kp.uout) + (kp.out_off ? kp.out_off[v] : (int64_t)v * kNV * n3);
  const T q = T(0.25);
  const SmallDiv<16> divx(ex), divy(ey);
  for (int f = t; f < nf; f += kCfNT) {
    const int q0 = divx(f), q1 = divy(q0);
    const int g[3] = {lo[0] + (f - q0 * ex), lo[1] + (q0 - q1 * ey), lo[2] + q1};
    // fine index relative to the central coarse block's corner, its coarse
    // cell (floor) and that cell's place under the slab
    const int fi[3] = {2 * co[0] + g[0] - kG, 2 * co[1] + g[1] - kG, 2 * co[2] + g[2] - kG};
    const int lc = ((fi[0] >> 1) - c0[0]) +
                   cnt[0] * (((fi[1] >> 1) - c0[1]) + cnt[1] * ((fi[2] >> 1) - c0[2]));
    if (!sgood[lc]) continue;
    const T dx = (fi[0] & 1) ? q : -q, dy = (fi[1] & 1) ? q : -q, dz = (fi[2] & 1) ? q : -q;
    const int64_t o = (g[0] - kG - ra[0] * n) + n * ((g[1] - kG - ra[1] * n) +
                                                       (int64_t)n * (g[2] - kG - ra[2] * n));
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
      T val = sbuf[(0 * kNV + k) * kCfNT + lc];
      val = val + dx * sbuf[(1 * kNV + k) * kCfNT + lc];
      val = val + dy * sbuf[(2 * kNV + k) * kCfNT + lc];
      val = val + dz * sbuf[(3 * kNV + k) * kCfNT + lc];
      d[(int64_t)k * n3 + o] = val;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kCfNT) void k_fill_coarse_fine(
    KParams kp, const int32_t* nbr, const T* cold, const T* cnew, T w, const int64_t* coff,
    int ncoarse, int cshift, const int32_t* cnbr, const int32_t* corigin) {
  // staged values [kNV][kCfStage], then slopes [4][kNV][kCfNT] (u, s_x, s_y, s_z)
  __shared__ T sbuf[4 * kNV * kCfNT];
  __shared__ int sgood[kCfNT];
  __shared__ int sok[kCfStage];
  __shared__ int32_t scb[27];
  // contiguous ranges of pairs per XCD: a block's regions, and neighbouring
  // blocks, whose coarse boxes overlap, meet in the same L2
  const int i = xcd_block(blockIdx.x, gridDim.x);
  fill_cf_pair<T>(kp, i / 26, i % 26, threadIdx.x, nbr, cold, cnew, w, coff, ncoarse, cshift, cnbr,
                  corigin, sbuf, sgood, sok, scb);
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


hipError_t launch_batched(int dtype, int order, const Variant& v, bool gather, const KParams& kp,
                          hipStream_t s) {
  if (dtype == 1) {
    if (v.edge == 16) return launch_batched_f32_e16(order, v, gather, kp, s);
    return launch_batched_f32_e8(order, v, gather, kp, s);
  }
  if (v.edge == 16) return hipErrorInvalidValue;  // FP64 edge 16 does not fit in LDS
  return launch_batched_f64_e8(order, v, gather, kp, s);
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
                                  const void* cin, const int64_t* coff, int ncoarse, int cedge,
                                  const int32_t* cnbr, const int32_t* corigin, hipStream_t s) {
  const int cshift = cedge == 16 ? 4 : 3;
  const int m = max_edge + 2 * kG;
  const int chunks = (m * m * m + kFillNT * kFillCPT - 1) / (kFillNT * kFillCPT);
  const dim3 grid((unsigned)kp.nblocks * chunks), block(kFillNT);
  if (dtype == 1)
    hipLaunchKernelGGL((k_fill_ghosts_amr<float>), grid, block, 0, s, kp, nbr, chunks,
                       static_cast<const float*>(cin), coff, ncoarse, cshift, cnbr, corigin);
  else
    hipLaunchKernelGGL((k_fill_ghosts_amr<double>), grid, block, 0, s, kp, nbr, chunks,
                       static_cast<const double*>(cin), coff, ncoarse, cshift, cnbr, corigin);
  return hipGetLastError();
}

hipError_t launch_fill_coarse_fine(int dtype, const KParams& kp, const int32_t* nbr,
                                   const void* cold, const void* cnew, double w,
                                   const int64_t* coff, int ncoarse, int cedge,
                                   const int32_t* cnbr, const int32_t* corigin, hipStream_t s) {
  const int cshift = cedge == 16 ? 4 : 3;
  const dim3 grid((unsigned)kp.nblocks * 26u), block(kCfNT);
  if (dtype == 1)
    hipLaunchKernelGGL((k_fill_coarse_fine<float>), grid, block, 0, s, kp, nbr,
                       static_cast<const float*>(cold), static_cast<const float*>(cnew), (float)w,
                       coff, ncoarse, cshift, cnbr, corigin);
  else
    hipLaunchKernelGGL((k_fill_coarse_fine<double>), grid, block, 0, s, kp, nbr,
                       static_cast<const double*>(cold), static_cast<const double*>(cnew), w,
                       coff, ncoarse, cshift, cnbr, corigin);
  return hipGetLastError();
}

__global__ void k_zero_f64(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0.0;
}

hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t want = (n + 255) / 256;
  const unsigned grid = (unsigned)(want < 4096 ? want : 4096);
  hipLaunchKernelGGL(k_zero_f64, dim3(grid), dim3(256), 0, s, p, n);
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

// grid-stride: any n up to the entry point's limit with a grid that stays
// far below the 2^32 work-item limit of a launch
__global__ void k_lerp_f32(int64_t n, const float* a, const float* b, float* out, float w) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = a[i] + w * (b[i] - a[i]);
}

__global__ void k_lerp_f64(int64_t n, const double* a, const double* b, double* out, double w) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = a[i] + w * (b[i] - a[i]);
}

hipError_t launch_lerp(int dtype, int64_t n, const void* a, const void* b, void* out, double w,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t want = (n + 255) / 256;
  const dim3 grid((unsigned)(want < (1 << 20) ? want : (1 << 20))), block(256);
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
