// The streamed advance: one step (sweep triple) of a chain of blocks that
// follow each other along the axis swept last (z for the forward order xyz,
// x for the backward order zyx).
//
// A workgroup of 256 threads owns a 16 x 16 tile of columns across the two
// axes swept first (the whole face of a 16^3 block, a quadrant of a 32^3
// block's face) and walks the chain plane by plane, in slabs of P planes:
//   phase A: the first sweep of the slab's planes, every pencil gathered
//            straight from HBM (the block's interior and its neighbours' for
//            the ghost cells), the 16 tile cells of each written to LDS;
//   phase B: the second sweep in LDS (the tile's 16 interior rows of each
//            plane, ghost rows of the first sweep included as inputs);
//   phase S: every thread pushes its column's cells of the slab through a
//            register ring that carries the third sweep's 1-D update along
//            the whole chain, and stores each finished cell to HBM.
// The third sweep therefore runs once over the chain instead of once per
// block with three ghost planes on each side: the region rule's redundant
// work shrinks from (n+6)^2 + n(n+6) + n^2 pencils per n^2 columns to
// (n+6) + n + n per column of the chain (plus three ghost planes at each
// chain end), and no LDS holds more than one slab.  The arithmetic of every
// cell is that of pencil_sweep, in the same order, so the results are
// bit-identical to the per-block advance (the region rule is exact).
//
// Scheme: Schive, Tsai & Chiueh, GAMER, Sec. 2.2 (equations cited in
// tvd_device.hpp); Sec. 3.1 for the one-block-per-thread-block design this
// replaces; signal speed Eq. (CFL), Sec. 3.4.
#pragma once

#include "tvd_block.hpp"
#include "tvd_stream_params.hpp"

namespace tvd {

constexpr int kStreamNT = 256;    // threads: one column of the 16 x 16 tile each
constexpr int kTile = 16;         // tile edge across the first two sweep axes
constexpr int kRows = kTile + 2 * kG;   // first-sweep rows of a plane (ghosts included)
constexpr int kStreamMaxChain = 64;     // blocks per chain at most
// Fourth word of a raw buffer resource on gfx950 (32-bit data format, no
// swizzle), and the vector types of the buffer stores' data.
constexpr int kBufferWord3 = 0x00020000;
typedef uint32_t U32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));

// Axes of the streamed advance: A (swept first), B (second), S (last,
// streamed).  Order 0 (xyz): A = x, B = y, S = z; order 1 (zyx): A = z,
// B = y, S = x.  Element strides of a block of edge E, and the neighbour
// region index of offsets (ra, rb, rs).
template <int ORDER, int E>
struct StreamAxes {
  static constexpr int A = ORDER == 0 ? 0 : 2;
  static constexpr int B = 1;
  static constexpr int S = ORDER == 0 ? 2 : 0;
  static constexpr int sa = ORDER == 0 ? 1 : E * E;
  static constexpr int sb = E;
  static constexpr int ss = ORDER == 0 ? E * E : 1;
  __device__ static constexpr int region(int ra, int rb, int rs) {
    return ORDER == 0 ? (ra + 1) + 3 * (rb + 1) + 9 * (rs + 1)
                      : (rs + 1) + 3 * (rb + 1) + 9 * (ra + 1);
  }
};

// LDS of one slab: P planes of kRows x 16 cells per variable, rows of the
// tile's 16 A-cells XOR-swizzled by (row + plane) and planes padded to a
// pitch of 16 mod 32 words, so that the three phases' access patterns
// spread over the banks.
template <int P>
struct SlabLayout {
  static constexpr int PL = kTile * kRows + kTile;   // plane pitch (368)
  static constexpr int VP = PL * P;                   // one variable
  __device__ static inline int idx(int a, int r, int p) {
    return (a ^ ((r + p) & (kTile - 1))) + kTile * r + PL * p;
  }
};

template <typename T, int P>
struct StreamLds {
  T s[kNV * SlabLayout<P>::VP];
  int64_t chain_off[kStreamMaxChain];  // interior offset of every chain block
  int64_t nb9[9];                      // the slab's 3 x 3 neighbour offsets (ra, rb)
  double red[kStreamNT / 64 * 2 * kNV];   // block-reduction scratch
  int nbad;
};

// Phase A source: the first-sweep pencil of row r (b = b0 - 3 + r) of one
// plane, cells a = a0 - 3 + j, j = 0 .. 21, gathered across the blocks at
// A-offsets -1, 0, +1 (p[0..2] point at the pencil's row in each, at A
// index 0).  For E = 16 the block of cell j is fixed; for E = 32 it depends
// on the tile's quadrant (a0 = 0 or 16), a value uniform over the
// workgroup.
template <typename T, int E, int SA, int D>
struct StreamPencilA {
  const T* p[3];
  int a0;
  // Along x (forward step, SA = 1) the tile's 16 interior cells of a row are
  // read four at a time with 16-byte loads (FP32), which cuts the first
  // sweep's load instructions and L1 requests; the ghost cells, 12-byte
  // pieces of the neighbours' rows, stay single loads.
  static constexpr bool kVec = SA == 1 && sizeof(T) == 4;
  mutable float4 buf[kNV];
  __device__ inline void load(int j, T u[kNV]) const {
    constexpr int E3 = E * E * E;
    if constexpr (kVec) {
      if (j >= kG && j < kG + kTile) {
        const int q = (j - kG) & 3;
        if (q == 0) {
          const float4* c = reinterpret_cast<const float4*>(p[1] + a0 + (j - kG));
#pragma unroll
          for (int k = 0; k < kNV; ++k) buf[k] = c[gcomp<D>(k) * (E3 / 4)];
        }
#pragma unroll
        for (int k = 0; k < kNV; ++k)
          u[k] = q == 0 ? buf[k].x : (q == 1 ? buf[k].y : (q == 2 ? buf[k].z : buf[k].w));
        return;
      }
    }
    const int a = a0 - kG + j;
    const T* c;
    if (E == kTile) {
      c = j < kG ? p[0] + (j - kG + E) * SA : (j < kG + E ? p[1] + (j - kG) * SA : p[2] + (j - kG - E) * SA);
    } else {
      c = a < 0 ? p[0] + (a + E) * SA : (a < E ? p[1] + a * SA : p[2] + (a - E) * SA);
    }
#pragma unroll
    for (int k = 0; k < kNV; ++k) u[k] = c[gcomp<D>(k) * E3];
  }
};

// Phase A sink: the 16 tile cells of a row into the slab.
template <typename T, int P, int D>
struct StreamSinkA {
  T* s;
  int r, p;
  __device__ inline void store(int i, const T u[kNV]) const {
    const int o = SlabLayout<P>::idx(i, r, p);
#pragma unroll
    for (int k = 0; k < kNV; ++k) s[gcomp<D>(k) * SlabLayout<P>::VP + o] = u[k];
  }
};

// Phase B: the second-sweep pencil at tile column a of plane p, in place
// (reads rows 0 .. 21, writes rows 3 .. 18).
template <typename T, int P, int D>
struct StreamPencilB {
  T* s;
  int a, p;
  __device__ inline void load(int j, T u[kNV]) const {
    const int o = SlabLayout<P>::idx(a, j, p);
#pragma unroll
    for (int k = 0; k < kNV; ++k) u[k] = s[gcomp<D>(k) * SlabLayout<P>::VP + o];
  }
  __device__ inline void store(int i, const T u[kNV]) const {
    const int o = SlabLayout<P>::idx(a, i + kG, p);
#pragma unroll
    for (int k = 0; k < kNV; ++k) s[gcomp<D>(k) * SlabLayout<P>::VP + o] = u[k];
  }
};

// The third sweep of one column, carried along the chain: the rolling
// windows of pencil_sweep (cell states, midpoint fluxes, the previous
// interface fluxes) kept across slabs.  step<J4>() takes the next cell
// (chain step j with j mod 4 = J4) and returns the finished cell j - 6 in
// `out`; the first six steps of a chain return nothing meaningful (their
// results are dropped by the caller).  The arithmetic per cell is that of
// pencil_sweep, operation for operation.
template <typename T>
struct StreamRing {
  T q[4][kNV];
  T FRh[4][kNV];
  T FLh[4][kNV];
  T FRp[kNV], Gp[kNV], Hp[kNV];

  __device__ inline void reset() {
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
      FRp[k] = Gp[k] = Hp[k] = T(0);
#pragma unroll
      for (int r = 0; r < 4; ++r) q[r][k] = FRh[r][k] = FLh[r][k] = T(0);
    }
  }

  template <int J4>
  __device__ inline void step(const T u[kNV], const Coef<T>& cf, T out[kNV]) {
    constexpr int a = J4, b = (J4 + 1) & 3, c = (J4 + 2) & 3, d = (J4 + 3) & 3;
    T* qj = q[J4];
#pragma unroll
    for (int k = 0; k < kNV; ++k) qj[k] = u[k];
    T FR[kNV], FL[kNV];
    split_flux(qj, cf, FR, FL);
    // first-order upwind flux at j-1/2, Eq. (MidpointValue) for cell j-1
    // and its midpoint fluxes
    T G[kNV], h[kNV];
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
      G[k] = FRp[k] - FL[k];
      h[k] = Num<T>::fma(-cf.hlam, G[k] - Gp[k], q[d][k]);
      Gp[k] = G[k];
      FRp[k] = FR[k];
    }
    split_flux(h, cf, FRh[d], FLh[d]);
    // second-order flux at interface (j-3)+1/2 from the midpoint fluxes of
    // cells j-4 .. j-1, then Eq. (FullstepValue) for cell j-3
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
      const T R = FRh[b][k] + vanleer(FRh[b][k] - FRh[a][k], FRh[c][k] - FRh[b][k]);
      const T L = FLh[c][k] + vanleer(FLh[c][k] - FLh[d][k], FLh[b][k] - FLh[c][k]);
      const T H = R - L;
      out[k] = Num<T>::fma(-cf.lam, H - Hp[k], q[b][k]);
      Hp[k] = H;
    }
  }
};

// Compile-time loop: f(std::integral_constant<int, I>{}) for I = B .. E-1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// One step of a chain on one tile (workgroup), see the top of this file.
//
// Chain planes are numbered g = -3 .. C*E+2 along the streamed axis: the
// three ghost planes before the first block (its S- neighbour), the blocks'
// planes, and three ghost planes after the last block (its S+ neighbour).
// Consuming plane g finishes cell g - 3 of every column.
//
// FLUX (0 none, 1 write, 2 add): the patch-boundary flux records of
// tvd_patch_advance_flux, w H through every plane at a multiple of 8 cells
// of every chain block, for the block's own face cells: the first two
// sweeps' planes from phases A and B (own rows and columns of the tile, the
// interface a tile shares with the one before it recorded by that one),
// the third sweep's from the ring, a plane between two chain blocks going
// to both blocks' records (as each block's own advance would record it).
template <typename T, int E, int ORDER, int P, bool SPLITB, int FLUX = 0>
struct StreamChain {
  using AX = StreamAxes<ORDER, E>;
  using SL = SlabLayout<P>;
  static constexpr int E3 = E * E * E;
  // 16-byte output runs along x in the backward order (x is the streamed
  // axis there, so a thread's finished cells are consecutive in memory)
  static constexpr int RUN = ORDER == 1 ? 16 / (int)sizeof(T) : 1;

  const KParams& kp;
  const StreamParams& sp;
  StreamLds<T, P>& sm;
  int tid, quad, a0, b0, chain0, C;
  int item;  // the workgroup's (chain, tile): the index of its diagnostics record
  Coef<T> cf;
  double dh;
  StreamRing<T> ring;
  CellDiag dg;
  // a 16-byte output run per variable (the backward order)
  typedef T RunVec __attribute__((ext_vector_type(RUN)));
  RunVec run[kNV];

  // flux record of block b (FLUX != 0)
  __device__ __forceinline__ T* record(int b) const {
    return reinterpret_cast<T*>(kp.flux) +
           (kp.flux_off ? kp.flux_off[b] : (int64_t)b * flux_record_size(E));
  }

  // Phase A and B of the slab planes pl in [lo, hi), plane pl being plane
  // s_lo + pl of block `cb` (rs = 0) or of its neighbour at S-offset rs (the
  // chain's ghost planes).  Chain ends use the same code with fewer planes,
  // so that one copy of each phase serves every slab.
  __device__ __forceinline__ void planes_ab(int cb, int rs, int s_lo, int lo, int hi, int rot) {
    // An opaque copy of the thread index: the per-lane LDS and HBM addresses
    // derived from it are recomputed in every slab instead of being hoisted
    // out of the slab loop, where the compiler keeps dozens of them alive
    // across all phases and spills them to scratch memory.
    int tid = this->tid;
    asm volatile("" : "+v"(tid));
    if (tid < 9) {
      const int ra = tid % 3 - 1, rb = tid / 3 - 1;
      const int nb = kp.nbr[27 * (int64_t)cb + AX::region(ra, rb, rs)];
      sm.nb9[tid] = kp.out_off ? kp.out_off[nb] : (int64_t)nb * kNV * E3;
    }
    __syncthreads();
    const T* __restrict__ uin = reinterpret_cast<const T*>(kp.uin);
    // phase A: 22 rows per plane, spread evenly over the four waves.  Along
    // x (forward step) each lane walks one contiguous row, so consecutive
    // lanes take consecutive rows; along z (backward step) the lanes of a row
    // take consecutive planes, i.e. consecutive x, so that one load
    // instruction reads whole 32-byte pieces of x-rows instead of one value
    // from each of 44 rows.
    {
      constexpr int npen = kRows * P;
      constexpr int per = (npen + 3) / 4;
      const int l = tid & 63, p = (tid >> 6) * per + l;
      const int r = ORDER == 0 ? p % kRows : p / P;
      const int pl = ORDER == 0 ? p / kRows : p % P;
      if (l < per && p < npen && pl >= lo && pl < hi) {
        const int b = b0 - kG + r;
        const int rb = b < 0 ? -1 : (b >= E ? 1 : 0);
        const int64_t row = (int64_t)(b - rb * E) * AX::sb + (int64_t)(s_lo + pl) * AX::ss;
        StreamPencilA<T, E, AX::sa, AX::A> src;
        src.a0 = a0;
#pragma unroll
        for (int ra = 0; ra < 3; ++ra) src.p[ra] = uin + sm.nb9[ra + 3 * (rb + 1)] + row;
        const StreamSinkA<T, P, AX::A> dst{sm.s, r, pl};
        if constexpr (FLUX != 0) {
          // own rows of the tile, planes of the chain's blocks: face
          // (z, y) = (s, b) of an x pencil, (y, x) = (b, s) of a z pencil
          const int s_ = s_lo + pl;
          T* fp = nullptr;
          if (rs == 0 && r >= kG && r < kG + kTile)
            fp = ORDER == 0 ? flux_entry<T, E>(record(cb), 0, s_, b)
                            : flux_entry<T, E>(record(cb), 2, b, s_);
          pencil_sweep<T, kTile>(src, tap<FLUX, T, E, AX::A>(dst, fp, a0, kp), cf);
        } else {
          pencil_sweep<T, kTile>(src, dst, cf);
        }
      }
    }
    __syncthreads();
    // phase B: the tile's 16 columns per plane, in place
    if constexpr (SPLITB) {
      const int p = tid >> 1, off = (tid & 1) * (kTile / 2);
      const int pl = p / kTile;
      const bool act = pl >= lo && pl < hi;   // 2 * 16 * P = 256 half pencils
      const Shifted<StreamPencilB<T, P, AX::B>> acc{{sm.s, p % kTile, pl}, off};
      Held<T, kTile / 2> held;
      if constexpr (FLUX != 0) {
        // face (z, x) = (s, a) of a y pencil (a, s: A and S coordinates)
        const int a = a0 + p % kTile, s_ = s_lo + pl;
        T* fp = nullptr;
        if (rs == 0)
          fp = ORDER == 0 ? flux_entry<T, E>(record(cb), 1, s_, a)
                          : flux_entry<T, E>(record(cb), 1, a, s_);
        if (act) pencil_sweep<T, kTile / 2>(acc, tap<FLUX, T, E, AX::B>(held, fp, b0 + off, kp), cf);
      } else {
        if (act) pencil_sweep<T, kTile / 2>(acc, held, cf);
      }
      __syncthreads();
      if (act) held.flush(acc);
    } else {
      // whole pencils packed densely into the fewest waves (two for P = 8),
      // the other waves idle; which waves work rotates from slab to slab
      // (rot), so that over two slabs every SIMD gets the same share
      constexpr int npen = kTile * P;
      const int l = tid & 63, p = (((tid >> 6) - rot) & 3) * 64 + l;
      const int pl = p / kTile;
      if (p < npen && pl >= lo && pl < hi) {
        const StreamPencilB<T, P, AX::B> acc{sm.s, p % kTile, pl};
        if constexpr (FLUX != 0) {
          const int a = a0 + p % kTile, s_ = s_lo + pl;
          T* fp = nullptr;
          if (rs == 0)
            fp = ORDER == 0 ? flux_entry<T, E>(record(cb), 1, s_, a)
                            : flux_entry<T, E>(record(cb), 1, a, s_);
          pencil_sweep<T, kTile>(acc, tap<FLUX, T, E, AX::B>(acc, fp, b0, kp), cf);
        } else {
          pencil_sweep<T, kTile>(acc, acc, cf);
        }
      }
    }
    __syncthreads();
  }

  // Store finished cell `cell` (0 .. C*E-1 along the chain) of this
  // thread's column and account for it in the diagnostics; with runs, the
  // cell waits in registers until its run is complete.  The stores are
  // buffer stores: the block's base (uniform over the workgroup) goes into
  // the resource, the variable and plane into the scalar offset, and the
  // lane's place in the plane (`lane`, bytes, fixed for the whole chain) is
  // the one vector operand, so that a store costs no vector address
  // arithmetic.
  template <int RPOS>
  __device__ __forceinline__ void emit(int cell, const T out[kNV]) {
    const uint32_t lane = (uint32_t)(((a0 + (tid & (kTile - 1))) * AX::sa + (b0 + tid / kTile) * AX::sb) * (int)sizeof(T));
    T ug[kNV];
#pragma unroll
    for (int k = 0; k < kNV; ++k) ug[gcomp<AX::S>(k)] = out[k];
    diag_cell<T>(dg, ug, kp.diag, kp.gamma, kp.pfloor);
    const int kk = cell / E, sl = cell % E;
    if constexpr (RUN != 1) {
#pragma unroll
      for (int k = 0; k < kNV; ++k) run[k][RPOS] = ug[k];
    }
    if constexpr (RPOS == RUN - 1 && sizeof(T) == 8) {
      // FP64: plain stores (the buffer-store form costs the FP64 kernels,
      // which already spill, more registers than it saves instructions)
      T* base = reinterpret_cast<T*>(kp.uout) + sm.chain_off[kk] + lane / sizeof(T);
#pragma unroll
      for (int k = 0; k < kNV; ++k) {
        if constexpr (RUN == 1)
          base[(int64_t)k * E3 + (int64_t)sl * AX::ss] = ug[k];
        else
          *reinterpret_cast<double2*>(base + (int64_t)k * E3 + (sl - RUN + 1)) =
              make_double2(run[k].x, run[k].y);
      }
    } else if constexpr (RPOS == RUN - 1) {
      const int64_t off = sm.chain_off[kk];
      const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)off);
      const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)off >> 32));
      T* blk = reinterpret_cast<T*>(kp.uout) + (int64_t)(((uint64_t)hi << 32) | lo);
      const __amdgpu_buffer_rsrc_t rs =
          __builtin_amdgcn_make_buffer_rsrc(blk, 0, (int)(kNV * E3 * sizeof(T)), kBufferWord3);
      // first cell of the run along S (RUN == 1: the cell itself)
      const int s0 = (sl - RUN + 1) * AX::ss;
#pragma unroll
      for (int k = 0; k < kNV; ++k) {
        const int so = (k * E3 + s0) * (int)sizeof(T);
        if constexpr (RUN == 1) {
          if constexpr (sizeof(T) == 4)
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(ug[k]), rs, lane, so, 0);
          else
            __builtin_amdgcn_raw_buffer_store_b64(
                U32x2{(uint32_t)__double_as_longlong(ug[k]), (uint32_t)((uint64_t)__double_as_longlong(ug[k]) >> 32)},
                rs, lane, so, 0);
        } else {
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U32x4, run[k]), rs, lane, so, 0);
        }
      }
    }
  }

  // The chain's diagnostics, once all its cells are finished, into the
  // partial record of its (chain, tile) item: one block reduction per chain
  // instead of one per block, and n_chains * tiles records to finalize.
  __device__ __forceinline__ void publish() {
    diag_publish<kStreamNT>(dg, item, dh, kp, sm.red, tid);
  }

  // The third sweep's flux through chain plane q (0 .. C*E, a multiple of
  // 8), just computed by the ring (ring.Hp), into the record of the block
  // above the plane and, on a boundary between two chain blocks, of the
  // block below it too.  Face (y, x) = (b, a) of a z column, (z, y) = (a, b)
  // of an x column.
  __device__ __forceinline__ void ring_flux(int q, int al, int bl) {
    if (q < 0 || q > C * E) return;
    const int a = a0 + al, b = b0 + bl;
    const T w = (T)kp.flux_w;
    auto put = [&](int blk, int plane) {
      T* f = (ORDER == 0 ? flux_entry<T, E>(record(blk), 2, b, a)
                         : flux_entry<T, E>(record(blk), 0, a, b)) +
             plane * (kNV * E * E);
#pragma unroll
      for (int k = 0; k < kNV; ++k) {
        T* c = f + gcomp<AX::S>(k) * (E * E);
        if constexpr (FLUX == 2) *c = *c + w * ring.Hp[k];
        else *c = w * ring.Hp[k];
      }
    };
    const int kk = q / E, r = q % E;
    if (kk < C) put(sp.blocks[chain0 + kk], r / kPatch);
    if (r == 0 && kk >= 1) put(sp.blocks[chain0 + kk - 1], E / kPatch);
  }

  // Phase S over the slab planes pl in [lo, hi): plane pl is chain plane
  // g = g0 + pl, chain step g + 3, ring position (3 + pl) mod 4 (g0 is a
  // multiple of 4 minus 0 for the blocks' planes and the closing ghost
  // planes, -8 for the opening ghost planes, which sit at pl = 5 .. 7).
  // `emit_from` is the first plane whose finished cell is kept.
  __device__ __forceinline__ void planes_s(int g0, int lo, int hi, int emit_from) {
    int tid = this->tid;  // opaque, as in planes_ab
    asm volatile("" : "+v"(tid));
    const int al = tid & (kTile - 1), bl = tid / kTile;
    static_for<0, P>([&](auto I) {
      constexpr int pl = decltype(I)::value;
      constexpr int j4 = (3 + pl) & 3;
      if (pl >= lo && pl < hi) {
        const int o = SL::idx(al, bl + kG, pl);
        T u[kNV], out[kNV];
#pragma unroll
        for (int k = 0; k < kNV; ++k) u[k] = sm.s[gcomp<AX::S>(k) * SL::VP + o];
        ring.template step<j4>(u, cf, out);
        if constexpr (FLUX != 0 && pl == 2) {
          // the flux of this step is that of chain plane g0 (the interface
          // below cell g0), a multiple of 8 for the blocks' slabs and the
          // closing ghost slab
          ring_flux(g0, al, bl);
        }
        // finished cell g - 3, at position (pl - 3) mod RUN of its 16-byte run
        constexpr int rpos = ((pl - kG) % RUN + RUN) % RUN;
        if (pl >= emit_from) emit<rpos>(g0 + pl - kG, out);
      }
    });
    __syncthreads();
  }

  __device__ __forceinline__ void run_chain() {
    static_assert(P == 8, "ring positions and run alignment assume slabs of 8 planes");
    ring.reset();
    diag_init(dg);
    // One loop over the chain's slabs, so that each phase exists once in the
    // code: slab 0 holds the three ghost planes before the chain (the last
    // planes of the head's S- neighbour) in slab planes 5 .. 7, chain steps
    // 0 .. 2, nothing finished; slabs 1 .. C*E/P hold the blocks' planes; the
    // last slab holds the three ghost planes after the chain (the first
    // planes of the tail's S+ neighbour), which finish the last block.
    const int nslab = C * (E / P) + 2;
    for (int t = 0; t < nslab; ++t) {
      int cb, rs, s_lo, lo, hi, g0, emit_from;
      if (t == 0) {
        cb = sp.blocks[chain0];
        rs = -1, s_lo = E - P, lo = P - kG, hi = P, g0 = -P, emit_from = P;
      } else if (t == nslab - 1) {
        cb = sp.blocks[chain0 + C - 1];
        rs = 1, s_lo = 0, lo = 0, hi = kG, g0 = C * E, emit_from = 0;
      } else {
        const int kk = (t - 1) / (E / P), m = (t - 1) % (E / P);
        cb = sp.blocks[chain0 + kk];
        rs = 0, s_lo = m * P, lo = 0, hi = P, g0 = kk * E + m * P;
        // the chain's first three planes finish nothing (cells -3 .. -1)
        emit_from = (kk == 0 && m == 0) ? kG : 0;
      }
      planes_ab(cb, rs, s_lo, lo, hi, (t & 1) * 2);
      planes_s(g0, lo, hi, emit_from);
    }
    publish();
  }
};

template <typename T, int E, int ORDER, int P, bool SPLITB, int FLUX = 0>
__global__ __launch_bounds__(kStreamNT) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_stream(
    KParams kp, StreamParams sp) {
  using AX = StreamAxes<ORDER, E>;
  __shared__ StreamLds<T, P> sm;
  const int tid = threadIdx.x;
  const int item = xcd_block(blockIdx.x, gridDim.x);
  const int chain = item / sp.quads, quad = item % sp.quads;
  const int c0 = sp.start[chain];
  const int C = sp.start[chain + 1] - c0;
  constexpr int kAlign = 16 / (int)sizeof(T);  // elements in 16 bytes
  // Validate the chain before touching anything: at most kStreamMaxChain
  // blocks of edge E, each the S+ neighbour of the one before, every
  // neighbour of every block present with edge E, one dt and dh.  A chain
  // that fails is not advanced (its cells are counted as non-physical and
  // its output is left untouched).
  const bool shape_ok = C >= 1 && C <= kStreamMaxChain && c0 >= 0 && c0 + C <= sp.n_members;
  if (tid == 0) sm.nbad = shape_ok ? 0 : 1;
  __syncthreads();
  if (sm.nbad == 0) {
    const int head = sp.blocks[c0];
    const bool head_ok = head >= 0 && head < kp.nblocks;
    for (int i = tid; i < C; i += kStreamNT) {
      const int b = sp.blocks[c0 + i];
      bool ok = head_ok && b >= 0 && b < kp.nblocks && block_edge(kp, b) == E;
      if (ok) {
        sm.chain_off[i] = kp.out_off ? kp.out_off[b] : (int64_t)b * kNV * E * E * E;
        // 16-byte loads of rows and 16-byte output runs stay aligned
        ok = sm.chain_off[i] % kAlign == 0;
        if (i + 1 < C) ok = kp.nbr[27 * (int64_t)b + AX::region(0, 0, 1)] == sp.blocks[c0 + i + 1];
        if (kp.d_dt) ok = ok && kp.d_dt[b] == kp.d_dt[head];
        if (kp.d_dh) ok = ok && kp.d_dh[b] == kp.d_dh[head];
      }
      if (!ok) atomicAdd(&sm.nbad, 1);
    }
    for (int w = tid; w < 27 * C; w += kStreamNT) {
      const int b = sp.blocks[c0 + w / 27];
      if (b < 0 || b >= kp.nblocks) continue;  // counted above
      const int nb = kp.nbr[27 * (int64_t)b + w % 27];
      if (!(nb >= 0 && nb < kp.nsrc && block_edge(kp, nb) == E &&
            (kp.out_off ? kp.out_off[nb] : (int64_t)nb * kNV * E * E * E) % kAlign == 0))
        atomicAdd(&sm.nbad, 1);
    }
  }
  __syncthreads();
  if (sm.nbad) {
    if (tid == 0) {
      if (shape_ok) atomicAdd(&kp.counters[1], (unsigned long long)C * (E * E * E / sp.quads));
      // the item's diagnostics record holds nothing
      if (kp.diag & kDiagSpeed) kp.ws_smax[item] = 0.0;
      if (kp.diag & kDiagSums)
        for (int k = 0; k < 2 * kNV; ++k) kp.ws_sums[(size_t)item * 2 * kNV + k] = 0.0;
    }
    return;  // uniform over the workgroup
  }
  StreamChain<T, E, ORDER, P, SPLITB, FLUX> ch{kp, sp, sm};
  ch.tid = tid;
  ch.quad = quad;
  ch.a0 = kTile * (quad & 1);
  ch.b0 = kTile * (quad >> 1);
  ch.chain0 = c0;
  ch.C = C;
  ch.item = item;
  ch.cf = make_coef<T>(kp, sp.blocks[c0], ch.dh);
  ch.run_chain();
}

}  // namespace tvd
