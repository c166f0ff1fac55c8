// Internal interface between the C ABI (tvd_capi.hip) and the kernels
// (tvd_kernels.hip).  Host-side only; no device code here.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvd {

// Fused diagnostics of an advance (KParams::diag bits).
constexpr int kDiagSpeed = 1;  // per-block max signal speed into ws_smax
constexpr int kDiagSums = 2;   // per-block compensated sums into ws_sums

// Everything a batch kernel needs, passed by value as the kernel argument.
struct KParams {
  const void* uin;
  void* uout;
  const int32_t* d_edge;
  const int64_t* in_off;
  const int64_t* out_off;
  const double* d_dt;
  const double* d_dh;
  double dt, dh, gamma, pfloor;
  int nblocks;
  int nsrc;                      // blocks a gathering advance may read as neighbours
                                 // (>= nblocks; the extra ones are sources only)
  int edge;                      // uniform edge (0 when d_edge is used)
  const int32_t* nbr;            // [nblocks][27] neighbour table (gather mode)
  int diag;                      // kDiagSpeed | kDiagSums
  double* ws_smax;               // [nblocks] per-block max signal speed
  double* ws_sums;               // [nblocks][10] per-block (sum, comp) x 5
  unsigned long long* counters;  // [0] floored, [1] non-physical
  void* flux;                    // patch-boundary flux records (null: none)
  const int64_t* flux_off;       // [nblocks] record offsets, or null for dense
  double flux_w;                 // records receive flux_w * H ...
  int flux_acc;                  // ... added to what they hold (1) or replacing it (0)
};

// Patch edge: boundary fluxes are recorded on the planes at its multiples.
constexpr int kPatch = 8;
// Values in one block's flux record: 3 axes x (edge/8 + 1) planes x 5
// variables x edge^2 face cells.
constexpr int64_t flux_record_size(int edge) {
  return 3 * (int64_t)(edge / kPatch + 1) * 5 * edge * edge;
}

// Variant of the batched kernel (chosen by the tuner or by default).
struct Variant {
  int edge;      // 8 or 16
  int threads;   // workgroup size
  int pad;       // LDS row padding (layout variant)
  int split;     // bit 0: sweep-1 tail pencils in halves; bit 1: sweep-2 pencils in halves
};

// Work plan of the persistent launch over mixed edges (device memory).
struct FusedPlan {
  int32_t* list;       // [nblocks] edge-16 blocks, then edge-8 blocks
  int32_t* count;      // [2] number of edge-16 and edge-8 blocks
  unsigned* next;      // [8] work counter of each XCD's queue
};

// Launchers.  All return a hipError_t from the launch.
// gather = true: the first sweep reads its pencils straight from the
// interiors of the block and its 26 neighbours (kp.nbr) instead of a
// ghosted copy; kp.uin then holds interior blocks at the out offsets.
hipError_t launch_batched(int dtype, int order, const Variant& v, bool gather, const KParams& kp,
                          hipStream_t s);
// Mixed edges (kp.d_edge, or a uniform kp.edge) in one persistent launch of `workgroups`
// workgroups, after a one-workgroup planning launch.  FP32 only.
hipError_t launch_fused(int dtype, int order, bool gather, const KParams& kp, const FusedPlan& pl,
                        int workgroups, hipStream_t s);
hipError_t launch_plain_f64(int order, const KParams& kp, hipStream_t s);
hipError_t launch_signal_speed(int dtype, int layout, const KParams& kp, hipStream_t s);
hipError_t launch_cons_sums(int dtype, int layout, const KParams& kp, hipStream_t s);
hipError_t launch_finalize_max(const double* ws, int n, double* out, hipStream_t s);
hipError_t launch_finalize_sums(const double* ws, int n, double* out, hipStream_t s);
hipError_t launch_dt_from_speed(const KParams& kp, const double* smax, double cfl,
                                double* dt_out, hipStream_t s);
hipError_t launch_fill_ghosts(int dtype, const KParams& kp, const int32_t* nbr, int max_edge,
                              hipStream_t s);
// Sibling copy, else Min-Mod limited interpolation from the coarse level's
// blocks of edge cedge (8 or 16; cin at coarse offsets coff, or dense); cnbr
// [27 per fine block], corigin [3 per fine block].
hipError_t launch_fill_ghosts_amr(int dtype, const KParams& kp, const int32_t* nbr, int max_edge,
                                  const void* cin, const int64_t* coff, int ncoarse, int cedge,
                                  const int32_t* cnbr, const int32_t* corigin, hipStream_t s);
// Coarse-fine ghost cells of a gathering advance into source-only blocks
// (kp.nblocks real fine blocks of uniform edge kp.edge, nbr entries >=
// kp.nblocks and < kp.nsrc name the stand-ins, interiors at kp.uout), the
// coarse level at old + w (new - old).
hipError_t launch_fill_coarse_fine(int dtype, const KParams& kp, const int32_t* nbr,
                                   const void* cold, const void* cnew, double w,
                                   const int64_t* coff, int ncoarse, int cedge,
                                   const int32_t* cnbr, const int32_t* corigin, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
// Closing step of a level pair: ck is the coarse level (interior blocks read
// and written at uout / out_off, flux records at flux / flux_off), fk the
// fine level (interior blocks read at uin with the interior offsets out_off,
// flux records at flux / flux_off).  rows: [nrows][5] restriction rows, or
// [nrows][8] face rows of one pass.
hipError_t launch_restrict(int dtype, const KParams& ck, const KParams& fk, const int32_t* rows,
                           int nrows, hipStream_t s);
hipError_t launch_flux_correct(int dtype, const KParams& ck, const KParams& fk, const int32_t* rows,
                               int nrows, hipStream_t s);
// Restriction rows and grouped face rows of a level pair in one launch.
hipError_t launch_close_level(int dtype, const KParams& ck, const KParams& fk,
                              const int32_t* rrows, int nr, const int32_t* frows, int nf,
                              const int32_t* start, int ngroups, hipStream_t s);
// The self-gravity operator on the interior blocks at kp.uout (uniform edge
// kp.edge, 8 or 16), potential [nblocks][(edge+2)^3].
hipError_t launch_gravity(int dtype, const KParams& kp, const void* phi, hipStream_t s);
// out[i] = a[i] + w (b[i] - a[i]) over n values.
hipError_t launch_lerp(int dtype, int64_t n, const void* a, const void* b, void* out, double w,
                       hipStream_t s);
// Red-black SOR on ngroups patch groups (18^3 potential in, 16^3 density in,
// 16^3 potential out).
hipError_t launch_sor(int dtype, int ngroups, const void* phi_in, const void* rho, void* phi_out,
                      const double* d_dh, double dh, double G, double omega, double tol,
                      int min_iter, int max_iter, int32_t* iters, double* resid, hipStream_t s);

// The streamed advance over chains of blocks (tvd_stream.hpp): grid = one
// workgroup per chain and 16 x 16 tile of a block face.
struct StreamParams;
hipError_t launch_stream_f32(int order, int edge, bool splitb, const KParams& kp,
                             const StreamParams& sp, hipStream_t s);
hipError_t launch_stream_f64(int order, int edge, bool splitb, const KParams& kp,
                             const StreamParams& sp, hipStream_t s);
// The streamed advance writing (accumulate false) or adding to the flux
// records at kp.flux (kp.flux_w, kp.flux_off): FP32, edge 16.
hipError_t launch_stream_flux_f32(int order, bool accumulate, const KParams& kp,
                                  const StreamParams& sp, hipStream_t s);
// Zero n doubles (fill kernel, capture-safe).
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s);

// The host-resident advance (tvd_pipeline.hip): n_blocks interior blocks of
// uniform edge in host memory (h_in, h_out), neighbour table h_nbr
// [n_blocks][27], advanced in launches of ns x ng blocks on the ns streams.
// kp carries dt, dh, gamma, p_floor and the health counters.
struct HostPipe {
  int dtype, edge, order;
  int64_t n_blocks;
  const int32_t* h_nbr;
  const void* h_in;
  void* h_out;
  int ns, ng, threads;
  bool concurrent;
  void* h_stage;   // page-locked: 2 x ns x ng ghosted blocks, then 2 x ns x ng interiors
  void* d_stage;   // per stream: ng ghosted blocks, then ng interiors
  const hipStream_t* streams;
  Variant variant;
  KParams kp;
};
// Runs the whole pipeline and returns when h_out holds every result;
// times (optional): wall, host preparation, host closing, the summed
// durations of the copies down, the advances and the copies up, and the
// GPU's span from the first copy down to the last copy up (ms).
hipError_t run_host_pipeline(const HostPipe& hp, double times[7]);

// Variants compiled into the library.
int variant_count();
Variant variant_at(int i);
bool variant_supported(int dtype, const Variant& v);

}  // namespace tvd
