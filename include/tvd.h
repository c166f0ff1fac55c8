/*
 * tvd.h -- C ABI of libtvd, the MI355X (gfx950) library that advances a
 * batch of ghosted cubic blocks of cells by one step of GAMER's dimensionally
 * split relaxing TVD scheme for the Euler equations (Schive, Tsai & Chiueh,
 * "GAMER: a GPU-Accelerated Adaptive Mesh Refinement Code for Astrophysics",
 * Sec. 2.2, Sec. 3.1 and Sec. 3.4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int status: 0 = TVD_OK, < 0 an error, > 0 a
 *   warning.  No exception crosses this boundary and nothing calls exit().
 *   Arguments are validated on the host before any launch; an invalid call
 *   launches nothing.  tvd_last_error() gives the text of the last failure.
 * - Pointers named d_* are device pointers on the context's device; they are
 *   owned by the caller, who keeps them alive until the work queued on the
 *   stream has finished.  The library never frees or keeps them.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Every call only enqueues work on that stream and returns; nothing
 *   synchronises except tvd_read_flags(), tvd_autotune() and the create,
 *   destroy and sequence-create calls.
 * - Variables are stored as five consecutive cubes per block, in the order
 *   (rho, m_x, m_y, m_z, e): mass density, momentum density, total energy
 *   density (Eqs. MassConserve-EnergyConserve, ThermalEnergy, EOS).  Within
 *   a cube x is fastest, then y, then z.  A "ghosted" block of interior edge
 *   n holds (n+6)^3 cells per variable: the n^3 interior plus three ghost
 *   zones on every side (the seven-point stencil of Sec. 2.2).  An
 *   "interior" block holds n^3 cells per variable.
 * - The element type of every state buffer is the batch dtype (TVD_F32:
 *   float, TVD_F64: double); time steps, zone sizes, gamma, speeds and sums
 *   are always double.
 * - A context is not thread safe: use one per host thread.  Its workspace
 *   (per-block partials, the persistent kernel's work plan) is shared by the
 *   calls made on it, so calls on one context that could run at the same time
 *   on different streams race: order them (one stream, or events).
 */
#ifndef TVD_H
#define TVD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
    TVD_OK = 0,
    TVD_WARN_FLOORED = 1,         /* tvd_read_flags: some cells had P < p_floor   */
    TVD_ERR_INVALID_ARG = -1,     /* a NULL pointer, a bad size or enum value      */
    TVD_ERR_UNSUPPORTED = -2,     /* valid request this build does not implement  */
    TVD_ERR_HIP = -3,             /* a HIP runtime call failed (text in last_error)*/
    TVD_ERR_NONPHYSICAL = -4,     /* tvd_read_flags: rho <= 0 or non-finite cells  */
    TVD_ERR_ALIAS = -5,           /* input and output buffers overlap              */
    TVD_ERR_STATE = -6            /* call not allowed in the current state         */
};

enum { TVD_F32 = 1, TVD_F64 = 2 };            /* state element type              */
enum { TVD_XYZ = 0, TVD_ZYX = 1 };            /* forward / backward sweep triple  */
enum { TVD_LAYOUT_GHOSTED = 0, TVD_LAYOUT_INTERIOR = 1 };

/* flags of tvd_patch_advance: which kernel runs */
enum {
    TVD_KERNEL_AUTO = 0,       /* uniform edge: BATCHED; mixed edges: PERSISTENT  */
    TVD_KERNEL_BATCHED = 1,    /* LDS-staged batched kernel, FP32 or FP64; with
                                  mixed edges one launch per edge               */
    TVD_KERNEL_PLAIN = 2,      /* plain FP64 kernel, one workgroup per 8^3 block  */
    TVD_KERNEL_PERSISTENT = 3  /* FP32, any edges, in one persistent launch:
                                  one workgroup per CU draws blocks from
                                  per-XCD work queues, edge 16 first; an
                                  edge-8 block takes a quarter of a workgroup */
};

typedef struct tvd_ctx tvd_ctx;

/*
 * A batch of blocks.  Every block b has an interior edge e_b (8 or 16), a
 * time step dt_b and a zone size dh_b.
 *   edge      uniform interior edge when d_edge == NULL: 8 or 16; also 32
 *             for tvd_patch_advance_stream, tvd_max_signal_speed,
 *             tvd_dt_from_speed, tvd_conservation_sums and tvd_fill_ghosts
 *             (the other entry points: TVD_ERR_INVALID_ARG).
 *   d_edge    [n_blocks] device int32 edges, or NULL.  When non-NULL the
 *             offsets below are required.
 *   d_in_off  [n_blocks] device int64: element offset of block b's ghosted
 *             data (5 cubes of (e_b+6)^3) from the base pointer, or NULL for
 *             dense packing b * 5 * (edge+6)^3.
 *   d_out_off [n_blocks] device int64: element offset of block b's interior
 *             data (5 cubes of e_b^3), or NULL for dense b * 5 * edge^3.
 *   d_dt,d_dh [n_blocks] device double, or NULL to use the scalars dt, dh.
 * Offsets must keep every block inside the buffers the caller passes; the
 * library cannot check device arrays and reads them as given.
 */
typedef struct tvd_batch {
    int32_t dtype;
    int32_t n_blocks;
    int32_t edge;
    int32_t reserved;
    const int32_t *d_edge;
    const int64_t *d_in_off;
    const int64_t *d_out_off;
    const double *d_dt;
    const double *d_dh;
    double dt;
    double dh;
} tvd_batch;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`: allocates the workspace that holds
 * per-block partial results and the health counters.  Synchronous. */
int tvd_create(tvd_ctx **out, int device);
/* Free the context and its workspace; waits for the device first. */
int tvd_destroy(tvd_ctx *ctx);
/* Static text for a status code. */
const char *tvd_status_string(int status);
/* Text of the last failing call on this context (empty if none). */
const char *tvd_last_error(const tvd_ctx *ctx);
/* Grow the workspace to hold per-block partials (and the persistent kernel's
 * work plan) of n_blocks blocks; tvd_create reserves 1024.  This is the only
 * call that allocates after tvd_create: the advance, signal-speed and sums
 * entry points never allocate or synchronise, and return TVD_ERR_STATE when
 * a batch needs more workspace than is reserved (fused d_smax / d_sums, the
 * persistent kernel, tvd_max_signal_speed, tvd_conservation_sums).
 * Synchronous (waits for the device before replacing the buffers).  Growing
 * the workspace retires every graph captured earlier on this context: their
 * tvd_graph_launch returns TVD_ERR_STATE.  TVD_ERR_STATE during a
 * tvd_graph_begin / tvd_graph_end capture; no-op if n_blocks is already
 * reserved. */
int tvd_reserve(tvd_ctx *ctx, int n_blocks);

/* ---- kernel variants (launch shape and LDS layout) ------------------------ */

/* Number of batched-kernel variants compiled into the library. */
int tvd_variant_count(void);
/* Describe variant `index`: block edge, workgroup size, the padding of the
 * LDS rows (layout) and how pencils map to threads (split bit 0: the tail of
 * the second sweep is done as half pencils by two threads each; bit 1: the
 * whole third sweep is).  TVD_ERR_INVALID_ARG for an index out of range.
 * Any output pointer may be NULL. */
int tvd_variant_info(int index, int32_t *edge, int32_t *threads, int32_t *lds_pad,
                     int32_t *split);
/* Select the variant used by TVD_KERNEL_AUTO / TVD_KERNEL_BATCHED for blocks of
 * (dtype, edge); index -1 restores the built-in default.  A variant of
 * another edge, or FP64 with edge 16, is TVD_ERR_UNSUPPORTED. */
int tvd_set_variant(tvd_ctx *ctx, int32_t dtype, int32_t edge, int32_t index);

/* Time every compiled variant serving the batch's (dtype, edge) on the
 * caller's data and select the fastest for later advances of that
 * (dtype, edge) on this context.  The time of a variant is the mean of `reps`
 * forward+backward pairs after one untimed pair.  With d_nbr != NULL the
 * gathering advance is timed (d_u_in interior blocks), else the advance of
 * ghosted blocks.  d_u_out is scratch and its contents are overwritten;
 * d_u_in is only read.  The batch must have a uniform edge.  Synchronous, on
 * a private stream of default priority; not for use during graph capture.
 * Writes the chosen variant index and its time per pair in ms (either
 * pointer may be NULL). */
int tvd_autotune(tvd_ctx *ctx, const tvd_batch *batch, const int32_t *d_nbr,
                 const void *d_u_in, void *d_u_out, double gamma, double p_floor,
                 int32_t reps, int32_t *chosen_index, float *best_ms);

/* ---- the hot path --------------------------------------------------------- */

/*
 * One step of the relaxing TVD scheme on every block (Sec. 2.2; Sec. 3.1 for
 * the one-block-per-workgroup design it re-thinks): per pencil, freezing
 * speed c = |v_d| + c_s and split fluxes F^R, F^L (Eq. LRFlux), the
 * first-order upwind half step (Eq. MidpointValue), fluxes recomputed at the
 * midpoint and corrected to second order with the van Leer limiter (Eqs.
 * 2ndTVDFluxCorr-2ndRFlux, the left-moving flux mirrored), and the full step
 * from u^t (Eq. FullstepValue); three sweeps in the order xyz
 * (sweep_order = TVD_XYZ) or zyx (TVD_ZYX) sharing one dt.
 *   d_u_in   ghosted blocks (read only), d_u_out interior blocks (written);
 *            the two must not overlap (TVD_ERR_ALIAS for equal base pointers
 *            or overlapping dense extents).
 *   gamma    ratio of specific heats (> 1, or exactly 1 for pressureless gas).
 *   p_floor  pressure floor: fluxes and sound speeds use max(P, p_floor); the
 *            stored energy is never changed.
 *   flags    TVD_KERNEL_* (PLAIN requires TVD_F64 and uniform edge 8;
 *            PERSISTENT requires TVD_F32).
 *            FP32 batches take edges 8 and 16, mixed through d_edge; FP64
 *            batches take uniform edge 8 only (else TVD_ERR_UNSUPPORTED).
 *            With mixed edges a block whose d_edge entry is neither 8 nor
 *            16 is not advanced (the persistent kernel also counts it once
 *            as non-physical).  The persistent kernel uses workspace of
 *            n_blocks entries (tvd_reserve; else TVD_ERR_STATE).
 *   d_smax   optional (NULL = skip): receives max over the output interior of
 *            c_s + max(|v_x|, |v_y|, |v_z|) in FP64 (Eq. CFL), fused.
 *   d_sums   optional (NULL = skip): receives the five sums over the output
 *            interior of u * dh_b^3, FP64 with Neumaier compensation and a
 *            fixed reduction order (deterministic), fused.
 * Output cells with rho <= 0 or non-finite values, and cells with
 * P < p_floor, are counted on the device (see tvd_read_flags).
 */
int tvd_patch_advance(tvd_ctx *ctx, const tvd_batch *batch, const void *d_u_in,
                      void *d_u_out, int32_t sweep_order, double gamma,
                      double p_floor, int32_t flags, double *d_smax,
                      double *d_sums, void *stream);

/*
 * The same step with the ghost zones gathered on the fly: d_u_in holds the
 * blocks' interiors only (5 cubes of e_b^3 each, at the batch's out offsets,
 * like d_u_out) and the first sweep of every block reads its ghost cells
 * straight from the interiors of the 26 neighbouring blocks named by
 * d_nbr[27*b + r] (region r as for tvd_fill_ghosts), which is the sibling
 * copy of Sec. 2.2 done inside the advance instead of as a separate pass.
 * Every neighbour must exist (index in [0, n_blocks)) and have the block's
 * edge; a block for which one does not is not advanced, its output is left
 * untouched and its e_b^3 cells are counted as non-physical.  d_u_in and
 * d_u_out must be different buffers (the neighbours' inputs are read while
 * outputs are written).  TVD_KERNEL_PLAIN is not available here.
 */
int tvd_patch_advance_gather(tvd_ctx *ctx, const tvd_batch *batch, const int32_t *d_nbr,
                             const void *d_u_in, void *d_u_out, int32_t sweep_order,
                             double gamma, double p_floor, int32_t flags, double *d_smax,
                             double *d_sums, void *stream);

/*
 * Chains of blocks for the streamed advance: chain c is the list
 * d_blocks[d_start[c] .. d_start[c+1]) (device arrays), each block the
 * neighbour of the one before at +1 along the axis that the step sweeps
 * last (z for TVD_XYZ, x for TVD_ZYX: neighbour region 22 resp. 14 of
 * d_nbr).  Every block should belong to exactly one chain; at most 64
 * blocks per chain.
 */
typedef struct {
    int32_t n_chains;
    int32_t n_members;        /* entries of d_blocks                           */
    const int32_t *d_start;   /* [n_chains + 1], d_start[0] = 0                 */
    const int32_t *d_blocks;  /* [n_members]                                    */
} tvd_chains;

/* flags of tvd_patch_advance_stream besides TVD_KERNEL_AUTO (which takes
 * half pencils in FP32 and whole pencils in FP64, the faster layout of
 * each: the FP64 half-pencil kernels run out of registers) */
enum {
    TVD_STREAM_WHOLE_B = 16,  /* second sweep in whole pencils               */
    TVD_STREAM_HALF_B = 32    /* second sweep in half pencils                */
};

/*
 * The same step as tvd_patch_advance_gather (interior blocks in, ghost
 * zones gathered from the 26 neighbours named by d_nbr, interior blocks
 * out; the same arithmetic per cell, so bit-identical results), organised
 * for the MI355X: one workgroup per chain and 16 x 16 tile of the block
 * face (1 tile for edge 16, 4 for edge 32) runs the first two sweeps of a
 * slab of 8 planes at a time in LDS and carries the third sweep's 1-D
 * update along the whole chain in registers.  This is the per-cell work of
 * Sec. 3.1's solver with the third sweep's ghost-zone work of every block
 * but the chain's ends removed; the region rule (three ghost planes on each
 * side) applies to the chain as a whole.
 *   batch    uniform edge 16 or 32 (d_edge NULL; else TVD_ERR_UNSUPPORTED),
 *            TVD_F32 or TVD_F64.
 *   d_u_in, d_u_out  16-byte aligned (else TVD_ERR_INVALID_ARG); block
 *            offsets (d_out_off, or the dense layout) must be multiples of
 *            16 bytes, since rows are read and written 16 bytes at a time.
 *   chains   chains along z for TVD_XYZ, along x for TVD_ZYX.  A chain whose
 *            blocks are not consecutive along that axis, or whose blocks
 *            lack a neighbour of the same edge, or differ in dt or dh, or
 *            has more than 64 blocks, or whose blocks or neighbours sit at
 *            offsets that are not multiples of 16 bytes, is not advanced:
 *            its output is left untouched and its cells are counted as
 *            non-physical.
 *   flags    TVD_KERNEL_AUTO, TVD_STREAM_WHOLE_B or TVD_STREAM_HALF_B (the
 *            layout of the second sweep; all give the same bits).
 *   d_smax, d_sums  as for tvd_patch_advance, over the chains' blocks; they
 *            use n_chains * (1 or 4) workspace entries, one per chain and
 *            tile (tvd_reserve; else TVD_ERR_STATE).
 * Asynchronous on stream; capture-safe.
 */
int tvd_patch_advance_stream(tvd_ctx *ctx, const tvd_batch *batch, const int32_t *d_nbr,
                             const tvd_chains *chains, const void *d_u_in, void *d_u_out,
                             int32_t sweep_order, double gamma, double p_floor, int32_t flags,
                             double *d_smax, double *d_sums, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as tvd_patch_advance_stream, with the same arguments and the same
 * results bit for bit, but the per-tile partials of the fused signal speed
 * and sums live in a static device array of the library (one per device,
 * 5.8 MB, held until the process ends) instead of the context's workspace.
 * It calls no hipMalloc, hipFree or allocating routine and needs no
 * tvd_reserve.
 *   Limit: with d_smax or d_sums, n_chains * (1 for edge 16, 4 for edge 32)
 *            must not exceed 65536 (else TVD_ERR_STATE, nothing launched).
 *   Sharing: every call on a device uses that device's one array; calls
 *            that overlap in time on one device (other streams, other
 *            contexts, other host threads) race and give wrong diagnostics.
 *            Each call's kernel writes every partial the call then reads
 *            (zeros for a refused chain), so nothing is left over from an
 *            earlier call.
 */
int tvd_patch_advance_stream_noalloc(tvd_ctx *ctx, const tvd_batch *batch,
                                     const int32_t *d_nbr, const tvd_chains *chains,
                                     const void *d_u_in, void *d_u_out, int32_t sweep_order,
                                     double gamma, double p_floor, int32_t flags,
                                     double *d_smax, double *d_sums, void *stream);

/* ---- host-resident advance (Sec. 3.1 stream objects, Sec. 3.5) ---------- */

/*
 * How tvd_patch_advance_host moves a host-resident level through the GPU.
 * A launch takes n_streams * groups_per_stream blocks (the paper's N_s x
 * N_g patch groups); stream s carries one copy down, one advance and one
 * copy up of groups_per_stream of them, so that one stream's copies overlap
 * another stream's advance.
 *   n_streams          N_s, 1 .. 16.
 *   groups_per_stream  N_g >= 1 (N_s * N_g <= 2^20).
 *   host_threads       threads of the host's preparation and closing steps,
 *                      1 .. 256.
 *   concurrent         1: the host prepares launch k+1 and closes launch k-1
 *                      while the GPU works on launch k (Sec. 3.5); 0: the
 *                      host waits for each launch before the next.
 *   streams            [n_streams] hipStream_t (void*), created by the caller
 *                      (default priority).
 *   h_stage            page-locked host memory (hipHostMalloc) of at least
 *                      the h_stage_bytes of tvd_pipeline_stage_bytes: two
 *                      launches of ghosted blocks, then two of interiors.
 *                      Pageable memory works but its copies do not overlap.
 *   d_stage            device memory of at least d_stage_bytes: per stream,
 *                      N_g ghosted blocks, then N_g interiors.
 * The staging buffers are the caller's and are overwritten by every call.
 */
typedef struct {
    int32_t n_streams;
    int32_t groups_per_stream;
    int32_t host_threads;
    int32_t concurrent;
    void *const *streams;
    void *h_stage;
    void *d_stage;
} tvd_host_pipeline;

/* Staging sizes in bytes for a pipeline of blocks of `edge` (8 or 16) and
 * `dtype`.  TVD_ERR_INVALID_ARG for sizes outside the limits above. */
int tvd_pipeline_stage_bytes(int32_t dtype, int32_t edge, const tvd_host_pipeline *pipe,
                             int64_t *h_stage_bytes, int64_t *d_stage_bytes);

/*
 * One step (one triple) of a level whose blocks live in host memory, as in
 * the paper's GPU solver (Sec. 3.1: preparation step, copy down, kernel, copy
 * up, closing step, with N_s stream objects; Sec. 3.5: the host's steps
 * overlapped with the GPU's).
 *   batch     dense, uniform edge (FP32: 8 or 16; FP64: 8), scalar dt and dh;
 *             no device arrays (else TVD_ERR_UNSUPPORTED).
 *   h_nbr     host int32 [n_blocks][27]: the block covering each of the 27
 *             regions around block b (region (rx+1) + 3(ry+1) + 9(rz+1)),
 *             every entry in [0, n_blocks) (checked; else
 *             TVD_ERR_INVALID_ARG).
 *   h_u_in    host: n_blocks interior blocks (5 cubes of edge^3 each);
 *   h_u_out   host: the advanced interiors, same layout; must not overlap
 *             h_u_in or h_stage (TVD_ERR_ALIAS).
 *   times     NULL, or double[7] receiving in ms: the call's wall time, the
 *             host's preparation and closing time, the durations of the
 *             copies down, the advances and the copies up summed over
 *             streams and launches (each measured on its stream), and the
 *             GPU's span from the first copy down to the end of the last
 *             copy up.
 * The preparation step copies each ghosted block from the interiors of the
 * block and its neighbours (sibling ghost zones), the closing step copies
 * each result back; the advance is the batched kernel of
 * tvd_patch_advance.  The results equal, bit for bit, tvd_fill_ghosts then
 * tvd_patch_advance on the device.  Synchronous: returns when h_u_out holds
 * every block.  Creates and destroys its HIP events; not capture-safe
 * (TVD_ERR_STATE while capturing).  Health counters as for
 * tvd_patch_advance.
 */
int tvd_patch_advance_host(tvd_ctx *ctx, const tvd_batch *batch, const int32_t *h_nbr,
                           const void *h_u_in, void *h_u_out, const tvd_host_pipeline *pipe,
                           int32_t sweep_order, double gamma, double p_floor, double *times);

/*
 * Eq. (CFL) signal speed: d_smax[0] = max over the interior cells of all
 * blocks of c_s + max(|v_x|, |v_y|, |v_z|), with c_s from max(P, p_floor);
 * evaluated in FP64 from the stored values.  layout selects ghosted or
 * interior blocks (ghost cells are skipped).  Uses n_blocks entries of the
 * workspace (tvd_reserve; else TVD_ERR_STATE).
 */
int tvd_max_signal_speed(tvd_ctx *ctx, const tvd_batch *batch, const void *d_u,
                         int32_t layout, double gamma, double p_floor,
                         double *d_smax, void *stream);

/*
 * Time step from a signal speed (Eq. CFL with Courant number cfl, Sec. 3.4):
 * d_dt_out[b] = cfl * dh_b / d_smax[0] for every block, on the device, so
 * that the next advance can read it through batch->d_dt without a host
 * round trip.
 */
int tvd_dt_from_speed(tvd_ctx *ctx, const tvd_batch *batch, const double *d_smax,
                      double cfl, double *d_dt_out, void *stream);

/*
 * Conservation sums: d_sums[k] = sum over blocks b and interior cells of
 * u_k * dh_b^3, k = 0..4, FP64, Neumaier-compensated, fixed order.  Uses
 * n_blocks entries of the workspace (tvd_reserve; else TVD_ERR_STATE).
 */
int tvd_conservation_sums(tvd_ctx *ctx, const tvd_batch *batch, const void *d_u,
                          int32_t layout, double *d_sums, void *stream);

/*
 * Health counters accumulated by every advance since the last read: output
 * cells with P < p_floor and output cells with rho <= 0 or non-finite values.
 * Synchronises `stream`, then resets the counters.  Returns
 * TVD_ERR_NONPHYSICAL if n_nonphysical > 0, else TVD_WARN_FLOORED if
 * n_floored > 0, else TVD_OK.  Either output pointer may be NULL.
 */
int tvd_read_flags(tvd_ctx *ctx, int64_t *n_floored, int64_t *n_nonphysical,
                   void *stream);

/*
 * Ghost-zone fill by sibling copy (Sec. 2.2: ghost zones of a patch are
 * copied from its siblings when they exist).  For every block b of the batch
 * and every ghost cell of its ghosted copy, the value is read from the
 * interior of the block that covers that cell: d_nbr[27*b + r] names that
 * block for the neighbour region r = (rx+1) + 3(ry+1) + 9(rz+1), rx, ry, rz in
 * {-1, 0, 1} (r = 13 is b itself, whose interior is copied too).  A negative
 * entry leaves that region untouched (the caller fills it, e.g. by
 * interpolation from a coarser level).  A neighbour must be a block of the
 * batch (index < n_blocks) with the same edge as b; otherwise the region is
 * left untouched and counted as non-physical.  d_interior uses the batch's out offsets, d_ghosted its in
 * offsets.
 */
int tvd_fill_ghosts(tvd_ctx *ctx, const tvd_batch *batch, const int32_t *d_nbr,
                    const void *d_interior, void *d_ghosted, void *stream);

/*
 * Ghost zones on a coarse-fine boundary (Sec. 2.2: a ghost cell is copied
 * from the sibling patch when it exists, otherwise filled by linear
 * interpolation with the Min-Mod limiter from the patches one level
 * coarser).  For every fine block b and every cell of its ghosted copy in
 * d_fine_ghosted (the fine batch's in offsets):
 *   - if d_nbr[27*b + r] >= 0 for the cell's region r (as for
 *     tvd_fill_ghosts, r = 13 being b itself), the cell is copied from that
 *     block's interior in d_fine_interior (the fine batch's out offsets);
 *   - otherwise, per variable, with f the cell's fine index relative to the
 *     corner of the central coarse block (f = 2 * d_corigin[3*b + axis] +
 *     cell - 3 along each axis), c = floor(f / 2) the coarse cell and
 *     d = -1/4 (f even) or
 *     +1/4 (f odd): u_c + dx s_x + dy s_y + dz s_z, summed in that order,
 *     s_axis = minmod(u_{c+1} - u_c, u_c - u_{c-1}) along the axis, minmod
 *     being 0 unless both differences are positive or both negative, else
 *     the one of smaller magnitude (the second on a tie).
 * The coarse level is a batch of blocks of uniform edge 8 (patches) or 16
 * (2^3 patch groups), interiors in d_coarse_interior at its out offsets,
 * same dtype.  d_cnbr[27*b + r] names the coarse block at offset r around
 * the central coarse block, the one holding b's parent patch (r = 13), and
 * d_corigin[3*b + 0..2] (x, y, z) is b's lower corner, in coarse cells,
 * relative to the central block's: 0 or 4 for 8^3 fine patches under 8^3
 * coarse patches, 0 for 16^3 fine groups under 8^3 patches, 0 or 8 for
 * 16^3 fine groups under 16^3 groups.  A cell whose coarse stencil leaves
 * those 27 blocks, or names a coarse index outside [0, coarse n_blocks), is
 * left untouched and counted as non-physical.  Proper nesting (every
 * refined patch has its 26 neighbours) makes every needed entry valid.
 * Asynchronous on stream.
 */
int tvd_fill_ghosts_amr(tvd_ctx *ctx, const tvd_batch *fine, const int32_t *d_nbr,
                        const void *d_fine_interior, void *d_fine_ghosted,
                        const tvd_batch *coarse, const void *d_coarse_interior,
                        const int32_t *d_cnbr, const int32_t *d_corigin, void *stream);

/*
 * The coarse-fine ghost zones of a gathering advance (Sec. 2.2: a ghost cell
 * is copied from the sibling when it exists, else interpolated from the
 * level one coarser; here the copy is the gathering advance's own read of
 * the sibling's interior, and only the interpolated cells are produced).
 * The fine level's interior buffer d_fine_interior holds n_sources blocks:
 * the fine batch's n_blocks real blocks (dense, uniform edge 8 or 16), then
 * source-only blocks that stand in for missing siblings.  For every real
 * block b and every ghost cell of b whose region r has d_nbr[27*b + r] =
 * s with n_blocks <= s < n_sources, the cell is interpolated exactly as in
 * tvd_fill_ghosts_amr (same corigin, cnbr and coarse batch conventions),
 * from the coarse level at time fraction w, each coarse value being
 * old + w (new - old) (w = 0: d_coarse_old alone; d_coarse_new may then be
 * NULL), and written into block s's interior at the cell's position
 * relative to s.  Cells with a real sibling (s < n_blocks) are left to the
 * advance.  A cell needed by several real blocks receives the same value
 * from each.  Then tvd_patch_advance_flux_gather with the same table and
 * n_sources advances the real blocks.  A source index at or beyond
 * n_sources, or a coarse stencil leaving the 27 coarse blocks, is counted
 * as non-physical and the cell left untouched.  The fine batch may hold at
 * most 1 290 555 blocks (one launch of 26 x 128 work-items per block);
 * more is TVD_ERR_UNSUPPORTED.  Asynchronous on stream.
 */
int tvd_fill_coarse_fine(tvd_ctx *ctx, const tvd_batch *fine, const int32_t *d_nbr,
                         int32_t n_sources, void *d_fine_interior, const tvd_batch *coarse,
                         const void *d_coarse_old, const void *d_coarse_new, double w,
                         const int32_t *d_cnbr, const int32_t *d_corigin, void *stream);

/* ---- closing step of a level pair (Sec. 2.1 step 3, Sec. 3.1) --------------- */

/*
 * Patch-boundary flux record of a block of edge e (a multiple of 8): the
 * fluxes across the boundaries of each 8^3 patch in it, which the closing
 * step of Sec. 3.1 routes to the coarse-fine flux correction of Sec. 2.1.
 * 3 * (e/8 + 1) * 5 * e^2 values of the batch's dtype:
 *   record[((d * (e/8 + 1) + q) * 5 + k) * e * e + a * e + b]
 * is the flux of variable k (rho, m_x, m_y, m_z, e) through the face plane
 * f = 8 q along axis d (0 = x), i.e. through interface f - 1/2, at face cell
 * (a, b) = the two other axes, the higher-numbered first (x: (z, y);
 * y: (z, x); z: (y, x)).  It is the flux H of Eq. (FullstepValue) in the
 * sweep along d (u_i -= dt/dh (H at i+1 - H at i)), so a patch changes by
 * exactly what its six faces carry.  Records are packed densely in block
 * order (offset b * record size) unless an int64 offset array is given.
 */

/*
 * tvd_patch_advance that also writes every block's flux record to d_flux
 * (at d_flux_off[b], or densely when NULL; required with mixed edges): each
 * entry receives w H with w = flux_weight rounded to the dtype, replacing
 * the entry (accumulate = 0) or added to it (accumulate = 1), so that the
 * records of a level's sub-steps can be summed with time weights (w = 1/2
 * for each of two sub-steps of half the coarse step; w = 1, accumulate = 0
 * gives H itself).  Ghosted input as for tvd_patch_advance; flags AUTO,
 * BATCHED or PERSISTENT (TVD_KERNEL_PLAIN is TVD_ERR_UNSUPPORTED).  The
 * batched kernel runs its default launch variant here whatever the tuner
 * chose.  d_flux must not overlap the state buffers.
 */
int tvd_patch_advance_flux(tvd_ctx *ctx, const tvd_batch *batch, const void *d_u_in,
                           void *d_u_out, void *d_flux, const int64_t *d_flux_off,
                           double flux_weight, int32_t accumulate, int32_t sweep_order,
                           double gamma, double p_floor, int32_t flags, double *d_smax,
                           double *d_sums, void *stream);

/*
 * tvd_patch_advance_flux reading its ghost zones from the neighbours'
 * interiors (as tvd_patch_advance_gather) instead of a ghosted copy: d_u_in
 * holds n_sources interior blocks (0: n_blocks), the batch's real blocks
 * first, then source-only blocks that d_nbr may name as neighbours but that
 * are not advanced (the stand-ins for missing siblings that
 * tvd_fill_coarse_fine fills).  Uniform edge, batched kernel (flags AUTO or
 * BATCHED); the other arguments as for tvd_patch_advance_flux.
 */
int tvd_patch_advance_flux_gather(tvd_ctx *ctx, const tvd_batch *batch, const int32_t *d_nbr,
                                  int32_t n_sources, const void *d_u_in, void *d_u_out,
                                  void *d_flux, const int64_t *d_flux_off, double flux_weight,
                                  int32_t accumulate, int32_t sweep_order, double gamma,
                                  double p_floor, int32_t flags, double *d_smax, double *d_sums,
                                  void *stream);

/*
 * tvd_patch_advance_flux_gather organised as tvd_patch_advance_stream
 * (chains of blocks along the axis swept last, the third sweep carried
 * along each chain in registers): the same state and the same flux records
 * bit for bit (Sec. 3.1, step 8: the fluxes across patch boundaries).  Each
 * chain block records the fluxes through its own planes at multiples of 8
 * cells, a plane between two chain blocks in both blocks' records, as the
 * per-block advance does.
 *   batch    TVD_F32, dense blocks of uniform edge 16 (else
 *            TVD_ERR_UNSUPPORTED); d_u_in holds n_sources blocks (real ones
 *            first, then source-only stand-ins), d_u_out n_blocks.
 *   chains   as for tvd_patch_advance_stream; every neighbour of a chain
 *            block must be a block below n_sources, of edge 16.  Blocks
 *            that no valid chain covers are neither advanced nor recorded.
 *   d_flux, d_flux_off, flux_weight, accumulate  as for
 *            tvd_patch_advance_flux; d_flux must not overlap the states.
 * No fused diagnostics.  Asynchronous on stream; capture-safe.
 */
int tvd_patch_advance_stream_flux(tvd_ctx *ctx, const tvd_batch *batch, const int32_t *d_nbr,
                                  int32_t n_sources, const tvd_chains *chains,
                                  const void *d_u_in, void *d_u_out, void *d_flux,
                                  const int64_t *d_flux_off, double flux_weight,
                                  int32_t accumulate, int32_t sweep_order, double gamma,
                                  double p_floor, void *stream);

/*
 * d_out[i] = d_a[i] + w (d_b[i] - d_a[i]), i < n, in the dtype (w rounded
 * to it): linear interpolation in time between two states of a level, e.g.
 * the coarse level half-way through its step for the ghost zones of a fine
 * sub-step (Sec. 2.1: the time step of level l may be half that of level
 * l-1).  d_out may be d_a or d_b; n <= 2^38.  Asynchronous on stream.
 */
int tvd_lerp(tvd_ctx *ctx, int32_t dtype, int64_t n, const void *d_a, const void *d_b,
             void *d_out, double w, void *stream);

/*
 * Restriction (Sec. 2.1: a coarse patch overlaid by its children takes the
 * spatial average of the fine-grid values).  d_rows[5*r .. 5*r+4] =
 * (f, c, ox, oy, oz): the (e_f/2)^3 coarse cells of coarse block c (interior
 * layout, d_coarse at the coarse batch's out offsets) starting at cell
 * (ox, oy, oz) become the means of their eight children in fine block f
 * (interior layout, d_fine at the fine batch's out offsets), summed in the
 * order (dz, dy, dx) = 000, 001, .., 111 and multiplied by 1/8.  Rows must
 * not write one cell twice, and no row may read a block another row writes.
 * A row naming a block out of range, an edge other than 8 or 16, or cells
 * outside its blocks is skipped and its cells counted as non-physical (once
 * when its fine block is not a block of the batch).  d_coarse and d_fine may
 * be the same buffer (one batch holding both
 * levels).  Asynchronous on stream.
 */
int tvd_restrict(tvd_ctx *ctx, const tvd_batch *coarse, void *d_coarse, const tvd_batch *fine,
                 const void *d_fine, const int32_t *d_rows, int32_t n_rows, void *stream);

/*
 * Coarse-fine flux correction (Sec. 2.1: the coarse cells next to a
 * coarse-fine interface are corrected with the difference between the
 * coarse-grid and fine-grid fluxes, so that what leaves the coarse side
 * enters the fine side).  Both levels were advanced with the same dt, and
 * their flux records (tvd_patch_advance_flux) are read, never written.
 * d_rows[8*r .. 8*r+7] = (c, d, s, qc, oa, ob, f, qf): on plane qc along
 * axis d of coarse block c, the face cells (oa + a, ob + b), a, b in
 * [0, e_f/2), are covered by the 2 x 2 face cells (2a + i, 2b + j) of plane
 * qf of fine block f.  The coarse cell on side s of the plane (s = 1: the
 * cell below it, whose + face the plane is; s = 0: the cell above it) gets
 *   u + lam (H_c - H_f)   (s = 1)   or   u - lam (H_c - H_f)   (s = 0),
 * lam = dt_c / dh_c of block c, H_f = (((f00 + f01) + f10) + f11) / 4.
 * Rows are grouped by pass p = 2 d + s (x-, x+, y-, y+, z-, z+) with
 * pass_count[p] rows each (a host array); the passes run in that order, one
 * launch each, and rows of one pass must not share a cell.  d_coarse is
 * read and written (interior layout, the coarse batch's out offsets); flux
 * offsets as for tvd_patch_advance_flux.  A row naming a block out of range
 * or cells outside its blocks is skipped and its cells counted as
 * non-physical (once when its fine block is not a block of the batch).
 * Asynchronous on stream.
 */
int tvd_flux_correct(tvd_ctx *ctx, const tvd_batch *coarse, void *d_coarse,
                     const void *d_coarse_flux, const int64_t *d_coarse_flux_off,
                     const tvd_batch *fine, const void *d_fine_flux,
                     const int64_t *d_fine_flux_off, const int32_t *d_rows,
                     const int32_t pass_count[6], void *stream);

/*
 * The closing of one level pair in a single launch: the restriction rows of
 * tvd_restrict and the face rows of tvd_flux_correct, the latter grouped by
 * coarse block instead of by pass.  Group g holds the rows
 * [d_face_start[g], d_face_start[g+1]) of d_face_rows (n_face_rows rows in
 * all, d_face_start has n_face_groups + 1 entries); all rows of a group name
 * the same coarse block, no two groups name the same one, and a group's
 * rows are sorted by pass 2 d + s.  Each group is applied by one workgroup in
 * that order, so a cell on several interfaces gets its corrections in the
 * order x-, x+, y-, y+, z-, z+, with the same arithmetic as
 * tvd_flux_correct: the result is bit for bit that of tvd_restrict followed
 * by tvd_flux_correct.  The restriction rows and the face rows must not
 * write the same cell (refined and unrefined patches never share one).  A
 * group whose rows name different coarse blocks or whose range leaves
 * [0, n_face_rows) is skipped and counted once as non-physical; rows as for
 * the two separate calls otherwise.  Asynchronous on stream.
 */
int tvd_close_level(tvd_ctx *ctx, const tvd_batch *coarse, void *d_coarse,
                    const void *d_coarse_flux, const int64_t *d_coarse_flux_off,
                    const tvd_batch *fine, const void *d_fine, const void *d_fine_flux,
                    const int64_t *d_fine_flux_off, const int32_t *d_restrict_rows,
                    int32_t n_restrict, const int32_t *d_face_rows, int32_t n_face_rows,
                    const int32_t *d_face_start, int32_t n_face_groups, void *stream);

/* ---- Poisson equation on patch groups (Sec. 2.3, Sec. 3.2) -------------------- */

/*
 * Red-black successive overrelaxation for the discrete Poisson equation
 * (Eq. DiscretePoisson, the 7-point Laplacian) on n_groups patch groups of
 * 16^3 cells, each with Dirichlet values in a one-cell ghost layer (Sec. 2.3:
 * refined levels are solved patch by patch with boundary values from the
 * coarser level; Sec. 3.2: a patch group holds 18^3 potentials and 16^3
 * densities).  Per iteration, the even cells (x + y + z even, interior
 * indices 0..15) are updated from the odd ones, then the odd cells from the
 * updated even ones, each by Eq. (Residual)
 *   R = (phi_x+1 + phi_y+1 + phi_z+1 + phi_x-1 + phi_y-1 + phi_z-1 - 6 phi) - s,
 *   s = (4 pi G dh^2) rho   (the factor computed in FP64, rounded once),
 * and Eq. (SOR) phi <- phi + (omega/6) R, summed in that order in the
 * batch's precision without contraction.  A group stops after max_iter
 * iterations, or, once min_iter are done, after the first iteration whose
 * residual one-norm (the |R| of that iteration's updates, summed in FP64) is
 * <= tol * (sum |s| + 6 sum |phi|).
 *   dtype      TVD_F32 or TVD_F64.
 *   d_phi_in   [n_groups][18][18][18] (x fastest): initial guess inside, the
 *              Dirichlet values on the ghost layer; read only.
 *   d_rho      [n_groups][16][16][16] densities.
 *   d_phi_out  [n_groups][16][16][16] the solution (must not overlap d_phi_in).
 *   G, dh      gravitational constant and zone size (d_dh: [n_groups] FP64
 *              zone sizes, or NULL).
 *   omega      in (0, 2); 0 selects 2 / (1 + sin(pi/17)), the optimum for a
 *              16^3 Dirichlet box.
 *   tol        in (0, 1); 0 selects 16 unit roundoffs of the dtype.
 *   d_iters    optional [n_groups] int32: iterations done per group.
 *   d_resid    optional [n_groups] FP64: the last residual one-norm.
 * Asynchronous on stream.
 */
int tvd_poisson_sor(tvd_ctx *ctx, int32_t dtype, int32_t n_groups, const void *d_phi_in,
                    const void *d_rho, void *d_phi_out, double G, double dh, const double *d_dh,
                    double omega, int32_t min_iter, int32_t max_iter, double tol,
                    int32_t *d_iters, double *d_resid, void *stream);

/*
 * The self-gravity source operator G (Sec. 2.3: accelerations from 3-point
 * central differences of the potential; Eqs. MomConserve and EnergyConserve
 * with the flux terms dropped; in the split order xyzGGzyx the two G merge
 * into one with twice the time step, so pass 2 dt there).  For every
 * interior cell of every block (uniform edge 8 or 16, interior layout at
 * the batch's out offsets, updated in place), with dt and dh of the block:
 *   m_d' = m_d + (a rho)(phi_-d - phi_+d),          a = dt / (2 dh),
 *   e'   = e + ((s_x + s_y) + s_z) b,  s_d = (m_d + m_d')(phi_-d - phi_+d),
 *                                                    b = dt / (4 dh),
 * a and b rounded once from FP64; rho unchanged.  The energy gain is the
 * work of the time-centred momentum, so the internal energy is unchanged.
 *   d_phi  [n_blocks][(edge+2)^3] potential with one ghost layer (x fastest),
 *          e.g. a tvd_poisson_sor input whose interior holds its output.
 * TVD_ERR_UNSUPPORTED with mixed edges; at most 2^38 cells per call.
 * Asynchronous on stream.
 */
int tvd_gravity(tvd_ctx *ctx, const tvd_batch *batch, void *d_u, const void *d_phi, void *stream);

/* ---- step sequences as HIP graphs --------------------------------------------- */

typedef struct tvd_graph tvd_graph;

/* Start capturing `stream` (a non-default hipStream_t) into a HIP graph, in
 * thread-local mode: the library calls made on that stream until
 * tvd_graph_end() are recorded, not run.  Every entry point except
 * tvd_read_flags, tvd_autotune and the create/destroy/reserve calls may be
 * recorded; reserve the workspace for the largest batch first.  The graph
 * keeps the pointers and scalars of the recorded calls; per-step data that
 * changes between replays (such as dt) must live in device memory. */
int tvd_graph_begin(tvd_ctx *ctx, void *stream);
/* Stop capturing and instantiate the graph; *out receives the handle. */
int tvd_graph_end(tvd_ctx *ctx, void *stream, tvd_graph **out);
/* Replay a recorded sequence on `stream` (asynchronous).  TVD_ERR_STATE, with
 * nothing launched, when tvd_reserve has replaced the context's workspace
 * since the capture, or the context has been destroyed. */
int tvd_graph_launch(tvd_graph *graph, void *stream);
/* Free a recorded sequence (the caller ensures no replay is in flight). */
int tvd_graph_destroy(tvd_graph *graph);

#ifdef __cplusplus
}
#endif

#endif /* TVD_H */
