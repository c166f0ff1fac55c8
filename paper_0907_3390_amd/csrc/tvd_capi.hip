// The C ABI of libtvd (declared in include/tvd.h): contexts, argument
// validation, workspace management and kernel dispatch.  Every check that
// can be made on the host is made before anything is launched.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "tvd.h"
#include "tvd_internal.hpp"
#include "tvd_stream_params.hpp"

#include <memory>
#include <mutex>

// Scratch of the allocation-free streamed advance
// (tvd_patch_advance_stream_noalloc): per-tile partials of the fused signal
// speed ([kScratchParts] doubles) followed by those of the compensated sums
// ([kScratchParts][10]), 5.8 MB.  Each device that loads the library holds
// its own copy until the process ends.  In host code `scratch` names a host
// stand-in, never the device memory: kernels and fills get the address that
// hipGetSymbolAddress returned for the current device (scratch_address).
constexpr int64_t kScratchParts = 65536;
static __device__ __align__(256) double scratch[11 * kScratchParts];

// Generation of a context's workspace, shared with the graphs captured on
// it: it changes whenever tvd_reserve replaces the workspace buffers (and
// when the context is destroyed), so that a graph holding the old pointers
// is refused instead of replayed into freed memory.
using WsGeneration = std::shared_ptr<unsigned long long>;
constexpr unsigned long long kWsGone = ~0ull;

struct tvd_graph {
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  WsGeneration ws_gen;            // the capturing context's generation counter
  unsigned long long gen = 0;     // its value when the capture ended
};

struct tvd_ctx {
  int device = 0;
  std::string err;
  // workspace: per-block partials and health counters
  double* ws_smax = nullptr;
  double* ws_sums = nullptr;
  unsigned long long* counters = nullptr;
  int ws_blocks = 0;
  WsGeneration ws_gen = std::make_shared<unsigned long long>(0ull);
  bool capturing = false;  // between tvd_graph_begin and tvd_graph_end
  // work plan of the persistent launch: list [ws_blocks], count [2], next [8]
  int32_t* plan_list = nullptr;
  int32_t* plan_small = nullptr;  // count[2] then next[8] (as unsigned)
  int cus = 256;                  // compute units (one persistent workgroup each)
  // tuned variants, per dtype (index 0: FP32, 1: FP64) and edge (0: 8, 1: 16)
  int tuned[2][2] = {{-1, -1}, {-1, -1}};
  // device address of this device's static scratch array
  double* scratch = nullptr;
};

namespace {

int fail(tvd_ctx* ctx, int status, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return status;
}

int hip_fail(tvd_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, TVD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Make `device` current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Device address of the static scratch array on `device`, looked up once per
// device (with that device current) and kept for the life of the process.
double* scratch_address(int device) {
  static std::mutex mu;
  static double* addr[64] = {};
  static bool done[64] = {};
  if (device < 0 || device >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!done[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    addr[device] = static_cast<double*>(p);
    done[device] = true;
  }
  return addr[device];
}

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}

// Grow the workspace to hold n blocks (tvd_create and tvd_reserve only: the
// other entry points never allocate).  Replacing the buffers moves the
// workspace generation on, which retires graphs captured before.
int reserve(tvd_ctx* ctx, int n) {
  if (n <= ctx->ws_blocks) return TVD_OK;
  ++*ctx->ws_gen;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
  (void)hipFree(ctx->ws_smax);
  (void)hipFree(ctx->ws_sums);
  (void)hipFree(ctx->plan_list);
  ctx->ws_smax = nullptr;
  ctx->ws_sums = nullptr;
  ctx->plan_list = nullptr;
  ctx->ws_blocks = 0;
  const int cap = n < 1024 ? 1024 : n;
  e = hipMalloc(&ctx->ws_smax, sizeof(double) * (size_t)cap);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(workspace)");
  e = hipMalloc(&ctx->ws_sums, sizeof(double) * 10 * (size_t)cap);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(workspace)");
  e = hipMalloc(&ctx->plan_list, sizeof(int32_t) * (size_t)cap);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(workspace)");
  ctx->ws_blocks = cap;
  return TVD_OK;
}

// The workspace must already hold n blocks: the hot entry points check, they
// do not allocate.
int need_workspace(tvd_ctx* ctx, int n) {
  if (n <= ctx->ws_blocks) return TVD_OK;
  return fail(ctx, TVD_ERR_STATE,
              "the workspace holds %d blocks and this batch has %d: call tvd_reserve first",
              ctx->ws_blocks, n);
}

size_t elem_size(int dtype) { return dtype == TVD_F32 ? 4 : 8; }

// Host-side checks of a batch descriptor.  Edge 32 only where the caller
// serves it (the streamed advance and the per-cell reductions and fills).
int check_batch(tvd_ctx* ctx, const tvd_batch* b, bool allow32 = false) {
  if (!b) return fail(ctx, TVD_ERR_INVALID_ARG, "batch is NULL");
  if (b->dtype != TVD_F32 && b->dtype != TVD_F64)
    return fail(ctx, TVD_ERR_INVALID_ARG, "dtype %d is neither TVD_F32 nor TVD_F64", b->dtype);
  if (b->n_blocks < 0) return fail(ctx, TVD_ERR_INVALID_ARG, "n_blocks %d < 0", b->n_blocks);
  if (b->d_edge == nullptr) {
    if (b->edge != 8 && b->edge != 16 && !(allow32 && b->edge == 32))
      return fail(ctx, TVD_ERR_INVALID_ARG, "edge %d is not 8 or 16%s", b->edge,
                  allow32 ? " or 32" : "");
  } else if (b->d_in_off == nullptr || b->d_out_off == nullptr) {
    return fail(ctx, TVD_ERR_INVALID_ARG, "mixed edges (d_edge) need d_in_off and d_out_off");
  }
  if (b->d_dt == nullptr && !(b->dt >= 0.0))
    return fail(ctx, TVD_ERR_INVALID_ARG, "dt %g must be >= 0", b->dt);
  if (b->d_dh == nullptr && !(b->dh > 0.0))
    return fail(ctx, TVD_ERR_INVALID_ARG, "dh %g must be > 0", b->dh);
  return TVD_OK;
}

int check_gamma(tvd_ctx* ctx, double gamma, double pfloor) {
  if (!(gamma >= 1.0) || !(gamma < 1e6))
    return fail(ctx, TVD_ERR_INVALID_ARG, "gamma %g must be >= 1", gamma);
  if (!(pfloor >= 0.0) || !(pfloor < 1e300))
    return fail(ctx, TVD_ERR_INVALID_ARG, "p_floor %g must be finite and >= 0", pfloor);
  return TVD_OK;
}

tvd::KParams make_params(tvd_ctx* ctx, const tvd_batch* b, const void* uin, void* uout,
                         double gamma, double pfloor) {
  tvd::KParams kp;
  kp.uin = uin;
  kp.uout = uout;
  kp.d_edge = b->d_edge;
  kp.in_off = b->d_in_off;
  kp.out_off = b->d_out_off;
  kp.d_dt = b->d_dt;
  kp.d_dh = b->d_dh;
  kp.dt = b->dt;
  kp.dh = b->dh;
  kp.gamma = gamma;
  kp.pfloor = pfloor;
  kp.nblocks = b->n_blocks;
  kp.nsrc = b->n_blocks;
  kp.edge = b->d_edge ? 0 : b->edge;
  kp.nbr = nullptr;
  kp.diag = 0;
  kp.ws_smax = ctx->ws_smax;
  kp.ws_sums = ctx->ws_sums;
  kp.counters = ctx->counters;
  kp.flux = nullptr;
  kp.flux_off = nullptr;
  kp.flux_w = 1.0;
  kp.flux_acc = 0;
  return kp;
}

tvd::Variant default_variant(int dtype, int edge) {
  if (edge == 16) return tvd::Variant{16, 512, 16, 3};
  return dtype == TVD_F32 ? tvd::Variant{8, 128, 8, 0} : tvd::Variant{8, 256, 8, 0};
}

tvd::Variant chosen_variant(const tvd_ctx* ctx, int dtype, int edge) {
  const int t = ctx->tuned[dtype == TVD_F32 ? 0 : 1][edge == 16 ? 1 : 0];
  if (t >= 0) return tvd::variant_at(t);
  return default_variant(dtype, edge);
}

}  // namespace

extern "C" {

const char* tvd_status_string(int status) {
  switch (status) {
    case TVD_OK: return "ok";
    case TVD_WARN_FLOORED: return "warning: pressure floor applied";
    case TVD_ERR_INVALID_ARG: return "invalid argument";
    case TVD_ERR_UNSUPPORTED: return "unsupported";
    case TVD_ERR_HIP: return "HIP runtime error";
    case TVD_ERR_NONPHYSICAL: return "non-physical state";
    case TVD_ERR_ALIAS: return "input and output overlap";
    case TVD_ERR_STATE: return "call not allowed in this state";
    default: return "unknown status";
  }
}

const char* tvd_last_error(const tvd_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

int tvd_create(tvd_ctx** out, int device) {
  if (!out) return TVD_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return TVD_ERR_INVALID_ARG;
  tvd_ctx* ctx = new tvd_ctx();
  ctx->device = device;
  DeviceGuard g(device);
  if (!g.ok) {
    delete ctx;
    return TVD_ERR_HIP;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      cus > 0)
    ctx->cus = cus;
  if (hipMalloc(&ctx->counters, 4 * sizeof(unsigned long long)) != hipSuccess ||
      hipMemset(ctx->counters, 0, 4 * sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&ctx->plan_small, 16 * sizeof(int32_t)) != hipSuccess ||
      hipMemset(ctx->plan_small, 0, 16 * sizeof(int32_t)) != hipSuccess ||
      reserve(ctx, 1024) != TVD_OK || (ctx->scratch = scratch_address(device)) == nullptr ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(ctx->counters);
    (void)hipFree(ctx->plan_small);
    (void)hipFree(ctx->plan_list);
    (void)hipFree(ctx->ws_smax);
    (void)hipFree(ctx->ws_sums);
    delete ctx;
    return TVD_ERR_HIP;
  }
  *out = ctx;
  return TVD_OK;
}

int tvd_destroy(tvd_ctx* ctx) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  *ctx->ws_gen = kWsGone;  // graphs captured on this context can no longer run
  {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(ctx->ws_smax);
    (void)hipFree(ctx->ws_sums);
    (void)hipFree(ctx->plan_list);
    (void)hipFree(ctx->plan_small);
    (void)hipFree(ctx->counters);
  }
  delete ctx;
  return TVD_OK;
}

int tvd_reserve(tvd_ctx* ctx, int n_blocks) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  if (n_blocks < 0) return fail(ctx, TVD_ERR_INVALID_ARG, "n_blocks %d < 0", n_blocks);
  DeviceGuard g(ctx->device);
  if (n_blocks <= ctx->ws_blocks) return TVD_OK;
  if (ctx->capturing)
    return fail(ctx, TVD_ERR_STATE, "tvd_reserve cannot run during a tvd_graph capture");
  return reserve(ctx, n_blocks);
}

int tvd_variant_count(void) { return tvd::variant_count(); }

int tvd_variant_info(int index, int32_t* edge, int32_t* threads, int32_t* lds_pad,
                     int32_t* split) {
  if (index < 0 || index >= tvd::variant_count()) return TVD_ERR_INVALID_ARG;
  const tvd::Variant v = tvd::variant_at(index);
  if (edge) *edge = v.edge;
  if (threads) *threads = v.threads;
  if (lds_pad) *lds_pad = v.pad;
  if (split) *split = v.split;
  return TVD_OK;
}

int tvd_set_variant(tvd_ctx* ctx, int32_t dtype, int32_t edge, int32_t index) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  if (dtype != TVD_F32 && dtype != TVD_F64)
    return fail(ctx, TVD_ERR_INVALID_ARG, "dtype %d", dtype);
  if (edge != 8 && edge != 16) return fail(ctx, TVD_ERR_INVALID_ARG, "edge %d", edge);
  if (index < -1 || index >= tvd::variant_count())
    return fail(ctx, TVD_ERR_INVALID_ARG, "variant index %d", index);
  if (index >= 0) {
    const tvd::Variant v = tvd::variant_at(index);
    if (v.edge != edge || !tvd::variant_supported(dtype == TVD_F32 ? 1 : 2, v))
      return fail(ctx, TVD_ERR_UNSUPPORTED, "variant %d does not serve dtype %d edge %d", index,
                  dtype, edge);
  }
  ctx->tuned[dtype == TVD_F32 ? 0 : 1][edge == 16 ? 1 : 0] = index;
  return TVD_OK;
}

}  // extern "C"

namespace {

// Shared body of tvd_patch_advance (nbr == NULL: ghosted input) and
// tvd_patch_advance_gather (nbr != NULL: interior input, ghosts gathered).
int advance_impl(tvd_ctx* ctx, const tvd_batch* batch, const void* d_u_in, void* d_u_out,
                 int32_t sweep_order, double gamma, double p_floor, int32_t flags,
                 double* d_smax, double* d_sums, void* stream, const int32_t* d_nbr,
                 void* d_flux = nullptr, const int64_t* d_flux_off = nullptr,
                 double flux_w = 1.0, int flux_acc = 0, int32_t n_sources = 0) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, batch);
  if (st) return st;
  if (n_sources == 0) n_sources = batch->n_blocks;
  if (n_sources < batch->n_blocks)
    return fail(ctx, TVD_ERR_INVALID_ARG, "n_sources %d < n_blocks %d", n_sources,
                batch->n_blocks);
  if (n_sources > batch->n_blocks && (batch->d_edge || !d_nbr))
    return fail(ctx, TVD_ERR_UNSUPPORTED,
                "source-only blocks need a gathering advance of uniform edge");
  if ((st = check_gamma(ctx, gamma, p_floor))) return st;
  if (sweep_order != TVD_XYZ && sweep_order != TVD_ZYX)
    return fail(ctx, TVD_ERR_INVALID_ARG, "sweep_order %d", sweep_order);
  if (flags != TVD_KERNEL_AUTO && flags != TVD_KERNEL_BATCHED && flags != TVD_KERNEL_PLAIN &&
      flags != TVD_KERNEL_PERSISTENT)
    return fail(ctx, TVD_ERR_INVALID_ARG, "flags %d", flags);
  if (batch->n_blocks == 0) return TVD_OK;
  if (!d_u_in || !d_u_out) return fail(ctx, TVD_ERR_INVALID_ARG, "state pointer is NULL");
  if (d_flux) {
    if (flags == TVD_KERNEL_PLAIN)
      return fail(ctx, TVD_ERR_UNSUPPORTED, "the plain kernel records no fluxes");
    if (batch->d_edge && !d_flux_off)
      return fail(ctx, TVD_ERR_INVALID_ARG, "mixed edges need flux record offsets");
    if (d_flux == d_u_in || d_flux == d_u_out)
      return fail(ctx, TVD_ERR_ALIAS, "the flux records overlap a state buffer");
  }
  if (flags == TVD_KERNEL_PLAIN) {
    if (d_nbr) return fail(ctx, TVD_ERR_UNSUPPORTED, "the plain kernel takes ghosted input only");
    if (batch->dtype != TVD_F64 || batch->d_edge || batch->edge != 8)
      return fail(ctx, TVD_ERR_UNSUPPORTED, "the plain kernel needs TVD_F64 and uniform edge 8");
  }
  if (flags == TVD_KERNEL_PERSISTENT && batch->dtype != TVD_F32)
    return fail(ctx, TVD_ERR_UNSUPPORTED, "the persistent kernel needs TVD_F32");
  if (batch->dtype == TVD_F64 && (batch->d_edge || batch->edge != 8))
    return fail(ctx, TVD_ERR_UNSUPPORTED,
                "FP64 batches take uniform edge 8 (edge 16 exceeds the 160 KB LDS)");
  if (d_u_in == d_u_out) return fail(ctx, TVD_ERR_ALIAS, "d_u_in == d_u_out");
  if (!batch->d_in_off && !batch->d_out_off && !batch->d_edge) {
    const size_t es = elem_size(batch->dtype);
    const size_t m = d_nbr ? batch->edge : batch->edge + 6, n = batch->edge;
    const char* a = (const char*)d_u_in;
    const char* b = (const char*)d_u_out;
    const size_t la = (size_t)n_sources * 5 * m * m * m * es;
    const size_t lb = (size_t)batch->n_blocks * 5 * n * n * n * es;
    if (a < b + lb && b < a + la) return fail(ctx, TVD_ERR_ALIAS, "input and output overlap");
  }
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, TVD_ERR_HIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const bool fuse = d_smax || d_sums;
  const bool persistent = flags == TVD_KERNEL_PERSISTENT ||
                          (batch->d_edge && flags == TVD_KERNEL_AUTO);
  if (d_flux && d_nbr && persistent)
    return fail(ctx, TVD_ERR_UNSUPPORTED,
                "the gathering flux-recording advance runs the batched kernel (uniform edge)");
  if ((fuse || persistent) && (st = need_workspace(ctx, batch->n_blocks))) return st;
  tvd::KParams kp = make_params(ctx, batch, d_u_in, d_u_out, gamma, p_floor);
  hipError_t e;
  // partials start at zero: a block the kernel does not advance (a missing
  // neighbour) then adds nothing, whatever an earlier call left there
  if (d_smax) e = tvd::launch_zero_f64(kp.ws_smax, batch->n_blocks, s);
  else e = hipSuccess;
  if (e == hipSuccess && d_sums) e = tvd::launch_zero_f64(kp.ws_sums, 10 * (int64_t)batch->n_blocks, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "partials reset launch");
  kp.nbr = d_nbr;
  kp.nsrc = n_sources;
  kp.diag = (d_smax ? tvd::kDiagSpeed : 0) | (d_sums ? tvd::kDiagSums : 0);
  kp.flux = d_flux;
  kp.flux_off = d_flux_off;
  kp.flux_w = flux_w;
  kp.flux_acc = flux_acc;
  const bool gather = d_nbr != nullptr;
  // the flux-recording advance has one variant per (type, edge): the default
  auto variant = [&](int edge) {
    return d_flux ? default_variant(batch->dtype, edge) : chosen_variant(ctx, batch->dtype, edge);
  };
  if (flags == TVD_KERNEL_PLAIN) {
    e = tvd::launch_plain_f64(sweep_order, kp, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "plain kernel launch");
  } else if (persistent) {
    tvd::FusedPlan pl;
    pl.list = ctx->plan_list;
    pl.count = ctx->plan_small;
    pl.next = reinterpret_cast<unsigned*>(ctx->plan_small + 2);
    // one workgroup per CU (the LDS of one edge-16 block fills a CU), never
    // more than there are blocks
    const int wg = batch->n_blocks < ctx->cus ? batch->n_blocks : ctx->cus;
    e = tvd::launch_fused(batch->dtype, sweep_order, gather, kp, pl, wg, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "persistent kernel launch");
  } else if (batch->d_edge) {
    // one launch per edge; a workgroup whose block has the other edge exits
    for (int edge : {16, 8}) {
      e = tvd::launch_batched(batch->dtype, sweep_order, variant(edge), gather, kp, s);
      if (e != hipSuccess) return hip_fail(ctx, e, "batched kernel launch");
    }
  } else {
    e = tvd::launch_batched(batch->dtype, sweep_order, variant(batch->edge), gather, kp, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "batched kernel launch");
  }
  if (d_smax) {
    e = tvd::launch_finalize_max(kp.ws_smax, batch->n_blocks, d_smax, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "finalize launch");
  }
  if (d_sums) {
    e = tvd::launch_finalize_sums(kp.ws_sums, batch->n_blocks, d_sums, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "finalize launch");
  }
  return TVD_OK;
}

}  // namespace

namespace {

// Shared body of tvd_patch_advance_stream (partials in the context's
// workspace) and tvd_patch_advance_stream_noalloc (partials in the static
// scratch array): ws_smax [cap] and ws_sums [10 * cap] hold the per-tile
// partials of the fused signal speed and sums.
// Flux records of the streamed advance (tvd_patch_advance_stream_flux).
struct StreamFlux {
  int32_t n_sources;
  void* flux;
  const int64_t* flux_off;
  double w;
  bool acc;
};

int stream_impl(tvd_ctx* ctx, const tvd_batch* batch, const int32_t* d_nbr,
                const tvd_chains* chains, const void* d_u_in, void* d_u_out, int32_t sweep_order,
                double gamma, double p_floor, int32_t flags, double* d_smax, double* d_sums,
                void* stream, double* ws_smax, double* ws_sums, int64_t cap,
                const char* cap_hint, const StreamFlux* fx = nullptr) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, batch, true);
  if (st) return st;
  if ((st = check_gamma(ctx, gamma, p_floor))) return st;
  if (sweep_order != TVD_XYZ && sweep_order != TVD_ZYX)
    return fail(ctx, TVD_ERR_INVALID_ARG, "sweep_order %d", sweep_order);
  if (flags != TVD_KERNEL_AUTO && flags != TVD_STREAM_WHOLE_B && flags != TVD_STREAM_HALF_B)
    return fail(ctx, TVD_ERR_INVALID_ARG,
                "flags %d (TVD_KERNEL_AUTO, TVD_STREAM_WHOLE_B or TVD_STREAM_HALF_B)", flags);
  if (batch->d_edge || (batch->edge != 16 && batch->edge != 32))
    return fail(ctx, TVD_ERR_UNSUPPORTED, "the streamed advance takes a uniform edge 16 or 32");
  if (!chains) return fail(ctx, TVD_ERR_INVALID_ARG, "chains is NULL");
  if (chains->n_chains < 0 || chains->n_members < 0 || chains->n_members > batch->n_blocks)
    return fail(ctx, TVD_ERR_INVALID_ARG, "%d chains of %d members for %d blocks",
                chains->n_chains, chains->n_members, batch->n_blocks);
  if (batch->n_blocks == 0 || chains->n_chains == 0) return TVD_OK;
  if (!chains->d_start || !chains->d_blocks || !d_nbr)
    return fail(ctx, TVD_ERR_INVALID_ARG, "NULL chain table or neighbour table");
  if (!d_u_in || !d_u_out) return fail(ctx, TVD_ERR_INVALID_ARG, "state pointer is NULL");
  if (d_u_in == d_u_out) return fail(ctx, TVD_ERR_ALIAS, "d_u_in == d_u_out");
  if ((reinterpret_cast<uintptr_t>(d_u_in) | reinterpret_cast<uintptr_t>(d_u_out)) & 15)
    return fail(ctx, TVD_ERR_INVALID_ARG, "the state pointers must be 16-byte aligned");
  const int quads = batch->edge == 32 ? 4 : 1;
  if (!batch->d_in_off && !batch->d_out_off) {
    const size_t n = batch->edge;
    const size_t blk = 5 * n * n * n * elem_size(batch->dtype);
    const size_t len_out = (size_t)batch->n_blocks * blk;
    const size_t len_in = (size_t)(fx ? fx->n_sources : batch->n_blocks) * blk;
    const char* a = (const char*)d_u_in;
    const char* b = (const char*)d_u_out;
    if (a < b + len_out && b < a + len_in)
      return fail(ctx, TVD_ERR_ALIAS, "input and output overlap");
    if (fx && !fx->flux_off) {
      const size_t len_f = (size_t)batch->n_blocks * tvd::flux_record_size(batch->edge) *
                           elem_size(batch->dtype);
      const char* f = (const char*)fx->flux;
      if ((f < a + len_in && a < f + len_f) || (f < b + len_out && b < f + len_f))
        return fail(ctx, TVD_ERR_ALIAS, "the flux records overlap a state");
    }
  }
  // one diagnostics record per (chain, tile) item
  const int64_t parts = (int64_t)chains->n_chains * quads;
  if ((d_smax || d_sums) && parts > 0x7fffffff)
    return fail(ctx, TVD_ERR_INVALID_ARG, "too many blocks for the fused diagnostics");
  if ((d_smax || d_sums) && parts > cap)
    return fail(ctx, TVD_ERR_STATE, "the fused diagnostics need %lld partials and %s holds %lld",
                (long long)parts, cap_hint, (long long)cap);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, TVD_ERR_HIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t s = (hipStream_t)stream;
  tvd::KParams kp = make_params(ctx, batch, d_u_in, d_u_out, gamma, p_floor);
  kp.nbr = d_nbr;
  kp.diag = (d_smax ? tvd::kDiagSpeed : 0) | (d_sums ? tvd::kDiagSums : 0);
  kp.ws_smax = ws_smax;
  kp.ws_sums = ws_sums;
  if (fx) {
    kp.nsrc = fx->n_sources;
    kp.flux = fx->flux;
    kp.flux_off = fx->flux_off;
    kp.flux_w = fx->w;
    kp.flux_acc = fx->acc ? 1 : 0;
  }
  tvd::StreamParams sp;
  sp.start = chains->d_start;
  sp.blocks = chains->d_blocks;
  sp.n_chains = chains->n_chains;
  sp.n_members = chains->n_members;
  sp.quads = quads;
  hipError_t e = hipSuccess;
  // every (chain, tile) workgroup writes its record, zeros for a chain that
  // is refused, so no reset is needed; blocks no chain covers add nothing
  // second sweep in half pencils: FP32 by default, FP64 only when asked
  // (its half-pencil kernels spill registers to scratch memory)
  const bool splitb = flags == TVD_STREAM_HALF_B || (flags == TVD_KERNEL_AUTO && batch->dtype == TVD_F32);
  if (fx)
    e = tvd::launch_stream_flux_f32(sweep_order, fx->acc, kp, sp, s);
  else
    e = batch->dtype == TVD_F32
            ? tvd::launch_stream_f32(sweep_order, batch->edge, splitb, kp, sp, s)
            : tvd::launch_stream_f64(sweep_order, batch->edge, splitb, kp, sp, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "streamed kernel launch");
  if (d_smax) {
    e = tvd::launch_finalize_max(ws_smax, (int)parts, d_smax, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "finalize launch");
  }
  if (d_sums) {
    e = tvd::launch_finalize_sums(ws_sums, (int)parts, d_sums, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "finalize launch");
  }
  return TVD_OK;
}

}  // namespace

extern "C" {

int tvd_patch_advance(tvd_ctx* ctx, const tvd_batch* batch, const void* d_u_in, void* d_u_out,
                      int32_t sweep_order, double gamma, double p_floor, int32_t flags,
                      double* d_smax, double* d_sums, void* stream) {
  return advance_impl(ctx, batch, d_u_in, d_u_out, sweep_order, gamma, p_floor, flags, d_smax,
                      d_sums, stream, nullptr);
}

int tvd_patch_advance_gather(tvd_ctx* ctx, const tvd_batch* batch, const int32_t* d_nbr,
                             const void* d_u_in, void* d_u_out, int32_t sweep_order,
                             double gamma, double p_floor, int32_t flags, double* d_smax,
                             double* d_sums, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  if (!d_nbr) return fail(ctx, TVD_ERR_INVALID_ARG, "d_nbr is NULL");
  return advance_impl(ctx, batch, d_u_in, d_u_out, sweep_order, gamma, p_floor, flags, d_smax,
                      d_sums, stream, d_nbr);
}

int tvd_patch_advance_stream(tvd_ctx* ctx, const tvd_batch* batch, const int32_t* d_nbr,
                             const tvd_chains* chains, const void* d_u_in, void* d_u_out,
                             int32_t sweep_order, double gamma, double p_floor, int32_t flags,
                             double* d_smax, double* d_sums, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  return stream_impl(ctx, batch, d_nbr, chains, d_u_in, d_u_out, sweep_order, gamma, p_floor,
                     flags, d_smax, d_sums, stream, ctx->ws_smax, ctx->ws_sums, ctx->ws_blocks,
                     "the workspace (tvd_reserve)");
}

int tvd_patch_advance_stream_noalloc(tvd_ctx* ctx, const tvd_batch* batch, const int32_t* d_nbr,
                                     const tvd_chains* chains, const void* d_u_in,
                                     void* d_u_out, int32_t sweep_order, double gamma,
                                     double p_floor, int32_t flags, double* d_smax,
                                     double* d_sums, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  if (!ctx->scratch)
    return fail(ctx, TVD_ERR_STATE, "the scratch array of device %d was not resolved",
                ctx->device);
  return stream_impl(ctx, batch, d_nbr, chains, d_u_in, d_u_out, sweep_order, gamma, p_floor,
                     flags, d_smax, d_sums, stream, ctx->scratch,
                     ctx->scratch + kScratchParts, kScratchParts, "the static scratch array");
}

int tvd_patch_advance_stream_flux(tvd_ctx* ctx, const tvd_batch* batch, const int32_t* d_nbr,
                                  int32_t n_sources, const tvd_chains* chains,
                                  const void* d_u_in, void* d_u_out, void* d_flux,
                                  const int64_t* d_flux_off, double flux_weight,
                                  int32_t accumulate, int32_t sweep_order, double gamma,
                                  double p_floor, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, batch, true);
  if (st) return st;
  if (batch->dtype != TVD_F32 || batch->d_edge || batch->edge != 16 || batch->d_in_off ||
      batch->d_out_off)
    return fail(ctx, TVD_ERR_UNSUPPORTED,
                "flux records of the streamed advance: FP32, dense blocks of edge 16");
  if (n_sources < batch->n_blocks)
    return fail(ctx, TVD_ERR_INVALID_ARG, "n_sources %d < n_blocks %d", n_sources,
                batch->n_blocks);
  if (!d_flux) return fail(ctx, TVD_ERR_INVALID_ARG, "d_flux is NULL");
  if (accumulate != 0 && accumulate != 1)
    return fail(ctx, TVD_ERR_INVALID_ARG, "accumulate %d (0 or 1)", accumulate);
  if (!(flux_weight > -1e300 && flux_weight < 1e300))
    return fail(ctx, TVD_ERR_INVALID_ARG, "flux_weight %g is not finite", flux_weight);
  const StreamFlux fx{n_sources, d_flux, d_flux_off, flux_weight, accumulate != 0};
  return stream_impl(ctx, batch, d_nbr, chains, d_u_in, d_u_out, sweep_order, gamma, p_floor,
                     TVD_KERNEL_AUTO, nullptr, nullptr, stream, ctx->ws_smax, ctx->ws_sums,
                     ctx->ws_blocks, "the workspace (tvd_reserve)", &fx);
}

int tvd_pipeline_stage_bytes(int32_t dtype, int32_t edge, const tvd_host_pipeline* pipe,
                             int64_t* h_stage_bytes, int64_t* d_stage_bytes) {
  if (!pipe || (dtype != TVD_F32 && dtype != TVD_F64) || (edge != 8 && edge != 16))
    return TVD_ERR_INVALID_ARG;
  if (pipe->n_streams < 1 || pipe->n_streams > 16 || pipe->groups_per_stream < 1 ||
      (int64_t)pipe->n_streams * pipe->groups_per_stream > (1 << 20))
    return TVD_ERR_INVALID_ARG;
  const int64_t es = dtype == TVD_F32 ? 4 : 8;
  const int64_t g = 5 * (int64_t)(edge + 6) * (edge + 6) * (edge + 6) * es;
  const int64_t i = 5 * (int64_t)edge * edge * edge * es;
  const int64_t per_launch = (int64_t)pipe->n_streams * pipe->groups_per_stream;
  if (h_stage_bytes) *h_stage_bytes = 2 * per_launch * (g + i);
  if (d_stage_bytes) *d_stage_bytes = per_launch * (g + i);
  return TVD_OK;
}

int tvd_patch_advance_host(tvd_ctx* ctx, const tvd_batch* batch, const int32_t* h_nbr,
                           const void* h_u_in, void* h_u_out, const tvd_host_pipeline* pipe,
                           int32_t sweep_order, double gamma, double p_floor, double* times) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, batch);
  if (st) return st;
  if ((st = check_gamma(ctx, gamma, p_floor))) return st;
  if (sweep_order != TVD_XYZ && sweep_order != TVD_ZYX)
    return fail(ctx, TVD_ERR_INVALID_ARG, "sweep_order %d", sweep_order);
  if (batch->d_edge || batch->d_in_off || batch->d_out_off || batch->d_dt || batch->d_dh)
    return fail(ctx, TVD_ERR_UNSUPPORTED,
                "the host-resident advance takes a dense batch of uniform edge with scalar dt "
                "and dh (no device arrays)");
  if (batch->dtype == TVD_F64 && batch->edge != 8)
    return fail(ctx, TVD_ERR_UNSUPPORTED, "FP64 blocks of edge %d (the batched kernel holds "
                "FP64 blocks of edge 8)", batch->edge);
  if (!pipe) return fail(ctx, TVD_ERR_INVALID_ARG, "pipe is NULL");
  int64_t hb = 0, db = 0;
  if (tvd_pipeline_stage_bytes(batch->dtype, batch->edge, pipe, &hb, &db) != TVD_OK)
    return fail(ctx, TVD_ERR_INVALID_ARG, "n_streams %d (1..16), groups_per_stream %d (>= 1)",
                pipe->n_streams, pipe->groups_per_stream);
  if (pipe->host_threads < 1 || pipe->host_threads > 256)
    return fail(ctx, TVD_ERR_INVALID_ARG, "host_threads %d (1..256)", pipe->host_threads);
  if (pipe->concurrent != 0 && pipe->concurrent != 1)
    return fail(ctx, TVD_ERR_INVALID_ARG, "concurrent %d is neither 0 nor 1", pipe->concurrent);
  if (batch->n_blocks == 0) {
    if (times)
      for (int k = 0; k < 7; ++k) times[k] = 0.0;
    return TVD_OK;
  }
  if (!h_nbr || !h_u_in || !h_u_out || !pipe->streams || !pipe->h_stage || !pipe->d_stage)
    return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  // host memory can be checked here, unlike the device arrays of a batch
  const int64_t nb = batch->n_blocks;
  for (int64_t k = 0; k < 27 * nb; ++k)
    if (h_nbr[k] < 0 || h_nbr[k] >= nb)
      return fail(ctx, TVD_ERR_INVALID_ARG, "h_nbr[%lld][%lld] = %d is not a block",
                  (long long)(k / 27), (long long)(k % 27), h_nbr[k]);
  const size_t len = (size_t)nb * 5 * batch->edge * batch->edge * batch->edge *
                     elem_size(batch->dtype);
  {
    const char* a = (const char*)h_u_in;
    const char* b = (const char*)h_u_out;
    if (a < b + len && b < a + len) return fail(ctx, TVD_ERR_ALIAS, "h_u_in and h_u_out overlap");
    const char* c = (const char*)pipe->h_stage;
    if ((c < a + len && a < c + hb) || (c < b + len && b < c + hb))
      return fail(ctx, TVD_ERR_ALIAS, "h_stage overlaps h_u_in or h_u_out");
  }
  if (ctx->capturing) return fail(ctx, TVD_ERR_STATE, "the host-resident advance cannot be captured");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, TVD_ERR_HIP, "hipSetDevice(%d) failed", ctx->device);
  for (int s = 0; s < pipe->n_streams; ++s)
    if (stream_capturing((hipStream_t)pipe->streams[s]))
      return fail(ctx, TVD_ERR_STATE, "stream %d is capturing", s);
  tvd::HostPipe hp;
  hp.dtype = batch->dtype;
  hp.edge = batch->edge;
  hp.order = sweep_order;
  hp.n_blocks = nb;
  hp.h_nbr = h_nbr;
  hp.h_in = h_u_in;
  hp.h_out = h_u_out;
  hp.ns = pipe->n_streams;
  hp.ng = pipe->groups_per_stream;
  hp.threads = pipe->host_threads;
  hp.concurrent = pipe->concurrent == 1;
  hp.h_stage = pipe->h_stage;
  hp.d_stage = pipe->d_stage;
  hp.streams = reinterpret_cast<const hipStream_t*>(pipe->streams);
  hp.variant = chosen_variant(ctx, batch->dtype, batch->edge);
  hp.kp = make_params(ctx, batch, nullptr, nullptr, gamma, p_floor);
  const hipError_t e = tvd::run_host_pipeline(hp, times);
  if (e != hipSuccess) return hip_fail(ctx, e, "host-resident pipeline");
  return TVD_OK;
}

int tvd_patch_advance_flux(tvd_ctx* ctx, const tvd_batch* batch, const void* d_u_in,
                           void* d_u_out, void* d_flux, const int64_t* d_flux_off,
                           double flux_weight, int32_t accumulate, int32_t sweep_order,
                           double gamma, double p_floor, int32_t flags, double* d_smax,
                           double* d_sums, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  if (!d_flux) return fail(ctx, TVD_ERR_INVALID_ARG, "d_flux is NULL");
  if (!(flux_weight == flux_weight) || flux_weight < -1e300 || flux_weight > 1e300)
    return fail(ctx, TVD_ERR_INVALID_ARG, "flux_weight %g", flux_weight);
  if (accumulate != 0 && accumulate != 1)
    return fail(ctx, TVD_ERR_INVALID_ARG, "accumulate %d is neither 0 nor 1", accumulate);
  return advance_impl(ctx, batch, d_u_in, d_u_out, sweep_order, gamma, p_floor, flags, d_smax,
                      d_sums, stream, nullptr, d_flux, d_flux_off, flux_weight, accumulate);
}

int tvd_patch_advance_flux_gather(tvd_ctx* ctx, const tvd_batch* batch, const int32_t* d_nbr,
                                  int32_t n_sources, const void* d_u_in, void* d_u_out,
                                  void* d_flux, const int64_t* d_flux_off, double flux_weight,
                                  int32_t accumulate, int32_t sweep_order, double gamma,
                                  double p_floor, int32_t flags, double* d_smax, double* d_sums,
                                  void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  if (!d_nbr) return fail(ctx, TVD_ERR_INVALID_ARG, "d_nbr is NULL");
  if (!d_flux) return fail(ctx, TVD_ERR_INVALID_ARG, "d_flux is NULL");
  if (n_sources < 0) return fail(ctx, TVD_ERR_INVALID_ARG, "n_sources %d < 0", n_sources);
  if (!(flux_weight == flux_weight) || flux_weight < -1e300 || flux_weight > 1e300)
    return fail(ctx, TVD_ERR_INVALID_ARG, "flux_weight %g", flux_weight);
  if (accumulate != 0 && accumulate != 1)
    return fail(ctx, TVD_ERR_INVALID_ARG, "accumulate %d is neither 0 nor 1", accumulate);
  if (flags == TVD_KERNEL_PLAIN || flags == TVD_KERNEL_PERSISTENT)
    return fail(ctx, TVD_ERR_UNSUPPORTED, "the gathering flux-recording advance is batched");
  return advance_impl(ctx, batch, d_u_in, d_u_out, sweep_order, gamma, p_floor, flags, d_smax,
                      d_sums, stream, d_nbr, d_flux, d_flux_off, flux_weight, accumulate,
                      n_sources);
}

int tvd_lerp(tvd_ctx* ctx, int32_t dtype, int64_t n, const void* d_a, const void* d_b,
             void* d_out, double w, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  if (dtype != TVD_F32 && dtype != TVD_F64) return fail(ctx, TVD_ERR_INVALID_ARG, "dtype %d", dtype);
  if (n < 0 || n > ((int64_t)1 << 38))
    return fail(ctx, TVD_ERR_INVALID_ARG, "n %lld outside [0, 2^38]", (long long)n);
  if (!(w == w) || w < -1e300 || w > 1e300) return fail(ctx, TVD_ERR_INVALID_ARG, "w %g", w);
  if (n == 0) return TVD_OK;
  if (!d_a || !d_b || !d_out) return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  DeviceGuard g(ctx->device);
  hipError_t e = tvd::launch_lerp(dtype == TVD_F32 ? 1 : 2, n, d_a, d_b, d_out, w,
                                  (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "lerp launch");
  return TVD_OK;
}

int tvd_restrict(tvd_ctx* ctx, const tvd_batch* coarse, void* d_coarse, const tvd_batch* fine,
                 const void* d_fine, const int32_t* d_rows, int32_t n_rows, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, coarse);
  if (st) return st;
  if ((st = check_batch(ctx, fine))) return st;
  if (coarse->dtype != fine->dtype)
    return fail(ctx, TVD_ERR_INVALID_ARG, "coarse and fine batches differ in dtype");
  if (n_rows < 0) return fail(ctx, TVD_ERR_INVALID_ARG, "n_rows %d", n_rows);
  if (n_rows == 0) return TVD_OK;
  if (!d_coarse || !d_fine || !d_rows) return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  DeviceGuard g(ctx->device);
  const tvd::KParams ck = make_params(ctx, coarse, nullptr, d_coarse, 1.0, 0.0);
  const tvd::KParams fk = make_params(ctx, fine, d_fine, nullptr, 1.0, 0.0);
  hipError_t e = tvd::launch_restrict(coarse->dtype, ck, fk, d_rows, n_rows, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "restriction launch");
  return TVD_OK;
}

int tvd_flux_correct(tvd_ctx* ctx, const tvd_batch* coarse, void* d_coarse,
                     const void* d_coarse_flux, const int64_t* d_coarse_flux_off,
                     const tvd_batch* fine, const void* d_fine_flux,
                     const int64_t* d_fine_flux_off, const int32_t* d_rows,
                     const int32_t pass_count[6], void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, coarse);
  if (st) return st;
  if ((st = check_batch(ctx, fine))) return st;
  if (coarse->dtype != fine->dtype)
    return fail(ctx, TVD_ERR_INVALID_ARG, "coarse and fine batches differ in dtype");
  if (!pass_count) return fail(ctx, TVD_ERR_INVALID_ARG, "pass_count is NULL");
  int64_t total = 0;
  for (int p = 0; p < 6; ++p) {
    if (pass_count[p] < 0) return fail(ctx, TVD_ERR_INVALID_ARG, "pass_count[%d] < 0", p);
    total += pass_count[p];
  }
  if (total > INT32_MAX) return fail(ctx, TVD_ERR_INVALID_ARG, "too many rows");
  if (total == 0) return TVD_OK;
  if (!d_coarse || !d_coarse_flux || !d_fine_flux || !d_rows)
    return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  if ((coarse->d_edge && !d_coarse_flux_off) || (fine->d_edge && !d_fine_flux_off))
    return fail(ctx, TVD_ERR_INVALID_ARG, "mixed edges need flux record offsets");
  if (d_coarse == d_coarse_flux || d_coarse == d_fine_flux)
    return fail(ctx, TVD_ERR_ALIAS, "the state overlaps a flux record buffer");
  DeviceGuard g(ctx->device);
  tvd::KParams ck = make_params(ctx, coarse, nullptr, d_coarse, 1.0, 0.0);
  ck.flux = const_cast<void*>(d_coarse_flux);
  ck.flux_off = d_coarse_flux_off;
  tvd::KParams fk = make_params(ctx, fine, nullptr, nullptr, 1.0, 0.0);
  fk.flux = const_cast<void*>(d_fine_flux);
  fk.flux_off = d_fine_flux_off;
  // one launch per pass, in the order x-, x+, y-, y+, z-, z+: a coarse cell
  // on several interfaces takes its corrections in that order
  int64_t first = 0;
  for (int p = 0; p < 6; ++p) {
    hipError_t e = tvd::launch_flux_correct(coarse->dtype, ck, fk, d_rows + 8 * first,
                                            pass_count[p], (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "flux correction launch");
    first += pass_count[p];
  }
  return TVD_OK;
}

int tvd_close_level(tvd_ctx* ctx, const tvd_batch* coarse, void* d_coarse,
                    const void* d_coarse_flux, const int64_t* d_coarse_flux_off,
                    const tvd_batch* fine, const void* d_fine, const void* d_fine_flux,
                    const int64_t* d_fine_flux_off, const int32_t* d_restrict_rows,
                    int32_t n_restrict, const int32_t* d_face_rows, int32_t n_face_rows,
                    const int32_t* d_face_start, int32_t n_face_groups, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, coarse);
  if (st) return st;
  if ((st = check_batch(ctx, fine))) return st;
  if (coarse->dtype != fine->dtype)
    return fail(ctx, TVD_ERR_INVALID_ARG, "coarse and fine batches differ in dtype");
  if (n_restrict < 0 || n_face_rows < 0 || n_face_groups < 0 ||
      (int64_t)n_restrict + n_face_groups > INT32_MAX)
    return fail(ctx, TVD_ERR_INVALID_ARG, "row counts");
  if (n_restrict + n_face_groups == 0) return TVD_OK;
  if (!d_coarse || (n_restrict && (!d_fine || !d_restrict_rows)) ||
      (n_face_groups && (!d_coarse_flux || !d_fine_flux || !d_face_rows || !d_face_start)))
    return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  if ((coarse->d_edge && !d_coarse_flux_off) || (fine->d_edge && !d_fine_flux_off))
    return fail(ctx, TVD_ERR_INVALID_ARG, "mixed edges need flux record offsets");
  if (d_coarse == d_coarse_flux || d_coarse == d_fine_flux)
    return fail(ctx, TVD_ERR_ALIAS, "the state overlaps a flux record buffer");
  DeviceGuard g(ctx->device);
  tvd::KParams ck = make_params(ctx, coarse, nullptr, d_coarse, 1.0, 0.0);
  ck.flux = const_cast<void*>(d_coarse_flux);
  ck.flux_off = d_coarse_flux_off;
  tvd::KParams fk = make_params(ctx, fine, d_fine, nullptr, 1.0, 0.0);
  fk.flux = const_cast<void*>(d_fine_flux);
  fk.flux_off = d_fine_flux_off;
  hipError_t e = tvd::launch_close_level(coarse->dtype, ck, fk, d_restrict_rows, n_restrict,
                                         d_face_rows, n_face_rows, d_face_start, n_face_groups,
                                         (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "closing launch");
  return TVD_OK;
}

int tvd_gravity(tvd_ctx* ctx, const tvd_batch* batch, void* d_u, const void* d_phi,
                void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, batch);
  if (st) return st;
  if (batch->d_edge) return fail(ctx, TVD_ERR_UNSUPPORTED, "the gravity operator takes a uniform edge");
  if (batch->n_blocks == 0) return TVD_OK;
  if ((int64_t)batch->n_blocks * batch->edge * batch->edge * batch->edge > ((int64_t)1 << 38))
    return fail(ctx, TVD_ERR_INVALID_ARG, "more than 2^38 cells in one call");
  if (!d_u || !d_phi) return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  if (d_u == d_phi) return fail(ctx, TVD_ERR_ALIAS, "state and potential are one buffer");
  DeviceGuard g(ctx->device);
  const tvd::KParams kp = make_params(ctx, batch, nullptr, d_u, 1.0, 0.0);
  hipError_t e = tvd::launch_gravity(batch->dtype == TVD_F32 ? 1 : 2, kp, d_phi, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "gravity launch");
  return TVD_OK;
}

int tvd_poisson_sor(tvd_ctx* ctx, int32_t dtype, int32_t n_groups, const void* d_phi_in,
                    const void* d_rho, void* d_phi_out, double G, double dh, const double* d_dh,
                    double omega, int32_t min_iter, int32_t max_iter, double tol,
                    int32_t* d_iters, double* d_resid, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  if (dtype != TVD_F32 && dtype != TVD_F64) return fail(ctx, TVD_ERR_INVALID_ARG, "dtype %d", dtype);
  if (n_groups < 0) return fail(ctx, TVD_ERR_INVALID_ARG, "n_groups %d", n_groups);
  if (!(G == G) || G < -1e300 || G > 1e300) return fail(ctx, TVD_ERR_INVALID_ARG, "G %g", G);
  if (!d_dh && !(dh > 0.0 && dh < 1e300)) return fail(ctx, TVD_ERR_INVALID_ARG, "dh %g", dh);
  if (omega == 0.0) omega = 2.0 / (1.0 + sin(3.141592653589793 / 17.0));
  if (!(omega > 0.0 && omega < 2.0)) return fail(ctx, TVD_ERR_INVALID_ARG, "omega %g", omega);
  if (max_iter < 1 || max_iter > 1000000 || min_iter < 0 || min_iter > max_iter)
    return fail(ctx, TVD_ERR_INVALID_ARG, "iteration limits %d..%d", min_iter, max_iter);
  if (tol == 0.0) tol = 16.0 * (dtype == TVD_F32 ? 5.9604644775390625e-08 : 1.1102230246251565e-16);
  if (!(tol > 0.0 && tol < 1.0)) return fail(ctx, TVD_ERR_INVALID_ARG, "tol %g", tol);
  if (n_groups == 0) return TVD_OK;
  if (!d_phi_in || !d_rho || !d_phi_out) return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  const size_t es = elem_size(dtype);
  const char* a = (const char*)d_phi_in;
  const char* b = (const char*)d_phi_out;
  const size_t la = (size_t)n_groups * 18 * 18 * 18 * es, lb = (size_t)n_groups * 4096 * es;
  if (a < b + lb && b < a + la) return fail(ctx, TVD_ERR_ALIAS, "phi_in and phi_out overlap");
  DeviceGuard g(ctx->device);
  hipError_t e = tvd::launch_sor(dtype == TVD_F32 ? 1 : 2, n_groups, d_phi_in, d_rho, d_phi_out,
                                 d_dh, dh, G, omega, tol, min_iter, max_iter, d_iters, d_resid,
                                 (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "SOR launch");
  return TVD_OK;
}

int tvd_autotune(tvd_ctx* ctx, const tvd_batch* batch, const int32_t* d_nbr, const void* d_u_in,
                 void* d_u_out, double gamma, double p_floor, int32_t reps,
                 int32_t* chosen_index, float* best_ms) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, batch);
  if (st) return st;
  if ((st = check_gamma(ctx, gamma, p_floor))) return st;
  if (batch->d_edge) return fail(ctx, TVD_ERR_UNSUPPORTED, "tune one edge at a time");
  if (batch->n_blocks == 0 || !d_u_in || !d_u_out || d_u_in == d_u_out)
    return fail(ctx, TVD_ERR_INVALID_ARG, "autotune needs a non-empty batch and two buffers");
  if (reps < 1 || reps > 1000) return fail(ctx, TVD_ERR_INVALID_ARG, "reps %d", reps);
  const int dt = batch->dtype == TVD_F32 ? 1 : 2;
  DeviceGuard g(ctx->device);
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamCreate");
  hipEvent_t a = nullptr, b = nullptr;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  tvd::KParams kp = make_params(ctx, batch, d_u_in, d_u_out, gamma, p_floor);
  kp.nbr = d_nbr;
  int best = -1;
  float best_t = 0.f;
  st = TVD_OK;
  for (int i = 0; i < tvd::variant_count() && st == TVD_OK; ++i) {
    const tvd::Variant v = tvd::variant_at(i);
    if (v.edge != batch->edge || !tvd::variant_supported(dt, v)) continue;
    // one untimed pair, then `reps` timed pairs (xyz + zyx)
    for (int o = 0; o < 2; ++o) e = tvd::launch_batched(dt, o, v, d_nbr != nullptr, kp, s);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r)
      for (int o = 0; o < 2 && e == hipSuccess; ++o)
        e = tvd::launch_batched(dt, o, v, d_nbr != nullptr, kp, s);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e != hipSuccess) {
      st = hip_fail(ctx, e, "autotune launch");
      break;
    }
    ms /= (float)reps;
    if (best < 0 || ms < best_t) {
      best = i;
      best_t = ms;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamDestroy(s);
  if (st != TVD_OK) return st;
  if (best < 0) return fail(ctx, TVD_ERR_UNSUPPORTED, "no variant serves this batch");
  ctx->tuned[dt == 1 ? 0 : 1][batch->edge == 16 ? 1 : 0] = best;
  if (chosen_index) *chosen_index = best;
  if (best_ms) *best_ms = best_t;
  return TVD_OK;
}

int tvd_graph_begin(tvd_ctx* ctx, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  if (!stream) return fail(ctx, TVD_ERR_INVALID_ARG, "capture needs a non-default stream");
  hipStream_t s = (hipStream_t)stream;
  if (stream_capturing(s)) return fail(ctx, TVD_ERR_STATE, "stream is already capturing");
  DeviceGuard g(ctx->device);
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamBeginCapture");
  ctx->capturing = true;
  return TVD_OK;
}

int tvd_graph_end(tvd_ctx* ctx, void* stream, tvd_graph** out) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  if (!stream || !out) return fail(ctx, TVD_ERR_INVALID_ARG, "NULL stream or output");
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard g(ctx->device);
  hipGraph_t graph = nullptr;
  ctx->capturing = false;
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(ctx, e, "hipGraphInstantiate");
  }
  tvd_graph* gr = new tvd_graph();
  gr->device = ctx->device;
  gr->graph = graph;
  gr->exec = exec;
  gr->ws_gen = ctx->ws_gen;
  gr->gen = *ctx->ws_gen;
  *out = gr;
  return TVD_OK;
}

int tvd_graph_launch(tvd_graph* graph, void* stream) {
  if (!graph) return TVD_ERR_INVALID_ARG;
  // captured before tvd_reserve replaced the workspace, or its context is gone
  if (*graph->ws_gen != graph->gen) return TVD_ERR_STATE;
  DeviceGuard g(graph->device);
  return hipGraphLaunch(graph->exec, (hipStream_t)stream) == hipSuccess ? TVD_OK : TVD_ERR_HIP;
}

int tvd_graph_destroy(tvd_graph* graph) {
  if (!graph) return TVD_ERR_INVALID_ARG;
  {
    DeviceGuard g(graph->device);
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
  }
  delete graph;
  return TVD_OK;
}

int tvd_max_signal_speed(tvd_ctx* ctx, const tvd_batch* batch, const void* d_u, int32_t layout,
                         double gamma, double p_floor, double* d_smax, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, batch, true);
  if (st) return st;
  if ((st = check_gamma(ctx, gamma, p_floor))) return st;
  if (layout != TVD_LAYOUT_GHOSTED && layout != TVD_LAYOUT_INTERIOR)
    return fail(ctx, TVD_ERR_INVALID_ARG, "layout %d", layout);
  if (!d_u || !d_smax) return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  if ((st = need_workspace(ctx, batch->n_blocks))) return st;
  const tvd::KParams kp = make_params(ctx, batch, d_u, nullptr, gamma, p_floor);
  hipError_t e = hipSuccess;
  if (batch->n_blocks > 0) e = tvd::launch_signal_speed(batch->dtype, layout, kp, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "signal speed launch");
  e = tvd::launch_finalize_max(ctx->ws_smax, batch->n_blocks, d_smax, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "finalize launch");
  return TVD_OK;
}

int tvd_dt_from_speed(tvd_ctx* ctx, const tvd_batch* batch, const double* d_smax, double cfl,
                      double* d_dt_out, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, batch, true);
  if (st) return st;
  if (!(cfl > 0.0) || !(cfl <= 1.0))
    return fail(ctx, TVD_ERR_INVALID_ARG, "cfl %g must lie in (0, 1]", cfl);
  if (!d_smax || !d_dt_out) return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  if (batch->n_blocks == 0) return TVD_OK;
  DeviceGuard g(ctx->device);
  const tvd::KParams kp = make_params(ctx, batch, nullptr, nullptr, 1.0, 0.0);
  hipError_t e = tvd::launch_dt_from_speed(kp, d_smax, cfl, d_dt_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "dt launch");
  return TVD_OK;
}

int tvd_conservation_sums(tvd_ctx* ctx, const tvd_batch* batch, const void* d_u, int32_t layout,
                          double* d_sums, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, batch, true);
  if (st) return st;
  if (layout != TVD_LAYOUT_GHOSTED && layout != TVD_LAYOUT_INTERIOR)
    return fail(ctx, TVD_ERR_INVALID_ARG, "layout %d", layout);
  if (!d_u || !d_sums) return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  if ((st = need_workspace(ctx, batch->n_blocks))) return st;
  const tvd::KParams kp = make_params(ctx, batch, d_u, nullptr, 1.0, 0.0);
  hipError_t e = hipSuccess;
  if (batch->n_blocks > 0) e = tvd::launch_cons_sums(batch->dtype, layout, kp, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "sums launch");
  e = tvd::launch_finalize_sums(ctx->ws_sums, batch->n_blocks, d_sums, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "finalize launch");
  return TVD_OK;
}

int tvd_read_flags(tvd_ctx* ctx, int64_t* n_floored, int64_t* n_nonphysical, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (stream_capturing(s)) return fail(ctx, TVD_ERR_STATE, "tvd_read_flags cannot be captured");
  DeviceGuard g(ctx->device);
  unsigned long long h[2] = {0, 0};
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  e = hipMemcpy(h, ctx->counters, sizeof(h), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(counters)");
  e = tvd::launch_zero_u64(ctx->counters, 2, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "counter reset launch");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  if (n_floored) *n_floored = (int64_t)h[0];
  if (n_nonphysical) *n_nonphysical = (int64_t)h[1];
  if (h[1]) return TVD_ERR_NONPHYSICAL;
  if (h[0]) return TVD_WARN_FLOORED;
  return TVD_OK;
}

int tvd_fill_ghosts(tvd_ctx* ctx, const tvd_batch* batch, const int32_t* d_nbr,
                    const void* d_interior, void* d_ghosted, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, batch, true);
  if (st) return st;
  if (batch->n_blocks == 0) return TVD_OK;
  if (!d_nbr || !d_interior || !d_ghosted)
    return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  if (d_interior == d_ghosted) return fail(ctx, TVD_ERR_ALIAS, "interior == ghosted");
  DeviceGuard g(ctx->device);
  const tvd::KParams kp = make_params(ctx, batch, d_ghosted, const_cast<void*>(d_interior), 1.0,
                                      0.0);
  const int max_edge = batch->d_edge ? 16 : batch->edge;
  hipError_t e = tvd::launch_fill_ghosts(batch->dtype, kp, d_nbr, max_edge, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "ghost fill launch");
  return TVD_OK;
}

int tvd_fill_ghosts_amr(tvd_ctx* ctx, const tvd_batch* fine, const int32_t* d_nbr,
                        const void* d_fine_interior, void* d_fine_ghosted,
                        const tvd_batch* coarse, const void* d_coarse_interior,
                        const int32_t* d_cnbr, const int32_t* d_corigin, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, fine);
  if (st) return st;
  if ((st = check_batch(ctx, coarse))) return st;
  if (coarse->dtype != fine->dtype)
    return fail(ctx, TVD_ERR_INVALID_ARG, "coarse and fine batches differ in dtype");
  if (coarse->d_edge || (coarse->edge != 8 && coarse->edge != 16))
    return fail(ctx, TVD_ERR_UNSUPPORTED,
                "coarse blocks must have a uniform edge of 8 (patches) or 16 (patch groups)");
  if (fine->n_blocks == 0) return TVD_OK;
  if (!d_nbr || !d_fine_interior || !d_fine_ghosted || !d_coarse_interior || !d_cnbr ||
      !d_corigin)
    return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  if (d_fine_interior == d_fine_ghosted || d_coarse_interior == d_fine_ghosted)
    return fail(ctx, TVD_ERR_ALIAS, "an input is the ghosted output");
  DeviceGuard g(ctx->device);
  const tvd::KParams kp = make_params(ctx, fine, d_fine_ghosted,
                                      const_cast<void*>(d_fine_interior), 1.0, 0.0);
  const int max_edge = fine->d_edge ? 16 : fine->edge;
  hipError_t e = tvd::launch_fill_ghosts_amr(fine->dtype, kp, d_nbr, max_edge, d_coarse_interior,
                                             coarse->d_out_off, coarse->n_blocks, coarse->edge,
                                             d_cnbr, d_corigin, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "coarse-fine ghost fill launch");
  return TVD_OK;
}

int tvd_fill_coarse_fine(tvd_ctx* ctx, const tvd_batch* fine, const int32_t* d_nbr,
                         int32_t n_sources, void* d_fine_interior, const tvd_batch* coarse,
                         const void* d_coarse_old, const void* d_coarse_new, double w,
                         const int32_t* d_cnbr, const int32_t* d_corigin, void* stream) {
  if (!ctx) return TVD_ERR_INVALID_ARG;
  int st = check_batch(ctx, fine);
  if (st) return st;
  if ((st = check_batch(ctx, coarse))) return st;
  if (coarse->dtype != fine->dtype)
    return fail(ctx, TVD_ERR_INVALID_ARG, "coarse and fine batches differ in dtype");
  if (fine->d_edge || fine->d_in_off || fine->d_out_off)
    return fail(ctx, TVD_ERR_UNSUPPORTED, "the fine batch must be dense with a uniform edge");
  if (coarse->d_edge || (coarse->edge != 8 && coarse->edge != 16))
    return fail(ctx, TVD_ERR_UNSUPPORTED,
                "coarse blocks must have a uniform edge of 8 (patches) or 16 (patch groups)");
  if (n_sources < fine->n_blocks)
    return fail(ctx, TVD_ERR_INVALID_ARG, "n_sources %d < n_blocks %d", n_sources,
                fine->n_blocks);
  if (!(w >= 0.0 && w <= 1.0)) return fail(ctx, TVD_ERR_INVALID_ARG, "w %g outside [0, 1]", w);
  if ((int64_t)fine->n_blocks * 26 * 128 >= (int64_t)1 << 32)
    return fail(ctx, TVD_ERR_UNSUPPORTED, "n_blocks %d > 1290555 (launch size)", fine->n_blocks);
  if (fine->n_blocks == 0 || n_sources == fine->n_blocks) return TVD_OK;
  if (!d_nbr || !d_fine_interior || !d_coarse_old || !d_cnbr || !d_corigin ||
      (w != 0.0 && !d_coarse_new))
    return fail(ctx, TVD_ERR_INVALID_ARG, "NULL pointer");
  if (d_fine_interior == d_coarse_old || d_fine_interior == d_coarse_new)
    return fail(ctx, TVD_ERR_ALIAS, "the fine interiors are a coarse state");
  DeviceGuard g(ctx->device);
  tvd::KParams kp = make_params(ctx, fine, nullptr, d_fine_interior, 1.0, 0.0);
  kp.nsrc = n_sources;
  hipError_t e = tvd::launch_fill_coarse_fine(
      fine->dtype, kp, d_nbr, d_coarse_old, w != 0.0 ? d_coarse_new : d_coarse_old, w,
      coarse->d_out_off, coarse->n_blocks, coarse->edge, d_cnbr, d_corigin, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "coarse-fine fill launch");
  return TVD_OK;
}

}  // extern "C"
