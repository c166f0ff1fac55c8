// Host-resident advance: the blocks of a level live in host memory and pass
// through the GPU in launches of N_s x N_g blocks, each of the N_s streams
// carrying one copy downstream, one advance and one copy upstream of its N_g
// blocks (Sec. 3.1, the stream objects and their N_s + 2 stages), while the
// host threads prepare the next launch's ghosted blocks and copy the
// previous launch's results back (Sec. 3.5, concurrent CPU and GPU work).
//
// The host's share is data movement only: the preparation step gathers each
// ghosted block from the interiors of the block and its 26 neighbours
// (sibling copies, Sec. 2.2 ghost zones), the closing step copies each
// advanced interior back to its block.  Every arithmetic operation of the
// scheme runs in the batched HIP kernel.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <thread>
#include <vector>

#include "tvd_internal.hpp"

namespace tvd {

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// f(i) for i in [0, n) on `threads` host threads (the caller's thread is one
// of them), in contiguous ranges.
template <class F>
void parallel_for(int64_t n, int threads, F&& f) {
  if (n <= 0) return;
  const int t = (int)std::min<int64_t>(threads, n);
  if (t <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> pool;
  pool.reserve(t - 1);
  auto range = [&](int w) {
    const int64_t lo = n * w / t, hi = n * (w + 1) / t;
    for (int64_t i = lo; i < hi; ++i) f(i);
  };
  for (int w = 1; w < t; ++w) pool.emplace_back(range, w);
  range(0);
  for (auto& th : pool) th.join();
}

// Preparation step of one block: the ghosted block (5 cubes of (e+6)^3) from
// the interiors (5 cubes of e^3) of the block and its neighbours, one row of
// e+6 cells at a time in three pieces (x neighbours -1, 0, +1).
void gather_block(size_t es, int e, const char* interior, const int32_t* nbr27, char* out) {
  const int m = e + 6;
  const size_t cube = (size_t)e * e * e;
  const size_t blk = 5 * cube;
  for (int v = 0; v < 5; ++v) {
    for (int z = -3; z < e + 3; ++z) {
      const int rz = z < 0 ? -1 : (z >= e ? 1 : 0);
      const int lz = z - rz * e;
      for (int y = -3; y < e + 3; ++y) {
        const int ry = y < 0 ? -1 : (y >= e ? 1 : 0);
        const int ly = y - ry * e;
        char* row = out + es * ((size_t)v * m * m * m + ((size_t)(z + 3) * m + (y + 3)) * m);
        const int64_t pieces[3][3] = {{-1, e - 3, 3}, {0, 0, e}, {1, 0, 3}};
        int x0 = 0;
        for (const auto& pc : pieces) {
          const int rx = (int)pc[0];
          const int nb = nbr27[(rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)];
          const char* src = interior + es * ((size_t)nb * blk + (size_t)v * cube +
                                             ((size_t)lz * e + ly) * e + (size_t)pc[1]);
          memcpy(row + es * x0, src, es * (size_t)pc[2]);
          x0 += (int)pc[2];
        }
      }
    }
  }
}

}  // namespace

hipError_t run_host_pipeline(const HostPipe& hp, double times[7]) {
  const auto t_start = Clock::now();
  const size_t es = hp.dtype == 1 ? 4 : 8;
  const int e = hp.edge;
  const size_t gsz = 5 * (size_t)(e + 6) * (e + 6) * (e + 6);  // ghosted block, elements
  const size_t isz = 5 * (size_t)e * e * e;                    // interior block
  const int64_t per_launch = (int64_t)hp.ns * hp.ng;
  const int64_t launches = (hp.n_blocks + per_launch - 1) / per_launch;
  // pinned host staging: P[2] (ghosted inputs of a launch), Q[2] (outputs)
  char* P[2] = {(char*)hp.h_stage, (char*)hp.h_stage + es * gsz * per_launch};
  char* Q[2] = {P[1] + es * gsz * per_launch, P[1] + es * gsz * per_launch + es * isz * per_launch};
  // device staging per stream: N_g ghosted blocks in, N_g interior blocks out
  auto d_in = [&](int s) { return (char*)hp.d_stage + es * (gsz + isz) * hp.ng * s; };
  auto d_out = [&](int s) { return d_in(s) + es * gsz * hp.ng; };

  std::vector<hipEvent_t> h2d_ev(2 * hp.ns, nullptr), d2h_ev(2 * hp.ns, nullptr);
  std::vector<bool> h2d_used(2 * hp.ns, false), d2h_used(2 * hp.ns, false);
  // stage timing: four events per stream and launch (before the copy down,
  // after it, after the advance, after the copy up)
  std::vector<hipEvent_t> tev;
  hipError_t err = hipSuccess;
  for (int i = 0; i < 2 * hp.ns && err == hipSuccess; ++i) {
    err = hipEventCreateWithFlags(&h2d_ev[i], hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&d2h_ev[i], hipEventDisableTiming);
  }
  if (times && err == hipSuccess) {
    tev.assign(4 * (size_t)hp.ns * launches, nullptr);
    for (auto& ev : tev) {
      if ((err = hipEventCreate(&ev)) != hipSuccess) break;
    }
  }
  double prep_ms = 0.0, close_ms = 0.0;

  auto count_of = [&](int64_t k) { return std::min<int64_t>(per_launch, hp.n_blocks - k * per_launch); };
  auto prepare = [&](int64_t k, int par) {
    const auto t0 = Clock::now();
    const int64_t b0 = k * per_launch;
    parallel_for(count_of(k), hp.threads, [&](int64_t i) {
      gather_block(es, e, (const char*)hp.h_in, hp.h_nbr + 27 * (b0 + i), P[par] + es * gsz * i);
    });
    prep_ms += ms_since(t0);
  };
  auto close = [&](int64_t k, int par) {
    const auto t0 = Clock::now();
    const int64_t b0 = k * per_launch;
    parallel_for(count_of(k), hp.threads, [&](int64_t i) {
      memcpy((char*)hp.h_out + es * isz * (b0 + i), Q[par] + es * isz * i, es * isz);
    });
    close_ms += ms_since(t0);
  };
  auto wait_all = [&](std::vector<hipEvent_t>& ev, std::vector<bool>& used, int par) {
    for (int s = 0; s < hp.ns; ++s) {
      if (!used[par * hp.ns + s]) continue;
      const hipError_t e2 = hipEventSynchronize(ev[par * hp.ns + s]);
      if (e2 != hipSuccess) return e2;
    }
    return hipSuccess;
  };
  // one launch: stream s takes blocks [s N_g, (s+1) N_g) of it
  auto enqueue = [&](int64_t k, int par) {
    const int64_t cnt = count_of(k);
    for (int s = 0; s < hp.ns; ++s) {
      const int64_t lo = (int64_t)s * hp.ng, hi = std::min<int64_t>(cnt, lo + hp.ng);
      h2d_used[par * hp.ns + s] = hi > lo;
      d2h_used[par * hp.ns + s] = hi > lo;
      if (hi <= lo) continue;
      hipStream_t st = hp.streams[s];
      hipEvent_t* te = times ? &tev[4 * ((size_t)k * hp.ns + s)] : nullptr;
      hipError_t e2 = hipSuccess;
      if (te) e2 = hipEventRecord(te[0], st);
      if (e2 == hipSuccess)
        e2 = hipMemcpyAsync(d_in(s), P[par] + es * gsz * lo, es * gsz * (hi - lo),
                            hipMemcpyHostToDevice, st);
      if (e2 == hipSuccess) e2 = hipEventRecord(h2d_ev[par * hp.ns + s], st);
      if (e2 == hipSuccess && te) e2 = hipEventRecord(te[1], st);
      if (e2 == hipSuccess) {
        KParams kp = hp.kp;
        kp.uin = d_in(s);
        kp.uout = d_out(s);
        kp.nblocks = kp.nsrc = (int)(hi - lo);
        e2 = launch_batched(hp.dtype, hp.order, hp.variant, false, kp, st);
      }
      if (e2 == hipSuccess && te) e2 = hipEventRecord(te[2], st);
      if (e2 == hipSuccess)
        e2 = hipMemcpyAsync(Q[par] + es * isz * lo, d_out(s), es * isz * (hi - lo),
                            hipMemcpyDeviceToHost, st);
      if (e2 == hipSuccess) e2 = hipEventRecord(d2h_ev[par * hp.ns + s], st);
      if (e2 == hipSuccess && te) e2 = hipEventRecord(te[3], st);
      if (e2 != hipSuccess) return e2;
    }
    return hipSuccess;
  };

  if (err == hipSuccess && launches > 0) {
    if (hp.concurrent) {
      // launch k runs on the GPU while the host prepares launch k+1 and
      // closes launch k-1; buffers of one parity serve every other launch
      prepare(0, 0);
      for (int64_t k = 0; k < launches && err == hipSuccess; ++k) {
        const int par = (int)(k & 1), nxt = par ^ 1;
        err = enqueue(k, par);
        if (err != hipSuccess) break;
        if (k + 1 < launches) {
          // launch k-1 read P[nxt]: its copies down must be done
          if (k >= 1 && (err = wait_all(h2d_ev, h2d_used, nxt)) != hipSuccess) break;
          prepare(k + 1, nxt);
        }
        if (k >= 1) {
          if ((err = wait_all(d2h_ev, d2h_used, nxt)) != hipSuccess) break;
          close(k - 1, nxt);
        }
      }
      if (err == hipSuccess) {
        const int par = (int)((launches - 1) & 1);
        err = wait_all(d2h_ev, d2h_used, par);
        if (err == hipSuccess) close(launches - 1, par);
      }
    } else {
      // the host waits for each launch before preparing the next
      for (int64_t k = 0; k < launches && err == hipSuccess; ++k) {
        prepare(k, 0);
        err = enqueue(k, 0);
        if (err == hipSuccess) err = wait_all(d2h_ev, d2h_used, 0);
        if (err == hipSuccess) close(k, 0);
      }
    }
  }
  if (err != hipSuccess) {
    // leave no copy in flight into buffers the caller may free
    for (int s = 0; s < hp.ns; ++s) (void)hipStreamSynchronize(hp.streams[s]);
  }
  if (times) {
    double h2d = 0.0, ker = 0.0, d2h = 0.0, span = 0.0;
    if (err == hipSuccess && launches > 0) {
      for (int64_t k = 0; k < launches; ++k) {
        const int64_t cnt = count_of(k);
        for (int s = 0; s < hp.ns; ++s) {
          if ((int64_t)s * hp.ng >= cnt) continue;
          hipEvent_t* te = &tev[4 * ((size_t)k * hp.ns + s)];
          float a = 0.f, b = 0.f, c = 0.f;
          if (hipEventElapsedTime(&a, te[0], te[1]) != hipSuccess ||
              hipEventElapsedTime(&b, te[1], te[2]) != hipSuccess ||
              hipEventElapsedTime(&c, te[2], te[3]) != hipSuccess)
            continue;
          h2d += a;
          ker += b;
          d2h += c;
          // the GPU's span: from the first copy down of the call (launch 0,
          // stream 0) to the end of the last copy up
          float d = 0.f;
          if (hipEventElapsedTime(&d, tev[0], te[3]) == hipSuccess) span = std::max(span, (double)d);
        }
      }
    }
    times[0] = ms_since(t_start);
    times[1] = prep_ms;
    times[2] = close_ms;
    times[3] = h2d;
    times[4] = ker;
    times[5] = d2h;
    times[6] = span;
  }
  for (auto ev : h2d_ev)
    if (ev) (void)hipEventDestroy(ev);
  for (auto ev : d2h_ev)
    if (ev) (void)hipEventDestroy(ev);
  for (auto ev : tev)
    if (ev) (void)hipEventDestroy(ev);
  return err;
}

}  // namespace tvd
