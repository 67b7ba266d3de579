// driver.hip -- the iteration driver of Alg. 2 (SND) and Alg. 3 (AND): start
// from tau_0 = d_s, sweep until a sweep changes nothing (the flag F of the
// algorithms), optionally stop early, and hand out per-sweep reports.
//
// Host round trips are amortised: sweeps are enqueued in chunks and each
// sweep kernel first reads the previous sweep's changed-counter and returns
// at once when it is zero, so sweeps queued past convergence cost only their
// launch.  For SND the two buffers then hold identical values, so the result
// is the same whichever was written last.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "api_util.h"
#include "internal.h"
#include "sweep_dev.h"

namespace nd {

namespace {

constexpr int kStatsRing = 1024;  // device counters kept per decomposition
constexpr int kMaxChunk = 16;     // sweeps enqueued per host round trip
constexpr int kGridPerCu = 64;    // sweep workgroups per CU (they stride;
                                  // measured best of 8..64 and uncapped)
constexpr int kGridPerCuFrontier = 40;  // with the frontier: mostly sparse
                                        // sweeps, where fewer workgroups
                                        // scan the flags sooner (24..64)

// Zero the counters of sweeps first .. first+count-1 (a kernel, not a
// memset, so that the sequence stays capturable).
__global__ void k_zero_stats(SweepStats *ring, int64_t first, int count) {
  constexpr int W = sizeof(SweepStats) / sizeof(unsigned long long);
  for (int i = threadIdx.x; i < count * W; i += blockDim.x) {
    unsigned long long *z =
        reinterpret_cast<unsigned long long *>(&ring[(first + i / W) % kStatsRing]);
    z[i % W] = 0;
  }
}

struct Timer {
  hipEvent_t a, b;
  Timer() {
    ND_HIP(hipEventCreate(&a));
    ND_HIP(hipEventCreate(&b));
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  void start(hipStream_t s) { ND_HIP(hipEventRecord(a, s)); }
  void stop(hipStream_t s) { ND_HIP(hipEventRecord(b, s)); }
  double ms() {
    ND_HIP(hipEventSynchronize(b));
    float m = 0;
    ND_HIP(hipEventElapsedTime(&m, a, b));
    return m;
  }
};

}  // namespace

// The sweep loop.  fixed_set (device, internal numbering, 1 = member) turns
// it into PartialAND: AND sweeps that recompute only the members, every
// other r-clique keeping tau_0 = d_s.
nd_status decompose_impl(nd_graph *g, nd_kind kind, const nd_opts *opts_in,
                         int32_t *kappa, int on_device, hipStream_t s,
                         nd_result *res, const uint8_t *fixed_set) {
  nd_opts opts;
  nd_opts_init(&opts);
  if (opts_in) opts = *opts_in;
  if (fixed_set) {
    opts.mode = ND_AND;
    opts.use_frontier = 0;
  }
  ND_REQUIRE(opts.mode == ND_SND || opts.mode == ND_AND, ND_ERR_INVALID,
             "unknown mode %d", (int)opts.mode);
  ND_REQUIRE(opts.stop_active_ratio >= 0 && opts.stop_active_ratio <= 1,
             ND_ERR_INVALID, "stop_active_ratio must be in [0,1]");
  ND_REQUIRE(kind_valid(kind), ND_ERR_UNSUPPORTED, "unknown kind %d",
             (int)kind);
  const bool was_ready = g->ks[kind].ready;
  prepare(g, kind, s);
  const KindState &ks = g->ks[kind];
  const int64_t nr = ks.nr;
  nd_result r{};
  r.n_rcliques = nr;
  r.n_incidence = ks.P;
  r.ms_prep = was_ready ? 0.0 : ks.ms_prep;
  r.max_sdegree = ks.max_ds;
  r.tau_bytes = ks.tau16 ? 2 : 4;
  ND_REQUIRE(kappa || nr == 0, ND_ERR_INVALID, "kappa is NULL");
  if (nr == 0) {
    r.converged = 1;
    if (res) *res = r;
    return ND_OK;
  }
  Allocator &al = g->ctx->alloc;
  const bool and_mode = opts.mode == ND_AND;
  // tau in the internal numbering, uint16 when it fits (ks.tau16)
  const int64_t tbytes = (ks.tau16 ? 2 : 4) * nr;
  DArr<uint8_t> tau0(al, tbytes), tau1;
  init_tau(ks, tau0.p, s);
  if (!and_mode) {
    tau1.reset(al, tbytes);
    ND_HIP(hipMemcpyAsync(tau1.p, tau0.p, tbytes, hipMemcpyDeviceToDevice, s));
  }
  void *buf[2] = {tau0.p, and_mode ? tau0.p : tau1.p};
  DArr<int32_t> snap;  // callback view, r-clique-id order, int32
  if (opts.on_iter) snap.reset(al, nr);
  // frontier flags (Section 4.3): act[t & 1] selects the r-cliques of sweep
  // t; every r-clique takes part in the first sweep
  DArr<uint8_t> act[2], act_sum[2];  // flags; one stamp per 64 r-cliques
  const bool frontier = opts.use_frontier != 0;
  // notifications start once a sweep changes at most 1/16 of the swept
  // r-cliques (ND_FRONTIER_SWITCH overrides the divisor; 0 = from the start)
  unsigned long long notify_below = 0;
  if (frontier) {
    act[0].reset(al, nr);
    act[1].reset(al, nr);
    fill_u8(act[0].p, 0, nr, s);  // no stamps yet
    fill_u8(act[1].p, 0, nr, s);
    const int64_t ng = (nr + (1 << dev::kGroupShift) - 1) >> dev::kGroupShift;
    act_sum[0].reset(al, ng);
    act_sum[1].reset(al, ng);
    fill_u8(act_sum[0].p, 0, ng, s);
    fill_u8(act_sum[1].p, 0, ng, s);
    int div = 16;
    if (const char *v = getenv("ND_FRONTIER_SWITCH")) div = atoi(v);
    notify_below = div <= 0 ? ~0ull : (unsigned long long)(ks.bin_lo[kBinZero] / div);
  }
  DArr<SweepStats> ring(al, kStatsRing);
  if (!g->ctx->host_stats)
    ND_HIP(hipHostMalloc(&g->ctx->host_stats, sizeof(SweepStats) * kStatsRing,
                         hipHostMallocDefault));
  SweepStats *hst = (SweepStats *)g->ctx->host_stats;

  // r-cliques whose h-index a sweep computes (d_s = 0 ones stay 0)
  const int64_t evaluated = ks.bin_lo[kBinZero];
  const bool step_by_step = opts.on_iter != nullptr || opts.stop_active_ratio > 0;
  int chunk = step_by_step ? 1 : 2;
  int64_t t = 0;  // sweeps enqueued
  int64_t sweeps = 0, updates = 0;
  bool converged = false, stop_ratio = false, stop_cb = false;
  Timer total, one;
  total.start(s);
  // Lemma 2: the iteration is exact after at most (number of degree levels)
  // <= |R| sweeps, so |R| + 1 sweeps always observe convergence; the cap only
  // guards against a defect turning into an endless loop.  A restricted
  // iteration ends too (some member drops by at least one in every sweep
  // but the last), without that bound.
  if (fixed_set) {
    if (opts.max_iters < 0) opts.max_iters = 0x7fffffff;
  } else if (opts.max_iters < 0 || opts.max_iters > nr + 1) {
    opts.max_iters = (int32_t)std::min<int64_t>(nr + 1, 0x7fffffff);
  }
  while (true) {
    if (t >= opts.max_iters) break;
    int nb = chunk;
    if (t + nb > opts.max_iters) nb = (int)(opts.max_iters - t);
    k_zero_stats<<<1, 256, 0, s>>>(ring.p, t, nb);
    ND_LAUNCHED();
    const int64_t t0 = t;
    for (int i = 0; i < nb; i++, t++) {
      SweepArgs a{};
      a.inc_off = ks.inc_off.p;
      a.inc_ids = ks.inc_ids.p;
      a.tau_in = buf[t & 1];
      a.tau_out = buf[(t + 1) & 1];
      a.stats = ring.p + (t % kStatsRing);
      a.prev = t > 0 ? ring.p + ((t - 1) % kStatsRing) : nullptr;
      a.cap_by_tau = 1;
      a.grid_cap = g->ctx->num_cu * (frontier ? kGridPerCuFrontier : kGridPerCu);
      if (frontier) {
        a.act = act[t & 1].p;
        a.act_next = act[(t + 1) & 1].p;
        a.act_sum = act_sum[t & 1].p;
        a.act_sum_next = act_sum[(t + 1) & 1].p;
        a.stamp = dev::sweep_stamp(t);
        a.notify_below = notify_below;
      } else if (fixed_set) {
        a.act = fixed_set;
        a.stamp = 1;
        a.fixed_set = 1;
      }
      if (step_by_step) one.start(s);
      launch_sweep(ks, a, and_mode, s);
      if (step_by_step) one.stop(s);
    }
    // read back this chunk's counters (the ring may wrap once)
    const int64_t f = t0 % kStatsRing;
    const int64_t first_n = std::min<int64_t>(nb, kStatsRing - f);
    ND_HIP(hipMemcpyAsync(hst + f, ring.p + f, sizeof(SweepStats) * first_n,
                          hipMemcpyDeviceToHost, s));
    if (first_n < nb)
      ND_HIP(hipMemcpyAsync(hst, ring.p, sizeof(SweepStats) * (nb - first_n),
                            hipMemcpyDeviceToHost, s));
    ND_HIP(hipStreamSynchronize(s));
    bool done = false;
    for (int64_t j = t0; j < t0 + nb && !done; j++) {
      const SweepStats &st = hst[j % kStatsRing];
      sweeps = j + 1;
      const int64_t changed = (int64_t)st.changed_total();
      const int64_t evald = (int64_t)st.evaluated_total();
      updates += evald;
      if (opts.on_iter) {
        to_original(ks, buf[(j + 1) & 1], ks.tau16, snap.p, s);
        ND_HIP(hipStreamSynchronize(s));
        nd_iter_info info{};
        info.iter = (int32_t)(j + 1);
        info.evaluated = evald;
        info.changed = changed;
        info.active_next = evaluated;
        info.tau_dev = snap.p;
        info.ms = one.ms();
        if (opts.on_iter(opts.user, &info)) stop_cb = true;
      }
      if (changed == 0) {
        converged = true;
        done = true;
      } else if (opts.stop_active_ratio > 0 &&
                 (double)changed < opts.stop_active_ratio * (double)nr) {
        stop_ratio = true;
        done = true;
      } else if (stop_cb) {
        done = true;
      }
    }
    if (done) break;
    chunk = std::min(chunk * 2, step_by_step ? 1 : kMaxChunk);
  }
  total.stop(s);
  r.ms_iterate = total.ms();
  r.sweeps = (int32_t)sweeps;
  r.converged = converged ? 1 : 0;
  r.updates = updates;
  const void *result = buf[sweeps & 1];
  if (on_device) {
    to_original(ks, result, ks.tau16, kappa, s);
  } else {
    DArr<int32_t> out(al, nr);
    to_original(ks, result, ks.tau16, out.p, s);
    ND_HIP(hipMemcpyAsync(kappa, out.p, sizeof(int32_t) * nr,
                          hipMemcpyDeviceToHost, s));
    ND_HIP(hipStreamSynchronize(s));
  }
  ND_HIP(hipStreamSynchronize(s));
  if (res) *res = r;
  if (converged || stop_ratio) return ND_OK;
  set_error("stopped after %lld sweeps without converging", (long long)sweeps);
  return ND_ERR_NOT_CONVERGED;
}

nd_status decompose(nd_graph *g, nd_kind kind, const nd_opts *opts,
                    int32_t *kappa, int on_device, hipStream_t s,
                    nd_result *res) {
  return decompose_impl(g, kind, opts, kappa, on_device, s, res, nullptr);
}

namespace {

// err = 1 if some id is outside [0, nr); else mark[inv[id]] = 1.
__global__ void k_mark_set(const int32_t *__restrict__ ids, int64_t count,
                           int64_t nr, const int32_t *__restrict__ inv,
                           uint8_t *__restrict__ mark, int32_t *__restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int32_t id = ids[i];
  if (id < 0 || id >= nr) {
    *err = 1;
    return;
  }
  mark[inv[id]] = 1;
}

__global__ void k_gather_ids(const int32_t *__restrict__ full,
                             const int32_t *__restrict__ ids, int64_t count,
                             int32_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = full[ids[i]];
}

}  // namespace

nd_status partial_and(nd_graph *g, nd_kind kind, const int32_t *ids,
                      int64_t count, const nd_opts *opts, int32_t *out,
                      int on_device, hipStream_t s, nd_result *res) {
  ND_REQUIRE(count >= 0 && (count == 0 || (ids && out)), ND_ERR_INVALID,
             "bad id list");
  prepare(g, kind, s);
  const KindState &ks = g->ks[kind];
  Allocator &al = g->ctx->alloc;
  const int64_t nr = ks.nr;
  DArr<int32_t> dids(al, std::max<int64_t>(count, 1));
  if (count > 0)
    ND_HIP(hipMemcpyAsync(dids.p, ids, sizeof(int32_t) * count,
                          on_device ? hipMemcpyDeviceToDevice
                                    : hipMemcpyHostToDevice, s));
  DArr<uint8_t> mark(al, std::max<int64_t>(nr, 1));
  DArr<int32_t> err(al, 1);
  fill_u8(mark.p, 0, std::max<int64_t>(nr, 1), s);
  fill_i32(err.p, 0, 1, s);
  if (count > 0) {
    k_mark_set<<<grid_for(count, 256), 256, 0, s>>>(dids.p, count, nr,
                                                     ks.inv.p, mark.p, err.p);
    ND_LAUNCHED();
  }
  int32_t herr = 0;
  ND_HIP(hipMemcpyAsync(&herr, err.p, sizeof herr, hipMemcpyDeviceToHost, s));
  ND_HIP(hipStreamSynchronize(s));
  ND_REQUIRE(herr == 0, ND_ERR_INVALID, "an r-clique id is outside [0, %lld)",
             (long long)nr);
  DArr<int32_t> full(al, std::max<int64_t>(nr, 1));
  const nd_status st =
      decompose_impl(g, kind, opts, full.p, 1, s, res, mark.p);
  if (st != ND_OK && st != ND_ERR_NOT_CONVERGED) return st;
  if (count > 0) {
    DArr<int32_t> got(al, count);
    k_gather_ids<<<grid_for(count, 256), 256, 0, s>>>(full.p, dids.p, count,
                                                       on_device ? out : got.p);
    ND_LAUNCHED();
    if (!on_device)
      ND_HIP(hipMemcpyAsync(out, got.p, sizeof(int32_t) * count,
                            hipMemcpyDeviceToHost, s));
    ND_HIP(hipStreamSynchronize(s));
  }
  return st;
}

}  // namespace nd

using namespace nd;

extern "C" nd_status nd_partial_and(nd_graph *g, nd_kind kind,
                                    const int32_t *ids, int64_t count,
                                    const nd_opts *opts, int32_t *out,
                                    int on_device, void *stream,
                                    nd_result *res) {
  nd_status outst = ND_OK;
  nd_status st = guarded([&] {
    ND_REQUIRE(g, ND_ERR_INVALID, "graph is NULL");
    ND_HIP(hipSetDevice(g->ctx->device));
    StreamScope scope((hipStream_t)stream);
    outst = partial_and(g, kind, ids, count, opts, out, on_device,
                        (hipStream_t)stream, res);
  });
  return st != ND_OK ? st : outst;
}

extern "C" nd_status nd_decompose(nd_graph *g, nd_kind kind,
                                  const nd_opts *opts, int32_t *kappa,
                                  int on_device, void *stream, nd_result *res) {
  nd_status out = ND_OK;
  nd_status st = guarded([&] {
    ND_REQUIRE(g, ND_ERR_INVALID, "graph is NULL");
    ND_HIP(hipSetDevice(g->ctx->device));
    StreamScope scope((hipStream_t)stream);
    out = decompose(g, kind, opts, kappa, on_device, (hipStream_t)stream, res);
  });
  return st != ND_OK ? st : out;
}
