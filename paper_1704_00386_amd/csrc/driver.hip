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

int frontier_switch(bool and_mode) {
  if (const char *v = getenv("ND_FRONTIER_SWITCH")) return atoi(v);
  (void)and_mode;
  return 8;
}


namespace {

constexpr int kStatsRing = 1024;  // device counters kept per decomposition
constexpr int kStaticRing = 64;   // the same, in the static workspace
constexpr int kMaxChunk = 16;     // sweeps enqueued per host round trip
static_assert(kMaxChunk < kStaticRing && kStaticRing <= kHostStatsRing &&
                  kStatsRing <= kHostStatsRing,
              "a chunk and its predecessor must fit every counter ring");
constexpr int64_t kSumsDiv = 256;  // see sums_after in sweep_loop
constexpr int kGridPerCu = 64;    // sweep workgroups per CU (they stride;
                                  // measured best of 8..64 and uncapped)

// Sweep workgroups per CU with the frontier (mostly sparse sweeps): about
// one wave per 4096 swept r-cliques (a wave's step of 64 flag groups), so
// that many short workgroups balance clustered flagged sets on big graphs,
// and few on small ones, where idle waves only add scheduling.  Measured
// per-CU grids of 16..384: the (3,4) block model (4.2e8 swept) best at 96,
// the Chung-Lu k-truss (8.6e6) and k-core (8.4e6) at 16..24.
int grid_per_cu_frontier(int64_t swept, int num_cu) {
  const int64_t waves_per_cu = swept / 4096 / std::max(num_cu, 1);
  return (int)std::min<int64_t>(96, std::max<int64_t>(16, waves_per_cu / 4));
}

// Zero the counters of sweeps first .. first+count-1 (a kernel, not a
// memset, so that the sequence stays capturable).
__global__ void k_zero_stats(SweepStats *ring, int ring_len, int64_t first,
                             int count) {
  constexpr int W = sizeof(SweepStats) / sizeof(unsigned long long);
  for (int i = threadIdx.x; i < count * W; i += blockDim.x) {
    unsigned long long *z =
        reinterpret_cast<unsigned long long *>(&ring[(first + i / W) % ring_len]);
    z[i % W] = 0;
  }
}

// The active-ratio indicator (Section 5.1.4): after a sweep, count the
// r-cliques flagged for the next one (act_next == stamp) into st->active,
// and clear the flags the sweep consumed (cur, sum_cur: the next sweep
// writes its notifications there), so that no stamp left from an earlier
// sweep is ever counted.  Four flags per thread step, compared as bytes:
// x = word ^ (stamp x 4) has a zero byte exactly where a flag matches, and
// ~(((x & 0x7f..) + 0x7f..) | x | 0x7f..) has the top bit of exactly those
// bytes set.
__global__ __launch_bounds__(256) void k_count_active(
    const uint8_t *__restrict__ next, uint8_t *__restrict__ cur,
    uint8_t *__restrict__ sum_cur, int64_t n, int64_t ngroups, uint8_t stamp,
    SweepStats *__restrict__ st) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const uint32_t pat = 0x01010101u * stamp;
  const int64_t n4 = n >> 2;
  unsigned long long c = 0;
  for (int64_t i = tid; i < n4; i += nth) {
    const uint32_t x = reinterpret_cast<const uint32_t *>(next)[i] ^ pat;
    const uint32_t y = ~(((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x | 0x7f7f7f7fu);
    c += __popc(y);
    reinterpret_cast<uint32_t *>(cur)[i] = 0;
  }
  for (int64_t i = 4 * n4 + tid; i < n; i += nth) {
    c += next[i] == stamp;
    cur[i] = 0;
  }
  for (int64_t i = tid; i < ngroups; i += nth) sum_cur[i] = 0;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
  if (lane_id() == 0 && c) atomicAdd(&st->active, c);
}

float elapsed_ms(hipEvent_t a, hipEvent_t b) {
  ND_HIP(hipEventSynchronize(b));
  float m = 0;
  ND_HIP(hipEventElapsedTime(&m, a, b));
  return m;
}

// Device buffers of one decomposition (see loop_layout for their sizes).
struct LoopBufs {
  void *tau[2] = {nullptr, nullptr};  // AND: both the same array
  uint8_t *act[2] = {nullptr, nullptr};      // flags (stamps)
  uint8_t *act_sum[2] = {nullptr, nullptr};  // one stamp per 64 r-cliques
  SweepStats *ring = nullptr;
  int ring_len = 0;
  int32_t *snap = nullptr;   // on_iter: tau_t in r-clique-id order
  int32_t *stage = nullptr;  // kappa on the device when it goes to the host
};

// Options as the loop runs them.
nd_opts effective_opts(const nd_opts *opts_in, bool fixed_set) {
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
  ND_REQUIRE(!fixed_set || opts.stop_active_ratio == 0, ND_ERR_UNSUPPORTED,
             "stop_active_ratio does not apply to PartialAND");
  return opts;
}

// The active-ratio indicator (notification flags counted after each sweep)
// is kept when asked for, or for the early stop that reads it.
bool wants_indicator(const nd_opts &o, bool fixed_set) {
  return !fixed_set && (o.count_active != 0 || o.stop_active_ratio > 0);
}

// Byte sizes of the buffers of a decomposition, each rounded to 256.
struct LoopLayout {
  int64_t tau, flags, sums, ring, snap, stage;
  int ntau;  // tau arrays: 2 for SND, 1 for AND (in place)
  int64_t total() const {
    return ntau * tau + 2 * flags + 2 * sums + ring + snap + stage;
  }
};
int64_t round256(int64_t b) { return (std::max<int64_t>(b, 1) + 255) / 256 * 256; }
LoopLayout loop_layout(const KindState &ks, const nd_opts &o, bool flags,
                       bool on_device, int ring_len) {
  const int64_t nr = ks.nr;
  LoopLayout L{};
  L.tau = round256(ks.tau_bytes * nr);
  L.ntau = o.mode == ND_AND ? 1 : 2;
  L.flags = flags ? round256(nr) : 0;
  L.sums = flags ? round256((nr + (1 << dev::kGroupShift) - 1) >> dev::kGroupShift) : 0;
  L.ring = round256((int64_t)sizeof(SweepStats) * ring_len);
  L.snap = o.on_iter ? round256(4 * nr) : 0;
  L.stage = on_device ? 0 : round256(4 * nr);
  return L;
}

// The sweep loop of Alg. 2 / Alg. 3 on prepared state, in the buffers b.
// fixed_set (device, internal numbering, 1 = member) turns it into
// PartialAND: AND sweeps that recompute only the members, every other
// r-clique keeping tau_0 = d_s.  r arrives with the sizes filled in.
nd_status sweep_loop(nd_graph *g, const KindState &ks, nd_opts opts,
                     int32_t *kappa, int on_device, hipStream_t s,
                     nd_result *res, nd_result r, const uint8_t *fixed_set,
                     const LoopBufs &b) {
  nd_ctx *ctx = g->ctx;
  const int64_t nr = ks.nr;
  const bool and_mode = opts.mode == ND_AND;
  const bool frontier = opts.use_frontier != 0;
  const bool indicator = wants_indicator(opts, fixed_set != nullptr);
  const bool flags = frontier || indicator;
  const int64_t tbytes = ks.tau_bytes * nr;
  init_tau(ks, b.tau[0], ks.tau_bytes, s);
  if (!and_mode)
    ND_HIP(hipMemcpyAsync(b.tau[1], b.tau[0], tbytes, hipMemcpyDeviceToDevice, s));
  const int64_t ng = (nr + (1 << dev::kGroupShift) - 1) >> dev::kGroupShift;
  // frontier flags (Section 4.3): act[t & 1] selects the r-cliques of sweep
  // t; every r-clique takes part in the first sweep.  Notifications start
  // once a sweep changes at most 1/frontier_switch() of the swept r-cliques;
  // with the indicator they run from the first sweep, so that every sweep's
  // active count is known.
  unsigned long long notify_below = 0, sums_after = 0;
  if (flags) {
    for (int i = 0; i < 2; i++) {
      fill_u8(b.act[i], 0, nr, s);  // no stamps yet
      fill_u8(b.act_sum[i], 0, ng, s);
    }
    const int div = frontier_switch(and_mode);
    notify_below = (indicator || div <= 0)
                       ? ~0ull
                       : (unsigned long long)(ks.bin_lo[kBinZero] / div);
    // Notifying sweeps after one that changed at least 1/256 of the swept
    // r-cliques leave the group summaries to k_group_sums (measured 1/16,
    // 1/64, 1/256 against in-sweep stores on the block model: SND 506 /
    // 501 / 497 ms against 505, AND 451 / 446 / 441 against 451; Chung-Lu
    // k-truss 0.5 ms faster, k-core unchanged).
    if (!indicator)
      sums_after = std::max<unsigned long long>(
          1, (unsigned long long)(ks.bin_lo[kBinZero] / kSumsDiv));
  }
  SweepStats *hst = (SweepStats *)ctx->host_stats;
  const int ring_len = b.ring_len;
  const int grid_per_cu =
      frontier ? grid_per_cu_frontier(ks.bin_lo[kBinZero], ctx->num_cu) : kGridPerCu;
  const bool step_by_step = opts.on_iter != nullptr || opts.stop_active_ratio > 0;
  int chunk = step_by_step ? 1 : 2;
  int64_t t = 0;  // sweeps enqueued
  int64_t sweeps = 0, updates = 0;
  bool converged = false, stop_ratio = false, stop_cb = false;
  hipEvent_t *ev = ctx->ev;  // ev[0..1]: whole loop; ev[2..3]: one sweep
  Phase sweeps_phase("nd.sweeps");
  ND_HIP(hipEventRecord(ev[0], s));
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
    k_zero_stats<<<1, 256, 0, s>>>(b.ring, ring_len, t, nb);
    ND_LAUNCHED();
    const int64_t t0 = t;
    for (int i = 0; i < nb; i++, t++) {
      SweepArgs a{};
      a.inc_off = ks.inc_off.p;
      a.inc_ids = ks.inc_ids.p;
      a.tau_in = b.tau[t & 1];
      a.tau_out = b.tau[(t + 1) & 1];
      a.stats = b.ring + (t % ring_len);
      a.prev = t > 0 ? b.ring + ((t - 1) % ring_len) : nullptr;
      a.cap_by_tau = 1;
      a.grid_cap = ctx->num_cu * grid_per_cu;
      if (flags) {
        a.act = b.act[t & 1];
        a.act_next = b.act[(t + 1) & 1];
        a.act_sum = b.act_sum[t & 1];
        a.act_sum_next = b.act_sum[(t + 1) & 1];
        a.stamp = dev::sweep_stamp(t);
        a.notify_below = notify_below;
        a.notify_first = indicator ? 1 : 0;
        a.flags_unused = frontier ? 0 : 1;
        a.sums_after = (frontier && !indicator) ? sums_after : 0;
      } else if (fixed_set) {
        a.act = fixed_set;
        a.stamp = 1;
        a.fixed_set = 1;
      }
      if (step_by_step) ND_HIP(hipEventRecord(ev[2], s));
      launch_sweep(ks, a, and_mode, s);
      launch_group_sums(ks, a, s);
      if (indicator) {
        const unsigned grid = (unsigned)std::min<int64_t>(
            std::max<int64_t>(1, ceil_div(nr, 4 * 256)), (int64_t)ctx->num_cu * 8);
        k_count_active<<<grid, 256, 0, s>>>(b.act[(t + 1) & 1], b.act[t & 1],
                                            b.act_sum[t & 1], nr, ng,
                                            dev::sweep_stamp(t + 1), a.stats);
        ND_LAUNCHED();
      }
      if (step_by_step) ND_HIP(hipEventRecord(ev[3], s));
    }
    // read back this chunk's counters (the ring may wrap once)
    const int64_t f = t0 % ring_len;
    const int64_t first_n = std::min<int64_t>(nb, ring_len - f);
    ND_HIP(hipMemcpyAsync(hst + f, b.ring + f, sizeof(SweepStats) * first_n,
                          hipMemcpyDeviceToHost, s));
    if (first_n < nb)
      ND_HIP(hipMemcpyAsync(hst, b.ring, sizeof(SweepStats) * (nb - first_n),
                            hipMemcpyDeviceToHost, s));
    ND_HIP(hipStreamSynchronize(s));
    bool done = false;
    for (int64_t j = t0; j < t0 + nb && !done; j++) {
      const SweepStats &st = hst[j % ring_len];
      sweeps = j + 1;
      const int64_t changed = (int64_t)st.changed_total();
      const int64_t evald = (int64_t)st.evaluated_total();
      updates += evald;
      const bool last = changed == 0 || j + 1 == opts.max_iters;
      if (opts.on_iter &&
          (opts.snapshot_every <= 1 || (j + 1) % opts.snapshot_every == 0 ||
           last)) {
        to_original(ks, b.tau[(j + 1) & 1], ks.tau_bytes, b.snap, s);
        ND_HIP(hipStreamSynchronize(s));
        nd_iter_info info{};
        info.iter = (int32_t)(j + 1);
        info.evaluated = evald;
        info.changed = changed;
        info.active_next = indicator ? (int64_t)st.active : -1;
        info.tau_dev = b.snap;
        info.ms = elapsed_ms(ev[2], ev[3]);
        if (opts.on_iter(opts.user, &info)) stop_cb = true;
      }
      if (changed == 0) {
        converged = true;
        done = true;
      } else if (opts.stop_active_ratio > 0 &&
                 (double)st.active < opts.stop_active_ratio * (double)nr) {
        stop_ratio = true;
        done = true;
      } else if (stop_cb) {
        done = true;
      }
    }
    if (done) break;
    chunk = std::min(chunk * 2, step_by_step ? 1 : kMaxChunk);
  }
  ND_HIP(hipEventRecord(ev[1], s));
  r.ms_iterate = elapsed_ms(ev[0], ev[1]);
  r.sweeps = (int32_t)sweeps;
  r.converged = converged ? 1 : 0;
  r.updates = updates;
  const void *result = b.tau[sweeps & 1];
  Phase out_phase("nd.output");
  if (on_device) {
    to_original(ks, result, ks.tau_bytes, kappa, s);
  } else {
    to_original(ks, result, ks.tau_bytes, b.stage, s);
    ND_HIP(hipMemcpyAsync(kappa, b.stage, sizeof(int32_t) * nr,
                          hipMemcpyDeviceToHost, s));
  }
  ND_HIP(hipStreamSynchronize(s));
  if (res) *res = r;
  if (converged || stop_ratio) return ND_OK;
  set_error("stopped after %lld sweeps without converging", (long long)sweeps);
  return ND_ERR_NOT_CONVERGED;
}

// Sizes known before the loop runs.
nd_result result_head(const KindState &ks, bool was_ready) {
  nd_result r{};
  r.n_rcliques = ks.nr;
  r.n_incidence = ks.P;
  r.ms_prep = was_ready ? 0.0 : ks.ms_prep;
  r.max_sdegree = ks.max_ds;
  r.tau_bytes = ks.tau_bytes;
  return r;
}

}  // namespace

// The decomposition with buffers from the context's allocator (prepares the
// kind first if needed).
nd_status decompose_impl(nd_graph *g, nd_kind kind, const nd_opts *opts_in,
                         int32_t *kappa, int on_device, hipStream_t s,
                         nd_result *res, const uint8_t *fixed_set) {
  const nd_opts opts = effective_opts(opts_in, fixed_set != nullptr);
  ND_REQUIRE(kind_valid(kind), ND_ERR_UNSUPPORTED, "unknown kind %d",
             (int)kind);
  const bool was_ready = g->ks[kind].ready;
  prepare(g, kind, s);
  const KindState &ks = g->ks[kind];
  const nd_result r = result_head(ks, was_ready);
  ND_REQUIRE(kappa || ks.nr == 0, ND_ERR_INVALID, "kappa is NULL");
  if (ks.nr == 0) {
    nd_result z = r;
    z.converged = 1;
    if (res) *res = z;
    return ND_OK;
  }
  Allocator &al = g->ctx->alloc;
  const bool flags =
      opts.use_frontier != 0 || wants_indicator(opts, fixed_set != nullptr);
  const LoopLayout L = loop_layout(ks, opts, flags, on_device != 0, kStatsRing);
  DArr<uint8_t> tau0(al, L.tau), tau1, act[2], sums[2], snap, stage;
  DArr<uint8_t> ring(al, L.ring);
  LoopBufs b;
  b.tau[0] = b.tau[1] = tau0.p;
  if (opts.mode != ND_AND) {
    tau1.reset(al, L.tau);
    b.tau[1] = tau1.p;
  }
  if (flags)
    for (int i = 0; i < 2; i++) {
      act[i].reset(al, L.flags);
      sums[i].reset(al, L.sums);
      b.act[i] = act[i].p;
      b.act_sum[i] = sums[i].p;
    }
  b.ring = (SweepStats *)ring.p;
  b.ring_len = kStatsRing;
  if (L.snap) {
    snap.reset(al, L.snap);
    b.snap = (int32_t *)snap.p;
  }
  if (L.stage) {
    stage.reset(al, L.stage);
    b.stage = (int32_t *)stage.p;
  }
  return sweep_loop(g, ks, opts, kappa, on_device, s, res, r, fixed_set, b);
}

// The same decomposition in the static workspace (nd_decompose_noalloc): no
// device or host memory is allocated.
nd_status decompose_noalloc(nd_graph *g, nd_kind kind, const nd_opts *opts_in,
                            int32_t *kappa, int on_device, hipStream_t s,
                            nd_result *res) {
  const nd_opts opts = effective_opts(opts_in, false);
  ND_REQUIRE(kind_valid(kind), ND_ERR_UNSUPPORTED, "unknown kind %d",
             (int)kind);
  const KindState &ks = g->ks[kind];
  ND_REQUIRE(ks.ready, ND_ERR_INVALID,
             "the graph is not prepared for this kind (call nd_prepare first)");
  const nd_result r = result_head(ks, true);
  ND_REQUIRE(kappa || ks.nr == 0, ND_ERR_INVALID, "kappa is NULL");
  if (ks.nr == 0) {
    nd_result z = r;
    z.converged = 1;
    if (res) *res = z;
    return ND_OK;
  }
  const bool flags = opts.use_frontier != 0 || wants_indicator(opts, false);
  const LoopLayout L = loop_layout(ks, opts, flags, on_device != 0, kStaticRing);
  ND_REQUIRE(L.total() <= (int64_t)kNoallocWorkspaceBytes, ND_ERR_OOM,
             "the decomposition needs %lld bytes of workspace; the static "
             "workspace holds %lld",
             (long long)L.total(), (long long)kNoallocWorkspaceBytes);
  uint8_t *w = (uint8_t *)noalloc_workspace(g->ctx->device);
  ND_REQUIRE(w != nullptr, ND_ERR_DEVICE,
             "no static workspace on device %d", g->ctx->device);
  auto take = [&](int64_t bytes) {
    uint8_t *p = w;
    w += bytes;
    return p;
  };
  LoopBufs b;
  b.tau[0] = b.tau[1] = take(L.tau);
  if (opts.mode != ND_AND) b.tau[1] = take(L.tau);
  if (flags)
    for (int i = 0; i < 2; i++) {
      b.act[i] = take(L.flags);
      b.act_sum[i] = take(L.sums);
    }
  b.ring = (SweepStats *)take(L.ring);
  b.ring_len = kStaticRing;
  if (L.snap) b.snap = (int32_t *)take(L.snap);
  if (L.stage) b.stage = (int32_t *)take(L.stage);
  return sweep_loop(g, ks, opts, kappa, on_device, s, res, r, nullptr, b);
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

extern "C" nd_status nd_decompose_noalloc(nd_graph *g, nd_kind kind,
                                          const nd_opts *opts, int32_t *kappa,
                                          int on_device, void *stream,
                                          nd_result *res) {
  nd_status out = ND_OK;
  nd_status st = guarded([&] {
    ND_REQUIRE(g, ND_ERR_INVALID, "graph is NULL");
    ND_HIP(hipSetDevice(g->ctx->device));
    StreamScope scope((hipStream_t)stream);
    out = decompose_noalloc(g, kind, opts, kappa, on_device,
                            (hipStream_t)stream, res);
  });
  return st != ND_OK ? st : out;
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
