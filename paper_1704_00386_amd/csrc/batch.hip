// batch.hip -- many graphs swept together.
//
// Every graph of a batch keeps its own internal numbering, incidence lists,
// tau buffers and per-sweep counters.  Their r-cliques are cut into tiles
// (graph, bin, id range) that form one combined work list; one epoch is one
// sweep of every graph still running, done by a persistent kernel whose
// workgroups pull tiles from an atomic counter until the list is exhausted
// (heaviest tiles first, so the tail of an epoch is short).  A graph whose
// previous sweep changed nothing is skipped tile by tile and dropped from the
// table at the next poll; graphs may join at any epoch (the server uses
// this), each counting its own sweeps from the epoch it joined.  All launch
// arguments are fixed device pointers and grid sizes -- the epoch number and
// table sizes live in device memory -- so a chunk of epochs is captured once
// in a HIP graph and replayed until the table outgrows its buffers.
//
// Tile and grid sizes come from a small autotuner, cached by (kind, mode,
// tau width, frontier, work bucket): a batch whose first sweep is short
// (launch-bound) times one trial sweep per candidate on scratch state and
// keeps the fastest; a longer one keeps the default, since there the
// configuration hardly matters and each trial would cost a whole sweep.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "api_util.h"
#include "batch.h"
#include "sweep_dev.h"

namespace nd {

namespace {

using namespace dev;

constexpr int kHubGrid = 256;
constexpr int kBeginGrid = 64;

// R's one 256-thread block pass covers, per bin type.
__host__ __device__ constexpr int rclq_per_pass(int type) {
  return type == kBinG1 ? 256 : type == kBinG4 ? 64 : type == kBinG16 ? 16 : 4;
}

// Largest incidence count of one pass, in units of 1024: passes of the
// G-bins cover at most 1024 incidences (R per pass x largest d_s of the
// bin); a pass of the wave bins (4 R of d_s < 2048, 1025, 513) up to 8x,
// 4x and 2x that.
constexpr int pass_units(int type) {
  return type == kBinWave ? 8 : type == kBinWave16 ? 4 : type == kBinWave8 ? 2 : 1;
}

__device__ __forceinline__ bool graph_live(const BGraph &G, int64_t e,
                                           int64_t *local) {
  *local = e - G.t0;
  if (*local < 0 || *local >= G.max_local) return false;
  return *local == 0 || changed_sum(&G.ring[(*local - 1) % kBatchRing]) != 0;
}

// Frontier state of graph G's sweep `local` (the rule of the one-graph
// sweep, per graph): flags are read only if the previous sweep wrote them,
// and notifications start once a sweep changed at most G.notify_below.
template <bool FR>
__device__ __forceinline__ void graph_frontier(const BGraph &G, int64_t local,
                                               SweepStats *sst,
                                               const uint8_t **act,
                                               uint8_t **act_next,
                                               uint8_t *stamp,
                                               const uint8_t **act_sum,
                                               uint8_t **sum_next) {
  *act = nullptr;
  *act_next = nullptr;
  *act_sum = nullptr;
  *sum_next = nullptr;
  *stamp = 0;
  if (!FR || local == 0) return;
  const SweepStats *prev = &G.ring[(local - 1) % kBatchRing];
  const bool valid = prev->notified != 0;
  const bool notify = valid || changed_sum(prev) <= G.notify_below;
  *act = valid ? G.act[local & 1] : nullptr;
  *act_next = notify ? G.act[(local + 1) & 1] : nullptr;
  *act_sum = valid ? G.act_sum[local & 1] : nullptr;
  *sum_next = notify ? G.act_sum[(local + 1) & 1] : nullptr;
  *stamp = sweep_stamp(local);
  if (notify && threadIdx.x == 0) sst->notified = 1;
}

// One epoch's tiles, pulled from a counter.  Two instances share the work:
// WIDE takes the tiles of the bins of 16 and 32 values per lane (tiles
// [0, nwide)), the other one every other bin, so that the registers of the
// wide lanes do not set the occupancy of the rest.
template <int K, typename T, bool AND, bool FR, bool WIDE>
__global__ __launch_bounds__(256) void k_batch_sweep(
    const BGraph *__restrict__ gs, const BTile *__restrict__ tiles,
    BState *__restrict__ st) {
  __shared__ int s_tile;
  const int64_t e = st->epoch;
  const int t_lo = WIDE ? 0 : st->nwide;
  const int t_hi = WIDE ? st->nwide : st->ntiles;
  unsigned int *counter = WIDE ? &st->counters[e % kCounterRing]
                               : &st->counters_narrow[e % kCounterRing];
  for (;;) {
    if (threadIdx.x == 0) s_tile = t_lo + (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int ti = s_tile;
    __syncthreads();
    if (ti >= t_hi) break;
    const BTile tile = tiles[ti];
    const BGraph &G = gs[tile.g];
    int64_t local;
    if (!graph_live(G, e, &local)) continue;
    const T *in = (const T *)G.tau[local & 1];
    T *out = (T *)G.tau[AND ? (local & 1) : ((local + 1) & 1)];
    SweepStats *sst = &G.ring[local % kBatchRing];
    const uint8_t *act, *act_sum;
    uint8_t *act_next, *sum_next, stamp;
    graph_frontier<FR>(G, local, sst, &act, &act_next, &stamp, &act_sum,
                       &sum_next);
    if (FR && act != nullptr) {
      // sparse sweep of the tile: flags tested a chunk at a time per wave
      unsigned long long n_ch = 0, n_ev = 0;
      const int64_t wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
      if constexpr (WIDE) {
        if (tile.type == kBinWave)
          sweep_sparse<K, 64, 32, T, AND>(G.inc_off, G.inc_ids, in, out, 1, tile.lo,
                                          tile.hi, wv, nw, act, act_next, stamp,
                                          &n_ch, &n_ev, act_sum, sum_next);
        else
          sweep_sparse<K, 64, 16, T, AND>(G.inc_off, G.inc_ids, in, out, 1, tile.lo,
                                          tile.hi, wv, nw, act, act_next, stamp,
                                          &n_ch, &n_ev, act_sum, sum_next);
      } else {
        switch (tile.type) {
          case kBinG1:
            sweep_sparse<K, 1, 4, T, AND>(G.inc_off, G.inc_ids, in, out, 1, tile.lo,
                                          tile.hi, wv, nw, act, act_next, stamp,
                                          &n_ch, &n_ev, act_sum, sum_next);
            break;
          case kBinG4:
            sweep_sparse<K, 4, 4, T, AND>(G.inc_off, G.inc_ids, in, out, 1, tile.lo,
                                          tile.hi, wv, nw, act, act_next, stamp,
                                          &n_ch, &n_ev, act_sum, sum_next);
            break;
          case kBinG16:
            sweep_sparse<K, 16, 4, T, AND>(G.inc_off, G.inc_ids, in, out, 1, tile.lo,
                                           tile.hi, wv, nw, act, act_next, stamp,
                                           &n_ch, &n_ev, act_sum, sum_next);
            break;
          case kBinG64:
            sweep_sparse<K, 64, 4, T, AND>(G.inc_off, G.inc_ids, in, out, 1, tile.lo,
                                           tile.hi, wv, nw, act, act_next, stamp,
                                           &n_ch, &n_ev, act_sum, sum_next);
            break;
          default:  // kBinWave8
            sweep_sparse<K, 64, 8, T, AND>(G.inc_off, G.inc_ids, in, out, 1, tile.lo,
                                           tile.hi, wv, nw, act, act_next, stamp,
                                           &n_ch, &n_ev, act_sum, sum_next);
            break;
        }
      }
      stat_add_counts(sst, n_ch, n_ev);
      continue;
    }
    const int per = rclq_per_pass(tile.type);
    for (int64_t base = tile.lo; base < tile.hi; base += per) {
      bool ch = false, ev = false;
      if constexpr (WIDE) {
        const int64_t R = base + threadIdx.x / 64;
        if (tile.type == kBinWave)
          ch = update_regs<K, 64, 32, T, AND, FR>(G.inc_off, G.inc_ids, in, out, 1,
                                              R, R < tile.hi, act, act_next, stamp, &ev, sum_next);
        else
          ch = update_regs<K, 64, 16, T, AND, FR>(G.inc_off, G.inc_ids, in, out, 1,
                                              R, R < tile.hi, act, act_next, stamp, &ev, sum_next);
      } else {
        switch (tile.type) {
          case kBinG1: {
            const int64_t R = base + threadIdx.x;
            ch = update_regs<K, 1, 4, T, AND, FR>(G.inc_off, G.inc_ids, in, out, 1, R,
                                              R < tile.hi, act, act_next, stamp, &ev, sum_next);
            break;
          }
          case kBinG4: {
            const int64_t R = base + threadIdx.x / 4;
            ch = update_regs<K, 4, 4, T, AND, FR>(G.inc_off, G.inc_ids, in, out, 1, R,
                                              R < tile.hi, act, act_next, stamp, &ev, sum_next);
            break;
          }
          case kBinG16: {
            const int64_t R = base + threadIdx.x / 16;
            ch = update_regs<K, 16, 4, T, AND, FR>(G.inc_off, G.inc_ids, in, out, 1,
                                               R, R < tile.hi, act, act_next, stamp, &ev, sum_next);
            break;
          }
          case kBinG64: {
            const int64_t R = base + threadIdx.x / 64;
            ch = update_regs<K, 64, 4, T, AND, FR>(G.inc_off, G.inc_ids, in, out, 1,
                                               R, R < tile.hi, act, act_next, stamp, &ev, sum_next);
            break;
          }
          default: {  // kBinWave8
            const int64_t R = base + threadIdx.x / 64;
            ch = update_regs<K, 64, 8, T, AND, FR>(G.inc_off, G.inc_ids, in, out, 1,
                                               R, R < tile.hi, act, act_next, stamp, &ev, sum_next);
            break;
          }
        }
      }
      stat_add(sst, ch, ev);
    }
  }
}

// r-cliques with d_s >= 2048: one workgroup each, grid-stride over the list.
template <int K, typename T, bool AND, bool FR>
__global__ __launch_bounds__(kBlockThreads) void k_batch_hubs(
    const BGraph *__restrict__ gs, const BHub *__restrict__ hubs,
    const BState *__restrict__ st) {
  __shared__ int32_t hist[kBlockHistBins];
  const int64_t e = st->epoch;
  const int nhubs = st->nhubs;
  for (int i = blockIdx.x; i < nhubs; i += gridDim.x) {
    const BHub hb = hubs[i];
    const BGraph &G = gs[hb.g];
    int64_t local;
    if (!graph_live(G, e, &local)) continue;
    const T *in = (const T *)G.tau[local & 1];
    T *out = (T *)G.tau[AND ? (local & 1) : ((local + 1) & 1)];
    SweepStats *sst = &G.ring[local % kBatchRing];
    const uint8_t *act, *act_sum;
    uint8_t *act_next, *sum_next, stamp;
    graph_frontier<FR>(G, local, sst, &act, &act_next, &stamp, &act_sum,
                       &sum_next);
    bool ev;
    const bool ch = update_block<K, T, AND, FR>(G.inc_off, G.inc_ids, in, out,
                                                1, hb.R, hist, act, act_next,
                                                stamp, &ev, sum_next);
    stat_add(sst, ch, ev);
  }
}

// Before an epoch: clear its tile counter and each live graph's counters.
__global__ void k_epoch_begin(const BGraph *__restrict__ gs,
                              BState *__restrict__ st) {
  const int64_t e = st->epoch;
  const int ng = st->ng;
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) {
    st->counters[e % kCounterRing] = 0;
    st->counters_narrow[e % kCounterRing] = 0;
  }
  for (int i = i0; i < ng; i += gridDim.x * blockDim.x) {
    const int64_t local = e - gs[i].t0;
    if (local >= 0 && local < gs[i].max_local) {
      SweepStats &z = gs[i].ring[local % kBatchRing];
      for (int q = 0; q < kStatParts; q++) {
        z.part[q].changed = 0;
        z.part[q].evaluated = 0;
      }
      z.notified = 0;
    }
  }
}

__global__ void k_epoch_end(BState *__restrict__ st) { st->epoch += 1; }

// Changed-counters of the last `n` epochs (ending before `e_end`), one row
// of kPollMax per graph; ~0 marks a sweep the graph did not run.
__global__ void k_collect(const BGraph *__restrict__ gs, int ng, int64_t e_end,
                          int n, unsigned long long *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng) return;
  for (int q = 0; q < n; q++) {
    const int64_t local = e_end - n + q - gs[i].t0;
    unsigned long long v = ~0ull;
    if (local >= 0 && local < gs[i].max_local)
      v = gs[i].ring[local % kBatchRing].changed_total();
    out[(int64_t)i * kPollMax + q] = v;
  }
}

struct TuneKey {
  int kind, mode, t16, fr, bucket;
  bool operator<(const TuneKey &o) const {
    return std::tie(kind, mode, t16, fr, bucket) <
           std::tie(o.kind, o.mode, o.t16, o.fr, o.bucket);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, BatchConfig> g_tune_cache;

int work_bucket(int64_t P) {
  int b = 0;
  while (P > 1) {
    P >>= 1;
    b++;
  }
  return b;
}

}  // namespace

// ------------------------------------------------------------ Batch

Batch::Batch(nd_ctx *ctx, nd_kind kind, nd_mode mode, bool tau16,
             bool frontier, hipStream_t caller)
    : ctx_(ctx), kind_(kind), mode_(mode), tau16_(tau16), frontier_(frontier) {
  cfg_ = default_config(ctx);
  if (const char *v = getenv("ND_FRONTIER_SWITCH")) notify_div_ = atoi(v);
  if (const char *v = getenv("ND_BATCH_NO_GRAPH")) use_graph = v[0] != '1';
  ND_HIP(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
  hipEvent_t ev;
  ND_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  ND_HIP(hipEventRecord(ev, caller));
  ND_HIP(hipStreamWaitEvent(s_, ev, 0));
  (void)hipEventDestroy(ev);
  StreamScope scope(s_);
  state_.reset(ctx->alloc, 1);
  BState z{};
  ND_HIP(hipMemcpyAsync(state_.p, &z, sizeof z, hipMemcpyHostToDevice, s_));
  ND_HIP(hipStreamSynchronize(s_));
}

Batch::~Batch() {
  (void)hipStreamSynchronize(s_);
  drop_graph();
  {
    StreamScope scope(s_);
    members_.clear();
    gs_.free();
    tiles_.free();
    hubs_.free();
    state_.free();
    poll_buf_.free();
  }
  ctx_->alloc.forget_stream(s_);
  (void)hipStreamDestroy(s_);
}

void Batch::drop_graph() {
  if (graph_exec_) {
    (void)hipGraphExecDestroy(graph_exec_);
    graph_exec_ = nullptr;
  }
}

BatchConfig Batch::default_config(nd_ctx *ctx) {
  BatchConfig c;
  c.grid = ctx->num_cu * 8;
  c.tiles_per_group = 8;
  return c;
}

Member *Batch::add(nd_graph *g, int32_t max_iters, void *user) {
  StreamScope scope(s_);
  KindState &ks = g->ks[kind_];
  ND_REQUIRE(ks.ready, ND_ERR_INVALID, "graph not prepared for the batch");
  ND_REQUIRE(ks.tau16 || !tau16_, ND_ERR_INVALID,
             "a 16-bit batch cannot hold a graph needing 32-bit tau");
  auto m = std::make_unique<Member>();
  m->g = g;
  m->user = user;
  m->t0 = epoch_;
  const int64_t cap = ks.nr + 1;  // Lemma 2: enough to observe convergence
  m->max_local = (max_iters < 0 || max_iters > cap) ? cap : max_iters;
  const int64_t tb = (tau16_ ? 2 : 4) * std::max<int64_t>(ks.nr, 1);
  m->tau0.reset(ctx_->alloc, tb);
  if (mode_ == ND_SND) m->tau1.reset(ctx_->alloc, tb);
  m->ring.reset(ctx_->alloc, kBatchRing);
  if (frontier_) {
    m->act0.reset(ctx_->alloc, std::max<int64_t>(ks.nr, 1));
    m->act1.reset(ctx_->alloc, std::max<int64_t>(ks.nr, 1));
    const int64_t ng = std::max<int64_t>((ks.nr + (1 << kGroupShift) - 1) >> kGroupShift, 1);
    m->sum0.reset(ctx_->alloc, ng);
    m->sum1.reset(ctx_->alloc, ng);
  }
  init_member_tau(*m);
  if (ks.nr == 0 || m->max_local == 0) {
    m->finished = true;
    m->converged = ks.nr == 0;
  }
  Member *raw = m.get();
  members_.push_back(std::move(m));
  dirty_ = true;
  return raw;
}

void Batch::init_member_tau(Member &m) {
  const KindState &ks = m.g->ks[kind_];
  if (ks.nr == 0) return;
  if (tau16_)
    init_tau(ks, m.tau0.p, s_);  // ks.tau16 holds (checked in add)
  else
    ND_HIP(hipMemcpyAsync(m.tau0.p, ks.ds.p, sizeof(int32_t) * ks.nr,
                          hipMemcpyDeviceToDevice, s_));
  if (mode_ == ND_SND)
    ND_HIP(hipMemcpyAsync(m.tau1.p, m.tau0.p, (tau16_ ? 2 : 4) * ks.nr,
                          hipMemcpyDeviceToDevice, s_));
  if (frontier_) {  // no stamps yet
    fill_u8(m.act0.p, 0, ks.nr, s_);
    fill_u8(m.act1.p, 0, ks.nr, s_);
    const int64_t ng = (ks.nr + (1 << kGroupShift) - 1) >> kGroupShift;
    fill_u8(m.sum0.p, 0, ng, s_);
    fill_u8(m.sum1.p, 0, ng, s_);
  }
}

std::vector<std::unique_ptr<Member>> Batch::take_finished() {
  std::vector<std::unique_ptr<Member>> out;
  std::vector<std::unique_ptr<Member>> keep;
  for (auto &m : members_)
    (m->finished ? out : keep).push_back(std::move(m));
  members_ = std::move(keep);
  if (!out.empty()) dirty_ = true;
  return out;
}

void Batch::rebuild() {
  StreamScope scope(s_);
  std::vector<BGraph> hg;
  std::vector<BTile> ht[kBinZero];  // per bin type; heaviest bins first
  std::vector<BHub> hh;
  int64_t work = 0;
  // Tile length: tiles hold about equal work bounds (pass_units) and an
  // epoch has about grid * tiles_per_group of them -- each costs one atomic
  // on the shared tile counter -- but never less than one block pass.
  int64_t units_total = 0;
  for (auto &mp : members_) {
    if (mp->finished) continue;
    const KindState &ks = mp->g->ks[kind_];
    for (int b = kBinWave; b < kBinZero; b++)
      units_total += (ks.bin_hi[b] - ks.bin_lo[b] + rclq_per_pass(b) - 1) /
                     rclq_per_pass(b) * pass_units(b);
  }
  const int64_t target = (int64_t)cfg_.grid * cfg_.tiles_per_group;
  const int64_t units = std::max<int64_t>(1, units_total / std::max<int64_t>(target, 1));
  for (auto &mp : members_) {
    Member &m = *mp;
    m.slot = -1;
    m.ntiles = 0;
    if (m.finished) continue;
    const KindState &ks = m.g->ks[kind_];
    const int32_t gi = (int32_t)hg.size();
    m.slot = gi;
    BGraph G{};
    G.inc_off = ks.inc_off.p;
    G.inc_ids = ks.inc_ids.p;
    G.tau[0] = m.tau0.p;
    G.tau[1] = mode_ == ND_SND ? m.tau1.p : m.tau0.p;
    G.ring = m.ring.p;
    G.t0 = m.t0;
    G.max_local = m.max_local;
    if (frontier_) {
      G.act[0] = m.act0.p;
      G.act[1] = m.act1.p;
      G.act_sum[0] = m.sum0.p;
      G.act_sum[1] = m.sum1.p;
      G.notify_below = notify_div_ <= 0
                           ? ~0ull
                           : (unsigned long long)(ks.bin_lo[kBinZero] / notify_div_);
    }
    hg.push_back(G);
    work += ks.P;
    for (int64_t R = ks.bin_lo[kBinBlock]; R < ks.bin_hi[kBinBlock]; R++)
      hh.push_back(BHub{gi, 0, R});
    for (int b = kBinWave; b < kBinZero; b++) {
      const int64_t lo = ks.bin_lo[b], hi = ks.bin_hi[b];
      const int64_t passes = std::max<int64_t>(1, units / pass_units(b));
      const int64_t step = (int64_t)rclq_per_pass(b) * passes;
      for (int64_t x = lo; x < hi; x += step) {
        ht[b].push_back(BTile{gi, b, x, std::min(hi, x + step)});
        m.ntiles++;
      }
    }
  }
  std::vector<BTile> all;
  for (int b = kBinWave; b < kBinZero; b++)
    all.insert(all.end(), ht[b].begin(), ht[b].end());
  ntiles_ = (int)all.size();
  nwide_ = (int)(ht[kBinWave].size() + ht[kBinWave16].size());  // first in `all`
  nhubs_ = (int)hh.size();
  ng_ = (int)hg.size();
  work_ = work;
  dead_tiles_ = 0;
  // Grow device tables (capacity doubles); a new buffer invalidates the
  // captured graph, whose kernels hold the table pointers.
  auto ensure = [&](auto &arr, int64_t need, int64_t &cap) {
    need = std::max<int64_t>(need, 1);
    if (need > cap) {
      cap = std::max<int64_t>(need, 2 * cap);
      arr.reset(ctx_->alloc, cap);
      drop_graph();
    }
  };
  ensure(gs_, (int64_t)hg.size(), gs_cap_);
  ensure(tiles_, (int64_t)all.size(), tiles_cap_);
  ensure(hubs_, (int64_t)hh.size(), hubs_cap_);
  ensure(poll_buf_, (int64_t)hg.size() * kPollMax, poll_cap_);
  if (!hg.empty())
    ND_HIP(hipMemcpyAsync(gs_.p, hg.data(), sizeof(BGraph) * hg.size(),
                          hipMemcpyHostToDevice, s_));
  if (!all.empty())
    ND_HIP(hipMemcpyAsync(tiles_.p, all.data(), sizeof(BTile) * all.size(),
                          hipMemcpyHostToDevice, s_));
  if (!hh.empty())
    ND_HIP(hipMemcpyAsync(hubs_.p, hh.data(), sizeof(BHub) * hh.size(),
                          hipMemcpyHostToDevice, s_));
  int32_t counts[4] = {ntiles_, nhubs_, ng_, nwide_};
  ND_HIP(hipMemcpyAsync(&state_.p->ntiles, counts, sizeof counts,
                        hipMemcpyHostToDevice, s_));
  ND_HIP(hipStreamSynchronize(s_));  // the host vectors go out of scope
  dirty_ = false;
}

template <int K, typename T, bool AND, bool FR>
void Batch::launch_epoch_t() {
  k_epoch_begin<<<kBeginGrid, 256, 0, s_>>>(gs_.p, state_.p);
  ND_LAUNCHED();
  k_batch_sweep<K, T, AND, FR, true><<<cfg_.grid, 256, 0, s_>>>(
      gs_.p, tiles_.p, state_.p);
  ND_LAUNCHED();
  k_batch_sweep<K, T, AND, FR, false><<<cfg_.grid, 256, 0, s_>>>(
      gs_.p, tiles_.p, state_.p);
  ND_LAUNCHED();
  k_batch_hubs<K, T, AND, FR><<<kHubGrid, kBlockThreads, 0, s_>>>(
      gs_.p, hubs_.p, state_.p);
  ND_LAUNCHED();
  k_epoch_end<<<1, 1, 0, s_>>>(state_.p);
  ND_LAUNCHED();
}

void Batch::launch_epoch() {
  const int k = kind_rs(kind_).k;
  const int key = (k * 2 + (tau16_ ? 1 : 0)) * 4 + (mode_ == ND_AND ? 2 : 0) +
                  (frontier_ ? 1 : 0);
#define ND_EPOCH_CASES(KK, T, BASE)                                   \
  case BASE + 0: launch_epoch_t<KK, T, false, false>(); break;       \
  case BASE + 1: launch_epoch_t<KK, T, false, true>(); break;        \
  case BASE + 2: launch_epoch_t<KK, T, true, false>(); break;        \
  case BASE + 3: launch_epoch_t<KK, T, true, true>(); break;
  switch (key) {
    ND_EPOCH_CASES(1, int32_t, 8)
    ND_EPOCH_CASES(1, uint16_t, 12)
    ND_EPOCH_CASES(2, int32_t, 16)
    ND_EPOCH_CASES(2, uint16_t, 20)
    ND_EPOCH_CASES(3, int32_t, 24)
    ND_EPOCH_CASES(3, uint16_t, 28)
    ND_EPOCH_CASES(5, int32_t, 40)
    ND_EPOCH_CASES(5, uint16_t, 44)
    default: ND_REQUIRE(false, ND_ERR_INVALID, "bad batch key %d", key);
  }
#undef ND_EPOCH_CASES
}

// Capture kGraphEpochs epochs into graph_exec_.  Relaxed mode: the capture
// itself makes no call that a capture forbids, and other threads of the
// process (a server's preparation thread allocating memory) must stay free
// to.  If the capture fails anyway, it is ended (so the stream leaves
// capture mode) and this batch launches its epochs directly from then on.
void Batch::capture() {
  hipGraph_t gr = nullptr;
  if (hipStreamBeginCapture(s_, hipStreamCaptureModeRelaxed) != hipSuccess) {
    (void)hipGetLastError();
    use_graph = false;
    return;
  }
  bool ok = true;
  try {
    for (int i = 0; i < kGraphEpochs; i++) launch_epoch();
  } catch (const Err &) {
    ok = false;
  }
  if (hipStreamEndCapture(s_, &gr) != hipSuccess) ok = false;
  if (ok && hipGraphInstantiate(&graph_exec_, gr, nullptr, nullptr, 0) != hipSuccess) {
    graph_exec_ = nullptr;
    ok = false;
  }
  if (gr) (void)hipGraphDestroy(gr);
  if (!ok) {
    (void)hipGetLastError();
    graph_exec_ = nullptr;
    use_graph = false;
  }
}

void Batch::run_epochs(int count) {
  if (dirty_) rebuild();
  if (ng_ == 0) return;
  if (use_graph && count == kGraphEpochs && !graph_exec_) capture();
  if (use_graph && count == kGraphEpochs && graph_exec_) {
    ND_HIP(hipGraphLaunch(graph_exec_, s_));
  } else {
    for (int i = 0; i < count; i++) launch_epoch();
  }
  epoch_ += count;
}

void Batch::poll(int epochs_run) {
  if (ng_ == 0 || epochs_run <= 0) return;
  ND_REQUIRE(epochs_run <= kPollMax, ND_ERR_INVALID, "poll window too large");
  k_collect<<<grid_for(ng_, 256), 256, 0, s_>>>(gs_.p, ng_, epoch_, epochs_run,
                                                 poll_buf_.p);
  ND_LAUNCHED();
  std::vector<unsigned long long> h((size_t)ng_ * kPollMax);
  ND_HIP(hipMemcpyAsync(h.data(), poll_buf_.p, sizeof(unsigned long long) * h.size(),
                        hipMemcpyDeviceToHost, s_));
  ND_HIP(hipStreamSynchronize(s_));
  for (auto &mp : members_) {
    Member &m = *mp;
    if (m.finished || m.slot < 0) continue;
    for (int q = 0; q < epochs_run && !m.finished; q++) {
      const int64_t local = epoch_ - epochs_run + q - m.t0;
      const unsigned long long v = h[(size_t)m.slot * kPollMax + q];
      if (local < 0 || local >= m.max_local || v == ~0ull) continue;
      m.sweeps = local + 1;
      if (v == 0) {
        m.converged = true;
        m.finished = true;
      }
    }
    if (!m.finished && m.sweeps >= m.max_local) m.finished = true;
    if (m.finished) dead_tiles_ += m.ntiles;
  }
  // drop finished graphs' tiles once they are a quarter of the table
  if (dead_tiles_ * 4 > ntiles_ && dead_tiles_ > 0) dirty_ = true;
}

const void *Batch::result_tau(const Member &m) const {
  if (mode_ == ND_AND) return m.tau0.p;
  return (m.sweeps & 1) ? m.tau1.p : m.tau0.p;
}

void Batch::set_config(const BatchConfig &c) {
  if (c.grid != cfg_.grid || c.tiles_per_group != cfg_.tiles_per_group) {
    cfg_ = c;
    dirty_ = true;
    drop_graph();
  }
}

// Pick the launch configuration.  The first epoch runs under the default
// configuration and counts as a real sweep; if it took kTuneSkipMs or more
// the batch is in the bandwidth-bound regime where the configuration hardly
// matters, and the default is kept (trials would cost whole sweeps).  A
// shorter (launch-bound) batch times one trial epoch per candidate on
// scratch state, then restores tau_0 and the epoch, so no epoch counts.
// Returns the real epochs run (0 or 1); the caller polls them.
int Batch::autotune() {
  StreamScope scope(s_);
  if (dirty_) rebuild();
  if (ng_ == 0) return 0;
  TuneKey key{(int)kind_, (int)mode_, tau16_ ? 1 : 0, frontier_ ? 1 : 0,
              work_bucket(work_)};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      set_config(it->second);
      return 0;
    }
  }
  hipEvent_t a, b;
  ND_HIP(hipEventCreate(&a));
  ND_HIP(hipEventCreate(&b));
  auto time_epoch = [&]() {
    ND_HIP(hipEventRecord(a, s_));
    launch_epoch();
    ND_HIP(hipEventRecord(b, s_));
    ND_HIP(hipEventSynchronize(b));
    float ms = 0;
    ND_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
  };
  const int64_t e0 = epoch_;
  const BatchConfig dflt = default_config(ctx_);
  set_config(dflt);
  if (dirty_) rebuild();
  const float first = time_epoch();
  int real = 0;
  BatchConfig best_cfg = dflt;
  float best = first;
  if (first >= kTuneSkipMs) {
    epoch_ += 1;
    real = 1;
  } else {
    const int cus = ctx_->num_cu;
    for (int gm : {4, 8, 16})
      for (int tpg : {4, 16}) {
        BatchConfig c;
        c.grid = cus * gm;
        c.tiles_per_group = tpg;
        set_config(c);
        rebuild();
        BState z{};
        z.epoch = e0;
        z.ntiles = ntiles_;
        z.nhubs = nhubs_;
        z.ng = ng_;
        z.nwide = nwide_;
        ND_HIP(hipMemcpyAsync(state_.p, &z, sizeof z, hipMemcpyHostToDevice, s_));
        const float ms = time_epoch();
        if (ms < best) {
          best = ms;
          best_cfg = c;
        }
      }
    for (auto &mp : members_) init_member_tau(*mp);
    set_config(best_cfg);
    rebuild();
    BState z{};
    z.epoch = e0;
    z.ntiles = ntiles_;
    z.nhubs = nhubs_;
    z.ng = ng_;
    z.nwide = nwide_;
    ND_HIP(hipMemcpyAsync(state_.p, &z, sizeof z, hipMemcpyHostToDevice, s_));
    ND_HIP(hipStreamSynchronize(s_));
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  tuned_ms = best;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = best_cfg;
  return real;
}

// ------------------------------------------------------- batch ABI

namespace {

constexpr int kPrepThreads = 4;

// Prepare the graphs that are not yet prepared for `kind`, on up to
// kPrepThreads host threads with a stream each (ordered after s), so that
// the short, launch-bound build phases of different graphs overlap; s then
// waits for every prep stream.  The first failure is rethrown.
void prepare_all(nd_ctx *ctx, int32_t count, nd_graph *const *graphs,
                 nd_kind kind, hipStream_t s) {
  std::vector<nd_graph *> todo;
  for (int i = 0; i < count; i++)
    if (!graphs[i]->ks[kind].ready &&
        std::find(todo.begin(), todo.end(), graphs[i]) == todo.end())
      todo.push_back(graphs[i]);
  if (todo.size() <= 1) {
    for (nd_graph *g : todo) prepare(g, kind, s);
    return;
  }
  const int nt = (int)std::min<size_t>(kPrepThreads, todo.size());
  hipEvent_t start;
  ND_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  ND_HIP(hipEventRecord(start, s));
  std::vector<hipStream_t> streams(nt, nullptr);
  for (int t = 0; t < nt; t++) {
    ND_HIP(hipStreamCreateWithFlags(&streams[t], hipStreamNonBlocking));
    ND_HIP(hipStreamWaitEvent(streams[t], start, 0));
  }
  (void)hipEventDestroy(start);
  std::atomic<size_t> next{0};
  std::atomic<bool> failed{false};
  std::vector<nd_status> codes(nt, ND_OK);
  std::vector<std::string> msgs(nt);
  std::vector<std::thread> threads;
  for (int t = 0; t < nt; t++)
    threads.emplace_back([&, t] {
      try {
        ND_HIP(hipSetDevice(ctx->device));
        StreamScope scope(streams[t]);
        for (size_t i; !failed && (i = next++) < todo.size();)
          prepare(todo[i], kind, streams[t]);
      } catch (const Err &e) {
        codes[t] = e.code;
        msgs[t] = nd_last_error();
        failed = true;
      } catch (const std::exception &e) {
        codes[t] = ND_ERR_DEVICE;
        msgs[t] = e.what();
        failed = true;
      }
    });
  for (auto &th : threads) th.join();
  for (int t = 0; t < nt; t++) {
    hipEvent_t done;
    ND_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    ND_HIP(hipEventRecord(done, streams[t]));
    ND_HIP(hipStreamWaitEvent(s, done, 0));
    (void)hipEventDestroy(done);
    ctx->alloc.forget_stream(streams[t]);
    (void)hipStreamDestroy(streams[t]);
  }
  for (int t = 0; t < nt; t++)
    if (codes[t] != ND_OK) {
      set_error("%s", msgs[t].c_str());
      throw Err(codes[t]);
    }
}

}  // namespace

nd_status batch_decompose(nd_ctx *ctx, int32_t count, nd_graph *const *graphs,
                          nd_kind kind, const nd_opts *opts_in,
                          int32_t *const *kappas, int on_device, hipStream_t s,
                          nd_result *res) {
  nd_opts opts;
  nd_opts_init(&opts);
  if (opts_in) opts = *opts_in;
  ND_REQUIRE(opts.mode == ND_SND || opts.mode == ND_AND, ND_ERR_INVALID,
             "unknown mode");
  ND_REQUIRE(opts.on_iter == nullptr && opts.stop_active_ratio == 0,
             ND_ERR_UNSUPPORTED,
             "batched decomposition supports mode, max_iters and use_frontier");
  bool all16 = true;
  std::vector<double> prep(count, 0.0);
  std::vector<bool> was(count);
  for (int i = 0; i < count; i++) {
    ND_REQUIRE(graphs[i] && graphs[i]->ctx == ctx, ND_ERR_INVALID,
               "graph %d is NULL or from another context", i);
    was[i] = graphs[i]->ks[kind].ready;
  }
  {
    Phase phase("nd.batch.prepare");
    prepare_all(ctx, count, graphs, kind, s);
  }
  for (int i = 0; i < count; i++) {
    prep[i] = was[i] ? 0.0 : graphs[i]->ks[kind].ms_prep;
    all16 &= graphs[i]->ks[kind].tau16;
  }
  Batch batch(ctx, kind, opts.mode, all16, opts.use_frontier != 0, s);
  hipStream_t bs = batch.stream();
  std::vector<Member *> ms;
  for (int i = 0; i < count; i++)
    ms.push_back(batch.add(graphs[i], opts.max_iters, nullptr));
  hipEvent_t a, b;
  ND_HIP(hipEventCreate(&a));
  ND_HIP(hipEventCreate(&b));
  ND_HIP(hipEventRecord(a, bs));
  Phase sweep_phase("nd.batch.sweeps");
  batch.poll(batch.autotune());
  int chunk = 2;
  for (;;) {
    bool any = false;
    for (Member *m : ms) any |= !m->finished;
    if (!any) break;
    batch.run_epochs(chunk);
    batch.poll(chunk);
    chunk = std::min(chunk * 2, Batch::kGraphEpochs);
  }
  ND_HIP(hipEventRecord(b, bs));
  ND_HIP(hipEventSynchronize(b));
  float ms_total = 0;
  ND_HIP(hipEventElapsedTime(&ms_total, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  nd_status out = ND_OK;
  StreamScope scope(bs);
  for (int i = 0; i < count; i++) {
    Member &m = *ms[i];
    const KindState &ks = graphs[i]->ks[kind];
    if (ks.nr > 0) {
      ND_REQUIRE(kappas && kappas[i], ND_ERR_INVALID, "kappas[%d] is NULL", i);
      if (on_device) {
        to_original(ks, batch.result_tau(m), batch.tau16(), kappas[i], bs);
      } else {
        DArr<int32_t> tmp(ctx->alloc, ks.nr);
        to_original(ks, batch.result_tau(m), batch.tau16(), tmp.p, bs);
        ND_HIP(hipMemcpyAsync(kappas[i], tmp.p, sizeof(int32_t) * ks.nr,
                              hipMemcpyDeviceToHost, bs));
        ND_HIP(hipStreamSynchronize(bs));
      }
    }
    if (res) {
      nd_result &r = res[i];
      memset(&r, 0, sizeof r);
      r.sweeps = (int32_t)m.sweeps;
      r.converged = m.converged ? 1 : 0;
      r.n_rcliques = ks.nr;
      r.n_incidence = ks.P;
      r.updates = ks.bin_lo[kBinZero] * m.sweeps;
      r.ms_prep = prep[i];
      r.ms_iterate = ms_total;  // shared by the whole batch
      r.max_sdegree = ks.max_ds;
      r.tau_bytes = batch.tau16() ? 2 : 4;
    }
    if (!m.converged) out = ND_ERR_NOT_CONVERGED;
  }
  ND_HIP(hipStreamSynchronize(bs));
  if (out != ND_OK) set_error("a graph of the batch stopped without converging");
  return out;
}

}  // namespace nd

using namespace nd;

extern "C" nd_status nd_batch_decompose(nd_ctx *ctx, int32_t count,
                                        nd_graph *const *graphs, nd_kind kind,
                                        const nd_opts *opts,
                                        int32_t *const *kappas, int on_device,
                                        void *stream, nd_result *res) {
  nd_status out = ND_OK;
  nd_status st = guarded([&] {
    ND_REQUIRE(ctx, ND_ERR_INVALID, "ctx is NULL");
    ND_REQUIRE(count >= 0 && (count == 0 || graphs), ND_ERR_INVALID,
               "bad graph list");
    ND_REQUIRE(kind_valid(kind),
               ND_ERR_UNSUPPORTED, "unknown kind");
    ND_HIP(hipSetDevice(ctx->device));
    StreamScope scope((hipStream_t)stream);
    if (count == 0) return;
    out = batch_decompose(ctx, count, graphs, kind, opts, kappas, on_device,
                          (hipStream_t)stream, res);
  });
  return st != ND_OK ? st : out;
}
