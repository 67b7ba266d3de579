// batch.hip -- many graphs swept together.
//
// Every graph of a batch keeps its own internal numbering, incidence lists,
// tau buffers and per-sweep counters.  Their r-cliques are cut into tiles
// (graph, bin, id range) that form one combined work list; one epoch is one
// sweep of every graph still running, one workgroup per tile, heaviest
// tiles first (dispatched first, so the tail of an epoch is short).  A
// graph whose
// previous sweep changed nothing is skipped tile by tile and dropped from the
// table at the next poll; graphs may join at any epoch (the server uses
// this), each counting its own sweeps from the epoch it joined.  All launch
// arguments are fixed device pointers and grid sizes -- the epoch number and
// table sizes live in device memory -- so a chunk of epochs is built once
// in a HIP graph and replayed until the table outgrows its buffers.
//
// Tile sizes come from a small autotuner, cached by (kind, mode,
// tau width, frontier, work bucket): a batch whose first sweep is short
// (launch-bound) times one trial sweep per candidate on scratch state and
// keeps the fastest; a longer one keeps the default, since there the
// configuration hardly matters and each trial would cost a whole sweep.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
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

// One epoch's tiles, one workgroup per tile (tile i of the kernel's range
// on workgroup i; the grid is the table's capacity, surplus workgroups
// exit at once).  Workgroups are short-lived, so the work of other streams
// (a server's preparations) is dispatched between them rather than waiting
// for the epoch to end.  Two instances share the work: WIDE takes the tiles
// of the bins of 16 and 32 values per lane (tiles [0, nwide)), the other
// one every other bin, so that the registers of the wide lanes do not set
// the occupancy of the rest.
template <int K, typename T, bool AND, bool FR, bool WIDE>
__global__ __launch_bounds__(256) void k_batch_sweep(
    const BGraph *__restrict__ gs, const BTile *__restrict__ tiles,
    const BState *__restrict__ st) {
  const int64_t e = st->epoch;
  const int t_lo = WIDE ? 0 : st->nwide;
  const int t_hi = WIDE ? st->nwide : st->ntiles;
  const int ti = t_lo + (int)blockIdx.x;
  if (ti >= t_hi) return;
  {
    const BTile tile = tiles[ti];
    const BGraph &G = gs[tile.g];
    int64_t local;
    if (!graph_live(G, e, &local)) return;
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
      return;
    }
    const int per = rclq_per_pass(tile.type);
    unsigned long long n_ch = 0, n_ev = 0;  // this wave's, over the passes
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
      n_ch += __popcll(ballot(ch));
      n_ev += __popcll(ballot(ev));
    }
    stat_add_counts(sst, n_ch, n_ev);
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

// Before an epoch: clear each live graph's counters.
__global__ void k_epoch_begin(const BGraph *__restrict__ gs,
                              const BState *__restrict__ st) {
  const int64_t e = st->epoch;
  const int ng = st->ng;
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
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
  notify_div_ = frontier_switch(mode == ND_AND);
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
    init_tau(ks, m.tau0.p, 2, s_);  // ks.tau16 holds (checked in add)
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
  // epoch has about grid * tiles_per_group of them -- each a workgroup of
  // its own -- but never less than one block pass.
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
  // epoch graph, whose kernel nodes hold the table pointers.
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
  // grids of the two tile kernels: the capacity of their tile ranges
  auto ensure_grid = [&](int64_t need, int64_t &cap) {
    need = std::max<int64_t>(need, 1);
    if (need > cap) {
      cap = std::max<int64_t>(need, 2 * cap);
      drop_graph();
    }
  };
  ensure_grid(nwide_, wide_grid_);
  ensure_grid((int64_t)ntiles_ - nwide_, narrow_grid_);
  int32_t counts[4] = {ntiles_, nhubs_, ng_, nwide_};
  ND_HIP(hipMemcpyAsync(&state_.p->ntiles, counts, sizeof counts,
                        hipMemcpyHostToDevice, s_));
  ND_HIP(hipStreamSynchronize(s_));  // the host vectors go out of scope
  dirty_ = false;
}

// The kernels of one epoch, in launch order, for the batch's instance.
struct EpochKernels {
  const void *fn[5];  // begin, wide tiles, other tiles, hubs, end
};

template <int K, typename T, bool AND, bool FR>
EpochKernels epoch_kernels_t() {
  return {{(const void *)k_epoch_begin,
           (const void *)k_batch_sweep<K, T, AND, FR, true>,
           (const void *)k_batch_sweep<K, T, AND, FR, false>,
           (const void *)k_batch_hubs<K, T, AND, FR>, (const void *)k_epoch_end}};
}

static EpochKernels epoch_kernels(int k, bool tau16, bool and_mode, bool fr) {
  const int key = (k * 2 + (tau16 ? 1 : 0)) * 4 + (and_mode ? 2 : 0) + (fr ? 1 : 0);
#define ND_EPOCH_CASES(KK, T, BASE)                                 \
  case BASE + 0: return epoch_kernels_t<KK, T, false, false>();    \
  case BASE + 1: return epoch_kernels_t<KK, T, false, true>();     \
  case BASE + 2: return epoch_kernels_t<KK, T, true, false>();     \
  case BASE + 3: return epoch_kernels_t<KK, T, true, true>();
  switch (key) {
    ND_EPOCH_CASES(1, int32_t, 8)
    ND_EPOCH_CASES(1, uint16_t, 12)
    ND_EPOCH_CASES(2, int32_t, 16)
    ND_EPOCH_CASES(2, uint16_t, 20)
    ND_EPOCH_CASES(3, int32_t, 24)
    ND_EPOCH_CASES(3, uint16_t, 28)
    ND_EPOCH_CASES(5, int32_t, 40)
    ND_EPOCH_CASES(5, uint16_t, 44)
    default: break;
  }
#undef ND_EPOCH_CASES
  ND_REQUIRE(false, ND_ERR_INVALID, "bad batch key %d", key);
  return {};
}

// Grid, block and arguments of kernel i of an epoch.  The argument values
// live in *this (table pointers), so `args` stays valid while they do.
struct EpochLaunch {
  const BGraph *gs;
  const BTile *tiles;
  const BHub *hubs;
  BState *st;
  void *a_begin[2], *a_tiles[3], *a_hubs[3], *a_end[1];
  dim3 grid[5], block[5];
  void **args[5];
  EpochLaunch(const BGraph *g, const BTile *t, const BHub *h, BState *s,
              int64_t wide_grid, int64_t narrow_grid)
      : gs(g), tiles(t), hubs(h), st(s) {
    a_begin[0] = &gs;
    a_begin[1] = &st;
    a_tiles[0] = &gs;
    a_tiles[1] = &tiles;
    a_tiles[2] = &st;
    a_hubs[0] = &gs;
    a_hubs[1] = &hubs;
    a_hubs[2] = &st;
    a_end[0] = &st;
    void **a[5] = {a_begin, a_tiles, a_tiles, a_hubs, a_end};
    const int64_t gr[5] = {kBeginGrid, wide_grid, narrow_grid, kHubGrid, 1};
    const int bl[5] = {256, 256, 256, kBlockThreads, 1};
    for (int i = 0; i < 5; i++) {
      args[i] = a[i];
      grid[i] = dim3((unsigned)gr[i]);
      block[i] = dim3(bl[i]);
    }
  }
  EpochLaunch(const EpochLaunch &) = delete;
};

void Batch::launch_epoch() {
  const EpochKernels ek =
      epoch_kernels(kind_rs(kind_).k, tau16_, mode_ == ND_AND, frontier_);
  EpochLaunch el(gs_.p, tiles_.p, hubs_.p, state_.p, wide_grid_, narrow_grid_);
  for (int i = 0; i < 5; i++) {
    ND_HIP(hipLaunchKernel(ek.fn[i], el.grid[i], el.block[i], el.args[i], 0, s_));
  }
}

// Build kGraphEpochs epochs as a HIP graph, node by node (no stream
// capture, so other threads stay free to use any stream, the legacy one
// included, while it is built); on failure this batch launches its epochs
// directly from then on.
void Batch::build_graph() {
  const EpochKernels ek =
      epoch_kernels(kind_rs(kind_).k, tau16_, mode_ == ND_AND, frontier_);
  EpochLaunch el(gs_.p, tiles_.p, hubs_.p, state_.p, wide_grid_, narrow_grid_);
  hipGraph_t gr = nullptr;
  bool ok = hipGraphCreate(&gr, 0) == hipSuccess;
  hipGraphNode_t prev = nullptr;
  for (int e = 0; ok && e < kGraphEpochs; e++)
    for (int i = 0; ok && i < 5; i++) {
      hipKernelNodeParams np{};
      np.func = const_cast<void *>(ek.fn[i]);
      np.gridDim = el.grid[i];
      np.blockDim = el.block[i];
      np.sharedMemBytes = 0;
      np.kernelParams = el.args[i];
      np.extra = nullptr;
      hipGraphNode_t node = nullptr;
      ok = hipGraphAddKernelNode(&node, gr, prev ? &prev : nullptr, prev ? 1 : 0,
                                 &np) == hipSuccess;
      prev = node;
    }
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
  if (use_graph && count == kGraphEpochs && !graph_exec_) build_graph();
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

constexpr int kPrepThreads = 2;

int prep_threads() {
  static const int n = [] {
    const char *v = getenv("ND_PREP_THREADS");
    const int x = v ? atoi(v) : kPrepThreads;
    return x < 1 ? 1 : x > 16 ? 16 : x;
  }();
  return n;
}

namespace {

// Prepares graphs for one kind on up to prep_threads() host threads, each
// with a stream of its own ordered after the caller's, largest graphs first
// (their sweeps are the longest, so they should start first).  Each
// prepared graph is handed to the consumer with an event recorded after its
// work, so the consumer's stream can wait for exactly that graph; the
// short, launch-bound build phases of different graphs overlap each other
// and the consumer's sweeps.
class PrepPool {
 public:
  PrepPool(nd_ctx *ctx, int32_t count, nd_graph *const *graphs, nd_kind kind,
           hipStream_t after)
      : ctx_(ctx), kind_(kind) {
    for (int i = 0; i < count; i++)
      if (!graphs[i]->ks[kind].ready &&
          std::find(todo_.begin(), todo_.end(), graphs[i]) == todo_.end())
        todo_.push_back(graphs[i]);
    std::stable_sort(todo_.begin(), todo_.end(),
                     [](const nd_graph *a, const nd_graph *b) { return a->nnz > b->nnz; });
    if (todo_.empty()) return;
    const int nt = (int)std::min<size_t>(prep_threads(), todo_.size());
    hipEvent_t start;
    ND_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    ND_HIP(hipEventRecord(start, after));
    for (int t = 0; t < nt; t++) {
      hipStream_t st = nullptr;
      const hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      if (e != hipSuccess) {
        (void)hipEventDestroy(start);
        ND_HIP(e);
      }
      streams_.push_back(st);
      ND_HIP(hipStreamWaitEvent(st, start, 0));
    }
    (void)hipEventDestroy(start);
    for (int t = 0; t < nt; t++) threads_.emplace_back([this, t] { run(t); });
  }

  ~PrepPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      failed_ = true;  // stop taking graphs
    }
    join();
    for (auto &d : done_) (void)hipEventDestroy(d.second);
    for (hipStream_t st : streams_) {
      ctx_->alloc.forget_stream(st);
      (void)hipStreamDestroy(st);
    }
  }

  int pending() const { return (int)todo_.size(); }

  // The next prepared graph and its event (owned by the caller).  Waits for
  // one when `block`; returns false when none is ready (not blocking), when
  // every graph has been handed out, or after a failure (see rethrow).
  bool next(bool block, nd_graph **g, hipEvent_t *ev) {
    std::unique_lock<std::mutex> lk(mu_);
    if (block)
      cv_.wait(lk, [&] { return !done_.empty() || failed_ || handed_ == todo_.size(); });
    if (done_.empty()) return false;
    *g = done_.front().first;
    *ev = done_.front().second;
    done_.pop_front();
    handed_++;
    return true;
  }

  // Every graph handed out.
  bool finished() {
    std::lock_guard<std::mutex> lk(mu_);
    return handed_ == todo_.size();
  }

  // A preparation failed (finish() throws it).
  bool failed() {
    std::lock_guard<std::mutex> lk(mu_);
    return code_ != ND_OK;
  }

  // Join the threads; make `s` wait for every preparation stream; throw the
  // first failure.
  void finish(hipStream_t s) {
    join();
    for (hipStream_t st : streams_) {
      hipEvent_t d;
      ND_HIP(hipEventCreateWithFlags(&d, hipEventDisableTiming));
      ND_HIP(hipEventRecord(d, st));
      ND_HIP(hipStreamWaitEvent(s, d, 0));
      (void)hipEventDestroy(d);
    }
    rethrow();
  }

  void rethrow() {
    std::lock_guard<std::mutex> lk(mu_);
    if (code_ != ND_OK) {
      set_error("%s", msg_.c_str());
      throw Err(code_);
    }
  }

 private:
  void join() {
    for (auto &th : threads_)
      if (th.joinable()) th.join();
  }

  void run(int t) {
    try {
      ND_HIP(hipSetDevice(ctx_->device));
      StreamScope scope(streams_[t]);
      for (;;) {
        nd_graph *g;
        {
          std::lock_guard<std::mutex> lk(mu_);
          if (failed_ || next_ == todo_.size()) return;
          g = todo_[next_++];
        }
        prepare(g, kind_, streams_[t]);
        hipEvent_t ev;
        ND_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        const hipError_t e = hipEventRecord(ev, streams_[t]);
        if (e != hipSuccess) {
          (void)hipEventDestroy(ev);
          ND_HIP(e);
        }
        std::lock_guard<std::mutex> lk(mu_);
        done_.emplace_back(g, ev);
        cv_.notify_all();
      }
    } catch (const Err &e) {
      fail(e.code, nd_last_error());
    } catch (const std::exception &e) {
      fail(ND_ERR_DEVICE, e.what());
    }
  }

  void fail(nd_status code, const std::string &msg) {
    std::lock_guard<std::mutex> lk(mu_);
    if (code_ == ND_OK) {
      code_ = code;
      msg_ = msg;
    }
    failed_ = true;
    cv_.notify_all();
  }

  nd_ctx *ctx_;
  nd_kind kind_;
  std::vector<nd_graph *> todo_;
  std::vector<hipStream_t> streams_;
  std::vector<std::thread> threads_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::pair<nd_graph *, hipEvent_t>> done_;
  size_t next_ = 0, handed_ = 0;
  bool failed_ = false;
  nd_status code_ = ND_OK;
  std::string msg_;
};

}  // namespace

void prepare_many(nd_ctx *ctx, int32_t count, nd_graph *const *graphs,
                  nd_kind kind, hipStream_t s) {
  PrepPool pool(ctx, count, graphs, kind, s);
  nd_graph *g;
  hipEvent_t ev;
  while (pool.next(true, &g, &ev)) (void)hipEventDestroy(ev);
  pool.finish(s);
}

// Incidence entries the live graphs must hold before sweeps run while
// other graphs are still being prepared.  Shorter epochs would mostly add
// launches and polls beside the preparation threads' own (whose build
// phases are launch-bound), slowing them more than the overlap gains.
constexpr int64_t kOverlapWork = (int64_t)1 << 24;

// The batched decomposition.  Graphs not yet prepared are prepared by a
// PrepPool while the graphs already prepared are being swept (once their
// sweeps are long enough, kOverlapWork): each joins the batch of its tau
// width (16 or 32 bits; two batches, on streams of their own, when the
// graphs need both) as soon as it is ready.
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
  std::vector<bool> was(count);
  for (int i = 0; i < count; i++) {
    ND_REQUIRE(graphs[i] && graphs[i]->ctx == ctx, ND_ERR_INVALID,
               "graph %d is NULL or from another context", i);
    was[i] = graphs[i]->ks[kind].ready;
  }
  for (int i = 0; i < count; i++)  // outputs of graphs already prepared
    ND_REQUIRE(!was[i] || graphs[i]->ks[kind].nr == 0 || (kappas && kappas[i]),
               ND_ERR_INVALID, "kappas[%d] is NULL", i);
  std::unique_ptr<Batch> batches[2];  // 16-bit, 32-bit tau
  bool tuned[2] = {false, false};
  std::map<nd_graph *, Member *> member;
  struct Events {  // the call's timing events, released on every exit
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } evs;
  ND_HIP(hipEventCreate(&evs.a));
  ND_HIP(hipEventCreate(&evs.b));
  hipEvent_t a = evs.a, b = evs.b;
  ND_HIP(hipEventRecord(a, s));
  auto join = [&](nd_graph *g, hipEvent_t ready) {
    const int w = g->ks[kind].tau16 ? 0 : 1;
    if (!batches[w])
      batches[w] = std::make_unique<Batch>(ctx, kind, opts.mode, w == 0,
                                           opts.use_frontier != 0, s);
    if (ready) ND_HIP(hipStreamWaitEvent(batches[w]->stream(), ready, 0));
    member[g] = batches[w]->add(g, opts.max_iters, nullptr);
  };
  {
    PrepPool pool(ctx, count, graphs, kind, s);
    Phase sweep_phase("nd.batch.sweeps");
    for (int i = 0; i < count; i++)
      if (was[i] && !member.count(graphs[i])) join(graphs[i], nullptr);
    int chunk = 2;
    while (!pool.failed()) {
      auto live_work = [&] {
        int64_t w = 0;
        for (auto &bt : batches)
          if (bt)
            for (Member *m : bt->live()) w += std::max<int64_t>(m->g->ks[kind].P, 1);
        return w;
      };
      int64_t work = live_work();
      // newcomers; wait for one while the sweeps would be too short to
      // overlap the preparations usefully
      nd_graph *g;
      hipEvent_t ev;
      while (pool.next(work < kOverlapWork && !pool.finished(), &g, &ev)) {
        try {
          join(g, ev);
        } catch (...) {
          (void)hipEventDestroy(ev);
          throw;
        }
        (void)hipEventDestroy(ev);
        work = live_work();
      }
      if (work == 0) {
        if (pool.finished()) break;
        continue;
      }
      int ran[2] = {0, 0};
      for (int w = 0; w < 2; w++) {
        if (!batches[w] || batches[w]->live().empty()) continue;
        if (!tuned[w]) {  // its first epoch, or trial epochs on scratch state
          ran[w] = batches[w]->autotune();
          tuned[w] = true;
        } else {
          batches[w]->run_epochs(chunk);
          ran[w] = chunk;
        }
      }
      for (int w = 0; w < 2; w++)
        if (ran[w]) batches[w]->poll(ran[w]);
      chunk = std::min(chunk * 2, Batch::kGraphEpochs);
    }
    pool.finish(s);
  }
  for (auto &bt : batches)
    if (bt) {
      hipEvent_t d;
      ND_HIP(hipEventCreateWithFlags(&d, hipEventDisableTiming));
      ND_HIP(hipEventRecord(d, bt->stream()));
      ND_HIP(hipStreamWaitEvent(s, d, 0));
      (void)hipEventDestroy(d);
    }
  ND_HIP(hipEventRecord(b, s));
  ND_HIP(hipEventSynchronize(b));
  float ms_total = 0;
  ND_HIP(hipEventElapsedTime(&ms_total, a, b));
  nd_status out = ND_OK;
  for (int i = 0; i < count; i++) {
    const Member &m = *member.at(graphs[i]);
    const KindState &ks = graphs[i]->ks[kind];
    const Batch &bt = *batches[ks.tau16 ? 0 : 1];
    hipStream_t bs = bt.stream();
    StreamScope scope(bs);
    if (ks.nr > 0) {
      ND_REQUIRE(kappas && kappas[i], ND_ERR_INVALID, "kappas[%d] is NULL", i);
      if (on_device) {
        to_original(ks, bt.result_tau(m), bt.tau16() ? 2 : 4, kappas[i], bs);
      } else {
        DArr<int32_t> tmp(ctx->alloc, ks.nr);
        to_original(ks, bt.result_tau(m), bt.tau16() ? 2 : 4, tmp.p, bs);
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
      r.ms_prep = was[i] ? 0.0 : ks.ms_prep;
      r.ms_iterate = ms_total;  // shared by the whole batch
      r.max_sdegree = ks.max_ds;
      r.tau_bytes = bt.tau16() ? 2 : 4;
    }
    if (!m.converged) out = ND_ERR_NOT_CONVERGED;
  }
  for (auto &bt : batches)
    if (bt) {
      ND_HIP(hipStreamSynchronize(bt->stream()));
      hipEvent_t d;  // the caller's later work follows the output kernels
      ND_HIP(hipEventCreateWithFlags(&d, hipEventDisableTiming));
      ND_HIP(hipEventRecord(d, bt->stream()));
      ND_HIP(hipStreamWaitEvent(s, d, 0));
      (void)hipEventDestroy(d);
    }
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

extern "C" nd_status nd_prepare_many(nd_ctx *ctx, int32_t count,
                                     nd_graph *const *graphs, nd_kind kind,
                                     void *stream) {
  return guarded([&] {
    ND_REQUIRE(ctx, ND_ERR_INVALID, "ctx is NULL");
    ND_REQUIRE(count >= 0 && (count == 0 || graphs), ND_ERR_INVALID,
               "bad graph list");
    ND_REQUIRE(kind_valid(kind), ND_ERR_UNSUPPORTED, "unknown kind");
    for (int i = 0; i < count; i++)
      ND_REQUIRE(graphs[i] && graphs[i]->ctx == ctx, ND_ERR_INVALID,
                 "graph %d is NULL or from another context", i);
    ND_HIP(hipSetDevice(ctx->device));
    StreamScope scope((hipStream_t)stream);
    prepare_many(ctx, count, graphs, kind, (hipStream_t)stream);
  });
}
