// batch.h -- the multi-graph sweep engine shared by nd_batch_decompose and
// the server.  Internal header.
#pragma once

#include <memory>
#include <vector>

#include "internal.h"

namespace nd {

constexpr int kBatchRing = 32;    // per-graph sweep counters kept
constexpr int kPollMax = 16;      // epochs between host polls, at most

// Device descriptor of one graph in a batch.
struct BGraph {
  const int64_t *inc_off;
  const int32_t *inc_ids;
  void *tau[2];        // sweep number t reads tau[t & 1] (SND)
  SweepStats *ring;    // counters of sweep t at ring[t % kBatchRing]
  int64_t t0;          // epoch at which the graph joined
  int64_t max_local;   // sweeps allowed
  uint8_t *act[2];     // frontier stamps: sweep t reads act[t & 1]
  uint8_t *act_sum[2]; // one stamp per 64 r-cliques, set with any of their flags
  unsigned long long notify_below;  // start notifying at <= this many changes
};

// A run of r-cliques of one graph and one sweep bin.
struct BTile {
  int32_t g;
  int32_t type;  // SweepBin
  int64_t lo, hi;
};

struct BHub {  // one r-clique with d_s >= 2048
  int32_t g;
  int32_t pad;
  int64_t R;
};

// Device-resident launch state: every kernel of an epoch reads it, so a
// chunk of epochs built as a HIP graph stays valid when the tables change.
struct BState {
  int64_t epoch;
  int32_t ntiles;
  int32_t nhubs;
  int32_t ng;
  int32_t nwide;  // tiles [0, nwide): 16 or 32 values per lane (k_batch_sweep<WIDE>)
};

// Tile length: an epoch is cut into about grid * tiles_per_group tiles of
// about equal work (one workgroup each).
struct BatchConfig {
  int grid = 2048;
  int tiles_per_group = 8;
};

// One graph taking part in a batch.
struct Member {
  nd_graph *g = nullptr;
  void *user = nullptr;
  int64_t t0 = 0;
  int64_t max_local = 0;
  int64_t sweeps = 0;
  bool converged = false;
  bool finished = false;
  int slot = -1;          // index in the device descriptor table
  int64_t ntiles = 0;     // tiles it contributes
  DArr<uint8_t> tau0, tau1;
  DArr<uint8_t> act0, act1;  // frontier batches only
  DArr<uint8_t> sum0, sum1;  // their group summaries (one per 64 r-cliques)
  DArr<SweepStats> ring;
};

class Batch {
 public:
  static constexpr int kGraphEpochs = 8;  // epochs per HIP graph

  // Work is issued on a private stream ordered after `caller`.
  Batch(nd_ctx *ctx, nd_kind kind, nd_mode mode, bool tau16, bool frontier,
        hipStream_t caller);
  ~Batch();
  Batch(const Batch &) = delete;
  Batch &operator=(const Batch &) = delete;

  // Add a prepared graph; it starts at the current epoch.
  Member *add(nd_graph *g, int32_t max_iters, void *user);
  // Drop finished members (their memory is released by the caller).
  std::vector<std::unique_ptr<Member>> take_finished();
  void run_epochs(int count);
  // Update sweeps/converged/finished of every member from the device.
  void poll(int epochs_run);
  // Pick tile and grid sizes (cached per shape).  Returns the number of
  // real epochs it ran (0 or 1), which the caller then polls.
  int autotune();
  static constexpr float kTuneSkipMs = 2.0f;
  const void *result_tau(const Member &m) const;
  bool tau16() const { return tau16_; }
  bool frontier() const { return frontier_; }
  nd_kind kind() const { return kind_; }
  nd_mode mode() const { return mode_; }
  hipStream_t stream() const { return s_; }
  size_t size() const { return members_.size(); }
  // Epochs run so far (the next epoch's number).
  int64_t epoch() const { return epoch_; }
  // Members still being swept (not finished).
  std::vector<Member *> live() const {
    std::vector<Member *> v;
    for (auto &m : members_)
      if (!m->finished) v.push_back(m.get());
    return v;
  }
  bool use_graph = true;
  float tuned_ms = 0;
  BatchConfig config() const { return cfg_; }
  static BatchConfig default_config(nd_ctx *ctx);

 private:
  void init_member_tau(Member &m);
  void rebuild();
  void set_config(const BatchConfig &c);
  void launch_epoch();
  void build_graph();
  void drop_graph();

  nd_ctx *ctx_;
  nd_kind kind_;
  nd_mode mode_;
  bool tau16_;
  bool frontier_;
  int notify_div_ = 4;
  hipStream_t s_ = nullptr;
  BatchConfig cfg_;
  std::vector<std::unique_ptr<Member>> members_;
  DArr<BGraph> gs_;
  DArr<BTile> tiles_;
  DArr<BHub> hubs_;
  DArr<BState> state_;
  DArr<unsigned long long> poll_buf_;
  int64_t gs_cap_ = 0, tiles_cap_ = 0, hubs_cap_ = 0, poll_cap_ = 0;
  int64_t wide_grid_ = 0, narrow_grid_ = 0;  // grids of the two tile kernels
  int ntiles_ = 0, nhubs_ = 0, ng_ = 0, nwide_ = 0;
  int64_t work_ = 0;
  int64_t epoch_ = 0;
  int64_t dead_tiles_ = 0;  // tiles of finished members still in the table
  bool dirty_ = true;
  hipGraphExec_t graph_exec_ = nullptr;
};

}  // namespace nd
