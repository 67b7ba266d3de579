// sweep.hip -- one application of the update operator U to every r-clique
// (Section 3, Defn. of U; the parallel loop of Alg. 2 and Alg. 3):
//
//   rho(S,R)  = min over the k other r-cliques R' of S of tau(R')  (gather+min)
//   tau'(R)   = H({rho(S,R)} over the d_s(R) s-cliques S containing R)
//   changed  += (tau'(R) != tau(R))                         (convergence flag)
//
// r-cliques are in the internal numbering (grouped by bin), so each bin is a
// contiguous id range and the incidence lists are read in one sequential,
// coalesced stream; the tau reads are the random part.  tau is stored as
// uint16 when every d_s fits (then every tau does: tau <= d_s), halving the
// bytes of the gathered array.
//
// H is computed exactly with a cap c (Section 4.4 "can the current value be
// preserved" check, made exact):
//   * H(min(K,c)) = min(H(K), c) for any multiset K and any c >= 0, and
//     H(K) <= |K| = d_s(R), so with c = d_s(R) the cap never changes H.
//   * For the iterates of SND/AND, U tau(R) <= tau(R) (Theorem 1, and the same
//     argument for in-place sweeps, whose inputs only decrease), so c = tau(R)
//     is exact there too and keeps the work small.
//   * If #{rho >= c} >= c then H = c (the preserve check).  Otherwise H is
//     the largest x < c with #{rho >= x} >= x, found by binary search on x
//     with counts reduced across the lanes that hold the rho values.
//
// Mappings by S-degree bin:
//   d_s <= 256     G = 1/4/16/64 lanes per r-clique, 4 rho values per lane;
//                  a full sweep gathers each run of r-cliques flat first
//                  (one lane per incidence entry, minima to LDS), then
//                  computes H from LDS (sweep_flat)
//   257..2047      one wave per r-clique, 8 / 16 / 32 rho values per lane
//                  (257..512 / 513..1024 / 1025..2047: fewer registers, more
//                  waves in flight for the shorter lists)
//   >= 2048        one 256-thread workgroup per r-clique; LDS histogram of
//                  min(rho, c) in up to 16384 bins; for larger c the values
//                  are binned coarsely and the coarse bin holding H is refined
//                  with a second gather.
// SND reads tau_t and writes tau_{t+1} (double buffer, race free, so every
// iterate is deterministic).  AND reads and writes one array in place with
// relaxed workgroup-scope atomics: a value read may predate another
// workgroup's write in the same sweep but never the sweep's start, and
// writes only ever lower values (Section 4.2; see load_tau).
#include <algorithm>

#include "sweep_dev.h"

namespace nd {

namespace {

using namespace dev;

// The previous sweep's changed count (1 for the first sweep: not converged).
__device__ __forceinline__ unsigned long long prev_changed(const SweepArgs &a) {
  return a.prev != nullptr ? changed_sum(a.prev) : 1ull;
}

// Frontier state of this sweep (uniform over the launch): flags are read
// only if the previous sweep wrote them (and a.flags_unused is clear); this
// sweep notifies once the previous one changed few enough r-cliques, and
// keeps notifying after; the first sweep notifies only with a.notify_first.
__device__ __forceinline__ void frontier_mode(const SweepArgs &a,
                                              unsigned long long prev_changed,
                                              const uint8_t **act,
                                              uint8_t **act_next,
                                              const uint8_t **act_sum,
                                              uint8_t **sum_next) {
  *act_sum = nullptr;
  *sum_next = nullptr;
  if (a.fixed_set) {
    *act = a.act;
    *act_next = nullptr;
    return;
  }
  const bool flags_valid =
      !a.flags_unused && a.prev != nullptr && a.prev->notified;
  const bool notify =
      a.prev != nullptr
          ? (a.prev->notified || prev_changed <= a.notify_below)
          : a.notify_first != 0;
  *act = flags_valid ? a.act : nullptr;
  *act_next = notify ? a.act_next : nullptr;
  *act_sum = flags_valid ? a.act_sum : nullptr;
  *sum_next = notify ? a.act_sum_next : nullptr;
  if (a.sums_after != 0 && prev_changed >= a.sums_after)
    *sum_next = nullptr;  // k_group_sums writes them
  if (notify && blockIdx.x == 0 && threadIdx.x == 0) a.stats->notified = 1;
}

// Workgroup LDS for sweep_flat: the minima of one run's incidence entries
// and the run's list offsets (relative to its first entry).
constexpr int kFlatRun = 4096;  // incidence entries per run, at most
template <typename T>
struct FlatLds {
  T rho[kFlatRun];
  int32_t off[kFlatRun / 4 + 1];
  // sweep_flat_fr: per entry, the listed members holding the minimum
  uint8_t mask[kFlatRun];
};

// A full sweep (no flags read, none written) of a bin of G lanes per
// r-clique with d_s <= 4G.  The workgroup takes one contiguous share of the
// bin in runs of kFlatRun / (4G) r-cliques (at most kFlatRun incidence
// entries).  The run's entries are gathered flat: lane t takes entries t,
// t + 256, ..., so the id stream is read in order and coalesced, and the
// values gathered by a run's r-cliques -- which share vertices -- are
// reused from the CU's cache; the minima go to LDS.  Then G lanes per
// r-clique read their values back from LDS and compute H as update_regs
// does.  Counts are added to *n_ch / *n_ev (wave totals).
template <int K, int G, typename T, bool AND>
__device__ __forceinline__ void sweep_flat(const SweepArgs &a, int64_t lo,
                                           int64_t hi, int64_t block,
                                           int64_t nblocks, FlatLds<T> *lds,
                                           unsigned long long *n_ch,
                                           unsigned long long *n_ev) {
  constexpr int M = 4;
  constexpr int kRun = kFlatRun / (G * M);  // r-cliques per run
  constexpr int kPerPass = 256 / G;         // r-cliques per h-index pass
  const T *tin = (const T *)a.tau_in;
  T *tout = (T *)a.tau_out;
  const int t = threadIdx.x;
  const int sl = lane_id() % G;
  const int64_t nruns = (hi - lo + kRun - 1) / kRun;
  const int64_t per = (nruns + nblocks - 1) / nblocks;
  const int64_t q1 = std::min<int64_t>(nruns, (block + 1) * per);
  for (int64_t q = block * per; q < q1; q++) {  // uniform over the workgroup
    const int64_t r0 = lo + q * kRun;
    const int n = (int)std::min<int64_t>(kRun, hi - r0);
    const int64_t e0 = a.inc_off[r0];
    for (int i = t; i <= n; i += blockDim.x)
      lds->off[i] = (int32_t)(a.inc_off[r0 + i] - e0);
    __syncthreads();
    const int ne = lds->off[n];
    for (int e = t; e < ne; e += blockDim.x)
      lds->rho[e] = (T)gather_rho<K, T, AND>(a.inc_ids, e0 + e, tin);
    __syncthreads();
    for (int p = 0; p < n; p += kPerPass) {  // uniform over the workgroup
      const int i = p + t / G;
      const bool active = i < n;
      int32_t told = 0, c = 0;
      int b = 0, d = 0;
      if (active) {
        told = (int32_t)tin[r0 + i];
        b = lds->off[i];
        d = lds->off[i + 1] - b;
        c = a.cap_by_tau ? told : d;
      }
      int32_t rho[M];
#pragma unroll
      for (int m = 0; m < M; m++) {
        const int j = sl + m * G;
        rho[m] = j < d ? (int32_t)lds->rho[b + j] : -1;
      }
      const int cnt = count_ge<G, M>(rho, c);
      const int32_t h = cnt >= c ? c : hindex_search<G, M>(rho, c);
      const bool lead = sl == 0;
      const bool ch = active && h != told;
      if (active && lead) store_tau<T, AND>(tout + r0 + i, h, ch);
      *n_ch += __popcll(ballot(lead && ch));
      *n_ev += __popcll(ballot(lead && active));
    }
    __syncthreads();  // the next run reuses the LDS
  }
}

// The full SND sweep that notifies (Section 4.3: the first sweep after the
// frontier switches on, or every sweep while active counts are taken), in
// the same runs as sweep_flat: the flat gather also keeps which members hold
// each minimum, and the subgroups write, self-activate on a change and
// notify through the kept minima (notify_kept), as update_regs does.
template <int K, int G, typename T>
__device__ __forceinline__ void sweep_flat_fr(const SweepArgs &a, int64_t lo,
                                              int64_t hi, int64_t block,
                                              int64_t nblocks, uint8_t *act_next,
                                              uint8_t *sum_next,
                                              FlatLds<T> *lds,
                                              unsigned long long *n_ch,
                                              unsigned long long *n_ev) {
  constexpr int M = 4;
  constexpr int kRun = kFlatRun / (G * M);
  constexpr int kPerPass = 256 / G;
  constexpr int kMaskWords = (K * M + 31) / 32;
  const T *tin = (const T *)a.tau_in;
  T *tout = (T *)a.tau_out;
  const uint8_t next = a.stamp == 255 ? 1 : a.stamp + 1;
  const int t = threadIdx.x;
  const int sl = lane_id() % G;
  const int64_t nruns = (hi - lo + kRun - 1) / kRun;
  const int64_t per = (nruns + nblocks - 1) / nblocks;
  const int64_t q1 = std::min<int64_t>(nruns, (block + 1) * per);
  for (int64_t q = block * per; q < q1; q++) {  // uniform over the workgroup
    const int64_t r0 = lo + q * kRun;
    const int n = (int)std::min<int64_t>(kRun, hi - r0);
    const int64_t e0 = a.inc_off[r0];
    for (int i = t; i <= n; i += blockDim.x)
      lds->off[i] = (int32_t)(a.inc_off[r0 + i] - e0);
    __syncthreads();
    const int ne = lds->off[n];
    for (int e = t; e < ne; e += blockDim.x) {
      uint32_t arg = 1;
      int32_t r;
      if constexpr (K > 1)
        r = gather_rho_arg<K, T>(a.inc_ids, e0 + e, tin, &arg);
      else
        r = gather_rho<K, T, false>(a.inc_ids, e0 + e, tin);
      lds->rho[e] = (T)r;
      lds->mask[e] = (uint8_t)arg;
    }
    __syncthreads();
    for (int p = 0; p < n; p += kPerPass) {  // uniform over the workgroup
      const int i = p + t / G;
      const bool active = i < n;
      int32_t told = 0, c = 0;
      int b = 0, d = 0;
      if (active) {
        b = lds->off[i];
        d = lds->off[i + 1] - b;
        told = (int32_t)tin[r0 + i];
        c = a.cap_by_tau ? told : d;
      }
      int32_t rho[M];
      uint32_t amask[kMaskWords];
#pragma unroll
      for (int w = 0; w < kMaskWords; w++) amask[w] = 0;
#pragma unroll
      for (int m = 0; m < M; m++) {
        const int j = sl + m * G;
        const bool in = j < d;
        rho[m] = in ? (int32_t)lds->rho[b + j] : -1;
        if (K > 1 && in) {
          const uint32_t am = lds->mask[b + j];
#pragma unroll
          for (int x = 0; x < K; x++) {
            const int bit = m * K + x;
            amask[bit >> 5] |= ((am >> x) & 1u) << (bit & 31);
          }
        }
      }
      const int cnt = count_ge<G, M>(rho, c);
      const int32_t h = cnt >= c ? c : hindex_search<G, M>(rho, c);
      const bool lead = sl == 0;
      const bool ch = active && h != told;
      const int64_t R = r0 + i;
      if (active && lead) store_tau<T, false>(tout + R, h, ch);
      if (ch) {
        if (lead) {
          act_next[R] = next;
          if (sum_next) sum_next[R >> kGroupShift] = next;
        }
        notify_kept<K, G, M>(a.inc_ids, e0 + b, d, sl, rho, amask, told, h,
                             act_next, next, sum_next);
      }
      *n_ch += __popcll(ballot(lead && ch));
      *n_ev += __popcll(ballot(lead && active));
    }
    __syncthreads();  // the next run reuses the LDS
  }
}

// One bin [lo, hi) of G lanes per r-clique with M values per lane, swept by
// the workgroups block .. of nblocks (a launch of its own, or a block range
// of k_sweep_small).  With `flat` LDS (small bins), a full sweep that
// notifies nobody runs as sweep_flat and a full SND sweep that notifies as
// sweep_flat_fr.  Sweeps that read flags find their flagged r-cliques per
// wave (sweep_sparse): run-based variants of those (marking, or compacting
// the flagged r-cliques of each run in LDS) measured no faster.
template <int K, int G, int M, typename T, bool AND, bool FR>
__device__ __forceinline__ void sweep_bin(const SweepArgs &a, int64_t lo,
                                          int64_t hi, int64_t block,
                                          int64_t nblocks, const uint8_t *act,
                                          uint8_t *act_next,
                                          const uint8_t *act_sum,
                                          uint8_t *sum_next,
                                          FlatLds<T> *flat = nullptr) {
  constexpr int kPerWave = kWave / G;
  const int64_t wave = (block * blockDim.x + threadIdx.x) / kWave;
  const int64_t waves = nblocks * (blockDim.x / kWave);
  const int sub = lane_id() / G;
  const T *tin = (const T *)a.tau_in;
  T *tout = (T *)a.tau_out;
  unsigned long long n_ch = 0, n_ev = 0;  // wave totals, from ballots
  constexpr bool kFlatFr = FR && !AND && M == 4;
  if (kFlatFr && flat != nullptr && act == nullptr && act_next != nullptr) {
    if constexpr (kFlatFr)
      sweep_flat_fr<K, G, T>(a, lo, hi, block, nblocks, act_next, sum_next,
                             flat, &n_ch, &n_ev);
  } else if (FR && act != nullptr) {
    sweep_sparse<K, G, M, T, AND>(a.inc_off, a.inc_ids, tin, tout, a.cap_by_tau,
                                  lo, hi, wave, waves, act, act_next, a.stamp,
                                  &n_ch, &n_ev, act_sum, sum_next);
  } else if (M == 4 && flat != nullptr && act == nullptr && act_next == nullptr) {
    if constexpr (M == 4)
      sweep_flat<K, G, T, AND>(a, lo, hi, block, nblocks, flat, &n_ch, &n_ev);
  } else {
    // Each workgroup takes one contiguous share of the bin (a multiple of
    // its waves' step), its waves striding inside it: the r-cliques of a
    // share have neighbouring ids and share vertices, so the values they
    // gather are reused from the CU's cache (measured against waves striding
    // over the whole bin: 11% less time per full (3,4) sweep of the
    // block-model workload, the same on the Chung-Lu ones).
    const int64_t wib = threadIdx.x / kWave;
    const int64_t step = (int64_t)(blockDim.x / kWave) * kPerWave;
    int64_t run = (hi - lo + nblocks - 1) / nblocks;
    run = (run + step - 1) / step * step;
    const int64_t c0 = lo + block * run;
    const int64_t c1 = std::min<int64_t>(hi, c0 + run);
    for (int64_t base = c0 + wib * kPerWave; base < c1; base += step) {
      const int64_t R = base + sub;
      bool ev;
      const bool changed = update_regs<K, G, M, T, AND, FR>(
          a.inc_off, a.inc_ids, tin, tout, a.cap_by_tau, R, R < c1, act,
          act_next, a.stamp, &ev, sum_next);
      n_ch += __popcll(ballot(changed));
      n_ev += __popcll(ballot(ev));
    }
  }
  stat_add_counts(a.stats, n_ch, n_ev);
}

template <int K, int G, int M, typename T, bool AND, bool FR>
__global__ __launch_bounds__(256) void k_sweep_regs(SweepArgs a, int64_t lo,
                                                    int64_t hi) {
  const unsigned long long pc = prev_changed(a);
  if (pc == 0) return;  // converged: a sweep queued past the end
  const uint8_t *act = nullptr, *act_sum = nullptr;
  uint8_t *act_next = nullptr, *sum_next = nullptr;
  if (FR) frontier_mode(a, pc, &act, &act_next, &act_sum, &sum_next);
  sweep_bin<K, G, M, T, AND, FR>(a, lo, hi, blockIdx.x, gridDim.x, act,
                                 act_next, act_sum, sum_next);
}

// The bins whose lanes hold at most 16 values (513..1024 down to 1..4) in
// one launch: their registers are alike enough that one occupancy suits
// all, a sparse sweep pays one launch for them instead of six, and the bins
// run side by side instead of each draining the chip before the next starts.
// Bin i (kFirstSmall + i) gets the workgroups [first[i], first[i+1]).
struct SmallBins {
  int64_t lo[kNumSmall], hi[kNumSmall];
  unsigned first[kNumSmall + 1];
};

template <int K, typename T, bool AND, bool FR>
__global__ __launch_bounds__(256) void k_sweep_small(SweepArgs a, SmallBins sb) {
  __shared__ FlatLds<T> flat;
  const unsigned long long pc = prev_changed(a);
  if (pc == 0) return;
  const uint8_t *act = nullptr, *act_sum = nullptr;
  uint8_t *act_next = nullptr, *sum_next = nullptr;
  if (FR) frontier_mode(a, pc, &act, &act_next, &act_sum, &sum_next);
  int i = 0;
  while (i + 1 < kNumSmall && blockIdx.x >= sb.first[i + 1]) i++;
  const int64_t block = blockIdx.x - sb.first[i];
  const int64_t nblocks = sb.first[i + 1] - sb.first[i];
  switch (kFirstSmall + i) {
    case kBinWave16:
      sweep_bin<K, 64, 16, T, AND, FR>(a, sb.lo[i], sb.hi[i], block, nblocks,
                                       act, act_next, act_sum, sum_next);
      break;
    case kBinWave8:
      sweep_bin<K, 64, 8, T, AND, FR>(a, sb.lo[i], sb.hi[i], block, nblocks,
                                      act, act_next, act_sum, sum_next);
      break;
    case kBinG64:
      sweep_bin<K, 64, 4, T, AND, FR>(a, sb.lo[i], sb.hi[i], block, nblocks,
                                      act, act_next, act_sum, sum_next, &flat);
      break;
    case kBinG16:
      sweep_bin<K, 16, 4, T, AND, FR>(a, sb.lo[i], sb.hi[i], block, nblocks,
                                      act, act_next, act_sum, sum_next, &flat);
      break;
    case kBinG4:
      sweep_bin<K, 4, 4, T, AND, FR>(a, sb.lo[i], sb.hi[i], block, nblocks,
                                     act, act_next, act_sum, sum_next, &flat);
      break;
    default:  // kBinG1
      sweep_bin<K, 1, 4, T, AND, FR>(a, sb.lo[i], sb.hi[i], block, nblocks,
                                     act, act_next, act_sum, sum_next, &flat);
      break;
  }
}

template <int K, typename T, bool AND, bool FR>
__global__ __launch_bounds__(kBlockThreads) void k_sweep_block(SweepArgs a,
                                                               int64_t lo,
                                                               int64_t hi) {
  __shared__ int32_t hist[kBlockHistBins];
  const unsigned long long pc = prev_changed(a);
  if (pc == 0) return;  // converged: a sweep queued past the end
  const uint8_t *act = nullptr, *act_sum = nullptr;
  uint8_t *act_next = nullptr, *sum_next = nullptr;
  if (FR) frontier_mode(a, pc, &act, &act_next, &act_sum, &sum_next);
  for (int64_t R = lo + blockIdx.x; R < hi; R += gridDim.x) {
    bool ev;
    const bool changed = update_block<K, T, AND, FR>(
        a.inc_off, a.inc_ids, (const T *)a.tau_in, (T *)a.tau_out,
        a.cap_by_tau, R, hist, act, act_next, a.stamp, &ev, sum_next);
    stat_add(a.stats, changed, ev);
  }
}

template <typename T>
__global__ void k_zero_range(T *__restrict__ tau, int64_t lo, int64_t hi) {
  const int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < hi) tau[i] = 0;
}

// Blocks for a bin of n r-cliques at G lanes each, at most a.grid_cap, and
// never more than grid_stride allows (the kernels stride over the rest).
inline unsigned regs_grid(const SweepArgs &a, int64_t n, int G) {
  const int64_t blocks = grid_stride(n, G);
  return (unsigned)(a.grid_cap > 0 ? std::min<int64_t>(blocks, a.grid_cap)
                                   : blocks);
}

template <int K, typename T, bool AND, bool FR>
void launch_bins(const KindState &ks, const SweepArgs &a, hipStream_t s) {
  for (int bin = kBinBlock; bin < kFirstSmall; bin++) {
    const int64_t lo = ks.bin_lo[bin], hi = ks.bin_hi[bin], n = hi - lo;
    if (n == 0) continue;
    switch (bin) {
      case kBinWave:
        k_sweep_regs<K, 64, 32, T, AND, FR><<<regs_grid(a, n, 64), 256, 0, s>>>(a, lo, hi);
        break;
      default: {
        const unsigned grid = (unsigned)(n < 65536 ? n : 65536);
        k_sweep_block<K, T, AND, FR><<<grid, kBlockThreads, 0, s>>>(a, lo, hi);
        break;
      }
    }
    ND_LAUNCHED();
  }
  constexpr int kLanes[kNumSmall] = {64, 64, 64, 16, 4, 1};  // G of each small bin
  SmallBins sb{};
  int64_t total = 0;
  for (int i = 0; i < kNumSmall; i++) {
    const int bin = kFirstSmall + i;
    sb.lo[i] = ks.bin_lo[bin];
    sb.hi[i] = ks.bin_hi[bin];
    sb.first[i] = (unsigned)total;
    if (sb.hi[i] > sb.lo[i]) total += regs_grid(a, sb.hi[i] - sb.lo[i], kLanes[i]);
  }
  sb.first[kNumSmall] = (unsigned)total;
  if (total > 0) {
    k_sweep_small<K, T, AND, FR><<<(unsigned)total, 256, 0, s>>>(a, sb);
    ND_LAUNCHED();
  }
}

template <int K, typename T, bool AND>
void launch_fr(const KindState &ks, const SweepArgs &a, hipStream_t s) {
  if (a.act)
    launch_bins<K, T, AND, true>(ks, a, s);
  else
    launch_bins<K, T, AND, false>(ks, a, s);
}

template <typename T>
void launch_typed(const KindState &ks, const SweepArgs &a, bool and_mode,
                  hipStream_t s) {
  if (!a.cap_by_tau) {
    // plain U on an arbitrary tau: r-cliques in no s-clique get H({}) = 0
    const int64_t lo = ks.bin_lo[kBinZero], hi = ks.bin_hi[kBinZero];
    if (hi > lo) {
      k_zero_range<T><<<grid_for(hi - lo, 256), 256, 0, s>>>((T *)a.tau_out, lo, hi);
      ND_LAUNCHED();
    }
  }
  switch (ks.k * 2 + (and_mode ? 1 : 0)) {
    case 2: launch_fr<1, T, false>(ks, a, s); break;
    case 3: launch_fr<1, T, true>(ks, a, s); break;
    case 4: launch_fr<2, T, false>(ks, a, s); break;
    case 5: launch_fr<2, T, true>(ks, a, s); break;
    case 6: launch_fr<3, T, false>(ks, a, s); break;
    case 7: launch_fr<3, T, true>(ks, a, s); break;
    case 10: launch_fr<5, T, false>(ks, a, s); break;
    case 11: launch_fr<5, T, true>(ks, a, s); break;
    default:
      ND_REQUIRE(false, ND_ERR_UNSUPPORTED, "no sweep kernel for k=%d", ks.k);
  }
}

// The group summaries of the flags a dense notifying sweep wrote without
// them: a thread per group of 64 flags (four 16-byte loads), striding, which
// stores the next stamp into the group's summary when any of its flags holds
// it.  Runs only when the sweep it follows took that path (the same test as
// frontier_mode, on the same counters); a small grid keeps the launches that
// find nothing to do cheap.
constexpr int kGroupSumsBlocks = 1024;

__global__ __launch_bounds__(256) void k_group_sums(SweepArgs a, int64_t nr) {
  const unsigned long long pc = prev_changed(a);
  if (pc == 0 || a.sums_after == 0 || pc < a.sums_after) return;
  const bool notify = a.prev != nullptr
                          ? (a.prev->notified || pc <= a.notify_below)
                          : a.notify_first != 0;
  if (!notify) return;
  const uint8_t next = a.stamp == 255 ? 1 : a.stamp + 1;
  const int64_t ng = (nr + (1 << kGroupShift) - 1) >> kGroupShift;
  const uint32_t pat = 0x01010101u * next;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f0 = g << kGroupShift;
    bool any = false;
    if (f0 + (1 << kGroupShift) <= nr) {
      const uint4 *p = reinterpret_cast<const uint4 *>(a.act_next + f0);
#pragma unroll
      for (int v = 0; v < (1 << kGroupShift) / 16; v++) {
        const uint4 w = p[v];
        const uint32_t x[4] = {w.x ^ pat, w.y ^ pat, w.z ^ pat, w.w ^ pat};
#pragma unroll
        for (int c = 0; c < 4; c++)  // a zero byte: a flag equal to next
          any |= ((x[c] - 0x01010101u) & ~x[c] & 0x80808080u) != 0;
      }
    } else {
      for (int64_t f = f0; f < nr; f++) any |= a.act_next[f] == next;
    }
    if (any) a.act_sum_next[g] = next;
  }
}

}  // namespace

void launch_group_sums(const KindState &ks, const SweepArgs &a, hipStream_t s) {
  if (a.sums_after == 0 || a.act_next == nullptr || a.act_sum_next == nullptr ||
      ks.nr == 0)
    return;
  const int64_t ng = (ks.nr + (1 << dev::kGroupShift) - 1) >> dev::kGroupShift;
  const unsigned grid =
      (unsigned)std::min<int64_t>(grid_for(ng, 256), kGroupSumsBlocks);
  k_group_sums<<<grid, 256, 0, s>>>(a, ks.nr);
  ND_LAUNCHED();
}

void launch_sweep(const KindState &ks, const SweepArgs &a, bool and_mode,
                  hipStream_t s) {
  if (ks.tau_bytes == 1)
    launch_typed<uint8_t>(ks, a, and_mode, s);
  else if (ks.tau_bytes == 2)
    launch_typed<uint16_t>(ks, a, and_mode, s);
  else
    launch_typed<int32_t>(ks, a, and_mode, s);
}

}  // namespace nd
