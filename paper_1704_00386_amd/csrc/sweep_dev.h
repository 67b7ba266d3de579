// sweep_dev.h -- device routines of one h-index update, shared by the
// single-graph sweep kernels (sweep.hip) and the batched tile kernel
// (batch.hip).  See sweep.hip for the method and the exactness argument.
#pragma once

#include "internal.h"

namespace nd {
namespace dev {

constexpr int kBlockThreads = 256;
// Frontier group summaries: one stamp per 64 consecutive r-cliques, set
// whenever a flag of the group is (see sweep_sparse).
constexpr int kGroupShift = 6;
constexpr int kBlockHistBins = 16384;  // 64 KiB of LDS

// AND reads and writes tau in place.  Reads and writes are relaxed atomics
// at workgroup scope: they may be served by (and stay in) this CU's L1 and
// this XCD's L2, which hold only values of the current launch (caches are
// made coherent at every kernel boundary), so a value read may be older than
// the latest write but never older than the sweep's start.  That keeps AND
// exact: values only fall, every value read lies between kappa and the
// previous iterate, so kappa <= AND_t <= SND_t still holds (H is monotone),
// and a sweep that changes nothing read only unchanged values, i.e. it
// certifies a fixed point.  Each value has one writer (the r-clique's own
// subgroup), so no write is lost.
template <typename T, bool AND>
__device__ __forceinline__ int32_t load_tau(const T *p) {
  if constexpr (AND) {
    return (int32_t)__hip_atomic_load(p, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
  } else {
    return (int32_t)*p;
  }
}

template <typename T, bool AND>
__device__ __forceinline__ void store_tau(T *p, int32_t h, bool changed) {
  if constexpr (AND) {
    if (changed)
      __hip_atomic_store(p, (T)h, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
  } else {
    *p = (T)h;
  }
}

// rho for the s-clique j of the incidence list (k = K ids per s-clique).
template <int K, typename T, bool AND>
__device__ __forceinline__ int32_t gather_rho(const int32_t *__restrict__ ids,
                                              int64_t j, const T *tau) {
  if constexpr (K == 1) {
    return load_tau<T, AND>(tau + ids[j]);
  } else if constexpr (K == 2) {
    const int2 p = *reinterpret_cast<const int2 *>(ids + 2 * j);
    return min(load_tau<T, AND>(tau + p.x), load_tau<T, AND>(tau + p.y));
  } else if constexpr (K == 3) {
    const int32_t *q = ids + 3 * j;
    const int32_t x = q[0], y = q[1], z = q[2];
    return min(min(load_tau<T, AND>(tau + x), load_tau<T, AND>(tau + y)),
               load_tau<T, AND>(tau + z));
  } else {
    const int32_t *q = ids + (int64_t)K * j;
    int32_t id[K];
#pragma unroll
    for (int x = 0; x < K; x++) id[x] = q[x];
    int32_t v = load_tau<T, AND>(tau + id[0]);
#pragma unroll
    for (int x = 1; x < K; x++) v = min(v, load_tau<T, AND>(tau + id[x]));
    return v;
  }
}

// gather_rho for SND with the frontier: also the members of the s-clique
// that hold the minimum (bit x set when the x-th listed id has tau = rho).
template <int K, typename T>
__device__ __forceinline__ int32_t gather_rho_arg(const int32_t *__restrict__ ids,
                                                  int64_t j, const T *tau,
                                                  uint32_t *arg) {
  int32_t v[K];
  if constexpr (K == 2) {
    const int2 p = *reinterpret_cast<const int2 *>(ids + 2 * j);
    v[0] = load_tau<T, false>(tau + p.x);
    v[1] = load_tau<T, false>(tau + p.y);
  } else {
    const int32_t *q = ids + (int64_t)K * j;
#pragma unroll
    for (int x = 0; x < K; x++) v[x] = load_tau<T, false>(tau + q[x]);
  }
  int32_t r = v[0];
#pragma unroll
  for (int x = 1; x < K; x++) r = min(r, v[x]);
  uint32_t a = 0;
#pragma unroll
  for (int x = 0; x < K; x++) a |= (uint32_t)(v[x] == r) << x;
  *arg = a;
  return r;
}

template <int G>
__device__ __forceinline__ int subgroup_sum(int x) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, G);
  return x;
}

// Add this wave's changed / recomputed r-cliques to the sweep's counters
// (one part per workgroup-and-wave hash, see SweepStats).
__device__ __forceinline__ void stat_add(SweepStats *st, bool changed,
                                         bool evald) {
  const uint64_t mc = ballot(changed), me = ballot(evald);
  if (lane_id() == 0 && (mc | me)) {
    StatPart &p = st->part[(blockIdx.x + threadIdx.x / kWave) % kStatParts];
    if (mc) atomicAdd(&p.changed, (unsigned long long)__popcll(mc));
    if (me) atomicAdd(&p.evaluated, (unsigned long long)__popcll(me));
  }
}

// Add wave-wide totals (the same on every lane, summed from ballots) to the
// sweep's counters: one atomic per wave and counter.
__device__ __forceinline__ void stat_add_counts(SweepStats *st,
                                                unsigned long long ch,
                                                unsigned long long ev) {
  if (lane_id() == 0 && (ch | ev)) {
    StatPart &p = st->part[(blockIdx.x + threadIdx.x / kWave) % kStatParts];
    if (ch) atomicAdd(&p.changed, ch);
    if (ev) atomicAdd(&p.evaluated, ev);
  }
}

// Total changed count of a finished sweep.  Every lane reads the same 16
// words (uniform addresses: scalar or broadcast loads), which costs far less
// at every wave's start than a cross-lane reduction.
__device__ __forceinline__ unsigned long long changed_sum(const SweepStats *st) {
  unsigned long long v = 0;
#pragma unroll
  for (int q = 0; q < kStatParts; q++) v += st->part[q].changed;
  return v;
}

// How many lanes of this lane's G-lane subgroup have p set: one wave ballot
// and a popcount (scalar for G = 64), no cross-lane data movement.
template <int G>
__device__ __forceinline__ int subgroup_count(bool p) {
  if constexpr (G == 1) {
    return p ? 1 : 0;
  } else {
    const uint64_t b = ballot(p);
    if constexpr (G == 64) {
      return __popcll(b);
    } else {
      const int sub = lane_id() / G;
      return __popcll((b >> (sub * G)) & (((uint64_t)1 << G) - 1));
    }
  }
}

// #{rho >= x} over the subgroup (G lanes x M values each).
template <int G, int M>
__device__ __forceinline__ int count_ge(const int32_t (&rho)[M], int32_t x) {
  int n = 0;
#pragma unroll
  for (int m = 0; m < M; m++) n += subgroup_count<G>(rho[m] >= x);
  return n;
}

// Largest x in [0, c-1] with #{rho >= x} >= x, given that x = 0 satisfies it;
// G lanes of a subgroup each hold M values (absent values are -1).  Binary
// search; every probe is M ballots.
template <int G, int M>
__device__ __forceinline__ int32_t hindex_search(const int32_t (&rho)[M],
                                                 int32_t c) {
  int32_t lo = 0, hi = c - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (count_ge<G, M>(rho, mid) >= mid)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Notification of Section 4.3: R changed from told to h.  A neighbour R'
// (another r-clique of an s-clique S containing R) can change at the next
// sweep only if some rho(S,R') falls from at least its next cap
// c' = tau_{t+1}(R') to below it.  Through S that needs rho_t(S,R') >= c' > h,
// i.e. both
//   h < tau(R')                 (tau_t(R') >= c'), and
//   h <= tau(Q) for every other member Q of S besides R and R'
// (rho_t(S,R') is a minimum over them and R).  In place (AND) the values read
// may already be newer; of several members of S that fell in one sweep, the
// one with the lowest new value still passes the test (<= keeps ties), so the
// s-clique is never lost.  SND reads tau_t exactly and self-activates every R
// that changed, so it only has to reach the R' that keep their value through
// sweep t+1: for those c' = tau_t(R'), and rho_t(S,R') >= c' also needs
// told >= c' and tau_t(Q) >= c' for the other members.  SND marks R' when
//   h < tau_t(R') <= told  and  tau_t(Q) >= tau_t(R') for every other Q,
// which keeps every R' that can change, so the iterates are those of full
// sweeps.  Byte stores of the same stamp race harmlessly.
template <int K, typename T, bool AND>
__device__ __forceinline__ void notify(const int32_t *__restrict__ ids,
                                       int64_t b, int64_t d, int first,
                                       int stride, int32_t told, int32_t h,
                                       const T *tau, uint8_t *act_next,
                                       uint8_t stamp_next, uint8_t *sum_next) {
  for (int64_t j = first; j < d; j += stride) {
    const int32_t *q = ids + K * (b + j);
    int32_t r[K], v[K];
#pragma unroll
    for (int x = 0; x < K; x++) {
      r[x] = q[x];
      v[x] = load_tau<T, AND>(tau + r[x]);
    }
#pragma unroll
    for (int x = 0; x < K; x++) {
      bool others_ok = true;
#pragma unroll
      for (int y = 0; y < K; y++)
        if (y != x) others_ok &= AND ? h <= v[y] : v[x] <= v[y];
      if (h < v[x] && (AND || v[x] <= told) && others_ok) {
        act_next[r[x]] = stamp_next;
        if (sum_next) sum_next[r[x] >> kGroupShift] = stamp_next;
      }
    }
  }
}

// The SND test of notify() from the values the update already gathered: R'
// passes it exactly when it holds the minimum rho of S and h < rho <= told,
// so the members to mark are those of the slots with rho in (h, told] whose
// bit is set in the argmin mask (bit m*K + x for slot m, member x; K = 1
// needs no mask).  Only their ids are read again, no tau.
template <int K, int G, int M>
__device__ __forceinline__ void notify_kept(const int32_t *__restrict__ ids,
                                            int64_t b, int64_t d, int sl,
                                            const int32_t *rho,
                                            const uint32_t *amask, int32_t told,
                                            int32_t h, uint8_t *act_next,
                                            uint8_t stamp_next,
                                            uint8_t *sum_next) {
#pragma unroll
  for (int m = 0; m < M; m++) {
    const int64_t j = sl + (int64_t)m * G;
    if (j < d && h < rho[m] && rho[m] <= told) {
      const int32_t *q = ids + K * (b + j);
#pragma unroll
      for (int x = 0; x < K; x++) {
        const int bit = m * K + x;
        if (K == 1 || ((amask[bit >> 5] >> (bit & 31)) & 1u)) {
          const int32_t r = q[x];
          act_next[r] = stamp_next;
          if (sum_next) sum_next[r >> kGroupShift] = stamp_next;
        }
      }
    }
  }
}

// The same test for lanes holding many values (no argmin mask kept): only the
// slots with rho in (h, told] read their members' tau again.
template <int K, int G, int M, typename T>
__device__ __forceinline__ void notify_slots(const int32_t *__restrict__ ids,
                                             int64_t b, int64_t d, int sl,
                                             const int32_t *rho, int32_t told,
                                             int32_t h, const T *tau,
                                             uint8_t *act_next,
                                             uint8_t stamp_next,
                                             uint8_t *sum_next) {
#pragma unroll
  for (int m = 0; m < M; m++) {
    const int64_t j = sl + (int64_t)m * G;
    if (j < d && h < rho[m] && rho[m] <= told) {
      const int32_t *q = ids + K * (b + j);
#pragma unroll
      for (int x = 0; x < K; x++) {
        const int32_t r = q[x];
        if (K == 1 || load_tau<T, false>(tau + r) == rho[m]) {
          act_next[r] = stamp_next;
          if (sum_next) sum_next[r >> kGroupShift] = stamp_next;
        }
      }
    }
  }
}

// Bit position of the t-th set bit (t counted from 0) of m; t < popc(m).
// Binary lifting: the largest p with popc(m below bit p) <= t is that bit.
__device__ __forceinline__ int nth_set_bit(uint64_t m, int t) {
  int p = 0;
#pragma unroll
  for (int w = 32; w > 0; w >>= 1) {
    const uint64_t below = m & ((((uint64_t)1) << (p + w)) - 1);
    if (__popcll(below) <= t) p += w;
  }
  return p;
}

// Frontier flags hold sweep stamps instead of booleans: sweep t takes part
// for r-cliques whose flag equals stamp(t) = t mod 255 + 1, and notifies by
// writing stamp(t+1) into the other array of the pair.  Old stamps never need
// clearing: a value left from sweep t' matches stamp(t) only when
// t' = t - 254k (harmless extra work; never a skipped r-clique).
__host__ __device__ __forceinline__ uint8_t sweep_stamp(int64_t t) {
  return (uint8_t)(t % 255 + 1);
}

// One r-clique per subgroup of G lanes (sl = lane within the subgroup), each
// lane holding M gathered values: d_s(R) <= G*M.  `active` false for a
// subgroup with no r-clique.  With a frontier (FR), an r-clique whose flag is
// clear is skipped: it cannot change.  SND writes only what it recomputes:
// a changed r-clique also flags itself for the next sweep (the self-activation
// of Alg. 3), so an r-clique skipped in sweep t+1 did not change in sweep t,
// and the output buffer of sweep t+1 (the input of sweep t) already holds
// its value.  Returns (on the subgroup's first lane only) whether R changed;
// *evald likewise whether it was recomputed.
template <int K, int G, int M, typename T, bool AND, bool FR>
__device__ __forceinline__ bool update_regs(const int64_t *__restrict__ inc_off,
                                            const int32_t *__restrict__ inc_ids,
                                            const T *tau_in, T *tau_out,
                                            int cap_by_tau, int64_t R,
                                            bool active, const uint8_t *act,
                                            uint8_t *act_next, uint8_t stamp,
                                            bool *evald,
                                            uint8_t *sum_next = nullptr) {
  const int sl = lane_id() % G;
  int32_t told = 0, c = 0;
  int64_t b = 0, d = 0;
  bool eval = active;
  if (active) {
    if (FR && act && act[R] != stamp) {
      eval = false;
    } else {
      told = (int32_t)tau_in[R];
      b = inc_off[R];
      d = inc_off[R + 1] - b;
      c = cap_by_tau ? told : (int32_t)d;
    }
  }
  // SND with the frontier keeps which members hold each minimum, so that
  // notifying needs no second gather (notify_kept).  Lanes with more than 4
  // values re-read only the qualifying s-cliques instead (notify_slots):
  // keeping masks past the search would cost those kernels occupancy.
  constexpr bool kKept = FR && !AND && M <= 4;
  constexpr bool kKeep = kKept && K > 1;
  constexpr int kMaskWords = kKeep ? (K * M + 31) / 32 : 1;
  int32_t rho[M];
  uint32_t amask[kMaskWords];
#pragma unroll
  for (int w = 0; w < kMaskWords; w++) amask[w] = 0;
#pragma unroll
  for (int m = 0; m < M; m++) {
    const int64_t j = sl + (int64_t)m * G;
    if (kKeep) {
      uint32_t a = 0;
      rho[m] = (j < d) ? gather_rho_arg<K, T>(inc_ids, b + j, tau_in, &a) : -1;
#pragma unroll
      for (int x = 0; x < K; x++) {
        const int bit = m * K + x;
        amask[bit >> 5] |= ((a >> x) & 1u) << (bit & 31);
      }
    } else {
      rho[m] = (j < d) ? gather_rho<K, T, AND>(inc_ids, b + j, tau_in) : -1;
    }
  }
  const int cnt = count_ge<G, M>(rho, c);
  const int32_t h = cnt >= c ? c : hindex_search<G, M>(rho, c);
  const bool ch = eval && h != told;  // uniform within the subgroup
  const bool lead = sl == 0;
  if (eval && lead) store_tau<T, AND>(tau_out + R, h, ch);
  if (FR && ch && act_next) {
    const uint8_t next = stamp == 255 ? 1 : stamp + 1;
    if (!AND && lead) {
      act_next[R] = next;
      if (sum_next) sum_next[R >> kGroupShift] = next;
    }
    if (kKept)
      notify_kept<K, G, M>(inc_ids, b, d, sl, rho, amask, told, h, act_next,
                           next, sum_next);
    else if (!AND)
      notify_slots<K, G, M, T>(inc_ids, b, d, sl, rho, told, h, tau_in,
                               act_next, next, sum_next);
    else
      notify<K, T, AND>(inc_ids, b, d, sl, G, told, h, tau_in, act_next, next,
                        sum_next);
  }
  *evald = lead && eval;
  return lead && ch;
}

// Sparse sweep of the r-cliques [lo, hi) of one bin of G lanes per
// r-clique, the frontier's flags being valid.  The calling wave (number
// `wave` of `nwaves`) runs only flagged r-cliques, 64/G at a time, found
// through ballots (nth_set_bit); skipped ones need no write (see
// update_regs).  It finds them either through the group summaries
// (act_sum: one stamp per 64 r-cliques, for the big bins, G <= 4: a step
// tests 64 groups, then loads the flags of flagged groups only), or by
// loading the flags of kU chunks of kChunk consecutive r-cliques at once
// (one lane per flag, coalesced, the loads in flight together).  A chunk
// holds at most 8 rounds of r-cliques, so a run of flagged hubs is not
// serialised on one wave for long.  Adds the wave's changed / recomputed
// counts to *n_ch / *n_ev.
template <int K, int G, int M, typename T, bool AND>
__device__ __forceinline__ void sweep_sparse(
    const int64_t *__restrict__ inc_off, const int32_t *__restrict__ inc_ids,
    const T *tin, T *tout, int cap_by_tau, int64_t lo, int64_t hi,
    int64_t wave, int64_t nwaves, const uint8_t *act, uint8_t *act_next,
    uint8_t stamp, unsigned long long *n_ch, unsigned long long *n_ev,
    const uint8_t *act_sum = nullptr, uint8_t *sum_next = nullptr) {
  constexpr int kPerWave = kWave / G;
  const int sub = lane_id() / G;
  const int lane = lane_id();
  // The flagged r-cliques found are queued, one per lane (lane l holds the
  // l-th), and run 64/G at a time when the queue is full or the share ends,
  // so that a group or chunk with one flagged r-clique does not take a whole
  // step of the wave.
  int64_t pend = 0;  // this lane's queued r-clique
  int np = 0;        // queued r-cliques (uniform)
  auto flush = [&]() {
    for (int r0 = 0; r0 < np; r0 += kPerWave) {  // uniform over the wave
      const int t = r0 + sub;
      const bool has = t < np;
      const int64_t R = __shfl(pend, has ? t : 0, kWave);
      bool ev;
      const bool changed = update_regs<K, G, M, T, AND, true>(
          inc_off, inc_ids, tin, tout, cap_by_tau, R, has, nullptr, act_next,
          stamp, &ev, sum_next);
      *n_ch += __popcll(ballot(changed));
      *n_ev += __popcll(ballot(ev));
    }
    np = 0;
  };
  // queues the flagged r-cliques of mask m (bit i: r-clique cb + i), running
  // the queue first when they would take it past `cap`
  auto queue = [&](uint64_t m, int64_t cb, int cap) {
    const int na = __popcll(m);
    if (np + na > cap) flush();
    const int slot = lane - np;  // the slot-th flagged r-clique of m
    if (slot >= 0 && slot < na) pend = cb + nth_set_bit(m, slot);
    np += na;
  };
  if (G <= 4 && act_sum != nullptr) {
    // Big bins: test 64 group summaries per step (one lane each), then the
    // flags of each flagged group only.  A sweep with few flagged r-cliques
    // reads 1/64 of the flags.
    const int64_t g_lo = lo >> kGroupShift;
    const int64_t g_hi = (hi + (1 << kGroupShift) - 1) >> kGroupShift;
    for (int64_t gb = g_lo + wave * kWave; gb < g_hi; gb += nwaves * kWave) {
      const int64_t gi = gb + lane;
      uint64_t gm = ballot(gi < g_hi && act_sum[gi] == stamp);
      while (gm) {  // uniform over the wave
        const int q = __ffsll((unsigned long long)gm) - 1;
        gm &= gm - 1;
        const int64_t cb = (gb + q) << kGroupShift;
        const int64_t Rl = cb + lane;
        queue(ballot(Rl >= lo && Rl < hi && act[Rl] == stamp), cb, kWave);
      }
    }
    if (np > 0) flush();
    return;
  }
  // At most 8 rounds of r-cliques per chunk and per queue, so that a run of
  // flagged hubs is not serialised on one wave for long.
  constexpr int kChunk = kPerWave * 8 < kWave ? kPerWave * 8 : kWave;
  // Several chunks per step only where a chunk is narrow work (G <= 4: the
  // big bins, where the flag scan dominates a sparse sweep); for wide
  // mappings a step of kU chunks would serialise up to 8 kU hub r-cliques
  // on one wave.
  constexpr int kU = G <= 4 ? 8 : 1;
  constexpr int64_t kStep = (int64_t)kChunk * kU;
  for (int64_t base = lo + wave * kStep; base < hi; base += nwaves * kStep) {
    bool on[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const int64_t Rl = base + (int64_t)u * kChunk + lane;
      on[u] = lane < kChunk && Rl < hi && act[Rl] == stamp;
    }
#pragma unroll
    for (int u = 0; u < kU; u++)
      queue(ballot(on[u]), base + (int64_t)u * kChunk, kChunk);
  }
  if (np > 0) flush();
}

// Bins hist[0..nb) count values, bin i standing for the value x0 + i*scale.
// Returns the largest i with base + sum_{i' >= i} hist[i'] >= x0 + i*scale,
// or -1 if there is none.  All NT threads of the block call it.
template <int NT>
__device__ int suffix_search(const int32_t *hist, int nb, int64_t base,
                             int64_t x0, int64_t scale) {
  __shared__ int64_t part[NT];
  __shared__ int best_s;
  const int t = threadIdx.x;
  const int chunk = (nb + NT - 1) / NT;
  const int lo = min(nb, t * chunk), hi = min(nb, lo + chunk);
  int64_t mine = 0;
  for (int i = lo; i < hi; i++) mine += hist[i];
  part[t] = mine;
  if (t == 0) best_s = -1;
  __syncthreads();
  int64_t above = base;  // the chunks above mine
  for (int q = t + 1; q < NT; q++) above += part[q];
  int found = -1;
  int64_t run = above;
  for (int i = hi - 1; i >= lo; i--) {
    run += hist[i];
    if (run >= x0 + (int64_t)i * scale) {
      found = i;
      break;
    }
  }
  if (found >= 0) atomicMax(&best_s, found);
  __syncthreads();
  const int r = best_s;
  __syncthreads();
  return r;
}

__device__ __forceinline__ int64_t block_sum(int64_t x) {
  __shared__ int64_t ws[kBlockThreads / kWave];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  if (lane_id() == 0) ws[threadIdx.x / kWave] = x;
  __syncthreads();
  int64_t s = 0;
#pragma unroll
  for (int w = 0; w < kBlockThreads / kWave; w++) s += ws[w];
  __syncthreads();
  return s;
}

// One r-clique per 256-thread workgroup, any d_s: LDS histogram of
// min(rho, c) in up to kBlockHistBins bins; for larger c values are binned
// coarsely and the coarse bin holding H is refined with a second gather.
// Returns whether R changed (thread 0 only); *evald likewise.
template <int K, typename T, bool AND, bool FR>
__device__ bool update_block(const int64_t *__restrict__ inc_off,
                             const int32_t *__restrict__ inc_ids,
                             const T *tau_in, T *tau_out, int cap_by_tau,
                             int64_t R, int32_t *hist, const uint8_t *act,
                             uint8_t *act_next, uint8_t stamp, bool *evald,
                             uint8_t *sum_next = nullptr) {
  const int t = threadIdx.x;
  if (FR && act && act[R] != stamp) {  // skipped: see update_regs
    *evald = false;
    return false;
  }
  const int32_t told = (int32_t)tau_in[R];
  const int64_t b = inc_off[R];
  const int64_t d = inc_off[R + 1] - b;
  const int32_t c = cap_by_tau ? told : (int32_t)d;
  const int64_t w = ((int64_t)c + kBlockHistBins) / kBlockHistBins;
  const int nb = (int)(((int64_t)c + w) / w);  // bins for values 0..c
  for (int x = t; x < nb; x += kBlockThreads) hist[x] = 0;
  __syncthreads();
  // One workgroup walks a long list: each thread keeps kU gathers in flight
  // (the ids, then the tau values, of kU list entries), or the walk is a
  // chain of dependent loads.  Values >= c are only counted (they enter the
  // search below as its starting suffix).
  constexpr int kU = 8;
  int64_t ge = 0;
  for (int64_t j0 = t; j0 < d; j0 += (int64_t)kBlockThreads * kU) {
    int32_t rho[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const int64_t j = j0 + (int64_t)u * kBlockThreads;
      rho[u] = j < d ? gather_rho<K, T, AND>(inc_ids, b + j, tau_in) : -1;
    }
#pragma unroll
    for (int u = 0; u < kU; u++) {
      if (rho[u] >= c)
        ge++;
      else if (rho[u] >= 0)
        atomicAdd(&hist[rho[u] / w], 1);
    }
  }
  ge = block_sum(ge);
  int32_t h = c;
  if (ge < c) {
    const int i = suffix_search<kBlockThreads>(hist, nb, ge, 0, w);
    if (w == 1) {
      h = i;
    } else {
      const int64_t x0 = (int64_t)i * w;
      const int64_t x1 = min(x0 + w, (int64_t)c + 1);  // exclusive
      const int nfine = (int)(x1 - x0);
      for (int x = t; x < nfine; x += kBlockThreads) hist[x] = 0;
      __syncthreads();
      int64_t above = 0;
      for (int64_t j0 = t; j0 < d; j0 += (int64_t)kBlockThreads * kU) {
        int32_t rho[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) {
          const int64_t j = j0 + (int64_t)u * kBlockThreads;
          rho[u] = j < d ? min(gather_rho<K, T, AND>(inc_ids, b + j, tau_in), c) : -1;
        }
#pragma unroll
        for (int u = 0; u < kU; u++) {
          if (rho[u] >= x1)
            above++;
          else if (rho[u] >= x0)
            atomicAdd(&hist[rho[u] - x0], 1);
        }
      }
      above = block_sum(above);
      const int f = suffix_search<kBlockThreads>(hist, nfine, above, x0, 1);
      h = (int32_t)(x0 + f);
    }
  }
  const bool ch = h != told;
  if (t == 0) store_tau<T, AND>(tau_out + R, h, ch);
  if (FR && ch && act_next) {
    const uint8_t next = stamp == 255 ? 1 : stamp + 1;
    if (!AND && t == 0) {
      act_next[R] = next;
      if (sum_next) sum_next[R >> kGroupShift] = next;
    }
    notify<K, T, AND>(inc_ids, b, d, t, kBlockThreads, told, h, tau_in,
                      act_next, next, sum_next);
  }
  __syncthreads();
  *evald = t == 0;
  return t == 0 && ch;
}

}  // namespace dev
}  // namespace nd
