// levels.hip -- degree levels (Defn. 4): L_0 holds the r-cliques of minimum
// S-degree; removing them removes every s-clique that contains one of them;
// L_1 holds the minimum-degree r-cliques of what is left, and so on.  Their
// number bounds the sweeps SND needs (level i is exact after i sweeps), the
// DL row of Table 3.
//
// One level per step, all on the device except a 3-integer read-back:
//   1. minimum current degree over the r-cliques still present (a compact
//      list of them, rebuilt every step),
//   2. split the list: degree == minimum -> this level (frontier), the rest
//      -> next list,
//   3. one wave per frontier r-clique walks its incidence list; an s-clique
//      still present (no member removed at an earlier level) is counted once,
//      by its frontier member of smallest id, and lowers the degree of each
//      member still present by one.
// The levels are fully determined by the definition, so the result is the
// same on every run.
#include <limits.h>

#include <algorithm>

#include "api_util.h"
#include "internal.h"

namespace nd {

namespace {

struct LevelCounters {
  int32_t min_deg;
  int32_t n_frontier;
  int32_t n_next;
  int32_t pad;
};

__global__ void k_level_reset(LevelCounters *c) {
  c->min_deg = INT_MAX;
  c->n_frontier = 0;
  c->n_next = 0;
}

__global__ __launch_bounds__(256) void k_level_min(
    const int32_t *__restrict__ alive, int64_t n, const int32_t *__restrict__ deg,
    LevelCounters *c) {
  int32_t m = INT_MAX;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = min(m, deg[alive[i]]);
  for (int o = kWave / 2; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o, kWave));
  if (lane_id() == 0 && m != INT_MAX) atomicMin(&c->min_deg, m);
}

// Wave-aggregated append of the lanes with `take` to list[*count ...].
__device__ __forceinline__ void wave_append(bool take, int32_t v, int32_t *list,
                                            int32_t *count) {
  const uint64_t b = ballot(take);
  if (!b) return;
  int32_t base = 0;
  if (lane_id() == __ffsll((long long)b) - 1)
    base = atomicAdd(count, (int32_t)__popcll(b));
  base = __shfl(base, __ffsll((long long)b) - 1, kWave);
  if (take) list[base + lanes_below(b)] = v;
}

__global__ __launch_bounds__(256) void k_level_split(
    const int32_t *__restrict__ alive, int64_t n, const int32_t *__restrict__ deg,
    int32_t level, int32_t *__restrict__ lvl, int32_t *__restrict__ frontier,
    int32_t *__restrict__ next, LevelCounters *c) {
  const int32_t m = c->min_deg;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // whole waves iterate together so that the ballots see every lane
  const int64_t n_up = (n + kWave - 1) / kWave * kWave;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_up;
       i += stride) {
    const bool valid = i < n;
    const int32_t R = valid ? alive[i] : 0;
    const bool now = valid && deg[R] == m;
    if (now) lvl[R] = level;
    wave_append(now, R, frontier, &c->n_frontier);
    wave_append(valid && !now, R, next, &c->n_next);
  }
}

template <int K>
__global__ __launch_bounds__(256) void k_level_peel(
    const int32_t *__restrict__ frontier, int64_t nf,
    const int64_t *__restrict__ inc_off, const int32_t *__restrict__ inc_ids,
    const int32_t *__restrict__ lvl, int32_t level, int32_t *__restrict__ deg) {
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t f = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
       f < nf; f += waves) {
    const int32_t R = frontier[f];
    const int64_t b = inc_off[R], d = inc_off[R + 1] - b;
    for (int64_t j = lane_id(); j < d; j += kWave) {
      const int32_t *o = inc_ids + (int64_t)K * (b + j);
      bool skip = false;
#pragma unroll
      for (int x = 0; x < K; x++) {
        const int32_t l = lvl[o[x]];
        skip |= (l >= 0 && l < level) || (l == level && o[x] < R);
      }
      if (skip) continue;
#pragma unroll
      for (int x = 0; x < K; x++)
        if (lvl[o[x]] < 0) atomicSub(&deg[o[x]], 1);
    }
  }
}

}  // namespace

nd_status levels(nd_graph *g, nd_kind kind, int32_t *level_out,
                 int32_t *num_levels, int on_device, hipStream_t s) {
  prepare(g, kind, s);
  const KindState &ks = g->ks[kind];
  Allocator &al = g->ctx->alloc;
  const int64_t nr = ks.nr;
  ND_REQUIRE(num_levels, ND_ERR_INVALID, "num_levels is NULL");
  ND_REQUIRE(level_out || nr == 0, ND_ERR_INVALID, "level is NULL");
  if (nr == 0) {
    *num_levels = 0;
    return ND_OK;
  }
  DArr<int32_t> deg(al, nr), lvl(al, nr), a0(al, nr), a1(al, nr), fr(al, nr);
  DArr<LevelCounters> cnt(al, 1);
  ND_HIP(hipMemcpyAsync(deg.p, ks.ds.p, sizeof(int32_t) * nr,
                        hipMemcpyDeviceToDevice, s));
  fill_i32(lvl.p, -1, nr, s);
  iota_i32(a0.p, nr, s);
  int32_t *alive = a0.p, *next = a1.p;
  int64_t nalive = nr;
  int32_t level = 0;
  const int max_grid = g->ctx->num_cu * 8;
  LevelCounters h{};
  while (nalive > 0) {
    const unsigned grid = (unsigned)std::min<int64_t>(grid_for(nalive, 256), max_grid);
    k_level_reset<<<1, 1, 0, s>>>(cnt.p);
    ND_LAUNCHED();
    k_level_min<<<grid, 256, 0, s>>>(alive, nalive, deg.p, cnt.p);
    ND_LAUNCHED();
    k_level_split<<<grid, 256, 0, s>>>(alive, nalive, deg.p, level, lvl.p, fr.p,
                                       next, cnt.p);
    ND_LAUNCHED();
    ND_HIP(hipMemcpyAsync(&h, cnt.p, sizeof h, hipMemcpyDeviceToHost, s));
    ND_HIP(hipStreamSynchronize(s));
    ND_REQUIRE(h.n_frontier > 0 && h.n_frontier + h.n_next == nalive,
               ND_ERR_DEVICE, "degree levels: inconsistent split");
    const unsigned pgrid =
        (unsigned)std::min<int64_t>(grid_for((int64_t)h.n_frontier * kWave, 256),
                                    max_grid);
    switch (ks.k) {
      case 1: k_level_peel<1><<<pgrid, 256, 0, s>>>(fr.p, h.n_frontier, ks.inc_off.p, ks.inc_ids.p, lvl.p, level, deg.p); break;
      case 2: k_level_peel<2><<<pgrid, 256, 0, s>>>(fr.p, h.n_frontier, ks.inc_off.p, ks.inc_ids.p, lvl.p, level, deg.p); break;
      default: k_level_peel<3><<<pgrid, 256, 0, s>>>(fr.p, h.n_frontier, ks.inc_off.p, ks.inc_ids.p, lvl.p, level, deg.p); break;
    }
    ND_LAUNCHED();
    std::swap(alive, next);
    nalive = h.n_next;
    level++;
  }
  *num_levels = level;
  if (on_device) {
    to_original(ks, lvl.p, false, level_out, s);
  } else {
    DArr<int32_t> out(al, nr);
    to_original(ks, lvl.p, false, out.p, s);
    ND_HIP(hipMemcpyAsync(level_out, out.p, sizeof(int32_t) * nr,
                          hipMemcpyDeviceToHost, s));
  }
  ND_HIP(hipStreamSynchronize(s));
  return ND_OK;
}

}  // namespace nd

using namespace nd;

extern "C" nd_status nd_levels(nd_graph *g, nd_kind kind, int32_t *level,
                               int32_t *num_levels, int on_device,
                               void *stream) {
  nd_status out = ND_OK;
  nd_status st = guarded([&] {
    ND_REQUIRE(g, ND_ERR_INVALID, "graph is NULL");
    ND_HIP(hipSetDevice(g->ctx->device));
    StreamScope scope((hipStream_t)stream);
    out = levels(g, kind, level, num_levels, on_device, (hipStream_t)stream);
  });
  return st != ND_OK ? st : out;
}
