// cliques.hip -- s-clique incidence lists (Section 3, Defn. of U, step 1).
//
// The paper finds the s-cliques containing an r-clique on the fly in every
// iteration (Section 5).  Here they are listed once, by intersecting sorted
// adjacency lists on the device, so that every sweep is a pure streaming
// gather:
//   k-truss (2,3): for edge (u,v) and every w in N(u) & N(v), the ids of the
//                  edges (u,w) and (v,w);
//   (3,4):         first the triangles (u,v,w), u<v<w, numbered
//                  lexicographically; then for triangle (u,v,w) and every x
//                  in N(u) & N(v) & N(w), the ids of the triangles {u,v,x},
//                  {u,w,x} and {v,w,x};
//   (1,3), (2,4):  from the triangle list (see below).
// Each is two passes: count, then (once every S-degree is known and the
// internal numbering is fixed, see build_layout) fill, which writes the lists
// in the internal order with internal ids.  The k-truss builder finds every
// triangle once, from its edge oriented by degree, and the (3,4) fill every
// 4-clique once, from its lowest triangle; entries that go to other lists
// take their slots from cursors (atomic, or per workgroup in LDS), so the
// order inside a list varies from run to run.  Nothing computed from a list
// depends on its order (min and H are order-free).  The k-core incidence is
// the CSR itself, re-indexed the same way.
//
// Work per item is proportional to the shortest adjacency list involved:
// each element of it is binary-searched in the others.  Items are binned by
// that length and each bin gets a subgroup of G lanes per item (G = 1, 4, 16,
// 64) that strides over the short list; matches are ordered with a ballot.
#include <algorithm>

#include "internal.h"

namespace nd {

namespace {

enum IsectMode : int {
  kCountTruss = 0,  // per edge: |N(u) & N(v)|
  kFillTruss,       // per edge: (eid(u,w), eid(v,w)) for each common w
  kCountTri,        // per edge: #{w > v common}
  kFillTri,         // per edge: tri_w / tri_e for each common w > v
};

struct EdgeIsectArgs {
  const int32_t *items;  // edge ids of this bin
  int64_t nitems;
  const int32_t *ev;     // edge endpoints (u, v), u < v
  const int64_t *row_off;
  const int32_t *col;
  const int32_t *eid;
  int32_t *count;        // count modes: per edge
  const int64_t *off;    // fill modes: output offset (truss: internal order)
  const int32_t *inv;    // truss fill: edge id -> internal id
  int32_t *out_a;        // fill: pair ids (truss) or tri_w (triangles)
  int32_t *out_b;        // fill: tri_e (triangles)
};

template <int G>
__device__ __forceinline__ uint64_t subgroup_mask() {
  if constexpr (G == 64) {
    return ~0ull;
  } else {
    const int sub = lane_id() / G;
    return (((uint64_t)1 << G) - 1) << (sub * G);
  }
}

template <int G, int MODE>
__global__ __launch_bounds__(256) void k_edge_isect(EdgeIsectArgs a) {
  const int sl = lane_id() % G;
  const int64_t nsub = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t gsub = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
       gsub < a.nitems; gsub += nsub) {  // uniform within the subgroup
  const int32_t e = a.items[gsub];
  const int32_t u = a.ev[2 * (int64_t)e], v = a.ev[2 * (int64_t)e + 1];
  const int64_t bu = a.row_off[u], eu = a.row_off[u + 1];
  const int64_t bv = a.row_off[v], ev = a.row_off[v + 1];
  const bool short_is_u = (eu - bu) <= (ev - bv);
  const int64_t sb = short_is_u ? bu : bv, se = short_is_u ? eu : ev;
  const int64_t lb = short_is_u ? bv : bu, le = short_is_u ? ev : eu;
  int64_t start = sb;
  if (MODE == kCountTri || MODE == kFillTri)
    start = lower_bound<int32_t>(a.col, sb, se, v + 1);  // only w > v
  const uint64_t smask = subgroup_mask<G>();
  int64_t written = 0;
  int64_t base = 0;
  if (MODE == kFillTruss) base = a.off[a.inv[e]];
  if (MODE == kFillTri) base = a.off[e];
  for (int64_t j0 = start; j0 < se; j0 += G) {
    const int64_t j = j0 + sl;
    bool found = false;
    int64_t q = 0;
    int32_t w = 0;
    if (j < se) {
      w = a.col[j];
      q = lower_bound<int32_t>(a.col, lb, le, w);
      found = q < le && a.col[q] == w;
    }
    const uint64_t m = ballot(found) & smask;
    if (MODE == kFillTruss && found) {
      const int64_t k = base + written + lanes_below(m);
      const int32_t id_short = a.inv[a.eid[j]], id_long = a.inv[a.eid[q]];
      a.out_a[2 * k] = short_is_u ? id_short : id_long;      // eid(u, w)
      a.out_a[2 * k + 1] = short_is_u ? id_long : id_short;  // eid(v, w)
    }
    if (MODE == kFillTri && found) {
      const int64_t k = base + written + lanes_below(m);
      a.out_a[k] = w;
      a.out_b[k] = e;
    }
    written += __popcll(m);
  }
  if ((MODE == kCountTruss || MODE == kCountTri) && sl == 0)
    a.count[e] = (int32_t)written;
  }
}

// Edges whose shorter list is long (both endpoints high-degree): one wave
// per edge streams the longer list through LDS in windows of kIsectWindow
// entries; the slice of the shorter list whose values fall inside a window is
// binary-searched in LDS rather than in global memory.  Windows cover
// increasing value ranges, so matches still come out in ascending order.
constexpr int kIsectWindow = 2048;

template <int MODE>
__global__ __launch_bounds__(kWave) void k_edge_isect_lds(EdgeIsectArgs a) {
  __shared__ int32_t win[kIsectWindow];
  const int lane = threadIdx.x;
  for (int64_t it = blockIdx.x; it < a.nitems; it += gridDim.x) {
    const int32_t e = a.items[it];
    const int32_t u = a.ev[2 * (int64_t)e], v = a.ev[2 * (int64_t)e + 1];
    const int64_t bu = a.row_off[u], eu = a.row_off[u + 1];
    const int64_t bv = a.row_off[v], ev = a.row_off[v + 1];
    const bool short_is_u = (eu - bu) <= (ev - bv);
    const int64_t sb = short_is_u ? bu : bv, se = short_is_u ? eu : ev;
    const int64_t lb = short_is_u ? bv : bu, le = short_is_u ? ev : eu;
    int64_t start = sb;
    if (MODE == kCountTri || MODE == kFillTri)
      start = lower_bound<int32_t>(a.col, sb, se, v + 1);  // only w > v
    int64_t base = 0;
    if (MODE == kFillTruss) base = a.off[a.inv[e]];
    if (MODE == kFillTri) base = a.off[e];
    int64_t written = 0;
    int64_t apos = start;  // shorter-list elements before apos are done
    for (int64_t w0 = lb; w0 < le && apos < se; w0 += kIsectWindow) {
      const int wn = (int)min((int64_t)kIsectWindow, le - w0);
      for (int i = lane; i < wn; i += kWave) win[i] = a.col[w0 + i];
      __syncthreads();
      const int32_t hi_val = win[wn - 1];
      // shorter-list elements <= hi_val that are not done yet
      const int64_t aend = lower_bound<int32_t>(a.col, apos, se, hi_val + 1);
      for (int64_t j0 = apos; j0 < aend; j0 += kWave) {
        const int64_t j = j0 + lane;
        bool found = false;
        int q = 0;
        int32_t w = 0;
        if (j < aend) {
          w = a.col[j];
          int lo = 0, hi = wn;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (win[mid] < w)
              lo = mid + 1;
            else
              hi = mid;
          }
          q = lo;
          found = q < wn && win[q] == w;
        }
        const uint64_t m = ballot(found);
        if (MODE == kFillTruss && found) {
          const int64_t k = base + written + lanes_below(m);
          const int32_t id_short = a.inv[a.eid[j]];
          const int32_t id_long = a.inv[a.eid[w0 + q]];
          a.out_a[2 * k] = short_is_u ? id_short : id_long;
          a.out_a[2 * k + 1] = short_is_u ? id_long : id_short;
        }
        if (MODE == kFillTri && found) {
          const int64_t k = base + written + lanes_below(m);
          a.out_a[k] = w;
          a.out_b[k] = e;
        }
        written += __popcll(m);
      }
      apos = aend;
      __syncthreads();  // the window is overwritten next
    }
    if ((MODE == kCountTruss || MODE == kCountTri) && lane == 0)
      a.count[e] = (int32_t)written;
  }
}

// ------------------------------------------------------------- (3,4)

struct TriIsectArgs {
  const int32_t *items;  // triangle ids of this bin
  int64_t nitems;
  const int32_t *ev;
  const int64_t *row_off;
  const int32_t *col;
  const int32_t *eid;
  const int64_t *toff;   // ne+1
  const int32_t *tri_w;
  const int32_t *tri_e;
  int32_t *count;        // count pass: S-degree of each triangle
  // count pass: its local 4-cliques (see below); fill pass: the cursor of
  // its remote entries, which start there
  int32_t *loc;
  const struct TriRec *rec;  // fill pass: each triangle's list (see below)
  int32_t *out;          // fill pass: 3 ids per 4-clique
  int32_t *err;          // set to 1 on an inconsistency (nothing written)
};

// Id of the triangle whose lowest edge (lexicographically) is e and whose
// third vertex is c: triangles are numbered by (lowest edge, third vertex).
__device__ __forceinline__ int32_t tri_in(const TriIsectArgs &t, int32_t e,
                                          int32_t c) {
  return (int32_t)lower_bound<int32_t>(t.tri_w, t.toff[e], t.toff[e + 1], c);
}

// Orders this wave's LDS accesses around it: the lanes of a subgroup (never
// wider than a wave) write a list into LDS that all of them then read.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Copies the two lists searched for every candidate into the subgroup's LDS
// slots when both fit (CAP entries each); returns whether they did.
template <int G, int CAP>
__device__ __forceinline__ bool n34_stage(const int32_t *__restrict__ col,
                                          int64_t b1, int64_t n1, int64_t b2,
                                          int64_t n2, int32_t *l1, int32_t *l2,
                                          int sl) {
  if (CAP == 0 || n1 > CAP || n2 > CAP) return false;
  wave_lds_sync();  // the subgroup's previous searches are done
  for (int i = sl; i < n1; i += G) l1[i] = col[b1 + i];
  for (int i = sl; i < n2; i += G) l2[i] = col[b2 + i];
  wave_lds_sync();
  return true;
}

// Binary searches of the (3,4) intersection take one dependent load per
// step; from LDS instead of the L2 they are several times shorter.
constexpr int n34_cap(int G) { return G == 16 ? 128 : G == 64 ? 512 : 0; }

// (3,4) count pass, one subgroup per triangle (the triangles whose lowest
// vertex is too big for the per-vertex builder below): the 4-cliques
// containing triangle (u,v,w), i.e. the x in N(u) & N(v) & N(w), and how
// many of them are local (x > u); G lanes stride over the shortest of the
// three lists and binary-search the other two (held in LDS when they fit).
template <int G>
__global__ __launch_bounds__(256) void k_n34_count(TriIsectArgs a) {
  constexpr int CAP = n34_cap(G);
  __shared__ int32_t lds[256 / G][2][CAP > 0 ? CAP : 1];
  const int sl = lane_id() % G;
  int32_t *l1 = lds[threadIdx.x / G][0], *l2 = lds[threadIdx.x / G][1];
  const int64_t nsub = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t gsub = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
       gsub < a.nitems; gsub += nsub) {  // uniform within the subgroup
    const int32_t t = a.items[gsub];
    const int32_t e = a.tri_e[t];
    const int32_t u = a.ev[2 * (int64_t)e], v = a.ev[2 * (int64_t)e + 1];
    const int32_t w = a.tri_w[t];
    const int64_t b[3] = {a.row_off[u], a.row_off[v], a.row_off[w]};
    const int64_t en[3] = {a.row_off[u + 1], a.row_off[v + 1], a.row_off[w + 1]};
    int sh = 0;
    if (en[1] - b[1] < en[sh] - b[sh]) sh = 1;
    if (en[2] - b[2] < en[sh] - b[sh]) sh = 2;
    const int o1 = sh == 0 ? 1 : 0, o2 = sh == 2 ? 1 : 2;
    const int64_t n1 = en[o1] - b[o1], n2 = en[o2] - b[o2];
    int found = 0, local = 0;
    if (n34_stage<G, CAP>(a.col, b[o1], n1, b[o2], n2, l1, l2, sl)) {
      for (int64_t j = b[sh] + sl; j < en[sh]; j += G) {
        const int32_t x = a.col[j];
        const int64_t q1 = lower_bound<int32_t>(l1, 0, n1, x);
        if (q1 >= n1 || l1[q1] != x) continue;
        const int64_t q2 = lower_bound<int32_t>(l2, 0, n2, x);
        const bool f = q2 < n2 && l2[q2] == x;
        found += f;
        local += f && x > u;
      }
    } else {
      for (int64_t j = b[sh] + sl; j < en[sh]; j += G) {
        const int32_t x = a.col[j];
        const int64_t q1 = lower_bound<int32_t>(a.col, b[o1], en[o1], x);
        if (q1 >= en[o1] || a.col[q1] != x) continue;
        const int64_t q2 = lower_bound<int32_t>(a.col, b[o2], en[o2], x);
        const bool f = q2 < en[o2] && a.col[q2] == x;
        found += f;
        local += f && x > u;
      }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      found += __shfl_xor(found, off, G);
      local += __shfl_xor(local, off, G);
    }
    if (sl == 0) {
      a.count[t] = found;
      a.loc[t] = local;
    }
  }
}

// ------------------------------------------- k-truss by orientation

// Orient every edge from the endpoint of lower (degree, id) to the higher one.
// Each triangle then has exactly one edge u->v whose out-lists N+(u), N+(v)
// both contain the third vertex, so intersecting out-lists lists every
// triangle once; out-lists are short (at most about sqrt(2|E|)) even when
// degrees are not.
__device__ __forceinline__ bool ranks_below(int64_t du, int32_t u, int64_t dv,
                                            int32_t v) {
  return du < dv || (du == dv && u < v);
}

__global__ void k_orient_flags(const int64_t *__restrict__ row_off,
                               const int32_t *__restrict__ col,
                               const int32_t *__restrict__ rowid, int64_t nnz,
                               int32_t *__restrict__ flag) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const int32_t u = rowid[p], v = col[p];
  const int64_t du = row_off[u + 1] - row_off[u], dv = row_off[v + 1] - row_off[v];
  flag[p] = ranks_below(du, u, dv, v) ? 1 : 0;
}

// Out-lists in CSR order (so sorted by vertex id) with each entry's edge id.
__global__ void k_orient_fill(const int32_t *__restrict__ col,
                              const int32_t *__restrict__ rowid,
                              const int32_t *__restrict__ eid,
                              const int32_t *__restrict__ flag,
                              const int64_t *__restrict__ pos, int64_t nnz,
                              int32_t *__restrict__ out_col,
                              int32_t *__restrict__ out_eid,
                              int32_t *__restrict__ out_src) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz || !flag[p]) return;
  const int64_t q = pos[p];
  out_col[q] = col[p];
  out_eid[q] = eid[p];
  out_src[q] = rowid[p];
}

// out_off[u] = first out-entry of u (entries are grouped by source, in order).
__global__ void k_orient_off(const int32_t *__restrict__ out_src, int64_t ne,
                             int32_t n, int64_t *__restrict__ out_off) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x > n) return;
  out_off[x] = lower_bound<int32_t>(out_src, 0, ne, (int32_t)x);
}

struct OrientArgs {
  const int32_t *items;   // oriented edges (out-entry index) of this bin
  int64_t nitems;
  const int64_t *out_off;
  const int32_t *out_col;
  const int32_t *out_eid;
  const int32_t *out_src;
  int32_t *count;         // count pass: per edge id
  const int32_t *inv;     // fill pass: edge id -> internal id
  unsigned long long *cursor;  // fill pass: next free side slot, internal
  int32_t *ids;           // fill pass: 2 ids per (edge, triangle)
  int32_t *count_base;    // count pass: base triangles per edge id
  const int64_t *base_off;  // fill pass: list start per internal id
  int lds_cap;            // k_orient_heavy: out-list entries held in LDS
  // count pass, when set: the triangles found from oriented edge q go to
  // tri_buf[tri_off[q] ...] as (e1, e2) pairs, for k_orient_scatter
  const int64_t *tri_off;
  int2 *tri_buf;
  // k_orient_heavy, count pass: side counts of the edges of out(u), summed
  // per source u (each edge lies in one out-list, so one source writes each)
  int32_t *hcount;
};

// One triangle (euv, e1 = (u,w), e2 = (v,w)) found from the oriented edge
// u->v.  Each edge's list holds first the triangles found from the edge
// itself (its "base" entries: their count and their places come from the
// subgroup that owns the edge, without atomics), then those where it is a
// side e1 or e2 (counted and placed with atomics).  Count pass: the side
// counts; fill pass: the three entries, the base one at base_pos.
template <bool FILL>
__device__ __forceinline__ void orient_emit(const OrientArgs &a, int32_t euv,
                                            int32_t e1, int32_t e2,
                                            int64_t base_pos) {
  if (!FILL) {
    atomicAdd(&a.count[e1], 1);
    atomicAdd(&a.count[e2], 1);
    if (a.tri_buf) a.tri_buf[base_pos] = make_int2(e1, e2);
  } else {
    const int32_t iuv = a.inv[euv], i1 = a.inv[e1], i2 = a.inv[e2];
    const int64_t p1 = (int64_t)atomicAdd(&a.cursor[i1], 1ull);
    const int64_t p2 = (int64_t)atomicAdd(&a.cursor[i2], 1ull);
    int2 *ids2 = reinterpret_cast<int2 *>(a.ids);  // one 8-byte store per entry
    ids2[base_pos] = make_int2(i1, i2);
    ids2[p1] = make_int2(iuv, i2);
    ids2[p2] = make_int2(iuv, i1);
  }
}

// After an edge's subgroup has found `run` base triangles: record them.
template <bool FILL>
__device__ __forceinline__ void orient_base_done(const OrientArgs &a,
                                                 int32_t euv, int run) {
  if (!FILL) {
    a.count_base[euv] = run;
    if (run) atomicAdd(&a.count[euv], run);
  }
}

template <int G, bool FILL>
__global__ __launch_bounds__(256) void k_orient_isect(OrientArgs a) {
  const int sl = lane_id() % G;
  const int64_t nsub = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t gsub = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
       gsub < a.nitems; gsub += nsub) {  // uniform within the subgroup
  const int64_t q = a.items[gsub];
  const int32_t u = a.out_src[q], v = a.out_col[q];
  const int32_t euv = a.out_eid[q];
  const int64_t bu = a.out_off[u], eu = a.out_off[u + 1];
  const int64_t bv = a.out_off[v], ev = a.out_off[v + 1];
  const bool short_is_u = (eu - bu) <= (ev - bv);
  const int64_t sb = short_is_u ? bu : bv, se = short_is_u ? eu : ev;
  const int64_t lb = short_is_u ? bv : bu, le = short_is_u ? ev : eu;
  const uint64_t smask = subgroup_mask<G>();
  const int64_t base = FILL ? a.base_off[a.inv[euv]]
                            : (a.tri_buf ? a.tri_off[q] : 0);
  int run = 0;
  for (int64_t j0 = sb; j0 < se; j0 += G) {  // uniform within the subgroup
    const int64_t j = j0 + sl;
    bool found = false;
    int64_t k = 0;
    if (j < se) {
      const int32_t w = a.out_col[j];
      k = lower_bound<int32_t>(a.out_col, lb, le, w);
      found = k < le && a.out_col[k] == w;
    }
    const uint64_t m = ballot(found) & smask;
    if (found) {
      const int32_t e1 = a.out_eid[short_is_u ? j : k];  // (u, w)
      const int32_t e2 = a.out_eid[short_is_u ? k : j];  // (v, w)
      orient_emit<FILL>(a, euv, e1, e2, base + run + lanes_below(m));
    }
    run += __popcll(m);
  }
  if (sl == 0) orient_base_done<FILL>(a, euv, run);
  }
}

// The oriented edges whose both out-lists are long (the 64-lane bin) are
// grouped by source u (they are sorted by it): one workgroup loads out(u)
// into LDS once, then each wave takes an edge u->v, streams out(v) from HBM
// (coalesced) and binary-searches each entry in the LDS copy of out(u).
// Degree orientation keeps out-lists short (at most sqrt(2|E|) entries), so
// out(u) fits LDS; the host falls back to k_orient_isect<64> otherwise.  In
// the count pass the side counts of the edges (u,w) of out(u) are summed in
// LDS and stored to hcount once per source (an edge lies in one out-list
// only), so only the (v,w) sides take a global atomic per triangle.  The
// triangle buffer then holds (index of (u,w) in out(u), edge (v,w)), for
// k_orient_scatter_heavy.
template <bool FILL>
__global__ __launch_bounds__(256) void k_orient_heavy(OrientArgs a,
                                                      const int32_t *__restrict__ seg_lo,
                                                      int64_t nseg) {
  extern __shared__ int32_t lds[];
  const int cap = a.lds_cap;
  int32_t *lc = lds, *le = lds + cap, *lcnt = lds + 2 * cap;  // lcnt: count pass
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
  constexpr int kWaves = 256 / kWave;
  for (int64_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
    const int64_t lo = seg_lo[sg];
    const int64_t hi = sg + 1 < nseg ? seg_lo[sg + 1] : a.nitems;
    const int32_t u = a.out_src[a.items[lo]];
    const int64_t bu = a.out_off[u];
    const int du = (int)(a.out_off[u + 1] - bu);  // <= cap (host-checked)
    __syncthreads();  // the previous segment is done with the LDS copy
    for (int i = t; i < du; i += 256) {
      lc[i] = a.out_col[bu + i];
      le[i] = a.out_eid[bu + i];
      if (!FILL) lcnt[i] = 0;
    }
    __syncthreads();
    for (int64_t e = lo + w; e < hi; e += kWaves) {  // one edge per wave
      const int64_t q = a.items[e];
      const int32_t v = a.out_col[q];
      const int32_t euv = a.out_eid[q];
      const int64_t bv = a.out_off[v], ev = a.out_off[v + 1];
      const int64_t base = FILL ? a.base_off[a.inv[euv]]
                                : (a.tri_buf ? a.tri_off[q] : 0);
      int run = 0;
      for (int64_t j0 = bv; j0 < ev; j0 += kWave) {  // uniform over the wave
        const int64_t j = j0 + lane;
        bool found = false;
        int l = 0;
        if (j < ev) {
          const int32_t x = a.out_col[j];
          int r = du;
          while (l < r) {
            const int mid = (l + r) >> 1;
            if (lc[mid] < x)
              l = mid + 1;
            else
              r = mid;
          }
          found = l < du && lc[l] == x;
        }
        const uint64_t m = ballot(found);
        if (found) {
          const int32_t e2 = a.out_eid[j];
          const int64_t bp = base + run + lanes_below(m);
          if (FILL) {
            orient_emit<true>(a, euv, le[l], e2, bp);
          } else {
            atomicAdd(&lcnt[l], 1);
            atomicAdd(&a.count[e2], 1);
            if (a.tri_buf) a.tri_buf[bp] = make_int2(l, e2);
          }
        }
        run += __popcll(m);
      }
      if (lane == 0) orient_base_done<FILL>(a, euv, run);
    }
    if (!FILL) {
      __syncthreads();  // every wave is done with this source
      for (int i = t; i < du; i += 256) a.hcount[le[i]] = lcnt[i];
    }
  }
}

// Fill pass from the triangles the count pass recorded: oriented edge q
// found count_base[euv] triangles, kept at tri_buf[tri_off[q] ...] in the
// order it found them; each goes into the lists of its three edges exactly as
// orient_emit places it, without intersecting the out-lists again.
template <int G>
__global__ __launch_bounds__(256) void k_orient_scatter(OrientArgs a) {
  const int sl = lane_id() % G;
  const int64_t nsub = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t gsub = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
       gsub < a.nitems; gsub += nsub) {
    const int64_t q = a.items[gsub];
    const int32_t euv = a.out_eid[q];
    const int32_t n = a.count_base[euv];
    if (n == 0) continue;
    const int64_t base = a.base_off[a.inv[euv]];
    const int2 *tb = a.tri_buf + a.tri_off[q];
    for (int i = sl; i < n; i += G) {
      const int2 p = tb[i];
      orient_emit<true>(a, euv, p.x, p.y, base + i);
    }
  }
}

// Fill pass of the 64-lane bin from the triangle buffer, one workgroup per
// source u as in the count pass.  The list of each edge (u,w) of out(u)
// keeps, right after its base entries, the hcount slots of the triangles
// where it is the (u,w) side, all found from this source: they are placed
// with LDS cursors; only the (v,w) sides take global atomic cursors.
__global__ __launch_bounds__(256) void k_orient_scatter_heavy(
    OrientArgs a, const int32_t *__restrict__ seg_lo, int64_t nseg) {
  extern __shared__ unsigned long long lds64[];
  const int cap = a.lds_cap;
  unsigned long long *lcur = lds64;                          // cap entries
  int32_t *linv = reinterpret_cast<int32_t *>(lds64 + cap);  // cap entries
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
  constexpr int kWaves = 256 / kWave;
  int2 *ids2 = reinterpret_cast<int2 *>(a.ids);
  for (int64_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
    const int64_t lo = seg_lo[sg];
    const int64_t hi = sg + 1 < nseg ? seg_lo[sg + 1] : a.nitems;
    const int32_t u = a.out_src[a.items[lo]];
    const int64_t bu = a.out_off[u];
    const int du = (int)(a.out_off[u + 1] - bu);  // <= cap (host-checked)
    __syncthreads();  // the previous source is done with the LDS cursors
    for (int i = t; i < du; i += 256) {
      const int32_t e = a.out_eid[bu + i];
      const int32_t ie = a.inv[e];
      linv[i] = ie;
      lcur[i] = (unsigned long long)(a.base_off[ie] + a.count_base[e]);
    }
    __syncthreads();
    for (int64_t e = lo + w; e < hi; e += kWaves) {  // one edge per wave
      const int64_t q = a.items[e];
      const int32_t euv = a.out_eid[q];
      const int32_t n = a.count_base[euv];
      const int32_t iuv = a.inv[euv];
      const int64_t base = a.base_off[iuv];
      const int2 *tb = a.tri_buf + a.tri_off[q];
      for (int i = lane; i < n; i += kWave) {
        const int2 p = tb[i];  // (index of (u,w) in out(u), edge (v,w))
        const int32_t i1 = linv[p.x], i2 = a.inv[p.y];
        const int64_t p1 = (int64_t)atomicAdd(&lcur[p.x], 1ull);
        const int64_t p2 = (int64_t)atomicAdd(&a.cursor[i2], 1ull);
        ids2[base + i] = make_int2(i1, i2);
        ids2[p1] = make_int2(iuv, i2);
        ids2[p2] = make_int2(iuv, i1);
      }
    }
  }
}

// Start of every run of equal source among the items: flag[i] = 1 there.
__global__ void k_seg_flags(const int32_t *__restrict__ items, int64_t n,
                            const int32_t *__restrict__ out_src,
                            int32_t *__restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n)
    flag[i] = (i == 0 || out_src[items[i]] != out_src[items[i - 1]]) ? 1 : 0;
}

__global__ void k_seg_fill(const int32_t *__restrict__ flag,
                           const int64_t *__restrict__ pos, int64_t n,
                           int32_t *__restrict__ seg_lo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) seg_lo[pos[i]] = (int32_t)i;
}

__global__ void k_max_outdeg(const int64_t *__restrict__ out_off, int32_t n,
                             int32_t *__restrict__ mx) {
  int32_t m = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x)
    m = max(m, (int32_t)(out_off[u + 1] - out_off[u]));
  for (int o = kWave / 2; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, kWave));
  if (lane_id() == 0) atomicMax(mx, m);
}

// Bin of oriented edge q by its shorter out-list, whose length also bounds
// the triangles found from q (cap).
__global__ void k_orient_bins(const int64_t *__restrict__ out_off,
                              const int32_t *__restrict__ out_col,
                              const int32_t *__restrict__ out_src, int64_t ne,
                              uint8_t *__restrict__ bin,
                              int32_t *__restrict__ cap) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ne) return;
  const int32_t u = out_src[q], v = out_col[q];
  const int64_t a = out_off[u + 1] - out_off[u], b = out_off[v + 1] - out_off[v];
  const int64_t m = min(a, b);
  bin[q] = m <= 4 ? 0 : m <= 16 ? 1 : m <= 64 ? 2 : 3;
  cap[q] = (int32_t)m;
}

// Side entries of internal r-clique i start after its base entries and, when
// given, after the blocks reserved per source (skip, by edge id).
__global__ void k_cursor_init(const int64_t *__restrict__ off,
                              const int32_t *__restrict__ perm,
                              const int32_t *__restrict__ count_base,
                              const int32_t *__restrict__ skip, int64_t nr,
                              unsigned long long *__restrict__ cursor) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nr)
    cursor[i] = (unsigned long long)(off[i] + (count_base ? count_base[perm[i]] : 0) +
                                     (skip ? skip[perm[i]] : 0));
}

__global__ void k_add_i32(int32_t *__restrict__ x, const int32_t *__restrict__ y,
                          int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += y[i];
}

// Segments of equal source in the 64-lane bin (for k_orient_heavy).
struct HeavySegs {
  DArr<int32_t> lo;
  int64_t n = 0;
};

template <bool FILL>
void run_orient(OrientArgs a, const int32_t *items, const int64_t *bin_off,
                const HeavySegs &hs, hipStream_t s) {
  for (int b = 0; b < 4; b++) {
    a.items = items + bin_off[b];
    a.nitems = bin_off[b + 1] - bin_off[b];
    if (a.nitems == 0) continue;
    switch (b) {
      case 0: k_orient_isect<1, FILL><<<grid_stride(a.nitems, 1), 256, 0, s>>>(a); break;
      case 1: k_orient_isect<4, FILL><<<grid_stride(a.nitems, 4), 256, 0, s>>>(a); break;
      case 2: k_orient_isect<16, FILL><<<grid_stride(a.nitems, 16), 256, 0, s>>>(a); break;
      default:
        if (a.lds_cap > 0) {
          const unsigned grid = (unsigned)std::min<int64_t>(hs.n, 65536);
          const size_t lds = sizeof(int32_t) * (FILL ? 2 : 3) * a.lds_cap;
          k_orient_heavy<FILL><<<grid, 256, lds, s>>>(a, hs.lo.p, hs.n);
        } else {
          k_orient_isect<64, FILL><<<grid_stride(a.nitems, 64), 256, 0, s>>>(a);
        }
        break;
    }
    ND_LAUNCHED();
  }
}

void run_scatter(OrientArgs a, const int32_t *items, const int64_t *bin_off,
                 const HeavySegs &hs, hipStream_t s) {
  for (int b = 0; b < 4; b++) {
    a.items = items + bin_off[b];
    a.nitems = bin_off[b + 1] - bin_off[b];
    if (a.nitems == 0) continue;
    switch (b) {
      case 0: k_orient_scatter<1><<<grid_stride(a.nitems, 1), 256, 0, s>>>(a); break;
      case 1: k_orient_scatter<4><<<grid_stride(a.nitems, 4), 256, 0, s>>>(a); break;
      case 2: k_orient_scatter<16><<<grid_stride(a.nitems, 16), 256, 0, s>>>(a); break;
      default:
        if (a.lds_cap > 0) {  // the count pass ran k_orient_heavy
          const unsigned grid = (unsigned)std::min<int64_t>(hs.n, 65536);
          const size_t lds = (sizeof(unsigned long long) + sizeof(int32_t)) * a.lds_cap;
          k_orient_scatter_heavy<<<grid, 256, lds, s>>>(a, hs.lo.p, hs.n);
        } else {
          k_orient_scatter<64><<<grid_stride(a.nitems, 64), 256, 0, s>>>(a);
        }
        break;
    }
    ND_LAUNCHED();
  }
}

// ------------------------------------------------------------- binning

constexpr int kIsectBins = 4;  // G = 1, 4, 16, 64

__device__ __forceinline__ uint8_t isect_bin(int64_t len) {
  return len <= 4 ? 0 : len <= 16 ? 1 : len <= 128 ? 2 : 3;
}

__global__ void k_edge_bins(const int32_t *__restrict__ ev,
                            const int64_t *__restrict__ row_off, int64_t ne,
                            uint8_t *__restrict__ bin) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int32_t u = ev[2 * e], v = ev[2 * e + 1];
  int64_t du = row_off[u + 1] - row_off[u], dv = row_off[v + 1] - row_off[v];
  bin[e] = isect_bin(min(du, dv));
}

__global__ void k_tri_bins(const int32_t *__restrict__ ev,
                           const int32_t *__restrict__ tri_e,
                           const int32_t *__restrict__ tri_w,
                           const int64_t *__restrict__ row_off, int64_t nt,
                           uint8_t *__restrict__ bin) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  int32_t e = tri_e[t];
  int32_t u = ev[2 * (int64_t)e], v = ev[2 * (int64_t)e + 1], w = tri_w[t];
  int64_t d = min(row_off[u + 1] - row_off[u], row_off[v + 1] - row_off[v]);
  d = min(d, row_off[w + 1] - row_off[w]);
  bin[t] = isect_bin(d);
}

template <int MODE>
void run_edge_isect(EdgeIsectArgs a, const int32_t *items,
                    const int64_t *bin_off, hipStream_t s) {
  for (int b = 0; b < kIsectBins; b++) {
    a.items = items + bin_off[b];
    a.nitems = bin_off[b + 1] - bin_off[b];
    if (a.nitems == 0) continue;
    switch (b) {
      case 0: k_edge_isect<1, MODE><<<grid_stride(a.nitems, 1), 256, 0, s>>>(a); break;
      case 1: k_edge_isect<4, MODE><<<grid_stride(a.nitems, 4), 256, 0, s>>>(a); break;
      case 2: k_edge_isect<16, MODE><<<grid_stride(a.nitems, 16), 256, 0, s>>>(a); break;
      default: {
        const unsigned grid = (unsigned)std::min<int64_t>(a.nitems, 1 << 20);
        k_edge_isect_lds<MODE><<<grid, kWave, 0, s>>>(a);
        break;
      }
    }
    ND_LAUNCHED();
  }
}

// Where a triangle's 4-cliques go in its list.  A 4-clique {p<q<r<s} is
// written by the builder of its lowest vertex p.  In the list of a triangle
// T, the "local" entries come first: the 4-cliques T + y with y above T's
// lowest vertex (their lowest vertex is T's, so T's own builder writes them,
// each at its rank, without atomics); then the "remote" ones (y below: T is
// the 4-clique's triangle without p, written by p's builder at a slot taken
// from T's cursor, which starts at T's local count) -- one atomic per
// 4-clique.

// What the (3,4) fill needs of triangle t, in one 16-byte load: its
// internal id and the place and length of its list.
struct alignas(16) TriRec {
  int64_t base;
  int32_t inv;
  int32_t len;
};

// Write the 3 ids of one entry at place `slot` of the list of r, if it lies
// inside the list (else flag an inconsistency).
__device__ __forceinline__ void n34_put(const TriIsectArgs &a, const TriRec &r,
                                        int64_t slot, int32_t i0, int32_t i1,
                                        int32_t i2) {
  if (slot < 0 || slot >= r.len) {
    *a.err = 1;
    return;
  }
  int32_t *o = a.out + 3 * (r.base + slot);
  o[0] = i0;
  o[1] = i1;
  o[2] = i2;
}

// Id of triangle p < q < r (-1 if it is not one): the edge (p,q) from p's
// adjacency, then r among that edge's third vertices.
__device__ __forceinline__ int32_t n34_tri_id(const TriIsectArgs &a, int32_t p,
                                              int32_t q, int32_t r) {
  const int64_t e0 = a.row_off[p], e1 = a.row_off[p + 1];
  const int64_t pos = lower_bound<int32_t>(a.col, e0, e1, q);
  if (pos >= e1 || a.col[pos] != q) return -1;
  const int32_t e = a.eid[pos];
  const int64_t t0 = a.toff[e], t1 = a.toff[e + 1];
  const int64_t t = lower_bound<int32_t>(a.tri_w, t0, t1, r);
  return (t < t1 && a.tri_w[t] == r) ? (int32_t)t : -1;
}

__device__ __forceinline__ int32_t n34_sorted_id(const TriIsectArgs &a,
                                                 int32_t x, int32_t y,
                                                 int32_t z) {
  // sort three distinct vertices
  const int32_t lo = min(x, min(y, z)), hi = max(x, max(y, z));
  const int32_t mid = x + y + z - lo - hi;
  return n34_tri_id(a, lo, mid, hi);
}

// (3,4) fill pass, one subgroup per triangle (u,v,w) whose lowest vertex u is
// too big for the per-vertex builder: its local entries (x > u in
// N(u) & N(v) & N(w)) at their rank, each with the three other triangles
// found by search, and, for the 4-cliques where it is the lowest triangle
// (x > w), the remote entry of the triangle {v,w,x}.
template <int G>
__global__ __launch_bounds__(256) void k_n34_fill_owner(TriIsectArgs a) {
  constexpr int CAP = n34_cap(G);
  __shared__ int32_t lds[256 / G][2][CAP > 0 ? CAP : 1];
  const int sl = lane_id() % G;
  const int sub = lane_id() / G;
  const uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1);
  int32_t *l1 = lds[threadIdx.x / G][0], *l2 = lds[threadIdx.x / G][1];
  const int64_t nsub = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t gsub = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
       gsub < a.nitems; gsub += nsub) {  // uniform within the subgroup
    const int32_t t = a.items[gsub];
    const int32_t e = a.tri_e[t];
    const int32_t u = a.ev[2 * (int64_t)e], v = a.ev[2 * (int64_t)e + 1];
    const int32_t w = a.tri_w[t];
    const int64_t b[3] = {a.row_off[u], a.row_off[v], a.row_off[w]};
    const int64_t en[3] = {a.row_off[u + 1], a.row_off[v + 1], a.row_off[w + 1]};
    int sh = 0;
    if (en[1] - b[1] < en[sh] - b[sh]) sh = 1;
    if (en[2] - b[2] < en[sh] - b[sh]) sh = 2;
    const int o1 = sh == 0 ? 1 : 0, o2 = sh == 2 ? 1 : 2;
    const int64_t n1 = en[o1] - b[o1], n2 = en[o2] - b[o2];
    const bool staged = n34_stage<G, CAP>(a.col, b[o1], n1, b[o2], n2, l1, l2, sl);
    const TriRec rt = a.rec[t];
    int64_t nloc = 0;  // local entries written so far (uniform)
    for (int64_t j0 = b[sh]; j0 < en[sh]; j0 += G) {  // uniform rounds
      const int64_t j = j0 + sl;
      bool hit = false;
      int32_t x = -1;
      if (j < en[sh]) {
        x = a.col[j];
        if (x > u) {
          if (staged) {
            const int64_t q1 = lower_bound<int32_t>(l1, 0, n1, x);
            const int64_t q2 = lower_bound<int32_t>(l2, 0, n2, x);
            hit = q1 < n1 && l1[q1] == x && q2 < n2 && l2[q2] == x;
          } else {
            const int64_t q1 = lower_bound<int32_t>(a.col, b[o1], en[o1], x);
            const int64_t q2 = lower_bound<int32_t>(a.col, b[o2], en[o2], x);
            hit = q1 < en[o1] && a.col[q1] == x && q2 < en[o2] && a.col[q2] == x;
          }
        }
      }
      const uint64_t m = (ballot(hit) >> (sub * G)) & gmask;
      if (hit) {
        const int rank = __popcll(m & ((1ull << sl) - 1));
        const int32_t tuv = n34_sorted_id(a, u, v, x);
        const int32_t tuw = n34_sorted_id(a, u, w, x);
        const int32_t tvw = n34_sorted_id(a, v, w, x);
        if (tuv < 0 || tuw < 0 || tvw < 0) {
          *a.err = 1;
        } else {
          const TriRec ruv = a.rec[tuv], ruw = a.rec[tuw], rvw = a.rec[tvw];
          n34_put(a, rt, nloc + rank, ruv.inv, ruw.inv, rvw.inv);
          if (x > w) {  // {u,v,w,x} seen from its lowest triangle: once
            const int32_t p = atomicAdd(&a.loc[tvw], 1);
            n34_put(a, rvw, p, rt.inv, ruv.inv, ruw.inv);
          }
        }
      }
      nloc += __popcll(m);
    }
  }
}

void run_n34_tri(TriIsectArgs a, bool fill, const int32_t *items,
                 const int64_t *bin_off, hipStream_t s) {
  for (int b = 0; b < kIsectBins; b++) {
    a.items = items + bin_off[b];
    a.nitems = bin_off[b + 1] - bin_off[b];
    if (a.nitems == 0) continue;
    const int G = b == 0 ? 1 : b == 1 ? 4 : b == 2 ? 16 : 64;
    const unsigned grid = grid_stride(a.nitems, G);
    switch (b * 2 + (fill ? 1 : 0)) {
      case 0: k_n34_count<1><<<grid, 256, 0, s>>>(a); break;
      case 1: k_n34_fill_owner<1><<<grid, 256, 0, s>>>(a); break;
      case 2: k_n34_count<4><<<grid, 256, 0, s>>>(a); break;
      case 3: k_n34_fill_owner<4><<<grid, 256, 0, s>>>(a); break;
      case 4: k_n34_count<16><<<grid, 256, 0, s>>>(a); break;
      case 5: k_n34_fill_owner<16><<<grid, 256, 0, s>>>(a); break;
      case 6: k_n34_count<64><<<grid, 256, 0, s>>>(a); break;
      default: k_n34_fill_owner<64><<<grid, 256, 0, s>>>(a); break;
    }
    ND_LAUNCHED();
  }
}

// ------------------------------------------- (3,4) per lowest vertex
//
// For a vertex p of degree d <= D, one wave holds N(p) = nb[0..d) in LDS
// (ascending) with its induced adjacency as bit rows: bit q of A[i] is set
// when nb[q] is adjacent to nb[i].  With nl = the number of neighbours below
// p (nb[i] > p iff i >= nl) and i >= nl:
//   * triangle (p, nb[i], nb[j]), i < j, exists iff bit j of A[i]; triangles
//     are numbered by lowest edge, then third vertex, so its id is
//     toff[edge (p, nb[i])] + #(bits of A[i] strictly between i and j);
//   * its 4-cliques are the bits of A[i] & A[j]: its S-degree is their
//     count, its local count (4th vertex above p) the count at bits >= nl;
//   * the 4-cliques with lowest vertex p are the triples i < j < k (all
//     >= nl) pairwise adjacent.  Three of their triangles contain p (ids and
//     local ranks from the bit rows); the fourth, (nb[i], nb[j], nb[k]), is
//     found by search and receives its remote entry.

constexpr int kN34VMax = 256;  // largest degree of the per-vertex builder

// LDS of one wave of the per-vertex builder.  Each pass holds only its own
// arrays (the other's shrink to one element): the workgroup is one wave, so
// LDS per wave sets how many waves a CU keeps in flight, and both passes
// wait on dependent loads.  Triangle ids fit 32 bits (at most 2^31 - 1
// r-cliques).
template <int D, bool FILL>
struct N34VLds {
  static constexpr int kC = FILL ? kWave : 1;  // fill-pass chunk arrays
  int32_t nb[D];
  int32_t len[D];      // |N(nb[i])|
  int64_t ro[D];       // row_off[nb[i]]
  int32_t pre[D + 1];  // exclusive prefix: bit-row work, then triangles
  int32_t st[D];       // where row i's walk of N(nb[i]) starts (row build)
  uint32_t A[D][D / 32];
  int32_t tb[D];       // toff of edge (p, nb[i]), i >= nl
  // fill pass: one chunk of up to 64 triangles with their lists (base,
  // internal id, length), and for each the range of triangles of edge
  // (nb[i], nb[j]) in which its 4-cliques' remote triangles lie (found once
  // per triangle, not once per 4-clique)
  int16_t ci[kC], cj[kC];
  int64_t cb[kC];
  int32_t cv[kC], cl[kC];
  int32_t coff[FILL ? kWave + 1 : 1];
  int32_t cs0[kC];
  int32_t cn[kC];
};

// Exclusive prefix sums of v[0..n) in place, v[n] = total (one wave).
__device__ void wave_scan_lds(int32_t *v, int n) {
  const int lane = lane_id();
  const int per = (n + kWave - 1) / kWave;
  const int lo = min(n, lane * per), hi = min(n, lo + per);
  int sum = 0;
  for (int i = lo; i < hi; i++) sum += v[i];
  int x = sum;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  const int total = __shfl(x, kWave - 1, kWave);
  int run = x - sum;
  for (int i = lo; i < hi; i++) {
    const int t = v[i];
    v[i] = run;
    run += t;
  }
  if (lane == 0) v[n] = total;
  wave_lds_sync();
}

// The row i of an exclusive prefix pre[0..n] (pre[n] > t) with
// pre[i] <= t < pre[i+1].
__device__ __forceinline__ int row_of(const int32_t *pre, int n, int32_t t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Bits [lo, hi) of the 32-bit word number w.
__device__ __forceinline__ uint32_t word_range(int w, int lo, int hi) {
  const int a = min(max(lo - 32 * w, 0), 32), b = min(max(hi - 32 * w, 0), 32);
  const uint32_t upto_b = b >= 32 ? 0xffffffffu : ((1u << b) - 1);
  const uint32_t from_a = a >= 32 ? 0u : ~((1u << a) - 1);
  return upto_b & from_a;
}

// Set bits of x & y in [lo, hi) (y may be x).
template <int W>
__device__ __forceinline__ int popc_and(const uint32_t *x, const uint32_t *y,
                                        int lo, int hi) {
  int c = 0;
#pragma unroll
  for (int w = 0; w < W; w++) c += __popc(x[w] & y[w] & word_range(w, lo, hi));
  return c;
}

// Position of the r-th (from 0) set bit of x & y at or above lo; -1 if none.
template <int W>
__device__ __forceinline__ int nth_and(const uint32_t *x, const uint32_t *y,
                                       int lo, int r) {
#pragma unroll
  for (int w = 0; w < W; w++) {
    uint32_t m = x[w] & y[w] & word_range(w, lo, 32 * W);
    const int pc = __popc(m);
    if (r < pc) {
      for (; r > 0; r--) m &= m - 1;
      return 32 * w + __ffs(m) - 1;
    }
    r -= pc;
  }
  return -1;
}

// Bit-row words kept per CSR entry between the count and the fill pass: the
// d rows of vertex p (D / 32 words each) lie packed from
// rows[row_off[p] * kN34RowWords], inside the region its entries own.
constexpr int kN34RowWords = 8;

struct N34VArgs {
  const int32_t *items;  // vertices of this degree class
  int64_t nitems;
  const int64_t *row_off;
  const int32_t *col;
  const int32_t *eid;
  const int32_t *nlow;
  const int64_t *eoff;
  // the bit rows: written by the first pass that builds them, read back by
  // the later ones (NULL: every pass builds its own)
  uint32_t *rows;
  int rows_ready;        // rows already holds every vertex's rows
  int32_t *tcnt;         // rows pass: triangles per edge (lowest edge)
  int32_t *tw, *te;      // triangles pass: tri_w / tri_e of those edges
  TriIsectArgs t;        // triangle tables, outputs and error flag
};

// Passes of the per-vertex builder: the bit rows and each edge's triangle
// count; the triangles themselves; the S-degrees and local counts of the
// triangles; the 4-cliques' entries.
constexpr int kVRows = 0, kVTris = 1, kVCount = 2, kVFill = 3;

// One wave per vertex p of degree <= D, one pass (MODE) over the triangles
// and 4-cliques whose lowest vertex is p: the bit rows (kept in a.rows) and
// the triangle count of each of p's upper edges; the triangles of those
// edges; the triangles' S-degrees and local counts; the 4-cliques' entries.
template <int D, int MODE>
__global__ __launch_bounds__(kWave) void k_n34_vertex(N34VArgs a) {
  constexpr int W = D / 32;
  constexpr bool FILL = MODE == kVFill;
  __shared__ N34VLds<D, FILL> L;
  const int lane = lane_id();
  const TriIsectArgs &T = a.t;
  for (int64_t it = blockIdx.x; it < a.nitems; it += gridDim.x) {
    const int32_t p = a.items[it];
    const int64_t base = a.row_off[p];
    const int d = (int)(a.row_off[p + 1] - base);
    const int nl = a.nlow[p];
    const int64_t e_lo = a.eoff[p];
    wave_lds_sync();  // the previous vertex's reads are done
    const bool reuse = MODE == kVTris || (MODE == kVCount && a.rows_ready) ||
                       (FILL && a.rows != nullptr);
    if (reuse) {
      for (int x = lane; x < d * W; x += kWave)
        L.A[x / W][x % W] = a.rows[base * kN34RowWords + x];
    } else {
      for (int x = lane; x < d * W; x += kWave) L.A[x / W][x % W] = 0;
    }
    for (int i = lane; i < d; i += kWave) {
      const int32_t v = a.col[base + i];
      L.nb[i] = v;
      L.ro[i] = a.row_off[v];
      L.len[i] = (int32_t)(a.row_off[v + 1] - L.ro[i]);
    }
    wave_lds_sync();
    if (!reuse) {
      // bit rows, which are symmetric: each pair i < q is looked at once,
      // from row i, and sets both bits.  A short row walks the part of
      // N(nb[i]) between nb[i] and the largest neighbour of p, finding each
      // entry among nb above i; a long one (a hub's) looks each nb[q], q > i,
      // up in N(nb[i]) instead.
      const int32_t top = L.nb[d - 1];
      for (int i = lane; i < d; i += kWave) {
        int32_t w = d - 1 - i;
        if (L.len[i] <= 4 * d) {
          const int64_t e1 = L.ro[i] + L.len[i];
          const int64_t b = lower_bound<int32_t>(T.col, L.ro[i], e1, L.nb[i] + 1);
          const int64_t e = lower_bound<int32_t>(T.col, b, e1, top + 1);
          L.st[i] = (int32_t)(b - L.ro[i]);
          w = (int32_t)(e - b);
        }
        L.pre[i] = w;
      }
      wave_lds_sync();
      wave_scan_lds(L.pre, d);
      const int32_t work = L.pre[d];
      for (int32_t t = lane; t < work; t += kWave) {
        const int i = row_of(L.pre, d, t);
        const int r = t - L.pre[i];
        int q = d;
        if (L.len[i] <= 4 * d) {
          const int32_t z = T.col[L.ro[i] + L.st[i] + r];
          q = (int)lower_bound<int32_t>(L.nb, i + 1, d, z);
          if (q < d && L.nb[q] != z) q = d;
        } else {
          const int32_t z = L.nb[i + 1 + r];
          const int64_t e1 = L.ro[i] + L.len[i];
          const int64_t pos = lower_bound<int32_t>(T.col, L.ro[i], e1, z);
          if (pos < e1 && T.col[pos] == z) q = i + 1 + r;
        }
        if (q < d) {
          atomicOr(&L.A[i][q >> 5], 1u << (q & 31));
          atomicOr(&L.A[q][i >> 5], 1u << (i & 31));
        }
      }
      wave_lds_sync();
      if (!FILL && a.rows != nullptr)  // keep them for the later passes
        for (int x = lane; x < d * W; x += kWave)
          a.rows[base * kN34RowWords + x] = L.A[x / W][x % W];
    }
    if constexpr (MODE == kVRows) {  // triangles (p, nb[i], w), w > nb[i]
      for (int i = lane; i < d; i += kWave)
        if (i >= nl) a.tcnt[e_lo + (i - nl)] = popc_and<W>(L.A[i], L.A[i], i + 1, d);
      continue;
    }
    // triangles (p, nb[i], nb[j]), i >= nl, i < j: row i holds those of
    // edge (p, nb[i]), numbered from tb[i]; every row must count exactly
    // the edge's triangles, so that every id below lies in the edge's range
    bool bad = false;
    for (int i = lane; i < d; i += kWave) {
      int c = 0;
      if (i >= nl) {
        const int64_t e = e_lo + (i - nl);
        c = popc_and<W>(L.A[i], L.A[i], i + 1, d);
        L.tb[i] = (int32_t)T.toff[e];
        bad |= (int64_t)c != T.toff[e + 1] - L.tb[i];
      }
      L.pre[i] = c;
    }
    if (ballot(bad)) {  // the triangle list disagrees: write nothing
      if (lane == 0) *T.err = 1;
      continue;
    }
    wave_lds_sync();
    wave_scan_lds(L.pre, d);
    const int32_t nt = L.pre[d];
    if constexpr (MODE == kVTris) {  // third vertices ascending, per edge
      for (int32_t t = lane; t < nt; t += kWave) {
        const int i = row_of(L.pre, d, t);
        const int r = t - L.pre[i];
        const int j = nth_and<W>(L.A[i], L.A[i], i + 1, r);
        const int64_t pos = (int64_t)L.tb[i] + r;
        a.tw[pos] = L.nb[j];
        a.te[pos] = (int32_t)(e_lo + (i - nl));
      }
      continue;
    }
    if constexpr (MODE == kVCount) {
      for (int32_t t = lane; t < nt; t += kWave) {
        const int i = row_of(L.pre, d, t);
        const int r = t - L.pre[i];
        const int j = nth_and<W>(L.A[i], L.A[i], i + 1, r);
        const int64_t id = L.tb[i] + r;
        T.count[id] = popc_and<W>(L.A[i], L.A[j], 0, d);
        T.loc[id] = popc_and<W>(L.A[i], L.A[j], nl, d);
      }
      continue;
    }
    if constexpr (FILL) {
    // fill: 64 triangles (i, j) at a time, then their 4-cliques (k > j)
    for (int32_t t0 = 0; t0 < nt; t0 += kWave) {
      const int32_t t = t0 + lane;
      int i = 0, j = 0, kc = 0;
      int64_t s0 = 0;
      int32_t sn = 0;
      TriRec rt{0, 0, 0};
      if (t < nt) {
        i = row_of(L.pre, d, t);
        const int r = t - L.pre[i];
        j = nth_and<W>(L.A[i], L.A[i], i + 1, r);
        rt = T.rec[L.tb[i] + r];
        kc = popc_and<W>(L.A[i], L.A[j], j + 1, d);
        if (kc > 0) {  // the remote triangles' edge: (nb[i], nb[j])
          const int64_t e1 = L.ro[i] + L.len[i];
          const int64_t pos = lower_bound<int32_t>(T.col, L.ro[i], e1, L.nb[j]);
          if (pos < e1 && T.col[pos] == L.nb[j]) {
            const int32_t e = a.eid[pos];
            s0 = T.toff[e];
            sn = (int32_t)(T.toff[e + 1] - s0);
          } else {
            *T.err = 1;
            kc = 0;
          }
        }
      }
      int x = kc;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
      }
      const int nq = __shfl(x, kWave - 1, kWave);
      L.ci[lane] = (int16_t)i;
      L.cj[lane] = (int16_t)j;
      L.cb[lane] = rt.base;
      L.cv[lane] = rt.inv;
      L.cl[lane] = rt.len;
      L.cs0[lane] = (int32_t)s0;
      L.cn[lane] = sn;
      L.coff[lane] = x - kc;
      if (lane == 0) L.coff[kWave] = nq;
      wave_lds_sync();
      for (int q = lane; q < nq; q += kWave) {
        const int c = row_of(L.coff, kWave, q);
        const int ii = L.ci[c], jj = L.cj[c];
        const int k = nth_and<W>(L.A[ii], L.A[jj], jj + 1, q - L.coff[c]);
        const int32_t tik = (int32_t)(L.tb[ii] + popc_and<W>(L.A[ii], L.A[ii], ii + 1, k));
        const int32_t tjk = (int32_t)(L.tb[jj] + popc_and<W>(L.A[jj], L.A[jj], jj + 1, k));
        // the triangle without p: third vertex nb[k] on edge (nb[ii], nb[jj])
        const int64_t s0 = L.cs0[c], s1 = s0 + L.cn[c];
        const int64_t s = lower_bound<int32_t>(T.tri_w, s0, s1, L.nb[k]);
        int32_t top = -1;
        if (s < s1 && T.tri_w[s] == L.nb[k]) top = (int32_t)s;
        if (top < 0) {
          *T.err = 1;
          continue;
        }
        TriRec rij;
        rij.base = L.cb[c];
        rij.inv = L.cv[c];
        rij.len = L.cl[c];
        const TriRec rik = T.rec[tik], rjk = T.rec[tjk], rtop = T.rec[top];
        n34_put(T, rij, popc_and<W>(L.A[ii], L.A[jj], nl, k), rik.inv, rjk.inv, rtop.inv);
        n34_put(T, rik, popc_and<W>(L.A[ii], L.A[k], nl, jj), rij.inv, rjk.inv, rtop.inv);
        n34_put(T, rjk, popc_and<W>(L.A[jj], L.A[k], nl, ii), rij.inv, rik.inv, rtop.inv);
        const int32_t slot = atomicAdd(&T.loc[top], 1);
        n34_put(T, rtop, slot, rij.inv, rik.inv, rjk.inv);
      }
      wave_lds_sync();  // before the next chunk overwrites ci .. coff
    }
    }  // FILL
  }
}

// Degree class of vertex p before the triangles exist: 0/1/2 for degree
// <= 64/128/256 when p has at least two neighbours above it (it may be the
// lowest vertex of a triangle), 3 for a larger degree, 4 otherwise.
__global__ void k_n34_degree_bins(const int64_t *__restrict__ row_off,
                                  const int32_t *__restrict__ nlow, int32_t n,
                                  uint8_t *__restrict__ bin) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t d = row_off[p + 1] - row_off[p];
  bin[p] = nlow[p] >= d - 1 ? 4 : d <= 64 ? 0 : d <= 128 ? 1 : d <= kN34VMax ? 2 : 3;
}

// Intersection bin of the edges whose lower endpoint is too big for the
// per-vertex builder; kIsectBins (skipped) for the others.
__global__ void k_edge_bins_big_low(const int32_t *__restrict__ ev,
                                    const int64_t *__restrict__ row_off,
                                    int64_t ne, uint8_t *__restrict__ bin) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int32_t u = ev[2 * e], v = ev[2 * e + 1];
  const int64_t du = row_off[u + 1] - row_off[u], dv = row_off[v + 1] - row_off[v];
  bin[e] = du <= kN34VMax ? (uint8_t)kIsectBins : isect_bin(min(du, dv));
}

// Degree class of vertex p for the per-vertex builder: 0/1/2 for degree
// <= 64/128/256 with at least one triangle whose lowest vertex is p, 3 for
// a larger degree (its triangles go per triangle), 4 for none.
__global__ void k_n34_vertex_bins(const int64_t *__restrict__ row_off,
                                  const int64_t *__restrict__ eoff,
                                  const int64_t *__restrict__ toff, int32_t n,
                                  uint8_t *__restrict__ bin) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t d = row_off[p + 1] - row_off[p];
  const bool any = toff[eoff[p + 1]] > toff[eoff[p]];
  bin[p] = !any ? 4 : d <= 64 ? 0 : d <= 128 ? 1 : d <= kN34VMax ? 2 : 3;
}

// Intersection bin of the triangles whose lowest vertex is too big for the
// per-vertex builder; kIsectBins (skipped) for the others.
__global__ void k_n34_tri_bins(const int32_t *__restrict__ ev,
                               const int32_t *__restrict__ tri_e,
                               const int32_t *__restrict__ tri_w,
                               const int64_t *__restrict__ row_off, int64_t nt,
                               uint8_t *__restrict__ bin) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int32_t e = tri_e[t];
  const int32_t u = ev[2 * (int64_t)e], v = ev[2 * (int64_t)e + 1], w = tri_w[t];
  const int64_t du = row_off[u + 1] - row_off[u];
  if (du <= kN34VMax) {
    bin[t] = kIsectBins;
    return;
  }
  int64_t m = min(du, row_off[v + 1] - row_off[v]);
  m = min(m, row_off[w + 1] - row_off[w]);
  bin[t] = isect_bin(m);
}

// The list of every triangle t: internal id inv[t], at inc_off[inv[t]].
__global__ void k_n34_rec(const int32_t *__restrict__ inv,
                          const int64_t *__restrict__ off, int64_t nt,
                          TriRec *__restrict__ rec) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int32_t x = inv[t];
  TriRec r;
  r.base = off[x];
  r.inv = x;
  r.len = (int32_t)(off[x + 1] - r.base);
  rec[t] = r;
}

// Every list full: each remote cursor ended at its list's length.
__global__ void k_n34_check_full(const int32_t *__restrict__ cur,
                                 const TriRec *__restrict__ rec, int64_t nt,
                                 int32_t *__restrict__ err) {
  bool bad = false;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt;
       t += (int64_t)gridDim.x * blockDim.x)
    bad |= cur[t] != rec[t].len;
  if (ballot(bad) && lane_id() == 0) atomicOr(err, 1);
}

template <int D>
void launch_n34_vertex(const N34VArgs &a, int mode, unsigned grid, hipStream_t s) {
  switch (mode) {
    case kVRows: k_n34_vertex<D, kVRows><<<grid, kWave, 0, s>>>(a); break;
    case kVTris: k_n34_vertex<D, kVTris><<<grid, kWave, 0, s>>>(a); break;
    case kVCount: k_n34_vertex<D, kVCount><<<grid, kWave, 0, s>>>(a); break;
    default: k_n34_vertex<D, kVFill><<<grid, kWave, 0, s>>>(a); break;
  }
}

void run_n34_vertex(N34VArgs a, int mode, const int32_t *items,
                    const int64_t *bin_off, hipStream_t s) {
  ND_REQUIRE((mode != kVRows && mode != kVTris) || a.rows != nullptr,
             ND_ERR_DEVICE, "internal error: bit-row pass without rows");
  for (int b = 0; b < 3; b++) {
    a.items = items + bin_off[b];
    a.nitems = bin_off[b + 1] - bin_off[b];
    if (a.nitems == 0) continue;
    const unsigned grid = (unsigned)std::min<int64_t>(a.nitems, 1 << 20);
    if (b == 0) launch_n34_vertex<64>(a, mode, grid, s);
    else if (b == 1) launch_n34_vertex<128>(a, mode, grid, s);
    else launch_n34_vertex<256>(a, mode, grid, s);
    ND_LAUNCHED();
  }
}

// Edges grouped by intersection bin (host offsets in bin_off).
void edge_schedule(nd_graph *g, DArr<int32_t> &items, int64_t *bin_off,
                   hipStream_t s) {
  Allocator &al = g->ctx->alloc;
  const int64_t ne = g->ne;
  DArr<uint8_t> bin(al, ne);
  items.reset(al, ne);
  if (ne > 0) {
    k_edge_bins<<<grid_for(ne, 256), 256, 0, s>>>(g->ev.p,
                                                   g->row_off.p, ne, bin.p);
    ND_LAUNCHED();
  }
  partition_by_bin(bin.p, ne, kIsectBins, items.p, bin_off, s, al);
}

EdgeIsectArgs edge_args(nd_graph *g) {
  EdgeIsectArgs a{};
  a.ev = g->ev.p;
  a.row_off = g->row_off.p;
  a.col = g->col.p;
  a.eid = g->eid.p;
  return a;
}

}  // namespace

// k-truss incidence: every triangle is listed once by the orientation above
// and written into the lists of its three edges.  Slots inside a list are
// taken with atomic cursors, so the order of s-cliques within a list varies
// from run to run; nothing computed from the lists depends on it (min and H
// are order-free).
void build_incidence_truss(nd_graph *g, KindState &ks, hipStream_t s) {
  build_edges(g, s);
  Allocator &al = g->ctx->alloc;
  const int64_t ne = g->ne, nnz = g->nnz;
  const int32_t n = g->n;
  DArr<int32_t> flag(al, nnz);
  DArr<int64_t> pos(al, nnz + 1);
  if (nnz > 0) {
    k_orient_flags<<<grid_for(nnz, 256), 256, 0, s>>>(g->row_off.p, g->col.p,
                                                       g->rowid.p, nnz, flag.p);
    ND_LAUNCHED();
  }
  exclusive_scan_i32(flag.p, pos.p, nnz, s, al);  // ne oriented entries
  DArr<int32_t> out_col(al, ne), out_eid(al, ne), out_src(al, ne);
  DArr<int64_t> out_off(al, (int64_t)n + 1);
  if (nnz > 0) {
    k_orient_fill<<<grid_for(nnz, 256), 256, 0, s>>>(
        g->col.p, g->rowid.p, g->eid.p, flag.p, pos.p, nnz, out_col.p,
        out_eid.p, out_src.p);
    ND_LAUNCHED();
  }
  flag.free();
  pos.free();
  k_orient_off<<<grid_for((int64_t)n + 1, 256), 256, 0, s>>>(out_src.p, ne, n,
                                                              out_off.p);
  ND_LAUNCHED();
  // oriented edges binned by their shorter out-list
  DArr<uint8_t> bin(al, ne);
  DArr<int32_t> items(al, ne), cap(al, ne);
  if (ne > 0) {
    k_orient_bins<<<grid_for(ne, 256), 256, 0, s>>>(out_off.p, out_col.p,
                                                     out_src.p, ne, bin.p,
                                                     cap.p);
    ND_LAUNCHED();
  }
  int64_t bin_off[5];
  partition_by_bin(bin.p, ne, 4, items.p, bin_off, s, al);
  bin.free();
  // Room for every triangle the count pass can find (the shorter out-list
  // bounds each edge's), so that the fill pass reads them back instead of
  // intersecting again.  The fill intersects again above kTriBufMax, or
  // under a device-memory budget when the buffer would take more than a
  // quarter of what is left of it (other work on the context, such as a
  // server preparing graphs while its caller builds more, keeps room).
  constexpr int64_t kTriBufMax = (int64_t)1 << 32;  // entries (32 GiB)
  DArr<int64_t> tri_off(al, ne + 1);
  exclusive_scan_i32(cap.p, tri_off.p, ne, s, al);
  cap.free();
  const int64_t tri_cap = read_i64(tri_off.p + ne, s);
  DArr<int2> tri_buf;
  const size_t tri_bytes = sizeof(int2) * (size_t)std::max<int64_t>(tri_cap, 1);
  const size_t live = al.live_bytes();
  const char *no_buf = getenv("ND_TRUSS_NO_TRIBUF");
  if (!(no_buf && no_buf[0] == '1') && tri_cap <= kTriBufMax &&
      (al.budget() == 0 ||
       (live < al.budget() && tri_bytes <= (al.budget() - live) / 4))) {
    try {
      tri_buf.reset(al, tri_cap);
    } catch (const Err &) {  // the device is short of memory: intersect twice
      tri_buf.p = nullptr;
    }
  }
  if (!tri_buf.p) tri_off.free();
  OrientArgs a{};
  a.out_off = out_off.p;
  a.out_col = out_col.p;
  a.out_eid = out_eid.p;
  a.out_src = out_src.p;
  // the 64-lane bin by source, when every out-list fits the LDS copy
  HeavySegs hs;
  const int64_t n3 = bin_off[4] - bin_off[3];
  if (n3 > 0) {
    DArr<int32_t> mx(al, 1);
    fill_i32(mx.p, 0, 1, s);
    k_max_outdeg<<<std::min<unsigned>(grid_for(n, 256), 1024), 256, 0, s>>>(
        out_off.p, n, mx.p);
    ND_LAUNCHED();
    const int32_t hmax = *PinnedChunk().read(mx.p, 1, s);
    constexpr int kMaxLdsEntries = 5120;  // 60 KiB: three int32 arrays
    const char *no_lds = getenv("ND_TRUSS_NO_LDS");
    if (hmax <= kMaxLdsEntries && !(no_lds && no_lds[0] == '1')) {
      a.lds_cap = std::max(hmax, 1);
      const int32_t *it3 = items.p + bin_off[3];
      DArr<int32_t> flag3(al, n3);
      DArr<int64_t> pos3(al, n3 + 1);
      k_seg_flags<<<grid_for(n3, 256), 256, 0, s>>>(it3, n3, out_src.p, flag3.p);
      ND_LAUNCHED();
      exclusive_scan_i32(flag3.p, pos3.p, n3, s, al);
      hs.n = read_i64(pos3.p + n3, s);
      hs.lo.reset(al, std::max<int64_t>(hs.n, 1));
      k_seg_fill<<<grid_for(n3, 256), 256, 0, s>>>(flag3.p, pos3.p, n3, hs.lo.p);
      ND_LAUNCHED();
    }
  }
  DArr<int32_t> cnt(al, ne), cbase(al, ne);
  fill_i32(cnt.p, 0, ne, s);
  a.count = cnt.p;
  a.count_base = cbase.p;  // every oriented edge stores its own
  a.tri_off = tri_buf.p ? tri_off.p : nullptr;
  a.tri_buf = tri_buf.p;
  // per-source side counts of k_orient_heavy; with the triangle buffer each
  // edge's list keeps those slots right after its base entries
  DArr<int32_t> hcount;
  if (a.lds_cap > 0) {
    hcount.reset(al, ne);
    fill_i32(hcount.p, 0, ne, s);
    a.hcount = hcount.p;
  }
  {
    Phase phase("nd.incidence.count");
    run_orient<false>(a, items.p, bin_off, hs, s);
  }
  if (hcount.p) {
    k_add_i32<<<grid_for(ne, 256), 256, 0, s>>>(cnt.p, hcount.p, ne);
    ND_LAUNCHED();
  }
  ks.nr = ne;
  build_layout(g, ks, cnt.p, s);
  cnt.free();
  ks.inc_ids.reset(al, 2 * ks.P);
  DArr<unsigned long long> cursor(al, ne);
  if (ne > 0) {
    k_cursor_init<<<grid_for(ne, 256), 256, 0, s>>>(
        ks.inc_off.p, ks.perm.p, cbase.p, tri_buf.p ? hcount.p : nullptr, ne,
        cursor.p);
    ND_LAUNCHED();
  }
  a.inv = ks.inv.p;
  a.cursor = cursor.p;
  a.ids = ks.inc_ids.p;
  a.base_off = ks.inc_off.p;
  Phase fill_phase("nd.incidence.fill");
  if (tri_buf.p)
    run_scatter(a, items.p, bin_off, hs, s);
  else
    run_orient<true>(a, items.p, bin_off, hs, s);
}

void build_triangles(nd_graph *g, hipStream_t s) {
  if (g->tris_ready) return;
  build_edges(g, s);
  Phase phase("nd.triangles");
  Allocator &al = g->ctx->alloc;
  const int64_t ne = g->ne;
  DArr<int32_t> items;
  int64_t bin_off[kIsectBins + 1];
  edge_schedule(g, items, bin_off, s);
  DArr<int32_t> cnt(al, ne);
  EdgeIsectArgs a = edge_args(g);
  a.count = cnt.p;
  run_edge_isect<kCountTri>(a, items.p, bin_off, s);
  g->toff.reset(al, ne + 1);
  exclusive_scan_i32(cnt.p, g->toff.p, ne, s, al);
  g->nt = read_i64(g->toff.p + ne, s);
  ND_REQUIRE(g->nt < ((int64_t)1 << 31), ND_ERR_INVALID,
             "%lld triangles: triangle ids must fit int32", (long long)g->nt);
  g->tri_w.reset(al, g->nt);
  g->tri_e.reset(al, g->nt);
  a.off = g->toff.p;
  a.out_a = g->tri_w.p;
  a.out_b = g->tri_e.p;
  run_edge_isect<kFillTri>(a, items.p, bin_off, s);
  g->tris_ready = true;
}

// The triangle list (the same arrays, in the same order, as build_triangles)
// from the per-vertex bit rows, which stay in `rows` for the (3,4) passes
// that follow: a wave per vertex p of degree <= kN34VMax counts, then lists,
// the triangles of each edge (p, v), v > p, from row v's bits above v; the
// edges whose lower endpoint has a larger degree are intersected as in
// build_triangles.
void build_triangles_rows(nd_graph *g, uint32_t *rows, hipStream_t s) {
  build_edges(g, s);
  Phase phase("nd.triangles");
  Allocator &al = g->ctx->alloc;
  const int32_t n = g->n;
  const int64_t ne = g->ne;
  DArr<uint8_t> vbin(al, std::max<int32_t>(n, 1));
  DArr<int32_t> vitems(al, std::max<int32_t>(n, 1));
  if (n > 0) {
    k_n34_degree_bins<<<grid_for(n, 256), 256, 0, s>>>(g->row_off.p, g->nlow.p, n,
                                                        vbin.p);
    ND_LAUNCHED();
  }
  int64_t voff[6];
  partition_by_bin(vbin.p, n, 5, vitems.p, voff, s, al);
  vbin.free();
  DArr<int32_t> eitems(al, std::max<int64_t>(ne, 1));
  int64_t ebin_off[kIsectBins + 2] = {0};
  if (voff[4] > voff[3]) {  // edges below a vertex too big for the rows
    DArr<uint8_t> ebin(al, std::max<int64_t>(ne, 1));
    k_edge_bins_big_low<<<grid_for(ne, 256), 256, 0, s>>>(g->ev.p, g->row_off.p,
                                                           ne, ebin.p);
    ND_LAUNCHED();
    partition_by_bin(ebin.p, ne, kIsectBins + 1, eitems.p, ebin_off, s, al);
  }
  DArr<int32_t> cnt(al, std::max<int64_t>(ne, 1)), err(al, 1);
  fill_i32(cnt.p, 0, ne, s);  // edges below a vertex without two upper ones
  fill_i32(err.p, 0, 1, s);
  EdgeIsectArgs ea = edge_args(g);
  ea.count = cnt.p;
  run_edge_isect<kCountTri>(ea, eitems.p, ebin_off, s);
  N34VArgs va{};
  va.row_off = g->row_off.p;
  va.col = g->col.p;
  va.eid = g->eid.p;
  va.nlow = g->nlow.p;
  va.eoff = g->eoff.p;
  va.rows = rows;
  va.tcnt = cnt.p;
  va.t.col = g->col.p;
  va.t.err = err.p;
  run_n34_vertex(va, kVRows, vitems.p, voff, s);
  g->toff.reset(al, ne + 1);
  exclusive_scan_i32(cnt.p, g->toff.p, ne, s, al);
  cnt.free();
  g->nt = read_i64(g->toff.p + ne, s);
  ND_REQUIRE(g->nt < ((int64_t)1 << 31), ND_ERR_INVALID,
             "%lld triangles: triangle ids must fit int32", (long long)g->nt);
  g->tri_w.reset(al, g->nt);
  g->tri_e.reset(al, g->nt);
  va.rows_ready = 1;
  va.t.toff = g->toff.p;
  va.tw = g->tri_w.p;
  va.te = g->tri_e.p;
  run_n34_vertex(va, kVTris, vitems.p, voff, s);
  ea.off = g->toff.p;
  ea.out_a = g->tri_w.p;
  ea.out_b = g->tri_e.p;
  run_edge_isect<kFillTri>(ea, eitems.p, ebin_off, s);
  const int32_t h = *PinnedChunk().read(err.p, 1, s);
  ND_REQUIRE(h == 0, ND_ERR_DEVICE,
             "internal error: the triangle counts of the bit rows disagree");
  g->tris_ready = true;
}

// (3,4) incidence: each 4-clique is written once, by the builder of its
// lowest vertex (per vertex for degrees up to kN34VMax, else per triangle),
// into the lists of its four triangles: the three that contain that vertex
// at ranks known from the count pass, the fourth at a cursor.
void build_incidence_n34(nd_graph *g, KindState &ks, hipStream_t s) {
  Allocator &al = g->ctx->alloc;
  // the bit rows of every vertex of degree <= kN34VMax, built once (with the
  // triangles when those do not exist yet, else by the count pass) and read
  // back by the later passes; skipped when they would take more than a
  // quarter of the budget left (every pass then builds them again)
  DArr<uint32_t> rows;
  const size_t rows_bytes =
      sizeof(uint32_t) * kN34RowWords * (size_t)std::max<int64_t>(g->nnz, 1);
  const size_t live = al.live_bytes();
  const char *no_rows = getenv("ND_N34_NO_ROWS");
  if (g->nnz > 0 && !(no_rows && no_rows[0] == '1') &&
      (al.budget() == 0 ||
       (live < al.budget() && rows_bytes <= (al.budget() - live) / 4))) {
    try {
      rows.reset(al, std::max<int64_t>(g->nnz, 1) * kN34RowWords);
    } catch (const Err &) {  // the device is short of memory
      rows.p = nullptr;
    }
  }
  bool rows_ready = false;
  if (!g->tris_ready && rows.p) {
    build_triangles_rows(g, rows.p, s);
    rows_ready = true;
  }
  build_triangles(g, s);
  const int64_t nt = g->nt;
  const int32_t n = g->n;
  // vertices by degree class; triangles of the big ones by intersection bin
  DArr<uint8_t> vbin(al, std::max<int32_t>(n, 1));
  DArr<int32_t> vitems(al, std::max<int32_t>(n, 1));
  if (n > 0) {
    k_n34_vertex_bins<<<grid_for(n, 256), 256, 0, s>>>(g->row_off.p, g->eoff.p,
                                                        g->toff.p, n, vbin.p);
    ND_LAUNCHED();
  }
  int64_t voff[6];
  partition_by_bin(vbin.p, n, 5, vitems.p, voff, s, al);
  vbin.free();
  DArr<uint8_t> bin(al, std::max<int64_t>(nt, 1));
  DArr<int32_t> items(al, std::max<int64_t>(nt, 1));
  int64_t bin_off[kIsectBins + 2] = {0};
  if (voff[4] > voff[3]) {  // vertices too big for the per-vertex builder
    k_n34_tri_bins<<<grid_for(nt, 256), 256, 0, s>>>(g->ev.p, g->tri_e.p,
                                                      g->tri_w.p, g->row_off.p,
                                                      nt, bin.p);
    ND_LAUNCHED();
    partition_by_bin(bin.p, nt, kIsectBins + 1, items.p, bin_off, s, al);
  }
  bin.free();
  DArr<int32_t> cnt(al, std::max<int64_t>(nt, 1)), loc(al, std::max<int64_t>(nt, 1));
  DArr<int32_t> err(al, 1);
  fill_i32(err.p, 0, 1, s);
  TriIsectArgs a{};
  a.ev = g->ev.p;
  a.row_off = g->row_off.p;
  a.col = g->col.p;
  a.eid = g->eid.p;
  a.toff = g->toff.p;
  a.tri_w = g->tri_w.p;
  a.tri_e = g->tri_e.p;
  a.count = cnt.p;
  a.loc = loc.p;
  a.err = err.p;
  N34VArgs va{};
  va.row_off = g->row_off.p;
  va.col = g->col.p;
  va.eid = g->eid.p;
  va.nlow = g->nlow.p;
  va.eoff = g->eoff.p;
  va.t = a;
  va.rows = rows.p;
  va.rows_ready = rows_ready ? 1 : 0;
  {
    Phase phase("nd.incidence.count");
    run_n34_vertex(va, kVCount, vitems.p, voff, s);
    run_n34_tri(a, false, items.p, bin_off, s);
  }
  ks.nr = nt;
  build_layout(g, ks, cnt.p, s);
  cnt.free();
  ks.inc_ids.reset(al, 3 * ks.P);
  DArr<TriRec> rec(al, std::max<int64_t>(nt, 1));
  if (nt > 0) {
    k_n34_rec<<<grid_for(nt, 256), 256, 0, s>>>(ks.inv.p, ks.inc_off.p, nt, rec.p);
    ND_LAUNCHED();
  }
  a.count = nullptr;
  a.rec = rec.p;  // loc: now the remote cursors
  a.out = ks.inc_ids.p;
  va.t = a;
  Phase fill_phase("nd.incidence.fill");
  run_n34_vertex(va, kVFill, vitems.p, voff, s);
  rows.free();
  run_n34_tri(a, true, items.p, bin_off, s);
  if (nt > 0) {
    const unsigned grid = (unsigned)std::min<int64_t>(grid_for(nt, 256), 65536);
    k_n34_check_full<<<grid, 256, 0, s>>>(loc.p, rec.p, nt, err.p);
    ND_LAUNCHED();
  }
  const int32_t h = *PinnedChunk().read(err.p, 1, s);
  ND_REQUIRE(h == 0, ND_ERR_DEVICE,
             "internal error: the (3,4) incidence lists are inconsistent");
}

// ------------------------------------------------------- (1,3) and (2,4)
//
// The generic variants of Section 5 listed from the triangles: for (1,3) a
// vertex's s-cliques are its triangles (the other two vertices listed); for
// (2,4) an edge's s-cliques are its 4-cliques (the other five edges listed).
// Counts and slots come from atomics, so list order varies from run to run.

namespace {

__global__ void k_n13_count(const int32_t *__restrict__ ev,
                            const int32_t *__restrict__ tri_e,
                            const int32_t *__restrict__ tri_w, int64_t nt,
                            int32_t *__restrict__ cnt) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = tri_e[t];
    atomicAdd(&cnt[ev[2 * e]], 1);
    atomicAdd(&cnt[ev[2 * e + 1]], 1);
    atomicAdd(&cnt[tri_w[t]], 1);
  }
}

// Triangle (u,v,w) into the lists of u, v and w, each entry the two other
// vertices (internal ids).
__global__ void k_n13_fill(const int32_t *__restrict__ ev,
                           const int32_t *__restrict__ tri_e,
                           const int32_t *__restrict__ tri_w, int64_t nt,
                           const int32_t *__restrict__ inv,
                           unsigned long long *__restrict__ cursor,
                           int32_t *__restrict__ ids) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = tri_e[t];
    const int32_t x[3] = {inv[ev[2 * e]], inv[ev[2 * e + 1]], inv[tri_w[t]]};
#pragma unroll
    for (int i = 0; i < 3; i++) {
      const int64_t p = (int64_t)atomicAdd(&cursor[x[i]], 1ull);
      ids[2 * p] = x[(i + 1) % 3];
      ids[2 * p + 1] = x[(i + 2) % 3];
    }
  }
}

struct K4Args {
  const int32_t *items;  // triangle ids of this bin
  int64_t nitems;
  const int32_t *ev;
  const int64_t *row_off;
  const int32_t *col;
  const int32_t *eid;
  const int32_t *tri_e;
  const int32_t *tri_w;
  int32_t *count;               // count pass: 4-cliques per edge id
  const int32_t *inv;           // fill pass: edge id -> internal id
  unsigned long long *cursor;   // fill pass: next slot per internal id
  int32_t *ids;                 // fill pass: 5 ids per (edge, 4-clique)
};

// Every 4-clique {u,v,w,x}, u<v<w<x, is found once, from its lowest
// triangle (u,v,w): x runs over the common neighbours of u, v and w above w.
// G lanes per triangle stride over the shortest of the three lists (from its
// first entry above w) and binary-search the other two.
template <int G, bool FILL>
__global__ __launch_bounds__(256) void k_k4_list(K4Args a) {
  const int sl = lane_id() % G;
  const int64_t nsub = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t gsub = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
       gsub < a.nitems; gsub += nsub) {
    const int32_t t = a.items[gsub];
    const int32_t euv = a.tri_e[t];
    const int32_t u = a.ev[2 * (int64_t)euv], v = a.ev[2 * (int64_t)euv + 1];
    const int32_t w = a.tri_w[t];
    const int64_t b[3] = {a.row_off[u], a.row_off[v], a.row_off[w]};
    const int64_t en[3] = {a.row_off[u + 1], a.row_off[v + 1], a.row_off[w + 1]};
    int sh = 0;
    if (en[1] - b[1] < en[sh] - b[sh]) sh = 1;
    if (en[2] - b[2] < en[sh] - b[sh]) sh = 2;
    const int o1 = sh == 0 ? 1 : 0, o2 = sh == 2 ? 1 : 2;
    const int64_t start = lower_bound<int32_t>(a.col, b[sh], en[sh], w + 1);
    if (start >= en[sh]) continue;  // uniform within the subgroup
    const int32_t euw = a.eid[lower_bound<int32_t>(a.col, b[0], en[0], w)];
    const int32_t evw = a.eid[lower_bound<int32_t>(a.col, b[1], en[1], w)];
    for (int64_t j = start + sl; j < en[sh]; j += G) {
      const int32_t x = a.col[j];
      const int64_t q1 = lower_bound<int32_t>(a.col, b[o1], en[o1], x);
      if (q1 >= en[o1] || a.col[q1] != x) continue;
      const int64_t q2 = lower_bound<int32_t>(a.col, b[o2], en[o2], x);
      if (q2 >= en[o2] || a.col[q2] != x) continue;
      int64_t pos[3];
      pos[sh] = j;
      pos[o1] = q1;
      pos[o2] = q2;
      // the six edges: uv, uw, vw, ux, vx, wx
      const int32_t e6[6] = {euv, euw, evw, a.eid[pos[0]], a.eid[pos[1]],
                             a.eid[pos[2]]};
      if (!FILL) {
#pragma unroll
        for (int i = 0; i < 6; i++) atomicAdd(&a.count[e6[i]], 1);
      } else {
        int32_t ie[6];
#pragma unroll
        for (int i = 0; i < 6; i++) ie[i] = a.inv[e6[i]];
#pragma unroll
        for (int i = 0; i < 6; i++) {
          const int64_t p = (int64_t)atomicAdd(&a.cursor[ie[i]], 1ull);
          int32_t *o = a.ids + 5 * p;
          int c = 0;
#pragma unroll
          for (int q = 0; q < 6; q++)
            if (q != i) o[c++] = ie[q];
        }
      }
    }
  }
}

template <bool FILL>
void run_k4(K4Args a, const int32_t *items, const int64_t *bin_off,
            hipStream_t s) {
  for (int b = 0; b < kIsectBins; b++) {
    a.items = items + bin_off[b];
    a.nitems = bin_off[b + 1] - bin_off[b];
    if (a.nitems == 0) continue;
    switch (b) {
      case 0: k_k4_list<1, FILL><<<grid_stride(a.nitems, 1), 256, 0, s>>>(a); break;
      case 1: k_k4_list<4, FILL><<<grid_stride(a.nitems, 4), 256, 0, s>>>(a); break;
      case 2: k_k4_list<16, FILL><<<grid_stride(a.nitems, 16), 256, 0, s>>>(a); break;
      default: k_k4_list<64, FILL><<<grid_stride(a.nitems, 64), 256, 0, s>>>(a); break;
    }
    ND_LAUNCHED();
  }
}

}  // namespace

void build_incidence_n13(nd_graph *g, KindState &ks, hipStream_t s) {
  build_triangles(g, s);
  Allocator &al = g->ctx->alloc;
  const int64_t nt = g->nt;
  const int32_t n = g->n;
  DArr<int32_t> cnt(al, n);
  fill_i32(cnt.p, 0, n, s);
  if (nt > 0) {
    k_n13_count<<<grid_stride(nt, 1), 256, 0, s>>>(g->ev.p, g->tri_e.p,
                                                   g->tri_w.p, nt, cnt.p);
    ND_LAUNCHED();
  }
  ks.nr = n;
  build_layout(g, ks, cnt.p, s);
  cnt.free();
  ks.inc_ids.reset(al, 2 * ks.P);
  DArr<unsigned long long> cursor(al, n);
  if (n > 0) {
    k_cursor_init<<<grid_for(n, 256), 256, 0, s>>>(ks.inc_off.p, ks.perm.p,
                                                    nullptr, nullptr, n, cursor.p);
    ND_LAUNCHED();
  }
  if (nt > 0) {
    k_n13_fill<<<grid_stride(nt, 1), 256, 0, s>>>(g->ev.p, g->tri_e.p,
                                                  g->tri_w.p, nt, ks.inv.p,
                                                  cursor.p, ks.inc_ids.p);
    ND_LAUNCHED();
  }
}

void build_incidence_n24(nd_graph *g, KindState &ks, hipStream_t s) {
  build_triangles(g, s);
  Allocator &al = g->ctx->alloc;
  const int64_t nt = g->nt, ne = g->ne;
  DArr<uint8_t> bin(al, nt);
  DArr<int32_t> items(al, nt);
  if (nt > 0) {
    k_tri_bins<<<grid_for(nt, 256), 256, 0, s>>>(g->ev.p, g->tri_e.p,
                                                  g->tri_w.p, g->row_off.p, nt,
                                                  bin.p);
    ND_LAUNCHED();
  }
  int64_t bin_off[kIsectBins + 1];
  partition_by_bin(bin.p, nt, kIsectBins, items.p, bin_off, s, al);
  bin.free();
  DArr<int32_t> cnt(al, ne);
  fill_i32(cnt.p, 0, ne, s);
  K4Args a{};
  a.ev = g->ev.p;
  a.row_off = g->row_off.p;
  a.col = g->col.p;
  a.eid = g->eid.p;
  a.tri_e = g->tri_e.p;
  a.tri_w = g->tri_w.p;
  a.count = cnt.p;
  run_k4<false>(a, items.p, bin_off, s);
  ks.nr = ne;
  build_layout(g, ks, cnt.p, s);
  cnt.free();
  ks.inc_ids.reset(al, 5 * ks.P);
  DArr<unsigned long long> cursor(al, ne);
  if (ne > 0) {
    k_cursor_init<<<grid_for(ne, 256), 256, 0, s>>>(ks.inc_off.p, ks.perm.p,
                                                     nullptr, nullptr, ne, cursor.p);
    ND_LAUNCHED();
  }
  a.inv = ks.inv.p;
  a.cursor = cursor.p;
  a.ids = ks.inc_ids.p;
  run_k4<true>(a, items.p, bin_off, s);
}

// ------------------------------------------------------------- (1,2)

namespace {

__global__ void k_degree(const int64_t *__restrict__ row_off, int32_t n,
                         int32_t *__restrict__ deg) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) deg[u] = (int32_t)(row_off[u + 1] - row_off[u]);
}

// The neighbour list of vertex perm[i], re-indexed, at inc_off[i].
template <int G>
__global__ __launch_bounds__(256) void k_csr_fill(
    const int64_t *__restrict__ row_off, const int32_t *__restrict__ col,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ inv,
    const int64_t *__restrict__ off, int64_t lo, int64_t hi,
    int32_t *__restrict__ out) {
  const int sl = lane_id() % G;
  const int64_t nsub = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t i = lo + ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
       i < hi; i += nsub) {
    const int32_t u = perm[i];
    const int64_t b = row_off[u], d = row_off[u + 1] - b, o = off[i];
    for (int64_t j = sl; j < d; j += G) out[o + j] = inv[col[b + j]];
  }
}

}  // namespace

void build_incidence_core(nd_graph *g, KindState &ks, hipStream_t s) {
  Allocator &al = g->ctx->alloc;
  const int32_t n = g->n;
  DArr<int32_t> deg(al, n);
  if (n > 0) {
    k_degree<<<grid_for(n, 256), 256, 0, s>>>(g->row_off.p, n, deg.p);
    ND_LAUNCHED();
  }
  ks.nr = n;
  build_layout(g, ks, deg.p, s);
  deg.free();
  ks.inc_ids.reset(al, ks.P);
  // high-degree vertices first in the internal order: a wave each; the rest
  // four lanes each
  const int64_t split = ks.bin_hi[kBinG64];
  if (split > 0) {
    k_csr_fill<64><<<grid_stride(split, 64), 256, 0, s>>>(
        g->row_off.p, g->col.p, ks.perm.p, ks.inv.p, ks.inc_off.p, 0, split,
        ks.inc_ids.p);
    ND_LAUNCHED();
  }
  if (n > split) {
    k_csr_fill<4><<<grid_stride(n - split, 4), 256, 0, s>>>(
        g->row_off.p, g->col.p, ks.perm.p, ks.inv.p, ks.inc_off.p, split, n,
        ks.inc_ids.p);
    ND_LAUNCHED();
  }
}

}  // namespace nd
