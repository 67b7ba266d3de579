// graph.hip -- the simple undirected graph on the device (Section 2):
// canonical CSR from a raw edge list (self-loops dropped, repeated pairs
// merged, adjacency sorted), validation of a caller-supplied CSR, the row of
// every adjacency entry, and the lexicographic numbering of edges (the
// r-cliques of the k-truss case).
#include "internal.h"

namespace nd {

namespace {

// Bits needed to hold values 0..x.
int bits_for(int64_t x) {
  int b = 1;
  while (b < 62 && ((int64_t)1 << b) <= x) b++;
  return b;
}

// Each raw pair {a,b}, a != b, becomes the two directed keys a<<bv|b and
// b<<bv|a.  Self-loops become the all-ones sentinel, which no real key can
// equal (it would need a == b) and which sorts last.
__global__ void k_make_keys(const int32_t *__restrict__ src,
                            const int32_t *__restrict__ dst, int64_t m,
                            int32_t n, int bv, uint64_t sentinel,
                            uint64_t *__restrict__ keys,
                            int32_t *__restrict__ err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int32_t a = src[i], b = dst[i];
  uint64_t k0 = sentinel, k1 = sentinel;
  if (a < 0 || a >= n || b < 0 || b >= n) {
    atomicOr(err, 1);
  } else if (a != b) {
    k0 = ((uint64_t)a << bv) | (uint64_t)b;
    k1 = ((uint64_t)b << bv) | (uint64_t)a;
  }
  keys[2 * i] = k0;
  keys[2 * i + 1] = k1;
}

__global__ void k_unique_flags(const uint64_t *__restrict__ keys, int64_t n,
                               uint64_t sentinel, int32_t *__restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k = keys[i];
  flag[i] = (k != sentinel && (i == 0 || keys[i - 1] != k)) ? 1 : 0;
}

__global__ void k_compact(const uint64_t *__restrict__ keys, int64_t n, int bv,
                          const int32_t *__restrict__ flag,
                          const int64_t *__restrict__ pos,
                          int32_t *__restrict__ col,
                          int32_t *__restrict__ rowid) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  uint64_t k = keys[i];
  int64_t p = pos[i];
  col[p] = (int32_t)(k & (((uint64_t)1 << bv) - 1));
  rowid[p] = (int32_t)(k >> bv);
}

// row_off[x] = first entry whose row is >= x, for x in [0, n].
__global__ void k_row_off(const int32_t *__restrict__ rowid, int64_t nnz,
                          int32_t n, int64_t *__restrict__ row_off) {
  int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x > n) return;
  row_off[x] = lower_bound<int32_t>(rowid, 0, nnz, (int32_t)x);
}

// Row structure of a caller CSR: row_off[0] = 0, non-decreasing, ends at nnz.
__global__ void k_check_rows(const int64_t *__restrict__ row_off, int32_t n,
                             int64_t nnz, int32_t *__restrict__ err) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u > n) return;
  int64_t a = row_off[u];
  if (u == 0 && a != 0) atomicOr(err, 1);
  if (u == n && a != nnz) atomicOr(err, 2);
  if (u < n && row_off[u + 1] < a) atomicOr(err, 4);
}

// Row of every entry: the u with row_off[u] <= p < row_off[u+1].
__global__ void k_rowid(const int64_t *__restrict__ row_off, int32_t n,
                        int64_t nnz, int32_t *__restrict__ rowid) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  // last u with row_off[u] <= p
  int64_t lo = 0, hi = n;  // answer in [0, n-1]
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (row_off[mid] <= p)
      lo = mid;
    else
      hi = mid - 1;
  }
  rowid[p] = (int32_t)lo;
}

// Entry-level checks: ids in range, no self-loop, strictly ascending rows,
// and symmetry (u must appear in N(v)).
__global__ void k_check_entries(const int64_t *__restrict__ row_off,
                                const int32_t *__restrict__ col,
                                const int32_t *__restrict__ rowid, int32_t n,
                                int64_t nnz, int32_t *__restrict__ err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  int32_t u = rowid[p], v = col[p];
  if (v < 0 || v >= n) {
    atomicOr(err, 8);
    return;
  }
  if (v == u) atomicOr(err, 16);
  if (p + 1 < row_off[u + 1] && col[p + 1] <= v) atomicOr(err, 32);
  int64_t b = row_off[v], e = row_off[v + 1];
  int64_t q = lower_bound<int32_t>(col, b, e, u);
  if (q >= e || col[q] != u) atomicOr(err, 64);
}

// Neighbours below u (u itself is never in N(u)).
__global__ void k_nlow(const int64_t *__restrict__ row_off,
                       const int32_t *__restrict__ col, int32_t n,
                       int32_t *__restrict__ nlow, int32_t *__restrict__ nup) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int64_t b = row_off[u], e = row_off[u + 1];
  int64_t q = lower_bound<int32_t>(col, b, e, (int32_t)u);
  nlow[u] = (int32_t)(q - b);
  nup[u] = (int32_t)(e - q);
}

// Edge (u,v), u < v, has id eoff[u] + (its rank among u's higher
// neighbours): the lexicographic order of the pairs.
__global__ void k_eid(const int64_t *__restrict__ row_off,
                      const int32_t *__restrict__ col,
                      const int32_t *__restrict__ rowid,
                      const int32_t *__restrict__ nlow,
                      const int64_t *__restrict__ eoff, int64_t nnz,
                      int32_t *__restrict__ eid, int32_t *__restrict__ ev) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  int32_t u = rowid[p], v = col[p];
  int64_t id;
  if (v > u) {
    id = eoff[u] + (p - row_off[u] - nlow[u]);
    ev[2 * id] = u;
    ev[2 * id + 1] = v;
  } else {
    int64_t q = lower_bound<int32_t>(col, row_off[v], row_off[v + 1], u);
    id = eoff[v] + (q - row_off[v] - nlow[v]);
  }
  eid[p] = (int32_t)id;
}

}  // namespace

void build_from_edges(nd_graph *g, int64_t m, const int32_t *src,
                      const int32_t *dst, hipStream_t s) {
  Allocator &al = g->ctx->alloc;
  const int32_t n = g->n;
  const int bv = bits_for(n > 0 ? n - 1 : 0);
  const int total_bits = 2 * bv;
  const uint64_t sentinel = (total_bits >= 64) ? ~0ull
                                               : (((uint64_t)1 << total_bits) - 1);
  const int64_t nk = 2 * m;
  DArr<int32_t> err(al, 1);
  fill_i32(err.p, 0, 1, s);
  DArr<uint64_t> keys(al, nk), tmp(al, nk);
  if (m > 0) {
    k_make_keys<<<grid_for(m, 256), 256, 0, s>>>(src, dst, m, n, bv, sentinel,
                                                  keys.p, err.p);
    ND_LAUNCHED();
  }
  const int32_t herr = *PinnedChunk().read(err.p, 1, s);
  ND_REQUIRE(herr == 0, ND_ERR_INVALID,
             "edge list has an endpoint outside [0, %d)", n);
  uint64_t *sorted = radix_sort_u64(keys.p, tmp.p, nk, 0, total_bits, s, al);
  DArr<int32_t> flag(al, nk);
  DArr<int64_t> pos(al, nk + 1);
  if (nk > 0) {
    k_unique_flags<<<grid_for(nk, 256), 256, 0, s>>>(sorted, nk, sentinel,
                                                      flag.p);
    ND_LAUNCHED();
  }
  exclusive_scan_i32(flag.p, pos.p, nk, s, al);
  const int64_t nnz = read_i64(pos.p + nk, s);
  g->nnz = nnz;
  g->col.reset(al, nnz);
  g->rowid.reset(al, nnz);
  g->row_off.reset(al, (int64_t)n + 1);
  if (nk > 0) {
    k_compact<<<grid_for(nk, 256), 256, 0, s>>>(sorted, nk, bv, flag.p, pos.p,
                                                 g->col.p, g->rowid.p);
    ND_LAUNCHED();
  }
  k_row_off<<<grid_for((int64_t)n + 1, 256), 256, 0, s>>>(g->rowid.p, nnz, n,
                                                           g->row_off.p);
  ND_LAUNCHED();
}

void validate_csr(nd_graph *g, hipStream_t s) {
  Allocator &al = g->ctx->alloc;
  DArr<int32_t> err(al, 1);
  fill_i32(err.p, 0, 1, s);
  k_check_rows<<<grid_for((int64_t)g->n + 1, 256), 256, 0, s>>>(
      g->row_off.p, g->n, g->nnz, err.p);
  ND_LAUNCHED();
  int32_t herr = *PinnedChunk().read(err.p, 1, s);
  ND_REQUIRE(herr == 0, ND_ERR_INVALID,
             "CSR row offsets malformed (flags 0x%x: 1 first != 0, 2 last != "
             "nnz, 4 decreasing)", herr);
  build_rowid(g, s);
  if (g->nnz > 0) {
    k_check_entries<<<grid_for(g->nnz, 256), 256, 0, s>>>(
        g->row_off.p, g->col.p, g->rowid.p, g->n, g->nnz, err.p);
    ND_LAUNCHED();
  }
  herr = *PinnedChunk().read(err.p, 1, s);
  ND_REQUIRE(herr == 0, ND_ERR_INVALID,
             "CSR is not a canonical simple graph (flags 0x%x: 8 id out of "
             "range, 16 self-loop, 32 row not strictly ascending, 64 not "
             "symmetric)", herr);
}

void build_rowid(nd_graph *g, hipStream_t s) {
  g->rowid.reset(g->ctx->alloc, g->nnz);
  if (g->nnz == 0) return;
  k_rowid<<<grid_for(g->nnz, 256), 256, 0, s>>>(g->row_off.p, g->n, g->nnz,
                                                 g->rowid.p);
  ND_LAUNCHED();
}

void build_edges(nd_graph *g, hipStream_t s) {
  if (g->edges_ready) return;
  Phase phase("nd.edges");
  Allocator &al = g->ctx->alloc;
  const int32_t n = g->n;
  g->nlow.reset(al, n);
  DArr<int32_t> nup(al, n);
  g->eoff.reset(al, (int64_t)n + 1);
  if (n > 0) {
    k_nlow<<<grid_for(n, 256), 256, 0, s>>>(g->row_off.p, g->col.p, n,
                                             g->nlow.p, nup.p);
    ND_LAUNCHED();
  }
  exclusive_scan_i32(nup.p, g->eoff.p, n, s, al);
  g->ne = read_i64(g->eoff.p + n, s);
  ND_REQUIRE(g->ne < ((int64_t)1 << 31), ND_ERR_INVALID,
             "%lld edges: edge ids must fit int32", (long long)g->ne);
  g->eid.reset(al, g->nnz);
  g->ev.reset(al, 2 * g->ne);  // also the k-truss r-clique table
  if (g->nnz > 0) {
    k_eid<<<grid_for(g->nnz, 256), 256, 0, s>>>(
        g->row_off.p, g->col.p, g->rowid.p, g->nlow.p, g->eoff.p, g->nnz,
        g->eid.p, g->ev.p);
    ND_LAUNCHED();
  }
  g->edges_ready = true;
}

}  // namespace nd
