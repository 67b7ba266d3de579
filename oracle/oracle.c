/*
 * oracle.c -- plain CPU reference for the local (r,s)-nucleus decomposition.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for obviousness, not
 * speed: s-cliques are found on the fly from sorted adjacency lists every
 * time they are needed (as the paper's own implementation does, Section 5),
 * r-cliques are looked up by binary search in their lexicographic list, and
 * the h-index is computed by sorting.
 *
 * Paper passages followed:
 *   - simple undirected graph, r-/s-cliques ............ Section 2
 *   - S-degree d_s(R) .................................. Section 2.1, Defn. of
 *                                                        S-degree
 *   - Alg. Peeling ..................................... Section 2.1, Alg. 1
 *   - h-index H ........................................ Section 2.2, Defn. of H
 *   - update operator U, rho(S,R) ...................... Section 3, Defn. of U
 *   - degree levels L_i ................................ Section 3.1, Defn. of
 *                                                        degree levels
 *   - asynchronous sweep ............................... Section 4.2, Alg. AND
 */
#include "oracle.h"

#include <pthread.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ errors */

static __thread char g_err[256];

static void set_err(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

const char *og_last_error(void) { return g_err; }

/* ------------------------------------------------------------------- graph */

struct og {
  int32_t n;
  int64_t nnz;
  int64_t *row_off; /* n+1 */
  int32_t *col;     /* nnz, each list ascending */
  /* r-clique lists, r = 1..4, lexicographic order of sorted tuples */
  int64_t nr[5];
  int32_t *rv[5];
  /* first[r][v]: index of the first r-clique whose smallest vertex is v */
  int64_t *first[5];
  int built[5];
  pthread_mutex_t lock;
};

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return (x > y) - (x < y);
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

static int cmp_i32_desc(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x < y) - (x > y);
}

og *og_new(int32_t n, int64_t m, const int32_t *src, const int32_t *dst) {
  if (n < 0 || m < 0) {
    set_err("og_new: negative size (n=%d, m=%lld)", n, (long long)m);
    return NULL;
  }
  for (int64_t i = 0; i < m; i++) {
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) {
      set_err("og_new: edge %lld has an endpoint outside [0,%d)", (long long)i,
              n);
      return NULL;
    }
  }
  og *g = (og *)calloc(1, sizeof(og));
  pthread_mutex_init(&g->lock, NULL);
  g->n = n;
  /* Unordered pairs {a,b} with a != b, as keys a<<32|b with a < b. */
  uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m ? m : 1));
  int64_t k = 0;
  for (int64_t i = 0; i < m; i++) {
    int32_t a = src[i], b = dst[i];
    if (a == b) continue; /* self-loop: not part of a simple graph */
    if (a > b) { int32_t t = a; a = b; b = t; }
    key[k++] = ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
  }
  qsort(key, (size_t)k, sizeof(uint64_t), cmp_u64);
  int64_t ne = 0; /* distinct pairs */
  for (int64_t i = 0; i < k; i++)
    if (i == 0 || key[i] != key[i - 1]) key[ne++] = key[i];
  /* Symmetric CSR: each pair {a,b} stored as b in N(a) and a in N(b). */
  g->row_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t i = 0; i < ne; i++) {
    g->row_off[(key[i] >> 32) + 1]++;
    g->row_off[(key[i] & 0xffffffffu) + 1]++;
  }
  for (int32_t v = 0; v < n; v++) g->row_off[v + 1] += g->row_off[v];
  g->nnz = 2 * ne;
  g->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->nnz ? g->nnz : 1));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  memcpy(fill, g->row_off, sizeof(int64_t) * ((size_t)n + 1));
  for (int64_t i = 0; i < ne; i++) {
    int32_t a = (int32_t)(key[i] >> 32), b = (int32_t)(key[i] & 0xffffffffu);
    g->col[fill[a]++] = b;
    g->col[fill[b]++] = a;
  }
  for (int32_t v = 0; v < n; v++)
    qsort(g->col + g->row_off[v], (size_t)(g->row_off[v + 1] - g->row_off[v]),
          sizeof(int32_t), cmp_i32);
  free(fill);
  free(key);
  return g;
}

void og_free(og *g) {
  if (!g) return;
  free(g->row_off);
  free(g->col);
  for (int r = 0; r < 5; r++) {
    free(g->rv[r]);
    free(g->first[r]);
  }
  pthread_mutex_destroy(&g->lock);
  free(g);
}

int32_t og_n(const og *g) { return g->n; }
int64_t og_nnz(const og *g) { return g->nnz; }

void og_csr(const og *g, int64_t *row_off, int32_t *col) {
  memcpy(row_off, g->row_off, sizeof(int64_t) * ((size_t)g->n + 1));
  memcpy(col, g->col, sizeof(int32_t) * (size_t)g->nnz);
}

/* Is v in the sorted list N(u)?  Binary search. */
static int adjacent(const og *g, int32_t u, int32_t v) {
  int64_t lo = g->row_off[u], hi = g->row_off[u + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (g->col[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo < g->row_off[u + 1] && g->col[lo] == v;
}

/* ------------------------------------------------------- growable int list */

typedef struct {
  int32_t *a;
  int64_t len, cap;
} ilist;

static void il_push(ilist *l, int32_t x) {
  if (l->len == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 64;
    l->a = (int32_t *)realloc(l->a, sizeof(int32_t) * (size_t)l->cap);
  }
  l->a[l->len++] = x;
}

/* ------------------------------------------------ r-clique enumeration */

/* Extend the clique tup[0..depth-1] (all of whose common higher neighbours
 * are in cand[0..nc-1], ascending) up to size r, appending in lexicographic
 * order. */
static void enum_rec(const og *g, int r, int32_t *tup, int depth,
                     const int32_t *cand, int64_t nc, ilist *out) {
  if (depth == r) {
    for (int j = 0; j < r; j++) il_push(out, tup[j]);
    return;
  }
  if (depth + 1 == r) { /* last position: every candidate completes it */
    for (int64_t i = 0; i < nc; i++) {
      tup[depth] = cand[i];
      for (int j = 0; j < r; j++) il_push(out, tup[j]);
    }
    return;
  }
  int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc ? nc : 1));
  for (int64_t i = 0; i < nc; i++) {
    int32_t x = cand[i];
    tup[depth] = x;
    /* candidates for the next position: later candidates adjacent to x,
     * i.e. cand[i+1..nc) & N(x), ascending.  Scan the shorter list and
     * binary-search the other. */
    int64_t nn = 0;
    const int64_t xb = g->row_off[x], xe = g->row_off[x + 1];
    if (xe - xb < nc - i - 1) {
      for (int64_t p = xb; p < xe; p++) {
        int32_t y = g->col[p];
        if (y <= x) continue;
        int64_t lo = i + 1, hi = nc;
        while (lo < hi) {
          int64_t mid = lo + (hi - lo) / 2;
          if (cand[mid] < y) lo = mid + 1;
          else hi = mid;
        }
        if (lo < nc && cand[lo] == y) next[nn++] = y;
      }
    } else {
      for (int64_t j = i + 1; j < nc; j++)
        if (adjacent(g, x, cand[j])) next[nn++] = cand[j];
    }
    enum_rec(g, r, tup, depth + 1, next, nn, out);
  }
  free(next);
}

static int build_rcliques(og *g, int r) {
  if (r < 1 || r > 4) {
    set_err("r=%d outside 1..4", r);
    return -1;
  }
  pthread_mutex_lock(&g->lock);
  if (g->built[r]) {
    pthread_mutex_unlock(&g->lock);
    return 0;
  }
  ilist out = {0};
  int32_t tup[4];
  for (int32_t v = 0; v < g->n; v++) {
    tup[0] = v;
    if (r == 1) {
      il_push(&out, v);
      continue;
    }
    /* higher neighbours of v, ascending */
    int64_t b = g->row_off[v], e = g->row_off[v + 1];
    int64_t s = b;
    while (s < e && g->col[s] < v) s++;
    enum_rec(g, r, tup, 1, g->col + s, e - s, &out);
  }
  g->nr[r] = out.len / r;
  g->rv[r] = out.a ? out.a : (int32_t *)malloc(sizeof(int32_t));
  g->first[r] = (int64_t *)malloc(sizeof(int64_t) * ((size_t)g->n + 1));
  int64_t i = 0;
  for (int32_t v = 0; v <= g->n; v++) {
    while (i < g->nr[r] && g->rv[r][i * r] < v) i++;
    g->first[r][v] = i;
  }
  g->built[r] = 1;
  pthread_mutex_unlock(&g->lock);
  return 0;
}

int64_t og_num_rcliques(og *g, int r) {
  if (build_rcliques(g, r)) return -1;
  return g->nr[r];
}

int og_rcliques(og *g, int r, int32_t *out) {
  if (build_rcliques(g, r)) return -1;
  memcpy(out, g->rv[r], sizeof(int32_t) * (size_t)(g->nr[r] * r));
  return 0;
}

/* Id of the sorted r-tuple t, or -1 when t is not an r-clique. */
static int64_t rclique_id(const og *g, int r, const int32_t *t) {
  int64_t lo = g->first[r][t[0]], hi = g->first[r][t[0] + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    const int32_t *x = g->rv[r] + mid * r;
    int c = 0;
    for (int j = 0; j < r && c == 0; j++) c = (x[j] > t[j]) - (x[j] < t[j]);
    if (c == 0) return mid;
    if (c < 0) lo = mid + 1;
    else hi = mid;
  }
  return -1;
}

/* ------------------------------------- s-cliques containing an r-clique */

typedef struct {
  const og *g;
  int r, s;
  const int32_t *R; /* sorted vertices of R */
  int64_t Rid;
  ilist cn;   /* common neighbours of R's vertices */
  int32_t ext[4];
  ilist *out; /* receives the other r-cliques' ids, or NULL to count only */
  int64_t count;
} scl_ctx;

/* Emit the s-clique S = R u ext: append the ids of its r-subsets other than
 * R, in lexicographic order of the position combinations. */
static void emit_s(scl_ctx *c) {
  c->count++;
  if (!c->out) return;
  int32_t S[4];
  int ns = 0;
  for (int j = 0; j < c->r; j++) S[ns++] = c->R[j];
  for (int j = 0; j < c->s - c->r; j++) S[ns++] = c->ext[j];
  /* insertion sort of at most 4 values */
  for (int i = 1; i < ns; i++)
    for (int j = i; j > 0 && S[j - 1] > S[j]; j--) {
      int32_t t = S[j]; S[j] = S[j - 1]; S[j - 1] = t;
    }
  int pos[4];
  for (int j = 0; j < c->r; j++) pos[j] = j;
  for (;;) {
    int32_t T[4];
    for (int j = 0; j < c->r; j++) T[j] = S[pos[j]];
    int same = 1;
    for (int j = 0; j < c->r; j++) same &= (T[j] == c->R[j]);
    if (!same) il_push(c->out, (int32_t)rclique_id(c->g, c->r, T));
    /* next combination of r positions out of s */
    int j = c->r - 1;
    while (j >= 0 && pos[j] == c->s - c->r + j) j--;
    if (j < 0) break;
    pos[j]++;
    for (int q = j + 1; q < c->r; q++) pos[q] = pos[q - 1] + 1;
  }
}

/* First index i >= lo of the sorted list a[0..len) with a[i] >= v. */
static int64_t first_ge(const int32_t *a, int64_t lo, int64_t len, int32_t v) {
  int64_t hi = len;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

/* Pick the extension vertices ext[depth..] from cn[start..], increasing,
 * each adjacent to the ones already picked.  Past the first pick the
 * candidates are also neighbours of the last one, so when that vertex has
 * fewer neighbours than cn has candidates left, its (ascending) list is
 * walked instead and each entry looked up in cn: the same vertices in the
 * same increasing order. */
static void extend_s(scl_ctx *c, int depth, int64_t start) {
  if (depth == c->s - c->r) {
    emit_s(c);
    return;
  }
  const og *g = c->g;
  if (depth > 0) {
    const int32_t last = c->ext[depth - 1];
    const int64_t b = g->row_off[last], e = g->row_off[last + 1];
    if (e - b < c->cn.len - start) {
      for (int64_t p = b; p < e; p++) {
        const int32_t x = g->col[p];
        const int64_t i = first_ge(c->cn.a, start, c->cn.len, x);
        if (i == c->cn.len || c->cn.a[i] != x) continue;
        int ok = 1;
        for (int j = 0; j < depth - 1 && ok; j++) ok = adjacent(g, c->ext[j], x);
        if (!ok) continue;
        c->ext[depth] = x;
        extend_s(c, depth + 1, i + 1);
      }
      return;
    }
  }
  for (int64_t i = start; i < c->cn.len; i++) {
    int32_t x = c->cn.a[i];
    int ok = 1;
    for (int j = 0; j < depth && ok; j++) ok = adjacent(g, c->ext[j], x);
    if (!ok) continue;
    c->ext[depth] = x;
    extend_s(c, depth + 1, i + 1);
  }
}

/* All s-cliques S containing r-clique Rid.  Vertices that may extend R are
 * exactly the common neighbours of R's vertices (none of R's own vertices is
 * its own neighbour in a simple graph). */
static int64_t scliques_of(scl_ctx *c, int64_t Rid) {
  const og *g = c->g;
  c->Rid = Rid;
  c->R = g->rv[c->r] + Rid * c->r;
  c->count = 0;
  c->cn.len = 0;
  /* scan the (ascending) neighbour list of R's lowest-degree vertex */
  int lo = 0;
  for (int j = 1; j < c->r; j++)
    if (g->row_off[c->R[j] + 1] - g->row_off[c->R[j]] <
        g->row_off[c->R[lo] + 1] - g->row_off[c->R[lo]])
      lo = j;
  int32_t v0 = c->R[lo];
  for (int64_t p = g->row_off[v0]; p < g->row_off[v0 + 1]; p++) {
    int32_t x = g->col[p];
    int ok = 1;
    for (int j = 0; j < c->r && ok; j++)
      if (j != lo) ok = adjacent(g, c->R[j], x);
    if (ok) il_push(&c->cn, x);
  }
  extend_s(c, 0, 0);
  return c->count;
}

static int check_rs(og *g, int r, int s) {
  if (r < 1 || s > 4 || r >= s) {
    set_err("unsupported (r,s)=(%d,%d): need 1 <= r < s <= 4", r, s);
    return -1;
  }
  return build_rcliques(g, r);
}

static int choose(int n, int k) {
  int c = 1;
  for (int i = 0; i < k; i++) c = c * (n - i) / (i + 1);
  return c;
}

int64_t og_members(og *g, int r, int s, int64_t R, int32_t *out, int64_t cap) {
  if (check_rs(g, r, s)) return -1;
  if (R < 0 || R >= g->nr[r]) {
    set_err("r-clique id %lld out of range", (long long)R);
    return -1;
  }
  ilist ids = {0};
  scl_ctx c = {.g = g, .r = r, .s = s, .out = &ids};
  int64_t d = scliques_of(&c, R);
  int64_t w = ids.len < cap ? ids.len : cap;
  if (w > 0) memcpy(out, ids.a, sizeof(int32_t) * (size_t)w);
  free(ids.a);
  free(c.cn.a);
  return d;
}

/* ----------------------------------------------------------- h-index */

/* Defn. of H: the largest k with at least k elements of K that are >= k.
 * Sort descending; then "at least i elements are >= i" holds exactly when the
 * i-th largest element is >= i, and it holds for every i up to the answer. */
int32_t og_hindex(const int32_t *K, int64_t len) {
  if (len <= 0) return 0;
  int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)len);
  memcpy(a, K, sizeof(int32_t) * (size_t)len);
  qsort(a, (size_t)len, sizeof(int32_t), cmp_i32_desc);
  int32_t h = 0;
  for (int64_t i = 1; i <= len; i++) {
    if (a[i - 1] >= i) h = (int32_t)i;
    else break;
  }
  free(a);
  return h;
}

/* ----------------------------------------------------- parallel loop */

typedef struct {
  int64_t lo, hi, chunk;
  int64_t next; /* guarded by lock */
  pthread_mutex_t lock;
  void (*body)(void *arg, int64_t i, void *scratch);
  void *arg;
} par_ctx;

typedef struct {
  par_ctx *p;
  scl_ctx sc;
  ilist ids;
} worker;

static void *par_worker(void *wv) {
  worker *w = (worker *)wv;
  par_ctx *p = w->p;
  for (;;) {
    pthread_mutex_lock(&p->lock);
    int64_t b = p->next;
    p->next += p->chunk;
    pthread_mutex_unlock(&p->lock);
    if (b >= p->hi) break;
    int64_t e = b + p->chunk < p->hi ? b + p->chunk : p->hi;
    for (int64_t i = b; i < e; i++) p->body(p->arg, i, w);
  }
  return NULL;
}

/* Run body(i) for i in [lo,hi) on `threads` threads, dynamic chunks of 100
 * (the scheduling the paper reports using, Section 4.4). */
static void par_for(int64_t lo, int64_t hi, int threads, const og *g, int r,
                    int s, void (*body)(void *, int64_t, void *), void *arg) {
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  par_ctx p = {.lo = lo, .hi = hi, .chunk = 100, .next = lo, .body = body,
               .arg = arg};
  pthread_mutex_init(&p.lock, NULL);
  worker *ws = (worker *)calloc((size_t)threads, sizeof(worker));
  pthread_t *th = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
  for (int t = 0; t < threads; t++) {
    ws[t].p = &p;
    ws[t].sc.g = g;
    ws[t].sc.r = r;
    ws[t].sc.s = s;
  }
  for (int t = 1; t < threads; t++)
    pthread_create(&th[t], NULL, par_worker, &ws[t]);
  par_worker(&ws[0]);
  for (int t = 1; t < threads; t++) pthread_join(th[t], NULL);
  for (int t = 0; t < threads; t++) {
    free(ws[t].sc.cn.a);
    free(ws[t].ids.a);
  }
  free(ws);
  free(th);
  pthread_mutex_destroy(&p.lock);
}

/* ------------------------------------------------------------ S-degree */

static void sdeg_body(void *arg, int64_t R, void *wv) {
  worker *w = (worker *)wv;
  w->sc.out = NULL; /* count only */
  ((int32_t *)arg)[R] = (int32_t)scliques_of(&w->sc, R);
}

int og_sdeg(og *g, int r, int s, int32_t *ds, int threads) {
  if (check_rs(g, r, s)) return -1;
  par_for(0, g->nr[r], threads, g, r, s, sdeg_body, ds);
  return 0;
}

/* ------------------------------------------------------ update operator */

typedef struct {
  const int32_t *tau_in;
  int32_t *tau_out;
  int k; /* other r-cliques per s-clique, C(s,r)-1 */
} upd_arg;

/* rho(S,R) for every S containing R, from the member list. */
static void rho_list(const ilist *ids, int64_t nS, int k, const int32_t *tau,
                     ilist *rho) {
  rho->len = 0;
  for (int64_t q = 0; q < nS; q++) {
    int32_t m = tau[ids->a[q * k]];
    for (int j = 1; j < k; j++)
      if (tau[ids->a[q * k + j]] < m) m = tau[ids->a[q * k + j]];
    il_push(rho, m);
  }
}

static void update_body(void *arg, int64_t R, void *wv) {
  upd_arg *u = (upd_arg *)arg;
  worker *w = (worker *)wv;
  w->ids.len = 0;
  w->sc.out = &w->ids;
  int64_t nS = scliques_of(&w->sc, R);
  ilist rho = {0};
  rho_list(&w->ids, nS, u->k, u->tau_in, &rho);
  u->tau_out[R] = og_hindex(rho.a, rho.len);
  free(rho.a);
}

int og_update(og *g, int r, int s, const int32_t *tau_in, int32_t *tau_out,
              int64_t lo, int64_t hi, int threads) {
  if (check_rs(g, r, s)) return -1;
  if (lo < 0) lo = 0;
  if (hi > g->nr[r]) hi = g->nr[r];
  upd_arg u = {.tau_in = tau_in, .tau_out = tau_out, .k = choose(s, r) - 1};
  if (lo < hi) par_for(lo, hi, threads, g, r, s, update_body, &u);
  return 0;
}

/* U on a list of r-clique ids (any order, repeats allowed). */
typedef struct {
  upd_arg u;
  const int32_t *ids;
} upd_set_arg;

static void update_set_body(void *arg, int64_t i, void *wv) {
  upd_set_arg *a = (upd_set_arg *)arg;
  update_body(&a->u, a->ids[i], wv);
}

int og_update_set(og *g, int r, int s, const int32_t *tau_in, int32_t *tau_out,
                  const int32_t *ids, int64_t count, int threads) {
  if (check_rs(g, r, s)) return -1;
  for (int64_t i = 0; i < count; i++)
    if (ids[i] < 0 || ids[i] >= g->nr[r]) {
      set_err("r-clique id %d out of range", ids[i]);
      return -1;
    }
  upd_set_arg a = {.u = {.tau_in = tau_in, .tau_out = tau_out,
                         .k = choose(s, r) - 1},
                   .ids = ids};
  if (count > 0) par_for(0, count, threads, g, r, s, update_set_body, &a);
  return 0;
}

/* ------------------------------------------------- asynchronous sweep */

int64_t og_and_sweep(og *g, int r, int s, int32_t *tau, const int64_t *order) {
  if (check_rs(g, r, s)) return -1;
  int k = choose(s, r) - 1;
  ilist ids = {0}, rho = {0};
  scl_ctx c = {.g = g, .r = r, .s = s, .out = &ids};
  int64_t changed = 0;
  for (int64_t i = 0; i < g->nr[r]; i++) {
    int64_t R = order ? order[i] : i;
    ids.len = 0;
    int64_t nS = scliques_of(&c, R);
    rho_list(&ids, nS, k, tau, &rho); /* reads the latest tau, in place */
    int32_t h = og_hindex(rho.a, rho.len);
    if (h != tau[R]) changed++;
    tau[R] = h;
  }
  free(ids.a);
  free(rho.a);
  free(c.cn.a);
  return changed;
}

/* --------------------------------------------------------------- peeling */

/* Alg. Peeling.  The bucket queue keeps r-cliques sorted by current d_s:
 * vert[] lists them in non-decreasing d_s, pos[R] is R's index in vert[],
 * bstart[d] is where bucket d begins.  Lowering d_s(R') by one moves R' to
 * the front of its bucket and shifts that bucket's start past it, which puts
 * it at the end of bucket d_s(R')-1 (Batagelj and Zaversnik's layout). */
int og_peel(og *g, int r, int s, int32_t *kappa, int threads) {
  if (check_rs(g, r, s)) return -1;
  int64_t nr = g->nr[r];
  int k = choose(s, r) - 1;
  int32_t *ds = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nr > 0 ? nr : 1));
  og_sdeg(g, r, s, ds, threads); /* counting is parallel, as in Section 5.2 */
  int32_t maxd = 0;
  for (int64_t i = 0; i < nr; i++) if (ds[i] > maxd) maxd = ds[i];
  int64_t *bstart = (int64_t *)calloc((size_t)maxd + 2, sizeof(int64_t));
  int64_t *vert = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nr > 0 ? nr : 1));
  int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nr > 0 ? nr : 1));
  char *done = (char *)calloc((size_t)(nr > 0 ? nr : 1), 1);
  for (int64_t i = 0; i < nr; i++) bstart[ds[i] + 1]++;
  for (int32_t d = 0; d <= maxd; d++) bstart[d + 1] += bstart[d];
  {
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)maxd + 2));
    memcpy(fill, bstart, sizeof(int64_t) * ((size_t)maxd + 2));
    for (int64_t i = 0; i < nr; i++) {
      pos[i] = fill[ds[i]]++;
      vert[pos[i]] = i;
    }
    free(fill);
  }
  ilist ids = {0};
  scl_ctx c = {.g = g, .r = r, .s = s, .out = &ids};
  for (int64_t i = 0; i < nr; i++) {
    int64_t R = vert[i]; /* an unprocessed r-clique of minimum d_s */
    kappa[R] = ds[R];
    ids.len = 0;
    int64_t nS = scliques_of(&c, R); /* s-cliques containing R, on the fly */
    for (int64_t q = 0; q < nS; q++) {
      const int32_t *m = ids.a + q * k;
      int skip = 0;
      for (int j = 0; j < k; j++) skip |= done[m[j]];
      if (skip) continue; /* S already destroyed by a processed r-clique */
      for (int j = 0; j < k; j++) {
        int64_t Rp = m[j];
        if (ds[Rp] > ds[R]) {
          int32_t du = ds[Rp];
          int64_t pu = pos[Rp], pw = bstart[du];
          int64_t W = vert[pw];
          if (W != Rp) { /* swap Rp with the first element of its bucket */
            vert[pu] = W; pos[W] = pu;
            vert[pw] = Rp; pos[Rp] = pw;
          }
          bstart[du]++;
          ds[Rp] = du - 1;
        }
      }
    }
    done[R] = 1;
  }
  free(ids.a);
  free(c.cn.a);
  free(ds);
  free(bstart);
  free(vert);
  free(pos);
  free(done);
  return 0;
}

/* ---------------------------------------------------------- degree levels */

/* Defn. of degree levels: L_0 holds the r-cliques of minimum S-degree; all of
 * them are removed together (removing an r-clique removes every s-clique
 * containing it); L_1 holds the minimum-degree r-cliques of what is left, and
 * so on.  Plain O(levels * |R|) scan for the minimum. */
int32_t og_levels(og *g, int r, int s, int32_t *level) {
  if (check_rs(g, r, s)) return -1;
  int64_t nr = g->nr[r];
  int k = choose(s, r) - 1;
  int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nr > 0 ? nr : 1));
  og_sdeg(g, r, s, deg, 1);
  for (int64_t i = 0; i < nr; i++) level[i] = -1; /* -1: still present */
  ilist ids = {0}, L = {0};
  scl_ctx c = {.g = g, .r = r, .s = s, .out = &ids};
  int64_t left = nr;
  int32_t lv = 0;
  while (left > 0) {
    int32_t mn = INT32_MAX;
    for (int64_t i = 0; i < nr; i++)
      if (level[i] < 0 && deg[i] < mn) mn = deg[i];
    L.len = 0;
    for (int64_t i = 0; i < nr; i++)
      if (level[i] < 0 && deg[i] == mn) il_push(&L, (int32_t)i);
    for (int64_t q = 0; q < L.len; q++) level[L.a[q]] = lv;
    left -= L.len;
    /* Each s-clique that was still present and loses a member now is
     * counted once: by its smallest-id member in L_lv. */
    for (int64_t q = 0; q < L.len; q++) {
      int64_t R = L.a[q];
      ids.len = 0;
      int64_t nS = scliques_of(&c, R);
      for (int64_t t = 0; t < nS; t++) {
        const int32_t *m = ids.a + t * k;
        int gone_before = 0, counted_by_other = 0;
        for (int j = 0; j < k; j++) {
          int32_t l = level[m[j]];
          if (l >= 0 && l < lv) gone_before = 1;
          if (l == lv && m[j] < R) counted_by_other = 1;
        }
        if (gone_before || counted_by_other) continue;
        for (int j = 0; j < k; j++)
          if (level[m[j]] < 0) deg[m[j]]--;
      }
    }
    lv++;
  }
  free(ids.a);
  free(L.a);
  free(c.cn.a);
  free(deg);
  return lv;
}
