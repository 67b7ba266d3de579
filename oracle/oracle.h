/*
 * oracle.h -- plain CPU reference for the local (r,s)-nucleus decomposition
 * of Sariyuce, Seshadhri and Pinar, "Local Algorithms for Hierarchical Dense
 * Subgraph Discovery" (PVLDB 12(1), 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * HIP implementation.
 *
 * Conventions
 *   - The graph is simple and undirected (Section 2).  og_new() turns a raw
 *     edge list into that form: self-loops dropped, repeated pairs merged,
 *     adjacency lists sorted ascending.
 *   - r-cliques are sorted vertex tuples, numbered in lexicographic order of
 *     those tuples ("natural order" of Section 5.1.1).  r = 1 numbers vertices
 *     by id, r = 2 numbers edges (u<v), r = 3 numbers triangles (u<v<w).
 *   - Supported (r,s): 1 <= r < s <= 4 (the paper's three cases (1,2), (2,3),
 *     (3,4) and the other small ones).
 *   - kappa / tau values and r-clique ids are int32; counts of (R,S) pairs and
 *     offsets are int64.
 *   - Functions returning int return 0 on success and -1 on error; the error
 *     text is available from og_last_error().
 */
#ifndef ND_ORACLE_H
#define ND_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct og og;

/* Build the simple undirected graph on vertices 0..n-1 from m raw pairs
 * (src[i], dst[i]).  Returns NULL (with og_last_error set) when n < 0, m < 0
 * or an endpoint is outside [0, n). */
og *og_new(int32_t n, int64_t m, const int32_t *src, const int32_t *dst);
void og_free(og *g);
const char *og_last_error(void);

int32_t og_n(const og *g);
/* Number of stored adjacency entries, 2|E|. */
int64_t og_nnz(const og *g);
/* Copy out the canonical CSR: row_off[n+1], col[nnz]. */
void og_csr(const og *g, int64_t *row_off, int32_t *col);

/* Number of r-cliques (builds the lexicographic list on first use). */
int64_t og_num_rcliques(og *g, int r);
/* Copy the r-clique list out: out[i*r + j] = j-th vertex of r-clique i. */
int og_rcliques(og *g, int r, int32_t *out);

/* h-index H(K) of a multiset (Defn. of H, Section 2.2): the largest k such
 * that at least k elements of K are >= k.  Computed by sorting. */
int32_t og_hindex(const int32_t *K, int64_t len);

/* S-degrees d_s(R) of all r-cliques (Defn. 1), s-cliques found on the fly. */
int og_sdeg(og *g, int r, int s, int32_t *ds, int threads);

/* Incidence of one r-clique R: for every s-clique S containing R (extension
 * tuples in lexicographic order), the ids of the C(s,r)-1 other r-cliques of
 * S (in lexicographic order of their vertex tuples).  Writes at most `cap`
 * ids into out and returns d_s(R), the number of such S; -1 on error. */
int64_t og_members(og *g, int r, int s, int64_t R, int32_t *out, int64_t cap);

/* kappa_s of every r-clique by Alg. Peeling (bucket queue on d_s). */
int og_peel(og *g, int r, int s, int32_t *kappa, int threads);

/* One application of the update operator U (Defn. of U, Section 3) to the
 * r-cliques with ids in [lo, hi):  tau_out[R] = H({rho(S,R)}_{S contains R})
 * with rho(S,R) = min over the other r-cliques R' of S of tau_in[R'].
 * Entries of tau_out outside [lo, hi) are not touched. */
int og_update(og *g, int r, int s, const int32_t *tau_in, int32_t *tau_out,
              int64_t lo, int64_t hi, int threads);

/* U applied to the r-cliques listed in ids[count] only (repeats allowed):
 * tau_out[R] = (U tau_in)(R) for each listed R; other entries untouched.
 * The step of PartialAND (Section 4.3, end), taken synchronously. */
int og_update_set(og *g, int r, int s, const int32_t *tau_in, int32_t *tau_out,
                  const int32_t *ids, int64_t count, int threads);

/* One in-place asynchronous sweep (Alg. AND without the notification lines):
 * visits r-cliques in the given order (NULL = id order), each time reading
 * the current tau.  Returns the number of r-cliques whose tau changed, or -1.
 */
int64_t og_and_sweep(og *g, int r, int s, int32_t *tau, const int64_t *order);

/* Degree levels (Defn. 4): level[R] = i for R in L_i.  Returns the number of
 * non-empty levels, or -1 on error. */
int32_t og_levels(og *g, int r, int s, int32_t *level);

#ifdef __cplusplus
}
#endif

#endif /* ND_ORACLE_H */
