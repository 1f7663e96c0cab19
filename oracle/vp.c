/* ORACLE (test infrastructure only; never part of the counting library).
 *
 * Vertex-priority counting of balanced and unbalanced butterflies in a signed
 * bipartite graph, written as plainly as possible from the paper:
 *   - Definition 3 (vertex priority): p(a) > p(b) iff deg(a) > deg(b), or the
 *     degrees are equal and id(a) > id(b), over all of U and V.
 *   - Algorithm 1, Phase 5: for every pivot u and every neighbour v of u with
 *     p(v) < p(u), every neighbour w of v with p(w) < p(u) is the end of a
 *     wedge u-v-w.  The wedge is symmetric (bucket B1) if the two edge signs
 *     agree, asymmetric (bucket B2) otherwise (Definitions 5 and 6).  Per
 *     endpoint w the pivot contributes C(B1[w],2) + C(B2[w],2) balanced
 *     butterflies (Lemma 1), after which the touched buckets are reset.
 *   - Theorem 1: every butterfly is counted once, at its highest-priority
 *     vertex.
 * Beyond the paper's balanced count this file also reports, per endpoint,
 * B1[w] * B2[w] unbalanced butterflies (a symmetric wedge paired with an
 * asymmetric one has an odd number of negative edges) and C(B1[w]+B2[w], 2)
 * butterflies in total, computed separately so that tests can check that the
 * two classes add up.  Optionally it also counts, per vertex and per edge,
 * the balanced and unbalanced butterflies containing that vertex or edge.
 *
 * Pivots are spread over POSIX threads; each thread has private buckets, as
 * in the paper's thread-private counters.  Integer sums are exact (int64).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t balanced, unbalanced, total, wedges, expansions;
} oracle_counts;

typedef struct {
  /* graph over global vertex indices 0..n-1: U first (0..n_u-1), then V */
  int64_t n;
  const int64_t *adj_off; /* [n+1] */
  const int32_t *adj;     /* neighbour global index */
  const int8_t *adj_sign; /* +1 / -1 */
  const int64_t *adj_eid; /* input record of each adjacency entry */
  const int64_t *deg;
  const int64_t *id; /* tie-break id per vertex */
  const int32_t *pivots;
  int64_t n_pivots;
  int64_t next; /* shared pivot cursor */
  pthread_mutex_t lock;
  int64_t *per_pivot_bal; /* optional [n] */
  int64_t *bal_vertex;    /* optional [n] */
  int64_t *unb_vertex;    /* optional [n] */
  int64_t *bal_edge;      /* optional [m], by input record */
  int64_t *unb_edge;      /* optional [m] */
  oracle_counts sum;
} job;

/* Definition 3: does a have higher priority than b? */
static inline int higher(const job *J, int64_t a, int64_t b) {
  if (J->deg[a] != J->deg[b]) return J->deg[a] > J->deg[b];
  return J->id[a] > J->id[b];
}

static inline int64_t choose2(int64_t x) { return x * (x - 1) / 2; }

static void add_vertex(int64_t *arr, int64_t x, int64_t val) {
  if (val) __atomic_fetch_add(&arr[x], val, __ATOMIC_RELAXED);
}

static void *worker(void *arg) {
  job *J = (job *)arg;
  int64_t n = J->n;
  int32_t *B1 = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  int32_t *B2 = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  oracle_counts c = {0, 0, 0, 0, 0};
  const int per_vertex = J->bal_vertex != NULL || J->unb_vertex != NULL;
  const int per_edge = J->bal_edge != NULL || J->unb_edge != NULL;
  for (;;) {
    int64_t k = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
    if (k >= J->n_pivots) break;
    int64_t u = J->pivots ? (int64_t)J->pivots[k] : k;
    int64_t nt = 0;
    /* enumerate wedges u - v - w with p(v) < p(u) and p(w) < p(u) */
    for (int64_t a = J->adj_off[u]; a < J->adj_off[u + 1]; ++a) {
      int64_t v = J->adj[a];
      if (!higher(J, u, v)) continue;
      c.expansions += 1;
      for (int64_t b = J->adj_off[v]; b < J->adj_off[v + 1]; ++b) {
        int64_t w = J->adj[b];
        if (!higher(J, u, w)) continue;
        c.wedges += 1;
        if (B1[w] == 0 && B2[w] == 0) touched[nt++] = (int32_t)w;
        if (J->adj_sign[a] == J->adj_sign[b])
          B1[w] += 1;
        else
          B2[w] += 1;
      }
    }
    int64_t pivot_bal = 0, pivot_unb = 0;
    for (int64_t t = 0; t < nt; ++t) {
      int64_t w = touched[t];
      int64_t bal = choose2(B1[w]) + choose2(B2[w]);
      int64_t unb = (int64_t)B1[w] * B2[w];
      pivot_bal += bal;
      pivot_unb += unb;
      c.total += choose2((int64_t)B1[w] + B2[w]);
      if (per_vertex) {
        if (J->bal_vertex) add_vertex(J->bal_vertex, w, bal);
        if (J->unb_vertex) add_vertex(J->unb_vertex, w, unb);
      }
    }
    c.balanced += pivot_bal;
    c.unbalanced += pivot_unb;
    if (J->per_pivot_bal) J->per_pivot_bal[u] = pivot_bal;
    if (per_vertex) {
      if (J->bal_vertex) add_vertex(J->bal_vertex, u, pivot_bal);
      if (J->unb_vertex) add_vertex(J->unb_vertex, u, pivot_unb);
    }
    if (per_vertex || per_edge) {
      /* A wedge u-v-w lies in the butterflies that pair it with another wedge
       * u-v'-w.  A symmetric one lies in B1[w] - 1 balanced butterflies (the
       * other symmetric wedges) and in B2[w] unbalanced ones (the asymmetric
       * wedges); an asymmetric one swaps the roles.  Each butterfly counted
       * at (u, w) is the union of exactly two such wedges, so this credit
       * goes once to the mid v and once to each of the wedge's two edges. */
      for (int64_t a = J->adj_off[u]; a < J->adj_off[u + 1]; ++a) {
        int64_t v = J->adj[a];
        if (!higher(J, u, v)) continue;
        int64_t bv = 0, uv = 0;
        for (int64_t b = J->adj_off[v]; b < J->adj_off[v + 1]; ++b) {
          int64_t w = J->adj[b];
          if (!higher(J, u, w)) continue;
          int64_t bw, uw;
          if (J->adj_sign[a] == J->adj_sign[b]) {
            bw = B1[w] - 1;
            uw = B2[w];
          } else {
            bw = B2[w] - 1;
            uw = B1[w];
          }
          bv += bw;
          uv += uw;
          if (J->bal_edge) {
            add_vertex(J->bal_edge, J->adj_eid[a], bw);
            add_vertex(J->bal_edge, J->adj_eid[b], bw);
          }
          if (J->unb_edge) {
            add_vertex(J->unb_edge, J->adj_eid[a], uw);
            add_vertex(J->unb_edge, J->adj_eid[b], uw);
          }
        }
        if (J->bal_vertex) add_vertex(J->bal_vertex, v, bv);
        if (J->unb_vertex) add_vertex(J->unb_vertex, v, uv);
      }
    }
    for (int64_t t = 0; t < nt; ++t) {
      B1[touched[t]] = 0;
      B2[touched[t]] = 0;
    }
  }
  pthread_mutex_lock(&J->lock);
  J->sum.balanced += c.balanced;
  J->sum.unbalanced += c.unbalanced;
  J->sum.total += c.total;
  J->sum.wedges += c.wedges;
  J->sum.expansions += c.expansions;
  pthread_mutex_unlock(&J->lock);
  free(B1);
  free(B2);
  free(touched);
  return NULL;
}

/* The graph in the form the worker walks: per global vertex index (U first,
 * then V) its adjacency list in input order, with each entry's sign and
 * input record, the degrees and the tie-break ids of Definition 3. */
typedef struct {
  int64_t n_u, n_v, m, n;
  int64_t *deg, *off, *ids, *adj_eid;
  int32_t *adj;
  int8_t *adj_sign;
} oracle_graph;

void oracle_graph_free(oracle_graph *G) {
  if (!G) return;
  free(G->deg);
  free(G->off);
  free(G->ids);
  free(G->adj);
  free(G->adj_sign);
  free(G->adj_eid);
  free(G);
}

/* Build the adjacency lists of the graph with edges (u[i], v[i], sign[i]).
 * Vertex x of U has global index x, vertex y of V has global index n_u + y.
 * id: tie-break id per global index (NULL: the global index itself).
 * Returns NULL on bad input (ids out of range, signs not +1 / -1) or when
 * memory runs out.  Duplicate (u, v) pairs are not allowed here. */
oracle_graph *oracle_graph_build(int64_t n_u, int64_t n_v, int64_t m, const int32_t *u,
                                 const int32_t *v, const int8_t *sign, const int64_t *id) {
  if (n_u < 0 || n_v < 0 || m < 0) return NULL;
  oracle_graph *G = (oracle_graph *)calloc(1, sizeof(oracle_graph));
  if (!G) return NULL;
  int64_t n = n_u + n_v;
  G->n_u = n_u;
  G->n_v = n_v;
  G->m = m;
  G->n = n;
  G->deg = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
  G->off = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
  int64_t *fill = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
  G->ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  G->adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
  G->adj_sign = (int8_t *)malloc((size_t)(2 * m + 1));
  G->adj_eid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
  if (!G->deg || !G->off || !fill || !G->ids || !G->adj || !G->adj_sign || !G->adj_eid) goto fail;
  for (int64_t i = 0; i < m; ++i) {
    if (u[i] < 0 || u[i] >= n_u || v[i] < 0 || v[i] >= n_v) goto fail;
    if (sign[i] != 1 && sign[i] != -1) goto fail;
    G->deg[u[i]] += 1;
    G->deg[n_u + v[i]] += 1;
  }
  for (int64_t x = 0; x < n; ++x) {
    G->off[x + 1] = G->off[x] + G->deg[x];
    G->ids[x] = id ? id[x] : x;
  }
  for (int64_t i = 0; i < m; ++i) {
    int64_t a = u[i], b = n_u + v[i];
    G->adj[G->off[a] + fill[a]] = (int32_t)b;
    G->adj_eid[G->off[a] + fill[a]] = i;
    G->adj_sign[G->off[a] + fill[a]++] = sign[i];
    G->adj[G->off[b] + fill[b]] = (int32_t)a;
    G->adj_eid[G->off[b] + fill[b]] = i;
    G->adj_sign[G->off[b] + fill[b]++] = sign[i];
  }
  free(fill);
  return G;
fail:
  free(fill);
  oracle_graph_free(G);
  return NULL;
}

/* Phase 5 over a built graph.
 * pivots / n_pivots: restrict Phase 5 to these global indices (NULL: all).
 * The per-vertex and per-pivot arrays (length n_u + n_v) and the per-edge
 * arrays (length m, indexed by input record) are optional and must be zeroed
 * by the caller.  Returns 0, or -1 on bad input / no memory. */
int oracle_graph_count(const oracle_graph *G, int nthreads, const int32_t *pivots, int64_t n_pivots,
                       int64_t *per_pivot_bal, int64_t *bal_vertex, int64_t *unb_vertex,
                       int64_t *bal_edge, int64_t *unb_edge, oracle_counts *out) {
  if (!G || !out) return -1;
  memset(out, 0, sizeof(*out));
  for (int64_t k = 0; pivots && k < n_pivots; ++k)
    if (pivots[k] < 0 || pivots[k] >= G->n) return -1;
  job J;
  memset(&J, 0, sizeof(J));
  J.n = G->n;
  J.adj_off = G->off;
  J.adj = G->adj;
  J.adj_sign = G->adj_sign;
  J.adj_eid = G->adj_eid;
  J.deg = G->deg;
  J.id = G->ids;
  J.pivots = pivots;
  J.n_pivots = pivots ? n_pivots : G->n;
  J.per_pivot_bal = per_pivot_bal;
  J.bal_vertex = bal_vertex;
  J.unb_vertex = unb_vertex;
  J.bal_edge = bal_edge;
  J.unb_edge = unb_edge;
  pthread_mutex_init(&J.lock, NULL);
  if (nthreads < 1) nthreads = 1;
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  if (!th) {
    pthread_mutex_destroy(&J.lock);
    return -1;
  }
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, worker, &J);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
  pthread_mutex_destroy(&J.lock);
  *out = J.sum;
  return 0;
}

/* Build, count and free in one call (arguments as above). */
int oracle_vp_count(int64_t n_u, int64_t n_v, int64_t m, const int32_t *u, const int32_t *v,
                    const int8_t *sign, const int64_t *id, int nthreads, const int32_t *pivots,
                    int64_t n_pivots, int64_t *per_pivot_bal, int64_t *bal_vertex,
                    int64_t *unb_vertex, int64_t *bal_edge, int64_t *unb_edge,
                    oracle_counts *out) {
  if (!out) return -1;
  memset(out, 0, sizeof(*out));
  oracle_graph *G = oracle_graph_build(n_u, n_v, m, u, v, sign, id);
  if (!G) return -1;
  int rc = oracle_graph_count(G, nthreads, pivots, n_pivots, per_pivot_bal, bal_vertex,
                              unb_vertex, bal_edge, unb_edge, out);
  oracle_graph_free(G);
  return rc;
}
