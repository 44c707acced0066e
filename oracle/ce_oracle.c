/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow, obviously-correct host implementation of what the edge
 * clustering of a dynamic multigraph computes. Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load this library; the
 * GPU product path never calls it and shares no code with it.
 *
 * Paper: "Scalable Edge Clustering of Dynamic Graphs via Weighted Line
 * Graphs" (arXiv 2311.10337). Passages followed:
 *   - dynamic multigraph model, incidence sets E_i, degree d_i  (Sec. 1.2.1)
 *   - undirected line graph: line-graph nodes are the temporal edges,
 *     adjacent when they share a vertex                          (Sec. 1.2.2)
 *   - node-local formation L = union_i L(i)                      (Sec. 2, Def. 2)
 *   - skeleton L* = union of node-local MSTs, and for |t_a-t_b|
 *     weights the node-local MST is the path through the
 *     time-sorted incidence list                                 (Alg. 3; Sec. 5.3)
 *   - hierarchical clustering: MST, sort, union-find dendrogram,
 *     condense with M, extract by stability ("volume")           (Alg. 1, Alg. 4)
 *   - weight-filtered connectivity and tie-breaking by a
 *     perturbation that fixes a deterministic order            (App. A, Thm 1-3)
 *
 * Readings where the paper is silent or garbled (listed again in the design
 * notes):
 *   R1 record order e < f  <=>  (t_e, e) < (t_f, f), ids = input indices.
 *   R2 line-graph edge {a,b}: tail = <-min, head = <-max, w = t_head - t_tail;
 *      a pair sharing both endpoints is ONE edge.
 *   R3 canonical key K = (w, head, 2^32-1-tail), lexicographic; keys are
 *      distinct, so the minimum spanning forest is unique.
 *   R4 forest: MSF + a virtual ROOT (id n+m) at w = infinity, lambda = 0.
 *   R5 lambda(w) = floor(2^63 / max(2w,1)) (u64); stability is exact u128.
 *   R6 condensing follows HDBSCAN (Campello et al. 2013, to which the paper
 *      defers): a split with both children >= M starts two clusters; one
 *      small child sheds its points; two small children end the cluster.
 *      At ROOT: components < M shed at lambda 0; if >= 2 components are
 *      >= M each starts a cluster at lambda 0; if exactly 1, ROOT continues
 *      into it.
 *   R7 excess-of-mass selection, ties keep the parent, ROOT never selected;
 *      label = the selected cluster above a point's exit cluster, else -1;
 *      labels numbered by ascending minimum member id.
 *
 * Readings of the causal mode (Def. 1 with Alg. 2):
 *   C1 list order of E_i: time, then in-edges before out-edges at equal
 *      times, then id; this is the order the perturbation in the proof of
 *      Thm 2 induces (in-edge offsets of order gamma^2 below out-edge ones).
 *   C2 arc r -> s: tail = r (arrives), head = s (leaves), w = t_s - t_r; the
 *      canonical key is K = (w, head, 2^32-1-tail) as in R3, so among arcs
 *      of one out-edge with equal w the later in-edge (larger id) is first.
 *   C3 an out-edge with an empty window emits nothing and the window stays
 *      empty.
 *   Direction only decides which pairs are arcs; the spanning forest,
 *   dendrogram and condensing treat arcs as undirected edges (Alg. 1).
 *
 * Readings of dynamic hypergraphs (Sec. 5.3, undirected):
 *   H1 a hyperedge is a set S_r of vertices with a time t_r, given as a CSR
 *      (offsets, members); a vertex listed twice in one hyperedge counts once,
 *      and an empty hyperedge is a line-graph node without neighbours.
 *   H2 two hyperedges are adjacent when their sets meet; as for graphs
 *      (R2) a pair is ONE line-graph edge however many vertices it shares,
 *      with w = |t_r - t_s| and the canonical key of R3.
 *   H3 the skeleton is, per vertex, the path through its incident
 *      hyperedges in the record order R1 (the node-local MST for |dt|).
 *
 * Output conventions (identical to the GPU library's documented ones):
 *   MSF rows (tail, head, w) in ascending K; m = n - (#components).
 *   Dendrogram row k creates node n+k: (left=min child, right=max child, w, size).
 *   Cluster id = dendrogram node id where the cluster is born, ROOT = n+m;
 *   cluster rows in ascending id (ROOT last).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum { OR_OK = 0, OR_EINVAL = -1, OR_ESELFLOOP = -2, OR_ERANGE = -3, OR_ENOMEM = -4 };

#define NONE32 0xffffffffu

/* ------------------------------------------------------------------ */
/* O0: validation                                                      */
/* ------------------------------------------------------------------ */
int oracle_validate(int64_t n, const int32_t *src, const int32_t *dst, const int64_t *t, int64_t V) {
  if (n < 0 || n > 2147483647LL || V < 0) return OR_EINVAL;
  if (n == 0) return OR_OK;
  int64_t tmin = t[0], tmax = t[0];
  for (int64_t i = 0; i < n; i++) {
    if (src[i] < 0 || dst[i] < 0 || (int64_t)src[i] >= V || (int64_t)dst[i] >= V) return OR_ERANGE;
    if (src[i] == dst[i]) return OR_ESELFLOOP;
    if (t[i] < tmin) tmin = t[i];
    if (t[i] > tmax) tmax = t[i];
  }
  if ((u128)((__int128)tmax - (__int128)tmin) >= ((u128)1 << 62)) return OR_ERANGE;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Line-graph edges and the canonical key                              */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t w;
  uint32_t tail, head;
} lg_edge;

static const int64_t *g_t; /* timestamps for the record order in qsort callbacks */

/* R1: strict total order on records */
static int rec_before(uint32_t a, uint32_t b) {
  if (g_t[a] != g_t[b]) return g_t[a] < g_t[b];
  return a < b;
}

static lg_edge make_edge(uint32_t a, uint32_t b) {
  lg_edge e;
  if (rec_before(a, b)) { e.tail = a; e.head = b; }
  else { e.tail = b; e.head = a; }
  e.w = g_t[e.head] - g_t[e.tail];
  return e;
}

/* R3: K = (w, head, 2^32-1-tail) */
static int cmp_key(const void *pa, const void *pb) {
  const lg_edge *a = (const lg_edge *)pa, *b = (const lg_edge *)pb;
  if (a->w != b->w) return a->w < b->w ? -1 : 1;
  if (a->head != b->head) return a->head < b->head ? -1 : 1;
  if (a->tail != b->tail) return a->tail > b->tail ? -1 : 1; /* larger tail = smaller key */
  return 0;
}

/* incidence lists E_i (Sec. 1.2.1): CSR of record ids per vertex, ascending id */
static int build_incidence(int64_t n, const int32_t *src, const int32_t *dst, int64_t V,
                           int64_t **off_out, uint32_t **lst_out) {
  int64_t *off = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
  uint32_t *lst = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(2 * n + 1));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(V + 1));
  if (!off || !lst || !fill) { free(off); free(lst); free(fill); return OR_ENOMEM; }
  for (int64_t i = 0; i < n; i++) { off[src[i] + 1]++; off[dst[i] + 1]++; }
  for (int64_t v = 0; v < V; v++) off[v + 1] += off[v];
  memcpy(fill, off, sizeof(int64_t) * (size_t)V);
  for (int64_t i = 0; i < n; i++) {
    lst[fill[src[i]]++] = (uint32_t)i;
    lst[fill[dst[i]]++] = (uint32_t)i;
  }
  free(fill);
  *off_out = off;
  *lst_out = lst;
  return OR_OK;
}

/*
 * Tier A, the definition (Sec. 1.2.2 undirected line graph; Sec. 2 formula for
 * |F| = sum_i C(d_i,2) before de-duplication): every unordered pair of distinct
 * records sharing a vertex is one line-graph edge (R2). A pair is emitted at
 * the smallest vertex the two records share, so pairs sharing both endpoints
 * appear once. If out == NULL only the count is returned.
 */
int64_t oracle_full_line_graph(int64_t n, const int32_t *src, const int32_t *dst, const int64_t *t,
                               int64_t V, lg_edge *out) {
  int64_t *off;
  uint32_t *lst;
  if (build_incidence(n, src, dst, V, &off, &lst)) return OR_ENOMEM;
  g_t = t;
  int64_t cnt = 0;
  for (int64_t x = 0; x < V; x++) {
    for (int64_t i = off[x]; i < off[x + 1]; i++)
      for (int64_t j = i + 1; j < off[x + 1]; j++) {
        uint32_t a = lst[i], b = lst[j];
        /* smallest shared vertex of the two records */
        int64_t best = -1;
        int32_t ea[2] = {src[a], dst[a]}, eb[2] = {src[b], dst[b]};
        for (int p = 0; p < 2; p++)
          for (int q = 0; q < 2; q++)
            if (ea[p] == eb[q] && (best < 0 || ea[p] < best)) best = ea[p];
        if (best != x) continue;
        if (out) out[cnt] = make_edge(a, b);
        cnt++;
      }
  }
  free(off);
  free(lst);
  return cnt;
}

/*
 * Tier B, the method's own steps (Alg. 3 with the undirected node-local MST of
 * Sec. 5.3): per vertex, its records in the record order R1, emit each
 * consecutive pair. Emits exactly sum_i (d_i - 1) over vertices with d_i >= 1
 * rows, i.e. 2n - V'. Rows are in vertex order, then list order.
 */
static int cmp_rec(const void *pa, const void *pb) {
  uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
  if (a == b) return 0;
  return rec_before(a, b) ? -1 : 1;
}

int64_t oracle_skeleton(int64_t n, const int32_t *src, const int32_t *dst, const int64_t *t, int64_t V,
                        lg_edge *out) {
  int64_t *off;
  uint32_t *lst;
  if (build_incidence(n, src, dst, V, &off, &lst)) return OR_ENOMEM;
  g_t = t;
  int64_t cnt = 0;
  for (int64_t x = 0; x < V; x++) {
    int64_t d = off[x + 1] - off[x];
    if (d < 2) continue;
    qsort(lst + off[x], (size_t)d, sizeof(uint32_t), cmp_rec); /* the vertex's records in time order */
    for (int64_t k = off[x] + 1; k < off[x + 1]; k++) {
      if (out) out[cnt] = make_edge(lst[k - 1], lst[k]);
      cnt++;
    }
  }
  free(off);
  free(lst);
  return cnt;
}

/*
 * CAUSAL mode, Tier A: the increment-weighted line graph of Def. 1. An arc
 * joins record r to record s when r's head vertex is s's tail vertex (P1,
 * tip-to-tail) and t_r <= t_s (P2), with weight t_s - t_r (P3). The arc is
 * found at that shared vertex i: r is an in-edge of i, s an out-edge. Rows are
 * (tail = r, head = s, w); the canonical key is the same K = (w, head,
 * 2^32-1-tail) (reading C2). Antiparallel arcs between one pair of records
 * (possible only at equal times) are two rows with different keys.
 */
int64_t oracle_causal_line_graph(int64_t n, const int32_t *src, const int32_t *dst, const int64_t *t,
                                 int64_t V, lg_edge *out) {
  int64_t *off;
  uint32_t *lst;
  if (build_incidence(n, src, dst, V, &off, &lst)) return OR_ENOMEM;
  int64_t cnt = 0;
  for (int64_t x = 0; x < V; x++) {
    for (int64_t i = off[x]; i < off[x + 1]; i++) {
      uint32_t r = lst[i];
      if (dst[r] != x) continue; /* r must arrive at x */
      for (int64_t j = off[x]; j < off[x + 1]; j++) {
        uint32_t q = lst[j];
        if (src[q] != x || t[r] > t[q]) continue; /* q must leave x, not earlier */
        if (out) {
          out[cnt].tail = r;
          out[cnt].head = q;
          out[cnt].w = t[q] - t[r];
        }
        cnt++;
      }
    }
  }
  free(off);
  free(lst);
  return cnt;
}

/*
 * CAUSAL mode, Tier B: at every vertex x the minimum spanning forest of the
 * node-local increment-weighted line graph (Def. 1 restricted to the arcs made
 * at x: every arrival joined to every departure that is not earlier), which
 * Thm 2 builds without that graph; the vertices' forests are united as in
 * Alg. 3. The records at x are ordered by time, arrivals before departures at
 * equal times, then by id (reading C1). A departure e then needs arcs only
 * from the arrivals since the departure before it, and from the latest
 * arrival before that departure: any earlier arrival a reaches that latest
 * arrival through the previous departure over arcs no heavier than t_e - t_a,
 * so its own arc to e is the heaviest on a cycle. The first departure takes
 * every arrival before it; with no arrival before the previous departure
 * nothing is carried (reading C3).
 */
static int32_t g_x;          /* the vertex whose list is being sorted */
static const int32_t *g_dst; /* record heads, to tell arrivals at g_x */

static int cmp_causal(const void *pa, const void *pb) {
  uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
  if (g_t[a] != g_t[b]) return g_t[a] < g_t[b] ? -1 : 1;
  int ia = g_dst[a] == g_x, ib = g_dst[b] == g_x; /* 1 = arrives at x */
  if (ia != ib) return ia ? -1 : 1;
  if (a != b) return a < b ? -1 : 1;
  return 0;
}

/* the arc from arrival a to departure e (Def. 1: weight t_e - t_a) */
static void put_arc(lg_edge *out, int64_t *cnt, uint32_t a, uint32_t e, const int64_t *t) {
  if (out) {
    out[*cnt].tail = a;
    out[*cnt].head = e;
    out[*cnt].w = t[e] - t[a];
  }
  (*cnt)++;
}

int64_t oracle_causal_skeleton(int64_t n, const int32_t *src, const int32_t *dst, const int64_t *t, int64_t V,
                               lg_edge *out) {
  int64_t *off;
  uint32_t *lst;
  if (build_incidence(n, src, dst, V, &off, &lst)) return OR_ENOMEM;
  g_t = t;
  g_dst = dst;
  int64_t cnt = 0;
  for (int64_t x = 0; x < V; x++) {
    int64_t d = off[x + 1] - off[x];
    if (d < 2) continue;
    g_x = (int32_t)x;
    qsort(lst + off[x], (size_t)d, sizeof(uint32_t), cmp_causal);
    int64_t since = off[x];  /* first position after the previous departure */
    int64_t carried = -1;    /* position of the latest arrival before the previous departure */
    int64_t latest = -1;     /* position of the latest arrival so far */
    for (int64_t k = off[x]; k < off[x + 1]; k++) {
      if (dst[lst[k]] == x) { latest = k; continue; }
      if (carried >= 0) put_arc(out, &cnt, lst[carried], lst[k], t);
      for (int64_t j = since; j < k; j++)
        if (dst[lst[j]] == x) put_arc(out, &cnt, lst[j], lst[k], t);
      carried = latest; since = k + 1;
    }
  }
  free(off);
  free(lst);
  return cnt;
}

/* progress lines on stderr for runs of billions of rows (CE_ORACLE_PROGRESS=1) */
static int progress_on(void) {
  static int on = -1;
  if (on < 0) {
    const char *e = getenv("CE_ORACLE_PROGRESS");
    on = e && e[0] == '1';
  }
  return on;
}
static void progress(const char *what, int64_t done, int64_t total) {
  if (!progress_on()) return;
  fprintf(stderr, "[oracle] %s %lld/%lld\n", what, (long long)done, (long long)total);
  fflush(stderr);
}
#define PROGRESS_EVERY(k, what, total) \
  do { if (((k) & ((1 << 26) - 1)) == 0) progress((what), (k), (total)); } while (0)

/* plain union-find with path halving */
static uint32_t uf_find(uint32_t *par, uint32_t x) {
  while (par[x] != x) {
    par[x] = par[par[x]];
    x = par[x];
  }
  return x;
}

/*
 * Alg. 1 steps 1-2: Kruskal in ascending K (R3) over the given line-graph
 * edges (sorted in place). Writes the MSF rows in ascending K; returns m.
 */
int64_t oracle_kruskal(int64_t n, int64_t E, lg_edge *edges, const int64_t *t, uint32_t *msf_tail,
                       uint32_t *msf_head, int64_t *msf_w) {
  g_t = t;
  qsort(edges, (size_t)E, sizeof(lg_edge), cmp_key);
  uint32_t *par = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
  if (!par) return OR_ENOMEM;
  for (int64_t i = 0; i < n; i++) par[i] = (uint32_t)i;
  int64_t m = 0;
  for (int64_t k = 0; k < E; k++) {
    uint32_t a = uf_find(par, edges[k].tail), b = uf_find(par, edges[k].head);
    if (a == b) continue;
    par[a] = b;
    msf_tail[m] = edges[k].tail;
    msf_head[m] = edges[k].head;
    msf_w[m] = edges[k].w;
    m++;
  }
  free(par);
  return m;
}

/*
 * Alg. 1 step 3: dendrogram by union-find over the MSF rows in order. Row k
 * merges the sets holding tail and head; the new node is n+k with
 * left = min(child ids), right = max(child ids), w, size = sum.
 */
int oracle_dendrogram(int64_t n, int64_t m, const uint32_t *msf_tail, const uint32_t *msf_head,
                      const int64_t *msf_w, uint32_t *left, uint32_t *right, int64_t *lw,
                      uint32_t *size) {
  uint32_t *par = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
  uint32_t *node = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
  uint32_t *sz = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
  if (!par || !node || !sz) { free(par); free(node); free(sz); return OR_ENOMEM; }
  for (int64_t i = 0; i < n; i++) { par[i] = (uint32_t)i; node[i] = (uint32_t)i; sz[i] = 1; }
  for (int64_t k = 0; k < m; k++) {
    PROGRESS_EVERY(k, "dendrogram rows", m);
    uint32_t a = uf_find(par, msf_tail[k]), b = uf_find(par, msf_head[k]);
    if (a == b) { free(par); free(node); free(sz); return OR_EINVAL; } /* not a forest */
    uint32_t na = node[a], nb = node[b];
    left[k] = na < nb ? na : nb;
    right[k] = na < nb ? nb : na;
    lw[k] = msf_w[k];
    size[k] = sz[a] + sz[b];
    par[a] = b;
    sz[b] = size[k];
    node[b] = (uint32_t)(n + k);
  }
  free(par); free(node); free(sz);
  return OR_OK;
}

/*
 * Checker for the cycle property of the minimum spanning forest (App. A):
 * with the forest rows in ascending K (R3), out[i] = 1 when query edge i's
 * two records are already joined by rows of smaller key. In the unique MSF,
 * every line-graph edge that is not a row closes a cycle on which it has the
 * largest key, so it is joined below; a row itself is not. Used to check a
 * forest at sizes where Kruskal over all edges is too slow.
 */
typedef struct {
  lg_edge e;
  int64_t idx;
} lg_query;

static int cmp_query(const void *pa, const void *pb) {
  return cmp_key(&((const lg_query *)pa)->e, &((const lg_query *)pb)->e);
}

int oracle_joined_below(int64_t n, int64_t m, const uint32_t *msf_tail, const uint32_t *msf_head,
                        const int64_t *msf_w, int64_t q, const uint32_t *q_tail, const uint32_t *q_head,
                        const int64_t *q_w, uint8_t *out) {
  lg_query *qs = (lg_query *)malloc(sizeof(lg_query) * (size_t)(q ? q : 1));
  uint32_t *par = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
  if (!qs || !par) { free(qs); free(par); return OR_ENOMEM; }
  for (int64_t i = 0; i < q; i++) {
    if (q_tail[i] >= (uint64_t)n || q_head[i] >= (uint64_t)n) { free(qs); free(par); return OR_EINVAL; }
    qs[i].e.w = q_w[i];
    qs[i].e.tail = q_tail[i];
    qs[i].e.head = q_head[i];
    qs[i].idx = i;
  }
  qsort(qs, (size_t)q, sizeof(lg_query), cmp_query);
  for (int64_t i = 0; i < n; i++) par[i] = (uint32_t)i;
  int64_t j = 0;
  for (int64_t k = 0; k < q; k++) {
    PROGRESS_EVERY(k, "cycle-property queries", q);
    while (j < m) {
      PROGRESS_EVERY(j, "cycle-property rows", m);
      lg_edge r;
      r.w = msf_w[j];
      r.tail = msf_tail[j];
      r.head = msf_head[j];
      if (cmp_key(&r, &qs[k].e) >= 0) break;
      uint32_t a = uf_find(par, r.tail), b = uf_find(par, r.head);
      if (a != b) par[a] = b;
      j++;
    }
    out[qs[k].idx] = uf_find(par, qs[k].e.tail) == uf_find(par, qs[k].e.head);
  }
  free(qs);
  free(par);
  return OR_OK;
}

/*
 * Alg. 5 as the paper computes it: the discrete dendrogram's level l is the
 * partition of the records into connected components of the line graph that
 * keeps only its edges with w <= thr[l]. The edges given may be the full
 * line graph, the skeleton or the forest (Thm 3: all three have the same
 * components at every threshold). Each level is computed on its own, from
 * scratch: union every kept edge, then label each record with the smallest
 * record id of its component. labels is level-major: labels[l*n + r].
 * Thresholds must be strictly increasing and >= 0.
 */
int oracle_level_components(int64_t n, int64_t E, const uint32_t *tail, const uint32_t *head, const int64_t *w,
                            int64_t q, const int64_t *thr, int32_t *labels) {
  if (n < 0 || E < 0 || q < 0 || n > 0x7fffffffLL) return OR_EINVAL;
  for (int64_t l = 0; l < q; l++)
    if (thr[l] < 0 || (l > 0 && thr[l] <= thr[l - 1])) return OR_EINVAL;
  for (int64_t e = 0; e < E; e++)
    if (tail[e] >= (uint64_t)n || head[e] >= (uint64_t)n) return OR_EINVAL;
  uint32_t *par = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
  uint32_t *low = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
  if (!par || !low) { free(par); free(low); return OR_ENOMEM; }
  for (int64_t l = 0; l < q; l++) {
    for (int64_t r = 0; r < n; r++) par[r] = (uint32_t)r;
    for (int64_t e = 0; e < E; e++) {
      if (w[e] > thr[l]) continue;
      uint32_t a = uf_find(par, tail[e]), b = uf_find(par, head[e]);
      if (a != b) par[a] = b;
    }
    /* smallest member of each component, kept at its root */
    for (int64_t r = 0; r < n; r++) low[r] = UINT32_MAX;
    for (int64_t r = 0; r < n; r++) {
      uint32_t root = uf_find(par, (uint32_t)r);
      if ((uint32_t)r < low[root]) low[root] = (uint32_t)r;
    }
    for (int64_t r = 0; r < n; r++) labels[l * n + r] = (int32_t)low[uf_find(par, (uint32_t)r)];
  }
  free(par);
  free(low);
  return OR_OK;
}

/* R5 */
static uint64_t lam(int64_t w) {
  if (w <= 0) return (uint64_t)1 << 63;
  return ((uint64_t)1 << 63) / (2 * (uint64_t)w);
}

typedef struct {
  int64_t n_clusters; /* rows written, ROOT included (last) */
  int64_t n_labels;
} condense_counts;

/*
 * Alg. 1 steps 4-5 (condense with M, extract by stability), HDBSCAN
 * semantics per R4-R7. Inputs: dendrogram rows. Outputs: per point the
 * cluster it leaves and the lambda at which it leaves; cluster rows in
 * ascending id; labels. Arrays cl_* must hold 2*floor(n/M)+1 rows.
 */
/*
 * dtop == NULL: the binary dendrogram, node n+k merging left[k] and right[k]
 * at lambda(lw[k]). dtop != NULL: the discrete dendrogram of Alg. 5 cut from
 * it (see oracle_condense_discrete): row k belongs to the D-node of its level
 * top dtop[k]; a D-node merges, at node_lam[its row], every child of its
 * block's rows that lies outside the block.
 */
static int condense_impl(int64_t n, int64_t m, const uint32_t *left, const uint32_t *right, const int64_t *lw,
                         const uint32_t *size, int64_t M, const uint32_t *dtop, const uint64_t *node_lam,
                         uint32_t *pt_cluster, uint64_t *pt_lambda, uint32_t *cl_id, uint32_t *cl_parent,
                         uint32_t *cl_size, uint64_t *cl_lambda_birth, uint64_t *cl_stab_hi,
                         uint64_t *cl_stab_lo, uint8_t *cl_selected, int32_t *labels, condense_counts *counts);

int oracle_condense(int64_t n, int64_t m, const uint32_t *left, const uint32_t *right,
                    const int64_t *lw, const uint32_t *size, int64_t M, uint32_t *pt_cluster,
                    uint64_t *pt_lambda, uint32_t *cl_id, uint32_t *cl_parent, uint32_t *cl_size,
                    uint64_t *cl_lambda_birth, uint64_t *cl_stab_hi, uint64_t *cl_stab_lo,
                    uint8_t *cl_selected, int32_t *labels, condense_counts *counts) {
  return condense_impl(n, m, left, right, lw, size, M, NULL, NULL, pt_cluster, pt_lambda, cl_id, cl_parent,
                       cl_size, cl_lambda_birth, cl_stab_hi, cl_stab_lo, cl_selected, labels, counts);
}

/*
 * Alg. 5 (discrete dendrogram) cut from the exact one: thresholds thr[0] <
 * ... < thr[q-1]; a row's level is the first threshold its weight does not
 * exceed (reading: comps(H, omega) keeps edges with w <= omega, App. A).
 * The rows must all satisfy w <= thr[q-1] (the caller drops the others: they
 * merge nothing below the last threshold). The components at a level are
 * the subtrees of rows of that level or lower; a component that first
 * appears at level i is a D-node, represented by its highest row (its level
 * top: a row whose parent has a higher level, or none). dd_level[k] is row
 * k's level, dd_top[k] the node n+j of its level top j. Condensing then
 * follows Campello et al. on this tree with several children per node: at a
 * D-node, children of size >= M are big; two or more big children each start
 * a cluster at the node's lambda = lambda(thr[level]); one continues the
 * cluster; small children shed their records at that lambda.
 */
int oracle_condense_discrete(int64_t n, int64_t m, const uint32_t *left, const uint32_t *right,
                             const int64_t *lw, const uint32_t *size, int64_t M, int64_t q, const int64_t *thr,
                             uint32_t *pt_cluster, uint64_t *pt_lambda, uint32_t *cl_id, uint32_t *cl_parent,
                             uint32_t *cl_size, uint64_t *cl_lambda_birth, uint64_t *cl_stab_hi,
                             uint64_t *cl_stab_lo, uint8_t *cl_selected, int32_t *labels, uint32_t *dd_level,
                             uint32_t *dd_top, condense_counts *counts) {
  if (q < 1) return OR_EINVAL;
  for (int64_t i = 1; i < q; i++)
    if (thr[i] <= thr[i - 1]) return OR_EINVAL;
  uint32_t *rowpar = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(m ? m : 1));
  uint64_t *nlam = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m ? m : 1));
  if (!rowpar || !nlam) { free(rowpar); free(nlam); return OR_ENOMEM; }
  for (int64_t k = 0; k < m; k++) {
    int64_t L = 0;
    while (L < q && lw[k] > thr[L]) L++;
    if (L == q) { free(rowpar); free(nlam); return OR_EINVAL; } /* above the last threshold */
    dd_level[k] = (uint32_t)L;
    nlam[k] = lam(thr[L]);
    rowpar[k] = NONE32;
  }
  for (int64_t k = 0; k < m; k++) {
    if (left[k] >= (uint64_t)n) rowpar[left[k] - n] = (uint32_t)k;
    if (right[k] >= (uint64_t)n) rowpar[right[k] - n] = (uint32_t)k;
  }
  /* parents are later rows: from the last row down, a row inherits its parent's top at equal level */
  for (int64_t k = m - 1; k >= 0; k--) {
    uint32_t p = rowpar[k];
    dd_top[k] = (p != NONE32 && dd_level[p] == dd_level[k]) ? dd_top[p] : (uint32_t)(n + k);
  }
  free(rowpar);
  int rc = condense_impl(n, m, left, right, lw, size, M, dd_top, nlam, pt_cluster, pt_lambda, cl_id, cl_parent,
                         cl_size, cl_lambda_birth, cl_stab_hi, cl_stab_lo, cl_selected, labels, counts);
  free(nlam);
  return rc;
}

static int condense_impl(int64_t n, int64_t m, const uint32_t *left, const uint32_t *right, const int64_t *lw,
                         const uint32_t *size, int64_t M, const uint32_t *dtop, const uint64_t *node_lam,
                         uint32_t *pt_cluster, uint64_t *pt_lambda, uint32_t *cl_id, uint32_t *cl_parent,
                         uint32_t *cl_size, uint64_t *cl_lambda_birth, uint64_t *cl_stab_hi,
                         uint64_t *cl_stab_lo, uint8_t *cl_selected, int32_t *labels, condense_counts *counts) {
  if (M < 2) return OR_EINVAL;
  int64_t N = n + m;            /* dendrogram nodes */
  uint32_t ROOT = (uint32_t)N;  /* virtual root */
  uint32_t *parent = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(N + 1));
  uint32_t *nsize = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(N + 1));
  uint32_t *clus = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(N + 1)); /* cluster of a big node */
  uint32_t *stack = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(N + 1));
  uint8_t *is_cluster = (uint8_t *)calloc((size_t)(N + 1), 1);
  uint32_t *cpar = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(N + 1)); /* parent cluster, by id */
  uint64_t *cbirth = (uint64_t *)calloc((size_t)(N + 1), sizeof(uint64_t));
  u128 *stab = (u128 *)calloc((size_t)(N + 1), sizeof(u128));
  if (!parent || !nsize || !clus || !stack || !is_cluster || !cpar || !cbirth || !stab) {
    free(parent); free(nsize); free(clus); free(stack); free(is_cluster); free(cpar); free(cbirth); free(stab);
    return OR_ENOMEM;
  }
  for (int64_t x = 0; x <= N; x++) { parent[x] = NONE32; clus[x] = NONE32; cpar[x] = NONE32; }
  for (int64_t x = 0; x < n; x++) nsize[x] = 1;
  for (int64_t k = 0; k < m; k++) {
    nsize[n + k] = size[k];
    parent[left[k]] = (uint32_t)(n + k);
    parent[right[k]] = (uint32_t)(n + k);
  }
  nsize[ROOT] = (uint32_t)n;
  is_cluster[ROOT] = 1;
  cbirth[ROOT] = 0;

  /* exits: every leaf under node y leaves cluster C at lambda L */
#define SHED(y, C, L)                                                      \
  do {                                                                     \
    int64_t sp_ = 0;                                                       \
    stack[sp_++] = (y);                                                    \
    while (sp_) {                                                          \
      uint32_t z_ = stack[--sp_];                                          \
      if (z_ < (uint32_t)n) { pt_cluster[z_] = (C); pt_lambda[z_] = (L); } \
      else { stack[sp_++] = left[z_ - n]; stack[sp_++] = right[z_ - n]; }  \
    }                                                                      \
  } while (0)

  progress("condense: parents", 1, 1);
  /* R6 at ROOT: count components of size >= M */
  int64_t nbig = 0;
  for (int64_t x = 0; x < N; x++)
    if (parent[x] == NONE32 && nsize[x] >= (uint64_t)M) nbig++;
  /* work list of (big node, its cluster) processed top-down */
  uint32_t *wl_node = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(N + 1));
  int64_t wl = 0;
  if (!wl_node) { free(parent); free(nsize); free(clus); free(stack); free(is_cluster); free(cpar); free(cbirth); free(stab); return OR_ENOMEM; }
  for (int64_t x = 0; x < N; x++) {
    if (parent[x] != NONE32) continue;
    if (nsize[x] < (uint64_t)M) { SHED((uint32_t)x, ROOT, 0); continue; }
    if (nbig >= 2) {
      is_cluster[x] = 1; cpar[x] = ROOT; cbirth[x] = 0; clus[x] = (uint32_t)x;
    } else {
      clus[x] = ROOT;
    }
    wl_node[wl++] = (uint32_t)x;
  }
  /* discrete: children of a D-node, gathered by walking its block */
  uint32_t *dch = dtop ? (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(N + 1)) : NULL;
  uint32_t *blk = dtop ? (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(N + 1)) : NULL;
  if (dtop && (!dch || !blk)) {
    free(dch); free(blk); free(wl_node);
    free(parent); free(nsize); free(clus); free(stack); free(is_cluster); free(cpar); free(cbirth); free(stab);
    return OR_ENOMEM;
  }
  while (wl && dtop) {
    uint32_t x = wl_node[--wl];
    uint32_t C = clus[x];
    uint64_t L = node_lam[x - n];
    int64_t nc = 0, nb = 0, bsp = 0;
    blk[bsp++] = x;
    while (bsp) {
      uint32_t y = blk[--bsp];
      uint32_t cs[2] = {left[y - n], right[y - n]};
      for (int h = 0; h < 2; h++) {
        uint32_t c = cs[h];
        if (c >= (uint32_t)n && dtop[c - n] == x) blk[bsp++] = c; /* same block */
        else dch[nc++] = c;
      }
    }
    for (int64_t i = 0; i < nc; i++) nb += nsize[dch[i]] >= (uint64_t)M;
    for (int64_t i = 0; i < nc; i++) {
      uint32_t c = dch[i];
      if (nsize[c] < (uint64_t)M) { SHED(c, C, L); continue; }
      if (nb >= 2) { is_cluster[c] = 1; cpar[c] = C; cbirth[c] = L; clus[c] = c; }
      else clus[c] = C;
      wl_node[wl++] = c;
    }
  }
  free(dch);
  free(blk);
  while (wl) {
    uint32_t x = wl_node[--wl];
    uint32_t C = clus[x];
    int64_t k = (int64_t)x - n;
    uint32_t c1 = left[k], c2 = right[k];
    uint64_t L = lam(lw[k]);
    int b1 = nsize[c1] >= (uint64_t)M, b2 = nsize[c2] >= (uint64_t)M;
    if (b1 && b2) {
      is_cluster[c1] = 1; cpar[c1] = C; cbirth[c1] = L; clus[c1] = c1;
      is_cluster[c2] = 1; cpar[c2] = C; cbirth[c2] = L; clus[c2] = c2;
      wl_node[wl++] = c1;
      wl_node[wl++] = c2;
    } else if (b1) {
      SHED(c2, C, L);
      clus[c1] = C;
      wl_node[wl++] = c1;
    } else if (b2) {
      SHED(c1, C, L);
      clus[c2] = C;
      wl_node[wl++] = c2;
    } else {
      SHED(x, C, L);
    }
  }
#undef SHED
  free(wl_node);

  progress("condense: exits", 1, 1);
  /* O8 stability: points that leave C, and child clusters born inside C */
  for (int64_t p = 0; p < n; p++) {
    uint32_t C = pt_cluster[p];
    stab[C] += (u128)(pt_lambda[p] - cbirth[C]);
  }
  for (int64_t x = 0; x < N; x++) {
    if (!is_cluster[x]) continue;
    uint32_t P = cpar[x];
    stab[P] += (u128)nsize[x] * (u128)(cbirth[x] - cbirth[P]);
  }

  /* cluster rows in ascending id, ROOT last */
  int64_t nc = 0;
  uint32_t *row = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(N + 1));
  for (int64_t x = 0; x <= N; x++) {
    if (!is_cluster[x]) continue;
    row[x] = (uint32_t)nc;
    cl_id[nc] = (uint32_t)x;
    cl_parent[nc] = (x == N) ? NONE32 : cpar[x];
    cl_size[nc] = nsize[x];
    cl_lambda_birth[nc] = cbirth[x];
    cl_stab_hi[nc] = (uint64_t)(stab[x] >> 64);
    cl_stab_lo[nc] = (uint64_t)stab[x];
    nc++;
  }

  progress("condense: stability", 1, 1);
  /* O9 excess of mass: explicit post-order over the cluster tree */
  int64_t *child_cnt = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
  u128 *best = (u128 *)calloc((size_t)nc, sizeof(u128));
  u128 *childsum = (u128 *)calloc((size_t)nc, sizeof(u128));
  uint8_t *sel = (uint8_t *)calloc((size_t)nc, 1);
  int64_t *pending = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
  int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc ? nc : 1));
  for (int64_t r = 0; r < nc - 1; r++) child_cnt[row[cl_parent[r]]]++;
  int64_t qh = 0, qt = 0;
  for (int64_t r = 0; r < nc; r++) {
    pending[r] = child_cnt[r];
    if (pending[r] == 0) queue[qt++] = r;
  }
  while (qh < qt) {
    int64_t r = queue[qh++];
    u128 S = ((u128)cl_stab_hi[r] << 64) | cl_stab_lo[r];
    if (child_cnt[r] == 0) { sel[r] = 1; best[r] = S; }
    else if (childsum[r] > S) { sel[r] = 0; best[r] = childsum[r]; }
    else { sel[r] = 1; best[r] = S; }
    if (r == nc - 1) continue; /* ROOT has no parent */
    int64_t pr = row[cl_parent[r]];
    childsum[pr] += best[r];
    if (--pending[pr] == 0) queue[qt++] = pr;
  }
  sel[nc - 1] = 0; /* ROOT is never selected */
  /* Final choice and labels, top-down (parents before children: the reverse
   * of the post-order above). A cluster is chosen when it is selected and no
   * proper ancestor below ROOT is selected; a point's label is the chosen
   * cluster on the path from its exit cluster up to ROOT, if any. */
  uint8_t *anc_sel = (uint8_t *)calloc((size_t)nc, 1);
  int32_t *lab_row = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc ? nc : 1));
  for (int64_t i = qt - 1; i >= 0; i--) {
    int64_t r = queue[i];
    if (r == nc - 1) { anc_sel[r] = 0; lab_row[r] = -1; cl_selected[r] = 0; continue; }
    int64_t pr = row[cl_parent[r]];
    anc_sel[r] = (uint8_t)(sel[pr] || anc_sel[pr]);
    int chosen = sel[r] && !anc_sel[r];
    cl_selected[r] = (uint8_t)chosen;
    lab_row[r] = chosen ? (int32_t)r : (anc_sel[r] ? lab_row[pr] : -1);
  }
  progress("condense: selection", 1, 1);
  /* O10 labels */
  int32_t *lab_of_row = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc ? nc : 1));
  int64_t *minmem = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc ? nc : 1));
  for (int64_t r = 0; r < nc; r++) { lab_of_row[r] = -1; minmem[r] = INT64_MAX; }
  for (int64_t p = 0; p < n; p++) {
    int64_t got = lab_row[row[pt_cluster[p]]];
    labels[p] = (int32_t)got; /* temporarily the row */
    if (got >= 0 && p < minmem[got]) minmem[got] = p;
  }
  /* number chosen clusters by ascending minimum member id */
  int64_t L = 0;
  for (int64_t p = 0; p < n; p++) {
    int32_t r = labels[p];
    if (r >= 0 && minmem[r] == p) lab_of_row[r] = (int32_t)L++;
  }
  for (int64_t p = 0; p < n; p++)
    if (labels[p] >= 0) labels[p] = lab_of_row[labels[p]];
  counts->n_clusters = nc;
  counts->n_labels = L;

  free(lab_of_row); free(minmem); free(anc_sel); free(lab_row);
  free(child_cnt); free(best); free(childsum); free(sel); free(pending); free(queue); free(row);
  free(parent); free(nsize); free(clus); free(stack); free(is_cluster); free(cpar); free(cbirth); free(stab);
  return OR_OK;
}

/*
 * Whole pipeline (Alg. 4): tier 0 = definition (full line graph), tier 1 =
 * skeleton (Alg. 3); causal = 0 for the undirected line graph, 1 for the
 * increment-weighted line graph of Def. 1 (Alg. 2 per vertex in tier 1).
 * max_dt >= 0 keeps only line-graph edges with w <= max_dt (the time-filtered
 * line graph of Sec. 5.1), in either tier; max_dt < 0 keeps all.
 * Output arrays are caller-allocated: msf_* and sl_* hold n-1 rows (n >= 1),
 * cl_* hold 2*floor(n/M)+1 rows. hdr = {status, m, n_clusters, n_labels}.
 */
/* Alg. 1 on the given line-graph edges (freed here): optional time filter,
 * Kruskal, dendrogram, condensing. */
static int finish_pipeline(int64_t n, int64_t E, lg_edge *edges, const int64_t *t, int64_t M, int64_t max_dt,
                           uint32_t *msf_tail, uint32_t *msf_head, int64_t *msf_w, uint32_t *sl_left,
                           uint32_t *sl_right, int64_t *sl_w, uint32_t *sl_size, uint32_t *pt_cluster,
                           uint64_t *pt_lambda, uint32_t *cl_id, uint32_t *cl_parent, uint32_t *cl_size,
                           uint64_t *cl_lambda_birth, uint64_t *cl_stab_hi, uint64_t *cl_stab_lo,
                           uint8_t *cl_selected, int32_t *labels, int64_t *hdr) {
  if (max_dt >= 0) { /* time-filtered line graph (Sec. 5.1): keep only w <= max_dt */
    int64_t k = 0;
    for (int64_t e = 0; e < E; e++)
      if (edges[e].w <= max_dt) edges[k++] = edges[e];
    E = k;
  }
  int64_t m = oracle_kruskal(n, E, edges, t, msf_tail, msf_head, msf_w);
  free(edges);
  if (m < 0) { hdr[0] = (int)m; return (int)m; }
  int rc = oracle_dendrogram(n, m, msf_tail, msf_head, msf_w, sl_left, sl_right, sl_w, sl_size);
  if (rc) { hdr[0] = rc; return rc; }
  condense_counts cc = {0, 0};
  rc = oracle_condense(n, m, sl_left, sl_right, sl_w, sl_size, M, pt_cluster, pt_lambda, cl_id,
                       cl_parent, cl_size, cl_lambda_birth, cl_stab_hi, cl_stab_lo, cl_selected,
                       labels, &cc);
  if (rc) { hdr[0] = rc; return rc; }
  hdr[1] = m;
  hdr[2] = cc.n_clusters;
  hdr[3] = cc.n_labels;
  return OR_OK;
}

int oracle_cluster(int64_t n, const int32_t *src, const int32_t *dst, const int64_t *t, int64_t V,
                   int64_t M, int tier, int causal, int64_t max_dt, uint32_t *msf_tail, uint32_t *msf_head, int64_t *msf_w,
                   uint32_t *sl_left, uint32_t *sl_right, int64_t *sl_w, uint32_t *sl_size,
                   uint32_t *pt_cluster, uint64_t *pt_lambda, uint32_t *cl_id, uint32_t *cl_parent,
                   uint32_t *cl_size, uint64_t *cl_lambda_birth, uint64_t *cl_stab_hi,
                   uint64_t *cl_stab_lo, uint8_t *cl_selected, int32_t *labels, int64_t *hdr) {
  hdr[0] = hdr[1] = hdr[2] = hdr[3] = 0;
  if (M < 2) { hdr[0] = OR_EINVAL; return OR_EINVAL; }
  int rc = oracle_validate(n, src, dst, t, V);
  if (rc) { hdr[0] = rc; return rc; }
  int64_t (*gen)(int64_t, const int32_t *, const int32_t *, const int64_t *, int64_t, lg_edge *) =
      causal ? (tier == 0 ? oracle_causal_line_graph : oracle_causal_skeleton)
             : (tier == 0 ? oracle_full_line_graph : oracle_skeleton);
  int64_t E = gen(n, src, dst, t, V, NULL);
  if (E < 0) { hdr[0] = (int)E; return (int)E; }
  lg_edge *edges = (lg_edge *)malloc(sizeof(lg_edge) * (size_t)(E ? E : 1));
  if (!edges) { hdr[0] = OR_ENOMEM; return OR_ENOMEM; }
  gen(n, src, dst, t, V, edges);
  return finish_pipeline(n, E, edges, t, M, max_dt, msf_tail, msf_head, msf_w, sl_left, sl_right, sl_w, sl_size,
                         pt_cluster, pt_lambda, cl_id, cl_parent, cl_size, cl_lambda_birth, cl_stab_hi, cl_stab_lo,
                         cl_selected, labels, hdr);
}

/* ------------------------------------------------------------------ */
/* Dynamic hypergraphs (Sec. 5.3), readings H1-H3                      */
/* ------------------------------------------------------------------ */
/* hyperedge r is the set of members[off[r] .. off[r+1]) with time t[r] */
int oracle_hyper_validate(int64_t n, const int64_t *off, const int32_t *members, const int64_t *t, int64_t V) {
  if (n < 0 || n > 2147483647LL || V < 0) return OR_EINVAL;
  if (off[0] != 0) return OR_EINVAL;
  for (int64_t r = 0; r < n; r++)
    if (off[r + 1] < off[r]) return OR_EINVAL;
  if (off[n] > 2147483647LL) return OR_EINVAL;
  for (int64_t k = 0; k < off[n]; k++)
    if (members[k] < 0 || (int64_t)members[k] >= V) return OR_ERANGE;
  if (n == 0) return OR_OK;
  int64_t tmin = t[0], tmax = t[0];
  for (int64_t r = 0; r < n; r++) {
    if (t[r] < tmin) tmin = t[r];
    if (t[r] > tmax) tmax = t[r];
  }
  if ((u128)((__int128)tmax - (__int128)tmin) >= ((u128)1 << 62)) return OR_ERANGE;
  return OR_OK;
}

/*
 * Tier A, the definition (H2): every unordered pair of distinct hyperedges
 * whose sets meet is one line-graph edge. For each hyperedge a its vertices
 * are stamped with a; a later hyperedge b is adjacent when one of its members
 * carries the stamp. If out == NULL only the count is returned.
 */
int64_t oracle_hyper_line_graph(int64_t n, const int64_t *off, const int32_t *members, const int64_t *t, int64_t V,
                                lg_edge *out) {
  int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(V ? V : 1));
  if (!stamp) return OR_ENOMEM;
  for (int64_t v = 0; v < V; v++) stamp[v] = -1;
  g_t = t;
  int64_t cnt = 0;
  for (int64_t a = 0; a < n; a++) {
    for (int64_t k = off[a]; k < off[a + 1]; k++) stamp[members[k]] = a;
    for (int64_t b = a + 1; b < n; b++) {
      int meet = 0;
      for (int64_t k = off[b]; k < off[b + 1] && !meet; k++) meet = stamp[members[k]] == a;
      if (!meet) continue;
      if (out) out[cnt] = make_edge((uint32_t)a, (uint32_t)b);
      cnt++;
    }
  }
  free(stamp);
  return cnt;
}

/*
 * Tier B, the method's steps for hypergraphs (H3, Sec. 5.3): the incident
 * hyperedges of every vertex (each once, H1) sorted by the record order R1,
 * then each consecutive pair. Emits sum_i (d_i - 1) rows over vertices with
 * d_i >= 1; a pair consecutive at several vertices appears once per vertex
 * (Kruskal keeps one).
 */
int64_t oracle_hyper_skeleton(int64_t n, const int64_t *off, const int32_t *members, const int64_t *t, int64_t V,
                              lg_edge *out) {
  int64_t nnz = off[n];
  int64_t *voff = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(V + 1));
  int64_t *last = (int64_t *)malloc(sizeof(int64_t) * (size_t)(V + 1));
  uint32_t *lst = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nnz + 1));
  if (!voff || !fill || !last || !lst) { free(voff); free(fill); free(last); free(lst); return OR_ENOMEM; }
  /* incidence lists E_i with each hyperedge once per vertex */
  for (int64_t v = 0; v < V; v++) last[v] = -1;
  for (int64_t r = 0; r < n; r++)
    for (int64_t k = off[r]; k < off[r + 1]; k++)
      if (last[members[k]] != r) { last[members[k]] = r; voff[members[k] + 1]++; }
  for (int64_t v = 0; v < V; v++) voff[v + 1] += voff[v];
  memcpy(fill, voff, sizeof(int64_t) * (size_t)V);
  for (int64_t v = 0; v < V; v++) last[v] = -1;
  for (int64_t r = 0; r < n; r++)
    for (int64_t k = off[r]; k < off[r + 1]; k++)
      if (last[members[k]] != r) { last[members[k]] = r; lst[fill[members[k]]++] = (uint32_t)r; }
  g_t = t;
  int64_t cnt = 0;
  for (int64_t x = 0; x < V; x++) {
    int64_t d = voff[x + 1] - voff[x];
    if (d < 2) continue;
    qsort(lst + voff[x], (size_t)d, sizeof(uint32_t), cmp_rec); /* incident hyperedges in time order */
    for (int64_t k = voff[x] + 1; k < voff[x + 1]; k++) {
      const uint32_t prev = lst[k - 1], cur = lst[k];
      if (out) out[cnt] = make_edge(prev, cur);
      cnt++;
    }
  }
  free(voff); free(fill); free(last); free(lst);
  return cnt;
}

/* Whole pipeline on a dynamic hypergraph; tier 0 = definition, 1 = skeleton;
 * outputs and hdr as in oracle_cluster, per hyperedge. */
int oracle_cluster_hyper(int64_t n, const int64_t *off, const int32_t *members, const int64_t *t, int64_t V,
                         int64_t M, int tier, int64_t max_dt, uint32_t *msf_tail, uint32_t *msf_head,
                         int64_t *msf_w, uint32_t *sl_left, uint32_t *sl_right, int64_t *sl_w, uint32_t *sl_size,
                         uint32_t *pt_cluster, uint64_t *pt_lambda, uint32_t *cl_id, uint32_t *cl_parent,
                         uint32_t *cl_size, uint64_t *cl_lambda_birth, uint64_t *cl_stab_hi,
                         uint64_t *cl_stab_lo, uint8_t *cl_selected, int32_t *labels, int64_t *hdr) {
  hdr[0] = hdr[1] = hdr[2] = hdr[3] = 0;
  if (M < 2) { hdr[0] = OR_EINVAL; return OR_EINVAL; }
  int rc = oracle_hyper_validate(n, off, members, t, V);
  if (rc) { hdr[0] = rc; return rc; }
  int64_t (*gen)(int64_t, const int64_t *, const int32_t *, const int64_t *, int64_t, lg_edge *) =
      tier == 0 ? oracle_hyper_line_graph : oracle_hyper_skeleton;
  int64_t E = gen(n, off, members, t, V, NULL);
  if (E < 0) { hdr[0] = (int)E; return (int)E; }
  lg_edge *edges = (lg_edge *)malloc(sizeof(lg_edge) * (size_t)(E ? E : 1));
  if (!edges) { hdr[0] = OR_ENOMEM; return OR_ENOMEM; }
  gen(n, off, members, t, V, edges);
  return finish_pipeline(n, E, edges, t, M, max_dt, msf_tail, msf_head, msf_w, sl_left, sl_right, sl_w, sl_size,
                         pt_cluster, pt_lambda, cl_id, cl_parent, cl_size, cl_lambda_birth, cl_stab_hi, cl_stab_lo,
                         cl_selected, labels, hdr);
}
