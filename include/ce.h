/*
 * ce.h -- C ABI of the MI355X (gfx950) edge-clustering library libce.so.
 *
 * Computes the hierarchical edge clustering of a dynamic multigraph
 * (arXiv 2311.10337, "Scalable Edge Clustering of Dynamic Graphs via
 * Weighted Line Graphs"). In the default undirected mode the line-graph
 * nodes are the temporal edges (Sec. 1.2.2), two are adjacent when they share
 * a vertex, with weight |t_a - t_b|; the causal mode (Def. 1), the time
 * cutoff (Sec. 5.1), the discrete dendrogram (Alg. 5) and dynamic hypergraphs
 * (Sec. 5.3) are described with their parameters and entry points below. The
 * library
 *   1. groups each vertex's incident temporal edges and sorts them by time
 *      (the per-vertex lists of Alg. 3, in time order as in Alg. 2),
 *   2. emits the line-graph skeleton L* = union of node-local MSTs, which for
 *      |t_a - t_b| weights is the path through each time-sorted list
 *      (Alg. 3; Sec. 5.3), never forming the line graph,
 *   3. runs Alg. 1 on L* (Alg. 4): minimum spanning forest, sorted MSF,
 *      union-find dendrogram, condensing with the minimum cluster size M,
 *      extraction by stability (HDBSCAN excess of mass).
 * The skeleton has the same weighted connectivity as the full line graph
 * (App. A, Thm 3), so every output equals that of the full line graph.
 *
 * Conventions (all ids 0-based; a temporal edge's id is its input index):
 *   record order  e < f  iff  (t_e, e) < (t_f, f)
 *   line-graph edge {a,b}: tail = <-min, head = <-max, w = t_head - t_tail
 *   canonical key K = (w, head, 2^32-1-tail), lexicographic -> unique MSF
 *   MSF rows (tail, head, w) in ascending K;  m = n - #components
 *   dendrogram row k creates node n+k: left = min(child ids),
 *     right = max(child ids), w, size (leaf nodes are the records 0..n-1)
 *   lambda(w) = floor(2^63 / max(2w,1)); virtual ROOT = node n+m, lambda 0
 *   clusters: id = dendrogram node at which the cluster is born; rows in
 *     ascending id, ROOT last; stability exact unsigned 128-bit (hi, lo)
 *   labels: -1 = noise, else 0..L-1 numbered by ascending minimum member id
 *
 * Memory: every pointer argument except `params`, `out` (the struct itself),
 * `counts` and the batch offset arrays is a DEVICE pointer on the current HIP
 * device. Inputs are read-only and owned by the caller. Outputs are owned by
 * the caller and must hold the documented row counts. Between calls the
 * library keeps only a 4 KiB pinned host page per calling thread (for the
 * small counts synchronous calls read back), the servers the caller creates,
 * and on each GPU where ce_cluster_edges_noalloc ran, its static workspace.
 *
 * Tuning (environment, optional, read on every call; outputs never depend
 * on them; a call's own ce_tuning takes precedence, see ce_tuning below):
 *   CE_KRT_LEVEL_BITS   1..12: largest number of row-index bits one global
 *                       dendrogram level takes
 *   CE_SPLIT_MIN_EDGES  live-edge count from which Boruvka splits its edges
 *                       at a pivot key (default 2^20; 0 = never)
 *   CE_RADIX_IPT        keys per thread of the radix sorts (4, 8, 16)
 *   CE_LIST_GRID        workgroups of the passes over live lists
 *   CE_TUNE_FILE        the autotuner's tuning file (per-bucket choices)
 *   CE_WEIGHT_RANKS     1: rank the weights even when they fit the key
 */
#ifndef CE_H
#define CE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CE_OK = 0,
  CE_EINVAL = -1,     /* bad argument: null pointer, n < 0, M < 2, unknown mode/flags */
  CE_ESELFLOOP = -2,  /* an input record has src == dst (the model excludes self loops, Sec. 1.2.1) */
  CE_ERANGE = -3,     /* vertex id outside [0, V), or a time span max t - min t >= 2^62 */
  CE_ENOMEM = -4,     /* workspace too small or device allocation failed */
  CE_EDEVICE = -5,    /* a HIP runtime call failed */
  CE_EBUSY = -6       /* serving queue full */
} ce_status;

/* UNDIRECTED: records sharing a vertex are adjacent, w = |t_a - t_b|, and the
 * skeleton is the time-sorted path through each vertex's records (Sec. 5.3).
 * CAUSAL: the increment-weighted line graph of Def. 1: an arc joins record r
 * to record s when r's head vertex is s's tail vertex and t_r <= t_s, with
 * w = t_s - t_r; the skeleton is Alg. 2 at every vertex (time order, in-edges
 * before out-edges at equal times, then id). MSF rows are (tail = r, head = s,
 * w) and the key is again K = (w, head, 2^32-1-tail); arcs are undirected for
 * the forest, dendrogram and condensing (Alg. 1).
 *
 * Time domain (all modes): any int64 times whose span max t - min t is below
 * 2^62 (Sec. 1.2.1 bounds nothing; the limit keeps every weight and lambda
 * exact). The key is one 63-bit word: w << s | tie bits when that fits, else
 * (wide spans) the rank of w among the skeleton's distinct weights in place
 * of w, which orders the same; the ranking costs one more sort of the
 * skeleton weights. The ranked key needs bits(rows - 1) + s <= 63, which
 * holds for every input of up to 2^30 records (undirected; causal and
 * hypergraph keys also add the tie width bits(c-1), c the largest number of
 * records arriving at one vertex at one time, or the longest run of equal
 * times). The environment variable CE_WEIGHT_RANKS=1 (read on every call)
 * ranks the weights even when w fits. */
typedef enum { CE_MODE_UNDIRECTED = 0, CE_MODE_CAUSAL = 1 } ce_mode;

/* Launch choices of one call: what the autotuner (paper_2311_10337_amd.autotune)
 * sweeps. None of them changes any output. A zero field takes the next
 * source: the environment variables CE_RADIX_IPT, CE_LIST_GRID,
 * CE_KRT_LEVEL_BITS and CE_SPLIT_MIN_EDGES (read on every call), then the
 * tuning file named by CE_TUNE_FILE (its entry for the call's bucket,
 * bits(n) and bits(num_vertices); lines "n_bits V_bits maxdeg_bits radix
 * list_grid krt_bits split" as the autotuner writes them), then the built-in
 * rules. */
typedef struct {
  uint32_t struct_size;           /* = sizeof(ce_tuning) */
  int32_t radix_keys_per_thread;  /* keys per thread of the radix sorts: 4 (sorts of up to 2^24 keys), 8
                                     (default) or 16 */
  int32_t list_grid;              /* workgroups of the passes over live lists (compaction, Boruvka minima,
                                     pointer jumping), 256..65536 (default 4096): with the list length it sets
                                     the items per thread, up to 16 */
  int32_t krt_level_bits;         /* dendrogram: the most bits one global level takes, 1..12 (default: a rule
                                     of the row count) */
  int64_t split_min_edges;        /* Boruvka's filter split runs from this many live edges (default 2^20);
                                     < 0: never */
} ce_tuning;

typedef struct {
  uint32_t struct_size;      /* = sizeof(ce_params); the earlier, shorter layouts are accepted (sizes below) */
  uint32_t mode;             /* ce_mode */
  int64_t min_cluster_size;  /* M >= 2 (Alg. 1 input) */
  int64_t num_vertices;      /* V > 0; vertex ids must lie in [0, V) */
  uint32_t flags;            /* must be 0 */
  uint32_t reserved;         /* must be 0 */
  int64_t max_dt;            /* >= 0: the time-filtered line graph (Sec. 5.1), only line-graph edges with
                                w <= max_dt; the forest is then the rows of the unfiltered one with
                                w <= max_dt (Thm 3 at that threshold). < 0: no cutoff */
  const int64_t *thresholds; /* HOST array of num_thresholds strictly increasing weights >= 0, or NULL */
  int64_t num_thresholds;    /* 0: the exact dendrogram. 1..CE_MAX_THRESHOLDS: the discrete dendrogram of
                                Alg. 5: a row's level is the first threshold its w does not exceed (rows
                                above the last one are dropped, as with max_dt); condensing runs on the
                                discrete tree, whose node at a level merges all of that level's joins at
                                once, at lambda(threshold): a node with two or more children of size >= M
                                starts a cluster for each of them; see dd_level / dd_top in ce_result */
  int64_t time_bits;         /* asynchronous calls: the caller's bound B on the time span, max t - min t <
                                2^B (0..62; 0 = 62). It fixes the key layout without reading the data
                                back (w itself when B + bits(n-1) + 1 <= 63, else ranked weights); a
                                wider span is reported as CE_ERANGE in the header. Synchronous calls
                                measure the span and ignore it. */
  const ce_tuning *tuning;   /* HOST, or NULL: launch choices (see ce_tuning) */
} ce_params;
#define CE_PARAMS_V1_SIZE 32 /* without max_dt */
#define CE_PARAMS_V2_SIZE 40 /* without the thresholds */
#define CE_PARAMS_V3_SIZE 56 /* without time_bits */
#define CE_PARAMS_V4_SIZE 64 /* without tuning */

/* The launch choices a call of n records over num_vertices vertices with
 * these params (NULL: none given) would take, after every source of
 * ce_tuning's fields; 0 in out->krt_level_bits is the built-in rule, -1 in
 * out->split_min_edges is no split. Pure host function; out->struct_size
 * must be set. Errors: CE_EINVAL. */
ce_status ce_resolve_tuning(int64_t n, int64_t num_vertices, const ce_params *params, ce_tuning *out);
#define CE_MAX_THRESHOLDS 64

/* Caller-allocated DEVICE output buffers. Any pointer may be NULL to skip
 * that output. Row capacities: rows of msf_* and sl_* >= max(n-1, 1);
 * pt_* and labels >= n; cl_* >= ce_max_clusters(n, M). */
typedef struct {
  uint32_t *msf_tail, *msf_head;
  int64_t *msf_w;
  uint32_t *sl_left, *sl_right;
  int64_t *sl_w;
  uint32_t *sl_size;
  uint32_t *pt_cluster;   /* cluster each record leaves (its exit), by record id */
  uint64_t *pt_lambda;    /* lambda at which it leaves */
  uint32_t *cl_id, *cl_parent, *cl_size; /* parent of ROOT = 0xFFFFFFFF */
  uint64_t *cl_lambda_birth;
  uint64_t *cl_stab_hi, *cl_stab_lo;
  uint8_t *cl_selected;   /* 1 = the cluster is one of the output labels */
  int32_t *labels;
  /* discrete dendrogram only (NULL otherwise), one entry per dendrogram row:
   * dd_level = the row's level (threshold index); dd_top = the node id n+j of
   * the row's level top j, the highest row reached through parents of the
   * same level: the discrete node (a component first present at that level)
   * the row belongs to. Discrete nodes are the rows with dd_top == own node;
   * a node's parent is the dd_top of its parent row. Cluster ids are such
   * node ids. */
  uint32_t *dd_level, *dd_top;
} ce_result;

/* Host-side counts filled when the call returns. */
typedef struct {
  int64_t m;           /* MSF / dendrogram rows */
  int64_t n_clusters;  /* cluster rows, ROOT included */
  int64_t n_labels;    /* L */
} ce_counts;

/* Upper bound on cluster rows, ROOT included: 2*floor(n/M) + 1. Pure. */
int64_t ce_max_clusters(int64_t n, int64_t min_cluster_size);

/* Bytes of device workspace ce_cluster_edges needs for n records over V
 * vertices. Pure host function; returns 0 on invalid arguments. */
size_t ce_workspace_bytes(int64_t n, int64_t num_vertices, const ce_params *params);

/*
 * Cluster the n temporal edges (src[i], dst[i], t[i]) (Alg. 4).
 *   src, dst : int32[n], vertex ids in [0, V), src[i] != dst[i]
 *   t        : int64[n], seconds (any unit); max(t) - min(t) < 2^62 (else
 *              CE_ERANGE); for n > 2^30 also bits(max-min) + bits(n-1) + 1 <= 63
 *   workspace: device buffer of >= ce_workspace_bytes(...) bytes, or NULL to
 *              let the library allocate (stream-ordered) and free it
 *   stream   : a hipStream_t (NULL = default stream)
 * Runs on `stream` and returns when every output is written (it waits on the
 * stream). Returns CE_OK or an error; on a data error (CE_ESELFLOOP,
 * CE_ERANGE) no output is written. Reentrant: concurrent calls need
 * distinct workspaces. ce_last_error() gives a message.
 */
ce_status ce_cluster_edges(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n,
                           const ce_params *params, const ce_result *out, ce_counts *counts,
                           void *workspace, size_t workspace_bytes, void *stream);

/*
 * Dynamic hypergraphs (Sec. 5.3, undirected). Record r is a hyperedge: the
 * vertex set members[offsets[r] .. offsets[r+1]) observed at time t[r]. Two
 * hyperedges are adjacent in the line graph when their sets meet, with weight
 * |t_r - t_s| (one line-graph edge per pair, however many vertices it
 * shares). The skeleton is, per vertex, the path through its incident
 * hyperedges in (t, id) order: sum_i (d_i - 1) <= nnz edges, the input size.
 * Everything after the skeleton is the graph pipeline, so the outputs have the
 * layout and conventions of ce_cluster_edges with hyperedges as records
 * (msf_tail/msf_head and point outputs are hyperedge ids).
 *   members  : int32[nnz] DEVICE, vertex ids in [0, params.num_vertices); a
 *              vertex listed twice in one hyperedge counts once
 *   offsets  : int64[n+1] DEVICE, offsets[0] = 0, non-decreasing,
 *              offsets[n] = nnz; an empty hyperedge is an isolated record
 *   t        : int64[n] DEVICE, seconds
 *   params   : mode must be CE_MODE_UNDIRECTED (directed hypergraphs are not
 *              supported: CE_EINVAL); max_dt and thresholds as for graphs
 * Limits: n <= 2^31-1, nnz <= 2^31-1, max t - min t < 2^62 (the key as for
 * graphs, with the longest run of equal times as its tie term). Errors:
 * CE_EINVAL for bad offsets, CE_ERANGE for a member outside [0, V) or a span
 * of 2^62 or more; no output is written on an error.
 */
/*
 * Alg. 5 by connected components, as the paper computes the discrete
 * dendrogram: one partition of the records per threshold, the components of
 * the line graph keeping only its edges with w <= threshold. By Thm 3 (at
 * every threshold) these are the components of the forest rows with
 * w <= threshold, so this runs on the sorted MSF rows that ce_cluster_edges,
 * ce_cluster_hyperedges or one graph of ce_cluster_batch wrote (any mode).
 * It is the direct counterpart of the discrete dendrogram those calls cut
 * from the exact one (dd_level / dd_top): a discrete node is a component
 * that first appears at a level.
 *   msf_tail, msf_head : uint32[m] DEVICE, record ids < n
 *   msf_w              : int64[m] DEVICE, ascending (the forest's row order)
 *   thresholds         : int64[q] HOST, >= 0, strictly increasing,
 *                        q <= CE_MAX_THRESHOLDS
 *   labels             : int32[q * n] DEVICE, level-major, caller-owned:
 *                        labels[l*n + r] = the smallest record id in r's
 *                        component at level l
 *   stream             : a hipStream_t (NULL = default stream)
 * Runs on `stream` and returns when the labels are written. Allocates
 * 8 (2q + 1) bytes of device memory for the call (stream-ordered) and no
 * workspace: each level's labels are the next level's union-find. q = 0 or
 * n = 0 writes nothing. Errors: CE_EINVAL for bad arguments or rows not in
 * ascending w, CE_ERANGE for a row naming a record >= n (labels then
 * untouched).
 */
ce_status ce_level_components(const uint32_t *msf_tail, const uint32_t *msf_head, const int64_t *msf_w, int64_t m,
                              int64_t n, const int64_t *thresholds, int64_t q, int32_t *labels, void *stream);

size_t ce_hyper_workspace_bytes(int64_t n, int64_t nnz, const ce_params *params);

ce_status ce_cluster_hyperedges(const int32_t *members, const int64_t *offsets, const int64_t *t, int64_t n,
                                int64_t nnz, const ce_params *params, const ce_result *out, ce_counts *counts,
                                void *workspace, size_t workspace_bytes, void *stream);

/*
 * Batches. Many independent graphs can be clustered in one call: graph g owns
 * the records [edge_offsets[g], edge_offsets[g+1]) of src/dst/t and the
 * vertex ids [0, vertex_offsets[g+1] - vertex_offsets[g]) (ids are local to
 * each graph). Two graphs share no vertex, so the line graph of the batch has
 * no edge between them (Sec. 1.2.2) and the batch is their disjoint union:
 * every graph's outputs equal those of ce_cluster_edges on that graph alone
 * (Alg. 4 applied per graph), in that graph's local ids:
 *   records 0..n_g-1 (input index - edge_offsets[g]), the k-th dendrogram row
 *   of the graph is node n_g + k, its virtual ROOT is node n_g + m_g.
 * Layout of the outputs (DEVICE buffers of one ce_result):
 *   msf_*, sl_*          rows of graph g at [row_offsets[g], row_offsets[g+1])
 *   pt_*, labels         by input index over the whole batch
 *   cl_*                 rows of graph g at [cluster_offsets[g], cluster_offsets[g+1]),
 *                        its ROOT last; labels are numbered per graph
 * Capacities: rows of msf_*, sl_* >= max(n, 1) where n = edge_offsets[G];
 *   pt_*, labels >= n; cl_* >= sum over graphs of ce_max_clusters(n_g, M)
 *   (at most 2*floor(n/M) + G).
 * Host arrays: edge_offsets, vertex_offsets (G+1 entries each, starting at 0,
 *   edge offsets non-decreasing, every graph with >= 1 vertex); counts (G
 *   entries), row_offsets and cluster_offsets (G+1 entries) are written.
 * params.num_vertices is not used (vertex_offsets gives every graph's V).
 * 1 <= G <= CE_MAX_GRAPHS; n <= 2^31-1; vertex_offsets[G] <= 2^31.
 * Errors as for ce_cluster_edges; a data error in any graph fails the call.
 */
#define CE_MAX_GRAPHS (1LL << 24)

/* Bytes of device workspace ce_cluster_batch needs; 0 on invalid arguments. */
size_t ce_batch_workspace_bytes(const int64_t *edge_offsets, const int64_t *vertex_offsets, int64_t num_graphs,
                                const ce_params *params);

ce_status ce_cluster_batch(const int32_t *src, const int32_t *dst, const int64_t *t,
                           const int64_t *edge_offsets, const int64_t *vertex_offsets, int64_t num_graphs,
                           const ce_params *params, const ce_result *out, ce_counts *counts,
                           int64_t *row_offsets, int64_t *cluster_offsets, void *workspace,
                           size_t workspace_bytes, void *stream);

/*
 * Asynchronous calls: enqueue only (the boundary of Alg. 4 with its input and
 * output on the device). Every data-dependent count of the pipeline (spanning
 * forest rows, Boruvka's live edges and components, births, pointer-jumping
 * rounds) lives in device memory: rounds are enqueued up to bounds that hold
 * for any input of n records and return at once when their work is done, so
 * a call returns as soon as its kernels are enqueued on `stream`, never waits
 * on the host, allocates nothing, and can be captured in a HIP graph and
 * replayed (with new contents in the same buffers).
 *
 * The call's header is written on the device, to hdr (caller-owned DEVICE
 * memory of CE_HDR_WORDS(G) int64, G = 1 for ce_cluster_edges_async):
 *   hdr[0]                 ce_status of the call's data: CE_OK, CE_ESELFLOOP,
 *                          CE_ERANGE (id outside [0, V), or a time span of
 *                          more than params.time_bits bits), CE_EINVAL (bad
 *                          device offsets), CE_EDEVICE (internal)
 *   hdr[1], hdr[2], hdr[3] total rows m, cluster rows, labels
 *   hdr[4 + 3g + {0,1,2}]  graph g's m, n_clusters, n_labels
 *   hdr[4 + 3G + g]        row_offsets[g]      (g = 0..G)
 *   hdr[5 + 4G + g]        cluster_offsets[g]  (g = 0..G)
 * On a data error no output is written. ce_result_status waits for the stream
 * and reads the header.
 *
 * Limits of the asynchronous form: undirected mode only (the causal key's tie
 * width is measured on the data); a workspace must be given; for n > 2^30
 * the key layout needs params.time_bits + bits(n-1) + 1 <= 63, checked when
 * the call is made (CE_ERANGE). A declared time_bits with
 * time_bits + bits(n-1) + 1 <= 63 keeps w itself in the key; a wider (or
 * undeclared, 0) one ranks the weights, which costs one more sort. Kernel
 * timing (ce_timing_enable) is not collected.
 */
#define CE_HDR_WORDS(G) (6 + 5 * (int64_t)(G))

/* Enqueues the clustering of n records (ce_cluster_edges's inputs, outputs
 * and workspace, all DEVICE memory); the counts go to the device header hdr
 * (CE_HDR_WORDS(1) int64). Host-checked argument errors are returned at once. */
ce_status ce_cluster_edges_async(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n,
                                 const ce_params *params, const ce_result *out, int64_t *hdr, void *workspace,
                                 size_t workspace_bytes, void *stream);

/* Enqueues a batch of G graphs (ce_cluster_batch's layout) whose offsets are
 * DEVICE arrays: edge_offsets[G+1] (edge_offsets[G] = n) and
 * vertex_offsets[G+1] (vertex_offsets[G] = num_vertices), checked on the
 * device. Capacities as for ce_cluster_batch; workspace of at least
 * ce_batch_workspace_bytes_for(n, G, params) bytes. */
ce_status ce_cluster_batch_async(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n,
                                 const int64_t *edge_offsets, const int64_t *vertex_offsets, int64_t num_graphs,
                                 int64_t num_vertices, const ce_params *params, const ce_result *out, int64_t *hdr,
                                 void *workspace, size_t workspace_bytes, void *stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ce_cluster_edges_async
 * with the workspace taken from a static device array of
 * CE_NOALLOC_SCRATCH_BYTES (128 MiB) inside the library, so the call itself
 * allocates nothing. Every GPU the library runs on holds its own copy of the
 * array until the process ends. Calls whose workspace (ce_workspace_bytes)
 * exceeds it return CE_ENOMEM (with the default M = 5 and V = n/20, about
 * 650 000 records fit). All calls on one GPU share its array: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller; the array keeps the last call's contents, and the
 * pipeline initialises everything it reads. Inputs, outputs and hdr as for
 * ce_cluster_edges_async.
 */
#define CE_NOALLOC_SCRATCH_BYTES (128LL << 20)
ce_status ce_cluster_edges_noalloc(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n,
                                   const ce_params *params, const ce_result *out, int64_t *hdr, void *stream);

/* Workspace of a batch of num_graphs graphs and n records in all. Pure. */
size_t ce_batch_workspace_bytes_for(int64_t n, int64_t num_graphs, const ce_params *params);

/* Waits for `stream`, reads the device header of an asynchronous call over
 * num_graphs graphs and returns its status; fills counts[G], row_offsets[G+1]
 * and cluster_offsets[G+1] (HOST arrays; any may be NULL) when it is CE_OK. */
ce_status ce_result_status(const int64_t *hdr, int64_t num_graphs, ce_counts *counts, int64_t *row_offsets,
                           int64_t *cluster_offsets, void *stream);

/*
 * Serving: continuous batching of independent clustering requests on one GPU.
 *
 * A server allocates its whole HBM budget once (ce_server_create) and never
 * allocates device memory afterwards. input_fraction_pct of it holds the
 * records of admitted requests, resident until they finish; the rest is work
 * memory. `workers` host threads each drive their own HIP stream: a free
 * worker takes the oldest queued requests that share min_cluster_size and fit
 * the free work memory (at most max_batch_records records, 0 = 2^26) and
 * clusters them as one batch (the ce_cluster_batch computation), so requests
 * that arrive while other batches run are admitted as memory frees up and the
 * batches of different workers overlap on the device. Each request's result
 * equals what ce_cluster_edges gives for it alone: graphs of a batch are
 * clustered independently (Alg. 4 per graph).
 */
typedef struct ce_server ce_server;

typedef struct {
  uint32_t struct_size;         /* = sizeof(ce_server_config) */
  int32_t device;               /* HIP device ordinal */
  uint32_t workers;             /* 1..16 worker threads / streams */
  uint32_t input_fraction_pct;  /* 1..90: share of the budget for resident request records */
  uint64_t hbm_budget_bytes;    /* device memory the server owns (>= 1 MiB) */
  int64_t max_inflight;         /* submitted but not yet polled-complete requests (>= 1) */
  int64_t max_batch_records;    /* records per batch, 0 = 2^26 */
} ce_server_config;

typedef struct {
  uint32_t struct_size;         /* = sizeof(ce_request) */
  uint32_t reserved;            /* 0 */
  const int32_t *src, *dst;     /* HOST arrays of n records, copied to the GPU before submit returns */
  const int64_t *t;
  int64_t n;
  ce_params params;             /* min_cluster_size, num_vertices as for ce_cluster_edges */
  ce_result out;                /* caller-owned DEVICE buffers with ce_cluster_edges capacities; written
                                   when the request completes and must stay valid until then */
} ce_request;

typedef struct {
  ce_status status;             /* the request's own outcome (e.g. CE_ESELFLOOP for its data) */
  uint32_t reserved;
  ce_counts counts;
  double queue_s;               /* submit -> its batch starts */
  double latency_s;             /* submit -> its outputs are written */
} ce_request_status;

typedef struct {
  int64_t requests_submitted, requests_done, requests_batched, batches;
  int64_t max_batch_requests, max_concurrent_batches;
  int64_t input_peak_bytes, work_peak_bytes, input_capacity_bytes, work_capacity_bytes;
} ce_server_stats;

/* Starts the workers. CE_ENOMEM if the budget cannot be allocated. */
ce_status ce_server_create(const ce_server_config *config, ce_server **server);

/* Finishes every queued request, stops the workers and frees the budget. */
ce_status ce_server_destroy(ce_server *server);

/* Device bytes one request of n records occupies while it runs alone (inputs
 * plus work memory): the admission footprint. Pure host function; 0 on
 * invalid arguments. */
size_t ce_server_request_bytes(int64_t n, const ce_params *params);

/* Admits a request and returns its ticket. CE_ENOMEM: the request can never
 * fit the budget; CE_EBUSY: max_inflight reached or input memory full now
 * (retry after polling); CE_EINVAL: bad arguments. Thread-safe. */
ce_status ce_server_submit(ce_server *server, const ce_request *request, uint64_t *ticket);

/* CE_OK when the request has finished (its outcome and counts are in
 * *status and the ticket is released), CE_EBUSY while it is still queued or
 * running (with wait = 0; wait != 0 blocks until it finishes), CE_EINVAL for
 * an unknown ticket. Thread-safe. */
ce_status ce_server_poll(ce_server *server, uint64_t ticket, int wait, ce_request_status *status);

/* Counters since creation (batches formed, largest batch, most batches
 * running at once, peak memory of each region). */
ce_status ce_server_get_stats(ce_server *server, ce_server_stats *stats);

/* Thread-local text of the last error on this thread (never NULL). */
const char *ce_last_error(void);

/*
 * Diagnostics: kernel timing with HIP events. ce_timing_enable(name) makes
 * every later launch of a library kernel whose name contains `name` record a
 * pair of events on the stream it is launched on (NULL or "" turns this off)
 * and resets the totals. ce_cluster_edges collects the elapsed times before
 * it returns; ce_timing_read gives the accumulated milliseconds and launch
 * count since the last enable. Process-wide; returns 0.
 */
int ce_timing_enable(const char *kernel_name);
int ce_timing_read(double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* CE_H */
