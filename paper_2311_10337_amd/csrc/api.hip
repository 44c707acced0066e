// C ABI of libce: argument checks, workspace layout, stage orchestration.
//
// One code path serves a single graph and a batch. A batch of G graphs is
// clustered as the disjoint union of its graphs (vertex ids shifted by each
// graph's vertex offset). The union's line graph has no edge between two
// graphs, so its spanning forest, dendrogram rows and clusters split exactly
// into the per-graph ones; each graph keeps its own virtual root, root rule and
// label numbering, and outputs are renumbered into each graph's local ids.
#include <string.h>
#include <sys/stat.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ce_internal.h"

namespace ce {

static thread_local std::string g_err = "no error";

void set_error(const std::string &msg) { g_err = msg; }

static std::mutex g_tmu;
static std::string g_tname;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_tev;
static double g_tms = 0.0;
static int64_t g_tcount = 0;

static thread_local bool t_timing_off = false;
TimingOff::TimingOff(bool off) : prev(t_timing_off) { t_timing_off = t_timing_off || off; }
TimingOff::~TimingOff() { t_timing_off = prev; }

bool timing_wants(const char *kernel) {
  if (t_timing_off) return false;
  std::lock_guard<std::mutex> l(g_tmu);
  return !g_tname.empty() && strstr(kernel, g_tname.c_str()) != nullptr;
}
void timing_push(hipEvent_t a, hipEvent_t b) {
  std::lock_guard<std::mutex> l(g_tmu);
  g_tev.emplace_back(a, b);
}
void timing_collect() {
  std::lock_guard<std::mutex> l(g_tmu);
  for (auto &pr : g_tev) {
    float ms = 0.f;
    if (hipEventSynchronize(pr.second) == hipSuccess && hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      g_tms += ms;
      g_tcount++;
    }
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  g_tev.clear();
}

namespace {

constexpr int B = 256;

__global__ __launch_bounds__(B) void k_iota32(uint32_t *p, Cnt nc) {
  const int64_t n = nc.get();
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) p[i] = (uint32_t)i;
}
__global__ __launch_bounds__(B) void k_zero32(uint32_t *p, Cnt nc) {
  const int64_t n = nc.get();
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) p[i] = 0u;
}

// graph of each MSF row (the graph of its tail record)
__global__ __launch_bounds__(B) void k_rowg(const uint64_t *msf_val, const uint32_t *grank, Cnt mc, uint32_t *rowg,
                                            uint32_t *key) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    const uint32_t g = grank[(uint32_t)msf_val[j]];
    rowg[j] = g;
    key[j] = g;
  }
}

// one graph: its rows are all rows
__global__ void k_moff_one(uint32_t *moff, const uint64_t *m) {
  if (threadIdx.x == 0) { moff[0] = 0; moff[1] = (uint32_t)*m; }
}

__global__ __launch_bounds__(B) void k_rowpos(const uint32_t *sorted_j, Cnt mc, uint32_t *rowpos) {
  const int64_t m = mc.get();
  for (int64_t p = (int64_t)blockIdx.x * B + threadIdx.x; p < m; p += (int64_t)gridDim.x * B)
    rowpos[sorted_j[p]] = (uint32_t)p;
}

// A record that is a child of row j joins at row j, so it is one of that row's
// two endpoints: its input id comes from the row itself (no gathers). Row j is
// written at its position in the batch, with its graph's local ids.
__global__ __launch_bounds__(B) void k_rows(const uint64_t *msf_w, const uint64_t *msf_val, const uint32_t *perm,
                                            const uint32_t *kc_u,
                                            const uint32_t *kc_v, const uint32_t *ksize, const uint32_t *rowg,
                                            const uint32_t *rowpos, const uint32_t *moff, const int64_t *eoff,
                                            Cnt mc, int64_t n, bool one, ce_result out) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    const uint64_t v = msf_val[j];
    const uint32_t tr = (uint32_t)v;
    const int64_t w = (int64_t)msf_w[j];
    // one graph: rows stay in place and local ids are the internal ones
    const uint32_t g = one ? 0u : rowg[j], p = one ? (uint32_t)j : rowpos[j], m0 = one ? 0u : moff[g];
    const uint32_t e0 = one ? 0u : (uint32_t)eoff[g], ng = one ? (uint32_t)n : (uint32_t)(eoff[g + 1] - eoff[g]);
    const uint32_t tid = perm[tr] - e0, hid = perm[v >> 32] - e0;
    if (out.msf_tail) out.msf_tail[p] = tid;
    if (out.msf_head) out.msf_head[p] = hid;
    if (out.msf_w) out.msf_w[p] = w;
    const uint32_t a = kc_u[j], b = kc_v[j];
    const uint32_t fa = a < (uint64_t)n ? (a == tr ? tid : hid) : (one ? a : ng + (rowpos[a - n] - m0));
    const uint32_t fb = b < (uint64_t)n ? (b == tr ? tid : hid) : (one ? b : ng + (rowpos[b - n] - m0));
    if (out.sl_left) out.sl_left[p] = fa < fb ? fa : fb;
    if (out.sl_right) out.sl_right[p] = fa < fb ? fb : fa;
    if (out.sl_w) out.sl_w[p] = w;
    if (out.sl_size) out.sl_size[p] = ksize[j];
  }
}

// At most one record in the whole batch: there is no line-graph edge, every
// graph's only cluster is its root (local id n_g, size n_g), and a record
// leaves its root at lambda 0 as noise.
__global__ void k_trivial(const int64_t *eoff, int64_t G, const uint64_t *hdr, ce_result out) {
  if (hdr[H_STATUS] != 0) return;  // a data error: no output is written
  for (int64_t g = threadIdx.x; g < G; g += blockDim.x) {
    const int64_t ng = eoff[g + 1] - eoff[g];
    if (ng == 1) {
      const int64_t id = eoff[g];
      if (out.pt_cluster) out.pt_cluster[id] = 1;
      if (out.pt_lambda) out.pt_lambda[id] = 0;
      if (out.labels) out.labels[id] = -1;
    }
    if (out.cl_id) out.cl_id[g] = (uint32_t)ng;
    if (out.cl_parent) out.cl_parent[g] = NONE32;
    if (out.cl_size) out.cl_size[g] = (uint32_t)ng;
    if (out.cl_lambda_birth) out.cl_lambda_birth[g] = 0;
    if (out.cl_stab_hi) out.cl_stab_hi[g] = 0;
    if (out.cl_stab_lo) out.cl_stab_lo[g] = 0;
    if (out.cl_selected) out.cl_selected[g] = 0;
  }
}

}  // namespace

size_t stage_graph_rows_scratch(int64_t n, int64_t G) {
  Ws w;
  for (int k = 0; k < 4; k++) w.alloc<uint32_t>(n);
  return w.off + radix_ws_bytes(n) + 4096;
}

// Position of every MSF row in the output: graphs in order, the rows of one
// graph in ascending key (a stable partition of the sorted MSF by graph).
// moff[g] = the first row of graph g.
ce_status stage_graph_rows(Bufs &b, Ws &ws, hipStream_t s) {
  const int64_t G = b.G, mb = b.n > 1 ? b.n - 1 : 1;
  const Cnt m(&b.hdr[H_M], mb);
  size_t m0 = ws.mark();
  uint32_t *key = ws.alloc<uint32_t>(mb), *val = ws.alloc<uint32_t>(mb);
  uint32_t *key2 = ws.alloc<uint32_t>(mb), *val2 = ws.alloc<uint32_t>(mb);
  CE_WS_CHECK(ws);
  if (G == 1) {
    CE_LAUNCH(k_zero32, dim3(grid_cap(mb, B)), dim3(B), 0, s, b.rowg, m);
    CE_LAUNCH(k_iota32, dim3(grid_cap(mb, B)), dim3(B), 0, s, b.rowpos, m);
    CE_LAUNCH(k_moff_one, dim3(1), dim3(64), 0, s, b.moff, &b.hdr[H_M]);
  } else {
    CE_LAUNCH(k_rowg, dim3(grid_cap(mb, B)), dim3(B), 0, s, b.msf_val, b.grank, m, b.rowg, key);
    CE_HIP(hipGetLastError());
    bool alt = false;
    CE_TRY((radix_sort_pairs<uint32_t, uint32_t>(key, val, key2, val2, m, 0, bits_for((uint64_t)(G - 1)), true,
                                                 &alt, ws, s)));
    CE_LAUNCH(k_rowpos, dim3(grid_cap(mb, B)), dim3(B), 0, s, alt ? val2 : val, m, b.rowpos);
    CE_TRY(segment_bounds_u32(alt ? key2 : key, m, G, b.moff, s));
  }
  CE_HIP(hipGetLastError());
  ws.release(m0);
  return CE_OK;
}

ce_status stage_write_rows(Bufs &b, const ce_result *out, hipStream_t s) {
  const int64_t mb = b.n > 1 ? b.n - 1 : 1;
  CE_LAUNCH(k_rows, dim3(grid_cap(mb, B)), dim3(B), 0, s, b.msf_key, b.msf_val, b.perm, b.kc_u, b.kc_v, b.ksize,
            b.rowg, b.rowpos, b.moff, b.eoff, Cnt(&b.hdr[H_M], mb), b.n, b.G == 1, *out);
  CE_HIP(hipGetLastError());
  return CE_OK;
}

// Workspace: a few persistent arrays, then a phase area holding
//   X  skeleton and Boruvka state (live until the MSF is sorted), at its start
//   Y  sorted MSF, dendrogram and row placement (live from the MSF sort on), at its end
// Scratch A (grouping, skeleton, Boruvka) follows X and may overlap Y; scratch
// M (MSF sort) lies between X and Y; scratch B (dendrogram, condensing) starts
// at the phase area and overlaps X.
// nnz >= 0: a hypergraph with nnz memberships (its skeleton has at most nnz rows)
static void layout(Bufs &b, Ws &ws, int64_t n, int64_t M, int64_t G, bool discrete, int64_t nnz) {
  const int64_t slots = nnz >= 0 ? (nnz > 0 ? nnz : 1) : 2 * n;
  b.slots = slots;
  b.hdr = ws.alloc<uint64_t>(kHdrWords);
  b.outhdr = ws.alloc<int64_t>(CE_HDR_WORDS(G));
  b.thr = ws.alloc<int64_t>(CE_MAX_THRESHOLDS);
  b.eoff = ws.alloc<int64_t>(G + 1);
  b.voff = ws.alloc<int64_t>(G + 1);
  b.perm = ws.alloc<uint32_t>(n);
  b.grank = ws.alloc<uint32_t>(n);
  b.rankof = ws.alloc<uint32_t>(n);
  const size_t base = ws.off;
  b.ts = ws.alloc<uint64_t>(n);
  b.skel_key = ws.alloc<uint64_t>(slots);
  b.skel_tail = ws.alloc<uint32_t>(slots);
  b.skel_tid = ws.alloc<uint32_t>(slots);
  b.best = ws.alloc<uint64_t>(n);
  b.msf_flag = ws.alloc<uint8_t>(slots);
  const size_t xbytes = ws.off - base;
  Ws y;
  y.alloc<uint64_t>(n);
  y.alloc<uint64_t>(n);
  for (int k = 0; k < 5; k++) y.alloc<uint32_t>(n);
  y.alloc<uint32_t>(G + 1);
  const size_t ybytes = y.off;
  size_t scr_a = stage_boruvka_scratch(n, slots);
  size_t x = nnz >= 0 ? stage_hyper_skeleton_scratch(n, nnz) : stage_sort_skeleton_scratch(n);
  if (x > scr_a) scr_a = x;
  x = nnz >= 0 ? 0 : stage_causal_skeleton_scratch(n);
  if (x > scr_a) scr_a = x;
  const size_t scr_m = stage_msf_sort_scratch(n);
  size_t scr_b = stage_dendrogram_scratch(n);
  x = stage_graph_rows_scratch(n, G);
  if (x > scr_b) scr_b = x;
  x = stage_condense_scratch(n, M, G, discrete);
  if (x > scr_b) scr_b = x;
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  size_t phase = xbytes + al(scr_a);
  if (xbytes + al(scr_m) + ybytes > phase) phase = xbytes + al(scr_m) + ybytes;
  if (al(scr_b) + ybytes > phase) phase = al(scr_b) + ybytes;
  ws.off = base + phase - ybytes;
  b.msf_key = ws.alloc<uint64_t>(n);
  b.msf_val = ws.alloc<uint64_t>(n);
  b.kc_u = ws.alloc<uint32_t>(n);
  b.kc_v = ws.alloc<uint32_t>(n);
  b.ksize = ws.alloc<uint32_t>(n);
  b.rowg = ws.alloc<uint32_t>(n);
  b.rowpos = ws.alloc<uint32_t>(n);
  b.moff = ws.alloc<uint32_t>(G + 1);
  char *pb = ws.base ? ws.base + base : nullptr;
  b.scratch_a = pb ? pb + xbytes : nullptr;
  b.scratch_a_bytes = phase - xbytes;
  b.scratch_m = b.scratch_a;
  b.scratch_m_bytes = phase - xbytes - ybytes;
  b.scratch_b = pb;
  b.scratch_b_bytes = phase - ybytes;
}

// fields the caller's struct has (earlier layouts end before them)
static int64_t max_dt_of(const ce_params *p) { return p->struct_size >= CE_PARAMS_V2_SIZE ? p->max_dt : -1; }

struct Thresholds {
  const int64_t *v = nullptr;
  int64_t q = 0;
};

static ce_status thresholds_of(const ce_params *p, Thresholds *th) {
  th->v = nullptr;
  th->q = 0;
  if (p->struct_size < CE_PARAMS_V3_SIZE || p->num_thresholds == 0) return CE_OK;
  if (p->num_thresholds < 0 || p->num_thresholds > CE_MAX_THRESHOLDS || !p->thresholds) {
    set_error("num_thresholds must be in [0, 64] with a thresholds array");
    return CE_EINVAL;
  }
  for (int64_t i = 0; i < p->num_thresholds; i++) {
    if (p->thresholds[i] < 0 || (i > 0 && p->thresholds[i] <= p->thresholds[i - 1])) {
      set_error("thresholds must be >= 0 and strictly increasing");
      return CE_EINVAL;
    }
  }
  th->v = p->thresholds;
  th->q = p->num_thresholds;
  return CE_OK;
}

// condensing on the discrete dendrogram needs room for nodes with many children
static bool discrete_of(const ce_params *p) { return p->struct_size >= CE_PARAMS_V3_SIZE && p->num_thresholds > 0; }

static size_t workspace_for(int64_t n, int64_t M, int64_t G, bool discrete, int64_t nnz = -1) {
  Bufs b;
  Ws ws;
  layout(b, ws, n, M, G, discrete, nnz);
  return ws.peak;
}

static ce_status check_params(const ce_params *p) {
  if (!p) { set_error("params is NULL"); return CE_EINVAL; }
  if (p->struct_size < CE_PARAMS_V1_SIZE) { set_error("params.struct_size too small"); return CE_EINVAL; }
  if (p->mode != CE_MODE_UNDIRECTED && p->mode != CE_MODE_CAUSAL) { set_error("unknown mode"); return CE_EINVAL; }
  if (p->flags != 0 || p->reserved != 0) { set_error("flags/reserved must be 0"); return CE_EINVAL; }
  if (p->min_cluster_size < 2) { set_error("min_cluster_size must be >= 2"); return CE_EINVAL; }
  return CE_OK;
}

static ce_status check_offsets(const int64_t *eoff, const int64_t *voff, int64_t G) {
  if (G < 1 || G > CE_MAX_GRAPHS) { set_error("number of graphs must be in [1, 2^24]"); return CE_EINVAL; }
  if (!eoff || !voff) { set_error("edge_offsets/vertex_offsets is NULL"); return CE_EINVAL; }
  if (eoff[0] != 0 || voff[0] != 0) { set_error("offsets must start at 0"); return CE_EINVAL; }
  for (int64_t g = 0; g < G; g++) {
    if (eoff[g + 1] < eoff[g]) { set_error("edge_offsets must be non-decreasing"); return CE_EINVAL; }
    if (voff[g + 1] <= voff[g]) { set_error("every graph needs at least one vertex"); return CE_EINVAL; }
    if (eoff[g + 1] > 0x7fffffffLL || voff[g + 1] > 0x80000000LL) {
      set_error("total records must be <= 2^31-1 and total vertices <= 2^31");
      return CE_EINVAL;
    }
  }
  return CE_OK;
}

// A dynamic hypergraph's memberships (device CSR), for run_call.
struct HyperIn {
  const int32_t *members;
  const int64_t *offsets;
  int64_t nnz;
};

// One clustering call: inputs, host-known sizes and where the offsets live.
struct Call {
  const int32_t *src = nullptr, *dst = nullptr;
  const int64_t *t = nullptr;
  int64_t n = 0, V = 0, G = 1;
  const int64_t *eoff_h = nullptr, *voff_h = nullptr;  // host offsets (G+1 each), or
  const int64_t *eoff_d = nullptr, *voff_d = nullptr;  // device offsets (asynchronous batches)
  const HyperIn *hy = nullptr;
  const ce_tuning *tuning = nullptr;
  int64_t M = 2;
  bool causal = false;
  int64_t max_dt = -1;
  Thresholds th;
  int time_bits = 0;  // asynchronous calls: the declared bound on bits(max t - min t)
};

// ---------------------------------------------------------------- tuning
namespace {

thread_local Tuning t_tuning;

struct TuneEntry {
  int nbits = 0, vbits = 0;
  Tuning t;
};
std::mutex g_tune_mu;
std::string g_tune_path;
long long g_tune_stamp = -1;
std::vector<TuneEntry> g_tune;

// The entries of the file named by CE_TUNE_FILE, read again when its name or
// time stamp changes. Lines: n_bits V_bits maxdeg_bits radix list_grid
// krt_bits split ('#' starts a comment line); the first entry of a bucket wins.
std::vector<TuneEntry> tune_entries() {
  const char *path = getenv("CE_TUNE_FILE");
  if (!path || !*path) return {};
  struct stat st;
  if (stat(path, &st) != 0) return {};
  const long long stamp = (long long)st.st_mtim.tv_sec * 1000000000LL + st.st_mtim.tv_nsec;
  std::lock_guard<std::mutex> l(g_tune_mu);
  if (g_tune_path != path || g_tune_stamp != stamp) {
    g_tune.clear();
    if (FILE *f = fopen(path, "r")) {
      char line[512];
      while (fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        TuneEntry e;
        int dbits = 0, ipt = 0, grid = 0, kb = 0;
        long long split = 0;
        if (sscanf(line, "%d %d %d %d %d %d %lld", &e.nbits, &e.vbits, &dbits, &ipt, &grid, &kb, &split) != 7)
          continue;
        if (ipt) e.t.radix_ipt = ipt;  // 0: the built-in choice
        if (grid) e.t.list_grid = grid;
        e.t.krt_level_bits = kb;
        e.t.split_min_edges = split < 0 ? INT64_MAX : (split > 0 ? split : e.t.split_min_edges);
        g_tune.push_back(e);
      }
      fclose(f);
    }
    g_tune_path = path;
    g_tune_stamp = stamp;
  }
  return g_tune;
}

}  // namespace

const Tuning &tuning() { return t_tuning; }
TuningScope::TuningScope(const Tuning &t) : prev(t_tuning) { t_tuning = t; }
TuningScope::~TuningScope() { t_tuning = prev; }

Tuning resolve_tuning(int64_t n, int64_t V, const ce_tuning *given) {
  Tuning t;
  const int nb = bits_for((uint64_t)(n > 0 ? n : 0)), vb = bits_for((uint64_t)(V > 0 ? V : 0));
  for (const TuneEntry &e : tune_entries())
    if (e.nbits == nb && e.vbits == vb) {
      t = e.t;
      break;
    }
  if (const char *e = getenv("CE_RADIX_IPT")) if (atoi(e)) t.radix_ipt = atoi(e);
  if (const char *e = getenv("CE_LIST_GRID")) if (atoi(e)) t.list_grid = atoi(e);
  if (const char *e = getenv("CE_KRT_LEVEL_BITS")) t.krt_level_bits = atoi(e);
  if (const char *e = getenv("CE_SPLIT_MIN_EDGES")) {
    const long long v = atoll(e);
    t.split_min_edges = v > 0 ? (int64_t)v : INT64_MAX;  // 0 turns the split off
  }
  if (given && given->struct_size >= sizeof(ce_tuning)) {
    if (given->radix_keys_per_thread) t.radix_ipt = given->radix_keys_per_thread;
    if (given->list_grid) t.list_grid = given->list_grid;
    if (given->krt_level_bits) t.krt_level_bits = given->krt_level_bits;
    if (given->split_min_edges) t.split_min_edges = given->split_min_edges > 0 ? given->split_min_edges : INT64_MAX;
  }
  if (t.radix_ipt != 4 && t.radix_ipt != 8 && t.radix_ipt != 16) t.radix_ipt = 8;
  if (t.list_grid < 256) t.list_grid = 256;
  if (t.list_grid > 65536) t.list_grid = 65536;
  if (t.krt_level_bits < 0) t.krt_level_bits = 0;
  if (t.krt_level_bits > 12) t.krt_level_bits = 12;
  return t;
}

namespace {

struct ThrArg {
  int64_t v[CE_MAX_THRESHOLDS];
};
__global__ void k_set_thresholds(int64_t *thr, ThrArg a, int q) {
  for (int i = threadIdx.x; i < q; i += blockDim.x) thr[i] = a.v[i];
}
__global__ void k_set_offsets_one(int64_t *eoff, int64_t *voff, int64_t n, int64_t V) {
  if (threadIdx.x == 0) { eoff[0] = 0; eoff[1] = n; voff[0] = 0; voff[1] = V; }
}
__global__ __launch_bounds__(B) void k_copy_i64(int64_t *dst, const int64_t *src, int64_t k) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < k; i += (int64_t)gridDim.x * B) dst[i] = src[i];
}
// device offsets of an asynchronous batch: start at 0, non-decreasing, every
// graph with a vertex, totals as declared; a violation is an argument error
__global__ __launch_bounds__(B) void k_check_offsets(const int64_t *eoff, const int64_t *voff, int64_t G, int64_t n,
                                                     int64_t V, uint64_t *hdr) {
  for (int64_t g = (int64_t)blockIdx.x * B + threadIdx.x; g <= G; g += (int64_t)gridDim.x * B) {
    bool bad = false;
    if (g == 0) bad = eoff[0] != 0 || voff[0] != 0;
    else bad = eoff[g] < eoff[g - 1] || voff[g] <= voff[g - 1];
    if (g == G) bad = bad || eoff[G] != n || voff[G] != V;
    if (bad) atomicOr((unsigned long long *)&hdr[H_STATUS], 4ull);
  }
}
// the call's header when there is at most one record: no rows, one cluster (the root) per graph
__global__ __launch_bounds__(B) void k_header_trivial(const uint64_t *hdr, int64_t G, int64_t *out) {
  for (int64_t g = (int64_t)blockIdx.x * B + threadIdx.x; g <= G; g += (int64_t)gridDim.x * B) {
    if (g == 0) {
      out[0] = status_of(hdr[H_STATUS]);
      out[1] = 0;
      out[2] = G;
      out[3] = 0;
    }
    if (g < G) {
      out[4 + 3 * g] = 0;
      out[4 + 3 * g + 1] = 1;
      out[4 + 3 * g + 2] = 0;
    }
    out[4 + 3 * G + g] = 0;
    out[4 + 3 * G + (G + 1) + g] = g;
  }
}

}  // namespace

// The whole pipeline on one stream. Synchronous calls (counts != nullptr)
// read the validation words back once (errors are returned at once and the
// time span's exact width sets the key layout) and the call's header at the
// end. Asynchronous calls (hdr_out, a device pointer) read nothing back: the
// key layout comes from the declared time_bits, and the header, status
// included, is written on the device.
static ce_status run_call(const Call &c, const ce_result *out, ce_counts *counts, int64_t *row_offsets,
                          int64_t *cluster_offsets, int64_t *hdr_out, void *workspace, size_t workspace_bytes,
                          hipStream_t s) {
  const TuningScope scope(resolve_tuning(c.n, c.V, c.tuning));
  const int64_t n = c.n, V = c.V, G = c.G;
  const bool sync = counts != nullptr;
  const TimingOff no_timing(!sync);
  const HyperIn *hy = c.hy;
  if (sync)
    for (int64_t g = 0; g < G; g++) counts[g] = ce_counts{0, 1, 0};
  if (hy) {
    if (!hy->offsets || (n > 0 && !c.t) || (hy->nnz > 0 && !hy->members)) {
      set_error("input pointer is NULL");
      return CE_EINVAL;
    }
  } else if (n > 0 && (!c.src || !c.dst || !c.t)) {
    set_error("input pointer is NULL");
    return CE_EINVAL;
  }
  const int64_t nnz = hy ? hy->nnz : -1;
  const size_t need = workspace_for(n, c.M, G, c.th.q > 0, nnz);
  void *base = workspace;
  bool own = false, async_alloc = true;
  if (!base) {
    if (!sync) {
      set_error("asynchronous calls need a workspace");
      return CE_EINVAL;
    }
    if (hipMallocAsync(&base, need, s) != hipSuccess) {
      (void)hipGetLastError();
      async_alloc = false;
      CE_HIP(hipMalloc(&base, need));
    }
    own = true;
  } else if (workspace_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return CE_ENOMEM;
  }
  struct Guard {
    void *p; bool own; bool async_alloc; hipStream_t s;
    ~Guard() {
      if (!own || !p) return;
      (void)hipStreamSynchronize(s);
      if (async_alloc) { (void)hipFreeAsync(p, s); (void)hipStreamSynchronize(s); }
      else (void)hipFree(p);
    }
  } guard{base, own, async_alloc, s};

  Ws ws;
  ws.base = (char *)base;
  ws.cap = need;
  Bufs b;
  layout(b, ws, n, c.M, G, c.th.q > 0, nnz);
  CE_WS_CHECK(ws);
  b.n = n;
  b.V = V;
  b.M = c.M;
  b.G = G;
  int64_t *hout = sync ? b.outhdr : hdr_out;
  // offsets and thresholds reach the device without host staging (a call may be captured in a graph)
  if (c.eoff_d) {
    CE_LAUNCH(k_copy_i64, dim3(grid_for(G + 1, B, 1024)), dim3(B), 0, s, (int64_t *)b.eoff, c.eoff_d, G + 1);
    CE_LAUNCH(k_copy_i64, dim3(grid_for(G + 1, B, 1024)), dim3(B), 0, s, (int64_t *)b.voff, c.voff_d, G + 1);
  } else if (G == 1) {
    CE_LAUNCH(k_set_offsets_one, dim3(1), dim3(64), 0, s, (int64_t *)b.eoff, (int64_t *)b.voff, n, V);
  } else {
    CE_HIP(hipMemcpyAsync((void *)b.eoff, c.eoff_h, sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
    CE_HIP(hipMemcpyAsync((void *)b.voff, c.voff_h, sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
  }
  int64_t max_dt = c.max_dt;
  if (c.th.q > 0) {
    ThrArg a;
    for (int64_t i = 0; i < c.th.q; i++) a.v[i] = c.th.v[i];
    CE_LAUNCH(k_set_thresholds, dim3(1), dim3(64), 0, s, (int64_t *)b.thr, a, (int)c.th.q);
    b.q = (int)c.th.q;
    // rows above the last threshold merge nothing in the discrete dendrogram
    if (max_dt < 0 || max_dt > c.th.v[c.th.q - 1]) max_dt = c.th.v[c.th.q - 1];
  }
  CE_HIP(hipGetLastError());
  if (hy) CE_TRY(stage_hyper_validate(hy->members, hy->offsets, c.t, nnz, b, s));
  else CE_TRY(stage_validate(c.src, c.dst, c.t, b, s));
  if (c.eoff_d)
    CE_LAUNCH(k_check_offsets, dim3(grid_for(G + 1, B, 1024)), dim3(B), 0, s, b.eoff, b.voff, G, n, V, b.hdr);
  CE_HIP(hipGetLastError());
  int tbits;
  if (sync) {
    uint64_t flags = 0;
    int64_t tmin = 0, tmax = 0;
    CE_TRY(read_validation(b, s, &flags, &tmin, &tmax));
    if (flags & 4) {
      set_error(hy ? "offsets must start at 0, be non-decreasing and end at nnz" : "bad graph offsets");
      return CE_EINVAL;
    }
    if (flags & 1) { set_error("self loop in input (src == dst)"); return CE_ESELFLOOP; }
    if (flags & 2) {
      set_error(hy ? "member outside [0, num_vertices)" : "vertex id outside [0, num_vertices) of its graph");
      return CE_ERANGE;
    }
    tbits = n > 0 ? bits_for((uint64_t)tmax - (uint64_t)tmin) : 0;
    if (tbits > 62) {
      set_error("time span (max t - min t) must be below 2^62");
      return CE_ERANGE;
    }
  } else {
    tbits = c.time_bits > 0 ? c.time_bits : 62;
  }
  b.tbits = tbits;
  b.idbits = bits_for((uint64_t)(n > 1 ? n - 1 : 0));
  b.vbits = bits_for((uint64_t)(V - 1));
  b.flat = c.causal || hy;
  b.hshift = 1;  // causal and hypergraph modes set their own shifts once the tie terms are known
  b.wshift = b.idbits + 1;
  // the all-ones word marks an absent edge, so a key may use at most 63 bits:
  // w itself when it fits, else its rank among the 2n slots' weights
  if (!b.flat && !choose_key_layout(b, b.slots)) {
    set_error("time span too wide for this many records: needs bits(span) + bits(n-1) + 1 <= 63, or n <= 2^30");
    return CE_ERANGE;
  }
  if (!sync) CE_TRY(stage_check_span(b, s));
  if (n <= 1) {
    CE_LAUNCH(k_trivial, dim3(1), dim3(256), 0, s, b.eoff, G, b.hdr, *out);
    CE_LAUNCH(k_header_trivial, dim3(grid_for(G + 1, B, 1024)), dim3(B), 0, s, b.hdr, G, hout);
    CE_HIP(hipGetLastError());
  } else {
    Ws wa, wm, wb;
    wa.base = b.scratch_a;
    wa.cap = b.scratch_a_bytes;
    wm.base = b.scratch_m;
    wm.cap = b.scratch_m_bytes;
    wb.base = b.scratch_b;
    wb.cap = b.scratch_b_bytes;
    if (hy) CE_TRY(stage_hyper_skeleton(hy->members, hy->offsets, c.t, nnz, b, wa, s));
    else if (c.causal) CE_TRY(stage_causal_skeleton(c.src, c.dst, c.t, b, wa, s));
    else CE_TRY(stage_sort_skeleton(c.src, c.dst, c.t, b, wa, s));
    CE_TRY(stage_boruvka(b, wa, s));
    CE_TRY(stage_msf_sort(b, wm, s));
    if (max_dt >= 0) CE_TRY(stage_time_filter(b, max_dt, s));
    CE_TRY(stage_dendrogram(b, wb, s));
    CE_TRY(stage_graph_rows(b, wb, s));
    CE_TRY(stage_write_rows(b, out, s));
    CE_TRY(stage_condense(b, out, wb, s, hout));
  }
  if (!sync) return CE_OK;
  std::vector<int64_t> h(CE_HDR_WORDS(G));
  CE_HIP(hipMemcpyAsync(h.data(), hout, sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost, s));
  CE_HIP(hipStreamSynchronize(s));
  timing_collect();
  if (h[0] != CE_OK) {
    set_error(h[0] == CE_EDEVICE ? "internal: a bounded loop did not converge" : "input data error");
    return (ce_status)h[0];
  }
  for (int64_t g = 0; g < G; g++) counts[g] = ce_counts{h[4 + 3 * g], h[4 + 3 * g + 1], h[4 + 3 * g + 2]};
  for (int64_t g = 0; g <= G; g++) {
    if (row_offsets) row_offsets[g] = h[4 + 3 * G + g];
    if (cluster_offsets) cluster_offsets[g] = h[4 + 3 * G + (G + 1) + g];
  }
  return CE_OK;
}

}  // namespace ce

using namespace ce;

extern "C" {

int64_t ce_max_clusters(int64_t n, int64_t M) {
  if (n < 0 || M < 2) return 0;
  return 2 * (n / M) + 1;
}

size_t ce_workspace_bytes(int64_t n, int64_t num_vertices, const ce_params *params) {
  ce_params p;
  memset(&p, 0, sizeof p);
  p.struct_size = sizeof p;
  p.min_cluster_size = 2;
  if (params) {  // a caller's struct may be the shorter earlier layout
    const size_t k = params->struct_size < sizeof p ? params->struct_size : sizeof p;
    memcpy(&p, params, k);
  }
  if (check_params(&p) != CE_OK) return 0;
  if (n < 0 || n > 0x7fffffffLL || num_vertices < 1 || num_vertices > 0x80000000LL) return 0;
  return workspace_for(n, p.min_cluster_size, 1, discrete_of(&p));
}

size_t ce_batch_workspace_bytes(const int64_t *edge_offsets, const int64_t *vertex_offsets, int64_t num_graphs,
                                const ce_params *params) {
  if (check_params(params) != CE_OK || check_offsets(edge_offsets, vertex_offsets, num_graphs) != CE_OK) return 0;
  return workspace_for(edge_offsets[num_graphs], params->min_cluster_size, num_graphs, discrete_of(params));
}

size_t ce_batch_workspace_bytes_for(int64_t n, int64_t num_graphs, const ce_params *params) {
  if (check_params(params) != CE_OK || n < 0 || n > 0x7fffffffLL || num_graphs < 1 || num_graphs > CE_MAX_GRAPHS)
    return 0;
  return workspace_for(n, params->min_cluster_size, num_graphs, discrete_of(params));
}

const char *ce_last_error(void) { return g_err.c_str(); }

int ce_timing_enable(const char *kernel_name) {
  std::lock_guard<std::mutex> l(g_tmu);
  g_tname = kernel_name ? kernel_name : "";
  g_tms = 0.0;
  g_tcount = 0;
  return 0;
}

int ce_timing_read(double *total_ms, int64_t *launches) {
  std::lock_guard<std::mutex> l(g_tmu);
  if (total_ms) *total_ms = g_tms;
  if (launches) *launches = g_tcount;
  return 0;
}

static const ce_tuning *tuning_of(const ce_params *p) {
  return p->struct_size >= sizeof(ce_params) ? p->tuning : nullptr;
}

static int time_bits_of(const ce_params *p) {
  return p->struct_size >= CE_PARAMS_V4_SIZE ? (int)p->time_bits : 0;
}

ce_status ce_resolve_tuning(int64_t n, int64_t num_vertices, const ce_params *params, ce_tuning *out) {
  if (!out || out->struct_size < sizeof(ce_tuning)) {
    set_error("out must be a ce_tuning with struct_size set");
    return CE_EINVAL;
  }
  if (params) CE_TRY(check_params(params));
  const Tuning t = resolve_tuning(n, num_vertices, params ? tuning_of(params) : nullptr);
  out->radix_keys_per_thread = t.radix_ipt;
  out->list_grid = t.list_grid;
  out->krt_level_bits = t.krt_level_bits;
  out->split_min_edges = t.split_min_edges == INT64_MAX ? -1 : t.split_min_edges;
  return CE_OK;
}

// The key layout of an asynchronous call comes from the declared time_bits; it is checked before anything
// is enqueued.
static ce_status check_async_key(int time_bits, int64_t n) {
  const int tb = time_bits > 0 ? time_bits : 62, idb = bits_for((uint64_t)(n > 1 ? n - 1 : 0));
  // w itself, or its rank among the 2n slots' weights
  if (tb + idb + 1 > 63 && bits_for((uint64_t)(2 * n - 1)) + idb + 1 > 63) {
    set_error("time span too wide for this many records: needs time_bits + bits(n-1) + 1 <= 63, or n <= 2^30");
    return CE_ERANGE;
  }
  return CE_OK;
}

static ce_status single_call(Call &c, const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n,
                             const ce_params *params) {
  CE_TRY(check_params(params));
  if (params->num_vertices < 1 || params->num_vertices > 0x80000000LL) {
    set_error("num_vertices must be in [1, 2^31]");
    return CE_EINVAL;
  }
  if (n < 0 || n > 0x7fffffffLL) { set_error("n must be in [0, 2^31-1]"); return CE_EINVAL; }
  if (time_bits_of(params) < 0 || time_bits_of(params) > 62) {
    set_error("time_bits must be in [0, 62]");
    return CE_EINVAL;
  }
  c.src = src;
  c.dst = dst;
  c.t = t;
  c.n = n;
  c.V = params->num_vertices;
  c.G = 1;
  c.M = params->min_cluster_size;
  c.tuning = tuning_of(params);
  c.causal = params->mode == CE_MODE_CAUSAL;
  c.max_dt = max_dt_of(params);
  c.time_bits = time_bits_of(params);
  return thresholds_of(params, &c.th);
}

ce_status ce_cluster_edges(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n, const ce_params *params,
                           const ce_result *out, ce_counts *counts, void *workspace, size_t workspace_bytes,
                           void *stream) {
  if (!out || !counts) { set_error("out/counts is NULL"); return CE_EINVAL; }
  Call c;
  CE_TRY(single_call(c, src, dst, t, n, params));
  return run_call(c, out, counts, nullptr, nullptr, nullptr, workspace, workspace_bytes, (hipStream_t)stream);
}

// The workspace of ce_cluster_edges_noalloc: a static device array, one copy
// on every GPU the library runs on, held until the process ends. Its
// address on a device comes from hipGetSymbolAddress with that device
// current (the array's name in host code is only a stand-in), taken on the
// first call on the device and kept.
static __device__ __align__(256) unsigned char scratch[CE_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static ce_status scratch_of_current_device(void **ptr) {
  int dev = -1;
  CE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device ordinal outside [0, 64)");
    return CE_EINVAL;
  }
  std::lock_guard<std::mutex> l(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(e));
      return CE_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return CE_OK;
}

ce_status ce_cluster_edges_async(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n,
                                 const ce_params *params, const ce_result *out, int64_t *hdr, void *workspace,
                                 size_t workspace_bytes, void *stream) {
  if (!out || !hdr) { set_error("out/hdr is NULL"); return CE_EINVAL; }
  Call c;
  CE_TRY(single_call(c, src, dst, t, n, params));
  if (c.causal) {
    set_error("asynchronous calls cluster the undirected line graph (mode must be CE_MODE_UNDIRECTED)");
    return CE_EINVAL;
  }
  CE_TRY(check_async_key(c.time_bits, n));
  return run_call(c, out, nullptr, nullptr, nullptr, hdr, workspace, workspace_bytes, (hipStream_t)stream);
}

ce_status ce_cluster_edges_noalloc(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n,
                                   const ce_params *params, const ce_result *out, int64_t *hdr, void *stream) {
  if (!out || !hdr) { set_error("out/hdr is NULL"); return CE_EINVAL; }
  Call c;
  CE_TRY(single_call(c, src, dst, t, n, params));
  if (c.causal) {
    set_error("asynchronous calls cluster the undirected line graph (mode must be CE_MODE_UNDIRECTED)");
    return CE_EINVAL;
  }
  CE_TRY(check_async_key(c.time_bits, n));
  const size_t need = workspace_for(n, c.M, 1, c.th.q > 0);
  if (need > (size_t)CE_NOALLOC_SCRATCH_BYTES) {
    set_error("the call needs " + std::to_string(need) + " bytes of workspace; the static scratch holds " +
              std::to_string((size_t)CE_NOALLOC_SCRATCH_BYTES));
    return CE_ENOMEM;
  }
  void *ws = nullptr;
  CE_TRY(scratch_of_current_device(&ws));
  return run_call(c, out, nullptr, nullptr, nullptr, hdr, ws, (size_t)CE_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream);
}

size_t ce_hyper_workspace_bytes(int64_t n, int64_t nnz, const ce_params *params) {
  if (check_params(params) != CE_OK || params->mode != CE_MODE_UNDIRECTED) return 0;
  if (n < 0 || n > 0x7fffffffLL || nnz < 0 || nnz > 0x7fffffffLL) return 0;
  if (params->num_vertices < 1 || params->num_vertices > 0x80000000LL) return 0;
  return workspace_for(n, params->min_cluster_size, 1, discrete_of(params), nnz);
}

ce_status ce_cluster_hyperedges(const int32_t *members, const int64_t *offsets, const int64_t *t, int64_t n,
                                int64_t nnz, const ce_params *params, const ce_result *out, ce_counts *counts,
                                void *workspace, size_t workspace_bytes, void *stream) {
  CE_TRY(check_params(params));
  if (params->mode != CE_MODE_UNDIRECTED) {
    set_error("hypergraphs are undirected: mode must be CE_MODE_UNDIRECTED");
    return CE_EINVAL;
  }
  if (!out || !counts) { set_error("out/counts is NULL"); return CE_EINVAL; }
  if (params->num_vertices < 1 || params->num_vertices > 0x80000000LL) {
    set_error("num_vertices must be in [1, 2^31]");
    return CE_EINVAL;
  }
  if (n < 0 || n > 0x7fffffffLL) { set_error("n must be in [0, 2^31-1]"); return CE_EINVAL; }
  if (nnz < 0 || nnz > 0x7fffffffLL) { set_error("nnz must be in [0, 2^31-1]"); return CE_EINVAL; }
  const HyperIn hy{members, offsets, nnz};
  Call c;
  c.t = t;
  c.n = n;
  c.V = params->num_vertices;
  c.M = params->min_cluster_size;
  c.tuning = tuning_of(params);
  c.max_dt = max_dt_of(params);
  c.hy = &hy;
  CE_TRY(thresholds_of(params, &c.th));
  return run_call(c, out, counts, nullptr, nullptr, nullptr, workspace, workspace_bytes, (hipStream_t)stream);
}

ce_status ce_cluster_batch(const int32_t *src, const int32_t *dst, const int64_t *t, const int64_t *edge_offsets,
                           const int64_t *vertex_offsets, int64_t num_graphs, const ce_params *params,
                           const ce_result *out, ce_counts *counts, int64_t *row_offsets, int64_t *cluster_offsets,
                           void *workspace, size_t workspace_bytes, void *stream) {
  CE_TRY(check_params(params));
  if (!out || !counts || !row_offsets || !cluster_offsets) {
    set_error("out/counts/row_offsets/cluster_offsets is NULL");
    return CE_EINVAL;
  }
  CE_TRY(check_offsets(edge_offsets, vertex_offsets, num_graphs));
  Call c;
  c.src = src;
  c.dst = dst;
  c.t = t;
  c.G = num_graphs;
  c.n = edge_offsets[num_graphs];
  c.V = vertex_offsets[num_graphs];
  c.eoff_h = edge_offsets;
  c.voff_h = vertex_offsets;
  c.M = params->min_cluster_size;
  c.tuning = tuning_of(params);
  c.causal = params->mode == CE_MODE_CAUSAL;
  c.max_dt = max_dt_of(params);
  CE_TRY(thresholds_of(params, &c.th));
  return run_call(c, out, counts, row_offsets, cluster_offsets, nullptr, workspace, workspace_bytes,
                  (hipStream_t)stream);
}

ce_status ce_cluster_batch_async(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n,
                                 const int64_t *edge_offsets, const int64_t *vertex_offsets, int64_t num_graphs,
                                 int64_t num_vertices, const ce_params *params, const ce_result *out, int64_t *hdr,
                                 void *workspace, size_t workspace_bytes, void *stream) {
  CE_TRY(check_params(params));
  if (!out || !hdr || !edge_offsets || !vertex_offsets) {
    set_error("out/hdr/edge_offsets/vertex_offsets is NULL");
    return CE_EINVAL;
  }
  if (num_graphs < 1 || num_graphs > CE_MAX_GRAPHS) { set_error("number of graphs must be in [1, 2^24]"); return CE_EINVAL; }
  if (n < 0 || n > 0x7fffffffLL) { set_error("n must be in [0, 2^31-1]"); return CE_EINVAL; }
  if (num_vertices < num_graphs || num_vertices > 0x80000000LL) {
    set_error("num_vertices must be in [num_graphs, 2^31]");
    return CE_EINVAL;
  }
  if (params->mode != CE_MODE_UNDIRECTED) {
    set_error("asynchronous calls cluster the undirected line graph (mode must be CE_MODE_UNDIRECTED)");
    return CE_EINVAL;
  }
  if (time_bits_of(params) < 0 || time_bits_of(params) > 62) {
    set_error("time_bits must be in [0, 62]");
    return CE_EINVAL;
  }
  CE_TRY(check_async_key(time_bits_of(params), n));
  Call c;
  c.src = src;
  c.dst = dst;
  c.t = t;
  c.G = num_graphs;
  c.n = n;
  c.V = num_vertices;
  c.eoff_d = edge_offsets;
  c.voff_d = vertex_offsets;
  c.M = params->min_cluster_size;
  c.tuning = tuning_of(params);
  c.max_dt = max_dt_of(params);
  c.time_bits = time_bits_of(params);
  CE_TRY(thresholds_of(params, &c.th));
  return run_call(c, out, nullptr, nullptr, nullptr, hdr, workspace, workspace_bytes, (hipStream_t)stream);
}

ce_status ce_result_status(const int64_t *hdr, int64_t num_graphs, ce_counts *counts, int64_t *row_offsets,
                           int64_t *cluster_offsets, void *stream) {
  if (!hdr || num_graphs < 1 || num_graphs > CE_MAX_GRAPHS) {
    set_error("hdr is NULL or num_graphs outside [1, 2^24]");
    return CE_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<int64_t> h(CE_HDR_WORDS(num_graphs));
  CE_HIP(hipMemcpyAsync(h.data(), hdr, sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost, s));
  CE_HIP(hipStreamSynchronize(s));
  const int64_t G = num_graphs;
  if (h[0] != CE_OK) {
    set_error(h[0] == CE_ESELFLOOP ? "self loop in input (src == dst)"
              : h[0] == CE_ERANGE  ? "vertex id outside [0, V) or time span wider than time_bits"
              : h[0] == CE_EINVAL  ? "bad graph offsets"
                                   : "internal: a bounded loop did not converge");
    return (ce_status)h[0];
  }
  for (int64_t g = 0; g < G; g++) {
    if (counts) counts[g] = ce_counts{h[4 + 3 * g], h[4 + 3 * g + 1], h[4 + 3 * g + 2]};
  }
  for (int64_t g = 0; g <= G; g++) {
    if (row_offsets) row_offsets[g] = h[4 + 3 * G + g];
    if (cluster_offsets) cluster_offsets[g] = h[4 + 3 * G + (G + 1) + g];
  }
  return CE_OK;
}

}  // extern "C"
