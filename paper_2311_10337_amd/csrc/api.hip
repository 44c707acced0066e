// C ABI of libce: argument checks, workspace layout, stage orchestration.
#include <string.h>

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

bool timing_wants(const char *kernel) {
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

// A record that is a child of row j joins at row j, so it is one of that row's
// two endpoints: its input id comes from the row itself (no gathers).
__global__ __launch_bounds__(B) void k_rows(const uint64_t *msf_key, const uint4 *msf_val, const uint32_t *kc_u,
                                            const uint32_t *kc_v, const uint32_t *ksize, int64_t m, int64_t n,
                                            int idbits, ce_result out) {
  const uint64_t idmask = (uint64_t(1) << idbits) - 1;
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    const uint4 v = msf_val[j];
    const uint64_t key = msf_key[j];
    const int64_t w = (int64_t)(key >> (idbits + 1));
    const uint32_t tr = v.x, tid = v.z, hid = (uint32_t)((key >> 1) & idmask);
    if (out.msf_tail) out.msf_tail[j] = tid;
    if (out.msf_head) out.msf_head[j] = hid;
    if (out.msf_w) out.msf_w[j] = w;
    uint32_t a = kc_u[j], b = kc_v[j];
    uint32_t fa = a < (uint64_t)n ? (a == tr ? tid : hid) : a, fb = b < (uint64_t)n ? (b == tr ? tid : hid) : b;
    if (out.sl_left) out.sl_left[j] = fa < fb ? fa : fb;
    if (out.sl_right) out.sl_right[j] = fa < fb ? fb : fa;
    if (out.sl_w) out.sl_w[j] = w;
    if (out.sl_size) out.sl_size[j] = ksize[j];
  }
}

// n == 0 or n == 1: no line-graph edges; every record leaves ROOT at lambda 0
__global__ void k_trivial(int64_t n, ce_result out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint32_t ROOT = (uint32_t)n;  // m = 0
  for (int64_t p = 0; p < n; p++) {
    if (out.pt_cluster) out.pt_cluster[p] = ROOT;
    if (out.pt_lambda) out.pt_lambda[p] = 0;
    if (out.labels) out.labels[p] = -1;
  }
  if (out.cl_id) out.cl_id[0] = ROOT;
  if (out.cl_parent) out.cl_parent[0] = NONE32;
  if (out.cl_size) out.cl_size[0] = (uint32_t)n;
  if (out.cl_lambda_birth) out.cl_lambda_birth[0] = 0;
  if (out.cl_stab_hi) out.cl_stab_hi[0] = 0;
  if (out.cl_stab_lo) out.cl_stab_lo[0] = 0;
  if (out.cl_selected) out.cl_selected[0] = 0;
}

}  // namespace

ce_status stage_write_rows(Bufs &b, int64_t m, const ce_result *out, hipStream_t s) {
  if (m <= 0) return CE_OK;
  CE_LAUNCH(k_rows, dim3(grid_for(m, B)), dim3(B), 0, s, b.msf_key, b.msf_val, b.kc_u, b.kc_v, b.ksize, m, b.n,
            b.idbits, *out);
  CE_HIP(hipGetLastError());
  return CE_OK;
}

static void layout(Bufs &b, Ws &ws, int64_t n, int64_t M) {
  b.hdr = ws.alloc<uint64_t>(16);
  b.ts = ws.alloc<uint64_t>(n);
  b.perm = ws.alloc<uint32_t>(n);
  b.skel_key = ws.alloc<uint64_t>(2 * n);
  b.skel_tail = ws.alloc<uint32_t>(2 * n);
  b.skel_tid = ws.alloc<uint32_t>(2 * n);
  b.best = ws.alloc<uint64_t>(n);
  b.msf_flag = ws.alloc<uint8_t>(2 * n);
  b.msf_key = ws.alloc<uint64_t>(n);
  b.msf_val = ws.alloc<uint4>(n);
  b.kc_u = ws.alloc<uint32_t>(n);
  b.kc_v = ws.alloc<uint32_t>(n);
  b.ksize = ws.alloc<uint32_t>(n);
  size_t sc = stage_sort_skeleton_scratch(n);
  size_t x = stage_boruvka_scratch(n);
  if (x > sc) sc = x;
  x = stage_msf_sort_scratch(n);
  if (x > sc) sc = x;
  x = stage_dendrogram_scratch(n);
  if (x > sc) sc = x;
  x = stage_condense_scratch(n, M);
  if (x > sc) sc = x;
  b.scratch = ws.alloc<char>(sc);
  b.scratch_bytes = sc;
}

static ce_status check_params(int64_t n, const ce_params *p) {
  if (!p) { set_error("params is NULL"); return CE_EINVAL; }
  if (p->struct_size < sizeof(ce_params)) { set_error("params.struct_size too small"); return CE_EINVAL; }
  if (p->mode != CE_MODE_UNDIRECTED) { set_error("unknown mode"); return CE_EINVAL; }
  if (p->flags != 0 || p->reserved != 0) { set_error("flags/reserved must be 0"); return CE_EINVAL; }
  if (p->min_cluster_size < 2) { set_error("min_cluster_size must be >= 2"); return CE_EINVAL; }
  if (p->num_vertices < 1 || p->num_vertices > 0x80000000LL) { set_error("num_vertices must be in [1, 2^31]"); return CE_EINVAL; }
  if (n < 0 || n > 0x7fffffffLL) { set_error("n must be in [0, 2^31-1]"); return CE_EINVAL; }
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
  if (params) p = *params;
  else { memset(&p, 0, sizeof p); p.struct_size = sizeof p; p.min_cluster_size = 2; }
  p.num_vertices = num_vertices;
  if (check_params(n, &p) != CE_OK) return 0;
  Bufs b;
  Ws ws;
  layout(b, ws, n, p.min_cluster_size);
  return ws.peak;
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

ce_status ce_cluster_edges(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n, const ce_params *params,
                           const ce_result *out, ce_counts *counts, void *workspace, size_t workspace_bytes,
                           void *stream) {
  CE_TRY(check_params(n, params));
  if (!out || !counts) { set_error("out/counts is NULL"); return CE_EINVAL; }
  if (n > 0 && (!src || !dst || !t)) { set_error("input pointer is NULL"); return CE_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  const int64_t M = params->min_cluster_size, V = params->num_vertices;
  counts->m = 0;
  counts->n_clusters = 1;
  counts->n_labels = 0;
  const size_t need = ce_workspace_bytes(n, V, params);
  void *base = workspace;
  bool own = false;
  bool async_alloc = true;
  if (!base) {
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
  layout(b, ws, n, M);
  CE_WS_CHECK(ws);
  b.n = n;
  b.V = V;
  b.M = M;
  uint64_t flags = 0;
  int64_t tmin = 0, tmax = 0;
  CE_TRY(stage_validate(src, dst, t, b, s, &flags, &tmin, &tmax));
  if (flags & 1) { set_error("self loop in input (src == dst)"); return CE_ESELFLOOP; }
  if (flags & 2) { set_error("vertex id outside [0, num_vertices)"); return CE_ERANGE; }
  if (n <= 1) {
    CE_LAUNCH(k_trivial, dim3(1), dim3(64), 0, s, n, *out);
    CE_HIP(hipGetLastError());
    CE_HIP(hipStreamSynchronize(s));
    return CE_OK;
  }
  const uint64_t span = (uint64_t)tmax - (uint64_t)tmin;
  b.tmin = tmin;
  b.tbits = bits_for(span);
  b.idbits = bits_for((uint64_t)(n - 1));
  b.vbits = bits_for((uint64_t)(V - 1));
  b.keybits = b.tbits + b.idbits + 1;
  if (b.keybits > 64) {
    set_error("time span too wide: bits(span) + bits(n-1) + 1 > 64");
    return CE_ERANGE;
  }
  Ws sw;
  sw.base = b.scratch;
  sw.cap = b.scratch_bytes;
  int64_t m = 0;
  CE_TRY(stage_sort_skeleton(src, dst, t, b, sw, s));
  CE_TRY(stage_boruvka(b, sw, s));
  CE_TRY(stage_msf_sort(b, sw, s, &m));
  CE_TRY(stage_dendrogram(b, m, sw, s));
  CE_TRY(stage_write_rows(b, m, out, s));
  CE_TRY(stage_condense(b, m, out, sw, s, counts));
  counts->m = m;
  CE_HIP(hipStreamSynchronize(s));
  timing_collect();
  return CE_OK;
}

}  // extern "C"
