// Serving: continuous batching of clustering requests on one GPU.
//
// A server owns one device allocation (its HBM budget), split into an input
// region, where each admitted request's records stay resident until it
// finishes, and a work region, from which every running batch takes one block
// (gathered inputs, workspace, outputs). Worker threads, each driving its own
// stream, repeatedly take the oldest queued requests that share a minimum
// cluster size and fit the free work memory, run them as one batch (each graph
// of a batch is clustered independently, so every result equals the one the
// request gets alone) and copy each request's rows into the caller's buffers.
// Requests that arrive while batches run are picked up by the next free
// worker, and batches on different streams overlap on the device.
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ce_internal.h"

namespace ce {
namespace {

constexpr int B = 256;
constexpr size_t ALIGN = 256;
constexpr int64_t MAX_BATCH_GRAPHS = 65535;  // one grid row per graph in the copy kernels
using Clock = std::chrono::steady_clock;

size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// first-fit allocator over one region, with coalescing of neighbours
class Arena {
 public:
  void init(size_t cap) {
    cap_ = cap;
    free_.clear();
    if (cap) free_[0] = cap;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = align_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      if (used_ > peak_) peak_ = used_;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes ? bytes : 1);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t cap() const { return cap_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t cap_ = 0, used_ = 0, peak_ = 0;
};

struct GatherDesc {
  const int32_t *src, *dst;
  const int64_t *t;
  int64_t n, off;
};

struct ScatterDesc {
  int64_t r0, m, p0, n, c0, nc;
  ce_result out;
};

// concatenates the requests' resident records into the batch input arrays
__global__ __launch_bounds__(B) void k_gather(const GatherDesc *d, int32_t *src, int32_t *dst, int64_t *t) {
  const GatherDesc q = d[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < q.n; i += (int64_t)gridDim.x * B) {
    src[q.off + i] = q.src[i];
    dst[q.off + i] = q.dst[i];
    t[q.off + i] = q.t[i];
  }
}

// copies each graph's slice of the batch outputs into its request's buffers
__global__ __launch_bounds__(B) void k_scatter(const ScatterDesc *d, ce_result s) {
  const ScatterDesc q = d[blockIdx.y];
  const ce_result &o = q.out;
  int64_t top = q.m > q.n ? q.m : q.n;
  if (q.nc > top) top = q.nc;
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < top; i += (int64_t)gridDim.x * B) {
    if (i < q.m) {
      const int64_t r = q.r0 + i;
      if (o.msf_tail) o.msf_tail[i] = s.msf_tail[r];
      if (o.msf_head) o.msf_head[i] = s.msf_head[r];
      if (o.msf_w) o.msf_w[i] = s.msf_w[r];
      if (o.sl_left) o.sl_left[i] = s.sl_left[r];
      if (o.sl_right) o.sl_right[i] = s.sl_right[r];
      if (o.sl_w) o.sl_w[i] = s.sl_w[r];
      if (o.sl_size) o.sl_size[i] = s.sl_size[r];
      if (o.dd_level && s.dd_level) o.dd_level[i] = s.dd_level[r];
      if (o.dd_top && s.dd_top) o.dd_top[i] = s.dd_top[r];
    }
    if (i < q.n) {
      const int64_t p = q.p0 + i;
      if (o.pt_cluster) o.pt_cluster[i] = s.pt_cluster[p];
      if (o.pt_lambda) o.pt_lambda[i] = s.pt_lambda[p];
      if (o.labels) o.labels[i] = s.labels[p];
    }
    if (i < q.nc) {
      const int64_t c = q.c0 + i;
      if (o.cl_id) o.cl_id[i] = s.cl_id[c];
      if (o.cl_parent) o.cl_parent[i] = s.cl_parent[c];
      if (o.cl_size) o.cl_size[i] = s.cl_size[c];
      if (o.cl_lambda_birth) o.cl_lambda_birth[i] = s.cl_lambda_birth[c];
      if (o.cl_stab_hi) o.cl_stab_hi[i] = s.cl_stab_hi[c];
      if (o.cl_stab_lo) o.cl_stab_lo[i] = s.cl_stab_lo[c];
      if (o.cl_selected) o.cl_selected[i] = s.cl_selected[c];
    }
  }
}

struct Request {
  uint64_t ticket = 0;
  int64_t n = 0, V = 0, M = 0;
  uint32_t mode = CE_MODE_UNDIRECTED;
  int64_t max_dt = -1;
  std::vector<int64_t> thr;  // discrete dendrogram thresholds (copied at submit)
  size_t in_off = 0, in_bytes = 0;
  ce_result out{};
  ce_counts counts{0, 1, 0};
  ce_status status = CE_OK;
  std::string err;
  Clock::time_point t_submit, t_start, t_done;
  bool done = false;
};

// output arrays of a batch of total n records and c cluster rows, laid out in one block
struct OutLayout {
  size_t off[19];
  size_t bytes;
};

OutLayout out_layout(int64_t n, int64_t c) {
  const size_t R = n > 1 ? (size_t)n : 1, P = n > 0 ? (size_t)n : 1, C = c > 0 ? (size_t)c : 1;
  const size_t sz[19] = {4u * R, 4u * R, 8u * R, 4u * R, 4u * R, 8u * R, 4u * R,   // msf_*, sl_*
                         4u * P, 8u * P,                                           // pt_*
                         4u * C, 4u * C, 4u * C, 8u * C, 8u * C, 8u * C, 1u * C,   // cl_*
                         4u * P,                                                   // labels
                         4u * R, 4u * R};                                          // dd_level, dd_top
  OutLayout L;
  size_t at = 0;
  for (int k = 0; k < 19; k++) {
    L.off[k] = at;
    at += align_up(sz[k]);
  }
  L.bytes = at;
  return L;
}

ce_result out_pointers(char *base, const OutLayout &L) {
  ce_result r;
  r.msf_tail = (uint32_t *)(base + L.off[0]);
  r.msf_head = (uint32_t *)(base + L.off[1]);
  r.msf_w = (int64_t *)(base + L.off[2]);
  r.sl_left = (uint32_t *)(base + L.off[3]);
  r.sl_right = (uint32_t *)(base + L.off[4]);
  r.sl_w = (int64_t *)(base + L.off[5]);
  r.sl_size = (uint32_t *)(base + L.off[6]);
  r.pt_cluster = (uint32_t *)(base + L.off[7]);
  r.pt_lambda = (uint64_t *)(base + L.off[8]);
  r.cl_id = (uint32_t *)(base + L.off[9]);
  r.cl_parent = (uint32_t *)(base + L.off[10]);
  r.cl_size = (uint32_t *)(base + L.off[11]);
  r.cl_lambda_birth = (uint64_t *)(base + L.off[12]);
  r.cl_stab_hi = (uint64_t *)(base + L.off[13]);
  r.cl_stab_lo = (uint64_t *)(base + L.off[14]);
  r.cl_selected = (uint8_t *)(base + L.off[15]);
  r.labels = (int32_t *)(base + L.off[16]);
  r.dd_level = (uint32_t *)(base + L.off[17]);
  r.dd_top = (uint32_t *)(base + L.off[18]);
  return r;
}

int64_t clusters_bound(int64_t n, int64_t M) { return 2 * (n / M) + 1; }

// work memory of a batch: gathered inputs, descriptor tables, outputs, workspace
size_t batch_bytes(const std::vector<Request *> &rs, int64_t M) {
  const int64_t G = (int64_t)rs.size();
  std::vector<int64_t> eoff(G + 1, 0), voff(G + 1, 0);
  int64_t C = 0;
  for (int64_t g = 0; g < G; g++) {
    eoff[g + 1] = eoff[g] + rs[g]->n;
    voff[g + 1] = voff[g] + rs[g]->V;
    C += clusters_bound(rs[g]->n, M);
  }
  const int64_t n = eoff[G];
  ce_params p;
  memset(&p, 0, sizeof p);
  p.struct_size = sizeof p;
  p.min_cluster_size = M;
  p.num_vertices = voff[G];
  p.num_thresholds = (int64_t)rs[0]->thr.size();  // sizing only looks at whether there are any
  p.thresholds = rs[0]->thr.data();
  size_t ws = ce_batch_workspace_bytes(eoff.data(), voff.data(), G, &p);
  if (G == 1) {
    const size_t w1 = ce_workspace_bytes(rs[0]->n, rs[0]->V, &p);
    return align_up(w1);  // one request runs straight into its own buffers
  }
  return align_up(4 * (size_t)n) * 2 + align_up(8 * (size_t)n) + align_up(sizeof(GatherDesc) * G) +
         align_up(sizeof(ScatterDesc) * G) + out_layout(n, C).bytes + align_up(ws);
}

}  // namespace
}  // namespace ce

using namespace ce;

struct ce_server {
  int device = 0;
  char *mem = nullptr;
  size_t in_cap = 0;
  Arena in_arena, work_arena;
  hipStream_t copy_stream = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  int64_t inflight = 0, max_inflight = 0, max_batch_records = 0;
  int running = 0;
  bool stop = false;
  ce_server_stats st{};

  void worker(int k);
  void run_batch(std::vector<Request *> &rs, size_t work_off, hipStream_t s);
};

// every request of a batch shares M, the mode and the cutoff
void ce_server::run_batch(std::vector<Request *> &rs, size_t work_off, hipStream_t s) {
  const int64_t M = rs[0]->M;
  const int64_t G = (int64_t)rs.size();
  char *in = mem, *work = mem + in_cap + work_off;
  ce_params p;
  memset(&p, 0, sizeof p);
  p.struct_size = sizeof p;
  p.min_cluster_size = M;
  p.mode = rs[0]->mode;
  p.max_dt = rs[0]->max_dt;
  p.thresholds = rs[0]->thr.empty() ? nullptr : rs[0]->thr.data();
  p.num_thresholds = (int64_t)rs[0]->thr.size();
  auto input = [&](Request *r, int k) -> char * {
    const size_t n = (size_t)r->n;
    const size_t offs[3] = {0, align_up(4 * n), 2 * align_up(4 * n)};
    return in + r->in_off + offs[k];
  };
  auto solo = [&](Request *r) {
    p.num_vertices = r->V;
    const size_t need = ce_workspace_bytes(r->n, r->V, &p);
    r->status = ce_cluster_edges((const int32_t *)input(r, 0), (const int32_t *)input(r, 1),
                                 (const int64_t *)input(r, 2), r->n, &p, &r->out, &r->counts, work, need, s);
    if (r->status != CE_OK) r->err = ce_last_error();
  };
  if (G == 1) {
    solo(rs[0]);
    return;
  }
  std::vector<int64_t> eoff(G + 1, 0), voff(G + 1, 0);
  int64_t C = 0;
  for (int64_t g = 0; g < G; g++) {
    eoff[g + 1] = eoff[g] + rs[g]->n;
    voff[g + 1] = voff[g] + rs[g]->V;
    C += clusters_bound(rs[g]->n, M);
  }
  const int64_t n = eoff[G];
  p.num_vertices = voff[G];
  size_t at = 0;
  int32_t *bsrc = (int32_t *)(work + at);
  at += align_up(4 * (size_t)n);
  int32_t *bdst = (int32_t *)(work + at);
  at += align_up(4 * (size_t)n);
  int64_t *bt = (int64_t *)(work + at);
  at += align_up(8 * (size_t)n);
  GatherDesc *gd = (GatherDesc *)(work + at);
  at += align_up(sizeof(GatherDesc) * G);
  ScatterDesc *sd = (ScatterDesc *)(work + at);
  at += align_up(sizeof(ScatterDesc) * G);
  const OutLayout L = out_layout(n, C);
  const ce_result bout = out_pointers(work + at, L);
  at += L.bytes;
  void *ws = work + at;
  const size_t ws_bytes = ce_batch_workspace_bytes(eoff.data(), voff.data(), G, &p);

  std::vector<GatherDesc> hg(G);
  int64_t maxn = 1;
  for (int64_t g = 0; g < G; g++) {
    Request *r = rs[g];
    hg[g] = GatherDesc{(const int32_t *)input(r, 0), (const int32_t *)input(r, 1), (const int64_t *)input(r, 2),
                       r->n, eoff[g]};
    if (r->n > maxn) maxn = r->n;
  }
  auto fail_all = [&](ce_status st, const char *msg) {
    for (Request *r : rs) { r->status = st; r->err = msg; }
  };
  if (hipMemcpyAsync(gd, hg.data(), sizeof(GatherDesc) * G, hipMemcpyHostToDevice, s) != hipSuccess) {
    fail_all(CE_EDEVICE, "descriptor upload failed");
    return;
  }
  const unsigned gx = (unsigned)((maxn + B - 1) / B < 1024 ? (maxn + B - 1) / B : 1024);
  hipLaunchKernelGGL(k_gather, dim3(gx, (unsigned)G), dim3(B), 0, s, gd, bsrc, bdst, bt);
  if (hipGetLastError() != hipSuccess) {
    fail_all(CE_EDEVICE, "gather launch failed");
    return;
  }
  std::vector<ce_counts> counts(G);
  std::vector<int64_t> roff(G + 1), coff(G + 1);
  ce_status st = ce_cluster_batch(bsrc, bdst, bt, eoff.data(), voff.data(), G, &p, &bout, counts.data(), roff.data(),
                                  coff.data(), ws, ws_bytes, s);
  if (st == CE_ESELFLOOP || st == CE_ERANGE) {
    // a data error fails the whole batch: run each request alone to find whose it is
    for (Request *r : rs) solo(r);
    return;
  }
  if (st != CE_OK) {
    fail_all(st, ce_last_error());
    return;
  }
  std::vector<ScatterDesc> hs(G);
  int64_t top = 1;
  for (int64_t g = 0; g < G; g++) {
    hs[g] = ScatterDesc{roff[g], roff[g + 1] - roff[g], eoff[g], rs[g]->n, coff[g], coff[g + 1] - coff[g], rs[g]->out};
    rs[g]->counts = counts[g];
    rs[g]->status = CE_OK;
    int64_t x = hs[g].m > hs[g].n ? hs[g].m : hs[g].n;
    if (hs[g].nc > x) x = hs[g].nc;
    if (x > top) top = x;
  }
  if (hipMemcpyAsync(sd, hs.data(), sizeof(ScatterDesc) * G, hipMemcpyHostToDevice, s) != hipSuccess) {
    fail_all(CE_EDEVICE, "descriptor upload failed");
    return;
  }
  const unsigned sx = (unsigned)((top + B - 1) / B < 1024 ? (top + B - 1) / B : 1024);
  hipLaunchKernelGGL(k_scatter, dim3(sx, (unsigned)G), dim3(B), 0, s, sd, bout);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) fail_all(CE_EDEVICE, "scatter failed");
}

void ce_server::worker(int k) {
  (void)hipSetDevice(device);
  hipStream_t s = streams[k];
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&] { return stop || !queue.empty(); });
    if (stop && queue.empty()) return;
    // the oldest request fixes M, the mode and the cutoff; take later
    // requests with the same ones while they fit
    const Request *head = queue.front();
    const int64_t M = head->M;
    std::vector<Request *> pick;
    int64_t recs = 0;
    for (Request *r : queue) {
      if (r->M != M || r->mode != head->mode || r->max_dt != head->max_dt || r->thr != head->thr) continue;
      if (!pick.empty() && (recs + r->n > max_batch_records || (int64_t)pick.size() >= MAX_BATCH_GRAPHS)) break;
      pick.push_back(r);
      recs += r->n;
    }
    size_t off = 0, bytes = 0;
    bool got = false;
    while (!pick.empty()) {
      bytes = batch_bytes(pick, M);
      if (work_arena.alloc(bytes, &off)) { got = true; break; }
      pick.pop_back();
    }
    if (!got) {
      if (running == 0) {
        // nothing else holds work memory, so the oldest request can never run
        Request *r = queue.front();
        queue.pop_front();
        r->status = CE_ENOMEM;
        r->err = "request does not fit the server's work memory";
        r->done = true;
        r->t_done = Clock::now();
        r->t_start = r->t_done;
        in_arena.release(r->in_off, r->in_bytes);
        st.requests_done++;
        cv_done.notify_all();
        continue;
      }
      cv_work.wait(lk);  // woken when a batch finishes and frees memory
      continue;
    }
    for (Request *r : pick) {
      for (auto it = queue.begin(); it != queue.end(); ++it)
        if (*it == r) { queue.erase(it); break; }
    }
    running++;
    st.batches++;
    st.requests_batched += (int64_t)pick.size();
    if ((int64_t)pick.size() > st.max_batch_requests) st.max_batch_requests = (int64_t)pick.size();
    if (running > st.max_concurrent_batches) st.max_concurrent_batches = running;
    if ((int64_t)work_arena.used() > st.work_peak_bytes) st.work_peak_bytes = (int64_t)work_arena.used();
    const auto t0 = Clock::now();
    for (Request *r : pick) r->t_start = t0;
    lk.unlock();
    run_batch(pick, off, s);
    const auto t1 = Clock::now();
    lk.lock();
    work_arena.release(off, bytes);
    running--;
    for (Request *r : pick) {
      in_arena.release(r->in_off, r->in_bytes);
      r->done = true;
      r->t_done = t1;
    }
    st.requests_done += (int64_t)pick.size();
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

extern "C" {

ce_status ce_server_create(const ce_server_config *cfg, ce_server **out) {
  if (!cfg || !out) { set_error("config/out is NULL"); return CE_EINVAL; }
  *out = nullptr;
  if (cfg->struct_size < sizeof(ce_server_config)) { set_error("config.struct_size too small"); return CE_EINVAL; }
  if (cfg->workers < 1 || cfg->workers > 16) { set_error("workers must be in [1, 16]"); return CE_EINVAL; }
  if (cfg->hbm_budget_bytes < (1u << 20)) { set_error("hbm_budget_bytes must be >= 1 MiB"); return CE_EINVAL; }
  if (cfg->max_inflight < 1) { set_error("max_inflight must be >= 1"); return CE_EINVAL; }
  if (cfg->input_fraction_pct < 1 || cfg->input_fraction_pct > 90) {
    set_error("input_fraction_pct must be in [1, 90]");
    return CE_EINVAL;
  }
  std::unique_ptr<ce_server> srv(new ce_server);
  srv->device = cfg->device;
  CE_HIP(hipSetDevice(cfg->device));
  const size_t budget = cfg->hbm_budget_bytes & ~(ALIGN - 1);
  srv->in_cap = (budget / 100 * cfg->input_fraction_pct) & ~(ALIGN - 1);
  if (hipMalloc((void **)&srv->mem, budget) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of the server budget failed");
    return CE_ENOMEM;
  }
  srv->in_arena.init(srv->in_cap);
  srv->work_arena.init(budget - srv->in_cap);
  srv->max_inflight = cfg->max_inflight;
  srv->max_batch_records = cfg->max_batch_records > 0 ? cfg->max_batch_records : (int64_t(1) << 26);
  if (hipStreamCreateWithFlags(&srv->copy_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(srv->mem);
    set_error("stream creation failed");
    return CE_EDEVICE;
  }
  for (uint32_t k = 0; k < cfg->workers; k++) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : srv->streams) (void)hipStreamDestroy(x);
      (void)hipStreamDestroy(srv->copy_stream);
      (void)hipFree(srv->mem);
      set_error("stream creation failed");
      return CE_EDEVICE;
    }
    srv->streams.push_back(s);
  }
  for (uint32_t k = 0; k < cfg->workers; k++) srv->workers.emplace_back(&ce_server::worker, srv.get(), (int)k);
  *out = srv.release();
  return CE_OK;
}

ce_status ce_server_destroy(ce_server *srv) {
  if (!srv) return CE_OK;
  {
    std::lock_guard<std::mutex> l(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto &t : srv->workers) t.join();
  (void)hipSetDevice(srv->device);
  for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
  (void)hipStreamDestroy(srv->copy_stream);
  (void)hipFree(srv->mem);
  delete srv;
  return CE_OK;
}

size_t ce_server_request_bytes(int64_t n, const ce_params *params) {
  if (!params || n < 0 || n > 0x7fffffffLL || params->min_cluster_size < 2 || params->num_vertices < 1) return 0;
  Request r;
  r.n = n;
  r.V = params->num_vertices;
  r.M = params->min_cluster_size;
  if (params->struct_size >= sizeof(ce_params) && params->num_thresholds > 0 && params->thresholds)
    r.thr.assign(params->thresholds, params->thresholds + params->num_thresholds);
  std::vector<Request *> one{&r};
  return batch_bytes(one, r.M) + align_up(4 * (size_t)n) * 2 + align_up(8 * (size_t)n);
}

ce_status ce_server_submit(ce_server *srv, const ce_request *req, uint64_t *ticket) {
  if (!srv || !req || !ticket) { set_error("server/request/ticket is NULL"); return CE_EINVAL; }
  if (req->struct_size < sizeof(ce_request)) { set_error("request.struct_size too small"); return CE_EINVAL; }
  const ce_params &p = req->params;
  if (p.struct_size < CE_PARAMS_V1_SIZE || (p.mode != CE_MODE_UNDIRECTED && p.mode != CE_MODE_CAUSAL) || p.flags ||
      p.reserved ||
      p.min_cluster_size < 2 || p.num_vertices < 1 || p.num_vertices > 0x80000000LL) {
    set_error("invalid request params");
    return CE_EINVAL;
  }
  const int64_t n = req->n;
  if (n < 0 || n > 0x7fffffffLL) { set_error("n must be in [0, 2^31-1]"); return CE_EINVAL; }
  if (n > 0 && (!req->src || !req->dst || !req->t)) { set_error("input pointer is NULL"); return CE_EINVAL; }
  const auto t_submit = Clock::now();
  auto r = std::make_unique<Request>();
  r->n = n;
  r->V = p.num_vertices;
  r->M = p.min_cluster_size;
  r->mode = p.mode;
  r->max_dt = p.struct_size >= CE_PARAMS_V2_SIZE ? p.max_dt : -1;
  if (p.struct_size >= sizeof(ce_params) && p.num_thresholds != 0) {
    if (p.num_thresholds < 0 || p.num_thresholds > CE_MAX_THRESHOLDS || !p.thresholds) {
      set_error("num_thresholds must be in [0, 64] with a thresholds array");
      return CE_EINVAL;
    }
    r->thr.assign(p.thresholds, p.thresholds + p.num_thresholds);
    for (size_t i = 0; i < r->thr.size(); i++)
      if (r->thr[i] < 0 || (i > 0 && r->thr[i] <= r->thr[i - 1])) {
        set_error("thresholds must be >= 0 and strictly increasing");
        return CE_EINVAL;
      }
  }
  r->out = req->out;
  r->t_submit = t_submit;
  r->in_bytes = 2 * align_up(4 * (size_t)n) + align_up(8 * (size_t)n);
  {
    std::vector<Request *> one{r.get()};
    if (batch_bytes(one, r->M) > srv->work_arena.cap() || r->in_bytes > srv->in_cap) {
      set_error("request needs more device memory than the server budget");
      return CE_ENOMEM;
    }
  }
  {
    std::lock_guard<std::mutex> l(srv->mu);
    if (srv->inflight >= srv->max_inflight) { set_error("too many requests in flight"); return CE_EBUSY; }
    if (!srv->in_arena.alloc(r->in_bytes, &r->in_off)) { set_error("input memory is full"); return CE_EBUSY; }
    srv->inflight++;
    if ((int64_t)srv->in_arena.used() > srv->st.input_peak_bytes) srv->st.input_peak_bytes = (int64_t)srv->in_arena.used();
  }
  // the records become resident in the server's input memory before submit returns
  char *in = srv->mem + r->in_off;
  hipError_t e = hipSuccess;
  if (n > 0) {
    e = hipMemcpyAsync(in, req->src, 4 * (size_t)n, hipMemcpyHostToDevice, srv->copy_stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(in + align_up(4 * (size_t)n), req->dst, 4 * (size_t)n, hipMemcpyHostToDevice,
                         srv->copy_stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(in + 2 * align_up(4 * (size_t)n), req->t, 8 * (size_t)n, hipMemcpyHostToDevice,
                         srv->copy_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(srv->copy_stream);
  }
  std::lock_guard<std::mutex> l(srv->mu);
  if (e != hipSuccess) {
    srv->in_arena.release(r->in_off, r->in_bytes);
    srv->inflight--;
    set_error(std::string("input copy failed: ") + hipGetErrorString(e));
    return CE_EDEVICE;
  }
  r->ticket = srv->next_ticket++;
  *ticket = r->ticket;
  srv->queue.push_back(r.get());
  srv->reqs.emplace(r->ticket, std::move(r));
  srv->st.requests_submitted++;
  srv->cv_work.notify_one();
  return CE_OK;
}

ce_status ce_server_poll(ce_server *srv, uint64_t ticket, int wait, ce_request_status *status) {
  if (!srv || !status) { set_error("server/status is NULL"); return CE_EINVAL; }
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) { set_error("unknown ticket"); return CE_EINVAL; }
  Request *r = it->second.get();
  if (!r->done) {
    if (!wait) return CE_EBUSY;
    srv->cv_done.wait(lk, [&] { return r->done; });
  }
  status->status = r->status;
  status->counts = r->counts;
  status->queue_s = std::chrono::duration<double>(r->t_start - r->t_submit).count();
  status->latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  set_error(r->status == CE_OK ? "no error" : r->err);
  srv->reqs.erase(it);
  srv->inflight--;
  return CE_OK;
}

ce_status ce_server_get_stats(ce_server *srv, ce_server_stats *out) {
  if (!srv || !out) { set_error("server/out is NULL"); return CE_EINVAL; }
  std::lock_guard<std::mutex> l(srv->mu);
  *out = srv->st;
  out->input_capacity_bytes = (int64_t)srv->in_arena.cap();
  out->work_capacity_bytes = (int64_t)srv->work_arena.cap();
  return CE_OK;
}

}  // extern "C"
