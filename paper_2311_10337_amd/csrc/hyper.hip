// Stages A1-A4 for dynamic hypergraphs (Sec. 5.3, undirected): record r is a
// hyperedge, the vertex set members[offsets[r] .. offsets[r+1]) at time t[r].
// Two hyperedges are adjacent when their sets meet, with weight |t_r - t_s|.
// The node-local MST of a vertex is the path through its incident hyperedges
// in time order, so the skeleton has sum_i (d_i - 1) <= nnz edges.
//
// 1. Hyperedges are sorted by (t, id) once (ranks).
// 2. The nnz membership entries are laid out in rank order (a prefix sum of
//    the degrees by rank; each entry finds its hyperedge by binary search) and
//    stably radix-sorted by vertex, so every vertex's list is in rank order.
// 3. Each entry whose predecessor in the list is another hyperedge of the same
//    vertex emits the row (predecessor, this). A vertex listed twice in one
//    hyperedge gives two equal neighbouring entries, which emit nothing. A
//    pair consecutive at several vertices is emitted once per vertex with the
//    same key; Boruvka keeps one copy.
//
// Key: the canonical order (w, head id, 2^32-1-tail id). Rows of one head with
// equal w have tails of equal time, and among records of equal time the rank
// order is the id order, so the tail term is replaced by the tail's distance
// to the end of its run of equal times: key = w << (idbits+jbits) |
// head id << jbits | (run end - 1 - tail rank), jbits = bits(longest run - 1).
// Duplicate rows get equal keys.
#include "ce_internal.h"

namespace ce {

namespace {

constexpr int B = 256;

__device__ inline uint64_t t_to_ord(int64_t t) { return (uint64_t)t ^ (uint64_t(1) << 63); }

// hdr[0] |= 2 member out of range, 4 bad offsets; hdr[1] = min t, hdr[2] = max t (ordered)
__global__ __launch_bounds__(B) void k_hvalidate(const int32_t *members, const int64_t *off, const int64_t *t,
                                                 int64_t n, int64_t nnz, int64_t V, uint64_t *hdr) {
  __shared__ uint64_t smin[B / 64], smax[B / 64];
  __shared__ uint32_t sflag;
  if (threadIdx.x == 0) sflag = 0;
  __syncthreads();
  uint64_t mn = NONE64, mx = 0;
  uint32_t flag = 0;
  const int64_t N = n > nnz ? n : nnz;
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < N; i += (int64_t)gridDim.x * B) {
    if (i < n) {
      if (off[i + 1] < off[i]) flag |= 4u;
      const uint64_t o = t_to_ord(t[i]);
      mn = o < mn ? o : mn;
      mx = o > mx ? o : mx;
    }
    if (i < nnz) {
      const int32_t v = members[i];
      if (v < 0 || (int64_t)v >= V) flag |= 2u;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (off[0] != 0 || off[n] != nnz)) flag |= 4u;
  for (int d = 32; d >= 1; d >>= 1) {
    uint64_t a = __shfl_xor(mn, d, 64), b = __shfl_xor(mx, d, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if (flag) atomicOr(&sflag, flag);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) { smin[w] = mn; smax[w] = mx; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < B / 64; q++) {
      mn = smin[q] < mn ? smin[q] : mn;
      mx = smax[q] > mx ? smax[q] : mx;
    }
    if (sflag) atomicOr((unsigned long long *)&hdr[0], (unsigned long long)sflag);
    atomicMin((unsigned long long *)&hdr[1], (unsigned long long)mn);
    atomicMax((unsigned long long *)&hdr[2], (unsigned long long)mx);
  }
}

__global__ void k_hinit_hdr(uint64_t *hdr) {
  for (int i = threadIdx.x; i < kHdrWords; i += blockDim.x) hdr[i] = i == H_TMIN ? NONE64 : 0;
}
__global__ void k_hzero(uint64_t *p) {
  if (threadIdx.x == 0) *p = 0;
}
__global__ __launch_bounds__(B) void k_hfill_best(uint64_t *best, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) best[i] = NONE64;
}

__global__ __launch_bounds__(B) void k_htkeys(const int64_t *t, int64_t n, const uint64_t *hdr, uint64_t *keys) {
  const int64_t tmin = (int64_t)(hdr[H_TMIN] ^ (uint64_t(1) << 63));
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B)
    keys[i] = (uint64_t)(t[i] - tmin);
}

// degree of every hyperedge by rank; the graph of every rank (one graph)
__global__ __launch_bounds__(B) void k_hdeg(const uint32_t *perm, const int64_t *off, int64_t n, uint32_t *deg,
                                            uint32_t *grank) {
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < n; r += (int64_t)gridDim.x * B) {
    const uint32_t id = perm[r];
    deg[r] = (uint32_t)(off[id + 1] - off[id]);
    grank[r] = 0u;
  }
}

// entry k of the rank-ordered membership list: its hyperedge rank r is the
// last one with roff[r] <= k (empty hyperedges share their start with the
// next one, so the last such r holds k); key = vertex, value = rank
__global__ __launch_bounds__(B) void k_hentries(const uint32_t *roff, const uint32_t *perm, const int64_t *off,
                                                const int32_t *members, int64_t n, int64_t nnz, uint32_t *ikey,
                                                uint32_t *ival) {
  for (int64_t k = (int64_t)blockIdx.x * B + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * B) {
    int64_t lo = 0, hi = n - 1;  // roff[0] = 0 <= k
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if ((int64_t)roff[mid] <= k) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t r = (uint32_t)lo;
    ikey[k] = (uint32_t)members[off[perm[r]] + (k - (int64_t)roff[r])];
    ival[k] = r;
  }
}

__device__ inline bool is_row(const uint32_t *sk, const uint32_t *sv, int64_t k) {
  return k > 0 && sk[k] == sk[k - 1] && sv[k] != sv[k - 1];
}

__global__ __launch_bounds__(B) void k_hrow_flags(const uint32_t *sk, const uint32_t *sv, int64_t nnz,
                                                  uint32_t *flag) {
  for (int64_t k = (int64_t)blockIdx.x * B + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * B)
    flag[k] = is_row(sk, sv, k) ? 1u : 0u;
}

// first rank of every run of equal times
__global__ __launch_bounds__(B) void k_hrun_flags(const uint64_t *ts, int64_t n, uint32_t *f) {
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < n; r += (int64_t)gridDim.x * B)
    f[r] = (r == 0 || ts[r] != ts[r - 1]) ? 1u : 0u;
}
// start[q] = first rank of run q, start[#runs] = n; the longest run - 1
__global__ __launch_bounds__(B) void k_hrun_starts(const uint32_t *f, const uint32_t *fx, int64_t n,
                                                   uint32_t *start) {
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < n; r += (int64_t)gridDim.x * B)
    if (f[r]) start[fx[r]] = (uint32_t)r;
  if (blockIdx.x == 0 && threadIdx.x == 0) start[fx[n]] = (uint32_t)n;
}
__global__ __launch_bounds__(B) void k_hrun_max(const uint32_t *start, const uint32_t *fx, int64_t n,
                                                unsigned int *maxtie) {
  const int64_t runs = fx[n];
  uint32_t mx = 0;
  for (int64_t q = (int64_t)blockIdx.x * B + threadIdx.x; q < runs; q += (int64_t)gridDim.x * B) {
    const uint32_t len = start[q + 1] - start[q];
    if (len - 1 > mx) mx = len - 1;
  }
  mx = wave_max_u32(mx);
  if (wave_lane() == 0 && mx) atomicMax(maxtie, mx);
}

__global__ __launch_bounds__(B) void k_hemit(const uint32_t *sk, const uint32_t *sv, const uint32_t *pos,
                                             int64_t nnz, const uint64_t *ts, const uint32_t *perm, const uint32_t *f,
                                             const uint32_t *fx, const uint32_t *start, int wshift, int hshift,
                                             uint64_t *skel_key, uint32_t *skel_tail, uint32_t *skel_head,
                                             uint64_t *best, uint64_t *wraw) {
  for (int64_t k = (int64_t)blockIdx.x * B + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * B) {
    if (pos[k + 1] == pos[k]) continue;
    const uint32_t tl = sv[k - 1], hd = sv[k], e = pos[k];
    const uint32_t tie = start[fx[tl] + f[tl]] - 1u - tl;
    skel_tail[e] = tl;
    skel_head[e] = hd;
    if (wraw) {  // weight ranks: the weight waits in wraw, the offers wait for the ranks
      skel_key[e] = ((uint64_t)perm[hd] << hshift) | (uint64_t)tie;
      wraw[e] = ts[hd] - ts[tl];
      continue;
    }
    const uint64_t key = ((ts[hd] - ts[tl]) << wshift) | ((uint64_t)perm[hd] << hshift) | (uint64_t)tie;
    skel_key[e] = key;
    // each row offers its key to both hyperedges' first Boruvka minimum
    atomicMin((unsigned long long *)&best[tl], (unsigned long long)key);
    atomicMin((unsigned long long *)&best[hd], (unsigned long long)key);
  }
}

__global__ void k_hput_u64(uint64_t *p, uint64_t v) { *p = v; }

}  // namespace

ce_status stage_hyper_validate(const int32_t *members, const int64_t *offsets, const int64_t *t, int64_t nnz,
                               Bufs &b, hipStream_t s) {
  CE_LAUNCH(k_hinit_hdr, dim3(1), dim3(64), 0, s, b.hdr);
  CE_LAUNCH(k_hvalidate, dim3(grid_for(b.n > nnz ? b.n : nnz, B, 4096)), dim3(B), 0, s, members, offsets, t, b.n,
            nnz, b.V, b.hdr);
  CE_HIP(hipGetLastError());
  return CE_OK;
}

size_t stage_hyper_skeleton_scratch(int64_t n, int64_t nnz) {
  Ws w;
  w.alloc<uint64_t>(nnz);  // raw weights, when the weights are ranked
  const size_t r0 = w.off;
  for (int k = 0; k < 4; k++) w.alloc<uint32_t>(nnz);  // ikey, ival and their ping-pong copies
  // phase 1: the time sort, then degrees and their prefix sum
  Ws a;
  a.alloc<uint64_t>(n);
  a.alloc<uint32_t>(n);
  const size_t p1a = a.off + radix_ws_bytes(n);
  Ws a2;
  a2.alloc<uint32_t>(n + 1);
  a2.alloc<uint32_t>(n + 1);
  const size_t p1b = a2.off + scan_ws_bytes(n + 1);
  // phase 2: the vertex sort; phase 3: row positions and runs of equal times
  const size_t p2 = radix_ws_bytes(nnz);
  Ws c;
  c.alloc<uint32_t>(nnz + 1);
  for (int k = 0; k < 3; k++) c.alloc<uint32_t>(n + 1);
  const size_t p3 = c.off + (scan_ws_bytes(nnz + 1) > scan_ws_bytes(n + 1) ? scan_ws_bytes(nnz + 1)
                                                                           : scan_ws_bytes(n + 1));
  size_t x = p1a > p1b ? p1a : p1b;
  if (p2 > x) x = p2;
  if (p3 > x) x = p3;
  x += w.off;
  const size_t rk = r0 + stage_rank_weights_scratch(nnz);
  return (x > rk ? x : rk) + 4096;
}

ce_status stage_hyper_skeleton(const int32_t *members, const int64_t *offsets, const int64_t *t, int64_t nnz,
                               Bufs &b, Ws &ws, hipStream_t s) {
  const int64_t n = b.n;
  size_t m0 = ws.mark();
  uint64_t *wraw = ws.alloc<uint64_t>(nnz);  // raw weights, when the weights are ranked
  const size_t mr = ws.mark();
  uint32_t *ikey = ws.alloc<uint32_t>(nnz);
  uint32_t *ival = ws.alloc<uint32_t>(nnz);
  uint32_t *ikey_alt = ws.alloc<uint32_t>(nnz);
  uint32_t *ival_alt = ws.alloc<uint32_t>(nnz);
  CE_WS_CHECK(ws);
  // 1. hyperedges by (t, id): ranks
  {
    size_t m1 = ws.mark();
    uint64_t *tkey_alt = ws.alloc<uint64_t>(n);
    uint32_t *pv_alt = ws.alloc<uint32_t>(n);
    CE_WS_CHECK(ws);
    CE_LAUNCH(k_htkeys, dim3(grid_for(n, B)), dim3(B), 0, s, t, n, b.hdr, b.ts);
    CE_HIP(hipGetLastError());
    bool alt = false;
    CE_TRY((radix_sort_pairs<uint64_t, uint32_t>(b.ts, b.perm, tkey_alt, pv_alt, n, 0, b.tbits, true, &alt, ws, s)));
    if (alt) {
      CE_HIP(hipMemcpyAsync(b.ts, tkey_alt, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
      CE_HIP(hipMemcpyAsync(b.perm, pv_alt, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    }
    ws.release(m1);
  }
  // 2. membership entries in rank order, then stably by vertex
  {
    size_t m1 = ws.mark();
    uint32_t *deg = ws.alloc<uint32_t>(n + 1), *roff = ws.alloc<uint32_t>(n + 1);
    CE_WS_CHECK(ws);
    CE_LAUNCH(k_hdeg, dim3(grid_for(n, B)), dim3(B), 0, s, b.perm, offsets, n, deg, b.grank);
    CE_HIP(hipGetLastError());
    CE_TRY(scan_exclusive_u32(deg, roff, n, ws, s));
    if (nnz > 0)
      CE_LAUNCH(k_hentries, dim3(grid_for(nnz, B)), dim3(B), 0, s, roff, b.perm, offsets, members, n, nnz, ikey,
                ival);
    CE_HIP(hipGetLastError());
    ws.release(m1);
  }
  bool alt = false;
  CE_TRY((radix_sort_pairs<uint32_t, uint32_t>(ikey, ival, ikey_alt, ival_alt, nnz, 0, b.vbits, false, &alt, ws, s)));
  const uint32_t *sk = alt ? ikey_alt : ikey;
  const uint32_t *sv = alt ? ival_alt : ival;
  // 3. row positions, runs of equal times (the key's tail term), rows
  uint32_t *pos = ws.alloc<uint32_t>(nnz + 1);
  uint32_t *f = ws.alloc<uint32_t>(n + 1), *fx = ws.alloc<uint32_t>(n + 1), *start = ws.alloc<uint32_t>(n + 1);
  CE_WS_CHECK(ws);
  CE_LAUNCH(k_hrow_flags, dim3(grid_for(nnz, B)), dim3(B), 0, s, sk, sv, nnz, pos);
  CE_HIP(hipGetLastError());
  CE_TRY(scan_exclusive_u32(pos, pos, nnz, ws, s));
  CE_LAUNCH(k_hrun_flags, dim3(grid_for(n, B)), dim3(B), 0, s, b.ts, n, f);
  CE_HIP(hipGetLastError());
  CE_TRY(scan_exclusive_u32(f, fx, n, ws, s));
  CE_LAUNCH(k_hzero, dim3(1), dim3(64), 0, s, &b.hdr[7]);
  CE_LAUNCH(k_hrun_starts, dim3(grid_for(n, B)), dim3(B), 0, s, f, fx, n, start);
  CE_LAUNCH(k_hrun_max, dim3(grid_for(n, B)), dim3(B), 0, s, start, fx, n, (unsigned int *)&b.hdr[7]);
  CE_HIP(hipGetLastError());
  uint64_t h[2];
  {
    uint32_t *pin = (uint32_t *)pinned_scratch();
    CE_HIP(hipMemcpyAsync(pin + 16, pos + nnz, 4, hipMemcpyDeviceToHost, s));
    CE_TRY(read_u64(&b.hdr[7], h, 1, s));  // synchronises the stream
    h[1] = pin[16];
  }
  const uint32_t maxtie = (uint32_t)h[0];
  const int64_t S = (int64_t)h[1];
  if (S > nnz) {
    set_error("internal: hypergraph skeleton larger than its input");
    return CE_EDEVICE;
  }
  b.S = S;
  b.jbits = bits_for(maxtie);
  b.hshift = b.jbits;
  b.wshift = b.idbits + b.jbits;
  if (!choose_key_layout(b, S)) {  // the all-ones word marks an absent edge
    set_error("too many hyperedges for the hypergraph key: bits(rows - 1) + bits(n-1) + bits(longest run of "
              "equal times - 1) > 63");
    return CE_ERANGE;
  }
  CE_LAUNCH(k_hfill_best, dim3(grid_for(n, B)), dim3(B), 0, s, b.best, n);
  if (nnz > 0)
    CE_LAUNCH(k_hemit, dim3(grid_for(nnz, B)), dim3(B), 0, s, sk, sv, pos, nnz, b.ts, b.perm, f, fx, start,
              b.wshift, b.hshift, b.skel_key, b.skel_tail, b.skel_tid, b.best, b.rank ? wraw : nullptr);
  CE_LAUNCH(k_hput_u64, dim3(1), dim3(1), 0, s, &b.hdr[H_C7], (uint64_t)S);  // the rows, for Boruvka's first round
  CE_HIP(hipGetLastError());
  ws.release(mr);
  if (b.rank) CE_TRY(stage_rank_weights(b, wraw, S, ws, s));
  ws.release(m0);
  return CE_OK;
}

}  // namespace ce
