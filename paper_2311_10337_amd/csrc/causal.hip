// Stages A2-A4 in CAUSAL mode: the increment-weighted line graph of Def. 1
// (an arc joins record r to record s when r arrives at the vertex s leaves,
// t_r <= t_s, weight t_s - t_r) and its skeleton by Alg. 2 at every vertex,
// united as in Alg. 3. The line graph is never formed.
//
// 1. Records are sorted by (t, id) once (ranks), as in undirected mode.
// 2. Every record has an in-entry at its head vertex and an out-entry at its
//    tail vertex. Entries are placed in (t, in before out, id) order without
//    a sort: inside a block of records with equal times, all in-entries come
//    first. A stable sort by vertex then yields every vertex's list in the
//    order Alg. 2 walks it.
// 3. Alg. 2's window at an out-entry s holds the in-entries since the previous
//    out-entry of the vertex, plus the last in-entry before that one (the
//    window is cut to its last element after each out-entry, and an empty
//    window stays empty). So the window is one contiguous run of the vertex's
//    in-entries, found with prefix counts; no sequential walk is needed.
// 4. Rows are written per out-entry at offsets from a prefix sum of window
//    sizes; windows longer than a wave are spread over a whole workgroup.
//
// Key: the canonical order (w, head id, 2^32-1-tail id). For one head, the
// rows with equal w have tails of equal time at the same vertex, so the tail
// term only has to order in-entries of equal time at one vertex: their tie
// index (how many equal-time in-entries with a larger id the vertex has)
// takes its place. key = w << (idbits+jbits) | head id << jbits | tie, with
// jbits = bits(largest tie index).
#include "ce_internal.h"

namespace ce {

namespace {

constexpr int B = 256;
constexpr uint32_t BIG_WINDOW = 64;

// first rank of every run of equal times
__global__ __launch_bounds__(B) void k_run_flags(const uint64_t *ts, int64_t n, uint32_t *f) {
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < n; r += (int64_t)gridDim.x * B)
    f[r] = (r == 0 || ts[r] != ts[r - 1]) ? 1u : 0u;
}
__global__ __launch_bounds__(B) void k_run_starts(const uint32_t *f, const uint32_t *fx, int64_t n, uint32_t *start) {
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < n; r += (int64_t)gridDim.x * B)
    if (f[r]) start[fx[r]] = (uint32_t)r;
  if (blockIdx.x == 0 && threadIdx.x == 0) start[fx[n]] = (uint32_t)n;
}

// entries at positions in (t, in before out, rank) order; value 2r + side,
// side 1 = in-entry (at the head vertex), 0 = out-entry (at the tail vertex)
__global__ __launch_bounds__(B) void k_causal_entries(const uint4 *vals, const uint32_t *f, const uint32_t *fx,
                                                      const uint32_t *start, int64_t n, uint32_t *perm,
                                                      uint32_t *grank, uint32_t *ikey, uint32_t *ival) {
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < n; r += (int64_t)gridDim.x * B) {
    const uint4 v = vals[r];
    perm[r] = v.x;
    grank[r] = v.w;
    const uint32_t run = fx[r] + f[r] - 1;
    const int64_t g0 = start[run], g1 = start[run + 1];
    const int64_t pin = 2 * g0 + (r - g0), pout = 2 * g0 + (g1 - g0) + (r - g0);
    ikey[pin] = v.z;
    ival[pin] = 2u * (uint32_t)r + 1u;
    ikey[pout] = v.y;
    ival[pout] = 2u * (uint32_t)r;
  }
}

__global__ __launch_bounds__(B) void k_in_flags(const uint32_t *sv, int64_t n2, uint32_t *isin) {
  for (int64_t k = (int64_t)blockIdx.x * B + threadIdx.x; k < n2; k += (int64_t)gridDim.x * B) isin[k] = sv[k] & 1u;
}

// positions of the q-th in-entry and of the q-th out-entry (n of each)
__global__ __launch_bounds__(B) void k_side_pos(const uint32_t *sv, const uint32_t *incount, int64_t n2,
                                                uint32_t *inpos, uint32_t *outpos) {
  for (int64_t k = (int64_t)blockIdx.x * B + threadIdx.x; k < n2; k += (int64_t)gridDim.x * B) {
    if (sv[k] & 1u) inpos[incount[k]] = (uint32_t)k;
    else outpos[k - incount[k]] = (uint32_t)k;
  }
}

// runs of in-entries with equal vertex and equal time, in in-entry order
__global__ __launch_bounds__(B) void k_tie_flags(const uint32_t *inpos, const uint32_t *sk, const uint32_t *sv,
                                                 const uint64_t *ts, int64_t n, uint32_t *gf) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) {
    uint32_t f = 1u;
    if (i > 0) {
      const uint32_t p = inpos[i], q = inpos[i - 1];
      f = (sk[p] != sk[q] || ts[sv[p] >> 1] != ts[sv[q] >> 1]) ? 1u : 0u;
    }
    gf[i] = f;
  }
}

// tie index of every in-entry: equal-time in-entries of its vertex after it
__global__ __launch_bounds__(B) void k_ties(const uint32_t *gf, const uint32_t *gx, const uint32_t *gstart, int64_t n,
                                            uint32_t *tie, unsigned int *maxtie) {
  uint32_t mx = 0;
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) {
    const uint32_t g = gx[i] + gf[i] - 1;
    const uint32_t tv = gstart[g + 1] - 1u - (uint32_t)i;
    tie[i] = tv;
    if (tv > mx) mx = tv;
  }
  mx = wave_max_u32(mx);
  if (wave_lane() == 0 && mx) atomicMax(maxtie, mx);
}

// Alg. 2 window of every out-entry as a run [a, a + cnt) of in-entry indices
__global__ __launch_bounds__(B) void k_windows(const uint32_t *sk, const uint32_t *incount, const uint32_t *inpos,
                                               const uint32_t *outpos, int64_t n, uint32_t *wa, uint32_t *wcnt) {
  for (int64_t q = (int64_t)blockIdx.x * B + threadIdx.x; q < n; q += (int64_t)gridDim.x * B) {
    const uint32_t k = outpos[q], v = sk[k];
    uint32_t a;
    const uint32_t prev = q > 0 ? outpos[q - 1] : NONE32;
    if (prev != NONE32 && sk[prev] == v) {
      // not the vertex's first out-entry: the in-entries after it, plus the
      // carried last in-entry before it if the vertex has one
      const uint32_t c = incount[prev];
      a = (c > 0 && sk[inpos[c - 1]] == v) ? c - 1 : c;
    } else {
      // the first out-entry: everything of the vertex before it is an in-entry;
      // find where the vertex's list starts (sk is sorted)
      uint32_t lo = prev != NONE32 ? prev + 1 : 0u, hi = k;
      while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (sk[mid] < v) lo = mid + 1;
        else hi = mid;
      }
      a = incount[lo];
    }
    wa[q] = a;
    wcnt[q] = incount[k] - a;
  }
}

// writes row e and offers its key to the tail's first Boruvka minimum; returns the key
// (weight ranks, wraw set: the key without its weight field, the weight to
// wraw, and no offer until the ranks are known)
__device__ inline uint64_t emit_row(int64_t e, uint32_t ii, uint32_t s, uint64_t hid, uint64_t th,
                                    const uint32_t *inpos, const uint32_t *sv, const uint64_t *ts,
                                    const uint32_t *tie, int wshift, int hshift, uint64_t *skel_key,
                                    uint32_t *skel_tail, uint32_t *skel_head, uint64_t *best, uint64_t *wraw) {
  const uint32_t r = sv[inpos[ii]] >> 1;
  skel_tail[e] = r;
  skel_head[e] = s;
  if (wraw) {
    skel_key[e] = (hid << hshift) | (uint64_t)tie[ii];
    wraw[e] = th - ts[r];
    return NONE64;
  }
  const uint64_t k = ((th - ts[r]) << wshift) | (hid << hshift) | (uint64_t)tie[ii];
  skel_key[e] = k;
  atomicMin((unsigned long long *)&best[r], (unsigned long long)k);
  return k;
}

// windows up to a wave long: one thread each; longer ones are listed
__global__ __launch_bounds__(B) void k_emit_small(const uint32_t *outpos, const uint32_t *wa, const uint32_t *wcnt,
                                                  const uint32_t *eoff, const uint32_t *inpos, const uint32_t *sv,
                                                  const uint64_t *ts, const uint32_t *perm, const uint32_t *tie,
                                                  int64_t n, int wshift, int hshift, uint64_t *skel_key,
                                                  uint32_t *skel_tail, uint32_t *skel_head, uint64_t *best,
                                                  uint64_t *wraw, uint32_t *big, unsigned long long *nbig) {
  for (int64_t q = (int64_t)blockIdx.x * B + threadIdx.x; q < n; q += (int64_t)gridDim.x * B) {
    const uint32_t c = wcnt[q];
    if (c == 0) continue;
    if (c > BIG_WINDOW) {
      big[atomicAdd(nbig, 1ull)] = (uint32_t)q;
      continue;
    }
    const uint32_t s = sv[outpos[q]] >> 1, a = wa[q];
    const uint64_t hid = perm[s], th = ts[s];
    const int64_t e0 = eoff[q];
    uint64_t mn = NONE64;
    for (uint32_t j = 0; j < c; j++) {
      const uint64_t k =
          emit_row(e0 + j, a + j, s, hid, th, inpos, sv, ts, tie, wshift, hshift, skel_key, skel_tail, skel_head, best,
                   wraw);
      mn = k < mn ? k : mn;
    }
    if (mn != NONE64) atomicMin((unsigned long long *)&best[s], (unsigned long long)mn);
  }
}

// one workgroup per long window
__global__ __launch_bounds__(B) void k_emit_big(const uint32_t *big, const uint32_t *outpos, const uint32_t *wa,
                                                const uint32_t *wcnt, const uint32_t *eoff, const uint32_t *inpos,
                                                const uint32_t *sv, const uint64_t *ts, const uint32_t *perm,
                                                const uint32_t *tie, int wshift, int hshift, uint64_t *skel_key,
                                                uint32_t *skel_tail, uint32_t *skel_head, uint64_t *best,
                                                uint64_t *wraw) {
  const uint32_t q = big[blockIdx.x];
  const uint32_t c = wcnt[q], s = sv[outpos[q]] >> 1, a = wa[q];
  const uint64_t hid = perm[s], th = ts[s];
  const int64_t e0 = eoff[q];
  uint64_t mn = NONE64;
  for (uint32_t j = threadIdx.x; j < c; j += B) {
    const uint64_t k =
        emit_row(e0 + j, a + j, s, hid, th, inpos, sv, ts, tie, wshift, hshift, skel_key, skel_tail, skel_head, best,
                 wraw);
    mn = k < mn ? k : mn;
  }
  mn = wave_min_u64(mn);
  if (wave_lane() == 0 && mn != NONE64) atomicMin((unsigned long long *)&best[s], (unsigned long long)mn);
}

__global__ __launch_bounds__(B) void k_fill_best(uint64_t *best, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) best[i] = NONE64;
}

__global__ void k_zero_u64(uint64_t *p) { *p = 0; }

__global__ void k_put_u64(uint64_t *p, uint64_t v) { *p = v; }

}  // namespace

size_t stage_causal_skeleton_scratch(int64_t n) {
  const int64_t n2 = 2 * n;
  Ws w;
  w.alloc<uint64_t>(n2);  // raw weights, when the weights are ranked
  const size_t r0 = w.off;
  for (int k = 0; k < 4; k++) w.alloc<uint32_t>(n2);  // ikey, ival and their ping-pong copies
  // phase 1: the time sort's arrays, then the runs of equal times beside them
  Ws a;
  a.alloc<uint64_t>(n);
  a.alloc<uint4>(n);
  a.alloc<uint4>(n);
  Ws r;
  for (int k = 0; k < 3; k++) r.alloc<uint32_t>(n + 1);
  size_t p1 = a.off + (radix_ws_bytes(n) > r.off + scan_ws_bytes(n + 1) ? radix_ws_bytes(n)
                                                                        : r.off + scan_ws_bytes(n + 1));
  // phase 2: the vertex sort; phase 3: side counts and positions, ties, windows
  const size_t p2 = radix_ws_bytes(n2);
  Ws c;
  c.alloc<uint32_t>(n2 + 1);
  for (int k = 0; k < 2; k++) c.alloc<uint32_t>(n);
  for (int k = 0; k < 8; k++) c.alloc<uint32_t>(n + 1);
  const size_t p3 = c.off + scan_ws_bytes(n2 + 1);
  size_t x = p1 > p2 ? p1 : p2;
  if (p3 > x) x = p3;
  x += w.off;
  const size_t rk = r0 + stage_rank_weights_scratch(n2);
  return (x > rk ? x : rk) + 4096;
}

ce_status stage_causal_skeleton(const int32_t *src, const int32_t *dst, const int64_t *t, Bufs &b, Ws &ws,
                                hipStream_t s) {
  const int64_t n = b.n, n2 = 2 * n;
  size_t m0 = ws.mark();
  uint64_t *wraw = ws.alloc<uint64_t>(n2);  // raw weights, when the weights are ranked
  const size_t mr = ws.mark();
  uint32_t *ikey = ws.alloc<uint32_t>(n2);
  uint32_t *ival = ws.alloc<uint32_t>(n2);
  uint32_t *ikey_alt = ws.alloc<uint32_t>(n2);
  uint32_t *ival_alt = ws.alloc<uint32_t>(n2);
  CE_WS_CHECK(ws);
  // 1-2. ranks, then entries in (t, in before out, rank) order
  {
    size_t m1 = ws.mark();
    const uint4 *vals = nullptr;
    CE_TRY(sort_records_by_time(src, dst, t, b, ws, s, &vals));
    uint32_t *f = ws.alloc<uint32_t>(n + 1), *fx = ws.alloc<uint32_t>(n + 1), *start = ws.alloc<uint32_t>(n + 1);
    CE_WS_CHECK(ws);
    CE_LAUNCH(k_run_flags, dim3(grid_for(n, B)), dim3(B), 0, s, b.ts, n, f);
    CE_HIP(hipGetLastError());
    CE_TRY(scan_exclusive_u32(f, fx, n, ws, s));
    CE_LAUNCH(k_run_starts, dim3(grid_for(n, B)), dim3(B), 0, s, f, fx, n, start);
    CE_LAUNCH(k_causal_entries, dim3(grid_for(n, B)), dim3(B), 0, s, vals, f, fx, start, n, b.perm, b.grank, ikey,
              ival);
    CE_HIP(hipGetLastError());
    ws.release(m1);
  }
  bool alt = false;
  CE_TRY((radix_sort_pairs<uint32_t, uint32_t>(ikey, ival, ikey_alt, ival_alt, n2, 0, b.vbits, false, &alt, ws, s)));
  const uint32_t *sk = alt ? ikey_alt : ikey;
  const uint32_t *sv = alt ? ival_alt : ival;
  // 3. side positions, tie indices, windows
  uint32_t *incount = ws.alloc<uint32_t>(n2 + 1);
  uint32_t *inpos = ws.alloc<uint32_t>(n), *outpos = ws.alloc<uint32_t>(n);
  uint32_t *gf = ws.alloc<uint32_t>(n + 1), *gx = ws.alloc<uint32_t>(n + 1);
  uint32_t *gstart = ws.alloc<uint32_t>(n + 1), *tie = ws.alloc<uint32_t>(n + 1);
  uint32_t *wa = ws.alloc<uint32_t>(n + 1), *wcnt = ws.alloc<uint32_t>(n + 1);
  uint32_t *eoff = ws.alloc<uint32_t>(n + 1), *big = ws.alloc<uint32_t>(n + 1);
  CE_WS_CHECK(ws);
  CE_LAUNCH(k_in_flags, dim3(grid_for(n2, B)), dim3(B), 0, s, sv, n2, incount);
  CE_HIP(hipGetLastError());
  CE_TRY(scan_exclusive_u32(incount, incount, n2, ws, s));
  CE_LAUNCH(k_side_pos, dim3(grid_for(n2, B)), dim3(B), 0, s, sv, incount, n2, inpos, outpos);
  CE_LAUNCH(k_tie_flags, dim3(grid_for(n, B)), dim3(B), 0, s, inpos, sk, sv, b.ts, n, gf);
  CE_HIP(hipGetLastError());
  CE_TRY(scan_exclusive_u32(gf, gx, n, ws, s));
  CE_LAUNCH(k_run_starts, dim3(grid_for(n, B)), dim3(B), 0, s, gf, gx, n, gstart);
  CE_LAUNCH(k_zero_u64, dim3(1), dim3(1), 0, s, &b.hdr[7]);
  CE_LAUNCH(k_ties, dim3(grid_for(n, B)), dim3(B), 0, s, gf, gx, gstart, n, tie, (unsigned int *)&b.hdr[7]);
  CE_LAUNCH(k_windows, dim3(grid_for(n, B)), dim3(B), 0, s, sk, incount, inpos, outpos, n, wa, wcnt);
  CE_HIP(hipGetLastError());
  CE_TRY(scan_exclusive_u32(wcnt, eoff, n, ws, s));
  uint64_t h[2];
  {
    uint32_t *pin = (uint32_t *)pinned_scratch();
    CE_HIP(hipMemcpyAsync(pin + 16, eoff + n, 4, hipMemcpyDeviceToHost, s));
    CE_TRY(read_u64(&b.hdr[7], h, 1, s));  // synchronises the stream
    h[1] = pin[16];
  }
  const uint32_t maxtie = (uint32_t)h[0];
  const int64_t S = (int64_t)h[1];
  if (S > n2) {
    set_error("internal: causal skeleton larger than 2n");
    return CE_EDEVICE;
  }
  b.S = S;
  b.jbits = bits_for(maxtie);
  b.hshift = b.jbits;
  b.wshift = b.idbits + b.jbits;
  if (!choose_key_layout(b, S)) {  // the all-ones word marks an absent edge
    set_error("too many records for the causal key: bits(rows - 1) + bits(n-1) + bits(largest equal-time "
              "in-degree - 1) > 63");
    return CE_ERANGE;
  }
  uint64_t *wr = b.rank ? wraw : nullptr;
  // 4. rows, each offering its key to both records' first Boruvka minimum
  CE_LAUNCH(k_fill_best, dim3(grid_for(n, B)), dim3(B), 0, s, b.best, n);
  CE_LAUNCH(k_zero_u64, dim3(1), dim3(1), 0, s, &b.hdr[7]);
  CE_LAUNCH(k_emit_small, dim3(grid_for(n, B)), dim3(B), 0, s, outpos, wa, wcnt, eoff, inpos, sv, b.ts, b.perm, tie, n,
            b.wshift, b.hshift, b.skel_key, b.skel_tail, b.skel_tid, b.best, wr, big,
            (unsigned long long *)&b.hdr[7]);
  CE_HIP(hipGetLastError());
  uint64_t nbig = 0;
  CE_TRY(read_u64(&b.hdr[7], &nbig, 1, s));
  if ((int64_t)nbig > n) {
    set_error("internal: long-window count");
    return CE_EDEVICE;
  }
  if (nbig > 0)
    CE_LAUNCH(k_emit_big, dim3((unsigned)nbig), dim3(B), 0, s, big, outpos, wa, wcnt, eoff, inpos, sv, b.ts, b.perm,
              tie, b.wshift, b.hshift, b.skel_key, b.skel_tail, b.skel_tid, b.best, wr);
  CE_LAUNCH(k_put_u64, dim3(1), dim3(1), 0, s, &b.hdr[H_C7], (uint64_t)S);  // the rows, for Boruvka's first round
  CE_HIP(hipGetLastError());
  ws.release(mr);
  if (b.rank) CE_TRY(stage_rank_weights(b, wraw, S, ws, s));
  ws.release(m0);
  return CE_OK;
}

}  // namespace ce
