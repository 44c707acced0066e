// Stages A1-A6: validate, group-and-sort by (vertex, time), emit the path
// skeleton, Boruvka minimum spanning forest, sort the MSF by canonical key.
//
// Grouping (Alg. 3 "adjacency list", Alg. 2 "Sort E_i by time"): the records
// are first sorted once by (t, id) with a stable radix sort on t - tmin; the
// position in that order is the record's rank. The 2n incidence entries
// (vertex, 2*rank+side) are then stably radix-sorted by vertex, so every
// vertex's list comes out in rank order, i.e. time order with ties by id,
// whatever its degree (hubs need no special splitting).
//
// Skeleton (Alg. 3 with the undirected node-local MST of Sec. 5.3): each list
// entry after the first links to its predecessor. The edge is stored at slot
// 2*head+side of its HEAD rank, so a record is the head of at most two skeleton
// edges. Its 64-bit key packs the canonical key (w, head id, 2^32-1-tail id):
//     key = w << (idbits+1) | head_id << 1 | bit
// where bit orders the (at most two) edges sharing a head by descending tail
// id. Edges with equal keys (a pair consecutive in both endpoint lists) are
// the same line-graph edge; one copy is dropped.
#include "ce_internal.h"

namespace ce {

namespace {

constexpr int B = 256;

__device__ inline uint64_t t_to_ord(int64_t t) { return (uint64_t)t ^ (uint64_t(1) << 63); }

// hdr[0] |= 1 self loop, 2 id out of range; hdr[1] = min t (ordered), hdr[2] = max t (ordered)
__global__ __launch_bounds__(B) void k_validate(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n,
                                                int64_t V, uint64_t *hdr) {
  __shared__ uint64_t smin[B / 64], smax[B / 64];
  __shared__ uint32_t sflag;
  if (threadIdx.x == 0) sflag = 0;
  __syncthreads();
  uint64_t mn = NONE64, mx = 0;
  uint32_t flag = 0;
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) {
    int32_t a = src[i], b = dst[i];
    if (a == b) flag |= 1u;
    if (a < 0 || b < 0 || (int64_t)a >= V || (int64_t)b >= V) flag |= 2u;
    uint64_t o = t_to_ord(t[i]);
    mn = o < mn ? o : mn;
    mx = o > mx ? o : mx;
  }
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

__global__ void k_init_hdr(uint64_t *hdr) {
  if (threadIdx.x < 16) hdr[threadIdx.x] = 0;
  if (threadIdx.x == 0) hdr[1] = NONE64;
}

__global__ __launch_bounds__(B) void k_tkeys(const int64_t *t, int64_t n, int64_t tmin, uint64_t *keys) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B)
    keys[i] = (uint64_t)(t[i] - tmin);
}

// incidence entries in rank order: (src, 2r), (dst, 2r+1)
__global__ __launch_bounds__(B) void k_incidence(const uint32_t *perm, const int32_t *src, const int32_t *dst,
                                                 int64_t n, uint32_t *ikey, uint32_t *ival) {
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < n; r += (int64_t)gridDim.x * B) {
    uint32_t id = perm[r];
    ikey[2 * r] = (uint32_t)src[id];
    ikey[2 * r + 1] = (uint32_t)dst[id];
    ival[2 * r] = (uint32_t)(2 * r);
    ival[2 * r + 1] = (uint32_t)(2 * r + 1);
  }
}

// every incidence entry names its slot; the entry's predecessor in the same
// vertex list is the tail of the skeleton edge stored there
__global__ __launch_bounds__(B) void k_skel_tails(const uint32_t *ikey, const uint32_t *ival, int64_t n2,
                                                  uint32_t *skel_tail) {
  for (int64_t k = (int64_t)blockIdx.x * B + threadIdx.x; k < n2; k += (int64_t)gridDim.x * B) {
    uint32_t slot = ival[k];
    skel_tail[slot] = (k > 0 && ikey[k - 1] == ikey[k]) ? (ival[k - 1] >> 1) : NONE32;
  }
}

// Also seeds the first Boruvka round: every record starts as its own
// component, so each edge offers its key to both of its records.
__global__ __launch_bounds__(B) void k_skel_keys(uint32_t *skel_tail, const uint64_t *ts, const uint32_t *perm,
                                                 int64_t n, int idbits, uint64_t *skel_key, uint64_t *best) {
  for (int64_t h = (int64_t)blockIdx.x * B + threadIdx.x; h < n; h += (int64_t)gridDim.x * B) {
    uint32_t t0 = skel_tail[2 * h], t1 = skel_tail[2 * h + 1];
    if (t0 != NONE32 && t0 == t1) {  // the same pair twice: one line-graph edge
      t1 = NONE32;
      skel_tail[2 * h + 1] = NONE32;
    }
    const uint64_t hid = perm[h];
    const uint64_t th = ts[h];
    uint32_t i0 = t0 != NONE32 ? perm[t0] : 0u, i1 = t1 != NONE32 ? perm[t1] : 0u;
    uint64_t k0 = NONE64, k1 = NONE64;
    if (t0 != NONE32) {
      uint64_t bit = (t1 != NONE32 && i0 < i1) ? 1u : 0u;
      k0 = ((th - ts[t0]) << (idbits + 1)) | (hid << 1) | bit;
    }
    if (t1 != NONE32) {
      uint64_t bit = (t0 != NONE32 && i1 < i0) ? 1u : 0u;
      k1 = ((th - ts[t1]) << (idbits + 1)) | (hid << 1) | bit;
    }
    skel_key[2 * h] = k0;
    skel_key[2 * h + 1] = k1;
    uint64_t mine = k0 < k1 ? k0 : k1;
    if (mine != NONE64) atomicMin((unsigned long long *)&best[h], (unsigned long long)mine);
    if (t0 != NONE32) atomicMin((unsigned long long *)&best[t0], (unsigned long long)k0);
    if (t1 != NONE32) atomicMin((unsigned long long *)&best[t1], (unsigned long long)k1);
  }
}

__global__ __launch_bounds__(B) void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) p[i] = v;
}
__global__ __launch_bounds__(B) void k_iota_u32(uint32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) p[i] = (uint32_t)i;
}
__global__ __launch_bounds__(B) void k_fill_u8(uint8_t *p, int64_t n, uint8_t v) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) p[i] = v;
}
__global__ __launch_bounds__(B) void k_rankof(const uint32_t *perm, int64_t n, uint32_t *rankof) {
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < n; r += (int64_t)gridDim.x * B) rankof[perm[r]] = (uint32_t)r;
}

// Boruvka: per component, the minimum key over live edges leaving it. A tile
// of 4096 live edges first takes per-component minima in an LDS hash (big
// components are hit by most edges of late rounds), then one atomicMin per
// component per tile; edges whose component finds no free slot go straight
// to global memory.
constexpr int MHS = 512;
__global__ __launch_bounds__(B) void k_bv_min(const uint32_t *live, int64_t nlive, const uint64_t *skel_key,
                                              const uint32_t *skel_tail, const uint32_t *comp, uint64_t *best) {
  __shared__ uint32_t hk[MHS];
  __shared__ unsigned long long hv[MHS];
  for (int i = threadIdx.x; i < MHS; i += B) { hk[i] = NONE32; hv[i] = NONE64; }
  __syncthreads();
  const int64_t tbase = (int64_t)blockIdx.x * (B * CT);
  for (int k = 0; k < CT; k++) {
    const int64_t i = tbase + (int64_t)k * B + threadIdx.x;
    unsigned long long key = NONE64;
    uint32_t cu = 0, cv = 0;
    bool act = false;
    if (i < nlive) {
      const uint32_t e = live[i];
      key = skel_key[e];
      cu = comp[skel_tail[e]];
      cv = comp[e >> 1];
      act = cu != cv;
    }
#pragma unroll
    for (int side = 0; side < 2; side++) {
      const uint32_t c = side ? cv : cu;
      unsigned long long kmin = key;
      const bool upd = wave_combine_first(act, c, [&](bool mine, int leader) {
        const unsigned long long v = wave_min_u64(mine ? key : NONE64);
        if ((int)wave_lane() == leader) kmin = v;
      });
      if (upd) {
        uint32_t sl = (c * 2654435761u) >> 23;  // 9 bits
        bool placed = false;
        for (int probe = 0; probe < 16 && !placed; probe++) {
          uint32_t old = atomicCAS(&hk[sl], NONE32, c);
          if (old == NONE32 || old == c) {
            if (kmin < hv[sl]) atomicMin(&hv[sl], kmin);
            placed = true;
          } else {
            sl = (sl + 1) & (MHS - 1);
          }
        }
        if (!placed && kmin < best[c]) atomicMin((unsigned long long *)&best[c], kmin);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < MHS; i += B) {
    const uint32_t c = hk[i];
    if (c == NONE32) continue;
    const unsigned long long v = hv[i];
    if (v < best[c]) atomicMin((unsigned long long *)&best[c], v);
  }
}

// slot of the (unique) edge with key k: its head is rank rankof[head id]; of
// the two slots of that head, the one holding k
__device__ inline uint32_t slot_of_key(uint64_t k, int idbits, const uint32_t *rankof, const uint64_t *skel_key) {
  uint32_t hid = (uint32_t)((k >> 1) & ((uint64_t(1) << idbits) - 1));
  uint32_t h = rankof[hid];
  return skel_key[2 * (uint64_t)h] == k ? 2 * h : 2 * h + 1;
}

// hook each component root onto the component across its minimum edge; of a
// mutual pair the smaller root stays; the hooking edge joins the forest.
// Roots that hook go to the active list for pointer jumping, the others to
// the list of roots of the next round (roots == nullptr: all records).
__global__ __launch_bounds__(B) void k_bv_hook(const uint32_t *roots, int64_t nroots, const uint32_t *comp,
                                               const uint64_t *best, const uint64_t *skel_key,
                                               const uint32_t *skel_tail, const uint32_t *rankof, int idbits,
                                               uint32_t *hook, uint8_t *msf_flag, uint32_t *active,
                                               unsigned long long *nactive, uint32_t *keep_roots,
                                               unsigned long long *nkeep) {
  bool hk[CT], st[CT];
  uint32_t vals[CT];
  const int64_t base = (int64_t)blockIdx.x * (B * CT) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < CT; k++) {
    const int64_t i = base + (int64_t)k * B;
    hk[k] = false;
    st[k] = false;
    vals[k] = 0;
    if (i >= nroots) continue;
    const uint32_t c = roots ? roots[i] : (uint32_t)i;
    vals[k] = c;
    uint32_t to = c;
    uint64_t bk = best[c];
    if (bk != NONE64) {
      uint32_t e = slot_of_key(bk, idbits, rankof, skel_key);
      uint32_t cu = comp[skel_tail[e]], cv = comp[e >> 1];
      uint32_t o = (cu == c) ? cv : cu;
      bool mutual = best[o] == bk;
      if (!(mutual && c < o)) {
        to = o;
        msf_flag[e] = 1;
        hk[k] = true;
      }
    }
    st[k] = !hk[k] && bk != NONE64;  // isolated components are final
    hook[c] = to;
  }
  tile_append(hk, vals, active, nactive);
  tile_append(st, vals, keep_roots, nkeep);
}

__global__ __launch_bounds__(B) void k_fill_best(const uint32_t *roots, int64_t nroots, uint64_t *best) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < nroots; i += (int64_t)gridDim.x * B)
    best[roots[i]] = NONE64;
}

// pointer jumping over the hooked roots; converged ones leave the list
__global__ __launch_bounds__(B) void k_bv_jump(const uint32_t *act, int64_t nact, uint32_t *hook, uint32_t *out,
                                               unsigned long long *nout) {
  bool keep[CT];
  uint32_t vals[CT];
  const int64_t base = (int64_t)blockIdx.x * (B * CT) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < CT; k++) {
    const int64_t i = base + (int64_t)k * B;
    keep[k] = false;
    vals[k] = 0;
    if (i >= nact) continue;
    uint32_t c = act[i];
    uint32_t h = hook[c];
    uint32_t hh = hook[h];
    if (hh != h) {
      hook[c] = hh;
      keep[k] = true;
      vals[k] = c;
    }
  }
  tile_append(keep, vals, out, nout);
}

__global__ __launch_bounds__(B) void k_bv_relabel(int64_t n, uint32_t *comp, const uint32_t *hook) {
  for (int64_t p = (int64_t)blockIdx.x * B + threadIdx.x; p < n; p += (int64_t)gridDim.x * B) comp[p] = hook[comp[p]];
}

// keep edges whose endpoints lie in different components (live == nullptr: all slots)
__global__ __launch_bounds__(B) void k_bv_filter(const uint32_t *live, int64_t nlive, const uint64_t *skel_key,
                                                 const uint32_t *skel_tail, const uint32_t *comp, uint32_t *out,
                                                 unsigned long long *cnt) {
  bool keep[CT];
  uint32_t vals[CT];
  const int64_t base = (int64_t)blockIdx.x * (B * CT) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < CT; k++) {
    const int64_t i = base + (int64_t)k * B;
    keep[k] = false;
    vals[k] = 0;
    if (i >= nlive) continue;
    uint32_t e = live ? live[i] : (uint32_t)i;
    if (!live && skel_key[e] == NONE64) continue;
    vals[k] = e;
    keep[k] = comp[skel_tail[e]] != comp[e >> 1];
  }
  tile_append(keep, vals, out, cnt);
}

__global__ __launch_bounds__(B) void k_msf_list(const uint8_t *flag, int64_t n2, uint32_t *out,
                                                unsigned long long *cnt) {
  bool keep[CT];
  uint32_t vals[CT];
  const int64_t base = (int64_t)blockIdx.x * (B * CT) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < CT; k++) {
    const int64_t e = base + (int64_t)k * B;
    keep[k] = e < n2 && flag[e];
    vals[k] = (uint32_t)e;
  }
  tile_append(keep, vals, out, cnt);
}

__global__ __launch_bounds__(B) void k_msf_gather(const uint32_t *list, int64_t m, const uint64_t *skel_key,
                                                  const uint32_t *skel_tail, uint64_t *okey, uint64_t *oval) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < m; i += (int64_t)gridDim.x * B) {
    uint32_t e = list[i];
    okey[i] = skel_key[e];
    oval[i] = ((uint64_t)(e >> 1) << 32) | skel_tail[e];
  }
}

}  // namespace

uint64_t *pinned_scratch() {
  static thread_local uint64_t *p = nullptr;
  if (!p) {
    if (hipHostMalloc((void **)&p, 4096, hipHostMallocDefault) != hipSuccess) p = nullptr;
  }
  return p;
}

ce_status read_u64(const uint64_t *dev, uint64_t *host_out, int count, hipStream_t s) {
  uint64_t *h = pinned_scratch();
  if (!h) {
    set_error("hipHostMalloc of the readback buffer failed");
    return CE_EDEVICE;
  }
  CE_HIP(hipMemcpyAsync(h, dev, sizeof(uint64_t) * count, hipMemcpyDeviceToHost, s));
  CE_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < count; i++) host_out[i] = h[i];
  return CE_OK;
}

ce_status stage_validate(const int32_t *src, const int32_t *dst, const int64_t *t, Bufs &b, hipStream_t s,
                         uint64_t *flags, int64_t *tmin, int64_t *tmax) {
  CE_LAUNCH(k_init_hdr, dim3(1), dim3(64), 0, s, b.hdr);
  CE_HIP(hipGetLastError());
  if (b.n > 0) {
    CE_LAUNCH(k_validate, dim3(grid_for(b.n, B, 4096)), dim3(B), 0, s, src, dst, t, b.n, b.V, b.hdr);
    CE_HIP(hipGetLastError());
  }
  uint64_t h[3];
  CE_TRY(read_u64(b.hdr, h, 3, s));
  *flags = h[0];
  *tmin = (int64_t)(h[1] ^ (uint64_t(1) << 63));
  *tmax = (int64_t)(h[2] ^ (uint64_t(1) << 63));
  return CE_OK;
}

__global__ void k_set_u64(uint64_t *p, uint64_t v) { *p = v; }

size_t stage_sort_skeleton_scratch(int64_t n) {
  Ws w;
  w.alloc<uint64_t>(n);      // tkey alt
  w.alloc<uint32_t>(n);      // perm alt
  size_t a = w.off + radix_ws_bytes(n);
  w = Ws();
  w.alloc<uint32_t>(2 * n);  // ikey
  w.alloc<uint32_t>(2 * n);  // ival
  w.alloc<uint32_t>(2 * n);  // ikey alt
  w.alloc<uint32_t>(2 * n);  // ival alt
  size_t b2 = w.off + radix_ws_bytes(2 * n);
  return (a > b2 ? a : b2) + 4096;
}

ce_status stage_sort_skeleton(const int32_t *src, const int32_t *dst, const int64_t *t, Bufs &b, Ws &ws,
                              hipStream_t s) {
  const int64_t n = b.n, n2 = 2 * n;
  size_t m0 = ws.mark();
  // 1. records by (t, id): stable radix sort on t - tmin; values start as ids
  {
    uint64_t *tkey_alt = ws.alloc<uint64_t>(n);
    uint32_t *perm_alt = ws.alloc<uint32_t>(n);
    CE_WS_CHECK(ws);
    CE_LAUNCH(k_tkeys, dim3(grid_for(n, B)), dim3(B), 0, s, t, n, b.tmin, b.ts);
    CE_HIP(hipGetLastError());
    bool alt = false;
    CE_TRY((radix_sort_pairs<uint64_t, uint32_t>(b.ts, b.perm, tkey_alt, perm_alt, n, 0, b.tbits, true, &alt, ws, s)));
    if (alt) {
      CE_HIP(hipMemcpyAsync(b.ts, tkey_alt, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
      CE_HIP(hipMemcpyAsync(b.perm, perm_alt, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    }
    ws.release(m0);
  }
  // 2. incidence entries (vertex, 2*rank+side), stably sorted by vertex
  uint32_t *ikey = ws.alloc<uint32_t>(n2);
  uint32_t *ival = ws.alloc<uint32_t>(n2);
  uint32_t *ikey_alt = ws.alloc<uint32_t>(n2);
  uint32_t *ival_alt = ws.alloc<uint32_t>(n2);
  CE_WS_CHECK(ws);
  CE_LAUNCH(k_incidence, dim3(grid_for(n, B)), dim3(B), 0, s, b.perm, src, dst, n, ikey, ival);
  CE_HIP(hipGetLastError());
  bool alt = false;
  CE_TRY((radix_sort_pairs<uint32_t, uint32_t>(ikey, ival, ikey_alt, ival_alt, n2, 0, b.vbits, true, &alt, ws, s)));
  const uint32_t *sk = alt ? ikey_alt : ikey;
  const uint32_t *sv = alt ? ival_alt : ival;
  // 3. skeleton: predecessor in the same vertex list, then packed keys
  CE_LAUNCH(k_skel_tails, dim3(grid_for(n2, B)), dim3(B), 0, s, sk, sv, n2, b.skel_tail);
  CE_LAUNCH(k_fill_u64, dim3(grid_for(n, B)), dim3(B), 0, s, b.best, n, NONE64);
  CE_HIP(hipGetLastError());
  CE_LAUNCH(k_skel_keys, dim3(grid_for(n, B)), dim3(B), 0, s, b.skel_tail, b.ts, b.perm, n, b.idbits,
                     b.skel_key, b.best);
  CE_HIP(hipGetLastError());
  ws.release(m0);
  return CE_OK;
}

size_t stage_boruvka_scratch(int64_t n) {
  Ws w;
  w.alloc<uint32_t>(n);      // comp
  w.alloc<uint32_t>(n);      // rankof
  w.alloc<uint32_t>(n);      // hook
  w.alloc<uint32_t>(n);      // active
  w.alloc<uint32_t>(n);      // active alt
  w.alloc<uint32_t>(n);      // roots
  w.alloc<uint32_t>(n);      // roots alt
  w.alloc<uint32_t>(2 * n);  // live
  w.alloc<uint32_t>(2 * n);  // live alt
  return w.off + 4096;
}

static unsigned tiles_for(int64_t n) { return (unsigned)((n + (int64_t)B * CT - 1) / ((int64_t)B * CT)); }

ce_status stage_boruvka(Bufs &b, Ws &ws, hipStream_t s) {
  const int64_t n = b.n, n2 = 2 * n;
  size_t m0 = ws.mark();
  uint32_t *comp = ws.alloc<uint32_t>(n);
  uint32_t *rankof = ws.alloc<uint32_t>(n);
  uint32_t *hook = ws.alloc<uint32_t>(n);
  uint32_t *act = ws.alloc<uint32_t>(n);
  uint32_t *act2 = ws.alloc<uint32_t>(n);
  uint32_t *roots = ws.alloc<uint32_t>(n);
  uint32_t *roots2 = ws.alloc<uint32_t>(n);
  uint32_t *live = ws.alloc<uint32_t>(n2);
  uint32_t *live2 = ws.alloc<uint32_t>(n2);
  CE_WS_CHECK(ws);
  uint64_t *best = b.best;  // seeded for the first round by k_skel_keys
  unsigned long long *cnt = (unsigned long long *)&b.hdr[4];
  unsigned long long *cnt2 = (unsigned long long *)&b.hdr[5];
  unsigned long long *cnt3 = (unsigned long long *)&b.hdr[7];
  CE_LAUNCH(k_fill_u8, dim3(grid_for(n2, B)), dim3(B), 0, s, b.msf_flag, n2, (uint8_t)0);
  CE_LAUNCH(k_iota_u32, dim3(grid_for(n, B)), dim3(B), 0, s, comp, n);
  CE_LAUNCH(k_rankof, dim3(grid_for(n, B)), dim3(B), 0, s, b.perm, n, rankof);
  CE_HIP(hipGetLastError());
  const uint32_t *cur = nullptr;  // first round: all slots
  const uint32_t *rcur = nullptr; // first round: all records are roots
  int64_t nlive = n2, nroots = n;
  int rounds = 0;
  while (nlive > 0) {
    if (++rounds > 64) {
      set_error("Boruvka did not converge");
      return CE_EDEVICE;
    }
    if (rounds > 1) {
      CE_LAUNCH(k_fill_best, dim3(grid_for(nroots, B)), dim3(B), 0, s, rcur, nroots, best);
      CE_LAUNCH(k_bv_min, dim3(tiles_for(nlive)), dim3(B), 0, s, cur, nlive, b.skel_key, b.skel_tail, comp, best);
    }
    CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[4], (uint64_t)0);
    CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[7], (uint64_t)0);
    CE_LAUNCH(k_bv_hook, dim3(tiles_for(nroots)), dim3(B), 0, s, rcur, nroots, comp, best, b.skel_key,
                       b.skel_tail, rankof, b.idbits, hook, b.msf_flag, act, cnt, roots, cnt3);
    CE_HIP(hipGetLastError());
    uint64_t hv[4];
    CE_TRY(read_u64(&b.hdr[4], hv, 4, s));
    uint64_t nact = hv[0];
    nroots = (int64_t)hv[3];
    rcur = roots;
    uint32_t *tr = roots; roots = roots2; roots2 = tr;
    for (int it = 0; nact > 0; it++) {
      if (it > 64) {
        set_error("Boruvka pointer jumping did not converge");
        return CE_EDEVICE;
      }
      CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[5], (uint64_t)0);
      CE_LAUNCH(k_bv_jump, dim3(tiles_for((int64_t)nact)), dim3(B), 0, s, act, (int64_t)nact, hook, act2,
                         cnt2);
      CE_HIP(hipGetLastError());
      CE_TRY(read_u64(&b.hdr[5], &nact, 1, s));
      uint32_t *t = act; act = act2; act2 = t;
    }
    CE_LAUNCH(k_bv_relabel, dim3(grid_for(n, B)), dim3(B), 0, s, n, comp, hook);
    CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[4], (uint64_t)0);
    CE_LAUNCH(k_bv_filter, dim3(tiles_for(nlive)), dim3(B), 0, s, cur, nlive, b.skel_key, b.skel_tail, comp,
                       live, cnt);
    CE_HIP(hipGetLastError());
    uint64_t nl = 0;
    CE_TRY(read_u64(&b.hdr[4], &nl, 1, s));
    nlive = (int64_t)nl;
    cur = live;
    uint32_t *t = live; live = live2; live2 = t;
  }
  ws.release(m0);
  return CE_OK;
}

size_t stage_msf_sort_scratch(int64_t n) {
  Ws w;
  w.alloc<uint64_t>(n);
  w.alloc<uint64_t>(n);
  w.alloc<uint32_t>(n);
  return w.off + radix_ws_bytes(n) + 4096;
}

ce_status stage_msf_sort(Bufs &b, Ws &ws, hipStream_t s, int64_t *m_out) {
  const int64_t n = b.n, n2 = 2 * n;
  size_t m0 = ws.mark();
  uint64_t *key_alt = ws.alloc<uint64_t>(n);
  uint64_t *val_alt = ws.alloc<uint64_t>(n);
  uint32_t *list = ws.alloc<uint32_t>(n);
  CE_WS_CHECK(ws);
  CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[6], (uint64_t)0);
  CE_LAUNCH(k_msf_list, dim3(tiles_for(n2)), dim3(B), 0, s, b.msf_flag, n2, list,
                     (unsigned long long *)&b.hdr[6]);
  CE_HIP(hipGetLastError());
  uint64_t m = 0;
  CE_TRY(read_u64(&b.hdr[6], &m, 1, s));
  if ((int64_t)m > n - 1) {
    set_error("spanning forest larger than n-1");
    return CE_EDEVICE;
  }
  if (m > 0)
    CE_LAUNCH(k_msf_gather, dim3(grid_for((int64_t)m, B)), dim3(B), 0, s, list, (int64_t)m, b.skel_key,
                       b.skel_tail, b.msf_key, b.msf_val);
  bool alt = false;
  CE_TRY((radix_sort_pairs<uint64_t, uint64_t>(b.msf_key, b.msf_val, key_alt, val_alt, (int64_t)m, 0, b.keybits,
                                                false, &alt, ws, s)));
  if (alt && m > 0) {
    CE_HIP(hipMemcpyAsync(b.msf_key, key_alt, sizeof(uint64_t) * m, hipMemcpyDeviceToDevice, s));
    CE_HIP(hipMemcpyAsync(b.msf_val, val_alt, sizeof(uint64_t) * m, hipMemcpyDeviceToDevice, s));
  }
  ws.release(m0);
  *m_out = (int64_t)m;
  return CE_OK;
}

}  // namespace ce
