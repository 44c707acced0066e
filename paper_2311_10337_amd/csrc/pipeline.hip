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
#include <algorithm>

#include "ce_internal.h"

namespace ce {

namespace {

constexpr int B = 256;

__device__ inline uint64_t t_to_ord(int64_t t) { return (uint64_t)t ^ (uint64_t(1) << 63); }

// hdr[0] |= 1 self loop, 2 id out of range; hdr[1] = min t (ordered), hdr[2] = max t (ordered).
// A record of graph g must name vertices in [0, voff[g+1] - voff[g]).
__global__ __launch_bounds__(B) void k_validate(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n,
                                                const int64_t *eoff, const int64_t *voff, int64_t G,
                                                uint64_t *hdr) {
  __shared__ uint64_t smin[B / 64], smax[B / 64];
  __shared__ uint32_t sflag;
  if (threadIdx.x == 0) sflag = 0;
  __syncthreads();
  uint64_t mn = NONE64, mx = 0;
  uint32_t flag = 0;
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) {
    int32_t a = src[i], b = dst[i];
    const uint32_t g = G > 1 ? graph_of(eoff, G, i) : 0u;
    const int64_t V = voff[g + 1] - voff[g];
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

// the time sort carries (id, src, dst, graph) along, so grouping needs no
// gathers; vertex ids become global (graph offset + local id)
__global__ __launch_bounds__(B) void k_tkeys(const int64_t *t, const int32_t *src, const int32_t *dst, int64_t n,
                                             const int64_t *eoff, const int64_t *voff, int64_t G, int64_t tmin,
                                             uint64_t *keys, uint4 *vals) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) {
    const uint32_t g = G > 1 ? graph_of(eoff, G, i) : 0u;
    const uint32_t vb = (uint32_t)voff[g];
    keys[i] = (uint64_t)(t[i] - tmin);
    vals[i] = make_uint4((uint32_t)i, vb + (uint32_t)src[i], vb + (uint32_t)dst[i], g);
  }
}

// incidence entries in rank order: key = vertex, value (implicit) = 2r+side
__global__ __launch_bounds__(B) void k_incidence(const uint4 *vals, int64_t n, uint32_t *perm, uint32_t *grank,
                                                 uint32_t *ikey) {
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < n; r += (int64_t)gridDim.x * B) {
    const uint4 v = vals[r];
    perm[r] = v.x;
    grank[r] = v.w;
    ikey[2 * r] = v.y;
    ikey[2 * r + 1] = v.z;
  }
}

// One graph whose time span fits 32 bits: the id rides in the key's low half,
// key = (t - tmin) << 32 | id, and the value is (src | dst << 32), so a radix
// pass over bits [32, 32 + bits(span)) moves 16 bytes per record instead of 24.
// Stability keeps ids in order within equal times either way.
__global__ __launch_bounds__(B) void k_tkeys_packed(const int64_t *t, const int32_t *src, const int32_t *dst,
                                                    int64_t n, int64_t tmin, uint64_t *keys, uint64_t *vals) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) {
    keys[i] = ((uint64_t)(t[i] - tmin) << 32) | (uint64_t)i;
    vals[i] = (uint64_t)(uint32_t)src[i] | ((uint64_t)(uint32_t)dst[i] << 32);
  }
}

// incidence entries from the packed sort; also t - tmin by rank (keys may be ts itself)
__global__ __launch_bounds__(B) void k_incidence_packed(const uint64_t *keys, const uint64_t *vals, int64_t n,
                                                        uint64_t *ts, uint32_t *perm, uint32_t *grank,
                                                        uint32_t *ikey) {
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < n; r += (int64_t)gridDim.x * B) {
    const uint64_t k = keys[r], v = vals[r];
    ts[r] = k >> 32;
    perm[r] = (uint32_t)k;
    grank[r] = 0;
    ikey[2 * r] = (uint32_t)v;
    ikey[2 * r + 1] = (uint32_t)(v >> 32);
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
// The low bit orders the two edges of a head by descending tail id; it only
// decides their order when they have the same weight (else w does), so the
// tails' ids are read only then.
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
    const uint64_t w0 = t0 != NONE32 ? th - ts[t0] : 0, w1 = t1 != NONE32 ? th - ts[t1] : 0;
    uint64_t b0 = 0, b1 = 0;
    if (t0 != NONE32 && t1 != NONE32 && w0 == w1) {
      const uint32_t i0 = perm[t0], i1 = perm[t1];
      b0 = i0 < i1 ? 1u : 0u;
      b1 = 1u - b0;
    }
    const uint64_t k0 = t0 != NONE32 ? (w0 << (idbits + 1)) | (hid << 1) | b0 : NONE64;
    const uint64_t k1 = t1 != NONE32 ? (w1 << (idbits + 1)) | (hid << 1) | b1 : NONE64;
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
__global__ __launch_bounds__(B) void k_fill_u8(uint8_t *p, int64_t n, uint8_t v) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) p[i] = v;
}
__global__ __launch_bounds__(B) void k_rankof(const uint32_t *perm, int64_t n, uint32_t *rankof) {
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < n; r += (int64_t)gridDim.x * B) rankof[perm[r]] = (uint32_t)r;
}

// slot of the (unique) edge with key k: its head is rank rankof[head id]; of
// the two slots of that head, the one holding k
__device__ inline uint32_t slot_of_key(uint64_t k, int idbits, const uint32_t *rankof, const uint64_t *skel_key) {
  uint32_t hid = (uint32_t)((k >> 1) & ((uint64_t(1) << idbits) - 1));
  uint32_t h = rankof[hid];
  return skel_key[2 * (uint64_t)h] == k ? 2 * h : 2 * h + 1;
}

// ---------------------------------------------------------------- Boruvka
// Round 1 runs on records (best[] was seeded while emitting the skeleton).
// Each later round runs on a CONTRACTED graph: components carry dense ids
// 0..C-1 and the live edges are records (key, endpoint ids, slot), so the
// per-round arrays shrink with C and stay cache resident after round 1.

// hook each component onto the component across its minimum edge; of a mutual
// pair the smaller id stays; the hooking edge joins the forest. Hooked
// components go to the active list for pointer jumping.
__global__ __launch_bounds__(B) void k_bv_hook_first(int64_t n, const uint64_t *best, const uint64_t *skel_key,
                                                     const uint32_t *skel_tail, const uint32_t *rankof, int idbits,
                                                     uint32_t *hook, uint8_t *msf_flag, uint32_t *active,
                                                     unsigned long long *nactive) {
  bool keep[CT];
  uint32_t vals[CT];
  const int64_t base = (int64_t)blockIdx.x * (B * CT) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < CT; k++) {
    const int64_t c = base + (int64_t)k * B;
    keep[k] = false;
    vals[k] = (uint32_t)c;
    if (c >= n) continue;
    uint32_t to = (uint32_t)c;
    const uint64_t bk = best[c];
    if (bk != NONE64) {
      // the minimum edge is one of c's own two head slots (read in order) or
      // one where c is the tail (found through its head's rank)
      const uint64_t k0 = skel_key[2 * c], k1 = skel_key[2 * c + 1];
      const uint32_t e = k0 == bk ? (uint32_t)(2 * c)
                                  : (k1 == bk ? (uint32_t)(2 * c + 1) : slot_of_key(bk, idbits, rankof, skel_key));
      const uint32_t tl = skel_tail[e], hd = e >> 1;
      const uint32_t o = (tl == (uint32_t)c) ? hd : tl;
      if (!(best[o] == bk && (uint32_t)c < o)) {
        to = o;
        msf_flag[e] = 1;
        keep[k] = true;
      }
    }
    hook[c] = to;
  }
  tile_append(keep, vals, active, nactive);
}

__global__ __launch_bounds__(B) void k_bv_hook(int64_t C, const uint64_t *best, const uint32_t *bidx,
                                               const uint32_t *eu, const uint32_t *ev, const uint32_t *eslot,
                                               uint32_t *hook, uint8_t *msf_flag, uint32_t *active,
                                               unsigned long long *nactive) {
  bool keep[CT];
  uint32_t vals[CT];
  const int64_t base = (int64_t)blockIdx.x * (B * CT) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < CT; k++) {
    const int64_t c = base + (int64_t)k * B;
    keep[k] = false;
    vals[k] = (uint32_t)c;
    if (c >= C) continue;
    uint32_t to = (uint32_t)c;
    const uint64_t bk = best[c];
    if (bk != NONE64) {
      const uint32_t i = bidx[c];
      const uint32_t o = eu[i] == (uint32_t)c ? ev[i] : eu[i];
      if (!(best[o] == bk && (uint32_t)c < o)) {
        to = o;
        msf_flag[eslot ? eslot[i] : i] = 1;
        keep[k] = true;
      }
    }
    hook[c] = to;
  }
  tile_append(keep, vals, active, nactive);
}

// pointer jumping over the hooked components; converged ones leave the list
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

// surviving roots get dense ids; records without any edge are left out
__global__ __launch_bounds__(B) void k_root_flags(int64_t C, const uint32_t *hook, const uint64_t *best,
                                                  uint32_t *flags) {
  for (int64_t c = (int64_t)blockIdx.x * B + threadIdx.x; c < C; c += (int64_t)gridDim.x * B)
    flags[c] = (hook[c] == (uint32_t)c && best[c] != NONE64) ? 1u : 0u;
}

// the dense id of every component's final root (one gather per component, so
// contraction reads one id per endpoint instead of a root and then its id)
__global__ __launch_bounds__(B) void k_final_ids(int64_t C, const uint32_t *hook, const uint32_t *newid,
                                                 uint32_t *fin) {
  for (int64_t c = (int64_t)blockIdx.x * B + threadIdx.x; c < C; c += (int64_t)gridDim.x * B)
    fin[c] = newid[hook[c]];
}

// contract: live edges between different final roots, endpoints renamed to dense ids
__global__ __launch_bounds__(B) void k_contract_first(int64_t n2, const uint64_t *skel_key, const uint32_t *skel_tail,
                                                      const uint32_t *fin, uint64_t *okey,
                                                      uint32_t *ou, uint32_t *ov, uint32_t *oslot,
                                                      unsigned long long *cnt) {
  bool keep[CT];
  uint32_t pos[CT], nu[CT], nv[CT];
  uint64_t kk[CT];
  const int64_t base = (int64_t)blockIdx.x * (B * CT) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < CT; k++) {
    const int64_t e = base + (int64_t)k * B;
    keep[k] = false;
    kk[k] = NONE64;
    nu[k] = nv[k] = 0;
    if (e >= n2) continue;
    kk[k] = skel_key[e];
    if (kk[k] == NONE64) continue;
    const uint32_t fu = fin[skel_tail[e]], fv = fin[e >> 1];
    if (fu == fv) continue;
    keep[k] = true;
    nu[k] = fu;
    nv[k] = fv;
  }
  tile_positions(keep, pos, cnt);
#pragma unroll
  for (int k = 0; k < CT; k++) {
    if (!keep[k]) continue;
    const uint32_t p = pos[k];
    okey[p] = kk[k];
    ou[p] = nu[k];
    ov[p] = nv[k];
    oslot[p] = (uint32_t)(base + (int64_t)k * B);
  }
}

__global__ __launch_bounds__(B) void k_contract(int64_t E, const uint64_t *key, const uint32_t *eu, const uint32_t *ev,
                                                const uint32_t *eslot, const uint32_t *fin,
                                                uint64_t *okey, uint32_t *ou, uint32_t *ov, uint32_t *oslot,
                                                unsigned long long *cnt) {
  bool keep[CT];
  uint32_t pos[CT], nu[CT], nv[CT];
  const int64_t base = (int64_t)blockIdx.x * (B * CT) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < CT; k++) {
    const int64_t i = base + (int64_t)k * B;
    keep[k] = false;
    nu[k] = nv[k] = 0;
    if (i >= E) continue;
    const uint32_t fu = fin[eu[i]], fv = fin[ev[i]];
    if (fu == fv) continue;
    keep[k] = true;
    nu[k] = fu;
    nv[k] = fv;
  }
  tile_positions(keep, pos, cnt);
#pragma unroll
  for (int k = 0; k < CT; k++) {
    if (!keep[k]) continue;
    const int64_t i = base + (int64_t)k * B;
    const uint32_t p = pos[k];
    okey[p] = key[i];
    ou[p] = nu[k];
    ov[p] = nv[k];
    oslot[p] = eslot ? eslot[i] : (uint32_t)i;
  }
}

// Filter split (Filter-Kruskal applied to Borůvka): the live edges with key
// below a pivot go to the front of the output lists, the others to their
// back, counted down from `cap`. Light and heavy together are E <= cap
// entries, so later contractions of the light part, which only shrink it,
// never reach the heavy part.
__global__ __launch_bounds__(B) void k_split(int64_t E, const uint64_t *key, const uint32_t *eu, const uint32_t *ev,
                                             const uint32_t *eslot, uint64_t pivot, int64_t cap, uint64_t *okey,
                                             uint32_t *ou, uint32_t *ov, uint32_t *oslot, unsigned long long *nlight,
                                             unsigned long long *nheavy) {
  bool lt[CT], ge[CT];
  uint32_t pl[CT], ph[CT];
  uint64_t kk[CT];
  const int64_t base = (int64_t)blockIdx.x * (B * CT) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < CT; k++) {
    const int64_t i = base + (int64_t)k * B;
    kk[k] = i < E ? key[i] : 0;
    lt[k] = i < E && kk[k] < pivot;
    ge[k] = i < E && kk[k] >= pivot;
  }
  tile_positions(lt, pl, nlight);
  tile_positions(ge, ph, nheavy);
#pragma unroll
  for (int k = 0; k < CT; k++) {
    if (!lt[k] && !ge[k]) continue;
    const int64_t i = base + (int64_t)k * B;
    const int64_t p = lt[k] ? (int64_t)pl[k] : cap - 1 - (int64_t)ph[k];
    okey[p] = kk[k];
    ou[p] = eu[i];
    ov[p] = ev[i];
    oslot[p] = eslot ? eslot[i] : (uint32_t)i;
  }
}

// root of every component of the split graph after another light round:
// hook maps this round's roots to their new roots
__global__ __launch_bounds__(B) void k_compose_roots(int64_t C, const uint32_t *hook, uint32_t *rootof, bool first) {
  for (int64_t c = (int64_t)blockIdx.x * B + threadIdx.x; c < C; c += (int64_t)gridDim.x * B)
    rootof[c] = hook[first ? (uint32_t)c : rootof[c]];
}

// evenly spaced keys of the live list, for the pivot
__global__ void k_sample_keys(int64_t E, const uint64_t *key, int S, uint64_t *out) {
  for (int i = threadIdx.x; i < S; i += blockDim.x) out[i] = key[(int64_t)((unsigned __int128)i * E / S)];
}

// per component, the minimum key over its live edges. A tile of 4096 edges
// first takes per-component minima in an LDS hash (late rounds send most
// edges to a few big components), then one atomicMin per component per tile.
constexpr int MHS = 512;
__global__ __launch_bounds__(B) void k_bv_min(int64_t E, const uint64_t *key, const uint32_t *eu, const uint32_t *ev,
                                              uint64_t *best) {
  __shared__ uint32_t hk[MHS];
  __shared__ unsigned long long hv[MHS];
  for (int i = threadIdx.x; i < MHS; i += B) { hk[i] = NONE32; hv[i] = NONE64; }
  __syncthreads();
  const int64_t tbase = (int64_t)blockIdx.x * (B * CT);
  for (int k = 0; k < CT; k++) {
    const int64_t i = tbase + (int64_t)k * B + threadIdx.x;
    const bool act = i < E;
    const unsigned long long kv = act ? key[i] : NONE64;
    const uint32_t cu = act ? eu[i] : 0u, cv = act ? ev[i] : 0u;
#pragma unroll
    for (int side = 0; side < 2; side++) {
      const uint32_t c = side ? cv : cu;
      unsigned long long kmin = kv;
      const bool upd = wave_combine_first(act, c, [&](bool mine, int leader) {
        const unsigned long long v = wave_min_u64(mine ? kv : NONE64);
        if ((int)wave_lane() == leader) kmin = v;
      });
      if (upd) {
        uint32_t sl = (c * 2654435761u) >> 23;  // 9 bits
        bool placed = false;
        for (int probe = 0; probe < HASH_PROBES && !placed; probe++) {
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

// the edge index holding each component's minimum (keys are unique)
__global__ __launch_bounds__(B) void k_bv_pick(int64_t E, const uint64_t *key, const uint32_t *eu, const uint32_t *ev,
                                               const uint64_t *best, uint32_t *bidx) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < E; i += (int64_t)gridDim.x * B) {
    const uint64_t k = key[i];
    const uint32_t a = eu[i], b = ev[i];
    if (best[a] == k) bidx[a] = (uint32_t)i;
    if (best[b] == k) bidx[b] = (uint32_t)i;
  }
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


// flat rows keep the head rank in skel_tid; the tail id comes from perm
__global__ __launch_bounds__(B) void k_msf_gather_causal(const uint32_t *list, int64_t m, const uint64_t *skel_key,
                                                         const uint32_t *skel_tail, const uint32_t *skel_head,
                                                         uint64_t *okey, uint64_t *oval) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < m; i += (int64_t)gridDim.x * B) {
    uint32_t e = list[i];
    okey[i] = skel_key[e];
    oval[i] = (uint64_t)skel_tail[e] | ((uint64_t)skel_head[e] << 32);
  }
}

__global__ __launch_bounds__(B) void k_msf_gather(const uint32_t *list, int64_t m, const uint64_t *skel_key,
                                                  const uint32_t *skel_tail, uint64_t *okey, uint64_t *oval) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < m; i += (int64_t)gridDim.x * B) {
    uint32_t e = list[i];
    okey[i] = skel_key[e];
    oval[i] = (uint64_t)skel_tail[e] | ((uint64_t)(e >> 1) << 32);
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

// Reads `count` (<= 8) u64 words through the first 64 bytes of the pinned page.
ce_status read_u64(const uint64_t *dev, uint64_t *host_out, int count, hipStream_t s) {
  if (count > 8) {
    set_error("internal: read_u64 count");
    return CE_EDEVICE;
  }
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
    CE_LAUNCH(k_validate, dim3(grid_for(b.n, B, 4096)), dim3(B), 0, s, src, dst, t, b.n, b.eoff, b.voff, b.G,
              b.hdr);
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
  for (int k = 0; k < 4; k++) w.alloc<uint32_t>(2 * n);  // ikey, ival and their ping-pong copies
  size_t base = w.off;
  w.alloc<uint64_t>(n);  // tkey alt
  w.alloc<uint4>(n);     // (id, src, dst)
  w.alloc<uint4>(n);     // ... ping-pong
  size_t a = w.off + radix_ws_bytes(n);
  size_t b2 = base + radix_ws_bytes(2 * n);
  return (a > b2 ? a : b2) + 4096;
}

// Records by (t, id): stable radix sort on t - tmin carrying (id, global src,
// global dst, graph). b.ts receives the sorted times; *vals points at the
// sorted payload inside ws (the caller releases it).
ce_status sort_records_by_time(const int32_t *src, const int32_t *dst, const int64_t *t, Bufs &b, Ws &ws,
                               hipStream_t s, const uint4 **vals) {
  const int64_t n = b.n;
  uint64_t *tkey_alt = ws.alloc<uint64_t>(n);
  uint4 *tval = ws.alloc<uint4>(n);
  uint4 *tval_alt = ws.alloc<uint4>(n);
  CE_WS_CHECK(ws);
  CE_LAUNCH(k_tkeys, dim3(grid_for(n, B)), dim3(B), 0, s, t, src, dst, n, b.eoff, b.voff, b.G, b.tmin, b.ts, tval);
  CE_HIP(hipGetLastError());
  bool alt = false;
  CE_TRY((radix_sort_pairs<uint64_t, uint4>(b.ts, tval, tkey_alt, tval_alt, n, 0, b.tbits, false, &alt, ws, s)));
  if (alt) CE_HIP(hipMemcpyAsync(b.ts, tkey_alt, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
  *vals = alt ? tval_alt : tval;
  return CE_OK;
}

ce_status stage_sort_skeleton(const int32_t *src, const int32_t *dst, const int64_t *t, Bufs &b, Ws &ws,
                              hipStream_t s) {
  const int64_t n = b.n, n2 = 2 * n;
  size_t m0 = ws.mark();
  uint32_t *ikey = ws.alloc<uint32_t>(n2);
  uint32_t *ival = ws.alloc<uint32_t>(n2);
  uint32_t *ikey_alt = ws.alloc<uint32_t>(n2);
  uint32_t *ival_alt = ws.alloc<uint32_t>(n2);
  CE_WS_CHECK(ws);
  // 1. records by (t, id)
  // 2. incidence entries (vertex, 2*rank+side) in rank order, perm by rank
  {
    size_t m1 = ws.mark();
    if (b.G == 1 && b.tbits <= 32) {
      uint64_t *kalt = ws.alloc<uint64_t>(n), *v0 = ws.alloc<uint64_t>(n), *v1 = ws.alloc<uint64_t>(n);
      CE_WS_CHECK(ws);
      CE_LAUNCH(k_tkeys_packed, dim3(grid_for(n, B)), dim3(B), 0, s, t, src, dst, n, b.tmin, b.ts, v0);
      CE_HIP(hipGetLastError());
      bool alt = false;
      CE_TRY((radix_sort_pairs<uint64_t, uint64_t>(b.ts, v0, kalt, v1, n, 32, 32 + b.tbits, false, &alt, ws, s)));
      CE_LAUNCH(k_incidence_packed, dim3(grid_for(n, B)), dim3(B), 0, s, alt ? kalt : b.ts, alt ? v1 : v0, n, b.ts,
                b.perm, b.grank, ikey);
    } else {
      const uint4 *vals = nullptr;
      CE_TRY(sort_records_by_time(src, dst, t, b, ws, s, &vals));
      CE_LAUNCH(k_incidence, dim3(grid_for(n, B)), dim3(B), 0, s, vals, n, b.perm, b.grank, ikey);
    }
    CE_HIP(hipGetLastError());
    ws.release(m1);
  }
  // stable sort by vertex keeps every list in rank order
  bool alt = false;
  CE_TRY((radix_sort_pairs<uint32_t, uint32_t>(ikey, ival, ikey_alt, ival_alt, n2, 0, b.vbits, true, &alt, ws, s)));
  const uint32_t *sk = alt ? ikey_alt : ikey;
  const uint32_t *sv = alt ? ival_alt : ival;
  // 3. skeleton: predecessor in the same vertex list, then packed keys
  CE_LAUNCH(k_skel_tails, dim3(grid_for(n2, B)), dim3(B), 0, s, sk, sv, n2, b.skel_tail);
  CE_LAUNCH(k_fill_u64, dim3(grid_for(n, B)), dim3(B), 0, s, b.best, n, NONE64);
  CE_HIP(hipGetLastError());
  CE_LAUNCH(k_skel_keys, dim3(grid_for(n, B)), dim3(B), 0, s, b.skel_tail, b.ts, b.perm, n, b.idbits, b.skel_key,
            b.best);
  CE_HIP(hipGetLastError());
  ws.release(m0);
  return CE_OK;
}

size_t stage_boruvka_scratch(int64_t n, int64_t slots) {
  Ws w;
  w.alloc<uint32_t>(n);      // hook
  w.alloc<uint32_t>(n);      // bidx
  w.alloc<uint32_t>(n + 1);  // root flags
  w.alloc<uint32_t>(n + 1);  // dense ids
  w.alloc<uint32_t>(n);      // active
  w.alloc<uint32_t>(n);      // active alt
  for (int k = 0; k < 2; k++) {  // edge lists (key, u, v, slot), ping-pong
    w.alloc<uint64_t>(slots);
    w.alloc<uint32_t>(slots);
    w.alloc<uint32_t>(slots);
    w.alloc<uint32_t>(slots);
  }
  return w.off + scan_ws_bytes(n + 1) + 4096;
}

static unsigned tiles_for(int64_t n) { return (unsigned)((n + (int64_t)B * CT - 1) / ((int64_t)B * CT)); }

// A contraction's edge count (a u64 counter on the device) and the number of
// components (the total of the dense-id scan, a u32): hv[0], hv[1].
static ce_status read_count_and_total(const uint64_t *count, const uint32_t *total, uint64_t *hv, hipStream_t s) {
  uint32_t *h = (uint32_t *)pinned_scratch();
  if (!h) {
    set_error("hipHostMalloc of the readback buffer failed");
    return CE_EDEVICE;
  }
  // word 16 of the pinned page is ours; read_u64 uses the first 64 bytes
  CE_HIP(hipMemcpyAsync(h + 16, total, 4, hipMemcpyDeviceToHost, s));
  CE_TRY(read_u64(count, hv, 1, s));  // synchronises the stream
  hv[1] = h[16];
  return CE_OK;
}

// The filter split runs when the live edges number at least 2^20 and more
// than twice the components. The environment variable CE_SPLIT_MIN_EDGES
// (read on every call) overrides the 2^20; 0 turns the split off.
constexpr int SPLIT_SAMPLES = 256;
static int64_t split_min_edges() {
  const char *e = getenv("CE_SPLIT_MIN_EDGES");
  if (!e) return int64_t(1) << 20;
  const long long v = atoll(e);
  return v > 0 ? (int64_t)v : INT64_MAX;
}

// Pivot of the filter split: about C edges (one per component) fall below it.
// The key of rank ~C*S/E among S evenly spaced samples of the live list.
// `dev` holds S keys of device scratch.
static ce_status split_pivot(const uint64_t *key, int64_t E, int64_t C, uint64_t *dev, hipStream_t s,
                             uint64_t *pivot) {
  uint64_t *h = pinned_scratch();
  if (!h) {
    set_error("hipHostMalloc of the readback buffer failed");
    return CE_EDEVICE;
  }
  uint64_t *hs = h + 128;  // bytes 1024 .. 3071 of the page
  CE_LAUNCH(k_sample_keys, dim3(1), dim3(B), 0, s, E, key, SPLIT_SAMPLES, dev);
  CE_HIP(hipGetLastError());
  CE_HIP(hipMemcpyAsync(hs, dev, sizeof(uint64_t) * SPLIT_SAMPLES, hipMemcpyDeviceToHost, s));
  CE_HIP(hipStreamSynchronize(s));
  std::sort(hs, hs + SPLIT_SAMPLES);
  int64_t q = (int64_t)((unsigned __int128)SPLIT_SAMPLES * (uint64_t)C / (uint64_t)E);
  if (q > SPLIT_SAMPLES - 1) q = SPLIT_SAMPLES - 1;
  *pivot = hs[q];
  return CE_OK;
}

// pointer jumping until every hooked component points at its final root
static ce_status jump_all(uint32_t *&act, uint32_t *&act2, uint64_t nact, uint32_t *hook, Bufs &b, hipStream_t s) {
  for (int it = 0; nact > 0; it++) {
    if (it > 64) {
      set_error("Boruvka pointer jumping did not converge");
      return CE_EDEVICE;
    }
    CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[5], (uint64_t)0);
    CE_LAUNCH(k_bv_jump, dim3(tiles_for((int64_t)nact)), dim3(B), 0, s, act, (int64_t)nact, hook, act2,
              (unsigned long long *)&b.hdr[5]);
    CE_HIP(hipGetLastError());
    CE_TRY(read_u64(&b.hdr[5], &nact, 1, s));
    uint32_t *t = act; act = act2; act2 = t;
  }
  return CE_OK;
}

ce_status stage_boruvka(Bufs &b, Ws &ws, hipStream_t s) {
  const int64_t n = b.n, n2 = b.slots;
  size_t m0 = ws.mark();
  uint32_t *hook = ws.alloc<uint32_t>(n);
  uint32_t *bidx = ws.alloc<uint32_t>(n);
  uint32_t *flags = ws.alloc<uint32_t>(n + 1);
  uint32_t *newid = ws.alloc<uint32_t>(n + 1);
  uint32_t *act = ws.alloc<uint32_t>(n);
  uint32_t *act2 = ws.alloc<uint32_t>(n);
  uint64_t *key[2];
  uint32_t *eu[2], *ev[2], *es[2];
  for (int k = 0; k < 2; k++) {
    key[k] = ws.alloc<uint64_t>(n2);
    eu[k] = ws.alloc<uint32_t>(n2);
    ev[k] = ws.alloc<uint32_t>(n2);
    es[k] = ws.alloc<uint32_t>(n2);
  }
  CE_WS_CHECK(ws);
  uint32_t *rankof = b.rankof;  // kept for writing the per-record outputs in input order
  CE_LAUNCH(k_rankof, dim3(grid_for(n, B)), dim3(B), 0, s, b.perm, n, rankof);
  uint64_t *best = b.best;  // seeded for round 1 while the skeleton was emitted
  unsigned long long *cnt = (unsigned long long *)&b.hdr[4];
  CE_LAUNCH(k_fill_u8, dim3(grid_for(n2, B)), dim3(B), 0, s, b.msf_flag, n2, (uint8_t)0);
  int64_t E = 0, C = 0;
  int rounds = 0;
  uint64_t nact = 0;
  uint64_t hv[2];
  // live edges of the current round (input) and the buffer the contraction writes
  const uint64_t *ik = key[0];
  const uint32_t *iu = eu[0], *iv = ev[0], *is = es[0];
  int ob = 1;
  bool seeded = false;
  if (b.flat) {
    // causal and hypergraph skeleton rows can share a head, so every round,
    // the first included, runs on the edge-list form with records as
    // components; the first reads the skeleton rows in place (slot = row)
    ik = b.skel_key;
    iu = b.skel_tail;
    iv = b.skel_tid;
    is = nullptr;
    ob = 0;
    seeded = true;
    E = b.S;
    C = n;
  } else {
    // round 1 on records
    CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[4], (uint64_t)0);
    CE_LAUNCH(k_bv_hook_first, dim3(tiles_for(n)), dim3(B), 0, s, n, best, b.skel_key, b.skel_tail, rankof,
              b.idbits, hook, b.msf_flag, act, cnt);
    CE_HIP(hipGetLastError());
    CE_TRY(read_u64(&b.hdr[4], &nact, 1, s));
    CE_TRY(jump_all(act, act2, nact, hook, b, s));
    CE_LAUNCH(k_root_flags, dim3(grid_for(n, B)), dim3(B), 0, s, n, hook, best, flags);
    CE_HIP(hipGetLastError());
    CE_TRY(scan_exclusive_u32(flags, newid, n, ws, s));
    CE_LAUNCH(k_final_ids, dim3(grid_for(n, B)), dim3(B), 0, s, n, hook, newid, flags);
    CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[4], (uint64_t)0);
    CE_LAUNCH(k_contract_first, dim3(tiles_for(n2)), dim3(B), 0, s, n2, b.skel_key, b.skel_tail, flags,
              key[0], eu[0], ev[0], es[0], cnt);
    CE_HIP(hipGetLastError());
    CE_TRY(read_count_and_total(&b.hdr[4], newid + n, hv, s));
    E = (int64_t)hv[0];
    C = (int64_t)hv[1];
    if (E > n2 || C > n) {
      set_error("internal: contracted graph larger than its input");
      return CE_EDEVICE;
    }
    rounds = 1;
  }
  // Filter split. When live edges far outnumber components, most of them run
  // between components that later rounds merge anyway, and every round would
  // scan them again. So the list is split at a pivot key: Borůvka runs on the
  // light edges (key below the pivot) alone until none is left, then the heavy
  // ones are contracted once and rounds go on with the survivors. Keys are
  // unique, so the forest is the same: a light edge outside the light forest
  // is the largest on a cycle of light edges, and contracting the light forest
  // keeps every heavy edge's cycles. During the light phase components keep
  // the ids they had at the split (no renumbering) and rootof, in newid, maps
  // each of them to its current root; the heavy edges wait at the back of the
  // output lists of buffer hb.
  const int64_t split_min = split_min_edges();
  bool light = false, first_light = false;
  int hb = 0;
  int64_t Eh = 0;
  uint32_t *rootof = newid;
  while (E > 0) {
    // (bidx, n words, holds the pivot samples)
    if (!light && !seeded && E >= split_min && E > 2 * C && n * 4 >= SPLIT_SAMPLES * 8) {
      uint64_t pivot = 0;
      CE_TRY(split_pivot(ik, E, C, (uint64_t *)bidx, s, &pivot));
      CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[4], (uint64_t)0);
      CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[5], (uint64_t)0);
      CE_LAUNCH(k_split, dim3(tiles_for(E)), dim3(B), 0, s, E, ik, iu, iv, is, pivot, n2, key[ob], eu[ob], ev[ob],
                es[ob], cnt, (unsigned long long *)&b.hdr[5]);
      CE_HIP(hipGetLastError());
      CE_TRY(read_u64(&b.hdr[4], hv, 2, s));
      if ((int64_t)(hv[0] + hv[1]) != E) {
        set_error("internal: filter split lost edges");
        return CE_EDEVICE;
      }
      const int64_t El = (int64_t)hv[0];
      Eh = (int64_t)hv[1];
      const int64_t off = El > 0 ? 0 : n2 - Eh;  // no light edge: the heavy ones are the whole list
      ik = key[ob] + off;
      iu = eu[ob] + off;
      iv = ev[ob] + off;
      is = es[ob] + off;
      if (El > 0) {
        light = first_light = true;
        hb = ob;
        E = El;
      }
      ob = 1 - ob;
    }
    if (++rounds > 64) {
      set_error("Boruvka did not converge");
      return CE_EDEVICE;
    }
    if (!seeded) {
      CE_LAUNCH(k_fill_u64, dim3(grid_for(C, B)), dim3(B), 0, s, best, C, NONE64);
      CE_LAUNCH(k_bv_min, dim3(tiles_for(E)), dim3(B), 0, s, E, ik, iu, iv, best);
    }
    seeded = false;
    CE_LAUNCH(k_bv_pick, dim3(grid_for(E, B)), dim3(B), 0, s, E, ik, iu, iv, best, bidx);
    CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[4], (uint64_t)0);
    CE_LAUNCH(k_bv_hook, dim3(tiles_for(C)), dim3(B), 0, s, C, best, bidx, iu, iv, is, hook, b.msf_flag, act, cnt);
    CE_HIP(hipGetLastError());
    CE_TRY(read_u64(&b.hdr[4], &nact, 1, s));
    CE_TRY(jump_all(act, act2, nact, hook, b, s));
    if (light) {
      // ids stay; the edges' endpoints are this round's roots, hook gives their new ones
      CE_LAUNCH(k_compose_roots, dim3(grid_for(C, B)), dim3(B), 0, s, C, hook, rootof, first_light);
      first_light = false;
      CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[4], (uint64_t)0);
      CE_LAUNCH(k_contract, dim3(tiles_for(E)), dim3(B), 0, s, E, ik, iu, iv, is, hook, key[ob], eu[ob], ev[ob],
                es[ob], cnt);
      CE_HIP(hipGetLastError());
      CE_TRY(read_u64(&b.hdr[4], hv, 1, s));
      if ((int64_t)hv[0] > E) {
        set_error("internal: contracted graph larger than its input");
        return CE_EDEVICE;
      }
      E = (int64_t)hv[0];
    } else {
      CE_LAUNCH(k_root_flags, dim3(grid_for(C, B)), dim3(B), 0, s, C, hook, best, flags);
      CE_HIP(hipGetLastError());
      CE_TRY(scan_exclusive_u32(flags, newid, C, ws, s));
      CE_LAUNCH(k_final_ids, dim3(grid_for(C, B)), dim3(B), 0, s, C, hook, newid, flags);
      CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[4], (uint64_t)0);
      CE_LAUNCH(k_contract, dim3(tiles_for(E)), dim3(B), 0, s, E, ik, iu, iv, is, flags, key[ob], eu[ob], ev[ob],
                es[ob], cnt);
      CE_HIP(hipGetLastError());
      CE_TRY(read_count_and_total(&b.hdr[4], newid + C, hv, s));
      if ((int64_t)hv[0] > E || (int64_t)hv[1] > C) {
        set_error("internal: contracted graph larger than its input");
        return CE_EDEVICE;
      }
      E = (int64_t)hv[0];
      C = (int64_t)hv[1];
    }
    ik = key[ob];
    iu = eu[ob];
    iv = ev[ob];
    is = es[ob];
    ob = 1 - ob;
    if (light && E == 0) {
      // light phase done: the heavy edges between different current roots
      // go on (ids of the split, not renumbered; the next round renumbers)
      const int64_t off = n2 - Eh;
      const int to = 1 - hb;
      CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[4], (uint64_t)0);
      CE_LAUNCH(k_contract, dim3(tiles_for(Eh)), dim3(B), 0, s, Eh, key[hb] + off, eu[hb] + off, ev[hb] + off,
                es[hb] + off, rootof, key[to], eu[to], ev[to], es[to], cnt);
      CE_HIP(hipGetLastError());
      CE_TRY(read_u64(&b.hdr[4], hv, 1, s));
      if ((int64_t)hv[0] > Eh) {
        set_error("internal: contracted graph larger than its input");
        return CE_EDEVICE;
      }
      E = (int64_t)hv[0];
      ik = key[to];
      iu = eu[to];
      iv = ev[to];
      is = es[to];
      ob = hb;
      light = false;
    }
  }
  ws.release(m0);
  return CE_OK;
}

// rows with key < limit (rows are sorted, so they are a prefix): one binary search
__global__ void k_prefix_below(const uint64_t *key, int64_t m, uint64_t limit, uint64_t *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (key[mid] < limit) lo = mid + 1;
    else hi = mid;
  }
  *out = (uint64_t)lo;
}

// Time-filtered line graph (Sec. 5.1): only edges with w <= max_dt. The
// filtered skeleton has the filtered line graph's components at every
// threshold up to max_dt (Thm 3), and Kruskal takes edges in key order, so
// its forest is the prefix of the sorted MSF with w <= max_dt.
ce_status stage_time_filter(Bufs &b, int64_t max_dt, hipStream_t s, int64_t *m) {
  if (*m <= 0 || max_dt < 0) return CE_OK;
  const unsigned __int128 lim = ((unsigned __int128)max_dt + 1) << b.wshift;
  if (lim > (unsigned __int128)NONE64) return CE_OK;  // every key is below it: no row is longer
  const uint64_t limit = (uint64_t)lim;
  CE_LAUNCH(k_prefix_below, dim3(1), dim3(64), 0, s, b.msf_key, *m, limit, &b.hdr[6]);
  CE_HIP(hipGetLastError());
  uint64_t k = 0;
  CE_TRY(read_u64(&b.hdr[6], &k, 1, s));
  if ((int64_t)k > *m) {
    set_error("internal: time filter");
    return CE_EDEVICE;
  }
  *m = (int64_t)k;
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
  const int64_t n = b.n, n2 = b.slots;
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
  // gather into the buffer pair from which an odd or even number of radix
  // passes ends in msf_key / msf_val, so no copy follows the sort
  const int passes = b.keybits > 8 ? (b.keybits + 7) / 8 : 1;
  uint64_t *gk = (passes & 1) ? key_alt : b.msf_key, *gv = (passes & 1) ? val_alt : b.msf_val;
  uint64_t *ok = (passes & 1) ? b.msf_key : key_alt, *ov = (passes & 1) ? b.msf_val : val_alt;
  if (m > 0 && b.flat)
    CE_LAUNCH(k_msf_gather_causal, dim3(grid_for((int64_t)m, B)), dim3(B), 0, s, list, (int64_t)m, b.skel_key,
              b.skel_tail, b.skel_tid, gk, gv);
  else if (m > 0)
    CE_LAUNCH(k_msf_gather, dim3(grid_for((int64_t)m, B)), dim3(B), 0, s, list, (int64_t)m, b.skel_key,
              b.skel_tail, gk, gv);
  bool alt = false;
  CE_TRY((radix_sort_pairs<uint64_t, uint64_t>(gk, gv, ok, ov, (int64_t)m, 0, b.keybits, false, &alt, ws, s)));
  if (m > 0 && (alt ? ok : gk) != b.msf_key) {  // (not reached: the pass count is as computed)
    CE_HIP(hipMemcpyAsync(b.msf_key, alt ? ok : gk, sizeof(uint64_t) * m, hipMemcpyDeviceToDevice, s));
    CE_HIP(hipMemcpyAsync(b.msf_val, alt ? ov : gv, sizeof(uint64_t) * m, hipMemcpyDeviceToDevice, s));
  }
  ws.release(m0);
  *m_out = (int64_t)m;
  return CE_OK;
}

}  // namespace ce
