// Stages A1-A6: validate, group-and-sort by (vertex, time), emit the path
// skeleton, Boruvka minimum spanning forest, sort the MSF by canonical key.
//
// Grouping (the per-vertex incidence lists of Alg. 3, time-sorted as in Alg. 2): the records
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
  for (int i = threadIdx.x; i < kHdrWords; i += blockDim.x) hdr[i] = i == H_TMIN ? NONE64 : 0;
}

// After validation: a time span wider than the plan's tbits bits is an error too (the keys would not fit).
__global__ void k_check_span(uint64_t *hdr, int64_t n, int tbits) {
  if (threadIdx.x != 0 || n == 0) return;
  const uint64_t span = hdr[H_TMAX] - hdr[H_TMIN];
  if (tbits < 64 && (span >> tbits) != 0) hdr[H_STATUS] |= 8;
}

__device__ inline int64_t tmin_of(const uint64_t *hdr) { return (int64_t)(hdr[H_TMIN] ^ (uint64_t(1) << 63)); }

// the time sort carries (id, src, dst, graph) along, so grouping needs no
// gathers; vertex ids become global (graph offset + local id)
__global__ __launch_bounds__(B) void k_tkeys(const int64_t *t, const int32_t *src, const int32_t *dst, int64_t n,
                                             const int64_t *eoff, const int64_t *voff, int64_t G,
                                             const uint64_t *hdr, uint64_t *keys, uint4 *vals) {
  const int64_t tmin = tmin_of(hdr);
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
                                                    int64_t n, const uint64_t *hdr, uint64_t *keys, uint64_t *vals) {
  const int64_t tmin = tmin_of(hdr);
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
// (an input that failed validation gets an empty skeleton, so everything after
// it runs on n isolated records and stays in bounds whatever the input held)
__global__ __launch_bounds__(B) void k_skel_tails(const uint32_t *ikey, const uint32_t *ival, int64_t n2,
                                                  const uint64_t *hdr, uint32_t *skel_tail) {
  const bool bad = hdr[H_STATUS] != 0;
  for (int64_t k = (int64_t)blockIdx.x * B + threadIdx.x; k < n2; k += (int64_t)gridDim.x * B) {
    uint32_t slot = ival[k];
    skel_tail[slot] = (!bad && k > 0 && ikey[k - 1] == ikey[k]) ? (ival[k - 1] >> 1) : NONE32;
  }
}

// Also seeds the first Boruvka round: every record starts as its own
// component, so each edge offers its key to both of its records.
// The low bit orders the two edges of a head by descending tail id; it only
// decides their order when they have the same weight (else w does), so the
// tails' ids are read only then.
// Weight ranks (wraw set): the keys get their tie bits only, the weights go
// to wraw, and the seeding waits for the ranks.
__global__ __launch_bounds__(B) void k_skel_keys(uint32_t *skel_tail, const uint64_t *ts, const uint32_t *perm,
                                                 int64_t n, int idbits, uint64_t *skel_key, uint64_t *best,
                                                 uint64_t *wraw) {
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
    if (wraw) {
      skel_key[2 * h] = t0 != NONE32 ? (hid << 1) | b0 : NONE64;
      skel_key[2 * h + 1] = t1 != NONE32 ? (hid << 1) | b1 : NONE64;
      wraw[2 * h] = w0;
      wraw[2 * h + 1] = w1;
      continue;
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
//
// Every count that steers the rounds (live edges E, components C, the phase of
// a filter split) lives in the call's control block, and every round kernel
// reads it when it starts. The host enqueues a fixed number of rounds, enough
// for any input of n records (live components at least halve per round); the
// rounds after the forest is complete find E = 0 and return at once. The last
// block of a round's final kernel advances the state (a ticket counter tells
// it that every other block is done).

// Boruvka state, words H_BV + k of the control block
enum : int {
  BV_E = 0,        // live edges of the current list
  BV_C = 1,        // components (ids 0..C-1)
  BV_PHASE = 2,    // 0 plain rounds, 1 light rounds of a filter split
  BV_IN = 3,       // the list: edge buffer 0 or 1, or 2 = the skeleton rows themselves
  BV_OFF = 4,      // its first entry in that buffer
  BV_HB = 5,       // buffer holding the heavy edges of a split at its back
  BV_EH = 6,       // heavy edges
  BV_SPLIT = 7,    // this round starts with a split at BV_PIVOT
  BV_PIVOT = 8,
  BV_FIRSTL = 9,   // first light round (the root map starts as the identity)
  BV_HEAVY = 10,   // the light edges are gone: contract the heavy ones next
  BV_SEEDED = 11,  // the minima of this round were seeded while the skeleton was emitted
  BV_SPLITDONE = 12,  // at most one split per call (it bounds the rounds)
  // gates: the live counts of the kernels of one phase, 0 while they have nothing to do
  BV_EN = 13, BV_CN = 14, BV_EL = 15, BV_CL = 16, BV_CG = 17, BV_EHG = 18,
  BV_TICKET = 19,  // last-block ticket, then two list counters
  BV_CNT1 = 20, BV_CNT2 = 21,
  BV_WORDS = 24
};

struct EdgeLists {
  uint64_t *key[3];
  uint32_t *u[3], *v[3], *s[3];  // s[2] == nullptr: the slot of a skeleton row is its index
  int64_t cap;                   // entries of buffers 0 and 1
};

__device__ inline uint64_t ld_coherent(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// the live list of the current round
struct Live {
  const uint64_t *key;
  const uint32_t *u, *v, *s;
  int64_t E;
};
__device__ inline Live live_list(const EdgeLists &L, const uint64_t *bv) {
  const int in = (int)bv[BV_IN];
  const int64_t off = (int64_t)bv[BV_OFF];
  return Live{L.key[in] + off, L.u[in] + off, L.v[in] + off, L.s[in] ? L.s[in] + off : nullptr, (int64_t)bv[BV_E]};
}
__device__ inline int out_buffer(const uint64_t *bv) {
  const int in = (int)bv[BV_IN];
  return in == 2 ? 0 : 1 - in;
}

// gates from the state (run by the block that last changed it)
__device__ inline void bv_publish(uint64_t *bv) {
  const bool light = bv[BV_PHASE] == 1, live = bv[BV_E] > 0;
  bv[BV_EN] = light ? 0 : bv[BV_E];
  bv[BV_CN] = (!light && live) ? bv[BV_C] : 0;
  bv[BV_EL] = light ? bv[BV_E] : 0;
  bv[BV_CL] = (light && live) ? bv[BV_C] : 0;
  bv[BV_CG] = live ? bv[BV_C] : 0;
  bv[BV_EHG] = bv[BV_HEAVY] ? bv[BV_EH] : 0;
}

// true in exactly one block, the last to arrive; all blocks must call it
__device__ inline bool last_block(uint64_t *ticket) {
  __shared__ bool last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned long long t = atomicAdd((unsigned long long *)ticket, 1ull);
    last = t == (unsigned long long)(gridDim.x - 1);
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

// first round, on records: hook each record onto the record across its
// minimum edge; of a mutual pair the smaller id stays; the hooking edge joins
// the forest. flags[c] = 1 for roots that have an edge (they get dense ids).
__global__ __launch_bounds__(B) void k_bv_hook_first(int64_t n, const uint64_t *best, const uint64_t *skel_key,
                                                     const uint32_t *skel_tail, const uint32_t *rankof, int idbits,
                                                     uint32_t *hook, uint8_t *msf_flag, uint32_t *flags) {
  for (int64_t c = (int64_t)blockIdx.x * B + threadIdx.x; c < n; c += (int64_t)gridDim.x * B) {
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
      }
    }
    hook[c] = to;
    flags[c] = (to == (uint32_t)c && bk != NONE64) ? 1u : 0u;
  }
}

// later rounds, on the contracted graph
__global__ __launch_bounds__(B) void k_bv_hook(EdgeLists L, const uint64_t *bv, const uint64_t *best,
                                               const uint32_t *bidx, uint32_t *hook, uint8_t *msf_flag,
                                               uint32_t *flags) {
  const Live lv = live_list(L, bv);
  const int64_t C = (int64_t)bv[BV_C];
  if (lv.E == 0) return;
  for (int64_t c = (int64_t)blockIdx.x * B + threadIdx.x; c < C; c += (int64_t)gridDim.x * B) {
    uint32_t to = (uint32_t)c;
    const uint64_t bk = best[c];
    if (bk != NONE64) {
      const uint32_t i = bidx[c];
      const uint32_t o = lv.u[i] == (uint32_t)c ? lv.v[i] : lv.u[i];
      if (!(best[o] == bk && (uint32_t)c < o)) {
        to = o;
        msf_flag[lv.s ? lv.s[i] : i] = 1;
      }
    }
    hook[c] = to;
    flags[c] = (to == (uint32_t)c && bk != NONE64) ? 1u : 0u;
  }
}

// Every component to its final root, in two passes. The first walks from
// every component and halves the path it follows (each store moves a link to
// a grandparent), so long hook chains shrink as in pointer jumping. Walks only
// ever store ancestors, so a stale link seen by another walk is still an
// ancestor and every walk ends at the root (hooks form a forest: keys are
// unique, and of a mutual pair only one side hooks). But a halving store can
// land after the owner of that entry stored its root, and put a lower
// ancestor back; so the second pass walks again, read only, and each
// component stores its own root alone. A walk longer than any forest allows
// marks the call failed and stops.
constexpr uint32_t MAX_WALK = 1u << 26;
__global__ __launch_bounds__(B) void k_bv_compress(Cnt C, uint32_t *hook, uint64_t *hdr) {
  const int64_t nc = C.get();
  for (int64_t c = (int64_t)blockIdx.x * B + threadIdx.x; c < nc; c += (int64_t)gridDim.x * B) {
    uint32_t x = hook[c];
    if (x == (uint32_t)c) continue;
    for (uint32_t steps = 0;; steps++) {
      const uint32_t p = __hip_atomic_load(&hook[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (p == x) break;
      const uint32_t gp = __hip_atomic_load(&hook[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (gp != p) __hip_atomic_store(&hook[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      x = gp;
      if (steps > MAX_WALK) {
        atomicOr((unsigned long long *)&hdr[H_STATUS], 16ull);
        break;
      }
    }
  }
}
__global__ __launch_bounds__(B) void k_bv_roots(Cnt C, uint32_t *hook, uint64_t *hdr) {
  const int64_t nc = C.get();
  for (int64_t c = (int64_t)blockIdx.x * B + threadIdx.x; c < nc; c += (int64_t)gridDim.x * B) {
    uint32_t x = __hip_atomic_load(&hook[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (x == (uint32_t)c) continue;
    for (uint32_t steps = 0;; steps++) {
      const uint32_t p = __hip_atomic_load(&hook[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (p == x) break;
      x = p;
      if (steps > MAX_WALK) {
        atomicOr((unsigned long long *)&hdr[H_STATUS], 16ull);
        break;
      }
    }
    __hip_atomic_store(&hook[c], x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// dense id of every component's final root (contraction reads one id per
// endpoint); the minima of the next round start empty
__global__ __launch_bounds__(B) void k_final_ids(Cnt C, const uint32_t *hook, const uint32_t *newid, uint32_t *fin,
                                                 uint64_t *best) {
  const int64_t nc = C.get();
  const int64_t cn = nc > 0 ? (int64_t)newid[nc] : 0;
  for (int64_t c = (int64_t)blockIdx.x * B + threadIdx.x; c < nc; c += (int64_t)gridDim.x * B) {
    fin[c] = newid[hook[c]];
    if (c < cn) best[c] = NONE64;
  }
}

// first contraction: skeleton slots between different final roots, endpoints renamed to dense ids
__global__ __launch_bounds__(B) void k_contract_first(int64_t n, const uint64_t *skel_key, const uint32_t *skel_tail,
                                                      const uint32_t *fin, const uint32_t *newid, EdgeLists L,
                                                      uint64_t *bv) {
  const int64_t n2 = 2 * n;
  unsigned long long *cnt = (unsigned long long *)&bv[BV_CNT1];
  const int ct = tile_items(n2);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < n2; tile += gridDim.x) {
    bool keep[CT];
    uint32_t pos[CT], nu[CT], nv[CT];
    uint64_t kk[CT];
    const int64_t base = tile * (B * ct) + threadIdx.x, end = tile_end(n2, tile, B * ct);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      const int64_t e = base + (int64_t)k * B;
      keep[k] = false;
      kk[k] = NONE64;
      nu[k] = nv[k] = 0;
      if (e >= end) continue;
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
      L.key[0][p] = kk[k];
      L.u[0][p] = nu[k];
      L.v[0][p] = nv[k];
      L.s[0][p] = (uint32_t)(base + (int64_t)k * B);
    }
  }
  if (last_block(&bv[BV_TICKET])) {
    if (threadIdx.x == 0) {
      bv[BV_E] = ld_coherent(&bv[BV_CNT1]);
      bv[BV_C] = newid[n];
      bv[BV_IN] = 0;
      bv[BV_OFF] = 0;
      bv[BV_PHASE] = 0;
      bv[BV_SEEDED] = 0;
      bv[BV_CNT1] = 0;
      bv[BV_TICKET] = 0;
      bv_publish(bv);
    }
  }
}

// Contraction of the live list (gated count E) with the map f: edges between
// different f-images go to the front of the output buffer, renamed. The last
// block advances the state: `mode` 0 = plain round (new ids from the scan),
// 1 = light round (ids stay), 2 = the heavy edges after the light phase.
__global__ __launch_bounds__(B) void k_contract(EdgeLists L, uint64_t *bv, const uint64_t *gate,
                                                const uint32_t *fmap, const uint32_t *newid, int mode) {
  const int64_t E = (int64_t)*gate;
  if (E == 0) return;  // uniform: every block returns, and the state does not change
  const int in = mode == 2 ? (int)bv[BV_HB] : (int)bv[BV_IN];
  const int64_t off = mode == 2 ? L.cap - (int64_t)bv[BV_EH] : (int64_t)bv[BV_OFF];
  const int ob = mode == 2 ? 1 - in : out_buffer(bv);
  const uint64_t *key = L.key[in] + off;
  const uint32_t *eu = L.u[in] + off, *ev = L.v[in] + off;
  const uint32_t *es = L.s[in] ? L.s[in] + off : nullptr;
  unsigned long long *cnt = (unsigned long long *)&bv[BV_CNT1];
  const int ct = tile_items(E);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < E; tile += gridDim.x) {
    bool keep[CT];
    uint32_t pos[CT], nu[CT], nv[CT];
    const int64_t base = tile * (B * ct) + threadIdx.x, end = tile_end(E, tile, B * ct);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      const int64_t i = base + (int64_t)k * B;
      keep[k] = false;
      nu[k] = nv[k] = 0;
      if (i >= end) continue;
      const uint32_t fu = fmap[eu[i]], fv = fmap[ev[i]];
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
      L.key[ob][p] = key[i];
      L.u[ob][p] = nu[k];
      L.v[ob][p] = nv[k];
      L.s[ob][p] = es ? es[i] : (uint32_t)i;
    }
  }
  if (last_block(&bv[BV_TICKET])) {
    if (threadIdx.x == 0) {
      const uint64_t c = ld_coherent(&bv[BV_CNT1]);
      if (mode == 0) bv[BV_C] = newid[bv[BV_C]];
      bv[BV_E] = c;
      bv[BV_IN] = (uint64_t)ob;
      bv[BV_OFF] = 0;
      bv[BV_SEEDED] = 0;
      if (mode == 1) {
        bv[BV_FIRSTL] = 0;
        if (c == 0) bv[BV_HEAVY] = 1;  // light edges used up: the heavy ones are contracted next
      }
      if (mode == 2) {
        bv[BV_PHASE] = 0;
        bv[BV_HEAVY] = 0;
      }
      bv[BV_CNT1] = 0;
      bv[BV_TICKET] = 0;
      bv_publish(bv);
    }
  }
}

// Filter split (Filter-Kruskal applied to Borůvka). A round may start with a
// split when live edges are at least `split_min` and more than twice the
// components: the pivot is the key of rank ~C*S/E among S evenly spaced
// samples of the list (sorted in LDS), so about one light edge per component.
constexpr int SPLIT_SAMPLES = 256;
__global__ __launch_bounds__(SPLIT_SAMPLES) void k_split_prep(EdgeLists L, uint64_t *bv, int64_t split_min) {
  __shared__ uint64_t sk[SPLIT_SAMPLES];
  const Live lv = live_list(L, bv);
  const int64_t C = (int64_t)bv[BV_C];
  const bool go = bv[BV_PHASE] == 0 && bv[BV_SEEDED] == 0 && bv[BV_SPLITDONE] == 0 && lv.E >= split_min &&
                  lv.E > 2 * C;
  if (!go) {
    if (threadIdx.x == 0) bv[BV_SPLIT] = 0;
    return;
  }
  const int i = threadIdx.x;
  sk[i] = lv.key[(int64_t)((unsigned __int128)i * (uint64_t)lv.E / SPLIT_SAMPLES)];
  __syncthreads();
  for (int k = 2; k <= SPLIT_SAMPLES; k <<= 1) {  // bitonic sort, ascending
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int p = i ^ j;
      if (p > i) {
        const uint64_t a = sk[i], b2 = sk[p];
        const bool up = (i & k) == 0;
        if ((a > b2) == up) { sk[i] = b2; sk[p] = a; }
      }
      __syncthreads();
    }
  }
  if (i == 0) {
    int64_t q = (int64_t)((unsigned __int128)SPLIT_SAMPLES * (uint64_t)C / (uint64_t)lv.E);
    if (q > SPLIT_SAMPLES - 1) q = SPLIT_SAMPLES - 1;
    bv[BV_PIVOT] = sk[q];
    bv[BV_SPLIT] = 1;
    bv[BV_CNT1] = 0;
    bv[BV_CNT2] = 0;
  }
}

// The live edges with key below the pivot go to the front of the output
// buffer, the others to its back, counted down from cap. Light and heavy
// together are E <= cap entries, so later contractions of the light part,
// which only shrink it, never reach the heavy part.
__global__ __launch_bounds__(B) void k_split(EdgeLists L, uint64_t *bv) {
  if (bv[BV_SPLIT] == 0) return;
  const Live lv = live_list(L, bv);
  const uint64_t pivot = bv[BV_PIVOT];
  const int ob = out_buffer(bv);
  const int64_t cap = L.cap;
  unsigned long long *nlight = (unsigned long long *)&bv[BV_CNT1];
  unsigned long long *nheavy = (unsigned long long *)&bv[BV_CNT2];
  const int ct = tile_items(lv.E);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < lv.E; tile += gridDim.x) {
    bool lt[CT], ge[CT];
    uint32_t pl[CT], ph[CT];
    uint64_t kk[CT];
    const int64_t base = tile * (B * ct) + threadIdx.x, end = tile_end(lv.E, tile, B * ct);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      const int64_t i = base + (int64_t)k * B;
      kk[k] = i < end ? lv.key[i] : 0;
      lt[k] = i < end && kk[k] < pivot;
      ge[k] = i < end && kk[k] >= pivot;
    }
    tile_positions(lt, pl, nlight);
    tile_positions(ge, ph, nheavy);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      if (!lt[k] && !ge[k]) continue;
      const int64_t i = base + (int64_t)k * B;
      const int64_t p = lt[k] ? (int64_t)pl[k] : cap - 1 - (int64_t)ph[k];
      L.key[ob][p] = kk[k];
      L.u[ob][p] = lv.u[i];
      L.v[ob][p] = lv.v[i];
      L.s[ob][p] = lv.s ? lv.s[i] : (uint32_t)i;
    }
  }
  if (last_block(&bv[BV_TICKET])) {
    if (threadIdx.x == 0) {
      const uint64_t el = ld_coherent(&bv[BV_CNT1]), eh = ld_coherent(&bv[BV_CNT2]);
      bv[BV_IN] = (uint64_t)ob;
      if (el > 0) {  // light rounds first; ids stay, the root map starts as the identity
        bv[BV_PHASE] = 1;
        bv[BV_FIRSTL] = 1;
        bv[BV_HB] = (uint64_t)ob;
        bv[BV_EH] = eh;
        bv[BV_E] = el;
        bv[BV_OFF] = 0;
      } else {  // no light edge: the heavy ones are the whole list
        bv[BV_E] = eh;
        bv[BV_OFF] = (uint64_t)(cap - (int64_t)eh);
      }
      bv[BV_SPLIT] = 0;
      bv[BV_SPLITDONE] = 1;
      bv[BV_CNT1] = 0;
      bv[BV_CNT2] = 0;
      bv[BV_TICKET] = 0;
      bv_publish(bv);
    }
  }
}

// light rounds: the root (in this round's hooks) of every component of the
// split; the minima of the next round start empty
__global__ __launch_bounds__(B) void k_compose_roots(Cnt C, const uint64_t *bv, const uint32_t *hook,
                                                     uint32_t *rootof, uint64_t *best) {
  const int64_t nc = C.get();
  const bool first = bv[BV_FIRSTL] != 0;
  for (int64_t c = (int64_t)blockIdx.x * B + threadIdx.x; c < nc; c += (int64_t)gridDim.x * B) {
    rootof[c] = hook[first ? (uint32_t)c : rootof[c]];
    best[c] = NONE64;
  }
}

// per component, the minimum key over its live edges. A tile of up to 4096 edges
// first takes per-component minima in an LDS hash (late rounds send most
// edges to a few big components), then one atomicMin per component per tile.
constexpr int MHS = 512;
__global__ __launch_bounds__(B) void k_bv_min(EdgeLists L, const uint64_t *bv, uint64_t *best) {
  if (bv[BV_SEEDED]) return;  // seeded while the skeleton was emitted
  const Live lv = live_list(L, bv);
  __shared__ uint32_t hk[MHS];
  __shared__ unsigned long long hv[MHS];
  const int ct = tile_items(lv.E);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < lv.E; tile += gridDim.x) {
    for (int i = threadIdx.x; i < MHS; i += B) { hk[i] = NONE32; hv[i] = NONE64; }
    __syncthreads();
    const int64_t tbase = tile * (B * ct);
    for (int k = 0; k < ct; k++) {
      const int64_t i = tbase + (int64_t)k * B + threadIdx.x;
      const bool act = i < lv.E;
      const unsigned long long kv = act ? lv.key[i] : NONE64;
      const uint32_t cu = act ? lv.u[i] : 0u, cv = act ? lv.v[i] : 0u;
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
    __syncthreads();
  }
}

// the edge index holding each component's minimum (keys are unique)
__global__ __launch_bounds__(B) void k_bv_pick(EdgeLists L, const uint64_t *bv, const uint64_t *best,
                                               uint32_t *bidx) {
  const Live lv = live_list(L, bv);
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < lv.E; i += (int64_t)gridDim.x * B) {
    const uint64_t k = lv.key[i];
    const uint32_t a = lv.u[i], b = lv.v[i];
    if (best[a] == k) bidx[a] = (uint32_t)i;
    if (best[b] == k) bidx[b] = (uint32_t)i;
  }
}

// state of a flat skeleton's first round: the rows themselves are the live
// list (S rows, counted on the device), records are the components, and the
// minima were seeded during emission
__global__ void k_bv_flat_init(uint64_t *bv, const uint64_t *rows, int64_t n) {
  if (threadIdx.x != 0) return;
  for (int k = 0; k < BV_WORDS; k++) bv[k] = 0;
  bv[BV_E] = *rows;
  bv[BV_C] = (uint64_t)n;
  bv[BV_IN] = 2;
  bv[BV_SEEDED] = 1;
  bv_publish(bv);
}

// after the last enqueued round every live edge must be gone (the round bound
// guarantees it); if not, the call fails instead of returning a partial forest
__global__ void k_bv_check(const uint64_t *bv, uint64_t *hdr) {
  if (threadIdx.x == 0 && (bv[BV_E] != 0 || bv[BV_HEAVY] != 0)) hdr[H_STATUS] |= 32;
}

__global__ __launch_bounds__(B) void k_msf_list(const uint8_t *flag, int64_t n2, uint32_t *out,
                                                unsigned long long *cnt) {
  const int ct = tile_items(n2);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < n2; tile += gridDim.x) {
    bool keep[CT];
    uint32_t vals[CT];
    const int64_t base = tile * (B * ct) + threadIdx.x, end = tile_end(n2, tile, B * ct);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      const int64_t e = base + (int64_t)k * B;
      keep[k] = e < end && flag[e];
      vals[k] = (uint32_t)e;
    }
    tile_append(keep, vals, out, cnt);
  }
}

// flat rows keep the head rank in skel_tid; the tail id comes from perm
__global__ __launch_bounds__(B) void k_msf_gather_causal(const uint32_t *list, Cnt mc, const uint64_t *skel_key,
                                                         const uint32_t *skel_tail, const uint32_t *skel_head,
                                                         uint64_t *okey, uint64_t *oval) {
  const int64_t m = mc.get();
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < m; i += (int64_t)gridDim.x * B) {
    uint32_t e = list[i];
    okey[i] = skel_key[e];
    oval[i] = (uint64_t)skel_tail[e] | ((uint64_t)skel_head[e] << 32);
  }
}

__global__ __launch_bounds__(B) void k_msf_gather(const uint32_t *list, Cnt mc, const uint64_t *skel_key,
                                                  const uint32_t *skel_tail, uint64_t *okey, uint64_t *oval) {
  const int64_t m = mc.get();
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < m; i += (int64_t)gridDim.x * B) {
    uint32_t e = list[i];
    okey[i] = skel_key[e];
    oval[i] = (uint64_t)skel_tail[e] | ((uint64_t)(e >> 1) << 32);
  }
}

__global__ void k_set_u64(uint64_t *p, uint64_t v) { *p = v; }

// a forest has at most n - 1 rows; more means the call failed (and the rows
// are dropped, so that later kernels stay in bounds)
__global__ void k_check_rows(uint64_t *hdr, int64_t n) {
  if (threadIdx.x == 0 && (int64_t)hdr[H_M] > (n > 1 ? n - 1 : 0)) {
    hdr[H_STATUS] |= 64;
    hdr[H_M] = 0;
  }
}

// rows with weight < limit (rows are sorted, so they are a prefix): one binary
// search; the prefix becomes the forest (the row count shrinks in place)
__global__ void k_prefix_below(const uint64_t *key, uint64_t *m, uint64_t limit) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t lo = 0, hi = (int64_t)*m;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (key[mid] < limit) lo = mid + 1;
    else hi = mid;
  }
  *m = (uint64_t)lo;
}

// ---------------------------------------------------------------- weight ranks
// When w << wshift does not fit the key word, the key's weight field holds the
// weight's rank among the distinct weights of the skeleton instead: ranks
// order exactly as the weights do, so every step that only compares keys is
// unchanged, and the weights themselves are read back from the times once the
// forest is known. Absent slots get the value 2^tbits, above every weight.
__global__ __launch_bounds__(B) void k_rank_absent(const uint64_t *skel_key, int64_t cnt, int tbits, uint64_t *wraw) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * B)
    if (skel_key[i] == NONE64) wraw[i] = uint64_t(1) << tbits;
}
// first position of every distinct present weight in sorted order
__global__ __launch_bounds__(B) void k_rank_flags(const uint64_t *w, int64_t cnt, int tbits, uint32_t *first) {
  const uint64_t absent = uint64_t(1) << tbits;
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * B)
    first[i] = w[i] != absent && (i == 0 || w[i] != w[i - 1]) ? 1u : 0u;
}
// rank = distinct weights before this one; the finished key is offered to both
// records' first Boruvka minimum (records start as their own components)
__global__ __launch_bounds__(B) void k_rank_apply(const uint64_t *w, const uint32_t *slot, const uint32_t *first,
                                                  const uint32_t *before, int64_t cnt, int tbits, int wshift, bool flat,
                                                  uint64_t *skel_key, const uint32_t *skel_tail,
                                                  const uint32_t *skel_tid, uint64_t *best) {
  const uint64_t absent = uint64_t(1) << tbits;
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * B) {
    if (w[i] == absent) continue;
    const uint32_t e = slot[i];
    const uint64_t rank = (uint64_t)(before[i] + first[i] - 1u);
    const uint64_t k = skel_key[e] | (rank << wshift);
    skel_key[e] = k;
    const uint32_t head = flat ? skel_tid[e] : e >> 1;
    atomicMin((unsigned long long *)&best[skel_tail[e]], (unsigned long long)k);
    atomicMin((unsigned long long *)&best[head], (unsigned long long)k);
  }
}
// sorted forest rows: the weight itself in place of the key (head minus tail time)
__global__ __launch_bounds__(B) void k_msf_weights(uint64_t *msf_key, const uint64_t *msf_val, const uint64_t *ts,
                                                   Cnt mc, int wshift, bool rank) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    const uint64_t v = msf_val[j];
    msf_key[j] = rank ? ts[v >> 32] - ts[(uint32_t)v] : msf_key[j] >> wshift;
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

// Enqueues validation: error bits, min and max time into the control block.
ce_status stage_validate(const int32_t *src, const int32_t *dst, const int64_t *t, Bufs &b, hipStream_t s) {
  CE_LAUNCH(k_init_hdr, dim3(1), dim3(64), 0, s, b.hdr);
  CE_HIP(hipGetLastError());
  if (b.n > 0) {
    CE_LAUNCH(k_validate, dim3(grid_for(b.n, B, 4096)), dim3(B), 0, s, src, dst, t, b.n, b.eoff, b.voff, b.G,
              b.hdr);
    CE_HIP(hipGetLastError());
  }
  return CE_OK;
}

// After the plan's key width is known: a wider time span is an error as well.
ce_status stage_check_span(Bufs &b, hipStream_t s) {
  CE_LAUNCH(k_check_span, dim3(1), dim3(64), 0, s, b.hdr, b.n, b.tbits);
  CE_HIP(hipGetLastError());
  return CE_OK;
}

// The validation words (error bits, min t, max t) on the host: one read back.
ce_status read_validation(Bufs &b, hipStream_t s, uint64_t *flags, int64_t *tmin, int64_t *tmax) {
  uint64_t h[3];
  CE_TRY(read_u64(b.hdr, h, 3, s));
  *flags = h[0];
  *tmin = (int64_t)(h[1] ^ (uint64_t(1) << 63));
  *tmax = (int64_t)(h[2] ^ (uint64_t(1) << 63));
  return CE_OK;
}

bool choose_key_layout(Bufs &b, int64_t rows) {
  // CE_WEIGHT_RANKS=1 (read on every call) ranks the weights even when they fit
  const char *e = getenv("CE_WEIGHT_RANKS");
  const bool force = e && atoi(e) == 1;
  if (!force && b.tbits + b.wshift <= 63) {
    b.rank = false;
    b.keybits = b.tbits + b.wshift;
    return true;
  }
  const int rb = bits_for((uint64_t)(rows > 1 ? rows - 1 : 1));
  if (rb + b.wshift > 63) return false;
  b.rank = true;
  b.keybits = rb + b.wshift;
  return true;
}

// Ranks the raw weights of the first cnt skeleton slots (wraw, overwritten)
// and completes their keys and the first Boruvka minima; the keys' other bits
// are in place. Scratch from ws.
ce_status stage_rank_weights(Bufs &b, uint64_t *wraw, int64_t cnt, Ws &ws, hipStream_t s) {
  if (cnt <= 0) return CE_OK;
  size_t m0 = ws.mark();
  uint32_t *slot = ws.alloc<uint32_t>(cnt), *slot_alt = ws.alloc<uint32_t>(cnt);
  uint64_t *w_alt = ws.alloc<uint64_t>(cnt);
  uint32_t *first = ws.alloc<uint32_t>(cnt + 1), *before = ws.alloc<uint32_t>(cnt + 1);
  CE_WS_CHECK(ws);
  const unsigned g = grid_cap(cnt, B);
  CE_LAUNCH(k_rank_absent, dim3(g), dim3(B), 0, s, b.skel_key, cnt, b.tbits, wraw);
  CE_HIP(hipGetLastError());
  bool alt = false;
  CE_TRY((radix_sort_pairs<uint64_t, uint32_t>(wraw, slot, w_alt, slot_alt, Cnt(cnt), 0, b.tbits + 1, true, &alt, ws,
                                               s)));
  const uint64_t *w = alt ? w_alt : wraw;
  const uint32_t *sl = alt ? slot_alt : slot;
  CE_LAUNCH(k_rank_flags, dim3(g), dim3(B), 0, s, w, cnt, b.tbits, first);
  CE_HIP(hipGetLastError());
  CE_TRY(scan_exclusive_u32(first, before, Cnt(cnt), ws, s));
  CE_LAUNCH(k_rank_apply, dim3(g), dim3(B), 0, s, w, sl, first, before, cnt, b.tbits, b.wshift, b.flat, b.skel_key,
            b.skel_tail, b.skel_tid, b.best);
  CE_HIP(hipGetLastError());
  ws.release(m0);
  return CE_OK;
}

size_t stage_rank_weights_scratch(int64_t cnt) {
  Ws w;
  w.alloc<uint32_t>(cnt);
  w.alloc<uint32_t>(cnt);
  w.alloc<uint64_t>(cnt);
  w.alloc<uint32_t>(cnt + 1);
  w.alloc<uint32_t>(cnt + 1);
  const size_t a = radix_ws_bytes(cnt), c = scan_ws_bytes(cnt + 1);
  return w.off + (a > c ? a : c) + 4096;
}

size_t stage_sort_skeleton_scratch(int64_t n) {
  Ws w;
  w.alloc<uint64_t>(2 * n);  // raw weights, when the weights are ranked
  const size_t r0 = w.off;
  for (int k = 0; k < 4; k++) w.alloc<uint32_t>(2 * n);  // ikey, ival and their ping-pong copies
  size_t base = w.off;
  w.alloc<uint64_t>(n);  // tkey alt
  w.alloc<uint4>(n);     // (id, src, dst)
  w.alloc<uint4>(n);     // ... ping-pong
  size_t a = w.off + radix_ws_bytes(n);
  size_t b2 = base + radix_ws_bytes(2 * n);
  size_t c = r0 + stage_rank_weights_scratch(2 * n);
  if (b2 > a) a = b2;
  return (a > c ? a : c) + 4096;
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
  CE_LAUNCH(k_tkeys, dim3(grid_for(n, B)), dim3(B), 0, s, t, src, dst, n, b.eoff, b.voff, b.G, b.hdr, b.ts, tval);
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
  uint64_t *wraw = b.rank ? ws.alloc<uint64_t>(n2) : nullptr;  // raw weights until they are ranked
  size_t m1 = ws.mark();
  uint32_t *ikey = ws.alloc<uint32_t>(n2);
  uint32_t *ival = ws.alloc<uint32_t>(n2);
  uint32_t *ikey_alt = ws.alloc<uint32_t>(n2);
  uint32_t *ival_alt = ws.alloc<uint32_t>(n2);
  CE_WS_CHECK(ws);
  // 1. records by (t, id)
  // 2. incidence entries (vertex, 2*rank+side) in rank order, perm by rank
  {
    size_t m2 = ws.mark();
    if (b.G == 1 && b.tbits <= 32) {
      uint64_t *kalt = ws.alloc<uint64_t>(n), *v0 = ws.alloc<uint64_t>(n), *v1 = ws.alloc<uint64_t>(n);
      CE_WS_CHECK(ws);
      CE_LAUNCH(k_tkeys_packed, dim3(grid_for(n, B)), dim3(B), 0, s, t, src, dst, n, b.hdr, b.ts, v0);
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
    ws.release(m2);
  }
  // stable sort by vertex keeps every list in rank order
  bool alt = false;
  CE_TRY((radix_sort_pairs<uint32_t, uint32_t>(ikey, ival, ikey_alt, ival_alt, n2, 0, b.vbits, true, &alt, ws, s)));
  const uint32_t *sk = alt ? ikey_alt : ikey;
  const uint32_t *sv = alt ? ival_alt : ival;
  // 3. skeleton: predecessor in the same vertex list, then packed keys
  CE_LAUNCH(k_skel_tails, dim3(grid_for(n2, B)), dim3(B), 0, s, sk, sv, n2, b.hdr, b.skel_tail);
  CE_LAUNCH(k_fill_u64, dim3(grid_for(n, B)), dim3(B), 0, s, b.best, n, NONE64);
  CE_HIP(hipGetLastError());
  CE_LAUNCH(k_skel_keys, dim3(grid_for(n, B)), dim3(B), 0, s, b.skel_tail, b.ts, b.perm, n, b.idbits, b.skel_key,
            b.best, wraw);
  CE_HIP(hipGetLastError());
  ws.release(m1);
  if (b.rank) CE_TRY(stage_rank_weights(b, wraw, n2, ws, s));
  ws.release(m0);
  return CE_OK;
}

size_t stage_boruvka_scratch(int64_t n, int64_t slots) {
  Ws w;
  w.alloc<uint32_t>(n);      // hook
  w.alloc<uint32_t>(n);      // bidx
  w.alloc<uint32_t>(n + 1);  // root flags
  w.alloc<uint32_t>(n + 1);  // dense ids
  w.alloc<uint32_t>(n);      // final ids
  w.alloc<uint32_t>(n);      // root map of a split
  for (int k = 0; k < 2; k++) {  // edge lists (key, u, v, slot), ping-pong
    w.alloc<uint64_t>(slots);
    w.alloc<uint32_t>(slots);
    w.alloc<uint32_t>(slots);
    w.alloc<uint32_t>(slots);
  }
  return w.off + scan_ws_bytes(n + 1) + 4096;
}

// The filter split runs when the live edges number at least 2^20 and more
// than twice the components. A call's tuning (ce_tuning.split_min_edges,
// CE_SPLIT_MIN_EDGES) overrides the 2^20 or turns the split off.
static int64_t split_min_edges() { return tuning().split_min_edges; }

// Rounds the host enqueues after the first: in every round the components
// that still have live edges at least halve, so bits(n) + 1 rounds end a run
// of plain rounds. With the (single) split, plain rounds before it and the
// light rounds together halve the components at least once per round, and so
// do the light rounds and the plain rounds after them: 2 (bits(n) + 1) + 1
// rounds cover both.
int boruvka_rounds(int64_t n, bool split_possible) {
  const int r = bits_for((uint64_t)n) + 1;
  return split_possible ? 2 * r + 1 : r;
}

ce_status stage_boruvka(Bufs &b, Ws &ws, hipStream_t s) {
  const int64_t n = b.n, n2 = b.slots;
  size_t m0 = ws.mark();
  uint32_t *hook = ws.alloc<uint32_t>(n);
  uint32_t *bidx = ws.alloc<uint32_t>(n);
  uint32_t *flags = ws.alloc<uint32_t>(n + 1);
  uint32_t *newid = ws.alloc<uint32_t>(n + 1);
  uint32_t *fin = ws.alloc<uint32_t>(n);
  uint32_t *rootof = ws.alloc<uint32_t>(n);
  EdgeLists L;
  for (int k = 0; k < 2; k++) {
    L.key[k] = ws.alloc<uint64_t>(n2);
    L.u[k] = ws.alloc<uint32_t>(n2);
    L.v[k] = ws.alloc<uint32_t>(n2);
    L.s[k] = ws.alloc<uint32_t>(n2);
  }
  CE_WS_CHECK(ws);
  L.key[2] = b.skel_key;
  L.u[2] = b.skel_tail;
  L.v[2] = b.skel_tid;
  L.s[2] = nullptr;
  L.cap = n2;
  uint64_t *bv = b.hdr + H_BV;
  uint32_t *rankof = b.rankof;  // kept for writing the per-record outputs in input order
  CE_LAUNCH(k_rankof, dim3(grid_for(n, B)), dim3(B), 0, s, b.perm, n, rankof);
  uint64_t *best = b.best;  // seeded for the first round while the skeleton was emitted
  CE_LAUNCH(k_fill_u8, dim3(grid_for(n2, B)), dim3(B), 0, s, b.msf_flag, n2, (uint8_t)0);
  const unsigned gN = grid_cap(n, B), gE = grid_cap(n2, B), tE = grid_cap(n2, B, tuning().list_grid);
  if (b.flat) {
    // causal and hypergraph skeleton rows can share a head, so every round,
    // the first included, runs on the edge-list form with records as
    // components; the first reads the skeleton rows in place (slot = row)
    CE_LAUNCH(k_bv_flat_init, dim3(1), dim3(64), 0, s, bv, &b.hdr[H_C7], n);
  } else {
    // first round on records, then its contraction into list 0
    CE_LAUNCH(k_bv_hook_first, dim3(gN), dim3(B), 0, s, n, best, b.skel_key, b.skel_tail, rankof, b.idbits, hook,
              b.msf_flag, flags);
    CE_LAUNCH(k_bv_compress, dim3(gN), dim3(B), 0, s, Cnt(n), hook, b.hdr);
    CE_LAUNCH(k_bv_roots, dim3(gN), dim3(B), 0, s, Cnt(n), hook, b.hdr);
    CE_HIP(hipGetLastError());
    CE_TRY(scan_exclusive_u32(flags, newid, Cnt(n), ws, s));
    CE_LAUNCH(k_final_ids, dim3(gN), dim3(B), 0, s, Cnt(n), hook, newid, fin, best);
    CE_LAUNCH(k_contract_first, dim3(tE), dim3(B), 0, s, n, b.skel_key, b.skel_tail, fin, newid, L, bv);
    CE_HIP(hipGetLastError());
  }
  // Filter split. When live edges far outnumber components, most of them run
  // between components that later rounds merge anyway, and every round would
  // scan them again. So the list is split at a pivot key: Borůvka runs on the
  // light edges (key below the pivot) alone until none is left, then the heavy
  // ones are contracted once and rounds go on with the survivors. Keys are
  // unique, so the forest is the same: a light edge outside the light forest
  // is the largest on a cycle of light edges, and contracting the light forest
  // keeps every heavy edge's cycles. During the light phase components keep
  // the ids they had at the split (no renumbering) and rootof maps each of
  // them to its current root; the heavy edges wait at the back of the buffer
  // the split wrote.
  const int64_t split_min = split_min_edges();
  const bool split_possible = n2 >= split_min;
  const int rounds = boruvka_rounds(n, split_possible);
  const Cnt CG(&bv[BV_CG], n), CN(&bv[BV_CN], n), CL(&bv[BV_CL], n);
  for (int r = 0; r < rounds; r++) {
    if (split_possible) {
      CE_LAUNCH(k_split_prep, dim3(1), dim3(SPLIT_SAMPLES), 0, s, L, bv, split_min);
      CE_LAUNCH(k_split, dim3(tE), dim3(B), 0, s, L, bv);
    }
    CE_LAUNCH(k_bv_min, dim3(tE), dim3(B), 0, s, L, bv, best);
    CE_LAUNCH(k_bv_pick, dim3(gE), dim3(B), 0, s, L, bv, best, bidx);
    CE_LAUNCH(k_bv_hook, dim3(gN), dim3(B), 0, s, L, bv, best, bidx, hook, b.msf_flag, flags);
    CE_LAUNCH(k_bv_compress, dim3(gN), dim3(B), 0, s, CG, hook, b.hdr);
    CE_LAUNCH(k_bv_roots, dim3(gN), dim3(B), 0, s, CG, hook, b.hdr);
    CE_HIP(hipGetLastError());
    if (split_possible) {
      // light round: ids stay; the edges' endpoints are this round's roots, hook gives their new ones
      CE_LAUNCH(k_compose_roots, dim3(gN), dim3(B), 0, s, CL, bv, hook, rootof, best);
      CE_LAUNCH(k_contract, dim3(tE), dim3(B), 0, s, L, bv, &bv[BV_EL], hook, newid, 1);
    }
    // plain round: dense ids for the surviving roots, then the contraction
    CE_TRY(scan_exclusive_u32(flags, newid, CN, ws, s));
    CE_LAUNCH(k_final_ids, dim3(gN), dim3(B), 0, s, CN, hook, newid, fin, best);
    CE_LAUNCH(k_contract, dim3(tE), dim3(B), 0, s, L, bv, &bv[BV_EN], fin, newid, 0);
    if (split_possible)  // after the light phase: the heavy edges between different current roots
      CE_LAUNCH(k_contract, dim3(tE), dim3(B), 0, s, L, bv, &bv[BV_EHG], rootof, newid, 2);
    CE_HIP(hipGetLastError());
  }
  CE_LAUNCH(k_bv_check, dim3(1), dim3(64), 0, s, bv, b.hdr);
  CE_HIP(hipGetLastError());
  ws.release(m0);
  return CE_OK;
}

// Time-filtered line graph (Sec. 5.1): only edges with w <= max_dt. The
// filtered skeleton has the filtered line graph's components at every
// threshold up to max_dt (Thm 3), and Kruskal takes edges in key order, so
// its forest is the prefix of the sorted MSF with w <= max_dt.
ce_status stage_time_filter(Bufs &b, int64_t max_dt, hipStream_t s) {
  if (max_dt < 0) return CE_OK;
  // the sorted rows' weights ascend
  CE_LAUNCH(k_prefix_below, dim3(1), dim3(64), 0, s, b.msf_key, &b.hdr[H_M], (uint64_t)max_dt + 1);
  CE_HIP(hipGetLastError());
  return CE_OK;
}

size_t stage_msf_sort_scratch(int64_t n) {
  Ws w;
  w.alloc<uint64_t>(n);
  w.alloc<uint64_t>(n);
  w.alloc<uint32_t>(n);
  return w.off + radix_ws_bytes(n) + 4096;
}

// The forest's rows (m on the device, at most n - 1) sorted by key into
// msf_key / msf_val.
ce_status stage_msf_sort(Bufs &b, Ws &ws, hipStream_t s) {
  const int64_t n = b.n, n2 = b.slots;
  size_t m0 = ws.mark();
  uint64_t *key_alt = ws.alloc<uint64_t>(n);
  uint64_t *val_alt = ws.alloc<uint64_t>(n);
  uint32_t *list = ws.alloc<uint32_t>(n);
  CE_WS_CHECK(ws);
  CE_LAUNCH(k_set_u64, dim3(1), dim3(1), 0, s, &b.hdr[H_M], (uint64_t)0);
  CE_LAUNCH(k_msf_list, dim3(grid_cap(n2, B, tuning().list_grid)), dim3(B), 0, s, b.msf_flag, n2, list,
            (unsigned long long *)&b.hdr[H_M]);
  CE_LAUNCH(k_check_rows, dim3(1), dim3(64), 0, s, b.hdr, n);
  CE_HIP(hipGetLastError());
  const Cnt m(&b.hdr[H_M], n > 1 ? n - 1 : 1);
  // gather into the buffer pair from which an odd or even number of radix
  // passes ends in msf_key / msf_val, so no copy follows the sort
  const int passes = b.keybits > 8 ? (b.keybits + 7) / 8 : 1;
  uint64_t *gk = (passes & 1) ? key_alt : b.msf_key, *gv = (passes & 1) ? val_alt : b.msf_val;
  uint64_t *ok = (passes & 1) ? b.msf_key : key_alt, *ov = (passes & 1) ? b.msf_val : val_alt;
  if (b.flat)
    CE_LAUNCH(k_msf_gather_causal, dim3(grid_cap(m.v, B)), dim3(B), 0, s, list, m, b.skel_key, b.skel_tail,
              b.skel_tid, gk, gv);
  else
    CE_LAUNCH(k_msf_gather, dim3(grid_cap(m.v, B)), dim3(B), 0, s, list, m, b.skel_key, b.skel_tail, gk, gv);
  bool alt = false;
  CE_TRY((radix_sort_pairs<uint64_t, uint64_t>(gk, gv, ok, ov, m, 0, b.keybits, false, &alt, ws, s)));
  if ((alt ? ok : gk) != b.msf_key) {  // (not reached: the pass count is as computed)
    set_error("internal: sorted forest is not in place");
    return CE_EDEVICE;
  }
  // the keys have done their work (the order); from here on msf_key holds each row's weight
  CE_LAUNCH(k_msf_weights, dim3(grid_cap(m.v, B)), dim3(B), 0, s, b.msf_key, b.msf_val, b.ts, m, b.wshift, b.rank);
  CE_HIP(hipGetLastError());
  ws.release(m0);
  return CE_OK;
}

}  // namespace ce
