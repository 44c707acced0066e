// Stage A7: exact single-linkage dendrogram from the sorted MSF (Alg. 1 step 3).
//
// The paper builds the dendrogram with a union-find pass over the sorted MST
// edges and calls that pass an expensive serial operation (Sec. 3). Here it is
// computed exactly in O(log m) parallel levels:
//
// For MSF row j (rows in key order), its two children are the dendrogram roots
// of the components of its endpoints in the forest of rows < j; the root of a
// component is its largest row (or the record itself when alone). Split the
// row range into aligned intervals. For an interval I=[a,b) the edges of I only
// see components of rows < a through their "labels" (roots at time a). The
// labels used inside one interval are disjoint from those of every other
// interval of the same length, because a root stays a root only until the
// first later row touching it. So one global union-find indexed by label can
// serve all intervals of a level at once. A level splits each interval into K
// sub-intervals processed in order: relabel the rows of sub-interval q to the
// roots after sub-intervals < q (largest row of the merged component), then
// union them. Sizes travel with labels. When intervals are small enough
// (512 rows) one workgroup finishes all remaining levels in LDS with binary
// splits, and the labels at the end are exactly the children.
//
// Within a level, the relabeling of sub-interval q and its unions run in one
// kernel: every hook records the sub-interval it was made in, so a find that
// must see the roots at the start of q stops at nodes hooked during q, and
// path halving never shortcuts such a link.
#include "ce_internal.h"

namespace ce {

namespace {

constexpr int B = 256;

__device__ inline void st(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One 16-byte entry per label keeps everything a level needs in a single
// cache line: x = parent, y = the sub-interval in which the node was hooked
// (NONE while it is a root), z = largest row + 1 of the component (0 = none),
// w = component size. x and y change together (one 64-bit CAS); z and w change
// only between kernels of a sub-interval. (The hot-root atomics are
// pre-aggregated in LDS.)
__device__ inline uint2 ld2(const uint4 *e) {
  const uint64_t v = __hip_atomic_load((const uint64_t *)e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}

// The same 8 bytes through the caches, possibly stale: what it returns was the
// entry's content at some time since the kernel started. A parent always has
// a smaller label than its child (hooks put the larger root under the smaller,
// halving moves a link to a grandparent), so a walk over stale links still
// ends, and every node it meets is an ancestor. Used where that is enough:
// finds that only follow links made by earlier kernels.
__device__ inline uint2 ld2_cached(const uint4 *e) {
  const uint64_t v = __hip_atomic_load((const uint64_t *)e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}

// root at the start of sub-interval q, from x and its entry e: links made
// during q (or later) are not followed, and every older link was made before
// this kernel, so a stale view of them is still exact
__device__ inline uint32_t g_find_before(uint4 *uf, uint32_t x, uint2 e, uint32_t q) {
  while (true) {
    if (e.x == x || e.y >= q) return x;
    const uint2 pe = ld2_cached(&uf[e.x]);
    if (pe.x == e.x || pe.y >= q) return e.x;
    st(&uf[x].x, pe.x);  // both links are older than q
    x = pe.x;
    e = ld2_cached(&uf[x]);
  }
}

// current root; halves only links older than q, so the roots at the start of
// q stay reachable for g_find_before
__device__ inline uint32_t g_find(uint4 *uf, uint32_t x, uint32_t q) {
  while (true) {
    const uint2 e = ld2(&uf[x]);
    if (e.x == x) return x;
    const uint2 pe = ld2(&uf[e.x]);
    if (pe.x == e.x) return e.x;
    if (e.y < q && pe.y < q) st(&uf[x].x, pe.x);
    x = pe.x;
  }
}

// the final root once every link of the level so far is in place (no hooks
// run concurrently, only halving): a stale view ends at the same root
__device__ inline uint32_t g_find_done(uint4 *uf, uint32_t x) {
  while (true) {
    const uint2 e = ld2_cached(&uf[x]);
    if (e.x == x) return x;
    const uint2 pe = ld2_cached(&uf[e.x]);
    if (pe.x == e.x) return e.x;
    st(&uf[x].x, pe.x);
    x = pe.x;
  }
}

// hooks the larger of the two roots under the smaller during sub-interval q;
// returns the hooked root. a and b are the roots at the start of q, so the
// first attempt hooks without another find: it fails only when the larger one
// was hooked during q, and the loop then finds the current roots.
__device__ inline uint32_t g_union(uint4 *uf, uint32_t a, uint32_t b, uint32_t q) {
  if (a == b) return NONE32;
  const unsigned long long to = (unsigned long long)q << 32;
  {
    const uint32_t hi = a > b ? a : b, lo = a > b ? b : a;
    const unsigned long long want = ((unsigned long long)NONE32 << 32) | hi;
    if (atomicCAS((unsigned long long *)&uf[hi], want, to | lo) == want) return hi;
  }
  while (true) {
    a = g_find(uf, a, q);
    b = g_find(uf, b, q);
    if (a == b) return NONE32;
    const uint32_t hi = a > b ? a : b, lo = a > b ? b : a;
    const unsigned long long want = ((unsigned long long)NONE32 << 32) | hi;
    if (atomicCAS((unsigned long long *)&uf[hi], want, to | lo) == want) return hi;
  }
}

__global__ __launch_bounds__(B) void k_krt_init(const uint64_t *msf_val, Cnt mc, uint32_t *lu, uint32_t *lv,
                                                uint32_t *su, uint32_t *sv) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    const uint64_t v = msf_val[j];
    lu[j] = (uint32_t)v;          // tail rank
    lv[j] = (uint32_t)(v >> 32);  // head rank
    su[j] = 1;
    sv[j] = 1;
  }
}

__global__ __launch_bounds__(B) void k_krt_reset(const uint32_t *lu, const uint32_t *lv, const uint32_t *su,
                                                 const uint32_t *sv, Cnt mc, uint4 *uf) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    uint32_t a = lu[j], b = lv[j];
    uf[a] = make_uint4(a, NONE32, 0u, su[j]);
    uf[b] = make_uint4(b, NONE32, 0u, sv[j]);
  }
}

// the first level's labels are exactly the records, each of size 1: a streaming fill
__global__ __launch_bounds__(B) void k_krt_reset_records(int64_t n, uint4 *uf) {
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < n; r += (int64_t)gridDim.x * B)
    uf[r] = make_uint4((uint32_t)r, NONE32, 0u, 1u);
}

__device__ inline int64_t step_row(int64_t tix, int lo, int hi, uint32_t q) {
  int64_t interval = tix >> lo;
  int64_t off = tix & ((int64_t(1) << lo) - 1);
  return (interval << (hi + 1)) | ((int64_t)q << lo) | off;
}

// Sub-interval q: relabel its rows to the roots at the start of q (for q >= 1:
// the largest row and size of the component after sub-intervals < q), then
// union them. Largest rows and sizes (z, w) are read while other threads hook
// roots, which changes only x and y.
__global__ __launch_bounds__(B) void k_krt_union(Cnt mc, int64_t n, int lo, int hi, uint32_t q, int64_t nthreads,
                                                 uint32_t *lu, uint32_t *lv, uint32_t *su, uint32_t *sv, uint4 *uf,
                                                 uint32_t *hooked) {
  const int64_t m = mc.get();
  if (((int64_t)q << lo) >= m) return;  // no interval reaches sub-interval q
  for (int64_t tix = (int64_t)blockIdx.x * B + threadIdx.x; tix < nthreads; tix += (int64_t)gridDim.x * B) {
    int64_t j = step_row(tix, lo, hi, q);
    if (j >= m) continue;
    uint32_t a = lu[j], b = lv[j];
    if (q) {
      const uint2 ea = ld2_cached(&uf[a]), eb = ld2_cached(&uf[b]);  // both walks start at once
      a = g_find_before(uf, a, ea, q);
      b = g_find_before(uf, b, eb, q);
      const uint4 na = uf[a];
      if (na.z) {
        lu[j] = (uint32_t)(n + na.z - 1);
        su[j] = na.w;
      }
      const uint4 nb = uf[b];
      if (nb.z) {
        lv[j] = (uint32_t)(n + nb.z - 1);
        sv[j] = nb.w;
      }
    }
    hooked[j] = g_union(uf, a, b, q);
  }
}

// Rows of a sub-interval are consecutive, so a tile of up to 4096 rows
// (kct per thread) mostly feeds few components (late steps: the giant one).
// Sizes and largest rows are summed per component root in an LDS hash first,
// then one atomic per root per tile; rows whose root finds no free slot go
// straight to global atomics.
constexpr int KHS = 256;
__global__ __launch_bounds__(B) void k_krt_accum(Cnt mc, int lo, int hi, uint32_t q, int64_t nthreads, int kct,
                                                 const uint32_t *hooked, uint4 *uf) {
  __shared__ uint32_t hk[KHS], hs[KHS], hm[KHS];
  const int64_t m = mc.get();
  if (((int64_t)q << lo) >= m) return;
  for (int i = threadIdx.x; i < KHS; i += B) { hk[i] = NONE32; hs[i] = 0; hm[i] = 0; }
  __syncthreads();
  const int64_t tbase = (int64_t)blockIdx.x * (B * kct);
  for (int k = 0; k < kct; k++) {
    const int64_t tix = tbase + (int64_t)k * B + threadIdx.x;
    const int64_t j = tix < nthreads ? step_row(tix, lo, hi, q) : m;
    uint32_t h = NONE32, f = 0, add = 0, mj = 0;
    if (j < m) h = hooked[j];
    if (h != NONE32) {
      f = g_find_done(uf, h);  // every link of sub-interval q is in place
      add = uf[h].w;
      mj = (uint32_t)(j + 1);
    }
    const bool upd = wave_combine_first(h != NONE32, f, [&](bool mine, int leader) {
      const uint32_t sa = wave_sum_u32(mine ? add : 0u), sm = wave_max_u32(mine ? mj : 0u);
      if ((int)wave_lane() == leader) { add = sa; mj = sm; }
    });
    if (upd) {
      uint32_t sl = (f * 2654435761u) >> 24;  // 8 bits
      bool placed = false;
      for (int probe = 0; probe < HASH_PROBES && !placed; probe++) {
        uint32_t old = atomicCAS(&hk[sl], NONE32, f);
        if (old == NONE32 || old == f) {
          atomicAdd(&hs[sl], add);
          atomicMax(&hm[sl], mj);
          placed = true;
        } else {
          sl = (sl + 1) & (KHS - 1);
        }
      }
      if (!placed) {
        atomicAdd(&uf[f].w, add);
        atomicMax(&uf[f].z, mj);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < KHS; i += B) {
    const uint32_t f = hk[i];
    if (f == NONE32) continue;
    atomicAdd(&uf[f].w, hs[i]);
    atomicMax(&uf[f].z, hm[i]);
  }
}

// ---------------------------------------------------------------- LDS level
constexpr int LS_BITS = 9;
constexpr int LS = 1 << LS_BITS;  // rows per workgroup
constexpr int HS = 4 * LS;        // hash slots (load factor <= 1/2)
constexpr int LB = 512;           // threads per interval: one per row
constexpr uint32_t EMPTY = 0xffffffffu;

// LDS union-find; relaxed workgroup-scope atomics (not volatile, which would
// turn the accesses into flat ones)
__device__ inline uint32_t l_ld(uint32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }

__device__ inline uint32_t l_find(uint32_t *uf, uint32_t x) {
  while (true) {
    uint32_t p = l_ld(&uf[x]);
    if (p == x) return x;
    uint32_t gp = l_ld(&uf[p]);
    if (gp == p) return p;
    __hip_atomic_store(&uf[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    x = gp;
  }
}

__device__ inline uint32_t l_union(uint32_t *uf, uint32_t a, uint32_t b) {
  while (true) {
    a = l_find(uf, a);
    b = l_find(uf, b);
    if (a == b) return EMPTY;
    uint32_t hi = a > b ? a : b, lo = a > b ? b : a;
    uint32_t want = hi;
    if (__hip_atomic_compare_exchange_strong(&uf[hi], &want, lo, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP))
      return hi;
  }
}

__device__ inline uint32_t hslot(uint32_t g) { return (g * 2654435761u) >> (32 - (LS_BITS + 2)); }

__global__ __launch_bounds__(LB) void k_krt_lds(const uint32_t *lu, const uint32_t *lv, const uint32_t *su,
                                               const uint32_t *sv, Cnt mc, int64_t n, uint32_t *kc_u,
                                               uint32_t *kc_v, uint32_t *ksize) {
  const int64_t m = mc.get();
  if ((int64_t)blockIdx.x * LS >= m) return;
  __shared__ uint32_t hkey[HS];
  __shared__ uint16_t hid[HS];
  __shared__ uint32_t glab[2 * LS];
  __shared__ uint32_t luf[3 * LS];
  __shared__ uint32_t lmx[3 * LS];
  __shared__ uint32_t lcs[3 * LS];
  __shared__ uint32_t lsz[3 * LS];
  __shared__ uint16_t elu[LS], elv[LS], ehk[LS];
  __shared__ uint32_t nloc;
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * LS;
  const int cnt = (int)((m - base) < LS ? (m - base) : LS);
  for (int i = tid; i < HS; i += LB) hkey[i] = EMPTY;
  if (tid == 0) nloc = 0;
  __syncthreads();
  // 1. distinct labels of this interval into an LDS hash set
  for (int i = tid; i < 2 * cnt; i += LB) {
    uint32_t g = (i & 1) ? lv[base + (i >> 1)] : lu[base + (i >> 1)];
    uint32_t s = hslot(g);
    while (true) {
      uint32_t old = atomicCAS(&hkey[s], EMPTY, g);
      if (old == EMPTY || old == g) break;
      s = (s + 1) & (HS - 1);
    }
  }
  __syncthreads();
  // 2. local ids for the distinct labels
  for (int s = tid; s < HS; s += LB) {
    uint32_t g = hkey[s];
    if (g != EMPTY) {
      uint32_t id = atomicAdd(&nloc, 1u);
      hid[s] = (uint16_t)id;
      glab[id] = g;
    }
  }
  __syncthreads();
  // 3. rows' labels as local ids, with sizes
  for (int i = tid; i < 2 * cnt; i += LB) {
    const bool isv = i & 1;
    const int r = i >> 1;
    uint32_t g = isv ? lv[base + r] : lu[base + r];
    uint32_t s = hslot(g);
    while (hkey[s] != g) s = (s + 1) & (HS - 1);
    uint16_t id = hid[s];
    if (isv) elv[r] = id; else elu[r] = id;
    lsz[id] = isv ? sv[base + r] : su[base + r];
  }
  __syncthreads();
  uint32_t *vuf = luf;
  // 4. binary levels inside the interval
  for (int bit = LS_BITS - 1; bit >= 0; bit--) {
    for (int i = tid; i < cnt; i += LB) {
      uint32_t a = elu[i], b = elv[i];
      luf[a] = a; luf[b] = b;
      lmx[a] = 0; lmx[b] = 0;
      lcs[a] = lsz[a]; lcs[b] = lsz[b];
    }
    __syncthreads();
    for (int i = tid; i < cnt; i += LB)
      if (!((i >> bit) & 1)) ehk[i] = (uint16_t)l_union(vuf, elu[i], elv[i]);
    __syncthreads();
    for (int i = tid; i < cnt; i += LB) {
      if ((i >> bit) & 1) continue;
      uint32_t h = ehk[i];
      if (h == 0xffffu) continue;
      uint32_t f = l_find(vuf, h);
      atomicAdd(&lcs[f], lcs[h]);
      atomicMax(&lmx[f], (uint32_t)(i + 1));
    }
    __syncthreads();
    for (int i = tid; i < cnt; i += LB) {
      if (!((i >> bit) & 1)) continue;
      uint32_t f = l_find(vuf, elu[i]);
      if (lmx[f]) {
        uint32_t nx = 2 * LS + lmx[f] - 1;
        lsz[nx] = lcs[f];
        elu[i] = (uint16_t)nx;
      }
      f = l_find(vuf, elv[i]);
      if (lmx[f]) {
        uint32_t nx = 2 * LS + lmx[f] - 1;
        lsz[nx] = lcs[f];
        elv[i] = (uint16_t)nx;
      }
    }
    __syncthreads();
  }
  // 5. children as internal labels (record rank < n, or n + row)
  for (int i = tid; i < cnt; i += LB) {
    uint32_t a = elu[i], b = elv[i];
    uint32_t ga = a < 2 * LS ? glab[a] : (uint32_t)(n + base + (a - 2 * LS));
    uint32_t gb = b < 2 * LS ? glab[b] : (uint32_t)(n + base + (b - 2 * LS));
    kc_u[base + i] = ga;
    kc_v[base + i] = gb;
    ksize[base + i] = lsz[a] + lsz[b];
  }
}

}  // namespace

// Largest number of bits one global level may take. The global bits
// (L - 9 for rows j < 2^L) are split into levels; a level of k bits runs 2^k
// sub-intervals one after another. Every level costs a pass of random
// accesses over all rows (its reset, relabels, unions and sums: about 0.4 ns
// per row, fitted to runs at 5e7 and 2^30 rows), and every sub-interval two
// dependent launches (about 20 us), every level one more (15 us). The plan
// takes the level count with the least modelled time: few wide levels for
// large m (two at 5e7 and 2^30 rows), narrow ones when launches dominate. A
// call's tuning (ce_tuning.krt_level_bits, CE_KRT_LEVEL_BITS) overrides it
// (1..12).
int krt_max_level_bits(int64_t m) {
  const int forced = tuning().krt_level_bits;
  if (forced > 0) return forced;
  const int gbits = bits_for((uint64_t)(m > 1 ? m - 1 : 1)) - 9;
  if (gbits <= 1) return 1;
  double best = 1e30;
  int kbest = gbits;
  for (int nlev = 1; nlev <= gbits; nlev++) {
    const int hi = (gbits + nlev - 1) / nlev, lo = gbits / nlev, nhi = gbits % nlev;
    if (hi > 12) continue;
    const double steps = (double)nhi * (double)(1 << hi) + (double)(nlev - nhi) * (double)(1 << lo);
    const double t = nlev * (0.4e-9 * (double)m + 15e-6) + steps * 20e-6;
    if (t < best) {
      best = t;
      kbest = hi;
    }
  }
  return kbest;
}

size_t stage_dendrogram_scratch(int64_t n) {
  Ws w;
  for (int k = 0; k < 5; k++) w.alloc<uint32_t>(n);  // lu lv su sv hooked
  w.alloc<uint4>(2 * n);  // packed union-find over labels < n + m
  return w.off + 4096;
}

// The row count m is on the device; the level plan is made for its bound n - 1
// (levels and sub-intervals past the live rows find nothing to do).
ce_status stage_dendrogram(Bufs &b, Ws &ws, hipStream_t s) {
  const int64_t n = b.n;
  if (n <= 1) return CE_OK;
  const int64_t mb = n - 1;
  const Cnt m(&b.hdr[H_M], mb);
  size_t m0 = ws.mark();
  uint32_t *lu = ws.alloc<uint32_t>(mb), *lv = ws.alloc<uint32_t>(mb);
  uint32_t *su = ws.alloc<uint32_t>(mb), *sv = ws.alloc<uint32_t>(mb);
  uint32_t *hooked = ws.alloc<uint32_t>(mb);
  uint4 *uf = ws.alloc<uint4>(n + mb);
  CE_WS_CHECK(ws);
  CE_LAUNCH(k_krt_init, dim3(grid_cap(mb, B)), dim3(B), 0, s, b.msf_val, m, lu, lv, su, sv);
  CE_HIP(hipGetLastError());
  const int L = bits_for((uint64_t)(mb - 1));  // rows are j < 2^L
  // the global bits L-1 .. LS_BITS in as few levels as the largest level
  // allows, spread evenly (the upper levels take the remainder)
  const int gbits = L - LS_BITS, kmax = krt_max_level_bits(mb);
  const int nlev = gbits > 0 ? (gbits + kmax - 1) / kmax : 0;
  int hi = L - 1, lev = 0;
  bool first = true;
  while (hi >= LS_BITS) {
    const int kb = gbits / nlev + (lev < gbits % nlev ? 1 : 0);
    lev++;
    int lo = hi - kb + 1;
    if (lo < LS_BITS) lo = LS_BITS;
    const uint32_t K = 1u << (hi - lo + 1);
    const int64_t nint = (mb + (int64_t(1) << (hi + 1)) - 1) >> (hi + 1);
    const int64_t nthreads = nint << lo;
    const unsigned g = grid_for(nthreads, B, 1 << 16);
    const int kct = items_per_thread(nthreads, B);
    if (first) CE_LAUNCH(k_krt_reset_records, dim3(grid_cap(n, B)), dim3(B), 0, s, n, uf);
    else CE_LAUNCH(k_krt_reset, dim3(grid_cap(mb, B)), dim3(B), 0, s, lu, lv, su, sv, m, uf);
    first = false;
    for (uint32_t q = 0; q < K; q++) {
      // sub-interval q exists in at least one interval of the bound (the kernels check the live rows)
      if (((int64_t)q << lo) >= mb) break;
      CE_LAUNCH(k_krt_union, dim3(g), dim3(B), 0, s, m, n, lo, hi, q, nthreads, lu, lv, su, sv, uf, hooked);
      CE_LAUNCH(k_krt_accum, dim3((unsigned)((nthreads + B * kct - 1) / (B * kct))), dim3(B), 0, s, m, lo, hi,
                q, nthreads, kct, hooked, uf);
    }
    CE_HIP(hipGetLastError());
    hi = lo - 1;
  }
  const int64_t nblk = (mb + LS - 1) / LS;
  CE_LAUNCH(k_krt_lds, dim3((unsigned)nblk), dim3(LB), 0, s, lu, lv, su, sv, m, n, b.kc_u, b.kc_v, b.ksize);
  CE_HIP(hipGetLastError());
  ws.release(m0);
  return CE_OK;
}

}  // namespace ce
