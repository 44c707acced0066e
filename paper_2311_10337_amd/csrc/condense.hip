// Stages A8-A9: condense the dendrogram with the minimum cluster size M,
// stability, excess-of-mass selection and labels (Alg. 1 steps 4-5, with the
// HDBSCAN semantics of Campello et al. 2013 to which the paper defers).
//
// Node space: records are ranks [0,n), row j of the sorted MSF is node n+j,
// the virtual root is n+m. A node is "big" if its size >= M.
//  - birth nodes: both children of a row whose two children are big; and the
//    big component roots of a graph when it has at least two of them. A
//    cluster is identified by its birth node.
//  - batches: every graph g of a packed batch has its own virtual root, node
//    n+m+g; cluster rows are laid out graph by graph (births in node order,
//    then the graph's root), and labels are numbered per graph.
//  - the cluster of a big node is its nearest birth ancestor-or-self, found by
//    pointer jumping over big nodes (chains can be as deep as the data).
//  - a record leaves the cluster of its lowest big ancestor y, at lambda(w_y);
//    with no big ancestor it leaves ROOT at lambda 0.
//  - stability sums exact 96-bit quantities as 32-bit limbs in u64 atomics.
//  - excess of mass is a tree DP; chains are contracted by composing
//    f(x) = max(a, x + b) (pointer jumping), leaves are raked each round.
//  - the highest selected cluster above each cluster is again pointer jumping.
#include <vector>

#include "ce_internal.h"

namespace ce {

namespace {

constexpr int B = 256;

__device__ inline uint32_t node_size(uint32_t x, int64_t n, const uint32_t *ksize) {
  return x < (uint64_t)n ? 1u : ksize[x - n];
}

__global__ __launch_bounds__(B) void k_fill32(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) p[i] = v;
}
__global__ __launch_bounds__(B) void k_fill64(uint64_t *p, int64_t n, uint64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) p[i] = v;
}
__global__ void k_set64(uint64_t *p, uint64_t v) { *p = v; }

__global__ __launch_bounds__(B) void k_cd_parents(const uint32_t *kc_u, const uint32_t *kc_v, Cnt mc, int64_t n,
                                                  uint32_t *kpar) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    kpar[kc_u[j]] = (uint32_t)(n + j);
    kpar[kc_v[j]] = (uint32_t)(n + j);
  }
}

// big component roots per graph
__global__ __launch_bounds__(B) void k_cd_bigroots(const uint32_t *kpar, const uint32_t *ksize, const uint32_t *rowg,
                                                   Cnt mc, int64_t n, int64_t M, uint32_t *nbig) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B)
    if (kpar[n + j] == NONE32 && ksize[j] >= (uint64_t)M) atomicAdd(&nbig[rowg[j]], 1u);
}

__global__ __launch_bounds__(B) void k_cd_birth(const uint32_t *kc_u, const uint32_t *kc_v, const uint32_t *ksize,
                                                const uint32_t *kpar, const uint64_t *rowL, bool discrete, Cnt mc,
                                                int64_t n, int64_t M, const uint32_t *nbig, const uint32_t *rowg,
                                                uint8_t *isbirth, uint64_t *birthL) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    uint32_t a = kc_u[j], b = kc_v[j];
    if (!discrete && node_size(a, n, ksize) >= (uint64_t)M && node_size(b, n, ksize) >= (uint64_t)M) {
      uint64_t L = rowL[j];
      isbirth[a - n] = 1;
      birthL[a - n] = L;
      isbirth[b - n] = 1;
      birthL[b - n] = L;
    }
    if (kpar[n + j] == NONE32 && ksize[j] >= (uint64_t)M && nbig[rowg[j]] >= 2) {
      isbirth[j] = 1;
      birthL[j] = 0;
    }
  }
}

// lambda of every row: of its weight, or with thresholds (the discrete
// dendrogram of Alg. 5) of its level's threshold, level = the first threshold
// the weight does not exceed
__global__ __launch_bounds__(B) void k_row_lambda(const uint64_t *msf_w, Cnt mc, const int64_t *thr, int q,
                                                  uint64_t *rowL, uint32_t *level) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    const int64_t w = (int64_t)msf_w[j];
    if (q == 0) {
      rowL[j] = lambda_of(w);
      continue;
    }
    int L = 0;
    while (L < q - 1 && w > thr[L]) L++;  // rows above the last threshold were dropped before
    rowL[j] = lambda_of(thr[L]);
    level[j] = (uint32_t)L;
  }
}

// Discrete dendrogram: a row's level top is its highest ancestor reached
// through parents of the same level (the component that first appears at that
// level, a D-node). First step: the parent if it has the same level.
__global__ __launch_bounds__(B) void k_dd_top_init(const uint32_t *kpar, const uint32_t *level, Cnt mc, int64_t n,
                                                   uint32_t *top) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    const uint32_t p = kpar[n + j];
    top[j] = (p != NONE32 && level[p - n] == level[j]) ? p : (uint32_t)(n + j);
  }
}
// rows whose level top is not known yet (their pointer is not a top)
__global__ __launch_bounds__(B) void k_dd_top_active(const uint32_t *top, Cnt mc, int64_t n, uint32_t *act,
                                                     unsigned long long *nact) {
  const int64_t m = mc.get();
  const int ct = tile_items(m);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < m; tile += gridDim.x) {
    bool keep[CT];
    uint32_t vals[CT];
    const int64_t base = tile * (B * ct) + threadIdx.x, end = tile_end(m, tile, B * ct);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      const int64_t j = base + (int64_t)k * B;
      keep[k] = false;
      vals[k] = (uint32_t)j;
      if (j >= end) continue;
      const uint32_t t = top[j];
      keep[k] = t != (uint32_t)(n + j) && top[t - n] != t;
    }
    tile_append(keep, vals, act, nact);
  }
}
// one pointer-doubling round over the active rows, in place: a row only reads
// pointers of rows above it, which stay valid ancestors of the same level
__global__ __launch_bounds__(B) void k_dd_top_jump(const uint32_t *act, const uint64_t *nact_in, int64_t n,
                                                   uint32_t *top, uint32_t *next, unsigned long long *nnext) {
  const int64_t nact = (int64_t)*nact_in;
  const int ct = tile_items(nact);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < nact; tile += gridDim.x) {
    bool keep[CT];
    uint32_t vals[CT];
    const int64_t base = tile * (B * ct) + threadIdx.x, end = tile_end(nact, tile, B * ct);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      const int64_t i = base + (int64_t)k * B;
      keep[k] = false;
      vals[k] = 0;
      if (i >= end) continue;
      const uint32_t j = act[i], t = top[j], tt = top[t - n];
      if (tt == t) continue;  // t is a top
      top[j] = tt;
      keep[k] = top[tt - n] != tt;
      vals[k] = j;
    }
    tile_append(keep, vals, next, nnext);
  }
}
// after the enqueued rounds every list must be empty (pointer doubling over
// a tree of m rows ends within bits(m) + 1 rounds); if not, the call fails
__global__ void k_loop_done(const uint64_t *cnt, uint64_t *hdr) {
  if (threadIdx.x == 0 && *cnt != 0) hdr[H_STATUS] |= 32;
}
// big children of every D-node: the level tops (rows that are their own top)
// hanging below its block; records are never big (M >= 2)
// big D-node children per D-node; a D-node can have millions of them, so the
// counts are combined per wave and per tile (LDS hash) before the atomics
constexpr int DHS = 512;
__global__ __launch_bounds__(B) void k_dd_bigcount(const uint32_t *kpar, const uint32_t *ksize, const uint32_t *top,
                                                   Cnt mc, int64_t n, int64_t M, int kct, uint32_t *bigcnt) {
  __shared__ uint32_t hk[DHS], hc[DHS];
  const int64_t m = mc.get();
  for (int i = threadIdx.x; i < DHS; i += B) { hk[i] = NONE32; hc[i] = 0; }
  __syncthreads();
  const int64_t tbase = (int64_t)blockIdx.x * (B * kct);
  for (int k = 0; k < kct; k++) {
    const int64_t j = tbase + (int64_t)k * B + threadIdx.x;
    uint32_t d = 0, add = 0;
    if (j < m) {
      const uint32_t p = kpar[n + j];
      if (p != NONE32 && top[j] == (uint32_t)(n + j) && ksize[j] >= (uint64_t)M) {
        d = top[p - n] - (uint32_t)n;
        add = 1;
      }
    }
    const bool upd = wave_combine_first(add != 0, d, [&](bool mine, int leader) {
      const uint32_t sum = wave_sum_u32(mine ? add : 0u);
      if ((int)wave_lane() == leader) add = sum;
    });
    if (upd) {
      uint32_t sl = (d * 2654435761u) >> 23;  // 9 bits
      bool placed = false;
      for (int probe = 0; probe < HASH_PROBES && !placed; probe++) {
        const uint32_t old = atomicCAS(&hk[sl], NONE32, d);
        if (old == NONE32 || old == d) {
          atomicAdd(&hc[sl], add);
          placed = true;
        } else {
          sl = (sl + 1) & (DHS - 1);
        }
      }
      if (!placed) atomicAdd(&bigcnt[d], add);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < DHS; i += B)
    if (hk[i] != NONE32) atomicAdd(&bigcnt[hk[i]], hc[i]);
}
// a big child of a D-node with two or more big children starts a cluster at
// the D-node's lambda
__global__ __launch_bounds__(B) void k_dd_birth(const uint32_t *kpar, const uint32_t *ksize, const uint32_t *top,
                                                const uint32_t *bigcnt, const uint64_t *rowL, Cnt mc, int64_t n,
                                                int64_t M, uint8_t *isbirth, uint64_t *birthL) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    const uint32_t p = kpar[n + j];
    if (p == NONE32 || top[j] != (uint32_t)(n + j) || ksize[j] < (uint64_t)M) continue;
    if (bigcnt[top[p - n] - n] < 2) continue;
    isbirth[j] = 1;
    birthL[j] = rowL[p - n];
  }
}

// a virtual root (n+m+g) or a birth node ends the jump
__device__ inline bool j_terminal(uint32_t x, int64_t n, int64_t m, const uint8_t *isbirth) {
  return x >= (uint64_t)(n + m) || isbirth[x - n];
}

// J[j] for big rows: self if birth, ROOT if a root, else the parent node.
// Rows whose J is not yet a birth node or ROOT go to the active list.
__global__ __launch_bounds__(B) void k_cd_jinit(const uint8_t *isbirth, const uint32_t *kpar, const uint32_t *ksize,
                                                const uint32_t *rowg, Cnt mc, int64_t n, int64_t M, uint32_t *J,
                                                uint32_t *act, unsigned long long *nact) {
  const int64_t m = mc.get();
  const int ct = tile_items(m);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < m; tile += gridDim.x) {
    bool keep[CT];
    uint32_t vals[CT];
    const int64_t base = tile * (B * ct) + threadIdx.x, end = tile_end(m, tile, B * ct);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      const int64_t j = base + (int64_t)k * B;
      keep[k] = false;
      vals[k] = (uint32_t)j;
      if (j >= end) continue;
      uint32_t v = NONE32;
      if (ksize[j] >= (uint64_t)M) {
        if (isbirth[j]) v = (uint32_t)(n + j);
        else if (kpar[n + j] == NONE32) v = (uint32_t)(n + m + rowg[j]);
        else {
          v = kpar[n + j];
          keep[k] = !j_terminal(v, n, m, isbirth);
        }
      }
      J[j] = v;
    }
    tile_append(keep, vals, act, nact);
  }
}

// one pointer-doubling round toward the nearest birth ancestor; finished rows
// leave the list (in place: J only moves up, so a pointer read while another
// row updates it is still an ancestor on the way)
__global__ __launch_bounds__(B) void k_cd_jstep(const uint32_t *act, const uint64_t *nact_in, uint32_t *J,
                                                const uint8_t *isbirth, Cnt mc, int64_t n, uint32_t *out,
                                                unsigned long long *nout) {
  const int64_t m = mc.get(), nact = (int64_t)*nact_in;
  const int ct = tile_items(nact);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < nact; tile += gridDim.x) {
    bool keep[CT];
    uint32_t vals[CT];
    const int64_t base = tile * (B * ct) + threadIdx.x, end = tile_end(nact, tile, B * ct);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      const int64_t i = base + (int64_t)k * B;
      keep[k] = false;
      vals[k] = 0;
      if (i >= end) continue;
      const uint32_t j = act[i];
      const uint32_t x = J[j];
      const uint32_t y = J[x - n];
      J[j] = y;
      if (!j_terminal(y, n, m, isbirth)) {
        keep[k] = true;
        vals[k] = j;
      }
    }
    tile_append(keep, vals, out, nout);
  }
}

__global__ __launch_bounds__(B) void k_u8_to_u32(const uint8_t *a, Cnt nc, uint32_t *o) {
  const int64_t n = nc.get();
  for (int64_t i = (int64_t)blockIdx.x * B + threadIdx.x; i < n; i += (int64_t)gridDim.x * B) o[i] = a[i];
}

__device__ inline uint32_t row_of(uint32_t c, int64_t n, int64_t m, const uint32_t *rowof, const uint32_t *rootrow) {
  return c >= (uint64_t)(n + m) ? rootrow[c - n - m] : rowof[c - n];
}

// cluster rows: node, size, birth lambda, parent row
__global__ __launch_bounds__(B) void k_cd_rows(const uint8_t *isbirth, const uint32_t *rowof, const uint32_t *rootrow,
                                               const uint32_t *ksize, const uint64_t *birthL, const uint32_t *kpar,
                                               const uint32_t *J, const uint32_t *rowg, Cnt mc, int64_t n,
                                               uint32_t *cnode, uint32_t *csize, uint64_t *cbirth, uint32_t *cprow) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    if (!isbirth[j]) continue;
    uint32_t r = rowof[j];
    cnode[r] = (uint32_t)(n + j);
    csize[r] = ksize[j];
    cbirth[r] = birthL[j];
    uint32_t par = kpar[n + j];
    uint32_t pc = par == NONE32 ? (uint32_t)(n + m + rowg[j]) : J[par - n];
    cprow[r] = row_of(pc, n, m, rowof, rootrow);
  }
}

// one root row per graph: size = the graph's records, born at lambda 0, no parent
__global__ __launch_bounds__(B) void k_cd_rootrows(const uint32_t *rootrow, const int64_t *eoff, int64_t G, Cnt mc,
                                                   int64_t n, uint32_t *cnode, uint32_t *csize, uint64_t *cbirth,
                                                   uint32_t *cprow) {
  const int64_t m = mc.get();
  for (int64_t g = (int64_t)blockIdx.x * B + threadIdx.x; g < G; g += (int64_t)gridDim.x * B) {
    const uint32_t r = rootrow[g];
    cnode[r] = (uint32_t)(n + m + g);
    csize[r] = (uint32_t)(eoff[g + 1] - eoff[g]);
    cbirth[r] = 0;
    cprow[r] = NONE32;
  }
}

// births in (graph, node) order: position p gives row p + g (each earlier graph adds its root row)
__global__ __launch_bounds__(B) void k_birth_list(const uint8_t *isbirth, const uint32_t *idx, const uint32_t *rowg,
                                                  Cnt mc, uint32_t *bkey, uint32_t *bval) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    if (!isbirth[j]) continue;
    const uint32_t i = idx[j];
    bkey[i] = rowg[j];
    bval[i] = (uint32_t)j;
  }
}
// births and cluster rows from the scan of the birth flags (idx[m] = births);
// more rows than the bound marks the call failed
__global__ void k_cluster_counts(const uint32_t *idx, const uint64_t *m, int64_t G, int64_t R, uint64_t *hdr) {
  if (threadIdx.x != 0) return;
  uint64_t nb = idx[*m];
  if ((int64_t)(nb + G) > R) {  // (cannot happen: every birth has at least M records) stay in bounds
    hdr[H_STATUS] |= 64;
    nb = 0;
  }
  hdr[H_NB] = nb;
  hdr[H_NROWS] = nb + (uint64_t)G;
}
// one graph: its births are rows 0..nb-1
__global__ void k_bstart_one(uint32_t *bstart, const uint64_t *hdr) {
  if (threadIdx.x == 0) { bstart[0] = 0; bstart[1] = (uint32_t)hdr[H_NB]; }
}
__global__ __launch_bounds__(B) void k_birth_rows(const uint32_t *sorted_j, const uint32_t *rowg, Cnt nbc,
                                                  uint32_t *rowof) {
  const int64_t nb = nbc.get();
  for (int64_t p = (int64_t)blockIdx.x * B + threadIdx.x; p < nb; p += (int64_t)gridDim.x * B) {
    const uint32_t j = sorted_j[p];
    rowof[j] = (uint32_t)p + rowg[j];
  }
}
__global__ __launch_bounds__(B) void k_root_rows(const uint32_t *bstart, int64_t G, uint32_t *rootrow) {
  for (int64_t g = (int64_t)blockIdx.x * B + threadIdx.x; g < G; g += (int64_t)gridDim.x * B)
    rootrow[g] = bstart[g + 1] + (uint32_t)g;
}

// exact sums of 32-bit limbs into a row's three u64 accumulators: the lanes
// sharing the wave's first row are summed first (one round; the others add on
// their own), zero limbs are skipped
__device__ inline void add_limbs(bool active, uint32_t row, uint64_t l0, uint64_t l1, uint64_t l2,
                                 unsigned long long *acc) {
  const bool upd = wave_combine_first(active, row, [&](bool mine, int leader) {
    const uint64_t a0 = wave_sum_u64(mine ? l0 : 0ull), a1 = wave_sum_u64(mine ? l1 : 0ull),
                   a2 = wave_sum_u64(mine ? l2 : 0ull);
    if ((int)wave_lane() == leader) { l0 = a0; l1 = a1; l2 = a2; }
  });
  if (!upd) return;
  if (l0) atomicAdd(&acc[3 * (uint64_t)row], (unsigned long long)l0);
  if (l1) atomicAdd(&acc[3 * (uint64_t)row + 1], (unsigned long long)l1);
  if (l2) atomicAdd(&acc[3 * (uint64_t)row + 2], (unsigned long long)l2);
}

constexpr int AHS = 512;  // LDS hash slots for per-cluster-row sums

// Point term of each cluster's stability: the records of a small child c of
// a big row j all leave the cluster of j at lambda_j, so they add size(c) *
// lambda_j; summed per cluster row in an LDS hash, then one atomic per limb,
// row and tile.
__global__ __launch_bounds__(B) void k_cd_point_terms(const uint32_t *kc_u, const uint32_t *kc_v,
                                                      const uint32_t *ksize, const uint32_t *J, const uint64_t *rowL,
                                                      const uint32_t *rowof, const uint32_t *rootrow, Cnt mc,
                                                      int64_t n, int64_t M, int kct,
                                                      unsigned long long *acc) {
  __shared__ uint32_t hk[AHS];
  const int64_t m = mc.get();
  __shared__ unsigned long long h0[AHS], h1[AHS], h2[AHS];
  for (int i = threadIdx.x; i < AHS; i += B) { hk[i] = NONE32; h0[i] = 0; h1[i] = 0; h2[i] = 0; }
  __syncthreads();
  const int64_t tbase = (int64_t)blockIdx.x * (B * kct);
  for (int k = 0; k < kct; k++) {
    const int64_t j = tbase + (int64_t)k * B + threadIdx.x;
    uint32_t cnt = 0, r = 0;
    uint64_t L = 0;
    if (j < m && ksize[j] >= (uint64_t)M) {
      L = rowL[j];
      const uint32_t su = node_size(kc_u[j], n, ksize), sv = node_size(kc_v[j], n, ksize);
      cnt = (su < (uint64_t)M ? su : 0u) + (sv < (uint64_t)M ? sv : 0u);
      if (cnt && L) r = row_of(J[j], n, m, rowof, rootrow);
    }
    const bool act = cnt != 0 && L != 0;
    const u128 prod = u128_mul64(cnt, L);
    uint64_t s0 = prod.lo & 0xffffffffull, s1 = prod.lo >> 32, s2 = prod.hi;
    const bool upd = wave_combine_first(act, r, [&](bool mine, int leader) {
      const uint64_t a0 = wave_sum_u64(mine ? s0 : 0ull), a1 = wave_sum_u64(mine ? s1 : 0ull),
                     a2 = wave_sum_u64(mine ? s2 : 0ull);
      if ((int)wave_lane() == leader) { s0 = a0; s1 = a1; s2 = a2; }
    });
    if (upd) {
      uint32_t sl = (r * 2654435761u) >> 23;  // 9 bits
      bool placed = false;
      for (int probe = 0; probe < HASH_PROBES && !placed; probe++) {
        uint32_t old = atomicCAS(&hk[sl], NONE32, r);
        if (old == NONE32 || old == r) {
          atomicAdd(&h0[sl], (unsigned long long)s0);
          atomicAdd(&h1[sl], (unsigned long long)s1);
          atomicAdd(&h2[sl], (unsigned long long)s2);
          placed = true;
        } else {
          sl = (sl + 1) & (AHS - 1);
        }
      }
      if (!placed) {
        atomicAdd(&acc[3 * (uint64_t)r], (unsigned long long)s0);
        atomicAdd(&acc[3 * (uint64_t)r + 1], (unsigned long long)s1);
        atomicAdd(&acc[3 * (uint64_t)r + 2], (unsigned long long)s2);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < AHS; i += B) {
    uint32_t r = hk[i];
    if (r == NONE32) continue;
    if (h0[i]) atomicAdd(&acc[3 * (uint64_t)r], h0[i]);
    if (h1[i]) atomicAdd(&acc[3 * (uint64_t)r + 1], h1[i]);
    if (h2[i]) atomicAdd(&acc[3 * (uint64_t)r + 2], h2[i]);
  }
}

// One 8-byte word per row for the exit walk: (parent node, size) for a small
// row, (cluster row of its cluster, size) for a big one.
__global__ __launch_bounds__(B) void k_cd_walk_words(const uint32_t *kpar, const uint32_t *ksize, const uint32_t *J,
                                                     const uint32_t *rowof, const uint32_t *rootrow, int64_t n,
                                                     Cnt mc, int64_t M, uint2 *wk) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    const uint32_t sz = ksize[j];
    wk[j] = make_uint2(sz < (uint64_t)M ? kpar[n + j] : row_of(J[j], n, m, rowof, rootrow), sz);
  }
}

// Exit of every record, in input order: from its leaf, up through the small
// subtrees (fewer than M records, so fewer than M steps) to the first big
// row y; it leaves the cluster of y at lambda_y, or its graph's root at 0 when
// no big row is above it. Writes the exit cluster row and the exit lambda.
__global__ __launch_bounds__(B) void k_cd_exit_ids(const uint32_t *rankof, const uint32_t *kpar, const uint2 *wk,
                                                   const uint64_t *rowL, const uint32_t *grank,
                                                   const uint32_t *rootrow, int64_t n, int64_t M, uint32_t *prow,
                                                   const uint64_t *hdr, uint64_t *pt_lambda) {
  if (hdr[H_STATUS] != 0) pt_lambda = nullptr;  // a data error: no output is written
  for (int64_t id = (int64_t)blockIdx.x * B + threadIdx.x; id < n; id += (int64_t)gridDim.x * B) {
    const uint32_t p = rankof[id];
    uint32_t y = kpar[p], r = NONE32;
    while (y != NONE32) {
      const uint2 e = wk[y - n];
      if (e.y >= (uint64_t)M) {
        r = e.x;
        break;
      }
      y = e.x;
    }
    uint64_t L = 0;
    if (y == NONE32) r = rootrow[grank[p]];
    else L = rowL[y - n];
    prow[id] = r;
    if (pt_lambda) pt_lambda[id] = L;
  }
}

__global__ __launch_bounds__(B) void k_cd_acc_children(const uint32_t *csize, const uint64_t *cbirth,
                                                       const uint32_t *cprow, Cnt nrc,
                                                       unsigned long long *acc) {
  const int64_t nrows = nrc.get();
  int64_t r = (int64_t)blockIdx.x * B + threadIdx.x;
  bool act = r < (int64_t)nrows && cprow[r] != NONE32;
  uint32_t pr = 0;
  u128 prod{0, 0};
  if (act) {
    pr = cprow[r];
    prod = u128_mul64(csize[r], cbirth[r]);
  }
  add_limbs(act, pr, prod.lo & 0xffffffffull, prod.lo >> 32, prod.hi, acc);
}

// S = sum - size * birth  (exact u128)
__global__ __launch_bounds__(B) void k_cd_stab(const unsigned long long *acc, const uint32_t *csize,
                                               const uint64_t *cbirth, Cnt nrc, uint64_t *shi, uint64_t *slo) {
  const int64_t nrows = nrc.get();
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * B) {
    u128 t0{acc[3 * r], 0};
    u128 t1 = u128_mul64(acc[3 * r + 1], uint64_t(1) << 32);
    u128 t2{0, acc[3 * r + 2]};
    u128 T = u128_add(u128_add(t0, t1), t2);
    u128 S = u128_sub(T, u128_mul64(csize[r], cbirth[r]));
    shi[r] = S.hi;
    slo[r] = S.lo;
  }
}

// root rows are the rows without a parent
__global__ __launch_bounds__(B) void k_cd_children(const uint32_t *cprow, Cnt nrc, uint32_t *nch, uint32_t *ch) {
  const int64_t nrows = nrc.get();
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * B) {
    uint32_t p = cprow[r];
    if (p == NONE32 || cprow[p] == NONE32) continue;
    uint32_t k = atomicAdd(&nch[p], 1u);
    if (k < 2) ch[2 * (uint64_t)p + k] = (uint32_t)r;
  }
}

// More than two child clusters (discrete dendrogram): children listed per
// parent, then a parent with k children gets a chain of k-2 virtual nodes
// (rows nrows..) of stability 0, so that every node has at most two children
// and a virtual node's value max(0, x + y) is the plain sum of its two.
// child lists by a sort of the rows by parent (a parent can have millions of
// children, so no per-parent atomics); rows that are not children of a
// non-root cluster get the key nrows and sort last
__global__ __launch_bounds__(B) void k_cd_child_keys(const uint32_t *cprow, Cnt nrc, uint32_t *key) {
  const int64_t nrows = nrc.get();
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * B) {
    const uint32_t p = cprow[r];
    key[r] = (p == NONE32 || cprow[p] == NONE32) ? (uint32_t)nrows : p;
  }
}
__global__ __launch_bounds__(B) void k_cd_child_counts(const uint32_t *choff, Cnt nrc, uint32_t *nch,
                                                       uint32_t *vcnt) {
  const int64_t nrows = nrc.get();
  for (int64_t p = (int64_t)blockIdx.x * B + threadIdx.x; p < nrows; p += (int64_t)gridDim.x * B) {
    const uint32_t k = choff[p + 1] - choff[p];
    nch[p] = k;
    vcnt[p] = k > 2 ? k - 2 : 0u;
  }
}
// p -> (L0, L1), or with k > 2 children p -> (L0, v0) (virtual nodes below)
__global__ __launch_bounds__(B) void k_cd_pairs(const uint32_t *nch, const uint32_t *choff, const uint32_t *clist,
                                                const uint32_t *vbase, Cnt nrc, uint32_t *ch) {
  const int64_t nrows = nrc.get();
  for (int64_t p = (int64_t)blockIdx.x * B + threadIdx.x; p < nrows; p += (int64_t)gridDim.x * B) {
    const uint32_t k = nch[p];
    if (k == 0) continue;
    const uint32_t *L = clist + choff[p];
    ch[2 * p] = L[0];
    ch[2 * p + 1] = k > 2 ? (uint32_t)nrows + vbase[p] : (k == 2 ? L[1] : L[0]);
  }
}
// virtual node v (the i-th of parent p): v_i -> (L_{i+1}, v_{i+1}); the last
// one -> (L_{k-2}, L_{k-1}); its parent is the last p with vbase[p] <= v
__global__ __launch_bounds__(B) void k_cd_virtual(const uint32_t *nch, const uint32_t *choff, const uint32_t *clist,
                                                  const uint32_t *vbase, Cnt nrc, Cnt nvc,
                                                  uint32_t *ch, uint32_t *vnch, uint64_t *shi, uint64_t *slo) {
  const int64_t nrows = nrc.get(), nvirt = nvc.get();
  for (int64_t v = (int64_t)blockIdx.x * B + threadIdx.x; v < nvirt; v += (int64_t)gridDim.x * B) {
    int64_t lo = 0, hi = (int64_t)nrows - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if ((int64_t)vbase[mid] <= v) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t p = (uint32_t)lo, i = (uint32_t)(v - vbase[p]), k = nch[p];
    const uint32_t *L = clist + choff[p];
    const uint64_t node = nrows + (uint64_t)v;
    ch[2 * node] = L[i + 1];
    ch[2 * node + 1] = (i + 3 < k) ? (uint32_t)(node + 1) : L[k - 1];
    vnch[node] = 2;
    shi[node] = 0;
    slo[node] = 0;
  }
}

// EOM state per row: st = 0 pending-binary, 1 pending-unary, 2 done
struct Eom {
  uint8_t *st;
  uint64_t *vhi, *vlo;  // value when done
  uint64_t *ahi, *alo, *bhi, *blo;  // unary f(x) = max(a, x + b)
  uint32_t *dep;
};

constexpr uint32_t COPY = 0x80000000u;  // list item flag: finished last round, copy state across buffers

__device__ inline void eom_store(const Eom &o, uint32_t r, uint8_t st, u128 v, u128 a, u128 bb, uint32_t dep) {
  o.st[r] = st;
  o.vhi[r] = v.hi; o.vlo[r] = v.lo;
  o.ahi[r] = a.hi; o.alo[r] = a.lo;
  o.bhi[r] = bb.hi; o.blo[r] = bb.lo;
  o.dep[r] = dep;
}

__global__ __launch_bounds__(B) void k_eom_init(const uint32_t *nch, const uint64_t *shi, const uint64_t *slo,
                                                const uint32_t *cprow, Cnt nrc, Cnt nec, Eom e0,
                                                Eom e1, uint32_t *act, unsigned long long *nact) {
  const int64_t nreal = nrc.get(), nrows = nec.get();
  const int ct = tile_items(nrows);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < nrows; tile += gridDim.x) {
    bool keep[CT];
    uint32_t vals[CT];
    const int64_t base = tile * (B * ct) + threadIdx.x, end = tile_end(nrows, tile, B * ct);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      const int64_t r = base + (int64_t)k * B;
      keep[k] = false;
      vals[k] = (uint32_t)r;
      if (r >= end) continue;
      // rows from nreal on are virtual sum nodes, never leaves
      bool leaf = r < nreal && (nch[r] == 0 || cprow[r] == NONE32);
      u128 S{slo[r], shi[r]}, z{0, 0};
      eom_store(e0, (uint32_t)r, leaf ? 2 : 0, S, z, z, NONE32);
      eom_store(e1, (uint32_t)r, leaf ? 2 : 0, S, z, z, NONE32);
      keep[k] = !leaf;
    }
    tile_append(keep, vals, act, nact);
  }
}

// One round over the pending rows: rake (both children done), turn into a
// unary f(x) = max(a, x + b) when one child is done, or compose along a chain
// of unary rows (pointer jumping). Reads `in`, writes `out`. A row that
// finishes goes once more to the next list, flagged COPY, so that both state
// buffers hold its final value; when the list is empty they agree everywhere.
__device__ inline bool eom_step(uint32_t item, const Eom &in, const Eom &out, const uint32_t *ch,
                                const uint64_t *shi, const uint64_t *slo, uint32_t *val) {
  const uint32_t r = item & ~COPY;
  uint8_t st = in.st[r];
  u128 v{in.vlo[r], in.vhi[r]}, a{in.alo[r], in.ahi[r]}, bb{in.blo[r], in.bhi[r]};
  uint32_t dep = in.dep[r];
  if (item & COPY) {
    eom_store(out, r, st, v, a, bb, dep);
    return false;
  }
  if (st == 0) {
    uint32_t c1 = ch[2 * (uint64_t)r], c2 = ch[2 * (uint64_t)r + 1];
    bool d1 = in.st[c1] == 2, d2 = in.st[c2] == 2;
    u128 S{slo[r], shi[r]};
    if (d1 && d2) {
      v = u128_max(S, u128_add(u128{in.vlo[c1], in.vhi[c1]}, u128{in.vlo[c2], in.vhi[c2]}));
      st = 2;
    } else if (d1 || d2) {
      uint32_t dn = d1 ? c1 : c2, pn = d1 ? c2 : c1;
      a = S;
      bb = u128{in.vlo[dn], in.vhi[dn]};
      dep = pn;
      st = 1;
    }
  } else if (st == 1) {
    uint8_t ds = in.st[dep];
    if (ds == 2) {
      v = u128_max(a, u128_add(u128{in.vlo[dep], in.vhi[dep]}, bb));
      st = 2;
    } else if (ds == 1) {
      u128 ad{in.alo[dep], in.ahi[dep]}, bd{in.blo[dep], in.bhi[dep]};
      a = u128_max(a, u128_add(ad, bb));
      bb = u128_add(bd, bb);
      dep = in.dep[dep];
    }
  }
  eom_store(out, r, st, v, a, bb, dep);
  *val = st == 2 ? (r | COPY) : r;
  return true;
}

__global__ __launch_bounds__(B) void k_eom_round(const uint32_t *act, const uint64_t *nact_in, Eom in, Eom out,
                                                 const uint32_t *ch, const uint64_t *shi, const uint64_t *slo,
                                                 uint32_t *next, unsigned long long *nnext) {
  const int64_t nact = (int64_t)*nact_in;
  const int ct = tile_items(nact);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < nact; tile += gridDim.x) {
    bool keep[CT];
    uint32_t vals[CT];
    const int64_t base = tile * (B * ct) + threadIdx.x, end = tile_end(nact, tile, B * ct);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      const int64_t i = base + (int64_t)k * B;
      keep[k] = false;
      vals[k] = 0;
      if (i < end) keep[k] = eom_step(act[i], in, out, ch, shi, slo, &vals[k]);
    }
    tile_append(keep, vals, next, nnext);
  }
}

// The rounds left after the enqueued ones, in one workgroup: lists and state
// buffers alternate as in the grid rounds (the state of round `parity` is
// read first); it stops when the list is empty. A round count beyond any
// tree marks the call failed.
constexpr int TB = 1024;
__global__ __launch_bounds__(TB) void k_eom_tail(uint32_t *l0, uint32_t *l1, const uint64_t *nact_in, int parity,
                                                 Eom e0, Eom e1, const uint32_t *ch, const uint64_t *shi,
                                                 const uint64_t *slo, uint64_t *hdr) {
  __shared__ uint32_t s_cnt;
  int64_t nact = (int64_t)*nact_in;
  int cur = parity;
  for (uint32_t round = 0; nact > 0; round++) {
    if (round > (1u << 20)) {
      if (threadIdx.x == 0) atomicOr((unsigned long long *)&hdr[H_STATUS], 32ull);
      return;
    }
    const uint32_t *in_list = cur ? l1 : l0;
    uint32_t *out_list = cur ? l0 : l1;
    const Eom &in = cur ? e1 : e0, &out = cur ? e0 : e1;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < nact; i += TB) {
      uint32_t v;
      if (eom_step(in_list[i], in, out, ch, shi, slo, &v)) out_list[atomicAdd(&s_cnt, 1u)] = v;
    }
    __threadfence_block();
    __syncthreads();
    nact = s_cnt;
    cur ^= 1;
    __syncthreads();
  }
}

// selection with ties kept by the parent; ROOT never selected
__global__ __launch_bounds__(B) void k_eom_select(const uint32_t *nch, const uint32_t *ch, Eom e, const uint64_t *shi,
                                                  const uint64_t *slo, Cnt nrc, uint32_t *top, uint32_t *nxt,
                                                  uint32_t *top2, uint32_t *nxt2, const uint32_t *cprow, uint32_t *act,
                                                  unsigned long long *nact) {
  const int64_t nrows = nrc.get();
  const int ct = tile_items(nrows);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < nrows; tile += gridDim.x) {
    bool keep[CT];
    uint32_t vals[CT];
    const int64_t base = tile * (B * ct) + threadIdx.x, end = tile_end(nrows, tile, B * ct);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      const int64_t r = base + (int64_t)k * B;
      keep[k] = false;
      vals[k] = (uint32_t)r;
      if (r >= end) continue;
      bool sel;
      if (cprow[r] == NONE32) sel = false;
      else if (nch[r] == 0) sel = true;
      else {
        uint32_t c1 = ch[2 * r], c2 = ch[2 * r + 1];
        u128 sum = u128_add(u128{e.vlo[c1], e.vhi[c1]}, u128{e.vlo[c2], e.vhi[c2]});
        sel = !u128_gt(sum, u128{slo[r], shi[r]});
      }
      uint32_t t = sel ? (uint32_t)r : NONE32;
      uint32_t p = cprow[r];
      uint32_t nx = (p == NONE32 || cprow[p] == NONE32) ? NONE32 : p;
      top[r] = t; top2[r] = t;
      nxt[r] = nx; nxt2[r] = nx;
      keep[k] = nx != NONE32;
    }
    tile_append(keep, vals, act, nact);
  }
}

// top[r] = highest selected row among r and its ancestors below ROOT
// (pointer doubling over (top, nxt); a row that finishes goes once more to the
// next list, flagged COPY, so both buffers agree when the list is empty)
__device__ inline bool top_step(uint32_t item, const uint32_t *tin, const uint32_t *nin, uint32_t *tout,
                                uint32_t *nout, uint32_t *val) {
  const uint32_t r = item & ~COPY;
  uint32_t nx = nin[r], t = tin[r];
  if (item & COPY) {
    tout[r] = t;
    nout[r] = nx;
    return false;
  }
  uint32_t tv = tin[nx];
  if (tv != NONE32) t = tv;
  nx = nin[nx];
  tout[r] = t;
  nout[r] = nx;
  *val = nx == NONE32 ? (r | COPY) : r;
  return true;
}

__global__ __launch_bounds__(B) void k_top_jump(const uint32_t *act, const uint64_t *nact_in, const uint32_t *tin,
                                                const uint32_t *nin, uint32_t *tout, uint32_t *nout, uint32_t *next,
                                                unsigned long long *nnext) {
  const int64_t nact = (int64_t)*nact_in;
  const int ct = tile_items(nact);
  for (int64_t tile = blockIdx.x; tile * (B * ct) < nact; tile += gridDim.x) {
    bool keep[CT];
    uint32_t vals[CT];
    const int64_t base = tile * (B * ct) + threadIdx.x, end = tile_end(nact, tile, B * ct);
#pragma unroll
    for (int k = 0; k < CT; k++) {
      const int64_t i = base + (int64_t)k * B;
      keep[k] = false;
      vals[k] = 0;
      if (i < end) keep[k] = top_step(act[i], tin, nin, tout, nout, &vals[k]);
    }
    tile_append(keep, vals, next, nnext);
  }
}

__global__ __launch_bounds__(TB) void k_top_tail(uint32_t *l0, uint32_t *l1, const uint64_t *nact_in, int parity,
                                                 uint32_t *top, uint32_t *nxt, uint32_t *top2, uint32_t *nxt2,
                                                 uint64_t *hdr) {
  __shared__ uint32_t s_cnt;
  int64_t nact = (int64_t)*nact_in;
  int cur = parity;
  for (uint32_t round = 0; nact > 0; round++) {
    if (round > (1u << 20)) {
      if (threadIdx.x == 0) atomicOr((unsigned long long *)&hdr[H_STATUS], 32ull);
      return;
    }
    const uint32_t *in_list = cur ? l1 : l0;
    uint32_t *out_list = cur ? l0 : l1;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < nact; i += TB) {
      uint32_t v;
      const bool keep = cur ? top_step(in_list[i], top2, nxt2, top, nxt, &v)
                            : top_step(in_list[i], top, nxt, top2, nxt2, &v);
      if (keep) out_list[atomicAdd(&s_cnt, 1u)] = v;
    }
    __threadfence_block();
    __syncthreads();
    nact = s_cnt;
    cur ^= 1;
    __syncthreads();
  }
}

// the smallest input id under each label (records in input order)
__global__ __launch_bounds__(B) void k_lab_rows(const uint32_t *prow, const uint32_t *top, const uint32_t *cprow,
                                                int64_t n, uint32_t *minmem) {
  for (int64_t id = (int64_t)blockIdx.x * B + threadIdx.x; id < n; id += (int64_t)gridDim.x * B) {
    const uint32_t r = prow[id];
    const uint32_t lr = cprow[r] == NONE32 ? NONE32 : top[r];
    if (lr != NONE32) atomicMin(&minmem[lr], (uint32_t)id);
  }
}

__global__ __launch_bounds__(B) void k_lab_flags(const uint32_t *top, const uint32_t *minmem, Cnt nrc,
                                                 uint32_t *flag) {
  const int64_t nrows = nrc.get();
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * B)
    if (top[r] == (uint32_t)r && minmem[r] != NONE32) flag[minmem[r]] = 1;
}

// node id inside its own graph: records keep their local ids; row j of graph g
// is node n_g + (its index among g's rows); the root of g is n_g + m_g
__device__ inline uint32_t local_node(uint32_t x, uint32_t g, int64_t n, int64_t m, const int64_t *eoff,
                                      const uint32_t *moff, const uint32_t *rowpos) {
  const uint32_t ng = (uint32_t)(eoff[g + 1] - eoff[g]);
  if (x >= (uint64_t)(n + m)) return ng + (moff[g + 1] - moff[g]);
  return ng + (rowpos[x - n] - moff[g]);
}

// per record, in input order: its exit row's node and label
__global__ __launch_bounds__(B) void k_out_points(const uint32_t *prow, const uint32_t *rlocal, const int32_t *rlab,
                                                  int64_t n, const uint64_t *hdr, uint32_t *pt_cluster,
                                                  int32_t *labels) {
  if (hdr[H_STATUS] != 0) return;  // a data error: no output is written
  for (int64_t id = (int64_t)blockIdx.x * B + threadIdx.x; id < n; id += (int64_t)gridDim.x * B) {
    const uint32_t r = prow[id];
    if (pt_cluster) pt_cluster[id] = rlocal[r];
    if (labels) labels[id] = rlab[r];
  }
}

__global__ __launch_bounds__(B) void k_out_clusters(const uint32_t *cnode, const uint32_t *cprow,
                                                    const uint32_t *csize, const uint64_t *cbirth,
                                                    const uint64_t *shi, const uint64_t *slo, const uint32_t *top,
                                                    const uint32_t *rowg, const int64_t *eoff, const uint32_t *moff,
                                                    const uint32_t *rowpos, int64_t n, Cnt mc, Cnt nrc,
                                                    const uint64_t *hdr, ce_result out) {
  if (hdr[H_STATUS] != 0) return;
  const int64_t m = mc.get(), nrows = nrc.get();
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * B) {
    const uint32_t c = cnode[r];
    const uint32_t g = c >= (uint64_t)(n + m) ? (uint32_t)(c - n - m) : rowg[c - n];
    if (out.cl_id) out.cl_id[r] = local_node(c, g, n, m, eoff, moff, rowpos);
    if (out.cl_parent)
      out.cl_parent[r] = cprow[r] == NONE32 ? NONE32 : local_node(cnode[cprow[r]], g, n, m, eoff, moff, rowpos);
    if (out.cl_size) out.cl_size[r] = csize[r];
    if (out.cl_lambda_birth) out.cl_lambda_birth[r] = cbirth[r];
    if (out.cl_stab_hi) out.cl_stab_hi[r] = shi[r];
    if (out.cl_stab_lo) out.cl_stab_lo[r] = slo[r];
    if (out.cl_selected) out.cl_selected[r] = (cprow[r] != NONE32 && top[r] == (uint32_t)r) ? 1 : 0;
  }
}

// discrete dendrogram per output row: level, and the row's D-node as a node id
__global__ __launch_bounds__(B) void k_out_discrete(const uint32_t *level, const uint32_t *top, const uint32_t *rowg,
                                                    const int64_t *eoff, const uint32_t *moff, const uint32_t *rowpos,
                                                    int64_t n, Cnt mc, uint32_t *dd_level, uint32_t *dd_top) {
  const int64_t m = mc.get();
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    const uint32_t g = rowg[j], p = rowpos[j];
    if (dd_level) dd_level[p] = level[j];
    if (dd_top) dd_top[p] = local_node(top[j], g, n, m, eoff, moff, rowpos);
  }
}

// labels per graph: the chosen clusters whose minimum member lies in g
// what a record exiting at cluster row r reports: the row's node in its
// graph's local ids, and the label of its selected ancestor (-1 if none)
__global__ __launch_bounds__(B) void k_row_point_vals(const uint32_t *cnode, const uint32_t *cprow,
                                                      const uint32_t *top, const uint32_t *minmem,
                                                      const uint32_t *fscan, const uint32_t *rowg,
                                                      const int64_t *eoff, const uint32_t *moff,
                                                      const uint32_t *rowpos, int64_t n, Cnt mc, Cnt nrc,
                                                      uint32_t *rlocal, int32_t *rlab) {
  const int64_t m = mc.get(), nrows = nrc.get();
  for (int64_t r = (int64_t)blockIdx.x * B + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * B) {
    const uint32_t c = cnode[r];
    const uint32_t g = c >= (uint64_t)(n + m) ? (uint32_t)(c - n - m) : rowg[c - n];
    rlocal[r] = local_node(c, g, n, m, eoff, moff, rowpos);
    const uint32_t lr = cprow[r] == NONE32 ? NONE32 : top[r];
    const uint32_t mm = lr == NONE32 ? NONE32 : minmem[lr];
    rlab[r] = mm == NONE32 ? -1 : (int32_t)(fscan[mm] - fscan[eoff[g]]);
  }
}

__global__ __launch_bounds__(B) void k_graph_labels(const uint32_t *fscan, const int64_t *eoff, int64_t G,
                                                    uint32_t *nl) {
  for (int64_t g = (int64_t)blockIdx.x * B + threadIdx.x; g < G; g += (int64_t)gridDim.x * B)
    nl[g] = fscan[eoff[g + 1]] - fscan[eoff[g]];
}

// per-graph counts and offsets of the call (its header): total and per-graph
// rows, cluster rows and labels, row and cluster offsets; the status from the
// error bits. Cluster rows of graph g start at bstart[g] + g (births, then its root).
__global__ __launch_bounds__(B) void k_header(const uint64_t *hdr, int64_t G, const uint32_t *moff,
                                              const uint32_t *bstart, const uint32_t *nlab, int64_t *out) {
  for (int64_t g = (int64_t)blockIdx.x * B + threadIdx.x; g <= G; g += (int64_t)gridDim.x * B) {
    if (g == 0) {
      uint64_t labels = 0;
      for (int64_t k = 0; k < G; k++) labels += nlab[k];
      out[0] = status_of(hdr[H_STATUS]);
      out[1] = moff[G];
      out[2] = (int64_t)bstart[G] + G;
      out[3] = (int64_t)labels;
    }
    if (g < G) {
      out[4 + 3 * g] = (int64_t)moff[g + 1] - moff[g];
      out[4 + 3 * g + 1] = (int64_t)bstart[g + 1] - bstart[g] + 1;
      out[4 + 3 * g + 2] = nlab[g];
    }
    out[4 + 3 * G + g] = moff[g];
    out[4 + 3 * G + (G + 1) + g] = (int64_t)bstart[g] + g;
  }
}

// virtual sum nodes of the discrete condensing (vbase[nrows]) and the EOM rows
__global__ void k_virtual_counts(const uint32_t *vbase, uint64_t *hdr, int64_t RE) {
  if (threadIdx.x != 0) return;
  const uint64_t nrows = hdr[H_NROWS];
  uint64_t nv = vbase[nrows];
  if ((int64_t)(nrows + nv) > RE) {  // (cannot happen: at most one virtual node per row) stay in bounds
    hdr[H_STATUS] |= 64;
    nv = 0;
  }
  hdr[H_NVIRT] = nv;
  hdr[H_NEOM] = nrows + nv;
}
__global__ void k_eom_count(uint64_t *hdr) {
  if (threadIdx.x == 0) hdr[H_NEOM] = hdr[H_NROWS];
}

}  // namespace

// Rounds of a pointer-doubling loop over a tree of up to k rows: bits(k) + 1
// end it; one more is a margin.
static int doubling_rounds(int64_t k) { return bits_for((uint64_t)k) + 2; }

// level tops (pointer doubling over same-level parents) and big children per
// D-node, then births; act and act2 hold m + 1 entries each, loop is the
// counter words of the rounds
static ce_status discrete_births(Bufs &b, Cnt m, const uint32_t *kpar, const uint32_t *level, const uint64_t *rowL,
                                 uint32_t *top, uint32_t *act, uint32_t *act2, uint64_t *loop, uint32_t *bigcnt,
                                 uint8_t *isbirth, uint64_t *birthL, hipStream_t s) {
  const int64_t n = b.n, M = b.M;
  const unsigned g = grid_cap(m.v, B), tg = grid_cap(m.v, B, tuning().list_grid);
  auto tiles = [](int64_t k, int per = CT) { return (unsigned)((k + (int64_t)B * per - 1) / ((int64_t)B * per)); };
  CE_LAUNCH(k_dd_top_init, dim3(g), dim3(B), 0, s, kpar, level, m, n, top);
  CE_LAUNCH(k_dd_top_active, dim3(tg), dim3(B), 0, s, top, m, n, act, (unsigned long long *)&loop[0]);
  const int R = doubling_rounds(m.v);
  uint32_t *lists[2] = {act, act2};
  for (int r = 0; r < R; r++)
    CE_LAUNCH(k_dd_top_jump, dim3(tg), dim3(B), 0, s, lists[r & 1], &loop[r], n, top, lists[1 - (r & 1)],
              (unsigned long long *)&loop[r + 1]);
  CE_LAUNCH(k_loop_done, dim3(1), dim3(64), 0, s, &loop[R], b.hdr);
  CE_LAUNCH(k_fill32, dim3(g), dim3(B), 0, s, bigcnt, m.v, 0u);
  const int kb = items_per_thread(m.v, B);
  CE_LAUNCH(k_dd_bigcount, dim3(tiles(m.v, kb)), dim3(B), 0, s, kpar, b.ksize, top, m, n, M, kb, bigcnt);
  CE_LAUNCH(k_dd_birth, dim3(g), dim3(B), 0, s, kpar, b.ksize, top, bigcnt, rowL, m, n, M, isbirth, birthL);
  CE_HIP(hipGetLastError());
  return CE_OK;
}

static int64_t cluster_row_bound(int64_t n, int64_t M, int64_t G) { return 2 * (n / M) + G + 1; }

size_t stage_condense_scratch(int64_t n, int64_t M, int64_t G, bool discrete) {
  const int64_t m = n, R = cluster_row_bound(n, M < 2 ? 2 : M, G), RE = discrete ? 2 * R : R;
  Ws w;
  w.alloc<uint32_t>(n + m + 1);  // kpar
  w.alloc<uint32_t>(m + 1); w.alloc<uint32_t>(m + 1); w.alloc<uint32_t>(m + 1);  // J, active lists
  w.alloc<uint8_t>(m + 4);       // isbirth
  w.alloc<uint64_t>(m + 1);      // birthL
  w.alloc<uint64_t>(m + 1);      // rowL (the discrete arrays reuse exc, exl, labrow and fl)
  w.alloc<uint32_t>(m + 2); w.alloc<uint32_t>(m + 2); w.alloc<uint32_t>(m + 1);  // flags32, idx, rowof
  for (int k = 0; k < 3; k++) w.alloc<uint32_t>(G + 2);  // nbig, bstart, rootrow
  w.alloc<uint32_t>(G + 1);  // labels per graph
  for (int k = 0; k < 4; k++) w.alloc<uint32_t>(R);  // birth sort keys/values
  w.alloc<uint32_t>(n); w.alloc<uint64_t>(n);  // exc exl
  w.alloc<uint32_t>(R); w.alloc<uint32_t>(R); w.alloc<uint64_t>(R); w.alloc<uint32_t>(R);  // cnode csize cbirth cprow
  w.alloc<uint64_t>(3 * R);  // acc
  w.alloc<uint64_t>(RE); w.alloc<uint64_t>(RE);  // shi slo (and virtual nodes)
  w.alloc<uint32_t>(RE); w.alloc<uint32_t>(2 * RE);  // nch ch
  if (discrete)
    for (int k = 0; k < 6; k++) w.alloc<uint32_t>(R + 1);  // child keys and lists (x2), offsets, virtual bases
  for (int k = 0; k < 2; k++) {
    w.alloc<uint8_t>(RE);
    for (int q = 0; q < 6; q++) w.alloc<uint64_t>(RE);
    w.alloc<uint32_t>(RE);
  }
  for (int k = 0; k < 4; k++) w.alloc<uint32_t>(R);  // top nxt x2
  w.alloc<uint32_t>(R);  // minmem
  w.alloc<uint32_t>(RE); w.alloc<uint32_t>(RE);  // row active lists
  w.alloc<uint32_t>(n);  // labrow
  w.alloc<uint32_t>(n + 1);  // flag / scan
  return w.off + scan_ws_bytes(n + 1) + scan_ws_bytes(m + 1) + scan_ws_bytes(G + 1) + scan_ws_bytes(R + 1) +
         radix_ws_bytes(R) + 8192;
}

// Grid rounds of the excess-of-mass and label pointer-jumping loops that the
// host enqueues for R cluster rows; what is left after them runs in one
// workgroup. Pointer doubling over a tree of R rows ends within bits(R) + 1
// rounds; the excess-of-mass rounds also rake, and measured runs end within
// about bits(R) + 2.
static int eom_rounds(int64_t R) { return bits_for((uint64_t)R) + 4; }
static int top_rounds(int64_t R) { return bits_for((uint64_t)R) + 2; }
// counter words of the bounded loops (from H_LOOP): level tops, J, excess of mass, label tops
constexpr int LOOP_DD = 0, LOOP_J = 40, LOOP_EOM = 80, LOOP_TOP = 130, LOOP_END = kHdrWords - H_LOOP;

// Sizes: m rows (device word, bound n - 1), nb births and nrows = nb + G
// cluster rows, nvirt virtual nodes (device words, bounds from R).
ce_status stage_condense(Bufs &b, const ce_result *out, Ws &ws, hipStream_t s, int64_t *hout) {
  const int64_t n = b.n, M = b.M, G = b.G, mb = n > 1 ? n - 1 : 1;
  const Cnt m(&b.hdr[H_M], mb);
  size_t m0 = ws.mark();
  const int64_t R = cluster_row_bound(n, M, G), RE = b.q > 0 ? 2 * R : R;
  const Cnt nb(&b.hdr[H_NB], R), nrows(&b.hdr[H_NROWS], R), nvirt(&b.hdr[H_NVIRT], R), neom(&b.hdr[H_NEOM], RE);
  uint32_t *kpar = ws.alloc<uint32_t>(n + mb + 1);
  uint32_t *J = ws.alloc<uint32_t>(mb + 1);
  uint32_t *jact = ws.alloc<uint32_t>(mb + 1), *jact2 = ws.alloc<uint32_t>(mb + 1);
  uint8_t *isbirth = ws.alloc<uint8_t>(mb + 4);
  uint64_t *birthL = ws.alloc<uint64_t>(mb + 1);
  uint64_t *rowL = ws.alloc<uint64_t>(mb + 1);
  uint32_t *flags32 = ws.alloc<uint32_t>(mb + 2), *idx = ws.alloc<uint32_t>(mb + 2), *rowof = ws.alloc<uint32_t>(mb + 1);
  uint32_t *nbig = ws.alloc<uint32_t>(G + 2), *bstart = ws.alloc<uint32_t>(G + 2);
  uint32_t *rootrow = ws.alloc<uint32_t>(G + 2);
  uint32_t *nlab = ws.alloc<uint32_t>(G + 1);
  uint32_t *bkey = ws.alloc<uint32_t>(R), *bval = ws.alloc<uint32_t>(R);
  uint32_t *bkey2 = ws.alloc<uint32_t>(R), *bval2 = ws.alloc<uint32_t>(R);
  uint32_t *exc = ws.alloc<uint32_t>(n);
  uint64_t *exl = ws.alloc<uint64_t>(n);
  uint32_t *cnode = ws.alloc<uint32_t>(R), *csize = ws.alloc<uint32_t>(R);
  uint64_t *cbirth = ws.alloc<uint64_t>(R);
  uint32_t *cprow = ws.alloc<uint32_t>(R);
  unsigned long long *acc = ws.alloc<unsigned long long>(3 * R);
  uint64_t *shi = ws.alloc<uint64_t>(RE), *slo = ws.alloc<uint64_t>(RE);
  uint32_t *nch = ws.alloc<uint32_t>(RE), *ch = ws.alloc<uint32_t>(2 * RE);
  uint32_t *choff = nullptr, *ckey = nullptr, *ckey2 = nullptr, *clist = nullptr, *clist2 = nullptr,
           *vbase = nullptr;
  if (b.q > 0) {
    choff = ws.alloc<uint32_t>(R + 1);
    ckey = ws.alloc<uint32_t>(R + 1);
    ckey2 = ws.alloc<uint32_t>(R + 1);
    clist = ws.alloc<uint32_t>(R + 1);
    clist2 = ws.alloc<uint32_t>(R + 1);
    vbase = ws.alloc<uint32_t>(R + 1);
  }
  Eom e[2];
  for (int k = 0; k < 2; k++) {
    e[k].st = ws.alloc<uint8_t>(RE);
    e[k].vhi = ws.alloc<uint64_t>(RE); e[k].vlo = ws.alloc<uint64_t>(RE);
    e[k].ahi = ws.alloc<uint64_t>(RE); e[k].alo = ws.alloc<uint64_t>(RE);
    e[k].bhi = ws.alloc<uint64_t>(RE); e[k].blo = ws.alloc<uint64_t>(RE);
    e[k].dep = ws.alloc<uint32_t>(RE);
  }
  uint32_t *top = ws.alloc<uint32_t>(R), *nxt = ws.alloc<uint32_t>(R);
  uint32_t *top2 = ws.alloc<uint32_t>(R), *nxt2 = ws.alloc<uint32_t>(R);
  uint32_t *minmem = ws.alloc<uint32_t>(R);
  uint32_t *ract = ws.alloc<uint32_t>(RE), *ract2 = ws.alloc<uint32_t>(RE);
  uint32_t *labrow = ws.alloc<uint32_t>(n);
  uint32_t *fl = ws.alloc<uint32_t>(n + 1);
  CE_WS_CHECK(ws);
  // discrete dendrogram: level, level tops and big-child counts per row live only until the
  // births are known and the per-row discrete outputs written, before exits, labels and flags use these
  uint32_t *level = exc, *dtop = labrow, *bigcnt = (uint32_t *)exl;
  auto tiles = [](int64_t k, int per = CT) { return (unsigned)((k + (int64_t)B * per - 1) / ((int64_t)B * per)); };
  uint64_t *loop = b.hdr + H_LOOP;  // counters of the bounded loops, zero from the start of the call

  const unsigned gN = grid_cap(n + mb + 1, B), gm = grid_cap(mb + 1, B), gG = grid_for(G + 1, B),
                 gR = grid_cap(R, B), gRE = grid_cap(RE, B);
  CE_LAUNCH(k_fill32, dim3(gN), dim3(B), 0, s, kpar, n + mb + 1, NONE32);
  CE_LAUNCH(k_fill32, dim3(gG), dim3(B), 0, s, nbig, G + 1, 0u);
  CE_LAUNCH(k_cd_parents, dim3(gm), dim3(B), 0, s, b.kc_u, b.kc_v, m, n, kpar);
  CE_LAUNCH(k_cd_bigroots, dim3(gm), dim3(B), 0, s, kpar, b.ksize, b.rowg, m, n, M, nbig);
  CE_LAUNCH(k_fill32, dim3(grid_cap((mb + 4) / 4, B)), dim3(B), 0, s, (uint32_t *)isbirth, (mb + 4) / 4, 0u);
  CE_HIP(hipGetLastError());
  CE_LAUNCH(k_row_lambda, dim3(gm), dim3(B), 0, s, b.msf_key, m, b.thr, b.q, rowL, level);
  CE_LAUNCH(k_cd_birth, dim3(gm), dim3(B), 0, s, b.kc_u, b.kc_v, b.ksize, kpar, rowL, b.q > 0, m, n, M, nbig, b.rowg,
            isbirth, birthL);
  CE_HIP(hipGetLastError());
  if (b.q > 0) {
    CE_TRY(discrete_births(b, m, kpar, level, rowL, dtop, jact, jact2, loop + LOOP_DD, bigcnt, isbirth, birthL, s));
    if (out->dd_level || out->dd_top)
      CE_LAUNCH(k_out_discrete, dim3(gm), dim3(B), 0, s, level, dtop, b.rowg, b.eoff, b.moff, b.rowpos, n, m,
                out->dd_level, out->dd_top);
    CE_HIP(hipGetLastError());
  }
  {
    uint64_t *jl = loop + LOOP_J;
    const unsigned tg = grid_cap(mb, B, tuning().list_grid);
    CE_LAUNCH(k_cd_jinit, dim3(tg), dim3(B), 0, s, isbirth, kpar, b.ksize, b.rowg, m, n, M, J, jact,
              (unsigned long long *)&jl[0]);
    const int R = doubling_rounds(mb);
    uint32_t *lists[2] = {jact, jact2};
    for (int r = 0; r < R; r++)
      CE_LAUNCH(k_cd_jstep, dim3(tg), dim3(B), 0, s, lists[r & 1], &jl[r], J, isbirth, m, n, lists[1 - (r & 1)],
                (unsigned long long *)&jl[r + 1]);
    CE_LAUNCH(k_loop_done, dim3(1), dim3(64), 0, s, &jl[R], b.hdr);
  }
  // cluster rows: births in (graph, node) order, each graph followed by its root row
  CE_LAUNCH(k_u8_to_u32, dim3(gm), dim3(B), 0, s, isbirth, m, flags32);
  CE_HIP(hipGetLastError());
  CE_TRY(scan_exclusive_u32(flags32, idx, m, ws, s));
  CE_LAUNCH(k_cluster_counts, dim3(1), dim3(64), 0, s, idx, &b.hdr[H_M], G, R, b.hdr);
  const uint32_t *rowmap = idx;  // one graph: a birth's row is its index among births
  if (G == 1) {
    CE_LAUNCH(k_bstart_one, dim3(1), dim3(64), 0, s, bstart, b.hdr);
  } else {
    CE_LAUNCH(k_birth_list, dim3(gm), dim3(B), 0, s, isbirth, idx, b.rowg, m, bkey, bval);
    CE_HIP(hipGetLastError());
    bool alt = false;
    CE_TRY((radix_sort_pairs<uint32_t, uint32_t>(bkey, bval, bkey2, bval2, nb, 0, bits_for((uint64_t)(G - 1)), false,
                                                 &alt, ws, s)));
    CE_LAUNCH(k_birth_rows, dim3(gR), dim3(B), 0, s, alt ? bval2 : bval, b.rowg, nb, rowof);
    CE_TRY(segment_bounds_u32(alt ? bkey2 : bkey, nb, Cnt(G), bstart, s));
    rowmap = rowof;
  }
  CE_HIP(hipGetLastError());
  CE_LAUNCH(k_root_rows, dim3(gG), dim3(B), 0, s, bstart, G, rootrow);
  CE_LAUNCH(k_cd_rows, dim3(gm), dim3(B), 0, s, isbirth, rowmap, rootrow, b.ksize, birthL, kpar, J, b.rowg, m, n,
            cnode, csize, cbirth, cprow);
  CE_LAUNCH(k_cd_rootrows, dim3(gG), dim3(B), 0, s, rootrow, b.eoff, G, m, n, cnode, csize, cbirth, cprow);
  CE_LAUNCH(k_fill64, dim3(grid_cap(3 * R, B)), dim3(B), 0, s, (uint64_t *)acc, 3 * R, (uint64_t)0);
  // point terms of the stabilities per big row; exits per record in input order
  const int kp = items_per_thread(mb, B);
  CE_LAUNCH(k_cd_point_terms, dim3(tiles(mb, kp)), dim3(B), 0, s, b.kc_u, b.kc_v, b.ksize, J, rowL, rowmap, rootrow, m,
            n, M, kp, acc);
  uint32_t *prow = labrow;
  uint2 *wk = (uint2 *)exl;  // m <= n words of 8 bytes
  CE_LAUNCH(k_cd_walk_words, dim3(gm), dim3(B), 0, s, kpar, b.ksize, J, rowmap, rootrow, n, m, M, wk);
  CE_LAUNCH(k_cd_exit_ids, dim3(grid_cap(n, B)), dim3(B), 0, s, b.rankof, kpar, wk, rowL, b.grank, rootrow, n, M,
            prow, b.hdr, out->pt_lambda);
  CE_LAUNCH(k_cd_acc_children, dim3((unsigned)((R + B - 1) / B)), dim3(B), 0, s, csize, cbirth, cprow, nrows, acc);
  CE_LAUNCH(k_cd_stab, dim3(gR), dim3(B), 0, s, acc, csize, cbirth, nrows, shi, slo);
  CE_LAUNCH(k_fill32, dim3(gR), dim3(B), 0, s, nch, R, 0u);
  CE_LAUNCH(k_fill32, dim3(grid_cap(2 * R, B)), dim3(B), 0, s, ch, 2 * R, 0u);
  if (b.q > 0) {
    // any number of child clusters: per-parent lists, then chains of virtual sum nodes
    CE_LAUNCH(k_cd_child_keys, dim3(gR), dim3(B), 0, s, cprow, nrows, ckey);
    CE_HIP(hipGetLastError());
    bool calt = false;
    CE_TRY((radix_sort_pairs<uint32_t, uint32_t>(ckey, clist, ckey2, clist2, nrows, 0, bits_for((uint64_t)R), true,
                                                 &calt, ws, s)));
    const uint32_t *sk = calt ? ckey2 : ckey;
    if (calt) clist = clist2;
    CE_TRY(segment_bounds_u32(sk, nrows, nrows, choff, s));
    CE_LAUNCH(k_cd_child_counts, dim3(gR), dim3(B), 0, s, choff, nrows, nch, vbase);
    CE_HIP(hipGetLastError());
    CE_TRY(scan_exclusive_u32(vbase, vbase, nrows, ws, s));
    CE_LAUNCH(k_virtual_counts, dim3(1), dim3(64), 0, s, vbase, b.hdr, RE);
    CE_LAUNCH(k_cd_pairs, dim3(gR), dim3(B), 0, s, nch, choff, clist, vbase, nrows, ch);
    CE_LAUNCH(k_cd_virtual, dim3(gR), dim3(B), 0, s, nch, choff, clist, vbase, nrows, nvirt, ch, nch, shi, slo);
    CE_HIP(hipGetLastError());
  } else {
    CE_LAUNCH(k_cd_children, dim3(gR), dim3(B), 0, s, cprow, nrows, nch, ch);
    CE_LAUNCH(k_eom_count, dim3(1), dim3(64), 0, s, b.hdr);
  }
  // excess of mass: enqueued rounds, then the rest in one workgroup
  uint64_t *el = loop + LOOP_EOM;
  const unsigned tRE = grid_cap(RE, B, tuning().list_grid);
  CE_LAUNCH(k_eom_init, dim3(tRE), dim3(B), 0, s, nch, shi, slo, cprow, nrows, neom, e[0], e[1], ract,
            (unsigned long long *)&el[0]);
  CE_HIP(hipGetLastError());
  uint32_t *lists[2] = {ract, ract2};
  const int EOM_ROUNDS = eom_rounds(RE), TOP_ROUNDS = top_rounds(R);
  if (LOOP_EOM + EOM_ROUNDS + 1 >= LOOP_TOP || LOOP_TOP + TOP_ROUNDS + 1 >= LOOP_END) {
    set_error("internal: too many bounded rounds");
    return CE_EDEVICE;
  }
  for (int r = 0; r < EOM_ROUNDS; r++)
    CE_LAUNCH(k_eom_round, dim3(tRE), dim3(B), 0, s, lists[r & 1], &el[r], e[r & 1], e[1 - (r & 1)], ch, shi, slo,
              lists[1 - (r & 1)], (unsigned long long *)&el[r + 1]);
  CE_LAUNCH(k_eom_tail, dim3(1), dim3(TB), 0, s, lists[0], lists[1], &el[EOM_ROUNDS], EOM_ROUNDS & 1, e[0], e[1],
            ch, shi, slo, b.hdr);
  CE_HIP(hipGetLastError());
  // the list is empty: both state buffers hold the final values
  uint64_t *tl = loop + LOOP_TOP;
  CE_LAUNCH(k_eom_select, dim3(grid_cap(R, B, tuning().list_grid)), dim3(B), 0, s, nch, ch, e[0], shi, slo, nrows,
            top, nxt, top2, nxt2, cprow, ract, (unsigned long long *)&tl[0]);
  CE_HIP(hipGetLastError());
  uint32_t *tops[2] = {top, top2}, *nxts[2] = {nxt, nxt2};
  for (int r = 0; r < TOP_ROUNDS; r++)
    CE_LAUNCH(k_top_jump, dim3(tRE), dim3(B), 0, s, lists[r & 1], &tl[r], tops[r & 1], nxts[r & 1],
              tops[1 - (r & 1)], nxts[1 - (r & 1)], lists[1 - (r & 1)], (unsigned long long *)&tl[r + 1]);
  CE_LAUNCH(k_top_tail, dim3(1), dim3(TB), 0, s, lists[0], lists[1], &tl[TOP_ROUNDS], TOP_ROUNDS & 1, top, nxt, top2,
            nxt2, b.hdr);
  CE_HIP(hipGetLastError());
  CE_LAUNCH(k_fill32, dim3(gR), dim3(B), 0, s, minmem, R, NONE32);
  CE_LAUNCH(k_lab_rows, dim3(grid_cap(n, B)), dim3(B), 0, s, prow, top, cprow, n, minmem);
  CE_LAUNCH(k_fill32, dim3(grid_cap(n + 1, B)), dim3(B), 0, s, fl, n + 1, 0u);
  CE_LAUNCH(k_lab_flags, dim3(gR), dim3(B), 0, s, top, minmem, nrows, fl);
  CE_HIP(hipGetLastError());
  CE_TRY(scan_exclusive_u32(fl, fl, Cnt(n), ws, s));
  // per cluster row first (small arrays), then every record reads its row's values
  uint32_t *rlocal = nxt;
  int32_t *rlab = (int32_t *)nxt2;
  CE_LAUNCH(k_row_point_vals, dim3(gR), dim3(B), 0, s, cnode, cprow, top, minmem, fl, b.rowg, b.eoff, b.moff,
            b.rowpos, n, m, nrows, rlocal, rlab);
  CE_LAUNCH(k_out_points, dim3(grid_cap(n, B)), dim3(B), 0, s, prow, rlocal, rlab, n, b.hdr, out->pt_cluster,
            out->labels);
  CE_LAUNCH(k_out_clusters, dim3(gR), dim3(B), 0, s, cnode, cprow, csize, cbirth, shi, slo, top, b.rowg, b.eoff,
            b.moff, b.rowpos, n, m, nrows, b.hdr, *out);
  CE_LAUNCH(k_graph_labels, dim3(gG), dim3(B), 0, s, fl, b.eoff, G, nlab);
  CE_LAUNCH(k_header, dim3(gG), dim3(B), 0, s, b.hdr, G, b.moff, bstart, nlab, hout);
  CE_HIP(hipGetLastError());
  (void)gRE;
  ws.release(m0);
  return CE_OK;
}

}  // namespace ce
