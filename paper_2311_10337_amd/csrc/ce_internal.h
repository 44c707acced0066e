// Internal declarations shared by the HIP translation units of libce.
// gfx950 (CDNA4) only: 64-wide wavefronts, 160 KB LDS per CU.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/ce.h"

namespace ce {

constexpr uint32_t NONE32 = 0xffffffffu;
constexpr uint64_t NONE64 = 0xffffffffffffffffull;

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);

#define CE_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::ce::set_error(std::string(#call " failed: ") + hipGetErrorString(e_));         \
      return CE_EDEVICE;                                                               \
    }                                                                                  \
  } while (0)

#define CE_WS_CHECK(ws)                                                   \
  do {                                                                    \
    if ((ws).overflow) {                                                  \
      ::ce::set_error("internal: workspace carve exceeds its capacity");  \
      return CE_ENOMEM;                                                   \
    }                                                                     \
  } while (0)

#define CE_TRY(expr)                   \
  do {                                 \
    ce_status s_ = (expr);             \
    if (s_ != CE_OK) return s_;        \
  } while (0)

// ------------------------------------------------------- kernel timing
// When enabled for a kernel name (ce_timing_enable), every launch whose name
// contains it carries a pair of HIP events in its own dispatch
// (hipExtLaunchKernel), stamped when the kernel starts and ends on the
// launch stream; the elapsed times are collected when a synchronous call
// returns. Asynchronous calls (which may be captured in a graph) are never
// timed: TimingOff holds timing off on the calling thread for their span.
bool timing_wants(const char *kernel);
struct TimingOff {
  bool prev;
  explicit TimingOff(bool off);
  ~TimingOff();
};
void timing_push(hipEvent_t a, hipEvent_t b);
void timing_collect();
struct KTime {
  hipEvent_t a = nullptr, b = nullptr;
  bool on;
  explicit KTime(const char *name) : on(timing_wants(name)) {
    if (on) {
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
    }
  }
  void stop() {
    if (on) timing_push(a, b);
  }
};
#define CE_LAUNCH(kernel, grid, block, shmem, stream, ...)                                     \
  do {                                                                                         \
    ::ce::KTime kt_(#kernel);                                                                  \
    if (kt_.on)                                                                                \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, kt_.a, kt_.b, 0, __VA_ARGS__); \
    else                                                                                       \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                     \
    kt_.stop();                                                                                \
  } while (0)

// ---------------------------------------------------------- workspace plan
// Bump allocator over one device buffer. With base == nullptr it only
// measures (used by ce_workspace_bytes), so the same layout code sizes and
// carves the workspace. Regions are 256-byte aligned.
struct Ws {
  char *base = nullptr;
  size_t off = 0;
  size_t peak = 0;
  size_t cap = ~size_t(0);
  bool overflow = false;  // set when a carve would pass cap; callers check before launching
  template <class T>
  T *alloc(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    if (off + bytes > cap) overflow = true;
    T *p = (base && !overflow) ? reinterpret_cast<T *>(base + off) : nullptr;
    off += bytes;
    if (off > peak) peak = off;
    return p;
  }
  size_t mark() const { return off; }
  void release(size_t m) { off = m; }
};

inline int bits_for(uint64_t v) {  // bits needed to represent v (0 -> 0)
  int b = 0;
  while (v) { b++; v >>= 1; }
  return b;
}

inline unsigned grid_for(int64_t work, int block, int64_t cap = 1 << 20) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ------------------------------------------------------ device-resident counts
// A size the host knows (p == nullptr: the value v), or one an earlier kernel
// of the same call wrote to device memory (p, read when a kernel starts; v is
// then an upper bound that sizes grids). Data-dependent sizes travel this way,
// so a call enqueues its whole pipeline without reading anything back.
// With sh > 0 the size is ceil(*p / 2^sh) (the tiles of a device count).
struct Cnt {
  const uint64_t *p;
  int64_t v;
  int sh;
  __host__ __device__ Cnt(int64_t x = 0) : p(nullptr), v(x), sh(0) {}
  __host__ __device__ Cnt(const uint64_t *q, int64_t bound, int shift = 0) : p(q), v(bound), sh(shift) {}
  __device__ inline int64_t get() const {
    return p ? (int64_t)((*p + ((uint64_t(1) << sh) - 1)) >> sh) : v;
  }
};

// Blocks for a grid-stride loop over at most `bound` items: the whole chip is
// covered several times over, and a launch whose live count turns out small
// (or zero) costs only its dispatch.
inline unsigned grid_cap(int64_t bound, int per_block, int64_t cap = 8192) {
  return grid_for(bound, per_block, cap);
}

// Words of a call's control block (Bufs::hdr, kHdrWords u64 at the start of
// the workspace).
enum : int {
  H_STATUS = 0,  // error bits: 1 self loop, 2 id out of range, 4 bad hypergraph offsets, 8 time span wider than
                 // the plan's key allows; every stage after validation treats the input as empty when set
  H_TMIN = 1,    // min t as an order-preserving u64
  H_TMAX = 2,    // max t likewise
  H_CNT = 4,     // list counters of the current stage
  H_CNT2 = 5,
  H_M = 6,       // rows of the spanning forest
  H_C7 = 7,      // stage-local counters
  H_C8 = 8,
  H_C9 = 9,
  H_NB = 10,     // cluster births
  H_NROWS = 11,  // cluster rows (births + one root per graph)
  H_NVIRT = 12,  // virtual sum nodes of the discrete condensing
  H_KEYW = 13,   // key layout of the flat skeletons: wshift | hshift << 8 | keybits << 16
  H_NEOM = 14,   // rows of the excess-of-mass tree (cluster rows + virtual nodes)
  H_BV = 16,     // Boruvka state (24 words)
  H_LOOP = 64,   // per-round counters of bounded loops
  kHdrWords = 256
};

// The ce_status of a call from its error bits (H_STATUS).
__host__ __device__ inline int64_t status_of(uint64_t bits) {
  if (bits & 1) return CE_ESELFLOOP;
  if (bits & 2) return CE_ERANGE;
  if (bits & 4) return CE_EINVAL;
  if (bits & 8) return CE_ERANGE;
  if (bits) return CE_EDEVICE;
  return CE_OK;
}

// ----------------------------------------------------------- u128 helpers
struct u128 {
  uint64_t lo, hi;
};
__host__ __device__ inline u128 u128_make(uint64_t hi, uint64_t lo) { return u128{lo, hi}; }
__host__ __device__ inline u128 u128_add(u128 a, u128 b) {
  u128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1 : 0);
  return r;
}
__host__ __device__ inline u128 u128_sub(u128 a, u128 b) {
  u128 r;
  r.lo = a.lo - b.lo;
  r.hi = a.hi - b.hi - (a.lo < b.lo ? 1 : 0);
  return r;
}
__host__ __device__ inline bool u128_gt(u128 a, u128 b) { return a.hi != b.hi ? a.hi > b.hi : a.lo > b.lo; }
__host__ __device__ inline u128 u128_max(u128 a, u128 b) { return u128_gt(b, a) ? b : a; }
__host__ __device__ inline u128 u128_mul64(uint64_t a, uint64_t b) {
  uint64_t a0 = a & 0xffffffffull, a1 = a >> 32, b0 = b & 0xffffffffull, b1 = b >> 32;
  uint64_t p00 = a0 * b0, p01 = a0 * b1, p10 = a1 * b0, p11 = a1 * b1;
  uint64_t mid = (p00 >> 32) + (p01 & 0xffffffffull) + (p10 & 0xffffffffull);
  u128 r;
  r.lo = (p00 & 0xffffffffull) | (mid << 32);
  r.hi = p11 + (p01 >> 32) + (p10 >> 32) + (mid >> 32);
  return r;
}

// graph g with eoff[g] <= i < eoff[g+1] (eoff non-decreasing, G >= 1)
__host__ __device__ inline uint32_t graph_of(const int64_t *eoff, int64_t G, int64_t i) {
  int64_t lo = 0, hi = G - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (eoff[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return (uint32_t)lo;
}

// lambda(w) = floor(2^63 / max(2w, 1)) for w >= 0
__host__ __device__ inline uint64_t lambda_of(int64_t w) {
  return w <= 0 ? (uint64_t(1) << 63) : ((uint64_t(1) << 63) / (2 * (uint64_t)w));
}

// ------------------------------------------------------ wave/block helpers
__device__ inline uint32_t wave_lane() { return threadIdx.x & 63u; }
__device__ inline uint64_t lanes_below(uint32_t lane) { return lane == 0 ? 0ull : (~0ull >> (64 - lane)); }

// One-shot wave combining for contended updates: the lanes holding the same
// key as the first active lane (the hot key, when one key dominates) are
// reduced into that lane by reduce(mine, leader), which every lane calls so
// it may shuffle. Returns whether this lane must still apply an update: the
// leader with the combined value, and every active lane with another key.
// (A loop over all distinct keys costs up to 64 rounds when keys differ;
// this costs one.)
template <class Fn>
__device__ inline bool wave_combine_first(bool active, uint32_t key, Fn reduce) {
  const uint64_t act = __ballot(active);
  if (act == 0) return false;
  const int leader = __ffsll((unsigned long long)act) - 1;
  const uint32_t k = __shfl(key, leader, 64);
  const bool mine = active && key == k;
  const uint64_t match = __ballot(mine);
  if (__popcll(match) < 2) return active;
  reduce(mine, leader);
  return active && (!mine || (int)wave_lane() == leader);
}
__device__ inline uint64_t wave_sum_u64(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}
__device__ inline uint32_t wave_sum_u32(uint32_t v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
  for (int d = 32; d >= 1; d >>= 1) { uint32_t o = __shfl_xor(v, d, 64); v = o > v ? o : v; }
  return v;
}
__device__ inline uint64_t wave_min_u64(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) { uint64_t o = __shfl_xor(v, d, 64); v = o < v ? o : v; }
  return v;
}

// Tile compaction: a 256-thread block keeps the elements of its tile
// [tile_base, tile_base + 256*CT) for which keep[k] is set and appends
// vals[k] to out[] with ONE atomic on the global counter per tile. Thread t
// owns elements tile_base + k*256 + t (coalesced loads). The output keeps
// element order inside the tile: per (k, wave) a ballot count, one 64-wide
// exclusive scan over the (k, wave) counts, then popcount ranks within the
// wave. Call from all threads of the block.
constexpr int CT = 16;
// Linear probes an LDS aggregation hash tries before a key goes straight to
// its global atomic: hot keys enter the table early, and a tile with many
// distinct keys should not pay a long probe sequence per element.
constexpr int HASH_PROBES = 4;
// Launch choices of the current call (ce_tuning resolved: the call's own
// fields, the environment, the tuning file, the built-in rules). Set by the
// entry points for the calling host thread.
struct Tuning {
  int radix_ipt = 8;
  int list_grid = 4096;
  int krt_level_bits = 0;  // 0: the rule of the row count
  int64_t split_min_edges = int64_t(1) << 20;  // INT64_MAX: no split
};
const Tuning &tuning();
struct TuningScope {
  Tuning prev;
  explicit TuningScope(const Tuning &t);
  ~TuningScope();
};
Tuning resolve_tuning(int64_t n, int64_t V, const ce_tuning *given);

// Items per thread of a tile loop over n items, at most CT: all CT once the
// launched grid is full, fewer when a short list (a small call, a late round)
// would otherwise sit in a few workgroups whose threads take their items one
// after another; then it spreads over the whole grid. Uniform over the grid.
__device__ inline int tile_items(int64_t n) {
  const int64_t span = (int64_t)blockDim.x * gridDim.x;
  const int64_t per = (n + span - 1) / span;
  return per < 1 ? 1 : (per > CT ? CT : (int)per);
}
// end of tile `tile` of `span` items in a list of n
__device__ inline int64_t tile_end(int64_t n, int64_t tile, int64_t span) {
  const int64_t e = (tile + 1) * span;
  return n < e ? n : e;
}
// Host side, for kernels that take a fixed number of items per thread over a
// list whose length the host knows (or bounds): enough items for the LDS
// aggregation to pay, but at least about 1024 workgroups while the list allows.
inline int items_per_thread(int64_t n, int block) {
  const int64_t per = n / ((int64_t)block * 1024);
  return per < 1 ? 1 : (per > CT ? CT : (int)per);
}
// Output positions for the kept elements of a tile (order as described
// above); pos[k] is valid where keep[k]. One atomic on `counter` per tile.
__device__ inline void tile_positions(const bool (&keep)[CT], uint32_t (&pos)[CT], unsigned long long *counter) {
  __shared__ uint32_t s_cnt[CT * 4];
  __shared__ uint32_t s_base;
  const uint32_t lane = wave_lane(), w = threadIdx.x >> 6;
  uint64_t mask[CT];
#pragma unroll
  for (int k = 0; k < CT; k++) {
    mask[k] = __ballot(keep[k]);
    if (lane == 0) s_cnt[k * 4 + w] = (uint32_t)__popcll(mask[k]);
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // CT * 4 == 64 counts in (k, wave) order
    uint32_t x = s_cnt[threadIdx.x], inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      uint32_t y = __shfl_up(inc, d, 64);
      if (threadIdx.x >= (uint32_t)d) inc += y;
    }
    uint32_t tot = __shfl(inc, 63, 64);
    s_cnt[threadIdx.x] = inc - x;
    if (threadIdx.x == 0) s_base = tot ? (uint32_t)atomicAdd(counter, (unsigned long long)tot) : 0u;
  }
  __syncthreads();
  const uint64_t below = lanes_below(lane);
#pragma unroll
  for (int k = 0; k < CT; k++) pos[k] = s_base + s_cnt[k * 4 + w] + (uint32_t)__popcll(mask[k] & below);
  __syncthreads();  // s_cnt / s_base may be reused by a later call
}

__device__ inline void tile_append(const bool (&keep)[CT], const uint32_t (&vals)[CT], uint32_t *out,
                                   unsigned long long *counter) {
  uint32_t pos[CT];
  tile_positions(keep, pos, counter);
#pragma unroll
  for (int k = 0; k < CT; k++)
    if (keep[k]) out[pos[k]] = vals[k];
}

// ------------------------------------------------------------ primitives
// Exclusive scan of n elements; out must hold n+1 (out[n] = total). In-place allowed.
// With a device count (n.p), n.v is the capacity and out[*n.p] gets the total.
ce_status scan_exclusive_u32(const uint32_t *in, uint32_t *out, Cnt n, Ws &ws, hipStream_t s);
size_t scan_ws_bytes(int64_t n);

// off[g] = first position whose key is >= g, for g in [0, G] (off[G] = n), from
// keys sorted ascending with values < G; no atomics, O(n + G) work.
ce_status segment_bounds_u32(const uint32_t *sorted_keys, Cnt n, Cnt G, uint32_t *off, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on bits [begin_bit, end_bit).
// Sorts the data in (k0, v0) using (k1, v1) as ping-pong buffers; on return
// *result_in_alt tells which pair holds the sorted output. With iota_values the
// values start as the identity 0..n-1 (v0's contents are not read).
template <class K, class V>
ce_status radix_sort_pairs(K *k0, V *v0, K *k1, V *v1, Cnt n, int begin_bit, int end_bit, bool iota_values,
                           bool *result_in_alt, Ws &ws, hipStream_t s);
size_t radix_ws_bytes(int64_t n);

}  // namespace ce

namespace ce {

// ---------------------------------------------------------------- pipeline
// Device buffers of one clustering call, carved from the workspace.
// Internal record ids are RANKS in the record order (t, id): rank r is the
// r-th record by time; perm[r] is its input id.
struct Bufs {
  int64_t n = 0, V = 0, M = 0;
  // batch of G independent graphs packed as a disjoint union: graph g owns
  // records [eoff[g], eoff[g+1]) and vertices [voff[g], voff[g+1]) (device copies)
  int64_t G = 1;
  const int64_t *eoff = nullptr, *voff = nullptr;
  uint32_t *grank = nullptr;    // [n] graph of each record, by rank
  uint32_t *rowg = nullptr;     // [n] graph of each MSF row
  uint32_t *rowpos = nullptr;   // [n] output position of each MSF row (graphs in order, rows in key order)
  uint32_t *moff = nullptr;     // [G+1] first output row of each graph
  int tbits = 0, idbits = 0, vbits = 0, keybits = 0;
  // packed key = w << wshift | head id << hshift | low bits (undirected: one
  // bit ordering the two edges of a head; causal: the tail's tie index)
  int wshift = 0, hshift = 0, jbits = 0;
  // weight ranks: the key's weight field holds the rank of w among the
  // skeleton's distinct weights (when w itself would not fit the key word)
  bool rank = false;
  // flat skeleton (causal and hypergraph modes): rows in slots 0..S-1, each
  // with its head rank in skel_tid; otherwise slot 2h+side belongs to head h
  bool flat = false;
  int64_t S = 0;
  int64_t slots = 0;  // capacity of the skeleton arrays: 2n, or nnz for hypergraphs
  // discrete dendrogram (Alg. 5): q thresholds on the device, 0 = exact
  const int64_t *thr = nullptr;
  int q = 0;
  int64_t tmin = 0;
  // persistent
  uint64_t *hdr = nullptr;      // [kHdrWords] the call's control block (H_* words)
  int64_t *outhdr = nullptr;    // [CE_HDR_WORDS(G)] the call's header (read back by synchronous calls)
  uint64_t *ts = nullptr;       // [n] t - tmin by rank
  uint32_t *perm = nullptr;     // [n] rank -> input id
  uint32_t *rankof = nullptr;   // [n] input id -> rank (from the MSF stage on)
  uint64_t *skel_key = nullptr; // [slots] slot 2h+s: key of the skeleton edge whose head is rank h
  uint32_t *skel_tail = nullptr;// [slots] tail rank of that edge or NONE
  uint32_t *skel_tid = nullptr; // [slots] input id of that tail (flat: the head rank)
  uint64_t *best = nullptr;     // [n] Boruvka: minimum key leaving each component
  uint8_t *msf_flag = nullptr;  // [slots]
  uint64_t *msf_key = nullptr;  // [n] sorted MSF keys
  uint64_t *msf_val = nullptr;  // [n] tail rank | head rank << 32; the head's id is in the key
  uint32_t *kc_u = nullptr, *kc_v = nullptr, *ksize = nullptr; // [n] dendrogram children (internal labels) and size
  // scratch arenas: A for grouping, skeleton and Boruvka (it may overlap the
  // MSF/dendrogram arrays, which are not live yet), M for sorting the MSF, B
  // for the dendrogram and condensing (it overlaps the dead skeleton arrays)
  char *scratch_a = nullptr, *scratch_m = nullptr, *scratch_b = nullptr;
  size_t scratch_a_bytes = 0, scratch_m_bytes = 0, scratch_b_bytes = 0;
};

// host pinned staging for small readbacks (per thread)
uint64_t *pinned_scratch();
ce_status read_u64(const uint64_t *dev, uint64_t *host_out, int count, hipStream_t s);

// Stages. Sizes that depend on the data (forest rows, births, list lengths)
// are device words of the control block; the stages enqueue work only.
ce_status stage_validate(const int32_t *src, const int32_t *dst, const int64_t *t, Bufs &b, hipStream_t s);
ce_status stage_check_span(Bufs &b, hipStream_t s);
ce_status read_validation(Bufs &b, hipStream_t s, uint64_t *flags, int64_t *tmin, int64_t *tmax);
ce_status stage_sort_skeleton(const int32_t *src, const int32_t *dst, const int64_t *t, Bufs &b, Ws &ws,
                              hipStream_t s);
ce_status stage_boruvka(Bufs &b, Ws &ws, hipStream_t s);
int boruvka_rounds(int64_t n, bool split_possible);
ce_status stage_msf_sort(Bufs &b, Ws &ws, hipStream_t s);
ce_status stage_dendrogram(Bufs &b, Ws &ws, hipStream_t s);
// condensing, stability, selection, labels; writes the call's header to hout
ce_status stage_condense(Bufs &b, const ce_result *out, Ws &ws, hipStream_t s, int64_t *hout);
ce_status stage_graph_rows(Bufs &b, Ws &ws, hipStream_t s);
size_t stage_graph_rows_scratch(int64_t n, int64_t G);
ce_status stage_write_rows(Bufs &b, const ce_result *out, hipStream_t s);

size_t stage_sort_skeleton_scratch(int64_t n);
// weight ranks of the first cnt skeleton slots from their raw weights (any mode)
ce_status stage_rank_weights(Bufs &b, uint64_t *wraw, int64_t cnt, Ws &ws, hipStream_t s);
size_t stage_rank_weights_scratch(int64_t cnt);
// the key layout for a time span of tbits bits: w itself, or its rank among at
// most `rows` distinct weights; false when neither fits the 63-bit key
bool choose_key_layout(Bufs &b, int64_t rows);
ce_status sort_records_by_time(const int32_t *src, const int32_t *dst, const int64_t *t, Bufs &b, Ws &ws,
                               hipStream_t s, const uint4 **vals);
ce_status stage_causal_skeleton(const int32_t *src, const int32_t *dst, const int64_t *t, Bufs &b, Ws &ws,
                                hipStream_t s);
size_t stage_causal_skeleton_scratch(int64_t n);
ce_status stage_time_filter(Bufs &b, int64_t max_dt, hipStream_t s);
size_t stage_boruvka_scratch(int64_t n, int64_t slots);
// dynamic hypergraphs (Sec. 5.3): members/offsets CSR per hyperedge
ce_status stage_hyper_validate(const int32_t *members, const int64_t *offsets, const int64_t *t, int64_t nnz,
                               Bufs &b, hipStream_t s);
ce_status stage_hyper_skeleton(const int32_t *members, const int64_t *offsets, const int64_t *t, int64_t nnz,
                               Bufs &b, Ws &ws, hipStream_t s);
size_t stage_hyper_skeleton_scratch(int64_t n, int64_t nnz);
size_t stage_msf_sort_scratch(int64_t n);
size_t stage_dendrogram_scratch(int64_t n);
size_t stage_condense_scratch(int64_t n, int64_t M, int64_t G, bool discrete);
int krt_max_level_bits(int64_t m);

}  // namespace ce
