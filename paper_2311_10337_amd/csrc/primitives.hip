// Device-wide primitives: exclusive scan and a stable LSD radix sort.
//
// The radix sort is a reduce-then-scan design tiled for 64-wide waves:
// each 256-thread block owns a 2048-key tile; the scatter pass ranks keys
// stably inside the tile with 8 ballots per 64-key chunk (lanes with equal
// digits form a peer mask), stages the tile in LDS in digit order and then
// writes it out in runs of consecutive addresses.
#include "ce_internal.h"

namespace ce {

namespace {

constexpr int SB = 256;          // scan block
constexpr int SIPT = 8;          // scan items per thread
constexpr int STILE = SB * SIPT; // 2048

__device__ inline uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// exclusive scan of one value per thread across a 256-thread block
__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t *lds_w /*[4]*/, uint32_t *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(x, lane);
  if (lane == 63) lds_w[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SB / 64; i++) {
    uint32_t v = lds_w[i];
    if (i < w) before += v;
    tot += v;
  }
  __syncthreads();
  if (total) *total = tot;
  return before + inc - x;
}

// Tiles of STILE elements; a block takes tiles blockIdx.x, + gridDim.x, ...
// up to the live count's tiles (the grid is capped, so a small or empty live
// count costs little).
__global__ __launch_bounds__(SB) void k_scan_reduce(const uint32_t *in, Cnt nc, uint32_t *sums) {
  __shared__ uint32_t lw[SB / 64];
  const int64_t n = nc.get();
  const int64_t tiles = (n + STILE - 1) / STILE;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t base = tile * STILE + (int64_t)threadIdx.x * SIPT;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < SIPT; k++)
      if (base + k < n) acc += in[base + k];
    uint32_t tot;
    block_excl_scan(acc, lw, &tot);
    if (threadIdx.x == 0) sums[tile] = tot;
  }
}

__global__ __launch_bounds__(SB) void k_scan_apply(const uint32_t *in, uint32_t *out, Cnt nc,
                                                   const uint32_t *sums_scanned) {
  __shared__ uint32_t lw[SB / 64];
  const int64_t n = nc.get();
  const int64_t tiles = (n + STILE - 1) / STILE;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t base = tile * STILE + (int64_t)threadIdx.x * SIPT;
    uint32_t v[SIPT];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < SIPT; k++) {
      v[k] = (base + k < n) ? in[base + k] : 0u;
      acc += v[k];
    }
    uint32_t run = block_excl_scan(acc, lw, nullptr) + sums_scanned[tile];
#pragma unroll
    for (int k = 0; k < SIPT; k++) {
      if (base + k < n) out[base + k] = run;
      run += v[k];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums_scanned[tiles];
}

// single-block exclusive scan for up to STILE elements; out[n] = total
__global__ __launch_bounds__(SB) void k_scan_small(const uint32_t *in, uint32_t *out, Cnt nc) {
  __shared__ uint32_t lw[SB / 64];
  const int64_t n = nc.get();
  int64_t base = (int64_t)threadIdx.x * SIPT;
  uint32_t v[SIPT];
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < SIPT; k++) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    acc += v[k];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(acc, lw, &tot);
#pragma unroll
  for (int k = 0; k < SIPT; k++) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) out[n] = tot;
}

}  // namespace

size_t scan_ws_bytes(int64_t n) {
  size_t b = 0;
  while (n > STILE) {
    int64_t nb = (n + STILE - 1) / STILE;
    b += 2 * (((size_t)(nb + 1) * 4 + 255) & ~size_t(255));
    n = nb;
  }
  return b + 512;
}

ce_status scan_exclusive_u32(const uint32_t *in, uint32_t *out, Cnt n, Ws &ws, hipStream_t s) {
  if (n.v <= STILE) {
    CE_LAUNCH(k_scan_small, dim3(1), dim3(SB), 0, s, in, out, n);
    CE_HIP(hipGetLastError());
    return CE_OK;
  }
  // one sum per tile of the live count; the sums are scanned with the tile count as their count
  int64_t nb = (n.v + STILE - 1) / STILE;
  size_t m = ws.mark();
  uint32_t *sums = ws.alloc<uint32_t>(nb + 1);
  uint32_t *sums_sc = ws.alloc<uint32_t>(nb + 1);
  CE_WS_CHECK(ws);
  const unsigned g = grid_for(nb, 1, 2048);
  CE_LAUNCH(k_scan_reduce, dim3(g), dim3(SB), 0, s, in, n, sums);
  CE_HIP(hipGetLastError());
  CE_TRY(scan_exclusive_u32(sums, sums_sc, n.p ? Cnt(n.p, nb, n.sh + 11) : Cnt(nb), ws, s));
  CE_LAUNCH(k_scan_apply, dim3(g), dim3(SB), 0, s, in, out, n, sums_sc);
  CE_HIP(hipGetLastError());
  ws.release(m);
  return CE_OK;
}

// ------------------------------------------------------------ segment bounds
namespace {

// off[g] = first position p with key[p] >= g, for g in [0, G]; each of the
// n+1 gaps between neighbouring keys writes the offsets that fall in it
__global__ __launch_bounds__(256) void k_seg_bounds(const uint32_t *key, Cnt nc, Cnt gc, uint32_t *off) {
  const int64_t n = nc.get(), G = gc.get();
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p <= n; p += (int64_t)gridDim.x * 256) {
    const int64_t lo = p == 0 ? 0 : (int64_t)key[p - 1] + 1;
    const int64_t hi = p == n ? G : (int64_t)key[p];
    for (int64_t g = lo; g <= hi; g++) off[g] = (uint32_t)p;
  }
}

}  // namespace

ce_status segment_bounds_u32(const uint32_t *sorted_keys, Cnt n, Cnt G, uint32_t *off, hipStream_t s) {
  CE_LAUNCH(k_seg_bounds, dim3(grid_cap(n.v + 1, 256)), dim3(256), 0, s, sorted_keys, n, G, off);
  CE_HIP(hipGetLastError());
  return CE_OK;
}

// ------------------------------------------------------------ radix sort
namespace {

constexpr int RB = 256;              // block
constexpr int RW = RB / 64;          // waves per block
// keys per thread (IPT): 4, 8 or 16 (a tuning choice); a tile is RB * IPT keys

template <class K, int IPT>
__global__ __launch_bounds__(RB) void k_rs_hist(const K *keys, Cnt nc, int shift, uint32_t *hist,
                                                int nblocks) {
  constexpr int TILE = RB * IPT;
  __shared__ uint32_t cnt[RW][256];
  const int64_t n = nc.get();  // tiles past a device count write zero counts
  const int w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < RW * 256; i += RB) (&cnt[0][0])[i] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * TILE;
#pragma unroll
  for (int k = 0; k < IPT; k++) {
    int64_t i = base + k * RB + threadIdx.x;
    if (i < n) atomicAdd(&cnt[w][(uint32_t)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += RB) {
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < RW; q++) c += cnt[q][d];
    hist[(int64_t)d * nblocks + blockIdx.x] = c;
  }
}

template <class V>
__device__ inline V iota_value(int64_t i) { return V(i); }
template <>
__device__ inline uint4 iota_value<uint4>(int64_t i) { return make_uint4((uint32_t)i, 0u, 0u, 0u); }

template <class K, class V, int IPT>
__global__ __launch_bounds__(RB) void k_rs_scatter(const K *kin, const V *vin, K *kout, V *vout, Cnt nc,
                                                   int shift, const uint32_t *hscan, int nblocks, int iota) {
  constexpr int TILE = RB * IPT, WT = TILE / RW;  // keys per tile, per wave (IPT chunks of 64)
  const int64_t n = nc.get();
  if ((int64_t)blockIdx.x * TILE >= n) return;
  __shared__ uint32_t wcnt[RW][256];
  __shared__ uint32_t dbase[256];
  __shared__ uint32_t lw[RB / 64];
  __shared__ K skey[TILE];
  __shared__ V sval[TILE];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < RW * 256; i += RB) (&wcnt[0][0])[i] = 0;
  __syncthreads();
  const int64_t tbase = (int64_t)blockIdx.x * TILE;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  K key[IPT];
  V val[IPT];
  uint32_t off[IPT];
  uint32_t dig[IPT];
#pragma unroll
  for (int c = 0; c < IPT; c++) {
    const int64_t i = tbase + (int64_t)w * WT + c * 64 + lane;
    const bool valid = i < n;
    K k = valid ? kin[i] : K(0);
    V v = valid ? (iota ? iota_value<V>(i) : vin[i]) : V{};
    uint32_t d = (uint32_t)(k >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const int leader = valid ? (__ffsll((unsigned long long)peers) - 1) : lane;
    uint32_t old = 0;
    if (valid && lane == leader) old = atomicAdd(&wcnt[w][d], (uint32_t)__popcll(peers));
    old = __shfl(old, leader, 64);
    key[c] = k;
    val[c] = v;
    dig[c] = valid ? d : 256u;
    off[c] = old + (uint32_t)__popcll(peers & below);
  }
  __syncthreads();
  // per digit: exclusive prefix over waves, then exclusive scan over digits
  uint32_t tot = 0;
  {
    const int d = tid;  // RB == 256 digits
    uint32_t run = 0;
#pragma unroll
    for (int q = 0; q < RW; q++) {
      uint32_t t = wcnt[q][d];
      wcnt[q][d] = run;
      run += t;
    }
    tot = run;
  }
  __syncthreads();
  uint32_t ex = block_excl_scan(tot, lw, nullptr);
  dbase[tid] = ex;
  __syncthreads();
#pragma unroll
  for (int c = 0; c < IPT; c++) {
    if (dig[c] < 256u) {
      uint32_t p = dbase[dig[c]] + wcnt[w][dig[c]] + off[c];
      skey[p] = key[c];
      sval[p] = val[c];
    }
  }
  __syncthreads();
  const int64_t rem = n - tbase;
  const int valid_n = rem < TILE ? (int)rem : TILE;
  for (int i = tid; i < valid_n; i += RB) {
    K k = skey[i];
    uint32_t d = (uint32_t)(k >> shift) & 255u;
    int64_t g = (int64_t)hscan[(int64_t)d * nblocks + blockIdx.x] + (i - (int64_t)dbase[d]);
    kout[g] = k;
    vout[g] = sval[i];
  }
}

// Up to 2^24 keys a sort may take 4 keys per thread (its histogram is sized
// for that); larger sorts take at least 8. A 16-key tile stages up to 24 B
// pairs in LDS: 96 KiB of the 160 KiB a gfx950 workgroup may use.
int radix_ipt(int64_t n) {
  int ipt = tuning().radix_ipt;
  if (ipt != 4 && ipt != 8 && ipt != 16) ipt = 8;
  if (ipt == 4 && n > (int64_t(1) << 24)) ipt = 8;
  return ipt;
}

template <class K, class V, int IPT>
ce_status radix_passes(K *k0, V *v0, K *k1, V *v1, Cnt n, int begin_bit, int end_bit, bool iota_values,
                       bool *result_in_alt, Ws &ws, hipStream_t s) {
  constexpr int TILE = RB * IPT;
  const int64_t nb64 = (n.v + TILE - 1) / TILE;
  if (nb64 > 0x7fffffff) return CE_EINVAL;
  const int nb = (int)nb64;
  size_t m = ws.mark();
  uint32_t *hist = ws.alloc<uint32_t>((size_t)nb * 256 + 1);
  uint32_t *hsc = ws.alloc<uint32_t>((size_t)nb * 256 + 1);
  CE_WS_CHECK(ws);
  K *ki = k0, *ko = k1;
  V *vi = v0, *vo = v1;
  bool alt = false;
  bool first = true;
  if (end_bit <= begin_bit) end_bit = begin_bit + 1;  // one stable pass still materialises identity values
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    CE_LAUNCH((k_rs_hist<K, IPT>), dim3((unsigned)nb), dim3(RB), 0, s, ki, n, shift, hist, nb);
    CE_HIP(hipGetLastError());
    CE_TRY(scan_exclusive_u32(hist, hsc, Cnt((int64_t)nb * 256), ws, s));
    CE_LAUNCH((k_rs_scatter<K, V, IPT>), dim3((unsigned)nb), dim3(RB), 0, s, ki, (const V *)vi, ko, vo, n,
                       shift, hsc, nb, (first && iota_values) ? 1 : 0);
    CE_HIP(hipGetLastError());
    first = false;
    K *tk = ki; ki = ko; ko = tk;
    V *tv = vi; vi = vo; vo = tv;
    alt = !alt;
  }
  *result_in_alt = alt;
  ws.release(m);
  return CE_OK;
}

}  // namespace

size_t radix_ws_bytes(int64_t n) {
  const int64_t tile = RB * (n > (int64_t(1) << 24) ? 8 : 4);  // the smallest tile a sort of n keys takes
  int64_t nb = (n + tile - 1) / tile;
  size_t h = (size_t)nb * 256;
  return 2 * (((h + 1) * 4 + 255) & ~size_t(255)) + scan_ws_bytes((int64_t)h) + 512;
}

template <class K, class V>
ce_status radix_sort_pairs(K *k0, V *v0, K *k1, V *v1, Cnt n, int begin_bit, int end_bit, bool iota_values,
                           bool *result_in_alt, Ws &ws, hipStream_t s) {
  *result_in_alt = false;
  if (n.v <= 0) return CE_OK;
  switch (radix_ipt(n.v)) {
    case 4:
      return radix_passes<K, V, 4>(k0, v0, k1, v1, n, begin_bit, end_bit, iota_values, result_in_alt, ws, s);
    case 16:
      return radix_passes<K, V, 16>(k0, v0, k1, v1, n, begin_bit, end_bit, iota_values, result_in_alt, ws, s);
    default:
      return radix_passes<K, V, 8>(k0, v0, k1, v1, n, begin_bit, end_bit, iota_values, result_in_alt, ws, s);
  }
}

template ce_status radix_sort_pairs<uint64_t, uint32_t>(uint64_t *, uint32_t *, uint64_t *, uint32_t *, Cnt, int,
                                                        int, bool, bool *, Ws &, hipStream_t);
template ce_status radix_sort_pairs<uint32_t, uint32_t>(uint32_t *, uint32_t *, uint32_t *, uint32_t *, Cnt, int,
                                                        int, bool, bool *, Ws &, hipStream_t);
template ce_status radix_sort_pairs<uint64_t, uint4>(uint64_t *, uint4 *, uint64_t *, uint4 *, Cnt, int, int,
                                                     bool, bool *, Ws &, hipStream_t);
template ce_status radix_sort_pairs<uint64_t, uint64_t>(uint64_t *, uint64_t *, uint64_t *, uint64_t *, Cnt, int,
                                                        int, bool, bool *, Ws &, hipStream_t);

}  // namespace ce
