// Alg. 5 by connected components: the discrete dendrogram's level l is the
// partition of the records into components of the line graph that keeps its
// edges with w <= threshold l. The paper computes it with one
// connected-components run per threshold. By Thm 3 (at every threshold) the
// components are those of the forest rows with w <= threshold, and the sorted
// forest rows of a level are a prefix of the rows, so each level adds its
// rows to the previous level's components:
//   level 0: labels = identity, union rows [0, p_0), compress;
//   level l: labels = level l-1, union rows [p_{l-1}, p_l), compress.
// The union-find hooks the larger root under the smaller and halving moves a
// link to a grandparent, so a parent always has a smaller id than its child
// and every component's root is its smallest member: after compression the
// labels are exactly the smallest member ids. The previous level's labels are
// the next level's union-find, so no workspace is needed.
#include "ce_internal.h"

namespace ce {

namespace {

constexpr int B = 256;

__device__ inline int32_t lc_ld(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void lc_st(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int32_t lc_find(int32_t *par, int32_t x) {
  while (true) {
    const int32_t p = lc_ld(&par[x]);
    if (p == x) return x;
    const int32_t g = lc_ld(&par[p]);
    if (g == p) return p;
    lc_st(&par[x], g);
    x = g;
  }
}

// flag |= 1: a row names a record >= n; |= 2: the rows are not in ascending w
__global__ __launch_bounds__(B) void k_lc_check(const uint32_t *tl, const uint32_t *hd, const int64_t *w, int64_t m,
                                                int64_t n, unsigned long long *flag) {
  uint32_t f = 0;
  for (int64_t j = (int64_t)blockIdx.x * B + threadIdx.x; j < m; j += (int64_t)gridDim.x * B) {
    if (tl[j] >= (uint64_t)n || hd[j] >= (uint64_t)n) f |= 1u;
    if (j + 1 < m && w[j] > w[j + 1]) f |= 2u;
  }
  if (__any(f != 0)) {
    const uint32_t all = (uint32_t)(__any(f & 1u) ? 1u : 0u) | (uint32_t)(__any(f & 2u) ? 2u : 0u);
    if (wave_lane() == 0) atomicOr(flag, (unsigned long long)all);
  }
}

// p[l] = number of rows with w <= thr[l] (rows ascending in w)
__global__ void k_lc_bounds(const int64_t *w, int64_t m, const int64_t *thr, int q, uint64_t *p) {
  for (int l = threadIdx.x; l < q; l += blockDim.x) {
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (w[mid] <= thr[l]) lo = mid + 1;
      else hi = mid;
    }
    p[l] = (uint64_t)lo;
  }
}

__global__ void k_lc_zero(uint64_t *p, int64_t k) {
  for (int64_t i = threadIdx.x; i < k; i += blockDim.x) p[i] = 0;
}

__global__ __launch_bounds__(B) void k_lc_iota(int32_t *lab, int64_t n) {
  for (int64_t x = (int64_t)blockIdx.x * B + threadIdx.x; x < n; x += (int64_t)gridDim.x * B) lab[x] = (int32_t)x;
}

// joins the components of the rows [a, b): the larger root goes under the smaller
__global__ __launch_bounds__(B) void k_lc_union(const uint32_t *tl, const uint32_t *hd, int64_t a, int64_t b,
                                                int32_t *par) {
  for (int64_t j = a + (int64_t)blockIdx.x * B + threadIdx.x; j < b; j += (int64_t)gridDim.x * B) {
    int32_t u = (int32_t)tl[j], v = (int32_t)hd[j];
    while (true) {
      u = lc_find(par, u);
      v = lc_find(par, v);
      if (u == v) break;
      const int32_t hi = u > v ? u : v, lo = u > v ? v : u;
      if (atomicCAS(&par[hi], hi, lo) == hi) break;
    }
  }
}

// root without halving: a halving store is an intermediate ancestor, and one
// landing after another thread stored the root would leave a non-root label
__device__ inline int32_t lc_root(const int32_t *par, int32_t x) {
  while (true) {
    const int32_t p = lc_ld(&par[x]);
    if (p == x) return x;
    x = p;
  }
}

// every record's root, its component's smallest member (no hooks run now).
// Only roots are stored, so every value a walk reads is an ancestor and the
// last store to each entry is its root.
__global__ __launch_bounds__(B) void k_lc_compress(int32_t *par, int64_t n) {
  for (int64_t x = (int64_t)blockIdx.x * B + threadIdx.x; x < n; x += (int64_t)gridDim.x * B) {
    const int32_t r = lc_root(par, (int32_t)x);
    if (r != (int32_t)x) lc_st(&par[x], r);
  }
}

}  // namespace

}  // namespace ce

using namespace ce;

extern "C" ce_status ce_level_components(const uint32_t *msf_tail, const uint32_t *msf_head, const int64_t *msf_w,
                                         int64_t m, int64_t n, const int64_t *thresholds, int64_t q,
                                         int32_t *labels, void *stream) {
  if (n < 0 || n > 0x7fffffffLL || m < 0 || m > 0x7fffffffLL) {
    set_error("n and m must be in [0, 2^31-1]");
    return CE_EINVAL;
  }
  if (q < 0 || q > CE_MAX_THRESHOLDS) {
    set_error("num_thresholds must be in [0, CE_MAX_THRESHOLDS]");
    return CE_EINVAL;
  }
  if (q > 0 && !thresholds) {
    set_error("thresholds is NULL");
    return CE_EINVAL;
  }
  for (int64_t l = 0; l < q; l++)
    if (thresholds[l] < 0 || (l > 0 && thresholds[l] <= thresholds[l - 1])) {
      set_error("thresholds must be >= 0 and strictly increasing");
      return CE_EINVAL;
    }
  if (q == 0 || n == 0) return CE_OK;
  if (!labels || (m > 0 && (!msf_tail || !msf_head || !msf_w))) {
    set_error("labels or a row array is NULL");
    return CE_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  uint64_t *h = pinned_scratch();
  if (!h) {
    set_error("hipHostMalloc of the readback buffer failed");
    return CE_EDEVICE;
  }
  // device words: [0] flags, [1..q] level bounds, then the thresholds
  const size_t words = 1 + (size_t)q + (size_t)q;
  void *dev = nullptr;
  CE_HIP(hipMallocAsync(&dev, sizeof(uint64_t) * words, s));
  struct Guard {
    void *p; hipStream_t s;
    ~Guard() { (void)hipFreeAsync(p, s); (void)hipStreamSynchronize(s); }
  } guard{dev, s};
  uint64_t *flag = (uint64_t *)dev, *p = flag + 1;
  int64_t *thr = (int64_t *)(p + q);
  CE_HIP(hipMemcpyAsync(thr, thresholds, sizeof(int64_t) * q, hipMemcpyHostToDevice, s));
  CE_LAUNCH(k_lc_zero, dim3(1), dim3(64), 0, s, flag, (int64_t)(1 + q));  // flags and bounds
  if (m > 0) {
    CE_LAUNCH(k_lc_check, dim3(grid_for(m, B)), dim3(B), 0, s, msf_tail, msf_head, msf_w, m, n,
              (unsigned long long *)flag);
    CE_LAUNCH(k_lc_bounds, dim3(1), dim3(64), 0, s, msf_w, m, thr, (int)q, p);
  }
  CE_HIP(hipGetLastError());
  uint64_t *hb = h + 128;  // bytes 1024 .. 1024 + 8 (q + 1) of the page
  CE_HIP(hipMemcpyAsync(hb, dev, sizeof(uint64_t) * (1 + q), hipMemcpyDeviceToHost, s));
  CE_HIP(hipStreamSynchronize(s));
  if (hb[0] & 1) {
    set_error("a row names a record >= n");
    return CE_ERANGE;
  }
  if (hb[0] & 2) {
    set_error("rows must be in ascending w (the order of the sorted forest)");
    return CE_EINVAL;
  }
  int64_t prev = 0;
  for (int64_t l = 0; l < q; l++) {
    int32_t *lab = labels + l * n;
    const int64_t end = (int64_t)hb[1 + l];
    if (end < prev || end > m) {
      set_error("internal: level bounds");
      return CE_EDEVICE;
    }
    if (l == 0) CE_LAUNCH(k_lc_iota, dim3(grid_for(n, B)), dim3(B), 0, s, lab, n);
    else CE_HIP(hipMemcpyAsync(lab, lab - n, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    if (end > prev) {
      CE_LAUNCH(k_lc_union, dim3(grid_for(end - prev, B)), dim3(B), 0, s, msf_tail, msf_head, prev, end, lab);
      CE_LAUNCH(k_lc_compress, dim3(grid_for(n, B)), dim3(B), 0, s, lab, n);
    }
    CE_HIP(hipGetLastError());
    prev = end;
  }
  CE_HIP(hipStreamSynchronize(s));
  return CE_OK;
}
