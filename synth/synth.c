/*
 * Seeded synthetic dynamic multigraphs (temporal edge lists).
 *
 * This module only draws inputs. It computes nothing of the clustering
 * method; both the CPU oracle and the GPU library consume the arrays it
 * writes. Every random number comes from a counter-based stream
 * (SplitMix64 of a per-stream key), so the output is identical for any
 * OpenMP thread count.
 *
 * Recipes (all timestamps are int64 seconds, vertex ids int32, no self-loops):
 *   chung_lu_bursts : Chung-Lu endpoint law w_i ~ (i+1)^(-1/(gamma-1)),
 *                     conversations as Poisson bursts coupled to a seed vertex.
 *   rmat_hawkes     : R-MAT endpoints (a,b,c,d), one self-exciting Hawkes
 *                     session per distinct (src,dst) pair supplies that
 *                     pair's timestamps; optional planted hub.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { uint64_t s; } rng_t;

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
static inline rng_t rng_stream(uint64_t seed, uint64_t domain, uint64_t idx) {
  rng_t r;
  r.s = mix64(mix64(seed * 0x9e3779b97f4a7c15ULL + domain) ^ (idx + 0x632be59bd9b4e019ULL));
  return r;
}
static inline uint64_t rng_next(rng_t *r) {
  r->s += 0x9e3779b97f4a7c15ULL;
  return mix64(r->s);
}
/* uniform in [0,1) with 53 bits */
static inline double rng_unif(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }
/* uniform integer in [0, k) */
static inline uint64_t rng_below(rng_t *r, uint64_t k) {
  return (uint64_t)(((unsigned __int128)rng_next(r) * k) >> 64);
}
static inline double rng_exp(rng_t *r, double mean) { return -mean * log1p(-rng_unif(r)); }
static inline int rng_poisson_small(rng_t *r, double lam) {
  double L = exp(-lam), p = 1.0;
  int k = 0;
  do { k++; p *= rng_unif(r); } while (p > L);
  return k - 1;
}

enum { D_PERM = 1, D_BSIZE = 2, D_BURST = 3, D_RMAT = 4, D_HUB = 5, D_HAWKES = 6, D_META = 7 };

/* Graph500-style random relabelling of vertices so hubs are not at id 0. */
static void make_perm(int32_t *perm, int64_t V, uint64_t seed) {
  rng_t r = rng_stream(seed, D_PERM, 0);
  for (int64_t i = 0; i < V; i++) perm[i] = (int32_t)i;
  for (int64_t i = V - 1; i > 0; i--) {
    int64_t j = (int64_t)rng_below(&r, (uint64_t)(i + 1));
    int32_t tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
  }
}

static inline int64_t cdf_pick(const double *cdf, int64_t V, double u) {
  int64_t lo = 0, hi = V - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (cdf[mid] > u) hi = mid; else lo = mid + 1;
  }
  return lo;
}

/*
 * Chung-Lu endpoints + Poisson-burst timestamps.
 * Bursts: centre c ~ U[0,T), size k ~ U{bmin..bmax}, a seed vertex u ~ w,
 * event times c, then + Exp(gap_mean) each; the other endpoint x ~ w (x != u)
 * with orientation u->x or x->u at probability 1/2; t = floor(tau) mod T.
 * The last burst is truncated so that exactly n edges are written.
 */
int synth_chung_lu_bursts(int64_t n, int64_t V, double gamma, int64_t T, int bmin, int bmax,
                          double gap_mean, uint64_t seed, int32_t *src, int32_t *dst, int64_t *t) {
  if (n < 0 || V < 2 || bmin < 1 || bmax < bmin || T < 1) return -1;
  if (n == 0) return 0;
  double *cdf = (double *)malloc(sizeof(double) * V);
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * V);
  if (!cdf || !perm) { free(cdf); free(perm); return -4; }
  double expo = -1.0 / (gamma - 1.0), acc = 0.0;
  for (int64_t i = 0; i < V; i++) { acc += pow((double)(i + 1), expo); cdf[i] = acc; }
  for (int64_t i = 0; i < V; i++) cdf[i] /= acc;
  cdf[V - 1] = 1.0;
  make_perm(perm, V, seed);

  /* burst sizes are drawn sequentially from one stream, then filled in parallel */
  int64_t cap = n / bmin + 2, nb = 0, tot = 0;
  int64_t *boff = (int64_t *)malloc(sizeof(int64_t) * (cap + 1));
  if (!boff) { free(cdf); free(perm); return -4; }
  rng_t rs = rng_stream(seed, D_BSIZE, 0);
  while (tot < n) {
    int64_t k = bmin + (int64_t)rng_below(&rs, (uint64_t)(bmax - bmin + 1));
    if (tot + k > n) k = n - tot;
    boff[nb++] = tot;
    tot += k;
  }
  boff[nb] = n;

#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t b = 0; b < nb; b++) {
    rng_t r = rng_stream(seed, D_BURST, (uint64_t)b);
    double tau = rng_unif(&r) * (double)T;
    int64_t u = cdf_pick(cdf, V, rng_unif(&r));
    for (int64_t e = boff[b]; e < boff[b + 1]; e++) {
      if (e > boff[b]) tau += rng_exp(&r, gap_mean);
      int64_t x;
      do { x = cdf_pick(cdf, V, rng_unif(&r)); } while (x == u);
      int orient = (int)(rng_next(&r) >> 63);
      int64_t tt = (int64_t)floor(tau) % T;
      src[e] = perm[orient ? x : u];
      dst[e] = perm[orient ? u : x];
      t[e] = tt;
    }
  }
  free(boff); free(cdf); free(perm);
  return 0;
}

/* LSD radix sort of (key,idx) pairs on the low `bits` bits of key; OpenMP-parallel
 * histogram + scatter per pass (stable). */
static int radix_sort_pairs(uint64_t *key, int64_t *idx, int64_t n, int bits) {
  uint64_t *k2 = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
  int64_t *i2 = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
  if (!k2 || !i2) { free(k2); free(i2); return -4; }
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  int64_t *cnt = (int64_t *)calloc((size_t)nth * 256, sizeof(int64_t));
  for (int shift = 0; shift < bits; shift += 8) {
    memset(cnt, 0, sizeof(int64_t) * nth * 256);
#pragma omp parallel num_threads(nth)
    {
      int tid = 0;
#ifdef _OPENMP
      tid = omp_get_thread_num();
#endif
      int64_t lo = n * tid / nth, hi = n * (tid + 1) / nth;
      int64_t *c = cnt + (size_t)tid * 256;
      for (int64_t i = lo; i < hi; i++) c[(key[i] >> shift) & 255]++;
#pragma omp barrier
#pragma omp single
      {
        int64_t run = 0;
        for (int d = 0; d < 256; d++)
          for (int th = 0; th < nth; th++) {
            int64_t v = cnt[(size_t)th * 256 + d];
            cnt[(size_t)th * 256 + d] = run;
            run += v;
          }
      }
      for (int64_t i = lo; i < hi; i++) {
        int64_t p = c[(key[i] >> shift) & 255]++;
        k2[p] = key[i];
        i2[p] = idx[i];
      }
    }
    memcpy(key, k2, sizeof(uint64_t) * n);
    memcpy(idx, i2, sizeof(int64_t) * n);
  }
  free(cnt); free(k2); free(i2);
  return 0;
}

static int cmp_dbl(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/*
 * R-MAT endpoints (scale levels, quadrant probabilities a,b,c,d=1-a-b-c; src bit
 * is set on c/d, dst bit on b/d), self-loops redrawn, vertices relabelled by a
 * random permutation. If hub_extra > 0, that many random endpoints are then
 * redirected to the largest R-MAT hub (unpermuted vertex 0), never creating a
 * self-loop. Timestamps: for each distinct (src,dst) pair with multiplicity k,
 * a Hawkes process (immigrant rate mu, branching ratio eta, exponential kernel
 * with mean delay beta) is started at s ~ U[0,T); the k earliest events give
 * the pair's times (ascending, in ascending edge-index order); t = floor mod T.
 */
int synth_rmat_hawkes(int64_t n, int scale, double a, double b, double c, int64_t T, double mu,
                      double eta, double beta, int64_t hub_extra, uint64_t seed, int32_t *src,
                      int32_t *dst, int64_t *t) {
  if (n < 0 || scale < 1 || scale > 30 || T < 1) return -1;
  if (n == 0) return 0;
  int64_t V = (int64_t)1 << scale;
  const uint32_t ta = (uint32_t)(a * 65536.0), tb = (uint32_t)((a + b) * 65536.0),
                 tc = (uint32_t)((a + b + c) * 65536.0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    rng_t r = rng_stream(seed, D_RMAT, (uint64_t)i);
    uint32_t s, d;
    do {
      s = 0; d = 0;
      uint64_t bitsrc = 0;
      int avail = 0;
      for (int l = 0; l < scale; l++) {
        if (avail == 0) { bitsrc = rng_next(&r); avail = 4; }
        uint32_t u = (uint32_t)(bitsrc & 0xffff);
        bitsrc >>= 16; avail--;
        uint32_t sb = (u >= tb) ? 1u : 0u;              /* c or d */
        uint32_t db = ((u >= ta && u < tb) || u >= tc) ? 1u : 0u; /* b or d */
        s = (s << 1) | sb;
        d = (d << 1) | db;
      }
    } while (s == d);
    src[i] = (int32_t)s;
    dst[i] = (int32_t)d;
  }
  if (hub_extra > 0) {
    rng_t r = rng_stream(seed, D_HUB, 0);
    for (int64_t j = 0; j < hub_extra; j++) {
      int64_t i = (int64_t)rng_below(&r, (uint64_t)n);
      int side = (int)(rng_next(&r) >> 63);
      if (side == 0 && dst[i] != 0) src[i] = 0;
      else if (side == 1 && src[i] != 0) dst[i] = 0;
    }
  }
  /* group by pair */
  uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * n);
  int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * n);
  if (!key || !idx) { free(key); free(idx); return -4; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    key[i] = ((uint64_t)(uint32_t)src[i] << scale) | (uint64_t)(uint32_t)dst[i];
    idx[i] = i;
  }
  int rc = radix_sort_pairs(key, idx, n, 2 * scale);
  if (rc) { free(key); free(idx); return rc; }
  /* group starts */
  int64_t ng = 0;
  int64_t *gs = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
  for (int64_t i = 0; i < n; i++)
    if (i == 0 || key[i] != key[i - 1]) gs[ng++] = i;
  gs[ng] = n;
  int fail = 0;
#pragma omp parallel
  {
    int64_t bcap = 256;
    double *ev = (double *)malloc(sizeof(double) * bcap);
#pragma omp for schedule(dynamic, 1024)
    for (int64_t g = 0; g < ng; g++) {
      int64_t k = gs[g + 1] - gs[g];
      rng_t r = rng_stream(seed, D_HAWKES, key[gs[g]]);
      double start = rng_unif(&r) * (double)T, imm = start;
      int64_t ne = 0;
      /* k immigrants with their full progeny contain the k earliest events */
      for (int64_t im = 0; im < k; im++) {
        if (im > 0) imm += rng_exp(&r, 1.0 / mu);
        int64_t head = ne;
        if (ne + 1 > bcap) { bcap *= 2; ev = (double *)realloc(ev, sizeof(double) * bcap); }
        ev[ne++] = imm;
        while (head < ne) {
          double pt = ev[head++];
          int kids = rng_poisson_small(&r, eta);
          for (int q = 0; q < kids; q++) {
            if (ne + 1 > bcap) { bcap *= 2; ev = (double *)realloc(ev, sizeof(double) * bcap); }
            ev[ne++] = pt + rng_exp(&r, beta);
          }
        }
      }
      if (!ev) { fail = 1; continue; }
      qsort(ev, (size_t)ne, sizeof(double), cmp_dbl);
      /* edge indices of this pair in ascending order get ascending times */
      int64_t *ix = idx + gs[g];
      for (int64_t p = 1; p < k; p++) { /* insertion sort, groups are small */
        int64_t v = ix[p], q = p - 1;
        while (q >= 0 && ix[q] > v) { ix[q + 1] = ix[q]; q--; }
        ix[q + 1] = v;
      }
      for (int64_t p = 0; p < k; p++) t[ix[p]] = (int64_t)floor(ev[p]) % T;
    }
    free(ev);
  }
  free(gs); free(key); free(idx);
  if (fail) return -4;
  /* relabel vertices */
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * V);
  if (!perm) return -4;
  make_perm(perm, V, seed);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) { src[i] = perm[src[i]]; dst[i] = perm[dst[i]]; }
  free(perm);
  return 0;
}

/* Per-item derived seed for batches of independent graphs / requests. */
uint64_t synth_child_seed(uint64_t seed, uint64_t item) { return mix64(mix64(seed + D_META) ^ (item * 0x9e3779b97f4a7c15ULL + 1)); }

/* Uniform / lognormal / exponential helper draws for batch and request metadata. */
void synth_lognormal_sizes(int64_t count, double median, double sigma, int64_t lo, int64_t hi,
                           uint64_t seed, int64_t *out) {
  for (int64_t i = 0; i < count; i++) {
    rng_t r = rng_stream(seed, D_META, (uint64_t)i);
    double u1 = rng_unif(&r), u2 = rng_unif(&r);
    double z = sqrt(-2.0 * log1p(-u1)) * cos(2.0 * 3.14159265358979323846 * u2);
    double v = median * exp(sigma * z);
    int64_t k = (int64_t)llround(v);
    if (k < lo) k = lo;
    if (k > hi) k = hi;
    out[i] = k;
  }
}

void synth_exp_gaps(int64_t count, double mean, uint64_t seed, double *out) {
  rng_t r = rng_stream(seed, D_META + 100, 0);
  for (int64_t i = 0; i < count; i++) out[i] = rng_exp(&r, mean);
}
