/*
 * graphgen.c -- seeded synthetic graph inputs shared by the oracle side and the
 * GPU side of the test and benchmark harness.
 *
 * This file holds input generation only: random edge lists, CSR assembly and
 * edge-weight samplers.  It contains none of the shortest-path arithmetic.
 *
 * Randomness: xoshiro256** seeded through splitmix64 (Blackman and Vigna,
 * "Scrambled linear pseudorandom number generators", 2021).  Every parallel
 * loop draws from a generator seeded per fixed-size chunk, so the output is
 * byte-identical for any thread count.
 *
 * Graph shapes stand in for the paper's SNAP / SuiteSparse inputs (Section 4.1,
 * Table 2), which are not available here:
 *   - directed Erdos-Renyi with uniform endpoints,
 *   - R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with quadrant probabilities a,b,c,d,
 *   - 2-D four-neighbour grids with a fraction of undirected pairs deleted.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GG_CHUNK ((int64_t)1 << 16)

typedef struct { uint64_t s[4]; } xo_t;

static uint64_t splitmix64_next(uint64_t* x) {
  uint64_t z = (*x += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* One independent stream per (seed, stream id). */
static void xo_seed(xo_t* r, uint64_t seed, uint64_t stream) {
  uint64_t x = seed ^ (stream * 0xD1B54A32D192ED03ULL + 0x632BE59BD9B4E019ULL);
  for (int i = 0; i < 4; i++) r->s[i] = splitmix64_next(&x);
}

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t xo_next(xo_t* r) {
  uint64_t* s = r->s;
  const uint64_t out = rotl64(s[1] * 5, 7) * 9;
  const uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl64(s[3], 45);
  return out;
}

/* Unbiased integer in [0, range) -- Lemire, "Fast random integer generation in
 * an interval", 2019 (multiply-shift with rejection). range >= 1. */
static inline uint32_t xo_bounded(xo_t* r, uint32_t range) {
  uint64_t x = xo_next(r) >> 32;
  uint64_t prod = x * (uint64_t)range;
  uint32_t low = (uint32_t)prod;
  if (low < range) {
    const uint32_t thresh = (uint32_t)(-range) % range;
    while (low < thresh) {
      x = xo_next(r) >> 32;
      prod = x * (uint64_t)range;
      low = (uint32_t)prod;
    }
  }
  return (uint32_t)(prod >> 32);
}

/* Uniform double in [0, 1) with 53 random bits. */
static inline double xo_unit(xo_t* r) { return (double)(xo_next(r) >> 11) * 0x1.0p-53; }

/* ------------------------------------------------------------------------- */
/* Edge lists                                                                 */
/* ------------------------------------------------------------------------- */

/* Directed Erdos-Renyi: m edges, endpoints uniform in [0,n); a self-loop is
 * redrawn so exactly m edges come out (parallel edges are kept). n >= 2. */
int64_t gg_er_edges(int64_t n, int64_t m, uint64_t seed, int32_t* src, int32_t* dst) {
  if (n < 2 || m < 0) return -1;
  const int64_t nchunks = (m + GG_CHUNK - 1) / GG_CHUNK;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nchunks; c++) {
    xo_t r;
    xo_seed(&r, seed, (uint64_t)c);
    const int64_t lo = c * GG_CHUNK, hi = (lo + GG_CHUNK < m) ? lo + GG_CHUNK : m;
    for (int64_t e = lo; e < hi; e++) {
      uint32_t a, b;
      do {
        a = xo_bounded(&r, (uint32_t)n);
        b = xo_bounded(&r, (uint32_t)n);
      } while (a == b);
      src[e] = (int32_t)a;
      dst[e] = (int32_t)b;
    }
  }
  return m;
}

/* R-MAT: m edge draws on 2^scale vertices.  At every level the quadrant is
 * (0,0) with probability a, (0,1) with b, (1,0) with c, (1,1) otherwise.
 * Self-loops are dropped (not redrawn); duplicates are kept.  If permute != 0
 * vertex ids are relabelled by a seeded uniform permutation.
 * Writes at most m edges and returns the number kept. */
int64_t gg_rmat_edges(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed,
                      int32_t permute, int32_t* src, int32_t* dst) {
  if (scale < 1 || scale > 30 || m < 0) return -1;
  const int64_t n = (int64_t)1 << scale;
  const double ab = a + b, abc = a + b + c;
  const int64_t nchunks = (m + GG_CHUNK - 1) / GG_CHUNK;
  uint8_t* keep = (uint8_t*)malloc((size_t)(m > 0 ? m : 1));
  if (!keep) return -2;
#pragma omp parallel for schedule(static)
  for (int64_t ch = 0; ch < nchunks; ch++) {
    xo_t r;
    xo_seed(&r, seed, (uint64_t)ch);
    const int64_t lo = ch * GG_CHUNK, hi = (lo + GG_CHUNK < m) ? lo + GG_CHUNK : m;
    for (int64_t e = lo; e < hi; e++) {
      uint32_t u = 0, v = 0;
      for (int32_t l = 0; l < scale; l++) {
        const double p = xo_unit(&r);
        uint32_t bu, bv;
        if (p < a) { bu = 0; bv = 0; }
        else if (p < ab) { bu = 0; bv = 1; }
        else if (p < abc) { bu = 1; bv = 0; }
        else { bu = 1; bv = 1; }
        u = (u << 1) | bu;
        v = (v << 1) | bv;
      }
      src[e] = (int32_t)u;
      dst[e] = (int32_t)v;
      keep[e] = (u != v);
    }
  }
  if (permute) {
    int32_t* perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!perm) { free(keep); return -2; }
    for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
    xo_t r;
    xo_seed(&r, seed, 0xFFFFFFFFull);
    for (int64_t i = n - 1; i > 0; i--) { /* Fisher-Yates */
      const int64_t j = (int64_t)xo_bounded(&r, (uint32_t)(i + 1));
      const int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; e++) {
      src[e] = perm[src[e]];
      dst[e] = perm[dst[e]];
    }
    free(perm);
  }
  int64_t k = 0;
  for (int64_t e = 0; e < m; e++) {
    if (keep[e]) { src[k] = src[e]; dst[k] = dst[e]; k++; }
  }
  free(keep);
  return k;
}

/* Number of undirected neighbour pairs of a rows x cols 4-neighbour grid. */
int64_t gg_grid_pairs(int32_t rows, int32_t cols) {
  return (int64_t)rows * (cols - 1) + (int64_t)(rows - 1) * cols;
}

/* 4-neighbour grid, vertex id = r*cols + c.  Undirected pairs are numbered
 * horizontal first (r*(cols-1)+c), then vertical.  ndel pairs, chosen uniformly
 * without replacement, are removed; every remaining pair is stored in both
 * directions.  Returns the number of directed edges written (2*(pairs-ndel)). */
int64_t gg_grid_edges(int32_t rows, int32_t cols, int64_t ndel, uint64_t seed, int32_t* src,
                      int32_t* dst) {
  if (rows < 1 || cols < 1) return -1;
  const int64_t np = gg_grid_pairs(rows, cols);
  if (ndel < 0 || ndel > np) return -1;
  uint8_t* dead = (uint8_t*)calloc((size_t)(np > 0 ? np : 1), 1);
  if (!dead) return -2;
  if (ndel > 0) {
    /* Partial Fisher-Yates over pair ids: the first ndel of a uniform shuffle. */
    int64_t* ids = (int64_t*)malloc((size_t)np * sizeof(int64_t));
    if (!ids) { free(dead); return -2; }
    for (int64_t i = 0; i < np; i++) ids[i] = i;
    xo_t r;
    xo_seed(&r, seed, 0);
    for (int64_t i = 0; i < ndel; i++) {
      const int64_t j = i + (int64_t)xo_bounded(&r, (uint32_t)(np - i));
      const int64_t t = ids[i]; ids[i] = ids[j]; ids[j] = t;
      dead[ids[i]] = 1;
    }
    free(ids);
  }
  const int64_t nh = (int64_t)rows * (cols - 1);
  int64_t k = 0;
  for (int64_t p = 0; p < np; p++) {
    if (dead[p]) continue;
    int64_t a, b;
    if (p < nh) {
      const int64_t r = p / (cols - 1), c = p % (cols - 1);
      a = r * cols + c; b = a + 1;
    } else {
      const int64_t q = p - nh;
      const int64_t r = q / cols, c = q % cols;
      a = r * cols + c; b = a + cols;
    }
    src[k] = (int32_t)a; dst[k] = (int32_t)b; k++;
    src[k] = (int32_t)b; dst[k] = (int32_t)a; k++;
  }
  free(dead);
  return k;
}

/* ------------------------------------------------------------------------- */
/* CSR assembly                                                               */
/* ------------------------------------------------------------------------- */

static int cmp_i32(const void* x, const void* y) {
  const int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
  return (a > b) - (a < b);
}

/* Edge list -> CSR by source (counting sort), each row sorted by column.
 * rowptr has n+1 entries, colidx m entries.  Returns 0, or -1 on a bad id. */
int32_t gg_csr_build(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, int32_t* rowptr,
                     int32_t* colidx) {
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -2;
  for (int64_t e = 0; e < m; e++) {
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) { free(cnt); return -1; }
    cnt[src[e] + 1]++;
  }
  for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
  for (int64_t i = 0; i <= n; i++) rowptr[i] = (int32_t)cnt[i];
  for (int64_t e = 0; e < m; e++) colidx[cnt[src[e]]++] = dst[e];
  free(cnt);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; i++) {
    const int64_t lo = rowptr[i], hi = rowptr[i + 1];
    if (hi - lo > 1) qsort(colidx + lo, (size_t)(hi - lo), sizeof(int32_t), cmp_i32);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Edge weights (indexed by CSR position)                                     */
/* ------------------------------------------------------------------------- */

/* Integers uniform in [lo, hi]. */
void gg_weights_u32(int64_t m, uint32_t lo, uint32_t hi, uint64_t seed, uint32_t* w) {
  const int64_t nchunks = (m + GG_CHUNK - 1) / GG_CHUNK;
  const uint32_t span = hi - lo + 1u; /* hi-lo < 2^32-1 assumed */
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nchunks; c++) {
    xo_t r;
    xo_seed(&r, seed, (uint64_t)c);
    const int64_t e0 = c * GG_CHUNK, e1 = (e0 + GG_CHUNK < m) ? e0 + GG_CHUNK : m;
    for (int64_t e = e0; e < e1; e++) w[e] = lo + xo_bounded(&r, span);
  }
}

/* fp32 uniform on (0,1]: (j+1) * 2^-24 with j uniform in [0, 2^24).  Every value
 * is exact in fp32 and every sum of < 2^29 of them is exact in fp64. */
void gg_weights_f32_unit(int64_t m, uint64_t seed, float* w) {
  const int64_t nchunks = (m + GG_CHUNK - 1) / GG_CHUNK;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nchunks; c++) {
    xo_t r;
    xo_seed(&r, seed, (uint64_t)c);
    const int64_t e0 = c * GG_CHUNK, e1 = (e0 + GG_CHUNK < m) ? e0 + GG_CHUNK : m;
    for (int64_t e = e0; e < e1; e++) w[e] = (float)((double)((xo_next(&r) >> 40) + 1) * 0x1.0p-24);
  }
}

/* fp32 on the closed range [0, 2]: j * 2^-23 with j uniform in [0, 2^24]. Zero
 * weights occur.  (The randomised weights of the paper's validation run,
 * Section 4.2.) */
void gg_weights_f32_range02(int64_t m, uint64_t seed, float* w) {
  const int64_t nchunks = (m + GG_CHUNK - 1) / GG_CHUNK;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nchunks; c++) {
    xo_t r;
    xo_seed(&r, seed, (uint64_t)c);
    const int64_t e0 = c * GG_CHUNK, e1 = (e0 + GG_CHUNK < m) ? e0 + GG_CHUNK : m;
    for (int64_t e = e0; e < e1; e++)
      w[e] = (float)((double)xo_bounded(&r, (1u << 24) + 1u) * 0x1.0p-23);
  }
}

/* fp32 lognormal(0,1): exp(z), z standard normal by Box-Muller in fp64. */
void gg_weights_f32_lognormal(int64_t m, uint64_t seed, float* w) {
  const int64_t nchunks = (m + GG_CHUNK - 1) / GG_CHUNK;
  const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nchunks; c++) {
    xo_t r;
    xo_seed(&r, seed, (uint64_t)c);
    const int64_t e0 = c * GG_CHUNK, e1 = (e0 + GG_CHUNK < m) ? e0 + GG_CHUNK : m;
    for (int64_t e = e0; e < e1; e++) {
      const double u1 = 1.0 - xo_unit(&r); /* (0,1] */
      const double u2 = xo_unit(&r);
      const double z = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
      w[e] = (float)exp(z);
    }
  }
}

/* k distinct vertices drawn uniformly from those with out-degree >= 1
 * (sequential partial shuffle of the eligible set).  Returns the number
 * written: min(k, eligible). */
int64_t gg_pick_sources(int64_t n, const int32_t* rowptr, int64_t k, uint64_t seed, int32_t* out) {
  int32_t* elig = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!elig) return -2;
  int64_t ne = 0;
  for (int64_t i = 0; i < n; i++)
    if (rowptr[i + 1] > rowptr[i]) elig[ne++] = (int32_t)i;
  if (k > ne) k = ne;
  xo_t r;
  xo_seed(&r, seed, 7);
  for (int64_t i = 0; i < k; i++) {
    const int64_t j = i + (int64_t)xo_bounded(&r, (uint32_t)(ne - i));
    const int32_t t = elig[i]; elig[i] = elig[j]; elig[j] = t;
    out[i] = elig[i];
  }
  free(elig);
  return k;
}

/* Uniform doubles in [0,1) for host-side schedulers (Poisson arrivals etc). */
void gg_uniform(int64_t count, uint64_t seed, double* out) {
  xo_t r;
  xo_seed(&r, seed, 11);
  for (int64_t i = 0; i < count; i++) out[i] = xo_unit(&r);
}
