/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously correct CPU
 * implementation of what the GOVM hot path computes.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header or constant with the HIP library.
 *
 * What the method computes.  GOVM (Section 3.4, Algorithm 2) repeats the
 * (min,+) vector-matrix step  p_ij = min_k (p_ik + a_kj)  over the rows whose
 * distance changed in the previous step and stops once no distance changes;
 * Section 3.1 argues this fixed point is the Floyd-Warshall recurrence's, and
 * Section 3.5 says it stops when the weights of all shortest paths no longer
 * change.  For non-negative weights that fixed point has a plain definition:
 *
 *     d(v) = min over directed s->v paths of the path weight,
 *     d(s) = 0, d(v) = INF when no path exists.
 *
 * So the distance oracle is that definition computed by textbook methods
 * (Section 2: Dijkstra, Floyd-Warshall; plus brute-force path enumeration), in
 * three arithmetic modes:
 *   - u32 weights, exact 64-bit sums, clipped to 0xFFFFFFFF (the uint32 INF);
 *   - f32 weights, exact-as-possible fp64 sums (the tolerance reference);
 *   - f32 weights, the fp32 left fold d' = fl32(d + w) (round to nearest even),
 *     which is the unique fixed point of the same iteration run in fp32.
 *
 * Every result also carries hops(v): the least hop count among optimal paths,
 * found with lexicographic (distance, hops) keys.
 *
 * The invariant checker verifies any candidate distance vector without a
 * reference (source is 0; no edge can be relaxed; every finite vertex has a
 * tight in-edge chain back to the source; INF exactly on unreachable vertices).
 *
 * Signed int32 weights (negative edges allowed) have their own reference,
 * Bellman-Ford with Algorithm 2's source guard (oracle_bellman_ford_i32).
 *
 * The one restatement of the method itself (oracle_govm_*) follows
 * Algorithm 2's steps in the paper's order.  It is used for step counts and
 * work counters (mu), never as the distance reference.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_INF32 0xFFFFFFFFu

/* ------------------------------------------------------------------------- */
/* Binary min-heap of (key, hops, vertex) with lazy deletion.                  */
/* ------------------------------------------------------------------------- */
typedef struct {
  double kd;   /* distance key (every mode's value fits a double exactly: u64 sums of
                  u32 weights stay below 2^53 for the sizes used, and fp32 values are
                  exact in double) */
  uint64_t ku; /* exact u64 key for the u32 mode */
  int32_t h;
  int32_t v;
} hent_t;

typedef struct {
  hent_t* a;
  int64_t size, cap;
  int use_u;
} heap_t;

static int hless(const heap_t* H, const hent_t* x, const hent_t* y) {
  if (H->use_u) {
    if (x->ku != y->ku) return x->ku < y->ku;
  } else {
    if (x->kd != y->kd) return x->kd < y->kd;
  }
  return x->h < y->h;
}

static int hpush(heap_t* H, hent_t e) {
  if (H->size == H->cap) {
    int64_t nc = H->cap ? 2 * H->cap : 1024;
    hent_t* na = (hent_t*)realloc(H->a, (size_t)nc * sizeof(hent_t));
    if (!na) return -1;
    H->a = na;
    H->cap = nc;
  }
  int64_t i = H->size++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (!hless(H, &e, &H->a[p])) break;
    H->a[i] = H->a[p];
    i = p;
  }
  H->a[i] = e;
  return 0;
}

static hent_t hpop(heap_t* H) {
  hent_t top = H->a[0];
  hent_t last = H->a[--H->size];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, c = i;
    const hent_t* best = &last;
    if (l < H->size && hless(H, &H->a[l], best)) { c = l; best = &H->a[l]; }
    if (r < H->size && hless(H, &H->a[r], best)) { c = r; best = &H->a[r]; }
    if (c == i) break;
    H->a[i] = H->a[c];
    i = c;
  }
  if (H->size > 0) H->a[i] = last;
  return top;
}

/* ------------------------------------------------------------------------- */
/* Dijkstra (Section 2.1), binary heap, lexicographic (distance, hops) keys.   */
/* ------------------------------------------------------------------------- */

/* u32 weights; sums in uint64; output clipped to 0xFFFFFFFF, which is also the
 * unreachable marker.  hops[v] = -1 when unreachable. Returns 0 or -1 (oom). */
int32_t oracle_sssp_u32(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                        const uint32_t* w, int32_t s, uint32_t* dist, int32_t* hops) {
  uint64_t* d = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
  int32_t* h = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  uint8_t* done = (uint8_t*)calloc((size_t)n, 1);
  heap_t H = {0};
  H.use_u = 1;
  if (!d || !h || !done) { free(d); free(h); free(done); return -1; }
  for (int32_t v = 0; v < n; v++) { d[v] = UINT64_MAX; h[v] = -1; }
  d[s] = 0;
  h[s] = 0;
  hent_t e0 = {0.0, 0, 0, s};
  if (hpush(&H, e0)) goto oom;
  while (H.size > 0) {
    hent_t t = hpop(&H);
    const int32_t u = t.v;
    if (done[u]) continue;
    if (t.ku != d[u] || t.h != h[u]) continue; /* stale entry */
    done[u] = 1;
    for (int32_t e = rowptr[u]; e < rowptr[u + 1]; e++) {
      const int32_t v = colidx[e];
      const uint64_t nd = d[u] + (uint64_t)w[e];
      const int32_t nh = h[u] + 1;
      if (nd < d[v] || (nd == d[v] && nh < h[v])) {
        d[v] = nd;
        h[v] = nh;
        hent_t x = {0.0, nd, nh, v};
        if (hpush(&H, x)) goto oom;
      }
    }
  }
  for (int32_t v = 0; v < n; v++) dist[v] = d[v] >= (uint64_t)OR_INF32 ? OR_INF32 : (uint32_t)d[v];
  /* A clipped (>= 2^32-1) distance reads as unreachable in uint32; keep hops of
   * real paths anyway. */
  if (hops) memcpy(hops, h, (size_t)n * sizeof(int32_t));
  free(d); free(h); free(done); free(H.a);
  return 0;
oom:
  free(d); free(h); free(done); free(H.a);
  return -1;
}

/* f32 weights.  mode 0: fp64 sums of the exact fp32 weight values, written to
 * dist64.  mode 1: fp32 left fold d' = fl32(d + w), written to dist32.
 * Unreachable = +inf.  Returns 0 or -1. */
static int32_t sssp_f32_impl(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                             const float* w, int32_t s, int mode, double* dist64, float* dist32,
                             int32_t* hops) {
  double* d = (double*)malloc((size_t)n * sizeof(double));
  int32_t* h = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  uint8_t* done = (uint8_t*)calloc((size_t)n, 1);
  heap_t H = {0};
  if (!d || !h || !done) { free(d); free(h); free(done); return -1; }
  for (int32_t v = 0; v < n; v++) { d[v] = INFINITY; h[v] = -1; }
  d[s] = 0.0;
  h[s] = 0;
  hent_t e0 = {0.0, 0, 0, s};
  if (hpush(&H, e0)) goto oom;
  while (H.size > 0) {
    hent_t t = hpop(&H);
    const int32_t u = t.v;
    if (done[u]) continue;
    if (t.kd != d[u] || t.h != h[u]) continue;
    done[u] = 1;
    for (int32_t e = rowptr[u]; e < rowptr[u + 1]; e++) {
      const int32_t v = colidx[e];
      double nd;
      if (mode == 0) {
        nd = d[u] + (double)w[e];
      } else {
        volatile float a = (float)d[u]; /* d[u] already holds an fp32 value */
        volatile float b = w[e];
        volatile float c = a + b;       /* one fp32 add, round to nearest even */
        nd = (double)c;
      }
      const int32_t nh = h[u] + 1;
      if (nd < d[v] || (nd == d[v] && nh < h[v])) {
        d[v] = nd;
        h[v] = nh;
        hent_t x = {nd, 0, nh, v};
        if (hpush(&H, x)) goto oom;
      }
    }
  }
  for (int32_t v = 0; v < n; v++) {
    if (mode == 0) dist64[v] = d[v];
    else dist32[v] = (float)d[v];
  }
  if (hops) memcpy(hops, h, (size_t)n * sizeof(int32_t));
  free(d); free(h); free(done); free(H.a);
  return 0;
oom:
  free(d); free(h); free(done); free(H.a);
  return -1;
}

int32_t oracle_sssp_f64(int32_t n, const int32_t* rowptr, const int32_t* colidx, const float* w,
                        int32_t s, double* dist, int32_t* hops) {
  return sssp_f32_impl(n, rowptr, colidx, w, s, 0, dist, NULL, hops);
}

int32_t oracle_sssp_f32fold(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                            const float* w, int32_t s, float* dist, int32_t* hops) {
  return sssp_f32_impl(n, rowptr, colidx, w, s, 1, NULL, dist, hops);
}

/* ------------------------------------------------------------------------- */
/* Floyd-Warshall (Section 2.3), dense n x n, row-major D[i*n+j].              */
/* ------------------------------------------------------------------------- */

/* u32 weights, uint64 entries, UINT64_MAX = no path.  Diagonal 0. */
void oracle_fw_u64(int32_t n, const int32_t* rowptr, const int32_t* colidx, const uint32_t* w,
                   uint64_t* D) {
  const size_t nn = (size_t)n * (size_t)n;
  for (size_t i = 0; i < nn; i++) D[i] = UINT64_MAX;
  for (int32_t i = 0; i < n; i++) {
    D[(size_t)i * n + i] = 0;
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      const size_t ij = (size_t)i * n + colidx[e];
      if ((uint64_t)w[e] < D[ij]) D[ij] = w[e];
    }
  }
  for (int32_t k = 0; k < n; k++)
    for (int32_t i = 0; i < n; i++) {
      const uint64_t dik = D[(size_t)i * n + k];
      if (dik == UINT64_MAX) continue;
      for (int32_t j = 0; j < n; j++) {
        const uint64_t dkj = D[(size_t)k * n + j];
        if (dkj == UINT64_MAX) continue;
        if (dik + dkj < D[(size_t)i * n + j]) D[(size_t)i * n + j] = dik + dkj;
      }
    }
}

/* f32 weights, fp64 entries, +inf = no path.  Diagonal 0. */
void oracle_fw_f64(int32_t n, const int32_t* rowptr, const int32_t* colidx, const float* w,
                   double* D) {
  const size_t nn = (size_t)n * (size_t)n;
  for (size_t i = 0; i < nn; i++) D[i] = INFINITY;
  for (int32_t i = 0; i < n; i++) {
    D[(size_t)i * n + i] = 0.0;
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      const size_t ij = (size_t)i * n + colidx[e];
      if ((double)w[e] < D[ij]) D[ij] = w[e];
    }
  }
  for (int32_t k = 0; k < n; k++)
    for (int32_t i = 0; i < n; i++) {
      const double dik = D[(size_t)i * n + k];
      if (dik == INFINITY) continue;
      for (int32_t j = 0; j < n; j++) {
        const double c = dik + D[(size_t)k * n + j];
        if (c < D[(size_t)i * n + j]) D[(size_t)i * n + j] = c;
      }
    }
}

/* ------------------------------------------------------------------------- */
/* Brute force: every simple path from s, depth first (tiny graphs only).      */
/* ------------------------------------------------------------------------- */
typedef struct {
  const int32_t* rowptr;
  const int32_t* colidx;
  const void* w;
  int mode; /* 0: u32 exact, 1: f32 -> f64 exact sum, 2: f32 left fold in fp32 */
  uint8_t* on_path;
  uint64_t* bu;
  double* bd;
  int32_t* bh;
} bf_t;

static void bf_visit(bf_t* B, int32_t u, uint64_t su, double sd, float sf, int32_t hops) {
  /* record the path ending at u */
  if (B->mode == 0) {
    if (su < B->bu[u] || (su == B->bu[u] && hops < B->bh[u])) { B->bu[u] = su; B->bh[u] = hops; }
  } else {
    const double val = (B->mode == 1) ? sd : (double)sf;
    if (val < B->bd[u] || (val == B->bd[u] && hops < B->bh[u])) { B->bd[u] = val; B->bh[u] = hops; }
  }
  B->on_path[u] = 1;
  for (int32_t e = B->rowptr[u]; e < B->rowptr[u + 1]; e++) {
    const int32_t v = B->colidx[e];
    if (B->on_path[v]) continue;
    if (B->mode == 0) {
      bf_visit(B, v, su + ((const uint32_t*)B->w)[e], 0.0, 0.0f, hops + 1);
    } else {
      const float we = ((const float*)B->w)[e];
      volatile float a = sf, b = we;
      volatile float c = a + b;
      bf_visit(B, v, 0, sd + (double)we, c, hops + 1);
    }
  }
  B->on_path[u] = 0;
}

/* mode 0: u32 weights -> dist_u64; mode 1: f32 weights -> exact fp64 sums in
 * dist_f64; mode 2: f32 weights -> fp32 left fold in dist_f64.  No path:
 * UINT64_MAX / +inf and hops -1.  n <= 12. */
int32_t oracle_brute(int32_t n, const int32_t* rowptr, const int32_t* colidx, const void* w,
                     int32_t s, int32_t mode, uint64_t* dist_u64, double* dist_f64,
                     int32_t* hops) {
  if (n > 12) return -1;
  uint8_t on_path[12] = {0};
  bf_t B = {rowptr, colidx, w, mode, on_path, dist_u64, dist_f64, hops};
  for (int32_t v = 0; v < n; v++) {
    if (mode == 0) dist_u64[v] = UINT64_MAX;
    else dist_f64[v] = INFINITY;
    hops[v] = -1;
  }
  bf_visit(&B, s, 0, 0.0, 0.0f, 0);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Breadth-first levels (reachability; the unit-weight special case).          */
/* ------------------------------------------------------------------------- */
/*
 * Signed int32 weights: Bellman-Ford (Section 2.2).  With negative weights a
 * shortest-path distance exists when no cycle of negative weight is reachable.
 * Algorithm 2 never lowers the source's own distance (its "index != source"
 * test), so the fixed point it reaches is the shortest-path distance of the
 * graph without the edges into s; that is what this computes: rounds over
 * every edge whose target is not s, exact 64-bit sums, until a round changes
 * nothing (return 1) or n rounds have all changed something, which only a
 * reachable negative cycle allows (return 0, dist then meaningless).
 * dist: int64, INT64_MAX = unreachable.
 */
int32_t oracle_bellman_ford_i32(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                                const int32_t* w, int32_t s, int64_t* dist) {
  for (int32_t v = 0; v < n; v++) dist[v] = INT64_MAX;
  dist[s] = 0;
  for (int32_t round = 0; round < n; round++) {
    int changed = 0;
    for (int32_t u = 0; u < n; u++) {
      if (dist[u] == INT64_MAX) continue;
      for (int32_t e = rowptr[u]; e < rowptr[u + 1]; e++) {
        const int32_t v = colidx[e];
        if (v == s) continue;
        const int64_t c = dist[u] + (int64_t)w[e];
        if (c < dist[v]) {
          dist[v] = c;
          changed = 1;
        }
      }
    }
    if (!changed) return 1;
  }
  return 0;
}

int32_t oracle_bfs(int32_t n, const int32_t* rowptr, const int32_t* colidx, int32_t s,
                   int32_t* level) {
  int32_t* q = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!q) return -1;
  for (int32_t v = 0; v < n; v++) level[v] = -1;
  int32_t head = 0, tail = 0;
  level[s] = 0;
  q[tail++] = s;
  while (head < tail) {
    const int32_t u = q[head++];
    for (int32_t e = rowptr[u]; e < rowptr[u + 1]; e++) {
      const int32_t v = colidx[e];
      if (level[v] < 0) { level[v] = level[u] + 1; q[tail++] = v; }
    }
  }
  free(q);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Invariant checker.                                                          */
/*   V1  d[s] == 0                                                              */
/*   V2  every edge (u,v,w) with d[u] < INF has d[v] <= d[u] (+) w              */
/*   V3  a search from s over tight edges (d[v] == d[u] (+) w, d[u] < INF)      */
/*       reaches every v with d[v] < INF                                        */
/*   V4  d[v] == INF for every v unreachable from s                             */
/* (+) is the saturating uint32 add, or the fp32 round-to-nearest add.  The     */
/* converse of V4 (reachable => finite) follows from V1 and V2 by induction     */
/* along a path, except where the saturating add makes INF the right answer,   */
/* so V2 is what rejects a reachable vertex wrongly reported as INF.            */
/* Returns 0 when all hold, else the first failing rule (1..4); *bad gets a     */
/* vertex that fails it.  -1 on allocation failure.                              */
/* ------------------------------------------------------------------------- */
static inline uint32_t sat_add_u32(uint32_t a, uint32_t b) {
  const uint64_t s = (uint64_t)a + b;
  return s >= OR_INF32 ? OR_INF32 : (uint32_t)s;
}

static inline float add_f32(float a, float b) {
  volatile float x = a, y = b;
  volatile float z = x + y;
  return z;
}

static int32_t check_impl(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                          const void* w, int32_t s, const void* dvec, int is_f32, int32_t* bad) {
  const uint32_t* du = (const uint32_t*)dvec;
  const float* df = (const float*)dvec;
  const uint32_t* wu = (const uint32_t*)w;
  const float* wf = (const float*)w;
#define D_FIN(x) (is_f32 ? (df[x] != INFINITY) : (du[x] != OR_INF32))
  *bad = -1;
  /* V1 */
  if (is_f32 ? !(df[s] == 0.0f && !signbit(df[s])) : (du[s] != 0)) { *bad = s; return 1; }
  /* V2 */
  for (int32_t u = 0; u < n; u++) {
    if (!D_FIN(u)) continue;
    for (int32_t e = rowptr[u]; e < rowptr[u + 1]; e++) {
      const int32_t v = colidx[e];
      if (is_f32) {
        if (!(df[v] <= add_f32(df[u], wf[e]))) { *bad = v; return 2; }
      } else {
        if (du[v] > sat_add_u32(du[u], wu[e])) { *bad = v; return 2; }
      }
    }
  }
  /* V3: search over tight edges */
  uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);
  int32_t* q = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* lvl = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!seen || !q || !lvl) { free(seen); free(q); free(lvl); return -1; }
  int32_t head = 0, tail = 0;
  seen[s] = 1;
  q[tail++] = s;
  while (head < tail) {
    const int32_t u = q[head++];
    if (!D_FIN(u)) continue;
    for (int32_t e = rowptr[u]; e < rowptr[u + 1]; e++) {
      const int32_t v = colidx[e];
      if (seen[v]) continue;
      const int tight = is_f32 ? (df[v] == add_f32(df[u], wf[e]))
                               : (du[v] == sat_add_u32(du[u], wu[e]));
      if (tight && D_FIN(v)) { seen[v] = 1; q[tail++] = v; }
    }
  }
  int32_t rc = 0;
  for (int32_t v = 0; v < n && !rc; v++)
    if (D_FIN(v) && !seen[v]) { *bad = v; rc = 3; }
  /* V4 */
  if (!rc) {
    oracle_bfs(n, rowptr, colidx, s, lvl);
    for (int32_t v = 0; v < n && !rc; v++)
      if (lvl[v] < 0 && D_FIN(v)) { *bad = v; rc = 4; }
  }
  free(seen); free(q); free(lvl);
  return rc;
#undef D_FIN
}

int32_t oracle_check_u32(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                         const uint32_t* w, int32_t s, const uint32_t* d, int32_t* bad) {
  return check_impl(n, rowptr, colidx, w, s, d, 0, bad);
}

int32_t oracle_check_f32(int32_t n, const int32_t* rowptr, const int32_t* colidx, const float* w,
                         int32_t s, const float* d, int32_t* bad) {
  return check_impl(n, rowptr, colidx, w, s, d, 1, bad);
}

/* ------------------------------------------------------------------------- */
/* Algorithm 2 (GOVM) restated sequentially, in the paper's order.             */
/*                                                                              */
/* Readings where the paper is silent:                                           */
/*   alpha starts at INF everywhere except alpha[source] = 0;                   */
/*   delta starts as {source}, beta empty;                                       */
/*   beta is cleared after it is copied into delta, so only vertices updated    */
/*   in the current step are expanded in the next one;                          */
/*   the strict improvement test and the index != source guard are kept;        */
/*   the step counter is capped at n.                                            */
/* order 0: rows in index order, in-place (a row may read a value lowered       */
/*          earlier in the same step); order 1: Jacobi (every row of a step      */
/*          reads the values the step started with); order 2: rows of each      */
/*          step visited in a seeded random order, in place.                      */
/* Outputs: dist (u32, or f32 as bits), and counters[5] = {steps, converged,     */
/* sum_t |delta_t| over rows with out-edges, edges scanned, improvements};       */
/* updates (optional, n entries): how many times each vertex's distance was     */
/* lowered (the paper's path updates, Section 4.2: 1 for a vertex whose first  */
/* path found is already shortest).                                              */
/* ------------------------------------------------------------------------- */
static uint64_t lcg_next(uint64_t* x) { *x = *x * 6364136223846793005ULL + 1442695040888963407ULL; return *x >> 33; }

int32_t oracle_govm(int32_t n, const int32_t* rowptr, const int32_t* colidx, const void* w,
                    int32_t is_f32, int32_t source, int32_t order, uint64_t seed, void* dist,
                    int64_t* counters, int32_t* updates) {
  uint32_t* au = (uint32_t*)dist;
  float* af = (float*)dist;
  uint8_t* delta = (uint8_t*)calloc((size_t)n, 1);
  uint8_t* beta = (uint8_t*)calloc((size_t)n, 1);
  uint32_t* snap = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
  int32_t* perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!delta || !beta || !snap || !perm) { free(delta); free(beta); free(snap); free(perm); return -1; }
  for (int32_t v = 0; v < n; v++) {
    if (is_f32) af[v] = INFINITY; else au[v] = OR_INF32;
    perm[v] = v;
    if (updates) updates[v] = 0;
  }
  if (is_f32) af[source] = 0.0f; else au[source] = 0;
  delta[source] = 1;
  int64_t steps = 0, converged = 0, fr = 0, scanned = 0, impr = 0;
  uint64_t rs = seed * 2862933555777941757ULL + 3037000493ULL;
  while (steps < n) {
    steps++;
    int ptr = 0;
    if (order == 1) memcpy(snap, dist, (size_t)n * sizeof(uint32_t));
    if (order == 2)
      for (int32_t i = n - 1; i > 0; i--) {
        int32_t j = (int32_t)(lcg_next(&rs) % (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
      }
    for (int32_t jj = 0; jj < n; jj++) {
      const int32_t j = perm[jj];
      const int32_t start = rowptr[j], end = rowptr[j + 1];
      if (!(delta[j] && start != end)) continue;
      fr++;
      const uint32_t aju = (order == 1) ? snap[j] : au[j];
      float ajf;
      { uint32_t bits = aju; memcpy(&ajf, &bits, 4); }
      for (int32_t k = start; k < end; k++) {
        const int32_t index = colidx[k];
        scanned++;
        if (is_f32) {
          const float cand = add_f32(ajf, ((const float*)w)[k]);
          if (af[index] > cand && index != source) {
            af[index] = cand;
            beta[index] = 1;
            ptr = 1;
            impr++;
            if (updates) updates[index]++;
          }
        } else {
          const uint32_t cand = sat_add_u32(aju, ((const uint32_t*)w)[k]);
          if (au[index] > cand && index != source) {
            au[index] = cand;
            beta[index] = 1;
            ptr = 1;
            impr++;
            if (updates) updates[index]++;
          }
        }
      }
    }
    if (!ptr) { converged = 1; break; }
    memcpy(delta, beta, (size_t)n);
    memset(beta, 0, (size_t)n);
  }
  counters[0] = steps;
  counters[1] = converged;
  counters[2] = fr;
  counters[3] = scanned;
  counters[4] = impr;
  free(delta); free(beta); free(snap); free(perm);
  return 0;
}
