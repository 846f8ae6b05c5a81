// govm_tile.hip -- GOVM for many sources at once on an [n x K] distance tile.
//
// Multi-source and all-pairs shortest paths repeat Algorithm 2 per source
// (Section 1; APSP cost mu * S_wcc * E_wcc in Section 3.4), and Section 3.5
// notes that work for different sources never updates the same path.  The
// tile runs K sources in lock-step: column j of D holds source j's alpha, and
// a per-vertex K-bit mask marks the sources whose alpha[v] changed in the last
// step (delta per source).  The union frontier is every vertex with any mask
// bit; one read of a row's edges then serves every source active there.
//
// Layout: D is vertex-major (the K distances of a vertex are contiguous, 4*K
// bytes), so for an edge (u, v) the active sources of one 64-column segment
// are served by 16 lanes loading 16 bytes each from D[v] -- one coalesced
// 256-byte read per (edge, segment) -- and segments with no active source at u
// are skipped.
//
// A step is two launches:
//  1. compaction: every vertex with a mask bit in the step's slot joins the
//     union frontier, binned by out-degree into a 16-lane-group tier, a
//     wavefront tier and workgroup chunks;
//  2. relaxation: for each frontier row and active segment, lanes hold the
//     row's distances of their 4 sources in registers and stream the row's
//     edges, 4 edges in flight per 16-lane group.  A candidate below the
//     target's distance (read with a plain load) is written with a
//     non-returning atomicMin and sets the target's bit in the next step's
//     mask.  No lane waits for an atomic: the plain value read is at least
//     the value just before the atomic (distances only decrease), so every
//     real improvement sets its bit; when another lane got there first, that
//     lane set the bit too.
// Masks and queues rotate over three slots (a slot is cleared one step after
// it was read), per-step counters and column-activity words over four.
#include <algorithm>

#include "govm_host.hpp"

namespace dawn {

constexpr int kTileU = 4;  // edges in flight per 16-lane group
// Persistent tile launches default to one 1024-thread workgroup per compute
// unit: each workgroup's arrival at a grid barrier costs serial time at the
// barrier word, and runs with thousands of steps (grids) pay two barriers per
// step (measured on a 2048 x 2048 grid: about 130 us per step instead of 335
// with four 256-thread workgroups per compute unit).
constexpr int kTilePersistentThreads = 1024;

// ---------------------------------------------------------------------------
// reset / seed / admit / evict
// ---------------------------------------------------------------------------
template <bool F32>
__global__ void tile_fill_kernel(TileArgs A) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nd4 = (int64_t)A.n * A.K / 4;
  const uint32_t inf = inf_bits<F32>();
  uint4* d4 = reinterpret_cast<uint4*>(A.D);
  if (A.D)
    for (int64_t i = tid; i < nd4; i += stride) d4[i] = make_uint4(inf, inf, inf, inf);
  const int64_t nm = (int64_t)A.n * A.nseg;
  for (int r = 0; r < 3; r++)
    for (int64_t i = tid; i < nm; i += stride) A.mk[r][i] = 0ull;
  if (A.vis)
    for (int64_t i = tid; i < nm; i += stride) A.vis[i] = 0ull;
  if (blockIdx.x == 0) {
    uint32_t* c = reinterpret_cast<uint32_t*>(A.ctl);
    for (int i = threadIdx.x; i < (int)(sizeof(TileCtl) / 4); i += blockDim.x) c[i] = 0u;
  }
}

// Put source s into column col before step t (the next step to run): alpha = 0
// at s and s active for col; the compaction of step t picks s up.
__device__ void tile_put_source(const TileArgs& A, int32_t col, int32_t s, uint32_t t) {
  TileCtl* C = A.ctl;
  const int seg = col >> 6;
  const unsigned long long bit = 1ull << (col & 63);
  if (A.D) A.D[(size_t)s * A.K + col] = 0u;
  atomicOr(&A.mk[t % 3][(size_t)s * A.nseg + seg], bit);
  atomicOr(&C->colact[t % kRot][seg], bit);
  atomicOr(&C->live[seg], bit);
  st_agent_i(&C->colsteps[col], 0);
}

// A source outside [0, n) ends the run before its first step, as failed
// validation does (converged = -1).
__global__ void tile_seed_kernel(TileArgs A, const int32_t* sources, int32_t count) {
  if (ld_agent(&A.ctl->done)) return;  // validation failed
  for (int32_t j = threadIdx.x; j < count; j += blockDim.x) {
    const int32_t s = sources[j];
    if (s >= 0 && s < A.n) {
      tile_put_source(A, j, s, 0u);
    } else {
      st_agent_i(&A.ctl->converged, -1);
      st_agent(&A.ctl->done, 1u);
    }
  }
}

template <bool F32>
__global__ void tile_col_fill_kernel(TileArgs A, int32_t col) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < A.n; v += stride)
    A.D[(size_t)v * A.K + col] = inf_bits<F32>();
}

__global__ void tile_admit_kernel(TileArgs A, int32_t col, int32_t s) {
  if (threadIdx.x != 0) return;
  TileCtl* C = A.ctl;
  tile_put_source(A, col, s, ld_agent(&C->step));
  st_agent(&C->done, 0u);
  st_agent_i(&C->converged, 0);
}

// Cancel column col.  Its distances were just reset to INF (tile_col_fill),
// so whatever mask bits it still has produce no candidate below INF and the
// column falls silent within one step; here it leaves the live and active sets.
__global__ void tile_evict_kernel(TileArgs A, int32_t col) {
  if (threadIdx.x != 0) return;
  TileCtl* C = A.ctl;
  const uint32_t t = ld_agent(&C->step);
  const unsigned long long keep = ~(1ull << (col & 63));
  atomicAnd(&C->colact[t % kRot][col >> 6], keep);
  atomicAnd(&C->live[col >> 6], keep);
}

// ---------------------------------------------------------------------------
// compaction: masks of the step -> union-frontier queues
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tile_prologue(TileCtl* C, uint32_t step, int K) {
  // zero the counters of the next step and count this step for active columns
  const int rz = (step + 1) % kRot, rc = step % kRot;
  if (threadIdx.x < 4) st_agent(&C->cnt[rz][threadIdx.x].v, 0u);
  if (threadIdx.x == 4) st_agent(&C->cstep, step);
  if (threadIdx.x < kCtrStripes) {
    st_agent64(&C->ctr[threadIdx.x].fedges[rz], 0ull);
    st_agent64(&C->ctr[threadIdx.x].fpairs[rz], 0ull);
  }
  if (threadIdx.x < kSegMax) st_agent64(&C->colact[rz][threadIdx.x], 0ull);
  for (int j = threadIdx.x; j < K; j += blockDim.x)
    if ((ld_agent64(&C->colact[rc][j >> 6]) >> (j & 63)) & 1ull)
      st_agent_i(&C->colsteps[j], ld_agent_i(&C->colsteps[j]) + 1);
}

// Value of a 64-bit register in lane `src` (wave-uniform), as a scalar.
__device__ __forceinline__ unsigned long long lane64(unsigned long long x, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), src);
  return ((unsigned long long)hi << 32) | lo;
}

// Queued vertices are gathered per workgroup in LDS (per tier) and written to
// the global queues with one atomicAdd per tier per flush; each workgroup
// scans a contiguous range of vertices, so the queues come out nearly sorted.
constexpr int kCompactLds = 2048;

struct CompactShared {
  int32_t q[2][kCompactLds];
  uint32_t cnt[2];
  uint32_t base[2];
  uint32_t nch, chbase;  // workgroup-chunk records of the current batch of vertices
};

__device__ __forceinline__ void compact_push(bool pred, int32_t v, int t, CompactShared& sh) {
  const unsigned long long b = __ballot(pred);
  if (b == 0ull) return;
  const int leader = __ffsll((long long)b) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(&sh.cnt[t], (uint32_t)__popcll(b));
  base = __shfl(base, leader, kWave);
  if (pred) sh.q[t][base + lanes_below(b)] = v;
}

// Write the gathered entries of both tiers to the global queues of slot q.
// Reached by the whole workgroup.
__device__ __forceinline__ void compact_flush(const TileArgs& A, int q, int rc,
                                              CompactShared& sh) {
  TileCtl* C = A.ctl;
  __syncthreads();
  if (threadIdx.x < 2) {
    const uint32_t c = sh.cnt[threadIdx.x];
    sh.base[threadIdx.x] = c ? atomicAdd(&C->cnt[rc][threadIdx.x].v, c) : 0u;
  }
  __syncthreads();
  for (int t = 0; t < 2; t++) {
    int32_t* gq = t == 0 ? A.qgrp[q] : A.qwave[q];
    const uint32_t c = sh.cnt[t], b = sh.base[t];
    for (uint32_t j = threadIdx.x; j < c; j += blockDim.x) {
      if (b + j < A.cap_v) gq[b + j] = sh.q[t][j];
      else atomicOr(&C->overflow, 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x < 2) sh.cnt[threadIdx.x] = 0u;
  __syncthreads();
}

// Counts, from step 1 on, the (vertex, source) pairs whose distance the
// previous step lowered (a pair lowered twice in one step counts once).
// UW (hop-count tiles): the pairs of the step's masks were reached by the
// previous step (or are the sources, at step 0): their distance is the step
// number t, recorded here in the bit planes (bit b of t set: the pair's bit
// in plane b set), and they join the reached set `vis`.  Plane b is written
// whole, zeros included, at step 2^b, its first use, so nothing clears it.
template <bool UW>
__device__ __forceinline__ void tile_compact(const TileArgs& A, uint32_t step, uint32_t gb,
                                             uint32_t nb, Acc& acc, CompactShared& sh) {
  TileCtl* C = A.ctl;
  const int q = step % 3, rc = step % kRot;
  const int nseg = A.nseg;
  const int64_t n = A.n, bd = blockDim.x;
  const int64_t per = ((n + nb - 1) / nb + bd - 1) / bd * bd;
  const int64_t lo = (int64_t)gb * per, hi = min(n, lo + per);
  if (threadIdx.x < 2) sh.cnt[threadIdx.x] = 0u;
  if (threadIdx.x == 0) sh.nch = 0u;
  __syncthreads();
  for (int64_t v0 = lo; v0 < hi; v0 += bd) {
    const int64_t v = v0 + threadIdx.x;
    unsigned long long* mp = A.mk[q] + v * nseg;
    unsigned long long any = 0ull;
    uint32_t pairs = 0u;
    unsigned long long xs[kSegMax];
#pragma unroll
    for (int s = 0; s < kSegMax; s++) {
      xs[s] = 0ull;
      if (s < nseg && v < hi) {
        const unsigned long long x = mp[s];
        any |= x;
        pairs += (uint32_t)__popcll(x);
        if constexpr (UW) xs[s] = x;
      }
    }
    if (step > 0) acc.im += pairs;
    if constexpr (UW) {
      const size_t pn = (size_t)n * nseg;
      const bool first = step > 0 && (step & (step - 1u)) == 0u;  // step = 2^b
      if (first && v < hi) {
        unsigned long long* pp = A.planes + (size_t)(__ffs(step) - 1) * pn + v * nseg;
#pragma unroll
        for (int s = 0; s < kSegMax; s++)
          if (s < nseg) pp[s] = xs[s];
      }
      if (any) {
        unsigned long long* vp = A.vis + v * nseg;
#pragma unroll
        for (int s = 0; s < kSegMax; s++)
          if (s < nseg && xs[s]) vp[s] |= xs[s];
        if (!first) {
          for (uint32_t bits = step; bits; bits &= bits - 1u) {
            unsigned long long* pp = A.planes + (size_t)(__ffs(bits) - 1) * pn + v * nseg;
#pragma unroll
            for (int s = 0; s < kSegMax; s++)
              if (s < nseg && xs[s]) pp[s] |= xs[s];
          }
        }
      }
    }
    int32_t start = 0, deg = 0;
    if (any) {
      start = A.rowptr[v];
      deg = A.rowptr[v + 1] - start;
      if (deg == 0)  // nothing to expand: the row never enters a queue
        for (int s = 0; s < nseg; s++) mp[s] = 0ull;
      else {
        acc.fe += 1;        // frontier rows
        acc.sa += pairs;    // frontier (row, source) pairs
        acc.es += (unsigned long long)deg;  // out-edges of the frontier rows
        acc.se += (unsigned long long)deg * pairs;  // out-edges of the (row, source) pairs
      }
    }
    {
      // frontier bitmap of the step: each wavefront owns 64 consecutive
      // vertices (ranges start at multiples of the workgroup size), so it
      // writes its two words whole and nothing needs clearing
      const unsigned long long fb = __ballot(any && deg > 0);
      const int64_t wbase = (v0 + (threadIdx.x & ~(kWave - 1))) >> 5;
      if (lane_id() == 0 && (wbase << 5) < n) A.fbm[step & 1][wbase] = (uint32_t)fb;
      if (lane_id() == 1 && ((wbase + 1) << 5) < n) A.fbm[step & 1][wbase + 1] = (uint32_t)(fb >> 32);
    }
    compact_push(any && deg > 0 && deg <= A.t_group, (int32_t)v, 0, sh);
    compact_push(any && deg > A.t_group && deg <= A.t_wave, (int32_t)v, 1, sh);
    // workgroup-chunk records: reserve within the workgroup, then one global
    // reservation per batch
    const bool hub = any && deg > A.t_wave;
    const uint32_t nch = hub ? (uint32_t)((deg + A.t_chunk - 1) / A.t_chunk) : 0u;
    uint32_t loc = 0u;
    if (hub) loc = atomicAdd(&sh.nch, nch);
    __syncthreads();
    if (threadIdx.x == 0) {
      sh.chbase = sh.nch ? atomicAdd(&C->cnt[rc][2].v, sh.nch) : 0u;
      sh.nch = 0u;
    }
    __syncthreads();
    // every wavefront reads the same counts: no push happens until the
    // barrier below
    const bool flush =
        sh.cnt[0] > (uint32_t)(kCompactLds - bd) || sh.cnt[1] > (uint32_t)(kCompactLds - bd);
    const uint32_t chbase = sh.chbase;
    for (uint32_t c = 0; c < nch; c++) {
      const int32_t off = (int32_t)c * A.t_chunk;
      const uint32_t p = chbase + loc + c;
      if (p < A.cap_wg)
        A.qwg[q][p] = make_int4((int32_t)v, start + off, min(A.t_chunk, deg - off), c == 0);
      else
        atomicOr(&C->overflow, 1u);
    }
    __syncthreads();
    if (flush) compact_flush(A, q, rc, sh);
  }
  compact_flush(A, q, rc, sh);
}

// ---------------------------------------------------------------------------
// relaxation
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t elem4(const uint4& x, int i) {
  return i == 0 ? x.x : i == 1 ? x.y : i == 2 ? x.z : x.w;
}

// OR over the 16 lanes of a row of the wavefront (lanes 16r..16r+15); every
// lane of the row gets the result.  DPP row rotations stay in the VALU (a
// cross-lane shuffle would go through the LDS crossbar).
__device__ __forceinline__ uint32_t row16_or(uint32_t x) {
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x121, 0xF, 0xF, false);  // row_ror:1
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x122, 0xF, 0xF, false);  // row_ror:2
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x124, 0xF, 0xF, false);  // row_ror:4
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false);  // row_ror:8
  return x;
}

// Value of lane n (0..15) of this lane's 16-lane row (DPP row_share, VALU
// only).  n must fold to a constant.
__device__ __forceinline__ int row_share(int x, int n) {
  switch (n) {
    case 0: return __builtin_amdgcn_update_dpp(0, x, 0x150, 0xF, 0xF, false);
    case 1: return __builtin_amdgcn_update_dpp(0, x, 0x151, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_update_dpp(0, x, 0x152, 0xF, 0xF, false);
    case 3: return __builtin_amdgcn_update_dpp(0, x, 0x153, 0xF, 0xF, false);
    case 4: return __builtin_amdgcn_update_dpp(0, x, 0x154, 0xF, 0xF, false);
    case 5: return __builtin_amdgcn_update_dpp(0, x, 0x155, 0xF, 0xF, false);
    case 6: return __builtin_amdgcn_update_dpp(0, x, 0x156, 0xF, 0xF, false);
    case 7: return __builtin_amdgcn_update_dpp(0, x, 0x157, 0xF, 0xF, false);
    case 8: return __builtin_amdgcn_update_dpp(0, x, 0x158, 0xF, 0xF, false);
    case 9: return __builtin_amdgcn_update_dpp(0, x, 0x159, 0xF, 0xF, false);
    case 10: return __builtin_amdgcn_update_dpp(0, x, 0x15A, 0xF, 0xF, false);
    case 11: return __builtin_amdgcn_update_dpp(0, x, 0x15B, 0xF, 0xF, false);
    case 12: return __builtin_amdgcn_update_dpp(0, x, 0x15C, 0xF, 0xF, false);
    case 13: return __builtin_amdgcn_update_dpp(0, x, 0x15D, 0xF, 0xF, false);
    case 14: return __builtin_amdgcn_update_dpp(0, x, 0x15E, 0xF, 0xF, false);
    default: return __builtin_amdgcn_update_dpp(0, x, 0x15F, 0xF, 0xF, false);
  }
}

// Relax edges [start, start+len) of one frontier row for the 4 sources of
// segment sg that this lane covers (`bits`; `du` = the row's distances of
// those sources).  `ngroups` 16-lane groups share the row; this lane's group
// is `gidx`.  Loop counts are uniform within a group.
//
// A group takes 16 edges at a time: lane j loads edge j's id and weight (one
// coalesced load each), and the 16 edges are walked kTileU at a time with the
// id and weight broadcast along the row (DPP); the next 16 are requested
// before the current ones are relaxed.  Within a batch all candidates are
// compared before any atomic is issued and the atomics go out back to back
// (gfx9's vector-memory counter also counts non-returning atomics, in order,
// so an atomic between two compares would make the second wait for it).
template <bool F32>
__device__ __forceinline__ void tile_seg_relax(const TileArgs& A, int32_t start, int32_t len,
                                               int sg, uint32_t bits, const uint4& du, int gidx,
                                               int ngroups, unsigned long long* mk_next,
                                               unsigned long long* sh_colact) {
  constexpr int U = kTileU;
  const int j16 = threadIdx.x & 15;
  const int col = sg * 64 + 4 * j16;
  const int K = A.K, nseg = A.nseg;
  const int32_t stride = ngroups * 16;
  int32_t eb = gidx * 16;
  if (eb >= len) return;
  int32_t cvn = -1;
  uint32_t cwn = 0u;
  if (eb + j16 < len) {
    cvn = A.colidx[start + eb + j16];
    cwn = A.w[start + eb + j16];
  }
  for (; eb < len; eb += stride) {
    const int32_t cv = cvn;
    const uint32_t cw = cwn;
    const int cnt = min(16, len - eb);
    if (eb + stride < len) {
      cvn = -1;
      cwn = 0u;
      if (eb + stride + j16 < len) {
        cvn = A.colidx[start + eb + stride + j16];
        cwn = A.w[start + eb + stride + j16];
      }
    }
#pragma unroll
    for (int i0 = 0; i0 < 16; i0 += U) {
      if (i0 >= cnt) break;
      int32_t v[U];
      uint32_t w[U];
#pragma unroll
      for (int i = 0; i < U; i++) {
        v[i] = i0 + i < cnt ? row_share(cv, i0 + i) : -1;
        w[i] = (uint32_t)row_share((int)cw, i0 + i);
      }
      uint4 dv[U];
#pragma unroll
      for (int i = 0; i < U; i++) {
        dv[i] = make_uint4(0u, 0u, 0u, 0u);
        if (v[i] >= 0 && bits) dv[i] = *reinterpret_cast<const uint4*>(A.D + (size_t)v[i] * K + col);
      }
      uint32_t imp[U];
#pragma unroll
      for (int i = 0; i < U; i++) {
        imp[i] = 0u;
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const uint32_t c = relax_add<F32>(elem4(du, t), w[i]);
          if (v[i] >= 0 && ((bits >> t) & 1u) && c < elem4(dv[i], t)) imp[i] |= 1u << t;
        }
      }
#pragma unroll
      for (int i = 0; i < U; i++) {
        if (imp[i]) {
          uint32_t* dp = A.D + (size_t)v[i] * K + col;
#pragma unroll
          for (int t = 0; t < 4; t++)
            if ((imp[i] >> t) & 1u) atomicMin(dp + t, relax_add<F32>(elem4(du, t), w[i]));
        }
      }
#pragma unroll
      for (int i = 0; i < U; i++) {
        // the group's 64 improvement bits of segment sg: lane j16 holds bits 4*j16..4*j16+3
        const uint32_t lo = row16_or(j16 < 8 ? imp[i] << (4 * j16) : 0u);
        const uint32_t hi = row16_or(j16 >= 8 ? imp[i] << (4 * (j16 - 8)) : 0u);
        const unsigned long long x = ((unsigned long long)hi << 32) | lo;
        if (j16 == 0 && x != 0ull) {
          atomicOr(mk_next + (size_t)v[i] * nseg + sg, x);
          atomicOr(&sh_colact[sg], x);
        }
      }
    }
  }
}

// Active-source mask word `s` of row u for this step; with skipping, minus the
// sources whose alpha[u] was already lowered again in this step (they are in
// the next step's mask and are expanded then, with the lower value).  The next
// mask was cleared before this step began (an earlier launch, or before a grid
// barrier), so a plain load returns only bits set in this step, or misses some
// of them -- which only means expanding a pair that could have waited.
__device__ __forceinline__ unsigned long long tile_row_mask(const TileArgs& A, int q, int qn,
                                                            int32_t u, int s) {
  const size_t i = (size_t)u * A.nseg + s;
  unsigned long long x = A.mk[q][i];
  if (A.skip && x) x &= ~A.mk[qn][i];
  return x;
}

// Relax edges [start, start+len) of row u for its few active sources, one
// edge per lane: lane t of a team of nt lanes takes edges t, t+nt, ...  For
// each active source (column j) the team streams the row once, each lane
// loading 4 bytes of its target's distances.  Used for rows with at most
// tile_sparse active sources, where the segment mapping (16 lanes per 64
// sources) would leave most lanes idle: early steps reach hub rows of
// thousands of edges for one or two sources.
template <bool F32>
__device__ __forceinline__ void tile_sparse_relax(const TileArgs& A, int32_t u, int32_t start,
                                                  int32_t len, int q, int qn, int t, int nt,
                                                  unsigned long long* mk_next,
                                                  unsigned long long* sh_colact) {
  const int K = A.K, nseg = A.nseg;
  for (int sg = 0; sg < nseg; sg++) {
    unsigned long long x = tile_row_mask(A, q, qn, u, sg);
    while (x) {
      const int b = __ffsll((long long)x) - 1;
      x &= x - 1ull;
      const int j = sg * 64 + b;
      const unsigned long long bit = 1ull << b;
      const uint32_t duj = A.D[(size_t)u * K + j];
      bool any = false;
      for (int32_t e0 = t; e0 < len; e0 += 2 * nt) {
        const int32_t e1 = e0 + nt;
        const int32_t v0 = A.colidx[start + e0];
        const uint32_t w0 = A.w[start + e0];
        int32_t v1 = -1;
        uint32_t w1 = 0u;
        if (e1 < len) {
          v1 = A.colidx[start + e1];
          w1 = A.w[start + e1];
        }
        const uint32_t d0 = A.D[(size_t)v0 * K + j];
        const uint32_t d1 = v1 >= 0 ? A.D[(size_t)v1 * K + j] : 0u;
        const uint32_t c0 = relax_add<F32>(duj, w0), c1 = relax_add<F32>(duj, w1);
        const bool i0 = c0 < d0, i1 = v1 >= 0 && c1 < d1;
        if (i0) {
          atomicMin(A.D + (size_t)v0 * K + j, c0);
          atomicOr(mk_next + (size_t)v0 * nseg + sg, bit);
        }
        if (i1) {
          atomicMin(A.D + (size_t)v1 * K + j, c1);
          atomicOr(mk_next + (size_t)v1 * nseg + sg, bit);
        }
        any |= i0 | i1;
      }
      if (any) atomicOr(&sh_colact[sg], bit);
    }
  }
}

// Lane l sets up row b0 + l of queue `qq` (count n): its vertex, row bounds
// and active segments (bit s: mask word s non-zero), and counts the row.
// Rows past the count get act = 0.
__device__ __forceinline__ void tile_row_setup(const TileArgs& A, const int32_t* qq, uint32_t n,
                                               uint32_t b0, int q, int qn, int32_t& u,
                                               int32_t& start, int32_t& deg, uint32_t& act,
                                               uint32_t& nsrc, unsigned long long& mask0) {
  const uint32_t i = b0 + (uint32_t)lane_id();
  u = 0;
  start = 0;
  deg = 0;
  act = 0u;
  nsrc = 0u;
  mask0 = 0ull;
  if (i >= n) return;
  u = ld_queue(qq + i);
  start = A.rowptr[u];
  deg = A.rowptr[u + 1] - start;
  unsigned long long ns = 0ull;
  for (int s = 0; s < A.nseg; s++) {
    const unsigned long long x = tile_row_mask(A, q, qn, u, s);
    if (s == 0) mask0 = x;
    if (x) {
      act |= 1u << s;
      ns += (unsigned long long)__popcll(x);
    }
  }
  nsrc = (uint32_t)ns;
}

// Staging of one wavefront's rows for tile_lane_rows.
struct TileLaneStage {
  int32_t incl[kWave];
  int32_t base[kWave];
  int32_t u[kWave];
  unsigned long long mask[kWave];
};

// Short rows of a one-segment tile (K <= 64) with few active sources, one
// edge per lane: lane i holds row i (its vertex, row bounds and active-source
// mask); the rows' edges are concatenated through an LDS prefix sum of their
// degrees and lane l takes edges l, l + 64, ...  For its edge (u, v) a lane
// relaxes each active source of u, four at a time with their loads in flight
// together.  A 16-lane group per row would keep only four rows in flight per
// wavefront, each waiting on its own chain of loads; here 64 edges are.
// Reached by the whole wavefront; rows with deg = 0 take no edge.
template <bool F32>
__device__ __forceinline__ void tile_lane_rows(const TileArgs& A, int32_t u, int32_t start,
                                               int32_t deg, unsigned long long mask,
                                               unsigned long long* mk_next,
                                               unsigned long long* sh_colact, TileLaneStage& st) {
  const int lane = lane_id();
  const int incl = wave_incl_scan(deg);
  const int total = __shfl(incl, kWave - 1, kWave);
  st.incl[lane] = incl;
  st.base[lane] = start - (incl - deg);
  st.u[lane] = u;
  st.mask[lane] = mask;
  wave_lds_sync();
  const int K = A.K;
  unsigned long long colact = 0ull;
  for (int k = lane; k < total; k += kWave) {
    int owner = 0;  // first lane whose inclusive prefix exceeds k
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
      if (st.incl[owner + s - 1] <= k) owner += s;
    const int32_t e = st.base[owner] + k;
    const uint32_t* du = A.D + (size_t)st.u[owner] * K;
    unsigned long long x = st.mask[owner];
    const int32_t v = A.colidx[e];
    const uint32_t w = A.w[e];
    uint32_t* dv = A.D + (size_t)v * K;
    unsigned long long got = 0ull;
    while (x) {
      int c[4];
      bool ok[4];
#pragma unroll
      for (int i = 0; i < 4; i++) {
        ok[i] = x != 0ull;
        c[i] = ok[i] ? __ffsll((long long)x) - 1 : 0;
        x &= x - 1ull;
      }
      uint32_t a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; i++) {
        a[i] = du[c[i]];
        b[i] = dv[c[i]];
      }
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const uint32_t cand = relax_add<F32>(a[i], w);
        if (ok[i] && cand < b[i]) {
          atomicMin(dv + c[i], cand);
          got |= 1ull << c[i];
        }
      }
    }
    if (got) {
      atomicOr(mk_next + v, got);  // one segment: row v's only mask word
      colact |= got;
    }
  }
  if (colact) atomicOr(&sh_colact[0], colact);
  wave_lds_sync();
}

// Clear the mask words of the previous step's frontier rows (slot read one
// step ago; it is written again from the next step on).
__device__ __forceinline__ void tile_clear_prev(const TileArgs& A, uint32_t step, uint32_t gb,
                                                uint32_t nb) {
  TileCtl* C = A.ctl;
  const int qp = (step + 2) % 3, rp = (step + 3) % kRot;
  const int nseg = A.nseg;
  {
    const uint32_t pg = min(ld_agent(&C->cnt[rp][0].v), A.cap_v);
    const uint32_t pw = min(ld_agent(&C->cnt[rp][1].v), A.cap_v);
    const uint32_t pc = min(ld_agent(&C->cnt[rp][2].v), A.cap_wg);
    const uint32_t tot = pg + pw + pc;
    for (uint32_t i = gb * blockDim.x + threadIdx.x; i < tot; i += nb * blockDim.x) {
      int32_t u;
      bool first = true;
      if (i < pg) {
        u = ld_queue(&A.qgrp[qp][i]);
      } else if (i < pg + pw) {
        u = ld_queue(&A.qwave[qp][i - pg]);
      } else {
        const int4 r = ld_queue4(&A.qwg[qp][i - pg - pw]);
        u = r.x;
        first = r.w != 0;
      }
      if (first) {
        unsigned long long* mp = A.mk[qp] + (size_t)u * nseg;
        for (int s = 0; s < nseg; s++) mp[s] = 0ull;
      }
    }
  }

}

template <bool F32>
__device__ void tile_relax(const TileArgs& A, uint32_t step, uint32_t gb, uint32_t nb,
                           unsigned long long* sh_colact) {
  const int q = step % 3, qn = (step + 1) % 3, qp = (step + 2) % 3;
  const int rc = step % kRot, rn = (step + 1) % kRot, rp = (step + 3) % kRot;
  TileCtl* C = A.ctl;
  const int lane = lane_id(), wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  const int j16 = lane & 15, gbase = lane & 48;
  const uint32_t gw = gb * W + wave, nwv = nb * W;
  const int nseg = A.nseg;
  unsigned long long* mkn = A.mk[qn];
  if (threadIdx.x < kSegMax) sh_colact[threadIdx.x] = 0ull;
  __syncthreads();

  tile_clear_prev(A, step, gb, nb);

  // (b) workgroup tier: the 16-lane groups of the workgroup share a chunk
  const uint32_t nc = min(ld_agent(&C->cnt[rc][2].v), A.cap_wg);
  for (uint32_t i = gb; i < nc; i += nb) {
    const int4 r = ld_queue4(&A.qwg[q][i]);
    const unsigned long long x = lane < nseg ? tile_row_mask(A, q, qn, r.x, lane) : 0ull;
    const uint32_t act = (uint32_t)__ballot(x != 0ull);
    if (act == 0u) continue;
    // The path must be the same for every wavefront of the workgroup (each
    // covers only its share of the chunk), so it is chosen from this step's
    // mask, which no lane changes during the step.
    int nsc = lane < nseg ? __popcll(A.mk[q][(size_t)r.x * nseg + lane]) : 0;
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) nsc += __shfl_xor(nsc, off, kWave);
    nsc = __builtin_amdgcn_readlane(nsc, 0);  // lanes 0..7 hold the sum; make it uniform
    if (nsc <= A.sparse) {
      tile_sparse_relax<F32>(A, r.x, r.y, r.z, q, qn, threadIdx.x, blockDim.x, mkn, sh_colact);
      continue;
    }
    for (uint32_t a = act; a; a &= a - 1u) {
      const int sg = __ffs(a) - 1;
      const unsigned long long xs = lane64(x, sg);
      const uint32_t bits = (uint32_t)(xs >> (4 * j16)) & 0xFu;
      uint4 du = make_uint4(0u, 0u, 0u, 0u);
      if (bits) du = *reinterpret_cast<const uint4*>(A.D + (size_t)r.x * A.K + sg * 64 + 4 * j16);
      tile_seg_relax<F32>(A, r.y, r.z, sg, bits, du, threadIdx.x >> 4, blockDim.x >> 4, mkn,
                          sh_colact);
    }
  }

  // (c) wave tier: one wavefront per row, its 4 groups share the row;
  // (d) group tier: one 16-lane group per row.
  // Rows are set up 64 at a time, one per lane (queue entry, row bounds,
  // active segments, counters), so the setup round trips of a batch overlap;
  // the rows are then walked from registers.
  // Each wavefront takes an even, contiguous share of a queue.
  const uint32_t nw = min(ld_agent(&C->cnt[rc][1].v), A.cap_v);
  const uint32_t pw = (nw + nwv - 1) / nwv, hw = min(nw, gw * pw + pw);
  for (uint32_t b0 = gw * pw; b0 < hw; b0 += kWave) {
    int32_t u, start, deg;
    uint32_t act, nsrc;
    unsigned long long mask0;
    tile_row_setup(A, A.qwave[q], hw, b0, q, qn, u, start, deg, act, nsrc, mask0);
    const int rows = (int)min((uint32_t)kWave, hw - b0);
    for (int r = 0; r < rows; r++) {
      const uint32_t ar = (uint32_t)__builtin_amdgcn_readlane((int)act, r);
      if (ar == 0u) continue;
      const int32_t ur = __builtin_amdgcn_readlane(u, r);
      const int32_t sr = __builtin_amdgcn_readlane(start, r);
      const int32_t dr = __builtin_amdgcn_readlane(deg, r);
      if ((int)__builtin_amdgcn_readlane((int)nsrc, r) <= A.sparse) {
        tile_sparse_relax<F32>(A, ur, sr, dr, q, qn, lane, kWave, mkn, sh_colact);
        continue;
      }
      for (uint32_t a = ar; a; a &= a - 1u) {
        const int sg = __ffs(a) - 1;
        const uint32_t bits = (uint32_t)(tile_row_mask(A, q, qn, ur, sg) >> (4 * j16)) & 0xFu;
        uint4 du = make_uint4(0u, 0u, 0u, 0u);
        if (bits) du = *reinterpret_cast<const uint4*>(A.D + (size_t)ur * A.K + sg * 64 + 4 * j16);
        tile_seg_relax<F32>(A, sr, dr, sg, bits, du, lane >> 4, 4, mkn, sh_colact);
      }
    }
  }

  const uint32_t ng = min(ld_agent(&C->cnt[rc][0].v), A.cap_v);
  const uint32_t pg = (ng + nwv - 1) / nwv, hg = min(ng, gw * pg + pg);
  const int grp = lane >> 4;
  // one-segment tiles: rows with few active sources go one edge per lane
  __shared__ TileLaneStage lst[kMaxWavesPerBlock];
  const bool lane_rows = nseg == 1;
  for (uint32_t b0 = gw * pg; b0 < hg; b0 += kWave) {
    int32_t u, start, deg;
    uint32_t act, nsrc;
    unsigned long long mask0;
    tile_row_setup(A, A.qgrp[q], hg, b0, q, qn, u, start, deg, act, nsrc, mask0);
    const int rows = (int)min((uint32_t)kWave, hg - b0);
    bool lr = false;
    if (lane_rows) {
      lr = act != 0u && (int)nsrc <= A.sparse;
      if (__ballot(lr) != 0ull)
        tile_lane_rows<F32>(A, u, start, lr ? deg : 0, lr ? mask0 : 0ull, mkn, sh_colact,
                            lst[wave]);
    }
    const uint32_t act_g = lr ? 0u : act;  // the rows left to the 16-lane groups
    // group g walks rows b0 + 4 r + g, held by lane 4 r + g
    for (int r = 0; 4 * r < rows; r++) {
      const int src = 4 * r + grp;
      const uint32_t ar = (uint32_t)__shfl((int)act_g, src, kWave);
      const int32_t ur = __shfl(u, src, kWave);
      const int32_t sr = __shfl(start, src, kWave);
      const int32_t dr = __shfl(deg, src, kWave);
      for (uint32_t a = ar; a; a &= a - 1u) {
        const int sg = __ffs(a) - 1;
        const uint32_t bits = (uint32_t)(tile_row_mask(A, q, qn, ur, sg) >> (4 * j16)) & 0xFu;
        uint4 du = make_uint4(0u, 0u, 0u, 0u);
        if (bits) du = *reinterpret_cast<const uint4*>(A.D + (size_t)ur * A.K + sg * 64 + 4 * j16);
        tile_seg_relax<F32>(A, sr, dr, sg, bits, du, 0, 1, mkn, sh_colact);
      }
    }
  }

  // (e) publish the workgroup's column activity
  __syncthreads();
  if ((int)threadIdx.x < nseg && sh_colact[threadIdx.x])
    or_new_bits(&C->colact[rn][threadIdx.x], sh_colact[threadIdx.x]);
}

__device__ __forceinline__ bool any_active(const TileCtl* C, int rn, int nseg) {
  unsigned long long a = 0ull;
  for (int s = 0; s < nseg; s++) a |= ld_agent64(&C->colact[rn][s]);
  return a != 0ull;
}

// All steps (up to max_steps, and at most n when cap_n) in one launch with a
// grid barrier after each compaction and each relaxation.
template <bool F32>
__global__ void __launch_bounds__(1024) tile_persistent_kernel(TileArgs A, int32_t max_steps,
                                                               int32_t cap_n) {
  __shared__ unsigned long long sh_colact[kSegMax];
  __shared__ CompactShared csh;
  TileCtl* C = A.ctl;
  if (ld_agent(&C->done)) return;
  Acc acc;  // every counter is taken by the compaction
  uint32_t epoch = 0;
  const uint32_t bar_base = ld_agent(&C->bar_base);
  uint32_t step = ld_agent(&C->step);
  const uint32_t stop = step + (uint32_t)max_steps;
  int32_t status = 1;
  bool finished = false;
  for (;;) {
    if (blockIdx.x == 0) tile_prologue(C, step, A.K);
    tile_compact<false>(A, step, blockIdx.x, gridDim.x, acc, csh);
    if (!grid_sync(&C->bar.v, &C->abort, gridDim.x, bar_base, epoch, A.bar_ticks)) {
      status = -2;
      finished = true;
      break;
    }
    tile_relax<F32>(A, step, blockIdx.x, gridDim.x, sh_colact);
    if (!grid_sync(&C->bar.v, &C->abort, gridDim.x, bar_base, epoch, A.bar_ticks)) {
      status = -2;
      finished = true;
      break;
    }
    const bool act = any_active(C, (step + 1) % kRot, A.nseg);
    step++;
    if (!act) { status = 1; finished = true; break; }
    if (cap_n && step >= (uint32_t)A.n) { status = 0; finished = true; break; }
    if (step == stop) break;
  }
  // (the frontier's out-edges per step decide pull steps of step launches only)
  CtrStripe& S = C->ctr[blockIdx.x % kCtrStripes];
  flush_acc(acc, &S.fe, &S.es, &S.im, &S.sa, &S.se);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st_agent(&C->step, step);
    st_agent(&C->bar_base, bar_base + epoch * gridDim.x);
    if (finished) {
      st_agent_i(&C->converged, status);
      st_agent(&C->done, 1u);
    }
  }
}

// Step launches: the compaction of a step, then its relaxation, whose last
// workgroup advances the step and detects the end.
template <bool UW>
__global__ void __launch_bounds__(1024) tile_compact_kernel(TileArgs A) {
  __shared__ CompactShared csh;
  TileCtl* C = A.ctl;
  if (ld_agent(&C->done)) return;
  const uint32_t step = ld_agent(&C->step);
  if (blockIdx.x == 0) tile_prologue(C, step, A.K);
  Acc acc;
  tile_compact<UW>(A, step, blockIdx.x, gridDim.x, acc, csh);
  // frontier rows and pairs, improvements, and the frontier's out-edges
  CtrStripe& S = C->ctr[blockIdx.x % kCtrStripes];
  flush_acc(acc, &S.fe, &S.es, &S.im, &S.sa, &S.se, &S.fedges[step % kRot], &S.fpairs[step % kRot]);
}

// A step is a pull step when the reverse graph is there, the frontier has at
// least pull_min out-edges and those carry at least pull_src active sources
// each on average (a pull step reads whole segment rows; with few active
// sources the push step reads far less).  Both counts come from the
// compaction, before both relaxation kernels of the step run, so both take
// the same decision.
__device__ __forceinline__ bool tile_is_pull_step(const TileArgs& A, uint32_t step) {
  if (A.T.hdr == nullptr || A.pull_min < 0) return false;
  const size_t off = offsetof(CtrStripe, fedges) + (step % kRot) * sizeof(unsigned long long);
  const unsigned long long fe = ctr_sum(A.ctl->ctr, off);
  if (fe < (unsigned long long)A.pull_min) return false;
  if (A.pull_src <= 0) return true;
  const size_t offp = offsetof(CtrStripe, fpairs) + (step % kRot) * sizeof(unsigned long long);
  return ctr_sum(A.ctl->ctr, offp) >= (unsigned long long)A.pull_src * fe;
}

// End of a step launch: the last workgroup advances the step and detects the end.
__device__ __forceinline__ void tile_end_step(const TileArgs& A, uint32_t step, int32_t cap_n) {
  TileCtl* C = A.ctl;
  if (last_block_arrive(&C->arrive) && threadIdx.x == 0) {
    const bool act = any_active(C, (step + 1) % kRot, A.nseg);
    const uint32_t ns = step + 1;
    st_agent(&C->step, ns);
    if (!act) {
      st_agent_i(&C->converged, 1);
      st_agent(&C->done, 1u);
    } else if (cap_n && ns >= (uint32_t)A.n) {
      st_agent_i(&C->converged, 0);
      st_agent(&C->done, 1u);
    }
  }
}

template <bool F32>
__global__ void __launch_bounds__(1024) tile_step_kernel(TileArgs A, int32_t cap_n) {
  __shared__ unsigned long long sh_colact[kSegMax];
  TileCtl* C = A.ctl;
  if (ld_agent(&C->done)) return;
  const uint32_t step = ld_agent(&C->step);
  if (tile_is_pull_step(A, step)) return;  // the pull kernel runs this step
  tile_relax<F32>(A, step, blockIdx.x, gridDim.x, sh_colact);
  tile_end_step(A, step, cap_n);
}

// ---------------------------------------------------------------------------
// pull steps
//
// When the frontier's rows carry a large share of the edges, the step walks
// the in-edges of every target instead (the reverse graph).  A wavefront takes
// one in-edge chunk of a target v and a quad of 64-source segments; each
// 16-lane group covers one segment (lane = 4 sources) and, when the quad has
// fewer than four segments, the groups that cover the same segment take
// different in-edges and combine at the end.  The best candidate of each
// source is kept in registers over all in-edges (u, v) whose u is in the
// step's frontier; v's improved distances and next-step mask word are then
// written with plain stores: no other lane writes them in this step.  Only
// targets whose in-edges span several chunks combine their chunks with atomics.
//
// Every source of a frontier row u is relaxed, not only those active at u:
// for a source c not active at u, u's distance for c has not changed since the
// step that last relaxed (u, v) for c (or is still INF), so that step left
// D[v][c] <= D[u][c] (+) w and the candidate cannot improve v.  The improved
// pairs -- hence the next frontier and the distances -- are exactly those of
// the push step.  Reading u's whole row costs no more memory traffic than
// reading its active sources (at 16 sources per 64-byte sector, a sector with
// no active source is rare in the steps dense enough to pull) and saves the
// gather of u's mask words.
// ---------------------------------------------------------------------------
constexpr int kPullThreads = 256;
constexpr int kPullU = 8;  // in-edges gathered at a time per 16-lane group

// E: in-edges taken at a time by the groups of one segment (4 / segments in
// the quad; 1 for quads of 3 or 4 segments)
template <bool F32, int E>
__device__ __forceinline__ void tile_pull_chunk(const TileArgs& A, const int4 ch, int p, int qn,
                                                const uint32_t* fbm,
                                                unsigned long long* sh_colact) {
  const int lane = lane_id(), j16 = lane & 15, g = lane >> 4;
  const int32_t v = ch.x, start = ch.y, len = ch.z;
  const bool split = ch.w != 0;
  const int nseg = A.nseg, K = A.K;
  const int nsq = min(4, nseg - 4 * p);  // segments in this quad
  const int e = g / nsq;                 // in-edge slot of this group
  const bool gok = e < E;                // false only for the idle group of a 3-segment quad
  const bool own = gok && e == 0;        // the group that writes v's segment
  const int s = 4 * p + g % nsq;
  const int col = s * 64 + 4 * j16;
  const uint32_t inf = inf_bits<F32>();
  uint32_t* dp = A.D + (size_t)v * K + col;
  // v's distances: read early when this chunk is v's only writer, else after
  // the loop (other chunks of v may lower them meanwhile)
  uint4 dv = make_uint4(0u, 0u, 0u, 0u);
  if (own && !split) dv = *reinterpret_cast<const uint4*>(dp);
  uint32_t best[4] = {inf, inf, inf, inf};
  for (int32_t b = 0; b < len; b += kWave) {
    const int cnt = min(kWave, len - b);
    // lane l: in-edge b + l -- its source and weight, kept if the source is in the frontier
    int32_t ul = 0;
    uint32_t wl = 0u;
    if (lane < cnt) {
      ul = A.T.colidx[start + b + lane];
      wl = A.T.w[start + b + lane];
    }
    const bool fr = lane < cnt && ((fbm[ul >> 5] >> (ul & 31)) & 1u);
    unsigned long long todo = __ballot(fr);
    while (todo) {
      int32_t ui[kPullU];
      uint32_t wi[kPullU];
      bool ok[kPullU];
      uint4 du[kPullU];
#pragma unroll
      for (int k = 0; k < kPullU; k++) {
        // the next E in-edges of the list go to slots 0 .. E-1
        ui[k] = 0;
        wi[k] = 0u;
        ok[k] = false;
#pragma unroll
        for (int t = 0; t < E; t++) {
          if (todo) {
            const int i = __ffsll((long long)todo) - 1;
            todo &= todo - 1ull;
            const int32_t ut = __builtin_amdgcn_readlane(ul, i);
            const uint32_t wt = (uint32_t)__builtin_amdgcn_readlane((int)wl, i);
            if (t == e) {
              ui[k] = ut;
              wi[k] = wt;
              ok[k] = gok;
            }
          }
        }
        du[k] = make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int k = 0; k < kPullU; k++)
        if (ok[k]) du[k] = *reinterpret_cast<const uint4*>(A.D + (size_t)ui[k] * K + col);
#pragma unroll
      for (int k = 0; k < kPullU; k++) {
        if (ok[k]) {
#pragma unroll
          for (int t = 0; t < 4; t++) best[t] = min(best[t], relax_add<F32>(elem4(du[k], t), wi[k]));
        }
      }
    }
  }
  // groups of one segment combine their candidates
#pragma unroll
  for (int off = 16 * (4 / E); off < kWave; off <<= 1) {
#pragma unroll
    for (int t = 0; t < 4; t++) best[t] = min(best[t], (uint32_t)__shfl_xor((int)best[t], off, kWave));
  }
  // write back the improved distances of v (this lane's 4 sources)
  if (own && split) dv = *reinterpret_cast<const uint4*>(dp);
  uint32_t imp = 0u;
  if (own && (best[0] != inf || best[1] != inf || best[2] != inf || best[3] != inf)) {
#pragma unroll
    for (int t = 0; t < 4; t++)
      if (best[t] < elem4(dv, t)) imp |= 1u << t;
    if (imp) {
      if (split) {
#pragma unroll
        for (int t = 0; t < 4; t++)
          if ((imp >> t) & 1u) atomicMin(dp + t, best[t]);
      } else {
        *reinterpret_cast<uint4*>(dp) = make_uint4(min(dv.x, best[0]), min(dv.y, best[1]),
                                                   min(dv.z, best[2]), min(dv.w, best[3]));
      }
    }
  }
  const uint32_t lo = row16_or(j16 < 8 ? imp << (4 * j16) : 0u);
  const uint32_t hi = row16_or(j16 >= 8 ? imp << (4 * (j16 - 8)) : 0u);
  const unsigned long long x = ((unsigned long long)hi << 32) | lo;
  if (j16 == 0 && own && x != 0ull) {
    unsigned long long* mp = A.mk[qn] + (size_t)v * nseg + s;
    if (split) atomicOr(mp, x);
    else *mp = x;
    atomicOr(&sh_colact[s], x);
  }
}

template <bool F32>
__global__ void __launch_bounds__(kPullThreads) tile_pull_kernel(TileArgs A, int32_t cap_n) {
  __shared__ unsigned long long sh_colact[kSegMax];
  TileCtl* C = A.ctl;
  if (ld_agent(&C->done)) return;
  const uint32_t step = ld_agent(&C->step);
  // after a push step the push kernel has already advanced the step: the new
  // one has no compaction yet
  if (step != ld_agent(&C->cstep)) return;
  if (!tile_is_pull_step(A, step)) return;  // the push kernel runs this step
  const int qn = (step + 1) % 3, rn = (step + 1) % kRot;
  tile_clear_prev(A, step, blockIdx.x, gridDim.x);
  if (threadIdx.x < kSegMax) sh_colact[threadIdx.x] = 0ull;
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const uint32_t gw = blockIdx.x * (kPullThreads / kWave) + wave;
  const uint32_t nwv = gridDim.x * (kPullThreads / kWave);
  const uint32_t nq = (uint32_t)((A.nseg + 3) / 4);
  const uint32_t nch = (uint32_t)min((long long)A.T.hdr->nchunks, (long long)A.T.cap_chunks);
  const uint32_t* fbm = A.fbm[step & 1];
  for (uint32_t task = gw; task < nch * nq; task += nwv) {
    const uint32_t c = task / nq;
    const int p = (int)(task - c * nq);
    const int nsq = min(4, A.nseg - 4 * p);
    const int4 ch = A.T.chunks[c];
    if (nsq >= 3) tile_pull_chunk<F32, 1>(A, ch, p, qn, fbm, sh_colact);
    else if (nsq == 2) tile_pull_chunk<F32, 2>(A, ch, p, qn, fbm, sh_colact);
    else tile_pull_chunk<F32, 4>(A, ch, p, qn, fbm, sh_colact);
  }
  __syncthreads();
  if ((int)threadIdx.x < A.nseg && sh_colact[threadIdx.x])
    or_new_bits(&C->colact[rn][threadIdx.x], sh_colact[threadIdx.x]);
  tile_end_step(A, step, cap_n);
}

// ---------------------------------------------------------------------------
// hop-count tiles (unit weights)
//
// With every weight 1 a (vertex, source) pair's distance is set once, to the
// number of the step that reaches it: the unweighted case, in which each
// shortest path is found exactly once (mu = 1) and a step is the boolean
// vector-matrix product of the Principle section.  A step then needs neither
// distances nor atomicMin.  Push: a frontier row's mask, restricted to the
// pairs not reached yet (`vis`), is ORed into each out-neighbour's next mask.
// Pull: a target ORs the masks of its frontier in-neighbours, restricted the
// same way, and stops reading in-edges once every pair it still lacks has
// been found.  The compaction of the next step writes the distances.
// ---------------------------------------------------------------------------

// 64-bit OR over the 16 lanes of this lane's row.
__device__ __forceinline__ unsigned long long row16_or64(unsigned long long x) {
  return ((unsigned long long)row16_or((uint32_t)(x >> 32)) << 32) | row16_or((uint32_t)x);
}

// 64-bit OR over the wavefront (wave-uniform result).
__device__ __forceinline__ unsigned long long wave_or64(unsigned long long x) {
  const unsigned long long r = row16_or64(x);
  return lane64(r, 0) | lane64(r, 16) | lane64(r, 32) | lane64(r, 48);
}

// 64-bit value of lane n (a constant, 0..15) of this lane's 16-lane row.
__device__ __forceinline__ unsigned long long row_share64(unsigned long long x, int n) {
  const uint32_t lo = (uint32_t)row_share((int)(uint32_t)x, n);
  const uint32_t hi = (uint32_t)row_share((int)(uint32_t)(x >> 32), n);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long shfl64(unsigned long long x, int src) {
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, src, kWave);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src, kWave);
  return ((unsigned long long)hi << 32) | lo;
}

// The nseg (<= S) mask words of a row: 16-byte loads when the row is a whole
// number of them (nseg = S = 2, 4 or 8: rows are then 16-byte aligned).
template <int S>
__device__ __forceinline__ void load_mask_row(const unsigned long long* p, int nseg,
                                              unsigned long long (&x)[S]) {
  if constexpr (S >= 2) {
    if (nseg == S) {
#pragma unroll
      for (int s = 0; s < S; s += 2) {
        const ulonglong2 t = *reinterpret_cast<const ulonglong2*>(p + s);
        x[s] = t.x;
        x[s + 1] = t.y;
      }
      return;
    }
  }
#pragma unroll
  for (int s = 0; s < S; s++) x[s] = s < nseg ? p[s] : 0ull;
}

// Push over the rows (or row chunks) held one per lane -- edges
// [start, start + len) of row u when ok -- one edge per lane over their
// concatenated edge lists.  colacc[s]: sources of segment s reached.
template <int S>
__device__ __forceinline__ void utile_push_rows(const TileArgs& A, int q, int qn, bool ok,
                                                int32_t u, int32_t start, int32_t len,
                                                unsigned long long (&colacc)[S]) {
  const int lane = lane_id(), nseg = A.nseg;
  unsigned long long xs[S];
#pragma unroll
  for (int s = 0; s < S; s++) xs[s] = 0ull;
  if (ok) load_mask_row<S>(A.mk[q] + (size_t)u * nseg, nseg, xs);
  const int32_t L = ok ? len : 0;
  int32_t incl = L;  // inclusive prefix sum of the lengths
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t y = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += y;
  }
  const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
  for (int32_t e0 = 0; e0 < total; e0 += kWave) {
    const int32_t g = e0 + lane;
    int r = 0;  // the row of edge g: first lane whose inclusive prefix exceeds g
    for (int st = kWave / 2; st > 0; st >>= 1)
      if (__shfl(incl, r + st - 1, kWave) <= g) r += st;
    const bool ge = g < total;
    const int32_t ir = __shfl(incl, r, kWave), lr = __shfl(L, r, kWave);
    const int32_t sr = __shfl(start, r, kWave);
    const int32_t v = ge ? A.colidx[sr + g - (ir - lr)] : 0;
#pragma unroll
    for (int s = 0; s < S; s++) {
      if (s < nseg) {
        const unsigned long long xw = shfl64(xs[s], r);
        if (ge && xw) {
          const size_t i = (size_t)v * nseg + s;
          const unsigned long long y = xw & ~A.vis[i] & ~A.mk[qn][i];
          if (y) {
            atomicOr(&A.mk[qn][i], y);
            colacc[s] |= y;
          }
        }
      }
    }
  }
}

// One push step of a hop-count tile over workgroups gb of nb (every thread of
// the workgroup calls it).
template <int S>
__device__ void utile_push_step(const TileArgs& A, uint32_t step, uint32_t gb, uint32_t nb,
                                unsigned long long* sh_colact) {
  TileCtl* C = A.ctl;
  const int q = step % 3, qn = (step + 1) % 3, rc = step % kRot, rn = (step + 1) % kRot;
  tile_clear_prev(A, step, gb, nb);
  if (threadIdx.x < kSegMax) sh_colact[threadIdx.x] = 0ull;
  __syncthreads();
  const int lane = lane_id(), W = blockDim.x >> 6;
  const uint32_t gw = gb * W + (threadIdx.x >> 6), nwv = nb * W;
  const uint32_t n0 = min(ld_agent(&C->cnt[rc][0].v), A.cap_v);
  const uint32_t n1 = min(ld_agent(&C->cnt[rc][1].v), A.cap_v);
  const uint32_t n2 = min(ld_agent(&C->cnt[rc][2].v), A.cap_wg);
  // batches: 64 rows of the group tier, 64 of the wave tier, 4 row chunks
  const uint32_t b0 = (n0 + 63) / 64, b1 = b0 + (n1 + 63) / 64, b2 = b1 + (n2 + 3) / 4;
  unsigned long long colacc[S];
#pragma unroll
  for (int s = 0; s < S; s++) colacc[s] = 0ull;
  for (uint32_t b = gw; b < b2; b += nwv) {
    bool ok = false;
    int32_t u = 0, start = 0, len = 0;
    if (b < b1) {
      const bool grp = b < b0;
      const uint32_t i = (grp ? b : b - b0) * 64 + (uint32_t)lane;
      ok = i < (grp ? n0 : n1);
      if (ok) {
        u = ld_queue(grp ? A.qgrp[q] + i : A.qwave[q] + i);
        start = A.rowptr[u];
        len = A.rowptr[u + 1] - start;
      }
    } else {
      const uint32_t i = (b - b1) * 4 + (uint32_t)lane;
      ok = lane < 4 && i < n2;
      if (ok) {
        const int4 r = ld_queue4(&A.qwg[q][i]);
        u = r.x;
        start = r.y;
        len = r.z;
      }
    }
    utile_push_rows<S>(A, q, qn, ok, u, start, len, colacc);
  }
#pragma unroll
  for (int s = 0; s < S; s++) {
    if (s < A.nseg) {
      const unsigned long long x = wave_or64(colacc[s]);
      if (lane == 0 && x) atomicOr(&sh_colact[s], x);
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < A.nseg && sh_colact[threadIdx.x])
    or_new_bits(&C->colact[rn][threadIdx.x], sh_colact[threadIdx.x]);
}

template <int S>
__global__ void __launch_bounds__(1024) utile_push_kernel(TileArgs A, int32_t cap_n) {
  __shared__ unsigned long long sh_colact[kSegMax];
  TileCtl* C = A.ctl;
  if (ld_agent(&C->done)) return;
  const uint32_t step = ld_agent(&C->step);
  if (tile_is_pull_step(A, step)) return;  // the pull kernel runs this step
  utile_push_step<S>(A, step, blockIdx.x, gridDim.x, sh_colact);
  tile_end_step(A, step, cap_n);
}

// The remaining steps of a hop-count tile in one launch (push steps only),
// with a grid barrier after each compaction and each push step; at most n
// steps in all.  As tile_persistent_kernel.
template <int S>
__global__ void __launch_bounds__(1024) utile_persistent_kernel(TileArgs A) {
  __shared__ unsigned long long sh_colact[kSegMax];
  __shared__ CompactShared csh;
  TileCtl* C = A.ctl;
  if (ld_agent(&C->done)) return;
  Acc acc;
  uint32_t epoch = 0;
  const uint32_t bar_base = ld_agent(&C->bar_base);
  uint32_t step = ld_agent(&C->step);
  int32_t status = 1;
  for (;;) {
    if (blockIdx.x == 0) tile_prologue(C, step, A.K);
    tile_compact<true>(A, step, blockIdx.x, gridDim.x, acc, csh);
    if (!grid_sync(&C->bar.v, &C->abort, gridDim.x, bar_base, epoch, A.bar_ticks)) {
      status = -2;
      break;
    }
    utile_push_step<S>(A, step, blockIdx.x, gridDim.x, sh_colact);
    if (!grid_sync(&C->bar.v, &C->abort, gridDim.x, bar_base, epoch, A.bar_ticks)) {
      status = -2;
      break;
    }
    const bool act = any_active(C, (step + 1) % kRot, A.nseg);
    step++;
    if (!act) break;
    if (step >= (uint32_t)A.n) { status = 0; break; }
  }
  CtrStripe& Sx = C->ctr[blockIdx.x % kCtrStripes];
  flush_acc(acc, &Sx.fe, &Sx.es, &Sx.im, &Sx.sa, &Sx.se);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st_agent(&C->step, step);
    st_agent(&C->bar_base, bar_base + epoch * gridDim.x);
    st_agent_i(&C->converged, status);
    st_agent(&C->done, 1u);
  }
}

// Pull: each 16-lane group takes one in-edge chunk of a target v, 16 in-edges
// at a time; lane j (< nseg) of the group holds v's segment-j words.
template <int S>
__global__ void __launch_bounds__(kPullThreads) utile_pull_kernel(TileArgs A, int32_t cap_n) {
  __shared__ unsigned long long sh_colact[kSegMax];
  TileCtl* C = A.ctl;
  if (ld_agent(&C->done)) return;
  const uint32_t step = ld_agent(&C->step);
  if (step != ld_agent(&C->cstep)) return;  // a push step ran (see tile_pull_kernel)
  if (!tile_is_pull_step(A, step)) return;  // the push kernel runs this step
  const int q = step % 3, qn = (step + 1) % 3, rn = (step + 1) % kRot;
  tile_clear_prev(A, step, blockIdx.x, gridDim.x);
  if (threadIdx.x < kSegMax) sh_colact[threadIdx.x] = 0ull;
  __syncthreads();
  const int lane = lane_id(), g = lane >> 4, j16 = lane & 15, nseg = A.nseg;
  const uint32_t gw = blockIdx.x * (kPullThreads / kWave) + (threadIdx.x >> 6);
  const uint32_t nwv = gridDim.x * (kPullThreads / kWave);
  const uint32_t nch = (uint32_t)min((long long)A.T.hdr->nchunks, (long long)A.T.cap_chunks);
  const uint32_t* fbm = A.fbm[step & 1];
  const unsigned long long live = j16 < nseg ? ld_agent64(&C->live[j16]) : 0ull;
  unsigned long long colacc = 0ull;  // lanes j16 < nseg: sources of segment j16 reached
  for (uint32_t c0 = gw * 4; c0 < nch; c0 += nwv * 4) {
    const uint32_t c = c0 + (uint32_t)g;
    const bool cok = c < nch;
    const int4 ch = cok ? A.T.chunks[c] : make_int4(0, 0, 0, 0);
    const int32_t v = ch.x, start = ch.y, len = ch.z;
    const bool split = ch.w != 0;
    // the pairs of v not reached yet
    const unsigned long long nd =
        (cok && j16 < nseg) ? (~A.vis[(size_t)v * nseg + j16] & live) : 0ull;
    unsigned long long need[S], acc[S];
    bool open = false;
#pragma unroll
    for (int s = 0; s < S; s++) {
      need[s] = s < nseg ? row_share64(nd, s) : 0ull;
      acc[s] = 0ull;
      open |= need[s] != 0ull;
    }
    for (int32_t b = 0; __ballot(open && b < len) != 0ull; b += 16) {
      const bool act = open && b + j16 < len;
      int32_t u = 0;
      bool fr = false;
      if (act) {
        u = A.T.colidx[start + b + j16];
        fr = ((fbm[u >> 5] >> (u & 31)) & 1u) != 0u;
      }
      unsigned long long m[S];
#pragma unroll
      for (int s = 0; s < S; s++) m[s] = 0ull;
      if (fr) load_mask_row<S>(A.mk[q] + (size_t)u * nseg, nseg, m);
      bool full = true;
#pragma unroll
      for (int s = 0; s < S; s++) {
        if (s < nseg) {
          acc[s] |= row16_or64(m[s] & need[s]);
          full = full && acc[s] == need[s];
        }
      }
      if (full) open = false;
    }
    // the pairs reached become v's next mask words, one lane per segment
    unsigned long long x = 0ull;
#pragma unroll
    for (int s = 0; s < S; s++)
      if (s == j16) x = acc[s];
    if (cok && j16 < nseg && x) {
      unsigned long long* mp = A.mk[qn] + (size_t)v * nseg + j16;
      if (split) atomicOr(mp, x);
      else *mp = x;
      colacc |= x;
    }
  }
  if (j16 < nseg && colacc) atomicOr(&sh_colact[j16], colacc);
  __syncthreads();
  if ((int)threadIdx.x < A.nseg && sh_colact[threadIdx.x])
    or_new_bits(&C->colact[rn][threadIdx.x], sh_colact[threadIdx.x]);
  tile_end_step(A, step, cap_n);
}

// ---------------------------------------------------------------------------
// outputs
// ---------------------------------------------------------------------------

// out[(j) * ld + v] = D[v][col0 + j] for j < count: 64 x 64 tiles through LDS so
// both the read (rows of D) and the write (rows of out) are contiguous.  Rows
// of D are read 16 bytes per lane (16 lanes per 64-column row segment); rows of
// out are written 16 bytes per lane when every output row starts 16-byte
// aligned (VEC), else 4 bytes per lane.
template <bool VEC>
__global__ void __launch_bounds__(256) tile_store_kernel(const uint32_t* D, int32_t n, int32_t K,
                                                         int32_t col0, int32_t count,
                                                         uint32_t* out, int64_t ld) {
  __shared__ uint32_t t[64][65];
  const int64_t v0 = (int64_t)blockIdx.x * 64;
  const int32_t c0 = blockIdx.y * 64;
  const int q = threadIdx.x & 15, r16 = threadIdx.x >> 4;  // 16 lanes per row, 16 rows at a time
  for (int r = r16; r < 64; r += 16) {
    const int64_t v = v0 + r;
    uint4 x = make_uint4(0u, 0u, 0u, 0u);
    // col0 and K are multiples of 64, so the 16-byte load is aligned; columns
    // past `count` are read (they exist in the tile) but never stored
    if (v < n) x = *reinterpret_cast<const uint4*>(D + (size_t)v * K + col0 + c0 + 4 * q);
    t[r][4 * q] = x.x;
    t[r][4 * q + 1] = x.y;
    t[r][4 * q + 2] = x.z;
    t[r][4 * q + 3] = x.w;
  }
  __syncthreads();
  if constexpr (VEC) {
    for (int r = r16; r < 64; r += 16) {
      const int32_t c = c0 + r;
      const int64_t v = v0 + 4 * q;
      if (c >= count || v >= n) continue;
      uint32_t* o = out + (size_t)c * ld + v;
      if (v + 3 < n) {
        *reinterpret_cast<uint4*>(o) = make_uint4(t[4 * q][r], t[4 * q + 1][r], t[4 * q + 2][r],
                                                  t[4 * q + 3][r]);
      } else {
        for (int i = 0; v + i < n; i++) o[i] = t[4 * q + i][r];
      }
    }
  } else {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
      const int32_t c = c0 + r;
      const int64_t v = v0 + tx;
      if (c < count && v < n) out[(size_t)c * ld + v] = t[tx][r];
    }
  }
}

// Hop-count tiles: out[(c - col0) * ld + v] for columns c in [col0, col0 +
// count): the pair's level assembled from the bit planes in use (levels up
// to the last step, whose compaction ran at step - 1), INF if never reached.
// A workgroup takes 64 vertices (lane = vertex) and one 64-column segment,
// four rows at a time, so every store is 64 contiguous words; the segment is
// the grid's second index, so the workgroups running together write the same
// 64 output rows.
__global__ void __launch_bounds__(256) utile_store_kernel(TileArgs A, int32_t col0, int32_t count,
                                                          uint32_t* out, int64_t ld) {
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t v = (int64_t)blockIdx.x * 64 + tx;
  const int nseg = A.nseg;
  const uint32_t last = ld_agent_block(&A.ctl->step);  // levels are <= last - 1
  int nb = 0;
  while (nb < A.nplanes && ((uint32_t)1 << nb) < last) nb++;  // planes 0 .. nb-1 are in use
  const size_t pn = (size_t)A.n * nseg;
  const int s = (col0 >> 6) + (int)blockIdx.y;
  // this thread's 16 columns of the segment: bits ty, ty + 4, ..., ty + 60
  uint32_t lvl[16];
#pragma unroll
  for (int i = 0; i < 16; i++) lvl[i] = 0u;
  for (int b = 0; b < nb; b++) {
    const unsigned long long w = v < A.n ? A.planes[(size_t)b * pn + v * nseg + s] >> ty : 0ull;
#pragma unroll
    for (int i = 0; i < 16; i++) lvl[i] |= (uint32_t)((w >> (4 * i)) & 1ull) << b;
  }
  const unsigned long long vw = v < A.n ? A.vis[v * nseg + s] >> ty : 0ull;
#pragma unroll
  for (int i = 0; i < 16; i++) {
    const int c = s * 64 + ty + 4 * i;
    if (c >= col0 && c < col0 + count && v < A.n)
      out[(size_t)(c - col0) * ld + v] = ((vw >> (4 * i)) & 1ull) ? lvl[i] : 0xFFFFFFFFu;
  }
}

__global__ void tile_read_col_kernel(const uint32_t* D, int32_t n, int32_t K, int32_t col,
                                     uint32_t* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    out[v] = D[(size_t)v * K + col];
}

__global__ void tile_done_bits_kernel(const TileCtl* C, int32_t k, uint32_t* done) {
  const int w = threadIdx.x;  // 32-bit words of the caller's k columns
  if (w >= (k + 31) / 32) return;
  const int rc = ld_agent(&C->step) % kRot;
  const int seg = w >> 1, half = (w & 1) * 32;
  const uint32_t live = (uint32_t)(ld_agent64(&C->live[seg]) >> half);
  const uint32_t act = (uint32_t)(ld_agent64(&C->colact[rc][seg]) >> half);
  const uint32_t valid = (w == (k - 1) / 32 && (k & 31)) ? ((1u << (k & 31)) - 1u) : ~0u;
  done[w] = live & ~act & valid;
}

// The run summary (info non-null), or the run's status into the run-status
// latch when it is not 1 (info null).
__global__ void tile_info_kernel(const TileCtl* C, int32_t K, dawn_run_info* info,
                                 uint32_t* latch) {
  __shared__ int32_t s_max;
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  int32_t mx = 0;
  for (int j = threadIdx.x; j < K; j += blockDim.x) mx = max(mx, ld_agent_i(&C->colsteps[j]));
  atomicMax(&s_max, mx);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int32_t conv = run_status(ld_agent_i(&C->converged), ld_agent(&C->abort),
                                  ld_agent(&C->overflow));
  if (!info) {
    latch_status(latch, conv);
    return;
  }
  info->steps = s_max;
  info->converged = conv;
  unsigned long long fe = 0, es = 0, im = 0, sa = 0, se = 0;
  for (int i = 0; i < kCtrStripes; ++i) {
    fe += ld_agent64(&C->ctr[i].fe);
    es += ld_agent64(&C->ctr[i].es);
    im += ld_agent64(&C->ctr[i].im);
    sa += ld_agent64(&C->ctr[i].sa);
    se += ld_agent64(&C->ctr[i].se);
  }
  info->frontier_entries = (int64_t)sa;
  info->edges_scanned = (int64_t)se;
  info->improvements = (int64_t)im;
  info->union_rows = (int64_t)fe;
  info->union_edges = (int64_t)es;
}

__global__ void tile_col_steps_kernel(const TileCtl* C, int32_t k, int32_t* out) {
  for (int j = threadIdx.x; j < k; j += blockDim.x) out[j] = ld_agent_i(&C->colsteps[j]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
TileLayout tile_layout(int64_t n, int64_t m, int32_t k, bool unweighted) {
  TileLayout L{};
  L.unweighted = unweighted;
  Carver c;
  L.nseg = (k + 63) / 64;
  L.K = L.nseg * 64;
  L.cap_v = (uint32_t)n;
  // rows above the smallest allowed threshold (32), each in at most deg/64 + 1
  // chunks (smallest allowed chunk 64)
  L.cap_wg = (uint32_t)(m / 33 + m / 64 + 2);
  L.ctl = c.take(sizeof(TileCtl));
  L.info = c.take(sizeof(dawn_run_info));
  // hop-count tiles keep their distances as bit planes (levels < n), not in D
  if (!unweighted) L.D = c.take((size_t)n * L.K * 4);
  for (int i = 0; i < 3; i++) L.mk[i] = c.take((size_t)n * L.nseg * 8);
  for (int i = 0; i < 3; i++) L.qgrp[i] = c.take((size_t)n * 4);
  for (int i = 0; i < 3; i++) L.qwave[i] = c.take((size_t)n * 4);
  for (int i = 0; i < 3; i++) L.qwg[i] = c.take((size_t)L.cap_wg * 16);
  for (int i = 0; i < 2; i++) L.fbm[i] = c.take((size_t)((n + 63) / 64) * 8);
  if (unweighted) {
    L.vis = c.take((size_t)n * L.nseg * 8);
    int32_t p = 1;
    while (p < 31 && ((int64_t)1 << p) < n) p++;
    L.nplanes = p;
    L.planes = c.take((size_t)p * n * L.nseg * 8);
  }
  L.total = c.off;
  return L;
}

TileArgs tile_args(const int32_t* rowptr, const int32_t* colidx, const void* w, int32_t n,
                   int32_t m, const TileLayout& L, void* ws) {
  const Tuning& T = tuning();
  char* base = static_cast<char*>(ws);
  TileArgs A{};
  A.rowptr = rowptr;
  A.colidx = colidx;
  A.w = static_cast<const uint32_t*>(w);
  A.D = L.unweighted ? nullptr : reinterpret_cast<uint32_t*>(base + L.D);
  A.n = n;
  A.m = m;
  A.K = L.K;
  A.nseg = L.nseg;
  A.t_wave = T.tile_t_wave;
  A.t_chunk = T.tile_t_chunk;
  A.t_group = T.tile_t_group;
  A.skip = T.tile_skip;
  A.sparse = T.tile_sparse;
  A.T = TGraph{};
  A.pull_min = -1;
  A.pull_src = 0;
  for (int i = 0; i < 3; i++) {
    A.mk[i] = reinterpret_cast<unsigned long long*>(base + L.mk[i]);
    A.qgrp[i] = reinterpret_cast<int32_t*>(base + L.qgrp[i]);
    A.qwave[i] = reinterpret_cast<int32_t*>(base + L.qwave[i]);
    A.qwg[i] = reinterpret_cast<int4*>(base + L.qwg[i]);
  }
  for (int i = 0; i < 2; i++) A.fbm[i] = reinterpret_cast<uint32_t*>(base + L.fbm[i]);
  A.cap_v = L.cap_v;
  A.cap_wg = L.cap_wg;
  A.ctl = reinterpret_cast<TileCtl*>(base + L.ctl);
  A.vis = L.unweighted ? reinterpret_cast<unsigned long long*>(base + L.vis) : nullptr;
  A.planes = L.unweighted ? reinterpret_cast<unsigned long long*>(base + L.planes) : nullptr;
  A.nplanes = L.unweighted ? L.nplanes : 0;
  A.bar_ticks = (unsigned long long)T.barrier_ms * kTicksPerMs;
  A.latch = dev_info().latch;
  return A;
}

static int grid_for(int64_t work, int threads) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (work + threads - 1) / threads));
}

dawn_status tile_reset(const TileArgs& a, bool f32, hipStream_t stream) {
  const int g = grid_for((int64_t)a.n * a.K / 4, 256);
  if (f32) hipLaunchKernelGGL(tile_fill_kernel<true>, dim3(g), dim3(256), 0, stream, a);
  else hipLaunchKernelGGL(tile_fill_kernel<false>, dim3(g), dim3(256), 0, stream, a);
  return hip_check(hipGetLastError(), "tile reset");
}

__global__ void ss_validate_kernel(const int32_t* rowptr, const int32_t* colidx,
                                   const uint32_t* w, int32_t n, int32_t m, int32_t is_f32,
                                   uint32_t* done, int32_t* converged);

dawn_status tile_seed_all(const TileArgs& a, const int32_t* sources_dev, int32_t count,
                          bool validate, bool f32, hipStream_t stream) {
  if (validate) {
    hipLaunchKernelGGL(ss_validate_kernel, dim3(grid_for(a.m, 256)), dim3(256), 0, stream,
                       a.rowptr, a.colidx, a.w, a.n, a.m, (int32_t)f32, &a.ctl->done,
                       &a.ctl->converged);
  }
  hipLaunchKernelGGL(tile_seed_kernel, dim3(1), dim3(512), 0, stream, a, sources_dev, count);
  return hip_check(hipGetLastError(), "tile seed");
}

dawn_status tile_admit(const TileArgs& a, bool f32, int32_t col, int32_t source,
                       hipStream_t stream) {
  const int g = grid_for(a.n, 256);
  if (f32) hipLaunchKernelGGL(tile_col_fill_kernel<true>, dim3(g), dim3(256), 0, stream, a, col);
  else hipLaunchKernelGGL(tile_col_fill_kernel<false>, dim3(g), dim3(256), 0, stream, a, col);
  hipLaunchKernelGGL(tile_admit_kernel, dim3(1), dim3(64), 0, stream, a, col, source);
  return hip_check(hipGetLastError(), "tile admit");
}

dawn_status tile_evict(const TileArgs& a, bool f32, int32_t col, hipStream_t stream) {
  const int g = grid_for(a.n, 256);
  if (f32) hipLaunchKernelGGL(tile_col_fill_kernel<true>, dim3(g), dim3(256), 0, stream, a, col);
  else hipLaunchKernelGGL(tile_col_fill_kernel<false>, dim3(g), dim3(256), 0, stream, a, col);
  hipLaunchKernelGGL(tile_evict_kernel, dim3(1), dim3(64), 0, stream, a, col);
  return hip_check(hipGetLastError(), "tile evict");
}

Residency tile_persistent_residency(int threads) {
  if (threads <= 0) threads = kTilePersistentThreads;
  return residency_of(tile_persistent_kernel<false>, threads);
}

Residency utile_persistent_residency(int threads) {
  if (threads <= 0) threads = kTilePersistentThreads;
  return residency_of(utile_persistent_kernel<4>, threads);
}

// Launch a persistent kernel on `grid` x `threads` (cooperatively when asked
// for and the stream is not being captured).
template <typename K, typename... Args>
static hipError_t launch_persistent(K kernel, int grid, int threads, hipStream_t stream,
                                    Args... args) {
  const Tuning& T = tuning();
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const bool capturing =
      hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
  if (dev_info().coop && T.coop && !capturing) {
    void* ptrs[] = {&args...};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kernel), dim3(grid),
                                      dim3(threads), ptrs, 0, stream);
  }
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), 0, stream, args...);
  return hipGetLastError();
}

dawn_status utile_persistent(const TileArgs& a, hipStream_t stream) {
  const Tuning& T = tuning();
  const int threads = T.wg_threads > 0 ? T.wg_threads : kTilePersistentThreads;
  auto k = a.nseg <= 1 ? utile_persistent_kernel<1> : a.nseg <= 2 ? utile_persistent_kernel<2>
         : a.nseg <= 4 ? utile_persistent_kernel<4> : utile_persistent_kernel<8>;
  int grid = residency_of(k, threads).grid;
  if (T.grid > 0 && T.grid < grid) grid = T.grid;
  void* tk = ktimer_begin(stream);
  const hipError_t e = launch_persistent(k, grid, threads, stream, a);
  ktimer_end(tk, stream, 1);
  return hip_check(e, "hop-count tile persistent launch");
}

template <bool F32>
static dawn_status tile_steps_t(const TileArgs& a, bool persistent, int32_t max_steps,
                                hipStream_t stream) {
  const Tuning& T = tuning();
  const int threads = T.wg_threads > 0 ? T.wg_threads : 256;
  const int32_t cap_n = persistent ? 1 : 0;
  if (persistent) {
    const int pthreads = T.wg_threads > 0 ? T.wg_threads : kTilePersistentThreads;
    int grid = residency_of(tile_persistent_kernel<F32>, pthreads).grid;
    if (T.grid > 0 && T.grid < grid) grid = T.grid;
    TileArgs aa = a;
    aa.pull_min = -1;  // pull steps need the step-launch path
    void* tk = ktimer_begin(stream);
    const hipError_t e =
        launch_persistent(tile_persistent_kernel<F32>, grid, pthreads, stream, aa, max_steps, cap_n);
    ktimer_end(tk, stream, 1);
    return hip_check(e, "tile persistent launch");
  }
  // push relaxation: 4 workgroups per CU, fewer for small graphs (about one
  // workgroup per 64 vertices, at least one per CU).  Each workgroup ends the
  // step with an agent-scope release (an L2 write-back) and an arrival on one
  // counter, about 50 ns of serial time apiece: on R-MAT scale 20, 16 per CU
  // made a push step with a near-empty frontier cost ~200 us instead of ~20.
  const int cus = dev_info().cus;
  const int grid = T.grid > 0 ? T.grid
                              : (int)std::max<int64_t>(cus, std::min<int64_t>(4 * cus, ((int64_t)a.n + 63) / 64));
  // compaction: one 1024-thread workgroup per CU (fewer for small graphs)
  const int cgrid = (int)std::max<int64_t>(1, std::min<int64_t>(cus, ((int64_t)a.n + 1023) / 1024));
  const bool pull = a.T.hdr != nullptr && a.pull_min >= 0;
  const int pgrid = 16 * cus;
  for (int s = 0; s < max_steps; s++) {
    hipLaunchKernelGGL(tile_compact_kernel<false>, dim3(cgrid), dim3(1024), 0, stream, a);
    void* tk = ktimer_begin(stream);
    hipLaunchKernelGGL(tile_step_kernel<F32>, dim3(grid), dim3(threads), 0, stream, a, 0);
    if (pull)
      hipLaunchKernelGGL(tile_pull_kernel<F32>, dim3(pgrid), dim3(kPullThreads), 0, stream, a, 0);
    ktimer_end(tk, stream, 1);
  }
  return hip_check(hipGetLastError(), "tile step launches");
}

dawn_status utile_steps(const TileArgs& a, int32_t max_steps, hipStream_t stream) {
  const Tuning& T = tuning();
  const int threads = T.wg_threads > 0 ? T.wg_threads : 256;
  const int cus = dev_info().cus;
  const int grid = T.grid > 0 ? T.grid
                              : (int)std::max<int64_t>(cus, std::min<int64_t>(4 * cus, ((int64_t)a.n + 63) / 64));
  const int cgrid = (int)std::max<int64_t>(1, std::min<int64_t>(cus, ((int64_t)a.n + 1023) / 1024));
  const bool pull = a.T.hdr != nullptr && a.pull_min >= 0;
  const int pgrid = 16 * cus;
  // kernels specialised for the largest segment count they serve
  auto push = a.nseg <= 1 ? utile_push_kernel<1> : a.nseg <= 2 ? utile_push_kernel<2>
            : a.nseg <= 4 ? utile_push_kernel<4> : utile_push_kernel<8>;
  auto pullk = a.nseg <= 1 ? utile_pull_kernel<1> : a.nseg <= 2 ? utile_pull_kernel<2>
             : a.nseg <= 4 ? utile_pull_kernel<4> : utile_pull_kernel<8>;
  for (int s = 0; s < max_steps; s++) {
    hipLaunchKernelGGL(tile_compact_kernel<true>, dim3(cgrid), dim3(1024), 0, stream, a);
    void* tk = ktimer_begin(stream);
    hipLaunchKernelGGL(push, dim3(grid), dim3(threads), 0, stream, a, 0);
    if (pull) hipLaunchKernelGGL(pullk, dim3(pgrid), dim3(kPullThreads), 0, stream, a, 0);
    ktimer_end(tk, stream, 1);
  }
  return hip_check(hipGetLastError(), "hop-count tile step launches");
}

dawn_status tile_steps(const TileArgs& a, bool f32, bool persistent, int32_t max_steps,
                       hipStream_t stream) {
  return f32 ? tile_steps_t<true>(a, persistent, max_steps, stream)
             : tile_steps_t<false>(a, persistent, max_steps, stream);
}

dawn_status tile_done_bits(const TileArgs& a, int32_t k, uint32_t* done_bits, hipStream_t stream) {
  hipLaunchKernelGGL(tile_done_bits_kernel, dim3(1), dim3(64), 0, stream, a.ctl, k, done_bits);
  return hip_check(hipGetLastError(), "tile done bits");
}

dawn_status tile_store(const TileArgs& a, int32_t col0, int32_t count, void* out, int64_t ld,
                       hipStream_t stream) {
  const dim3 grid((unsigned)((a.n + 63) / 64), (unsigned)((count + 63) / 64));
  const bool vec = ld % 4 == 0 && (reinterpret_cast<uintptr_t>(out) & 15u) == 0;
  if (vec)
    hipLaunchKernelGGL(tile_store_kernel<true>, grid, dim3(256), 0, stream, a.D, a.n, a.K, col0,
                       count, static_cast<uint32_t*>(out), ld);
  else
    hipLaunchKernelGGL(tile_store_kernel<false>, grid, dim3(256), 0, stream, a.D, a.n, a.K, col0,
                       count, static_cast<uint32_t*>(out), ld);
  return hip_check(hipGetLastError(), "tile store");
}

dawn_status utile_store(const TileArgs& a, int32_t col0, int32_t count, uint32_t* out, int64_t ld,
                        hipStream_t stream) {
  if (count < 1) return DAWN_OK;
  const unsigned segs = (unsigned)(((col0 + count - 1) >> 6) - (col0 >> 6) + 1);
  hipLaunchKernelGGL(utile_store_kernel, dim3((unsigned)((a.n + 63) / 64), segs), dim3(256), 0,
                     stream, a, col0, count, out, ld);
  return hip_check(hipGetLastError(), "hop-count tile store");
}

dawn_status tile_read_col(const TileArgs& a, int32_t col, void* out, hipStream_t stream) {
  hipLaunchKernelGGL(tile_read_col_kernel, dim3(grid_for(a.n, 256)), dim3(256), 0, stream, a.D,
                     a.n, a.K, col, static_cast<uint32_t*>(out));
  return hip_check(hipGetLastError(), "tile read");
}

dawn_status tile_info(const TileArgs& a, dawn_run_info* info, hipStream_t stream) {
  hipLaunchKernelGGL(tile_info_kernel, dim3(1), dim3(256), 0, stream, a.ctl, a.K, info, a.latch);
  return hip_check(hipGetLastError(), "tile info");
}

dawn_status tile_col_steps(const TileArgs& a, int32_t k, int32_t* out, hipStream_t stream) {
  hipLaunchKernelGGL(tile_col_steps_kernel, dim3(1), dim3(256), 0, stream, a.ctl, k, out);
  return hip_check(hipGetLastError(), "tile steps");
}

}  // namespace dawn
