// govm_sssp.hip -- single-source GOVM (Section 3.4, Algorithm 2) on gfx950.
//
// One step expands every row in the frontier delta (the rows whose distance
// changed in the previous step, Algorithm 2's `delta[j] = true and start != end`
// test): for each out-edge (u, v, w) it forms cand = alpha[u] (+) w and lowers
// alpha[v] to cand if cand is strictly smaller (with the `index != source`
// guard).  Every v lowered this step is recorded in beta; beta becomes the next
// delta and the loop stops after a step that lowers nothing (`ptr` false) or
// after n steps.
//
// Mapping to the device:
// - delta is the beta bitmap of the step, split by out-degree:
//     lane tier (deg <= t_lane): found by scanning the bitmap a block of words
//       at a time, 64 rows per wavefront; the wavefront's rows are concatenated
//       through an LDS prefix sum so each lane takes one edge;
//     wave tier (deg <= t_wave): also queued; one wavefront per row, lanes
//       stride the row;
//     workgroup tier: also queued, the row cut into t_chunk-edge chunks, one
//       workgroup each.
// - the lane whose atomicOr first sets a long row's bit appends it to the
//   right next-step queue (wavefront ballot + mbcnt prefix, gathered per
//   workgroup in LDS, one atomicAdd per tier and workgroup).  The scan clears
//   the bitmap of the current step, n/32 words per step.
// - The relaxation reads alpha[v] with a plain load first (a stale value can
//   only be higher, so skipping on it is safe) and uses atomicMin only when
//   the candidate is smaller.  Order of updates inside a step does not matter:
//   the fixed point is unique (Section 3.5: the method does not care in which
//   order paths appear).
// - Step loop: one persistent launch with a grid barrier per step, or a fixed
//   number of launches of one step each (last-block bookkeeping) followed by
//   the persistent launch for the remaining steps.  The host never waits.
#include <stdio.h>

#include <algorithm>

#include "govm_host.hpp"

namespace dawn {

// ---------------------------------------------------------------------------
// init
// ---------------------------------------------------------------------------
// hv (may be null): bit v set when row v has more than t_lane edges, the rows
// that steps take from the wave and workgroup queues rather than from the bitmap.
template <int WT>
__global__ void ss_fill_kernel(uint32_t* dist, int64_t n, uint32_t* bm0, uint32_t* bm1,
                               int64_t nwords, SsCtl* ctl, const int32_t* rowptr, uint32_t* hv,
                               int32_t t_lane) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < n; i += stride) dist[i] = inf_key<WT>();
  for (int64_t i = tid; i < nwords; i += stride) { bm0[i] = 0; bm1[i] = 0; }
  if (hv) {
    // a wavefront per 64 vertices: the ballot's halves are two bitmap words
    // (blockDim and the grid's thread count are multiples of 64)
    const int lane = lane_id();
    for (int64_t v0 = tid - lane; v0 < n; v0 += stride) {
      const int64_t v = v0 + lane;
      const bool heavy = v < n && rowptr[v + 1] - rowptr[v] > t_lane;
      const unsigned long long b = __ballot(heavy);
      const int64_t wi = v0 / 32 + (lane >> 5);
      if ((lane & 31) == 0 && wi < nwords) hv[wi] = (uint32_t)(b >> (lane & 32));
    }
  }
  if (blockIdx.x == 0) {
    uint32_t* c = reinterpret_cast<uint32_t*>(ctl);
    for (int i = threadIdx.x; i < (int)(sizeof(SsCtl) / 4); i += blockDim.x) c[i] = 0;
  }
}

// CSR checks (tuning field `validate`): rowptr[0] == 0, rowptr[n] == m,
// non-decreasing rows, column ids in range, fp32 weights finite with the sign
// bit clear.  A failure marks the run done with converged = -1.
__global__ void ss_validate_kernel(const int32_t* rowptr, const int32_t* colidx,
                                   const uint32_t* w, int32_t n, int32_t m, int32_t is_f32,
                                   uint32_t* done, int32_t* converged) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  if (tid == 0) bad = rowptr[0] != 0 || rowptr[n] != m;
  for (int64_t i = tid; i < n; i += stride) bad |= rowptr[i + 1] < rowptr[i];
  for (int64_t e = tid; e < m; e += stride) {
    const int32_t v = colidx[e];
    bad |= v < 0 || v >= n;
    if (is_f32) bad |= (w[e] & 0x80000000u) != 0 || (w[e] & 0x7F800000u) == 0x7F800000u;
  }
  if (bad) {
    st_agent_i(converged, -1);
    st_agent(done, 1u);
  }
}

// Put the seeds in step 0's delta: alpha[s] = 0, beta bit set, row queued.
template <int WT>
__global__ void ss_seed_kernel(SsArgs A, const int32_t* sources, const int64_t* voff,
                               int32_t count, int32_t single) {
  SsCtl* C = A.ctl;
  if (ld_agent(&C->done)) return;
  for (int j = threadIdx.x; j < count; j += blockDim.x) {
    int64_t s = sources ? (int64_t)sources[j] : (int64_t)single;
    if (voff) s += voff[j];
    A.dist[s] = zero_key<WT>();
    const uint32_t bit = 1u << (s & 31);
    const uint32_t old = atomicOr(&A.bm[0][s >> 5], bit);
    if (old & bit) continue;  // duplicate seed
    const int32_t start = A.rowptr[s], deg = A.rowptr[s + 1] - start;
    if (deg == 0) continue;
    atomicAdd(&C->ctr.fedges[0], (unsigned long long)deg);
    atomicAdd(&C->ctr.frows[0], 1ull);
    if (deg <= A.t_lane) {
      // short row: step 0 finds it by its bit
    } else if (deg <= A.t_wave) {
      const uint32_t p = atomicAdd(&C->cnt[0][1].v, 1u);
      A.qwave[0][p] = (int32_t)s;
    } else {
      const uint32_t nch = (deg + A.t_chunk - 1) / A.t_chunk;
      const uint32_t p = atomicAdd(&C->cnt[0][2].v, nch);
      for (uint32_t c = 0; c < nch; c++) {
        const int32_t off = (int32_t)c * A.t_chunk;
        if (p + c < A.cap_wg)
          A.qwg[0][p + c] = make_int4((int32_t)s, start + off, min(A.t_chunk, deg - off), c == 0);
      }
    }
  }
}

// int32 weights: keys back to int32 values (INF -> INT32_MAX).
__global__ void ss_decode_i32_kernel(uint32_t* dist, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dist[i] ^= 0x80000000u;
}

// The end of a run's bookkeeping (one thread): the run's status (see
// run_status; with int32 weights a path sum that left the int32 range also
// makes the run count as not converged) and counters go to `info`, or, when
// the caller gave none, a status other than 1 goes to the run-status latch.
template <int WT>
__device__ void ss_report(SsCtl* C, dawn_run_info* info, uint32_t* latch) {
  int32_t conv = run_status(ld_agent_i(&C->converged), ld_agent(&C->abort), ld_agent(&C->overflow));
  if (WT == kWI32 && conv == 1 && ld_agent(&C->negfloor)) conv = 0;
  if (!info) {
    latch_status(latch, conv);
    return;
  }
  const unsigned long long fe = ld_agent64(&C->ctr.fe);
  const unsigned long long es = ld_agent64(&C->ctr.es);
  const unsigned long long im = ld_agent64(&C->ctr.im);
  info->steps = (int32_t)ld_agent(&C->step);
  info->converged = conv;
  info->frontier_entries = (int64_t)fe;
  info->edges_scanned = (int64_t)es;
  info->improvements = (int64_t)im;
  info->union_rows = (int64_t)fe;
  info->union_edges = (int64_t)es;
}

template <int WT>
__global__ void ss_finalize_kernel(SsCtl* C, dawn_run_info* info, uint32_t* latch) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  ss_report<WT>(C, info, latch);
}

// ---------------------------------------------------------------------------
// one step
// ---------------------------------------------------------------------------

// Next-frontier entries found by a workgroup are gathered in LDS and written
// to the global queues once at the end of the step with one atomicAdd per
// tier per workgroup (a queue that fills up spills straight to global memory).
constexpr int kLdsQWave = 512;
constexpr int kUnroll = 4;      // edges in flight per lane (wave and workgroup tiers)
constexpr int kUnrollLane = 4;  // edges in flight per lane (lane tier)

struct SsShared {
  int stage[kMaxWavesPerBlock * 3 * kWave];      // lane-tier batch: prefix, row base, distance
  uint32_t scan[kMaxWavesPerBlock * 2 * kWave];  // bitmap block: short-row bits, their prefix
  int32_t qw[kLdsQWave];
  uint32_t nqw, upd, gbase_w;
};

// Push `v` for lanes with `pred` into the workgroup's LDS queue; lanes past
// its capacity go to the global queue.  Reached by the whole wavefront.
__device__ __forceinline__ void block_push(bool pred, int32_t v, int32_t* sq, uint32_t* sn,
                                           uint32_t lcap, int32_t* gq, uint32_t* gcnt,
                                           uint32_t gcap, uint32_t* overflow) {
  const unsigned long long b = __ballot(pred);
  if (b == 0) return;
  const int leader = __ffsll((long long)b) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(sn, (uint32_t)__popcll(b));
  base = __shfl(base, leader, kWave);
  const uint32_t pos = base + lanes_below(b);
  const bool spill = pred && pos >= lcap;
  if (pred && !spill) sq[pos] = v;
  wave_push(spill, v, gq, gcnt, gcap, overflow);
}

// Record improvements of alpha[v[i]] (lanes with imp[i]): the ptr flag, the
// beta bitmap, and for the first setter of a bit whose row has more than
// t_lane edges, the next-step queue of its degree tier (shorter rows are found
// by the next step's bitmap scan).  Reached by the whole wavefront.  CNT: also
// count the next frontier's rows and out-edges (the pull decision of the next
// step).
template <int WT, int U, bool CNT>
__device__ __forceinline__ void ss_enqueue(const SsArgs& A, const bool (&imp)[U],
                                           const int32_t (&v)[U], const uint32_t (&cand)[U],
                                           int nxt, int rn, Acc& acc, SsShared& sh) {
  bool any = false;
#pragma unroll
  for (int i = 0; i < U; i++) any |= imp[i];
  if (__ballot(any) == 0) return;
  SsCtl* C = A.ctl;
  if (any) sh.upd = 1u;
  bool newv[U];
  uint32_t hvw[U];  // heavy-row words, loaded beside the test-and-set
#pragma unroll
  for (int i = 0; i < U; i++) hvw[i] = imp[i] && !CNT ? A.hv[v[i] >> 5] : 0u;
#pragma unroll
  for (int i = 0; i < U; i++) {
    newv[i] = false;
    if (imp[i]) {
      const uint32_t bit = 1u << (v[i] & 31);
      newv[i] = (atomicOr(&A.bm[nxt][v[i] >> 5], bit) & bit) == 0u;
    }
  }
#pragma unroll
  for (int i = 0; i < U; i++) {
    if (imp[i]) {
      // unit weights: every candidate of a step is the same level (the
      // frontier holds exactly the vertices of the previous level), so the
      // writers agree and a plain store will do
      if constexpr (WT == kWUNIT) A.dist[v[i]] = cand[i];
      else atomicMin(&A.dist[v[i]], cand[i]);  // result unused: not waited for
    }
  }
#pragma unroll
  for (int i = 0; i < U; i++)
    if (newv[i]) acc.im += 1;  // a vertex lowered in this step counts once
  int32_t start[U], deg[U];
#pragma unroll
  for (int i = 0; i < U; i++) {
    start[i] = 0;
    deg[i] = 0;
    if (newv[i] && (CNT || ((hvw[i] >> (v[i] & 31)) & 1u))) {
      start[i] = A.rowptr[v[i]];
      deg[i] = A.rowptr[v[i] + 1] - start[i];
      if (CNT && deg[i] > 0) {
        acc.sa += (unsigned long long)deg[i];  // the next frontier's out-edges
        acc.se += 1;                           // and rows
      }
    }
  }
#pragma unroll
  for (int i = 0; i < U; i++) {
    const bool tw = newv[i] && deg[i] > A.t_lane && deg[i] <= A.t_wave;
    block_push(tw, v[i], sh.qw, &sh.nqw, kLdsQWave, A.qwave[nxt], &C->cnt[rn][1].v, A.cap_v,
               &C->overflow);
    if (newv[i] && deg[i] > A.t_wave) {
      const uint32_t nch = (uint32_t)((deg[i] + A.t_chunk - 1) / A.t_chunk);
      const uint32_t base = atomicAdd(&C->cnt[rn][2].v, nch);
      for (uint32_t c = 0; c < nch; c++) {
        const int32_t off = (int32_t)c * A.t_chunk;
        if (base + c < A.cap_wg)
          A.qwg[nxt][base + c] = make_int4(v[i], start[i] + off, min(A.t_chunk, deg[i] - off), c == 0);
        else
          atomicOr(&C->overflow, 1u);
      }
    }
  }
}

// Relax U edges per lane: all column/weight loads, then all target-distance
// loads, then the atomic mins of the lanes whose candidate is smaller.
template <int WT, int U>
__device__ __forceinline__ void ss_relax_n(const SsArgs& A, const int32_t (&e)[U],
                                           const bool (&valid)[U], const uint32_t (&du)[U],
                                           bool (&imp)[U], int32_t (&v)[U]) {
  uint32_t cand[U];
#pragma unroll
  for (int i = 0; i < U; i++) {
    v[i] = 0;
    cand[i] = 0u;
    if (valid[i]) {
      v[i] = A.colidx[e[i]];
      cand[i] = relax_key<WT>(du[i], WT == kWUNIT ? 1u : A.w[e[i]]);
      if constexpr (WT == kWI32)
        if (cand[i] == 0u) atomicOr(&A.ctl->negfloor, 1u);  // sum left the int32 range
    }
  }
  uint32_t cur[U];
#pragma unroll
  for (int i = 0; i < U; i++) cur[i] = valid[i] ? A.dist[v[i]] : 0u;
#pragma unroll
  for (int i = 0; i < U; i++) {
    imp[i] = false;
    if (valid[i] && cand[i] < cur[i] && v[i] != A.src) imp[i] = cand[i] < atomicMin(&A.dist[v[i]], cand[i]);
  }
}

// Candidates and the plain-load pre-check only, for ss_enqueue: it issues the
// next-frontier test-and-set first and the non-returning atomicMin after it,
// so waiting for the test-and-set does not wait for the atomicMin too (gfx9's
// vector-memory counter retires in order).  A candidate that passes the
// pre-check but loses to a lower value written in the same step only sets a
// bit that the writer of that value sets as well.
template <int WT, int U>
__device__ __forceinline__ void ss_relax_pre(const SsArgs& A, const int32_t (&e)[U],
                                             const bool (&valid)[U], const uint32_t (&du)[U],
                                             bool (&imp)[U], int32_t (&v)[U],
                                             uint32_t (&cand)[U]) {
#pragma unroll
  for (int i = 0; i < U; i++) {
    v[i] = 0;
    cand[i] = 0u;
    if (valid[i]) {
      v[i] = A.colidx[e[i]];
      cand[i] = relax_key<WT>(du[i], WT == kWUNIT ? 1u : A.w[e[i]]);
      if constexpr (WT == kWI32)
        if (cand[i] == 0u) atomicOr(&A.ctl->negfloor, 1u);  // sum left the int32 range
    }
  }
  uint32_t cur[U];
#pragma unroll
  for (int i = 0; i < U; i++) cur[i] = valid[i] ? A.dist[v[i]] : 0u;
#pragma unroll
  for (int i = 0; i < U; i++) imp[i] = valid[i] && cand[i] < cur[i] && v[i] != A.src;
}

// Minimum over the 16 lanes of this lane's row (DPP row rotations).
__device__ __forceinline__ uint32_t row16_min(uint32_t x) {
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x121, 0xF, 0xF, false));
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x122, 0xF, 0xF, false));
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x124, 0xF, 0xF, false));
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false));
  return x;
}

// A pull step (step launches on a dense frontier): each 16-lane group takes
// one in-edge chunk of a target v from the reverse graph and relaxes the
// in-edges whose source is in the step's frontier (its bit in the current
// bitmap), 16 at a time; the best candidate goes through the same enqueue as
// a push step's.  The (edge) relaxations are exactly the push step's; no
// atomicMin per edge, one per improved target (a target whose in-edges span
// several chunks may be improved from each).  The current bitmap is read
// throughout and not cleared here (the step's last workgroup clears it).
template <int WT>
__device__ __forceinline__ void ss_pull(const SsArgs& A, int cur, int nxt, int rn, uint32_t gw,
                                        uint32_t nwv, Acc& acc, SsShared& sh) {
  const int lane = lane_id(), g = lane >> 4, j16 = lane & 15;
  const uint32_t nch = (uint32_t)min((long long)A.T.hdr->nchunks, (long long)A.T.cap_chunks);
  const uint32_t* fb = A.bm[cur];
  for (uint32_t c0 = gw * 4; c0 < nch; c0 += nwv * 4) {
    const uint32_t c = c0 + (uint32_t)g;
    const bool cok = c < nch;
    const int4 ch = cok ? A.T.chunks[c] : make_int4(0, 0, 0, 0);
    const int32_t v = ch.x, start = ch.y, len = ch.z;
    uint32_t best = inf_key<WT>();
    for (int32_t b = 0; __ballot(cok && b < len) != 0ull; b += 16) {
      if (cok && b + j16 < len) {
        const int32_t u = A.T.colidx[start + b + j16];
        if ((fb[u >> 5] >> (u & 31)) & 1u) {
          const uint32_t w = WT == kWUNIT ? 1u : A.T.w[start + b + j16];
          const uint32_t cand = relax_key<WT>(A.dist[u], w);
          if constexpr (WT == kWI32)
            if (cand == 0u) atomicOr(&A.ctl->negfloor, 1u);  // sum left the int32 range
          best = min(best, cand);
          acc.es += 1;
        }
      }
    }
    best = row16_min(best);
    bool imp[1] = {cok && j16 == 0 && v != A.src && best < A.dist[v]};
    const int32_t vv[1] = {v};
    const uint32_t cc[1] = {best};
    ss_enqueue<WT, 1, true>(A, imp, vv, cc, nxt, rn, acc, sh);
  }
}

// With skipping (tuning ss_skip): a frontier row whose distance another row
// lowered again during this step is already marked for the next step, where
// it is expanded with a value at least as low; expanding it now as well would
// only repeat that work.  Its current-bitmap word is still cleared.
// Position of the set bit of x that has r set bits below it (x has more than
// r set bits): a binary search on the population counts of its low halves.
__device__ __forceinline__ int nth_set_bit(uint32_t x, int r) {
  int pos = 0;
#pragma unroll
  for (int s = 16; s >= 1; s >>= 1) {
    const int lo = __popc(x & ((1u << s) - 1u));
    if (r >= lo) {
      r -= lo;
      x >>= s;
      pos += s;
    }
  }
  return pos;
}

__device__ __forceinline__ bool ss_skip_row(const SsArgs& A, int nxt, int32_t u) {
  return A.skip && ((ld_agent(&A.bm[nxt][u >> 5]) >> (u & 31)) & 1u);
}

// Returns true when the step was a pull step.
// PULL: pull steps may run (step launches with a reverse graph); the push-only
// instance keeps none of their code.
// The step's queue counts (lane, wave, workgroup-chunk tiers); read at the
// start of a step launch, or by the persistent kernel together with the
// previous step's update flag, right after the barrier that ends that step.
struct SsCounts {
  uint32_t w, g;  // wave-tier rows, workgroup-tier chunks
};

__device__ __forceinline__ SsCounts ss_counts(const SsArgs& A, uint32_t step) {
  const SsCtl* C = A.ctl;
  const int rc = step % kRot;
  // Entries past a queue's capacity were never written (the pushes that
  // counted them set the overflow flag, and the run reports -3), so the
  // counts are read up to the capacities only.
  return SsCounts{min(ld_agent(&C->cnt[rc][1].v), A.cap_v), min(ld_agent(&C->cnt[rc][2].v), A.cap_wg)};
}

template <int WT, bool PULL>
__device__ bool ss_step(const SsArgs& A, uint32_t step, uint32_t gb, uint32_t nb, Acc& acc,
                        SsShared& sh, SsCounts counts) {
  const int cur = step & 1, nxt = cur ^ 1;
  const int rc = step % kRot, rn = (step + 1) % kRot;
  SsCtl* C = A.ctl;
  const int lane = lane_id(), wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  // wave-major: consecutive work items go to different workgroups, so a
  // frontier smaller than the grid's waves is spread over every compute unit
  const uint32_t gw = (uint32_t)wave * nb + gb, nwv = nb * W;
  if (threadIdx.x == 0) {
    sh.nqw = 0u;
    sh.upd = 0u;
  }
  __syncthreads();
  const uint32_t nw = counts.w, ng = counts.g;
  const bool pull = PULL && A.T.hdr != nullptr && A.pull_min >= 0 &&
                    ld_agent64(&C->ctr.fedges[rc]) >= (unsigned long long)A.pull_min;
  if (pull) {
    if (gb == 0 && threadIdx.x == 0) acc.fe += ld_agent64(&C->ctr.frows[rc]);
    ss_pull<WT>(A, cur, nxt, rn, gw, nwv, acc, sh);
  } else {

    // workgroup tier: one chunk of one row per workgroup
    for (uint32_t i = gb; i < ng; i += nb) {
      const int4 r = ld_queue4(&A.qwg[cur][i]);
      const int32_t u = r.x, start = r.y;
      const uint32_t du = ld_agent(&A.dist[u]);
      const int32_t len = ss_skip_row(A, nxt, u) ? 0 : r.z;
      if (threadIdx.x == 0) {
        acc.es += (unsigned long long)len;
        if (r.w) acc.fe += 1;
      }
      const int32_t stride = (int32_t)blockDim.x;
      for (int32_t base = 0; base < len; base += stride * kUnroll) {
        int32_t e[kUnroll], v[kUnroll];
        bool ok[kUnroll], imp[kUnroll];
        uint32_t d[kUnroll], cand[kUnroll];
  #pragma unroll
        for (int j = 0; j < kUnroll; j++) {
          const int32_t k = base + j * stride + (int32_t)threadIdx.x;
          ok[j] = k < len;
          e[j] = start + k;
          d[j] = du;
        }
        ss_relax_pre<WT, kUnroll>(A, e, ok, d, imp, v, cand);
        ss_enqueue<WT, kUnroll, PULL>(A, imp, v, cand, nxt, rn, acc, sh);
      }
    }

    // wave tier: one wavefront per row
    for (uint32_t i = gw; i < nw; i += nwv) {
      const int32_t u = ld_queue(&A.qwave[cur][i]);
      const int32_t start = A.rowptr[u];
      const int32_t end = ss_skip_row(A, nxt, u) ? start : A.rowptr[u + 1];
      const uint32_t du = ld_agent(&A.dist[u]);
      if (lane == 0) {
        acc.fe += 1;
        acc.es += (unsigned long long)(end - start);
      }
      for (int32_t base = start; base < end; base += kWave * kUnroll) {
        int32_t e[kUnroll], v[kUnroll];
        bool ok[kUnroll], imp[kUnroll];
        uint32_t d[kUnroll], cand[kUnroll];
  #pragma unroll
        for (int j = 0; j < kUnroll; j++) {
          e[j] = base + j * kWave + lane;
          ok[j] = e[j] < end;
          d[j] = du;
        }
        ss_relax_pre<WT, kUnroll>(A, e, ok, d, imp, v, cand);
        ss_enqueue<WT, kUnroll, PULL>(A, imp, v, cand, nxt, rn, acc, sh);
      }
    }

    // lane tier: rows of at most t_lane edges are not queued.  Each wavefront
    // scans blocks of bw words of the step's bitmap (bw <= 64, halved until
    // there are at least as many blocks as wavefronts; the rows come in index
    // order), clears them, and takes their short rows 64 at a time; the rows'
    // edges are dealt out to the lanes through an LDS prefix sum of the row
    // lengths.  The scan clears every word, heavy rows' bits included: nothing
    // else reads this bitmap during a push step.
    int* l_incl = sh.stage + wave * 3 * kWave;
    int* l_base = l_incl + kWave;
    int* l_du = l_base + kWave;
    uint32_t* s_bits = sh.scan + wave * 2 * kWave;
    uint32_t* s_pre = s_bits + kWave;
    const int64_t nwords = ((int64_t)A.n + 31) / 32;
    int bw = kWave;
    while (bw > 1 && (nwords + bw - 1) / bw < (int64_t)nwv) bw >>= 1;
    const uint32_t nblk = (uint32_t)((nwords + bw - 1) / bw);
    for (uint32_t blk = gw; blk < nblk; blk += nwv) {
      const int64_t wi = (int64_t)blk * bw + lane;
      uint32_t bits = 0u;
      if (lane < bw && wi < nwords) {
        const uint32_t word = ld_agent(&A.bm[cur][wi]);
        if (word) {
          A.bm[cur][wi] = 0u;
          bits = word & ~A.hv[wi];
        }
      }
      const int cnt = __popc(bits);
      const int incl = wave_incl_scan(cnt);
      const int nrows = __shfl(incl, kWave - 1, kWave);
      if (nrows == 0) continue;
      s_bits[lane] = bits;
      s_pre[lane] = (uint32_t)(incl - cnt);
      wave_lds_sync();
      for (int r0 = 0; r0 < nrows; r0 += kWave) {
        const int j = r0 + lane;
        const bool has = j < nrows;
        int32_t start = 0, deg = 0;
        uint32_t du = 0;
        if (has) {
          int o = 0;  // the last word whose exclusive prefix is <= j (o + s <= 63 throughout)
  #pragma unroll
          for (int s = 32; s >= 1; s >>= 1)
            if (s_pre[o + s] <= (uint32_t)j) o += s;
          const int pos = nth_set_bit(s_bits[o], j - (int)s_pre[o]);
          const int32_t u = (int32_t)(((int64_t)blk * bw + o) * 32 + pos);
          start = A.rowptr[u];
          deg = A.rowptr[u + 1] - start;
          du = ld_agent(&A.dist[u]);
          const bool skipped = ss_skip_row(A, nxt, u);
          if (deg > 0) acc.fe += 1;  // a frontier row (rows without edges are not counted)
          if (skipped) deg = 0;
          acc.es += (unsigned long long)deg;
        }
        const int dincl = wave_incl_scan(deg);
        const int total = __shfl(dincl, kWave - 1, kWave);
        l_incl[lane] = dincl;
        l_base[lane] = start - (dincl - deg);
        l_du[lane] = (int)du;
        wave_lds_sync();
        for (int base = 0; base < total; base += kWave * kUnrollLane) {
          int32_t e[kUnrollLane], v[kUnrollLane];
          bool ok[kUnrollLane], imp[kUnrollLane];
          uint32_t d[kUnrollLane], cand[kUnrollLane];
  #pragma unroll
          for (int jj = 0; jj < kUnrollLane; jj++) {
            const int k = base + jj * kWave + lane;
            int owner = 0;  // first lane whose inclusive prefix exceeds k
  #pragma unroll
            for (int s = 32; s >= 1; s >>= 1)
              if (l_incl[owner + s - 1] <= k) owner += s;
            ok[jj] = k < total;
            e[jj] = l_base[owner] + k;
            d[jj] = (uint32_t)l_du[owner];
          }
          ss_relax_pre<WT, kUnrollLane>(A, e, ok, d, imp, v, cand);
          ss_enqueue<WT, kUnrollLane, PULL>(A, imp, v, cand, nxt, rn, acc, sh);
        }
        wave_lds_sync();
      }
    }

  }

  // publish the workgroup's next-frontier entries and ptr flag
  __syncthreads();
  const uint32_t n_w = min(sh.nqw, (uint32_t)kLdsQWave);
  if (threadIdx.x == 0) {
    if (n_w) sh.gbase_w = atomicAdd(&C->cnt[rn][1].v, n_w);
    if (sh.upd) st_agent(&C->upd[rn], 1u);
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < n_w; j += blockDim.x) {
    const uint32_t p = sh.gbase_w + j;
    if (p < A.cap_v) A.qwave[nxt][p] = sh.qw[j];
    else atomicOr(&C->overflow, 1u);
  }
  return pull;
}

__device__ __forceinline__ void ss_zero_rotation(SsCtl* C, uint32_t step) {
  const int rz = (step + 2) % kRot;
  for (int t = 0; t < 4; t++) st_agent(&C->cnt[rz][t].v, 0u);
  st_agent(&C->upd[rz], 0u);
  st_agent64(&C->ctr.fedges[rz], 0ull);
  st_agent64(&C->ctr.frows[rz], 0ull);
}

// All steps in one launch; a grid barrier separates the steps.  The grid must
// be co-resident: its size is what the compute units hold at once by the
// kernel's compiled resources (residency_of); should a barrier wait still give
// up, the run ends with status -2, reported to the caller.
template <int WT>
__global__ void __launch_bounds__(1024) ss_persistent_kernel(SsArgs A) {
  __shared__ SsShared sh;
  SsCtl* C = A.ctl;
  if (ld_agent(&C->done)) return;
  Acc acc;
  uint32_t epoch = 0;
  const uint32_t bar_base = ld_agent(&C->bar_base);
  uint32_t step = ld_agent(&C->step);
  SsCounts counts = ss_counts(A, step);
  int32_t status = 1;
  for (;;) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ss_zero_rotation(C, step);
    ss_step<WT, false>(A, step, blockIdx.x, gridDim.x, acc, sh, counts);
    if (!grid_sync(&C->bar.v, &C->abort, gridDim.x, bar_base, epoch, A.bar_ticks)) {
      status = -2;
      break;
    }
    // the step's update flag and the next step's queue counts, one round trip
    // (all were written before the barrier; nothing writes them during the
    // next step, whose pushes count in the rotation slot after)
    const uint32_t upd = ld_agent(&C->upd[(step + 1) % kRot]);
    counts = ss_counts(A, step + 1);
    step++;
    if (!upd) { status = 1; break; }
    if (step >= (uint32_t)A.n) { status = 0; break; }
  }
  SsCounters& S = C->ctr;
  flush_acc(acc, &S.fe, &S.es, &S.im, nullptr, nullptr);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st_agent(&C->step, step);
    st_agent_i(&C->converged, status);
    st_agent(&C->done, 1u);
    st_agent(&C->bar_base, bar_base + epoch * gridDim.x);
  }
}

// One step per launch; the last block to finish advances the step.
template <int WT, bool PULL>
__global__ void __launch_bounds__(1024) ss_step_kernel(SsArgs A) {
  __shared__ SsShared sh;
  SsCtl* C = A.ctl;
  if (ld_agent(&C->done)) return;
  const uint32_t step = ld_agent(&C->step);
  if (blockIdx.x == 0 && threadIdx.x == 0) ss_zero_rotation(C, step);
  Acc acc;
  const bool pulled = ss_step<WT, PULL>(A, step, blockIdx.x, gridDim.x, acc, sh, ss_counts(A, step));
  // counters, and the next frontier's out-edges and rows (its pull decision)
  SsCounters& S = C->ctr;
  flush_acc(acc, &S.fe, &S.es, &S.im, &S.fedges[(step + 1) % kRot], &S.frows[(step + 1) % kRot]);
  if (last_block_arrive(&C->arrive)) {
    // a pull step read the current bitmap throughout: clear it now, before it
    // serves as the next step's next-frontier bitmap
    if (pulled)
      for (int64_t i = threadIdx.x; i < ((int64_t)A.n + 31) / 32; i += blockDim.x)
        A.bm[step & 1][i] = 0u;
    if (threadIdx.x != 0) return;
    const uint32_t upd = ld_agent(&C->upd[(step + 1) % kRot]);
    const uint32_t ns = step + 1;
    st_agent(&C->step, ns);
    if (!upd) {
      st_agent_i(&C->converged, 1);
      st_agent(&C->done, 1u);
    } else if (ns >= (uint32_t)A.n) {
      st_agent_i(&C->converged, 0);
      st_agent(&C->done, 1u);
    }
  }
}

// ---------------------------------------------------------------------------
// small graphs: one workgroup runs the whole loop
//
// When the edge list is short, a step's work is a few microseconds and the
// grid barrier between steps (device-scope fences over the L2s of all XCDs)
// would dominate.  One workgroup then runs init, seeding and every step in a
// single launch, with a workgroup barrier between steps.  delta is one queue:
// each wavefront takes 64 rows and deals their edges out to its lanes through
// an LDS prefix sum of the row lengths (the lane tier's scheme, any degree).
// Data that one step writes and a later step reads (distances, the beta
// bitmaps, queue entries) go through device-scope atomics, as in the other
// kernels; the queue length and the ptr flag live in LDS.
// ---------------------------------------------------------------------------
struct SsSmallShared {
  int stage[kMaxWavesPerBlock * 3 * kWave];  // per wavefront: prefix, row base, distance
  uint32_t cnt_next, upd;
};

template <int WT>
__global__ void __launch_bounds__(1024) ss_small_kernel(SsArgs A, const int32_t* sources,
                                                        const int64_t* voff, int32_t count,
                                                        int32_t single, int32_t check_valid,
                                                        dawn_run_info* info) {
  __shared__ SsSmallShared sh;
  SsCtl* C = A.ctl;
  const int lane = lane_id(), wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  const int64_t n = A.n, nwords = (n + 31) / 32;
  uint32_t step = 0;
  int32_t status = 1;
  Acc acc;
  if (check_valid && ld_agent(&C->done)) {
    status = -1;
  } else {
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) A.dist[i] = inf_key<WT>();
    for (int64_t i = threadIdx.x; i < nwords; i += blockDim.x) {
      A.bm[0][i] = 0u;
      A.bm[1][i] = 0u;
    }
    if (threadIdx.x == 0) {
      sh.cnt_next = 0u;
      sh.upd = 0u;
      // the status words the report reads: the workspace may hold an earlier
      // run's (atomics, as the later reports are)
      atomicExch(&C->negfloor, 0u);
      atomicExch(&C->abort, 0u);
      atomicExch(&C->overflow, 0u);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // seeds: alpha = 0, queued once (a repeated seed finds its bit set)
    for (int j = threadIdx.x; j < count; j += blockDim.x) {
      int64_t s = sources ? (int64_t)sources[j] : (int64_t)single;
      if (voff) s += voff[j];
      st_agent(&A.dist[s], zero_key<WT>());
      const uint32_t bit = 1u << (s & 31);
      if (atomicOr(&A.bm[0][s >> 5], bit) & bit) continue;
      st_agent_i(&A.qlane[0][atomicAdd(&sh.cnt_next, 1u)], (int32_t)s);
    }
    __syncthreads();
    uint32_t cnt = sh.cnt_next;
    __syncthreads();
    if (threadIdx.x == 0) sh.cnt_next = 0u;
    __syncthreads();
    int* l_incl = sh.stage + wave * 3 * kWave;
    int* l_base = l_incl + kWave;
    int* l_du = l_base + kWave;
    for (;;) {
      const int cur = step & 1, nxt = cur ^ 1;
      for (uint32_t bi = wave; (uint64_t)bi * kWave < cnt; bi += W) {
        const uint32_t i = bi * kWave + lane;
        int32_t u = 0, start = 0, deg = 0;
        uint32_t du = 0;
        if (i < cnt) {
          u = ld_queue(&A.qlane[cur][i]);
          start = A.rowptr[u];
          deg = A.rowptr[u + 1] - start;
          du = ld_agent(&A.dist[u]);
          st_agent(&A.bm[cur][u >> 5], 0u);
          if (deg > 0) {
            acc.fe += 1;
            acc.es += (unsigned long long)deg;
          }
        }
        const int incl = wave_incl_scan(deg);
        const int total = __shfl(incl, kWave - 1, kWave);
        l_incl[lane] = incl;
        l_base[lane] = start - (incl - deg);
        l_du[lane] = (int)du;
        wave_lds_sync();
        for (int base = 0; base < total; base += kWave * kUnrollLane) {
          int32_t e[kUnrollLane], v[kUnrollLane];
          bool ok[kUnrollLane], imp[kUnrollLane];
          uint32_t d[kUnrollLane];
#pragma unroll
          for (int j = 0; j < kUnrollLane; j++) {
            const int k = base + j * kWave + lane;
            int owner = 0;  // first lane whose inclusive prefix exceeds k
#pragma unroll
            for (int s = 32; s >= 1; s >>= 1)
              if (l_incl[owner + s - 1] <= k) owner += s;
            ok[j] = k < total;
            e[j] = l_base[owner] + k;
            d[j] = (uint32_t)l_du[owner];
          }
          ss_relax_n<WT, kUnrollLane>(A, e, ok, d, imp, v);
#pragma unroll
          for (int j = 0; j < kUnrollLane; j++) {
            bool newv = false;
            if (imp[j]) {
              acc.im += 1;
              sh.upd = 1u;
              const uint32_t bit = 1u << (v[j] & 31);
              newv = (atomicOr(&A.bm[nxt][v[j] >> 5], bit) & bit) == 0u;
            }
            const unsigned long long b = __ballot(newv);
            if (b != 0ull) {
              const int leader = __ffsll((long long)b) - 1;
              uint32_t pos = 0;
              if (lane == leader) pos = atomicAdd(&sh.cnt_next, (uint32_t)__popcll(b));
              pos = __shfl(pos, leader, kWave) + lanes_below(b);
              if (newv) {
                if (pos < A.cap_v) st_agent_i(&A.qlane[nxt][pos], v[j]);
                else atomicOr(&C->overflow, 1u);
              }
            }
          }
        }
        wave_lds_sync();
      }
      __syncthreads();
      const uint32_t upd = sh.upd, cn = min(sh.cnt_next, A.cap_v);
      __syncthreads();
      if (threadIdx.x == 0) {
        sh.upd = 0u;
        sh.cnt_next = 0u;
      }
      __syncthreads();
      step++;
      cnt = cn;
      if (!upd) { status = 1; break; }
      if (step >= (uint32_t)A.n) { status = 0; break; }
    }
  }
  // counters, state and run info
  // thread i zeroes the counter that it then adds to (flush_acc: fe, es, im)
  SsCounters& S = C->ctr;
  if (threadIdx.x == 0) st_agent64(&S.fe, 0ull);
  if (threadIdx.x == 1) st_agent64(&S.es, 0ull);
  if (threadIdx.x == 2) st_agent64(&S.im, 0ull);
  flush_acc(acc, &S.fe, &S.es, &S.im, nullptr, nullptr);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (status != -1) {
      st_agent(&C->step, step);
      st_agent_i(&C->converged, status);
      st_agent(&C->done, 1u);
    }
    ss_report<WT>(C, info, A.latch);
  }
}

// ---------------------------------------------------------------------------
// tiny graphs: the whole state in LDS
//
// With n <= kTinyN the distances, both beta bitmaps and both frontier queues
// fit in one workgroup's LDS, so every step runs on LDS atomics (a few
// hundred cycles) instead of device-scope atomics; only the CSR is read from
// global memory.  The final distances are copied out once.
// ---------------------------------------------------------------------------
constexpr int kTinyN = 6144;

struct SsTinyShared {
  int stage[kMaxWavesPerBlock * 3 * kWave];
  uint32_t dist[kTinyN];
  uint16_t q[2][kTinyN];
  uint32_t bm[2][kTinyN / 32];
  uint32_t cnt_next, upd;
};

template <int WT>
__global__ void __launch_bounds__(1024) ss_tiny_kernel(SsArgs A, const int32_t* sources,
                                                       const int64_t* voff, int32_t count,
                                                       int32_t single, int32_t check_valid,
                                                       dawn_run_info* info) {
  __shared__ SsTinyShared sh;
  SsCtl* C = A.ctl;
  const int lane = lane_id(), wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  const int n = A.n, nwords = (n + 31) / 32;
  uint32_t step = 0;
  int32_t status = 1;
  Acc acc;
  if (check_valid && ld_agent(&C->done)) {
    status = -1;
  } else {
    for (int i = threadIdx.x; i < n; i += blockDim.x) sh.dist[i] = inf_key<WT>();
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) {
      sh.bm[0][i] = 0u;
      sh.bm[1][i] = 0u;
    }
    if (threadIdx.x == 0) {
      sh.cnt_next = 0u;
      sh.upd = 0u;
      // the status words the report reads: the workspace may hold an earlier
      // run's (atomics, as the later reports are)
      atomicExch(&C->negfloor, 0u);
      atomicExch(&C->abort, 0u);
      atomicExch(&C->overflow, 0u);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    __syncthreads();
    for (int j = threadIdx.x; j < count; j += blockDim.x) {
      int64_t s = sources ? (int64_t)sources[j] : (int64_t)single;
      if (voff) s += voff[j];
      sh.dist[s] = zero_key<WT>();
      const uint32_t bit = 1u << (s & 31);
      if (atomicOr(&sh.bm[0][s >> 5], bit) & bit) continue;
      sh.q[0][atomicAdd(&sh.cnt_next, 1u)] = (uint16_t)s;
    }
    __syncthreads();
    uint32_t cnt = sh.cnt_next;
    __syncthreads();
    if (threadIdx.x == 0) sh.cnt_next = 0u;
    __syncthreads();
    int* l_incl = sh.stage + wave * 3 * kWave;
    int* l_base = l_incl + kWave;
    int* l_du = l_base + kWave;
    for (;;) {
      const int cur = step & 1, nxt = cur ^ 1;
      for (uint32_t bi = wave; (uint64_t)bi * kWave < cnt; bi += W) {
        const uint32_t i = bi * kWave + lane;
        int32_t u = 0, start = 0, deg = 0;
        uint32_t du = 0;
        if (i < cnt) {
          u = sh.q[cur][i];
          start = A.rowptr[u];
          deg = A.rowptr[u + 1] - start;
          du = sh.dist[u];
          sh.bm[cur][u >> 5] = 0u;
          if (deg > 0) {
            acc.fe += 1;
            acc.es += (unsigned long long)deg;
          }
        }
        const int incl = wave_incl_scan(deg);
        const int total = __shfl(incl, kWave - 1, kWave);
        l_incl[lane] = incl;
        l_base[lane] = start - (incl - deg);
        l_du[lane] = (int)du;
        wave_lds_sync();
        for (int base = 0; base < total; base += kWave * kUnrollLane) {
          int32_t v[kUnrollLane];
          uint32_t cand[kUnrollLane];
          bool ok[kUnrollLane];
#pragma unroll
          for (int j = 0; j < kUnrollLane; j++) {
            const int k = base + j * kWave + lane;
            int owner = 0;  // first lane whose inclusive prefix exceeds k
#pragma unroll
            for (int s = 32; s >= 1; s >>= 1)
              if (l_incl[owner + s - 1] <= k) owner += s;
            ok[j] = k < total;
            v[j] = 0;
            cand[j] = 0u;
            if (ok[j]) {
              const int32_t e = l_base[owner] + k;
              uint32_t we = 1u;
              v[j] = A.colidx[e];
              if constexpr (WT != kWUNIT) we = A.w[e];
              cand[j] = relax_key<WT>((uint32_t)l_du[owner], we);
              if constexpr (WT == kWI32)
                if (cand[j] == 0u) atomicOr(&A.ctl->negfloor, 1u);  // sum left the int32 range
            }
          }
#pragma unroll
          for (int j = 0; j < kUnrollLane; j++) {
            bool newv = false;
            if (ok[j] && v[j] != A.src && cand[j] < sh.dist[v[j]] &&
                cand[j] < atomicMin(&sh.dist[v[j]], cand[j])) {
              acc.im += 1;
              sh.upd = 1u;
              const uint32_t bit = 1u << (v[j] & 31);
              newv = (atomicOr(&sh.bm[nxt][v[j] >> 5], bit) & bit) == 0u;
            }
            const unsigned long long b = __ballot(newv);
            if (b != 0ull) {
              const int leader = __ffsll((long long)b) - 1;
              uint32_t pos = 0;
              if (lane == leader) pos = atomicAdd(&sh.cnt_next, (uint32_t)__popcll(b));
              pos = __shfl(pos, leader, kWave) + lanes_below(b);
              if (newv) sh.q[nxt][pos] = (uint16_t)v[j];
            }
          }
        }
        wave_lds_sync();
      }
      __syncthreads();
      const uint32_t upd = sh.upd, cn = sh.cnt_next;
      __syncthreads();
      if (threadIdx.x == 0) {
        sh.upd = 0u;
        sh.cnt_next = 0u;
      }
      __syncthreads();
      step++;
      cnt = cn;
      if (!upd) { status = 1; break; }
      if (step >= (uint32_t)A.n) { status = 0; break; }
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) A.dist[i] = sh.dist[i];
  }
  // thread i zeroes the counter that it then adds to (flush_acc: fe, es, im)
  SsCounters& S = C->ctr;
  if (threadIdx.x == 0) st_agent64(&S.fe, 0ull);
  if (threadIdx.x == 1) st_agent64(&S.es, 0ull);
  if (threadIdx.x == 2) st_agent64(&S.im, 0ull);
  flush_acc(acc, &S.fe, &S.es, &S.im, nullptr, nullptr);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (status != -1) {
      st_agent(&C->step, step);
      st_agent_i(&C->converged, status);
      st_agent(&C->done, 1u);
    }
    ss_report<WT>(C, info, A.latch);
  }
}

// ---------------------------------------------------------------------------
// graphs that fit whole in LDS: edge-parallel steps
//
// With n <= kTinyN and m <= kLdsM a workgroup of kLdsThreads threads holds the
// whole run: the distances, the frontier bitmaps and the weights in LDS, and
// each thread's edges t, t + kLdsThreads, ... (at most kLdsEdges) in
// registers, as packed (source, target) ids.  A step then needs no queue: a thread
// relaxes each of its edges whose source's bit is set in the step's frontier
// bitmap.  Those are exactly the out-edges of the frontier, the relaxations
// Algorithm 2 makes, and every thread gets the same number of edges whatever
// the degrees.  A target lowered in the step gets its bit in the next bitmap.
// Three bitmaps and three update flags rotate, so one barrier per step
// suffices: step t reads bitmap t mod 3, sets bits in (t+1) mod 3 and clears
// (t+2) mod 3, which step t-1 read and step t+1 fills.
// ---------------------------------------------------------------------------
constexpr int kLdsThreads = 1024;
constexpr int kLdsEdges = 16;  // edges per thread
constexpr int kLdsM = kLdsThreads * kLdsEdges;
constexpr int kLdsRows = kTinyN / kLdsThreads;  // vertices per thread
constexpr int kLdsHalf = kLdsEdges / 2;

struct SsLdsShared {
  uint32_t dist[kTinyN];
  uint32_t bm[3][kTinyN / 32];
  uint32_t upd[3];
  uint16_t src[kLdsM];  // each edge's source, read once to fill the registers
  uint32_t w[kLdsM];
  unsigned long long part[kLdsThreads / kWave][3];
};

template <int WT>
__global__ void __launch_bounds__(kLdsThreads) ss_lds_kernel(SsArgs A, const int32_t* sources,
                                                             const int64_t* voff, int32_t count,
                                                             int32_t single, int32_t check_valid,
                                                             dawn_run_info* info) {
  __shared__ SsLdsShared sh;
  SsCtl* C = A.ctl;
  const int n = A.n, m = A.m, nwords = (n + 31) / 32, t = threadIdx.x;
  uint32_t step = 0;
  int32_t status = 1;
  Acc acc;
  if (check_valid && ld_agent(&C->done)) {
    status = -1;
  } else {
    if (t == 0) {
      // the status words the report reads: the workspace may hold an earlier
      // run's
      atomicExch(&C->negfloor, 0u);
      atomicExch(&C->abort, 0u);
      atomicExch(&C->overflow, 0u);
    }
    // this thread's edges and rows: every global load issued before any use
    uint32_t tv[kLdsEdges], we[kLdsEdges];
#pragma unroll
    for (int j = 0; j < kLdsEdges; j++) {
      const int e = t + j * kLdsThreads;
      tv[j] = e < m ? (uint32_t)A.colidx[e] : 0u;
      we[j] = (WT != kWUNIT && e < m) ? A.w[e] : 1u;
    }
#pragma unroll
    for (int j = 0; j < kLdsEdges; j++)
      if (t + j * kLdsThreads < m) sh.w[t + j * kLdsThreads] = we[j];
    int32_t ra[kLdsRows], rb[kLdsRows];
#pragma unroll
    for (int i = 0; i < kLdsRows; i++) {
      const int u = t + i * kLdsThreads;
      ra[i] = u < n ? A.rowptr[u] : 0;
      rb[i] = u < n ? A.rowptr[u + 1] : 0;
    }
#pragma unroll
    for (int i = 0; i < kLdsRows; i++) {
      const int u = t + i * kLdsThreads;
      if (u < n) {
        for (int32_t e = ra[i]; e < rb[i]; e++) sh.src[e] = (uint16_t)u;
        sh.dist[u] = inf_key<WT>();
      }
    }
    for (int i = t; i < nwords; i += kLdsThreads) {
      sh.bm[0][i] = 0u;
      sh.bm[1][i] = 0u;
      sh.bm[2][i] = 0u;
    }
    if (t < 3) sh.upd[t] = 0u;
    __syncthreads();
    // (source, target) of each edge packed in one register; bit j of `first`:
    // edge j is its row's first edge (counts the row once per step)
    uint32_t uv[kLdsEdges];
    uint32_t first = 0u;
#pragma unroll
    for (int j = 0; j < kLdsEdges; j++) {
      const int e = t + j * kLdsThreads;
      uv[j] = 0u;
      if (e < m) {
        const uint32_t u = sh.src[e];
        uv[j] = u | (tv[j] << 16);
        if (e == 0 || sh.src[e - 1] != u) first |= 1u << j;
      }
    }
    for (int j = t; j < count; j += kLdsThreads) {
      int64_t s = sources ? (int64_t)sources[j] : (int64_t)single;
      if (voff) s += voff[j];
      sh.dist[s] = zero_key<WT>();
      atomicOr(&sh.bm[0][s >> 5], 1u << (s & 31));
    }
    __syncthreads();
    for (;;) {
      const uint32_t* bc = sh.bm[step % 3];
      uint32_t* bn = sh.bm[(step + 1) % 3];
      bool upd = false;
      // Values derived from the edge ids (word indices, bit masks, LDS
      // addresses) are recomputed each step rather than kept in registers
      // across steps, which would not fit: the empty asm marks the ids as
      // changed here.
#pragma unroll
      for (int j = 0; j < kLdsEdges; j++) asm volatile("" : "+v"(uv[j]));
      // Frontier test of every edge, then the distances of the active ones,
      // then the atomics.  Every LDS read is unconditional (edges past m read
      // edge 0's slots, vertex 0), so a round's reads go out back to back and
      // are waited for once; a read under a branch would be waited for alone.
      uint32_t act = 0u;
      {
        uint32_t wd[kLdsEdges];
#pragma unroll
        for (int j = 0; j < kLdsEdges; j++) wd[j] = bc[(uv[j] & 0xFFFFu) >> 5];
#pragma unroll
        for (int j = 0; j < kLdsEdges; j++)
          act |= ((wd[j] >> (uv[j] & 31u)) & (t + j * kLdsThreads < m ? 1u : 0u)) << j;
      }
      // the active edges in halves of kLdsHalf (registers for their candidates)
#pragma unroll
      for (int h = 0; h < kLdsEdges; h += kLdsHalf) {
        if (!((act >> h) & ((1u << kLdsHalf) - 1u))) continue;
        uint32_t cand[kLdsHalf], dv[kLdsHalf];
#pragma unroll
        for (int i = 0; i < kLdsHalf; i++) {
          const int j = h + i, e = t + j * kLdsThreads;
          cand[i] = relax_key<WT>(sh.dist[uv[j] & 0xFFFFu], sh.w[e < m ? e : 0]);
          dv[i] = sh.dist[uv[j] >> 16];
        }
        uint32_t need = 0u;
#pragma unroll
        for (int i = 0; i < kLdsHalf; i++) {
          const int j = h + i;
          const uint32_t v = uv[j] >> 16;
          if ((act >> j) & 1u) {
            acc.es += 1;
            acc.fe += (first >> j) & 1u;
            if constexpr (WT == kWI32)
              if (cand[i] == 0u) atomicOr(&A.ctl->negfloor, 1u);  // sum left the int32 range
            if ((int32_t)v != A.src && cand[i] < dv[i]) need |= 1u << i;
          }
        }
        // returning atomics, all issued before any result is used
        uint32_t old[kLdsHalf];
#pragma unroll
        for (int i = 0; i < kLdsHalf; i++) {
          old[i] = 0u;
          if ((need >> i) & 1u) old[i] = atomicMin(&sh.dist[uv[h + i] >> 16], cand[i]);
        }
#pragma unroll
        for (int i = 0; i < kLdsHalf; i++) {
          const uint32_t v = uv[h + i] >> 16;
          if (((need >> i) & 1u) && cand[i] < old[i]) {
            acc.im += 1;
            upd = true;
            __hip_atomic_fetch_or(&bn[v >> 5], 1u << (v & 31), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
      for (int i = t; i < nwords; i += kLdsThreads) sh.bm[(step + 2) % 3][i] = 0u;
      if (t == 0) sh.upd[(step + 2) % 3] = 0u;
      if (upd) sh.upd[(step + 1) % 3] = 1u;
      __syncthreads();
      const uint32_t more = sh.upd[(step + 1) % 3];
      step++;
      if (!more) { status = 1; break; }
      if (step >= (uint32_t)n) { status = 0; break; }
    }
    for (int i = t; i < n; i += kLdsThreads) A.dist[i] = sh.dist[i];
  }
  // One workgroup owns the counters: they are summed in LDS and stored, not
  // added to, and the report is made from the values this workgroup holds.
  {
    const unsigned long long v0 = wave_sum64(acc.fe), v1 = wave_sum64(acc.es),
                             v2 = wave_sum64(acc.im);
    if (lane_id() == 0) {
      sh.part[t / kWave][0] = v0;
      sh.part[t / kWave][1] = v1;
      sh.part[t / kWave][2] = v2;
    }
  }
  // the int32 range flag is set by any thread's atomic
  if (WT == kWI32 || status == -1) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (t == 0) {
    unsigned long long fe = 0, es = 0, im = 0;
    for (int i = 0; i < kLdsThreads / kWave; i++) {
      fe += sh.part[i][0];
      es += sh.part[i][1];
      im += sh.part[i][2];
    }
    SsCounters& S = C->ctr;
    st_agent64(&S.fe, fe);
    st_agent64(&S.es, es);
    st_agent64(&S.im, im);
    if (status == -1) {
      // failed validation: report what the control words record
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      ss_report<WT>(C, info, A.latch);
    } else {
      if (WT == kWI32) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const uint32_t ab = ld_agent(&C->abort), ov = ld_agent(&C->overflow);
      const uint32_t nf = WT == kWI32 ? ld_agent(&C->negfloor) : 0u;
      st_agent(&C->step, step);
      st_agent_i(&C->converged, status);
      st_agent(&C->done, 1u);
      int32_t conv = run_status(status, ab, ov);
      if (WT == kWI32 && conv == 1 && nf) conv = 0;
      if (!info) {
        latch_status(A.latch, conv);
      } else {
        info->steps = (int32_t)step;
        info->converged = conv;
        info->frontier_entries = (int64_t)fe;
        info->edges_scanned = (int64_t)es;
        info->improvements = (int64_t)im;
        info->union_rows = (int64_t)fe;
        info->union_edges = (int64_t)es;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
SsLayout ss_layout(int64_t n, int64_t m) {
  SsLayout L{};
  Carver c;
  L.cap_v = (uint32_t)n;
  // at most m/65 rows exceed the smallest allowed t_wave (64), each cut into at
  // most deg/256 + 1 chunks (smallest allowed t_chunk 256)
  L.cap_wg = (uint32_t)(m / 65 + m / 256 + 2);
  L.nwords = (n + 31) / 32;
  L.ctl = c.take(sizeof(SsCtl));
  for (int i = 0; i < 2; i++) L.qwave[i] = c.take((size_t)n * 4);
  // The one-workgroup kernel's queues share the wave-tier queues' memory: a
  // one-workgroup run has no wave tier, and the other runs queue no short rows.
  for (int i = 0; i < 2; i++) L.qlane[i] = L.qwave[i];
  for (int i = 0; i < 2; i++) L.qwg[i] = c.take((size_t)L.cap_wg * 16);
  for (int i = 0; i < 2; i++) L.bm[i] = c.take((size_t)L.nwords * 4);
  L.hv = c.take((size_t)L.nwords * 4);
  L.total = c.off;
  return L;
}

Residency ss_persistent_residency(int threads) {
  if (threads <= 0) threads = 1024;
  return residency_of(ss_persistent_kernel<kWU32>, threads);
}

template <int WT>
static dawn_status ss_run_t(const SsArgs& A, const int32_t* rowptr, const int32_t* colidx,
                            const SsSeeds& seeds, const SsLayout& L, dawn_run_info* info,
                            hipStream_t stream, bool capture) {
  const Tuning& T = tuning();
  const DevInfo& di = dev_info();
  // mode 0 picks: one workgroup when m <= small_m; step launches first when
  // m >= step_min_m; otherwise the persistent launch alone.  Measured on
  // MI355X: on R-MAT scale 22 (67M edges) step launches of 512-thread
  // workgroups take a third of the time of the persistent launch; on
  // 16.7M-edge graphs (R-MAT scale 20, the 2048^2 grid) the persistent launch
  // of 1024-thread workgroups is faster.
  int mode = T.mode;
  if (mode == 0) mode = (int64_t)A.m <= (int64_t)T.small_m ? 3
                        : (int64_t)A.m >= (int64_t)T.step_min_m ? 1 : 2;
  const int threads = T.wg_threads > 0 ? T.wg_threads : mode == 1 ? 512 : 1024;
  const int fill_blocks = (int)std::min<int64_t>(4096, (A.n + 255) / 256 + 1);
  dawn_status st;
  if (mode == 3) {
    // one workgroup, one launch (after the optional device validation)
    if (T.validate) {
      hipLaunchKernelGGL(ss_fill_kernel<WT>, dim3(fill_blocks), dim3(256), 0, stream, A.dist,
                         (int64_t)A.n, A.bm[0], A.bm[1], L.nwords, A.ctl, nullptr, nullptr, 0);
      const int vb = (int)std::min<int64_t>(4096, ((int64_t)A.m + 255) / 256 + 1);
      hipLaunchKernelGGL(ss_validate_kernel, dim3(vb), dim3(256), 0, stream, rowptr, colidx, A.w,
                         A.n, A.m, (int32_t)(WT == kWF32), &A.ctl->done, &A.ctl->converged);
    }
    void* tk = capture ? nullptr : ktimer_begin(stream);
    if (A.n <= kTinyN && A.m <= kLdsM)  // its own workgroup size (the whole graph in registers)
      hipLaunchKernelGGL(ss_lds_kernel<WT>, dim3(1), dim3(kLdsThreads), 0, stream, A,
                         seeds.sources_dev, seeds.voff_dev, seeds.count, seeds.source,
                         (int32_t)(T.validate != 0), info);
    else if (A.n <= kTinyN)
      hipLaunchKernelGGL(ss_tiny_kernel<WT>, dim3(1), dim3(threads), 0, stream, A,
                         seeds.sources_dev, seeds.voff_dev, seeds.count, seeds.source,
                         (int32_t)(T.validate != 0), info);
    else
      hipLaunchKernelGGL(ss_small_kernel<WT>, dim3(1), dim3(threads), 0, stream, A,
                         seeds.sources_dev, seeds.voff_dev, seeds.count, seeds.source,
                         (int32_t)(T.validate != 0), info);
    ktimer_end(tk, stream, 1);
    if constexpr (WT == kWI32)
      hipLaunchKernelGGL(ss_decode_i32_kernel, dim3(fill_blocks), dim3(256), 0, stream, A.dist,
                         (int64_t)A.n);
    return hip_check(hipGetLastError(), "small-graph launch");
  }
  hipLaunchKernelGGL(ss_fill_kernel<WT>, dim3(fill_blocks), dim3(256), 0, stream, A.dist,
                     (int64_t)A.n, A.bm[0], A.bm[1], L.nwords, A.ctl, rowptr, A.hv, A.t_lane);
  if (T.validate) {
    const int vb = (int)std::min<int64_t>(4096, ((int64_t)A.m + 255) / 256 + 1);
    hipLaunchKernelGGL(ss_validate_kernel, dim3(vb), dim3(256), 0, stream, rowptr, colidx, A.w,
                       A.n, A.m, (int32_t)(WT == kWF32), &A.ctl->done, &A.ctl->converged);
  }
  hipLaunchKernelGGL(ss_seed_kernel<WT>, dim3(1), dim3(256), 0, stream, A, seeds.sources_dev,
                     seeds.voff_dev, seeds.count, seeds.source);
  if ((st = hip_check(hipGetLastError(), "init launch")) != DAWN_OK) return st;

  // Mode 1: `step_launches` step launches, then one persistent launch for
  // whatever steps remain.  Nothing waits on the host: every launch after the
  // run has ended returns at once, so the call is a fixed launch sequence that
  // a HIP graph can capture.
  if (mode == 1) {
    const int grid = T.grid > 0 ? T.grid : 4 * di.cus;
    auto stepk = A.pull_min >= 0 ? ss_step_kernel<WT, true> : ss_step_kernel<WT, false>;
    const int chunk = (int)std::min<int64_t>(T.step_launches, (int64_t)A.n + 1);
    void* tk = capture ? nullptr : ktimer_begin(stream);
    for (int s = 0; s < chunk; s++)
      hipLaunchKernelGGL(stepk, dim3(grid), dim3(threads), 0, stream, A);
    ktimer_end(tk, stream, chunk);
    if ((st = hip_check(hipGetLastError(), "step launches")) != DAWN_OK) return st;
  }
  {
    const Residency r = residency_of(ss_persistent_kernel<WT>, threads);
    int grid = r.grid;
    if (T.grid > 0 && T.grid < grid) grid = T.grid;
    if (T.ss_tail_grid > 0 && T.ss_tail_grid < grid) grid = T.ss_tail_grid;
    SsArgs a = A;
    a.pull_min = -1;  // pull steps need step launches (the last workgroup clears the bitmap)
    void* args[] = {&a};
    hipError_t e;
    void* tk = capture ? nullptr : ktimer_begin(stream);
    if (!capture && di.coop && T.coop) {
      e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&ss_persistent_kernel<WT>),
                                     dim3(grid), dim3(threads), args, 0, stream);
    } else {
      hipLaunchKernelGGL(ss_persistent_kernel<WT>, dim3(grid), dim3(threads), 0, stream, a);
      e = hipGetLastError();
    }
    ktimer_end(tk, stream, 1);
    if ((st = hip_check(e, "persistent launch")) != DAWN_OK) return st;
  }
  hipLaunchKernelGGL(ss_finalize_kernel<WT>, dim3(1), dim3(64), 0, stream, A.ctl, info, A.latch);
  if ((st = hip_check(hipGetLastError(), "finalize launch")) != DAWN_OK) return st;
  if constexpr (WT == kWI32) {
    hipLaunchKernelGGL(ss_decode_i32_kernel, dim3(fill_blocks), dim3(256), 0, stream, A.dist,
                       (int64_t)A.n);
    st = hip_check(hipGetLastError(), "decode launch");
  }
  return st;
}

dawn_status ss_run(const int32_t* rowptr, const int32_t* colidx, const void* w, int wt,
                   int32_t n, int32_t m, const SsSeeds& seeds, bool guard_source, void* dist,
                   void* ws, dawn_run_info* info, hipStream_t stream, bool capture,
                   const void* tgraph) {
  const Tuning& T = tuning();
  const SsLayout L = ss_layout(n, m);
  char* base = static_cast<char*>(ws);
  SsArgs A{};
  A.rowptr = rowptr;
  A.colidx = colidx;
  A.w = static_cast<const uint32_t*>(w);
  A.dist = static_cast<uint32_t*>(dist);
  A.n = n;
  A.m = m;
  A.src = guard_source ? seeds.source : -1;
  A.t_lane = T.t_lane;
  A.skip = T.ss_skip;
  A.T = TGraph{};
  A.pull_min = -1;
  if (tgraph && T.ss_pull <= 1000) {
    A.T = tgraph_view(tgraph, n, m);
    A.pull_min = (long long)m * T.ss_pull / 1000;
  }
  A.t_wave = T.t_wave;
  A.t_chunk = T.t_chunk;
  for (int i = 0; i < 2; i++) {
    A.qlane[i] = reinterpret_cast<int32_t*>(base + L.qlane[i]);
    A.qwave[i] = reinterpret_cast<int32_t*>(base + L.qwave[i]);
    A.qwg[i] = reinterpret_cast<int4*>(base + L.qwg[i]);
    A.bm[i] = reinterpret_cast<uint32_t*>(base + L.bm[i]);
  }
  A.hv = reinterpret_cast<uint32_t*>(base + L.hv);
  A.cap_v = L.cap_v;
  A.cap_wg = L.cap_wg;
  A.ctl = reinterpret_cast<SsCtl*>(base + L.ctl);
  A.bar_ticks = (unsigned long long)T.barrier_ms * kTicksPerMs;
  A.latch = dev_info().latch;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    capture = true;
  if (wt == kWF32) return ss_run_t<kWF32>(A, rowptr, colidx, seeds, L, info, stream, capture);
  if (wt == kWUNIT) return ss_run_t<kWUNIT>(A, rowptr, colidx, seeds, L, info, stream, capture);
  if (wt == kWI32) return ss_run_t<kWI32>(A, rowptr, colidx, seeds, L, info, stream, capture);
  return ss_run_t<kWU32>(A, rowptr, colidx, seeds, L, info, stream, capture);
}

}  // namespace dawn
