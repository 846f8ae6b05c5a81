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
// are served by 16 lanes loading 16 bytes each from D[u] and D[v] -- two
// coalesced 256-byte reads per (edge, segment) -- and segments with no active
// source at u are skipped.  Improvements use atomicMin per element; the
// 16 lanes OR their improvement bits into one 64-bit word that is atomically
// OR-ed into v's next-step mask, and the first improvement of v in a step
// appends v to the next union frontier (bitmap dedup + wavefront ballot).
//
// Buffers rotate with the step: masks and queues over three slots (a slot is
// cleared one step after it was read), the union dedup bitmap over two,
// per-step counters and column-activity words over four.
#include <algorithm>

#include "govm_host.hpp"

namespace dawn {

// ---------------------------------------------------------------------------
// reset / seed / admit / evict
// ---------------------------------------------------------------------------
template <bool F32>
__global__ void tile_fill_kernel(TileArgs A, int64_t nwords) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nd4 = (int64_t)A.n * A.K / 4;
  const uint32_t inf = inf_bits<F32>();
  uint4* d4 = reinterpret_cast<uint4*>(A.D);
  for (int64_t i = tid; i < nd4; i += stride) d4[i] = make_uint4(inf, inf, inf, inf);
  const int64_t nm = (int64_t)A.n * A.nseg;
  for (int r = 0; r < 3; r++)
    for (int64_t i = tid; i < nm; i += stride) A.mk[r][i] = 0ull;
  for (int64_t i = tid; i < nwords; i += stride) {
    A.ubm[0][i] = 0u;
    A.ubm[1][i] = 0u;
  }
  if (blockIdx.x == 0) {
    uint32_t* c = reinterpret_cast<uint32_t*>(A.ctl);
    for (int i = threadIdx.x; i < (int)(sizeof(TileCtl) / 4); i += blockDim.x) c[i] = 0u;
  }
}

// Put source s into column col at step `t` (the next step to run).
__device__ void tile_put_source(const TileArgs& A, int32_t col, int32_t s, uint32_t t) {
  TileCtl* C = A.ctl;
  const int q = t % 3, rc = t % kRot, cur = t & 1;
  const int seg = col >> 6;
  const unsigned long long bit = 1ull << (col & 63);
  A.D[(size_t)s * A.K + col] = 0u;
  atomicOr(&A.mk[q][(size_t)s * A.nseg + seg], bit);
  atomicOr(&C->colact[rc][seg], bit);
  atomicOr(&C->live[seg], bit);
  st_agent_i(&C->colsteps[col], 0);
  const uint32_t vb = 1u << (s & 31);
  if (atomicOr(&A.ubm[cur][s >> 5], vb) & vb) return;  // already in the union frontier
  const int32_t start = A.rowptr[s], deg = A.rowptr[s + 1] - start;
  if (deg == 0) return;
  if (deg <= A.t_wave) {
    const uint32_t p = atomicAdd(&C->cnt[rc][1], 1u);
    if (p < A.cap_v) A.qwave[q][p] = s;
    else atomicOr(&C->overflow, 1u);
  } else {
    const uint32_t nch = (uint32_t)((deg + A.t_chunk - 1) / A.t_chunk);
    const uint32_t p = atomicAdd(&C->cnt[rc][2], nch);
    for (uint32_t c = 0; c < nch; c++) {
      const int32_t off = (int32_t)c * A.t_chunk;
      if (p + c < A.cap_wg) A.qwg[q][p + c] = make_int4(s, start + off, min(A.t_chunk, deg - off), c == 0);
      else atomicOr(&C->overflow, 1u);
    }
  }
}

__global__ void tile_seed_kernel(TileArgs A, const int32_t* sources, int32_t count) {
  if (ld_agent(&A.ctl->done)) return;  // validation failed
  // one thread per column; shared words are updated with atomics and the
  // union-bitmap test-and-set picks one thread to queue a repeated source
  for (int32_t j = threadIdx.x; j < count; j += blockDim.x) tile_put_source(A, j, sources[j], 0u);
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

// Cancel column col: drop its bit from every mask of the current frontier.
__global__ void tile_evict_kernel(TileArgs A, int32_t col) {
  TileCtl* C = A.ctl;
  const uint32_t t = ld_agent(&C->step);
  const int q = t % 3, rc = t % kRot;
  const int seg = col >> 6;
  const unsigned long long keep = ~(1ull << (col & 63));
  const uint32_t nw = ld_agent(&C->cnt[rc][1]), ng = ld_agent(&C->cnt[rc][2]);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)nw + ng; i += stride) {
    const int32_t u = i < nw ? ld_queue(&A.qwave[q][i]) : ld_queue(&A.qwg[q][i - nw].x);
    atomicAnd(&A.mk[q][(size_t)u * A.nseg + seg], keep);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    atomicAnd(&C->colact[rc][seg], keep);
    atomicAnd(&C->live[seg], keep);
  }
}

// ---------------------------------------------------------------------------
// one step
// ---------------------------------------------------------------------------
constexpr int kTileLdsQ = 1024;  // next union-frontier entries gathered per workgroup
constexpr int kTileUnroll = 2;   // (edge, segment) units in flight per 16-lane group

// Dynamic LDS of a tile launch: the distances of each wavefront's current row
// (K words per wavefront) and of the workgroup's current chunk row (K words).
__host__ __device__ inline size_t tile_dyn_lds(int K, int waves) {
  return (size_t)(waves + 1) * (size_t)K * 4u;
}

struct TileShared {
  unsigned long long rowmask[kMaxWavesPerBlock][kSegMax];  // masks of each wave's row
  unsigned long long blkmask[kSegMax];                     // masks of the workgroup's chunk
  unsigned long long colact[kSegMax];                      // columns improved (this workgroup)
  int32_t q[kTileLdsQ];
  uint32_t nq, gbase;
};

__device__ __forceinline__ void tile_block_push(bool pred, int32_t v, TileShared& sh,
                                                int32_t* gq, uint32_t* gcnt, uint32_t gcap,
                                                uint32_t* overflow) {
  const unsigned long long b = __ballot(pred);
  if (b == 0) return;
  const int leader = __ffsll((long long)b) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(&sh.nq, (uint32_t)__popcll(b));
  base = __shfl(base, leader, kWave);
  const uint32_t pos = base + lanes_below(b);
  const bool spill = pred && pos >= (uint32_t)kTileLdsQ;
  if (pred && !spill) sh.q[pos] = v;
  wave_push(spill, v, gq, gcnt, gcap, overflow);
}

template <bool F32>
__device__ __forceinline__ void tile_enqueue(const TileArgs& A, bool newv, int32_t v, int qn,
                                             int rn, TileShared& sh) {
  TileCtl* C = A.ctl;
  int32_t start = 0, deg = 0;
  if (newv) {
    start = A.rowptr[v];
    deg = A.rowptr[v + 1] - start;
  }
  const bool tw = newv && deg > 0 && deg <= A.t_wave;
  const bool tg = newv && deg > A.t_wave;
  tile_block_push(tw, v, sh, A.qwave[qn], &C->cnt[rn][1], A.cap_v, &C->overflow);
  if (tg) {
    const uint32_t nch = (uint32_t)((deg + A.t_chunk - 1) / A.t_chunk);
    const uint32_t base = atomicAdd(&C->cnt[rn][2], nch);
    for (uint32_t c = 0; c < nch; c++) {
      const int32_t off = (int32_t)c * A.t_chunk;
      if (base + c < A.cap_wg)
        A.qwg[qn][base + c] = make_int4(v, start + off, min(A.t_chunk, deg - off), c == 0);
      else
        atomicOr(&C->overflow, 1u);
    }
  }
}

__device__ __forceinline__ uint32_t elem4(const uint4& x, int i) {
  return i == 0 ? x.x : i == 1 ? x.y : i == 2 ? x.z : x.w;
}

// Process the (edge, active segment) units of edges [start, start+len) of row
// u, whose masks are in `rowmask` (LDS).  `ngroups` groups of 16 lanes
// cooperate (a wavefront: 4; a workgroup: blockDim/16); `gidx` is this lane's
// group, j16 its lane in the group.  The loop count is uniform over the
// cooperating lanes.  Each lane covers 4 consecutive sources of a segment.
template <bool F32>
__device__ __forceinline__ void tile_units(const TileArgs& A, int32_t start, int32_t len,
                                           const unsigned long long* rowmask,
                                           const uint32_t* rowdu, uint32_t actseg, int nact,
                                           int gidx, int ngroups, int qn, int rn, int nxt,
                                           Acc& acc, TileShared& sh) {
  constexpr int U = kTileUnroll;
  const int j16 = threadIdx.x & 15;
  const uint32_t units = (uint32_t)len * (uint32_t)nact;
  for (uint32_t ub = 0; ub < units; ub += (uint32_t)(ngroups * U)) {
    int32_t v[U];
    int sg[U];
    uint32_t w[U], bits[U];
#pragma unroll
    for (int i = 0; i < U; i++) {
      const uint32_t unit = ub + (uint32_t)(i * ngroups + gidx);
      v[i] = 0;
      sg[i] = 0;
      w[i] = 0u;
      bits[i] = 0u;
      if (unit < units) {
        const uint32_t eo = unit / (uint32_t)nact;
        uint32_t si = unit - eo * (uint32_t)nact;
        uint32_t am = actseg;
        while (si--) am &= am - 1u;
        sg[i] = __ffs(am) - 1;
        const int32_t e = start + (int32_t)eo;
        v[i] = A.colidx[e];
        w[i] = A.w[e];
        bits[i] = (uint32_t)(rowmask[sg[i]] >> (4 * j16)) & 0xFu;
      }
    }
    uint4 du[U], dv[U];
#pragma unroll
    for (int i = 0; i < U; i++) {
      if (bits[i]) {
        const int col = sg[i] * 64 + 4 * j16;
        du[i] = *reinterpret_cast<const uint4*>(rowdu + col);
        dv[i] = *reinterpret_cast<const uint4*>(A.D + (size_t)v[i] * A.K + col);
      } else {
        du[i] = make_uint4(0u, 0u, 0u, 0u);
        dv[i] = du[i];
      }
    }
    uint32_t imp[U];
#pragma unroll
    for (int i = 0; i < U; i++) {
      imp[i] = 0u;
      const size_t ov = (size_t)v[i] * A.K + sg[i] * 64 + 4 * j16;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        if ((bits[i] >> t) & 1u) {
          const uint32_t c = relax_add<F32>(elem4(du[i], t), w[i]);
          if (c < elem4(dv[i], t) && c < atomicMin(&A.D[ov + t], c)) imp[i] |= 1u << t;
        }
      }
    }
    bool newv[U];
#pragma unroll
    for (int i = 0; i < U; i++) {
      unsigned long long x = (unsigned long long)imp[i] << (4 * j16);
      x |= __shfl_xor(x, 1, kWave);
      x |= __shfl_xor(x, 2, kWave);
      x |= __shfl_xor(x, 4, kWave);
      x |= __shfl_xor(x, 8, kWave);
      newv[i] = false;
      if (j16 == 0 && x != 0ull) {
        atomicOr(&A.mk[qn][(size_t)v[i] * A.nseg + sg[i]], x);
        atomicOr(&sh.colact[sg[i]], x);
        acc.im += (unsigned long long)__popcll(x);
        const uint32_t vb = 1u << (v[i] & 31);
        newv[i] = (atomicOr(&A.ubm[nxt][v[i] >> 5], vb) & vb) == 0u;
      }
    }
#pragma unroll
    for (int i = 0; i < U; i++) tile_enqueue<F32>(A, newv[i], v[i], qn, rn, sh);
  }
}

template <bool F32>
__device__ void tile_step(const TileArgs& A, uint32_t step, uint32_t gb, uint32_t nb, Acc& acc,
                          TileShared& sh, uint32_t* dyn) {
  const int q = step % 3, qn = (step + 1) % 3, qp = (step + 2) % 3;
  const int cur = step & 1, nxt = cur ^ 1;
  const int rc = step % kRot, rn = (step + 1) % kRot, rp = (step + 3) % kRot;
  TileCtl* C = A.ctl;
  const int lane = lane_id(), wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  const uint32_t gw = gb * W + wave, nwv = nb * W;
  const int nseg = A.nseg;
  if (threadIdx.x < kSegMax) sh.colact[threadIdx.x] = 0ull;
  if (threadIdx.x == 0) sh.nq = 0u;
  __syncthreads();

  // (a) clear the masks of the previous step's frontier (read one step ago)
  {
    const uint32_t pw = ld_agent(&C->cnt[rp][1]), pg = ld_agent(&C->cnt[rp][2]);
    const uint32_t tot = pw + pg;
    for (uint32_t i = gb * blockDim.x + threadIdx.x; i < tot; i += nb * blockDim.x) {
      const int32_t u = i < pw ? ld_queue(&A.qwave[qp][i]) : ld_queue(&A.qwg[qp][i - pw].x);
      unsigned long long* mp = A.mk[qp] + (size_t)u * nseg;
      for (int s = 0; s < nseg; s++) mp[s] = 0ull;
    }
  }

  // (b) workgroup tier: one chunk of a long row per workgroup
  uint32_t* bdu = dyn + (size_t)W * A.K;
  const uint32_t ng = ld_agent(&C->cnt[rc][2]);
  for (uint32_t i = gb; i < ng; i += nb) {
    const int4 r = ld_queue4(&A.qwg[q][i]);
    __syncthreads();  // the previous chunk is done with blkmask / bdu
    if ((int)threadIdx.x < nseg) sh.blkmask[threadIdx.x] = A.mk[q][(size_t)r.x * nseg + threadIdx.x];
    for (int c = threadIdx.x; c < A.K; c += blockDim.x) bdu[c] = A.D[(size_t)r.x * A.K + c];
    __syncthreads();
    uint32_t act = 0u;
    int nsrc = 0;
    for (int s = 0; s < nseg; s++) {
      const unsigned long long x = sh.blkmask[s];
      if (x) {
        act |= 1u << s;
        nsrc += __popcll(x);
      }
    }
    if (threadIdx.x == 0) {
      acc.es += (unsigned long long)r.z;
      acc.se += (unsigned long long)r.z * (unsigned long long)nsrc;
      if (r.w) {
        A.ubm[cur][r.x >> 5] = 0u;
        acc.fe += 1;
        acc.sa += (unsigned long long)nsrc;
      }
    }
    tile_units<F32>(A, r.y, r.z, sh.blkmask, bdu, act, __popc(act), threadIdx.x >> 4,
                    blockDim.x >> 4, qn, rn, nxt, acc, sh);
  }

  // (c) wave tier: one wavefront per row
  const uint32_t nw = ld_agent(&C->cnt[rc][1]);
  unsigned long long* wmask = sh.rowmask[wave];
  uint32_t* wdu = dyn + (size_t)wave * A.K;
  for (uint32_t i = gw; i < nw; i += nwv) {
    const int32_t u = ld_queue(&A.qwave[q][i]);
    const int32_t start = A.rowptr[u], deg = A.rowptr[u + 1] - start;
    unsigned long long x = 0ull;
    if (lane < nseg) x = A.mk[q][(size_t)u * nseg + lane];
    const unsigned long long actb = __ballot(x != 0ull);
    const int cnt = __popcll(x);
    int nsrc = cnt;
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) nsrc += __shfl_xor(nsrc, off, kWave);
    nsrc = __shfl(nsrc, 0, kWave);
    if (lane < nseg) wmask[lane] = x;
    const uint32_t act = (uint32_t)actb & 0xFFu;
    for (int sgm = 0; sgm < nseg; sgm++)
      if ((act >> sgm) & 1u) wdu[sgm * 64 + lane] = A.D[(size_t)u * A.K + sgm * 64 + lane];
    wave_lds_sync();
    if (lane == 0) {
      A.ubm[cur][u >> 5] = 0u;
      acc.fe += 1;
      acc.es += (unsigned long long)deg;
      acc.sa += (unsigned long long)nsrc;
      acc.se += (unsigned long long)deg * (unsigned long long)nsrc;
    }
    tile_units<F32>(A, start, deg, wmask, wdu, act, __popc(act), lane >> 4, kWave / 16, qn, rn,
                    nxt, acc, sh);
    wave_lds_sync();
  }

  // (d) publish the workgroup's next-frontier entries and column activity
  __syncthreads();
  const uint32_t n_q = min(sh.nq, (uint32_t)kTileLdsQ);
  if (threadIdx.x == 0 && n_q) sh.gbase = atomicAdd(&C->cnt[rn][1], n_q);
  if ((int)threadIdx.x < nseg && sh.colact[threadIdx.x])
    atomicOr(&C->colact[rn][threadIdx.x], sh.colact[threadIdx.x]);
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < n_q; j += blockDim.x) {
    const uint32_t p = sh.gbase + j;
    if (p < A.cap_v) A.qwave[qn][p] = sh.q[j];
    else atomicOr(&C->overflow, 1u);
  }
}

__device__ __forceinline__ void tile_step_prologue(TileCtl* C, uint32_t step, int K) {
  // zero the counters two steps ahead and count this step for active columns
  if (blockIdx.x == 0) {
    const int rz = (step + 2) % kRot, rc = step % kRot;
    if (threadIdx.x < 4) st_agent(&C->cnt[rz][threadIdx.x], 0u);
    if (threadIdx.x < kSegMax) st_agent64(&C->colact[rz][threadIdx.x], 0ull);
    for (int j = threadIdx.x; j < K; j += blockDim.x)
      if ((ld_agent64(&C->colact[rc][j >> 6]) >> (j & 63)) & 1ull)
        st_agent_i(&C->colsteps[j], ld_agent_i(&C->colsteps[j]) + 1);
  }
}

__device__ __forceinline__ bool any_active(const TileCtl* C, int rn, int nseg) {
  unsigned long long a = 0ull;
  for (int s = 0; s < nseg; s++) a |= ld_agent64(&C->colact[rn][s]);
  return a != 0ull;
}

// All steps (up to max_steps, and at most n when cap_n) in one launch with a
// grid barrier between steps.
template <bool F32>
__global__ void __launch_bounds__(1024) tile_persistent_kernel(TileArgs A, int32_t max_steps,
                                                               int32_t cap_n) {
  __shared__ TileShared sh;
  extern __shared__ uint32_t tile_dyn[];
  TileCtl* C = A.ctl;
  if (ld_agent(&C->done)) return;
  Acc acc;
  uint32_t epoch = 0;
  const uint32_t bar_base = ld_agent(&C->bar_base);
  uint32_t step = ld_agent(&C->step);
  const uint32_t stop = step + (uint32_t)max_steps;
  int32_t status = 1;
  bool finished = false;
  for (;;) {
    tile_step_prologue(C, step, A.K);
    tile_step<F32>(A, step, blockIdx.x, gridDim.x, acc, sh, tile_dyn);
    if (!grid_sync(&C->bar, &C->abort, gridDim.x, bar_base, epoch)) {
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
  flush_acc(acc, &C->fe, &C->es, &C->im, &C->sa, &C->se);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st_agent(&C->step, step);
    st_agent(&C->bar_base, bar_base + epoch * gridDim.x);
    if (finished) {
      st_agent_i(&C->converged, status);
      st_agent(&C->done, 1u);
    }
  }
}

// One step per launch; the last block advances the step.
template <bool F32>
__global__ void __launch_bounds__(1024) tile_step_kernel(TileArgs A, int32_t cap_n) {
  __shared__ TileShared sh;
  extern __shared__ uint32_t tile_dyn[];
  TileCtl* C = A.ctl;
  if (ld_agent(&C->done)) return;
  const uint32_t step = ld_agent(&C->step);
  tile_step_prologue(C, step, A.K);
  Acc acc;
  tile_step<F32>(A, step, blockIdx.x, gridDim.x, acc, sh, tile_dyn);
  flush_acc(acc, &C->fe, &C->es, &C->im, &C->sa, &C->se);
  if (last_block_done(&C->blocks_done)) {
    st_agent(&C->blocks_done, 0u);
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

// ---------------------------------------------------------------------------
// outputs
// ---------------------------------------------------------------------------

// out[(j) * ld + v] = D[v][col0 + j] for j < count: 64 x 64 tiles through LDS so
// both the read (rows of D) and the write (rows of out) are contiguous.
__global__ void tile_store_kernel(const uint32_t* D, int32_t n, int32_t K, int32_t col0,
                                  int32_t count, uint32_t* out, int64_t ld) {
  __shared__ uint32_t t[64][65];
  const int64_t v0 = (int64_t)blockIdx.x * 64;
  const int32_t c0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 256 threads: 4 rows at a time
  for (int r = ty; r < 64; r += 4) {
    const int64_t v = v0 + r;
    const int32_t c = c0 + tx;
    t[r][tx] = (v < n && c < count) ? D[(size_t)v * K + col0 + c] : 0u;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int32_t c = c0 + r;
    const int64_t v = v0 + tx;
    if (c < count && v < n) out[(size_t)c * ld + v] = t[tx][r];
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

__global__ void tile_info_kernel(const TileCtl* C, int32_t K, dawn_run_info* info) {
  __shared__ int32_t s_max;
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  int32_t mx = 0;
  for (int j = threadIdx.x; j < K; j += blockDim.x) mx = max(mx, ld_agent_i(&C->colsteps[j]));
  atomicMax(&s_max, mx);
  __syncthreads();
  if (threadIdx.x != 0) return;
  int32_t conv = ld_agent_i(&C->converged);
  if (ld_agent(&C->abort)) conv = -2;
  info->steps = s_max;
  info->converged = conv;
  info->frontier_entries = (int64_t)ld_agent64(&C->sa);
  info->edges_scanned = (int64_t)ld_agent64(&C->se);
  info->improvements = (int64_t)ld_agent64(&C->im);
  info->union_rows = (int64_t)ld_agent64(&C->fe);
  info->union_edges = (int64_t)ld_agent64(&C->es);
}

__global__ void tile_col_steps_kernel(const TileCtl* C, int32_t k, int32_t* out) {
  for (int j = threadIdx.x; j < k; j += blockDim.x) out[j] = ld_agent_i(&C->colsteps[j]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
TileLayout tile_layout(int64_t n, int64_t m, int32_t k) {
  TileLayout L{};
  Carver c;
  L.nseg = (k + 63) / 64;
  L.K = L.nseg * 64;
  L.cap_v = (uint32_t)n;
  // rows above the smallest allowed threshold (32), each in at most deg/64 + 1
  // chunks (smallest allowed chunk 64)
  L.cap_wg = (uint32_t)(m / 33 + m / 64 + 2);
  L.nwords = (n + 31) / 32;
  L.ctl = c.take(sizeof(TileCtl));
  L.info = c.take(sizeof(dawn_run_info));
  L.D = c.take((size_t)n * L.K * 4);
  for (int i = 0; i < 3; i++) L.mk[i] = c.take((size_t)n * L.nseg * 8);
  for (int i = 0; i < 3; i++) L.qwave[i] = c.take((size_t)n * 4);
  for (int i = 0; i < 3; i++) L.qwg[i] = c.take((size_t)L.cap_wg * 16);
  for (int i = 0; i < 2; i++) L.ubm[i] = c.take((size_t)L.nwords * 4);
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
  A.D = reinterpret_cast<uint32_t*>(base + L.D);
  A.n = n;
  A.m = m;
  A.K = L.K;
  A.nseg = L.nseg;
  A.t_wave = T.tile_t_wave;
  A.t_chunk = T.tile_t_chunk;
  for (int i = 0; i < 3; i++) {
    A.mk[i] = reinterpret_cast<unsigned long long*>(base + L.mk[i]);
    A.qwave[i] = reinterpret_cast<int32_t*>(base + L.qwave[i]);
    A.qwg[i] = reinterpret_cast<int4*>(base + L.qwg[i]);
  }
  for (int i = 0; i < 2; i++) A.ubm[i] = reinterpret_cast<uint32_t*>(base + L.ubm[i]);
  A.cap_v = L.cap_v;
  A.cap_wg = L.cap_wg;
  A.ctl = reinterpret_cast<TileCtl*>(base + L.ctl);
  return A;
}

static int grid_for(int64_t work, int threads) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (work + threads - 1) / threads));
}

dawn_status tile_reset(const TileArgs& a, bool f32, hipStream_t stream) {
  const int64_t nwords = ((int64_t)a.n + 31) / 32;
  const int g = grid_for((int64_t)a.n * a.K / 4, 256);
  if (f32) hipLaunchKernelGGL(tile_fill_kernel<true>, dim3(g), dim3(256), 0, stream, a, nwords);
  else hipLaunchKernelGGL(tile_fill_kernel<false>, dim3(g), dim3(256), 0, stream, a, nwords);
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

dawn_status tile_evict(const TileArgs& a, int32_t col, hipStream_t stream) {
  hipLaunchKernelGGL(tile_evict_kernel, dim3(grid_for(a.n, 256)), dim3(256), 0, stream, a, col);
  return hip_check(hipGetLastError(), "tile evict");
}

template <typename K>
static int persistent_grid_t(K kernel, int threads, int* per_cu_out = nullptr, size_t dyn = 0) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, dyn) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  // Measured on MI355X: the occupancy query reports twice the workgroups per CU
  // that are resident together (a 2048-workgroup grid of 256 threads never
  // completed its first barrier; 1024 did), so a persistent grid takes half.
  per_cu = std::max(1, per_cu / 2);
  if (per_cu_out) *per_cu_out = per_cu;
  return per_cu * dev_info().cus;
}

void tile_persistent_occupancy(int threads, int* per_cu, int* grid) {
  if (threads <= 0) threads = 256;
  *grid = persistent_grid_t(tile_persistent_kernel<false>, threads, per_cu,
                            tile_dyn_lds(256, threads / 64));
}

template <bool F32>
static dawn_status tile_steps_t(const TileArgs& a, bool persistent, int32_t max_steps,
                                hipStream_t stream) {
  const Tuning& T = tuning();
  const int threads = T.wg_threads > 0 ? T.wg_threads : 256;
  const int32_t cap_n = persistent ? 1 : 0;
  const size_t dyn = tile_dyn_lds(a.K, threads / 64);
  if (persistent) {
    int grid = persistent_grid_t(tile_persistent_kernel<F32>, threads, nullptr, dyn);
    if (T.grid > 0 && T.grid < grid) grid = T.grid;
    TileArgs aa = a;
    int32_t ms = max_steps, cn = cap_n;
    void* args[] = {&aa, &ms, &cn};
    hipError_t e;
    void* tk = ktimer_begin(stream);
    if (dev_info().coop && T.coop) {
      e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&tile_persistent_kernel<F32>),
                                     dim3(grid), dim3(threads), args, (unsigned)dyn, stream);
    } else {
      hipLaunchKernelGGL(tile_persistent_kernel<F32>, dim3(grid), dim3(threads), dyn, stream, aa,
                         ms, cn);
      e = hipGetLastError();
    }
    ktimer_end(tk, stream, 1);
    return hip_check(e, "tile persistent launch");
  }
  const int grid = T.grid > 0 ? T.grid : 16 * dev_info().cus;
  void* tk = ktimer_begin(stream);
  for (int s = 0; s < max_steps; s++)
    hipLaunchKernelGGL(tile_step_kernel<F32>, dim3(grid), dim3(threads), dyn, stream, a, 0);
  ktimer_end(tk, stream, max_steps);
  return hip_check(hipGetLastError(), "tile step launches");
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
  hipLaunchKernelGGL(tile_store_kernel, grid, dim3(256), 0, stream, a.D, a.n, a.K, col0, count,
                     static_cast<uint32_t*>(out), ld);
  return hip_check(hipGetLastError(), "tile store");
}

dawn_status tile_read_col(const TileArgs& a, int32_t col, void* out, hipStream_t stream) {
  hipLaunchKernelGGL(tile_read_col_kernel, dim3(grid_for(a.n, 256)), dim3(256), 0, stream, a.D,
                     a.n, a.K, col, static_cast<uint32_t*>(out));
  return hip_check(hipGetLastError(), "tile read");
}

dawn_status tile_info(const TileArgs& a, dawn_run_info* info, hipStream_t stream) {
  hipLaunchKernelGGL(tile_info_kernel, dim3(1), dim3(256), 0, stream, a.ctl, a.K, info);
  return hip_check(hipGetLastError(), "tile info");
}

dawn_status tile_col_steps(const TileArgs& a, int32_t k, int32_t* out, hipStream_t stream) {
  hipLaunchKernelGGL(tile_col_steps_kernel, dim3(1), dim3(256), 0, stream, a.ctl, k, out);
  return hip_check(hipGetLastError(), "tile steps");
}

}  // namespace dawn
