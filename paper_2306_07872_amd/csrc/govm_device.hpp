// govm_device.hpp -- device-side building blocks of the GOVM kernels (gfx950).
//
// GOVM (Section 3.4, Algorithm 2) keeps three vectors: alpha (distances),
// delta (rows to expand this step) and beta (rows changed this step).  Here:
//   alpha -> the caller's distance array (uint32, or fp32 kept as its bits);
//   delta -> per-tier frontier queues of vertex ids (compacted, no dense scan);
//   beta  -> a bitmap that deduplicates the next frontier, whose first setter
//            of each bit appends the vertex to the next queues with a
//            wavefront ballot + prefix count (one atomic per wavefront);
//   ptr   -> a per-step "something improved" flag.
// Distances only decrease, so the relaxation is an atomic min; for
// non-negative fp32 values the bit patterns order like uint32, so one uint32
// atomic min serves both weight types.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dawn {

constexpr uint32_t kInfU32 = 0xFFFFFFFFu;
constexpr uint32_t kInfF32 = 0x7F800000u;  // +inf bits
constexpr int kWave = 64;
constexpr int kMaxWavesPerBlock = 16;      // 1024-thread workgroups
constexpr int kRot = 4;                    // rotation of per-step counters
constexpr int kSegMax = 8;                 // 8 x 64 = 512 tile columns

// Tile counters are striped: workgroup b adds to stripe b % kCtrStripes, each
// on its own 256-byte line; a reader sums the stripes.
constexpr int kCtrStripes = 32;

// A 32-bit control word alone on its cache line.
struct alignas(128) LineU32 {
  uint32_t v;
};

// Counters of a single-source run.  Every workgroup of a step adds to them
// (memory-side atomics): on one line of their own they measured faster than
// striped over 32 lines, and faster than beside the queue and step words.
struct alignas(256) SsCounters {
  unsigned long long fe, es, im;  // frontier rows, edges scanned, improvements
  // [step % 4]: out-edges and rows of the step's frontier, counted as the
  // previous step builds it (the pull decision of step launches)
  unsigned long long fedges[kRot], frows[kRot];
};

// Per-run control block in device memory (zeroed before a run).  Words that
// workgroups update concurrently sit on lines of their own, apart from the
// words every workgroup reads at the start of a step.
struct alignas(256) SsCtl {
  uint32_t step;              // next step to run
  uint32_t done;              // 1 once the loop has stopped
  int32_t converged;          // see dawn_run_info
  uint32_t abort;             // set when a barrier wait gives up
  uint32_t overflow;          // a queue capacity was exceeded (cannot happen on valid input)
  uint32_t bar_base;          // value of `bar` when the next persistent launch starts
  uint32_t negfloor;          // int32 weights: a path sum fell to or below INT32_MIN
  alignas(128) uint32_t upd[kRot];  // [step % 4]: any improvement during the previous step
  LineU32 bar;                // grid barrier arrivals (monotone within a launch)
  LineU32 arrive;             // last-block detection of step launches
  LineU32 cnt[kRot][4];       // [step % 4][tier]: lane, wave, workgroup-chunk records
  SsCounters ctr;
};

// Counters of a tile run.
struct alignas(256) CtrStripe {
  unsigned long long fe, es, im, sa, se;  // union rows, union edges, improvements,
                                          // per-source rows, per-source edges
  unsigned long long fedges[kRot];        // [step % 4]: out-edges of the step's frontier rows
  unsigned long long fpairs[kRot];        // [step % 4]: their (edge, active source) pairs
};

struct alignas(256) TileCtl {
  unsigned long long colact[kRot][kSegMax];  // [step % 4]: columns improved in step-1
  unsigned long long live[kSegMax];    // admitted columns
  uint32_t step, done;
  int32_t converged;
  uint32_t abort, overflow, bar_base;
  uint32_t cstep;                      // the step whose compaction ran last
  LineU32 bar;                         // grid barrier arrivals (monotone within a launch)
  LineU32 arrive;                      // last-block detection of step launches
  LineU32 cnt[kRot][4];                // [step % 4][tier]: group, wave, workgroup-chunk
  CtrStripe ctr[kCtrStripes];           // statistics, summed over the stripes
  int32_t colsteps[kSegMax * 64];
};

struct Acc {
  unsigned long long fe = 0, es = 0, im = 0, sa = 0, se = 0;
};

// ---------------------------------------------------------------------------
// arithmetic: d (+) w
// ---------------------------------------------------------------------------
template <bool F32>
__device__ __forceinline__ uint32_t relax_add(uint32_t d, uint32_t w) {
  if constexpr (F32) {
    // One IEEE fp32 add, round to nearest even (no FMA: nothing to contract).
    return __float_as_uint(__uint_as_float(d) + __uint_as_float(w));
  } else {
    const uint32_t s = d + w;
    return s < d ? kInfU32 : s;  // saturate
  }
}

// Weight modes of the single-source path.  Distances are kept as uint32 keys
// that order like the values they stand for: the uint32 value; the fp32 bit
// pattern (non-negative floats order like their bits); or, for int32 weights
// of either sign, the int32 value with its sign bit flipped.
// kWUNIT: every weight 1 and not read (hop counts, uint32 keys).
constexpr int kWU32 = 0, kWF32 = 1, kWI32 = 2, kWUNIT = 3;

template <int WT>
__device__ __forceinline__ constexpr uint32_t inf_key() {
  return WT == kWF32 ? 0x7F800000u : 0xFFFFFFFFu;  // int32: the key of INT32_MAX
}

template <int WT>
__device__ __forceinline__ constexpr uint32_t zero_key() {
  return WT == kWI32 ? 0x80000000u : 0u;
}

// d (+) w on keys.  uint32 and fp32 as relax_add.  int32: exact sum; a sum at
// or above INT32_MAX reads as INF (as uint32 sums saturate), a sum at or
// below INT32_MIN becomes key 0, which the caller reports (it cannot be a
// distance: finite distances lie strictly between the two).
template <int WT>
__device__ __forceinline__ uint32_t relax_key(uint32_t d, uint32_t w) {
  if constexpr (WT == kWUNIT) {
    return d + 1u;  // levels stay below n
  } else if constexpr (WT == kWI32) {
    if (d == 0xFFFFFFFFu) return d;
    const int64_t s = (int64_t)(int32_t)(d ^ 0x80000000u) + (int64_t)(int32_t)w;
    if (s >= (int64_t)INT32_MAX) return 0xFFFFFFFFu;
    if (s <= (int64_t)INT32_MIN) return 0u;
    return (uint32_t)(int32_t)s ^ 0x80000000u;
  } else {
    return relax_add<WT == kWF32>(d, w);
  }
}

template <bool F32>
__device__ __forceinline__ constexpr uint32_t inf_bits() {
  return F32 ? kInfF32 : kInfU32;
}

// ---------------------------------------------------------------------------
// memory-model helpers (agent scope = the whole device, all XCDs)
//
// Control state (step counter, done flag, per-step counts and column-activity
// words) is written by one kernel and read by later, often tiny, kernels that
// may run on any XCD.  Every such access goes through these agent-scope atomic
// loads and stores, so no read can be served from a cache line another XCD
// holds from before the write.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_agent64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent64(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_agent_i(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_i(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Queue entries are rewritten every step and often read at a wave- or
// block-uniform address, which a plain load may serve from the scalar cache;
// these loads always go to the coherent level.
__device__ __forceinline__ int32_t ld_queue(const int32_t* p) { return ld_agent_i(p); }
__device__ __forceinline__ int4 ld_queue4(const int4* p) {
  const int32_t* q = reinterpret_cast<const int32_t*>(p);
  return make_int4(ld_agent_i(q), ld_agent_i(q + 1), ld_agent_i(q + 2), ld_agent_i(q + 3));
}

// ---------------------------------------------------------------------------
// wavefront helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ int wave_incl_scan(int x) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  return x;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// Orders this wavefront's LDS writes before its own later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Append `val` for every lane with `pred` set: one atomic per wavefront
// reserves the range, each lane writes at base + (number of lanes below it).
// Must be reached by the whole wavefront.
__device__ __forceinline__ void wave_push(bool pred, int32_t val, int32_t* q, uint32_t* count,
                                          uint32_t cap, uint32_t* overflow) {
  const unsigned long long b = __ballot(pred);
  if (b == 0) return;
  const int leader = __ffsll((long long)b) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(count, (uint32_t)__popcll(b));
  base = __shfl(base, leader, kWave);
  if (pred) {
    const uint32_t pos = base + lanes_below(b);
    if (pos < cap) q[pos] = val;
    else atomicOr(overflow, 1u);
  }
}

// ---------------------------------------------------------------------------
// grid barrier for persistent launches
//
// Arrivals increment one monotone counter; a block waits until the counter
// reaches base + epoch * nblocks (`base` = the counter's value when the launch
// started, so the counter is never reset while a block may still be waiting).  Release/acquire fences at agent scope make every
// write before the barrier visible to every read after it, across the L2s of
// all XCDs.  The wait is bounded by wall-clock time (s_memrealtime runs at
// 100 MHz): past the bound the block raises `abort` and every block leaves, so
// the kernel always terminates.  The bound (`ticks`, tuning field barrier_ms)
// is a kernel argument; 0 gives up at the first wait that is not already
// satisfied, which lets a test force the failure path from the host.
// ---------------------------------------------------------------------------
constexpr unsigned long long kTicksPerMs = 100000ull;  // s_memrealtime: 100 MHz

__device__ __forceinline__ bool grid_sync(uint32_t* bar, uint32_t* abort_flag, uint32_t nblocks,
                                          uint32_t base, uint32_t& epoch,
                                          unsigned long long ticks) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    epoch += 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t target = base + epoch * nblocks;
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    int ok = 1;
    // every poll of the barrier word is a memory-side load that queues with
    // the arrivals on that address: poll every few hundred cycles and check
    // the abort flag only every 8th time (measured: a barrier of 256
    // workgroups takes 7.7 us instead of 19)
    for (uint32_t it = 0;; it++) {
      const uint32_t cur = ld_agent(bar);
      if ((int32_t)(cur - target) >= 0) break;
      if ((it & 7u) == 7u && ld_agent(abort_flag)) { ok = 0; break; }
      if (__builtin_amdgcn_s_memrealtime() - t0 > ticks) {
        st_agent(abort_flag, 1u);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Last-block detection for step launches: returns true in every thread of
// the workgroup that arrives last, once all other workgroups' writes are
// visible to it, and leaves the arrival word at zero for the next launch.
// Every thread must call it.  (Arrivals in two levels, over striped words,
// measured no faster: a step's workgroups do not finish all at once.)
__device__ __forceinline__ bool last_block_arrive(LineU32* arrive) {
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    int last = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (__hip_atomic_fetch_add(&arrive->v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
        gridDim.x - 1) {
      st_agent(&arrive->v, 0u);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      last = 1;
    }
    s_last = last;
  }
  __syncthreads();
  return s_last != 0;
}

// OR x into a word that only gains bits during a step, unless they are all
// there already: a memory-side load instead of a memory-side atomic, and in a
// dense step most workgroups find every bit set.
__device__ __forceinline__ void or_new_bits(unsigned long long* p, unsigned long long x) {
  if ((ld_agent64(p) & x) != x) atomicOr(p, x);
}

// Sum per-thread counters over the workgroup (wavefront sums, then LDS) and
// add each total to its counter with one atomic (null pointer: not counted;
// es2 / se2: second counters that also take the es / se totals).
// One add per workgroup rather than per wavefront: device-scope atomics on one
// address are serialised where they execute.  Every thread must call it.
__device__ __forceinline__ void flush_acc(const Acc& a, unsigned long long* fe,
                                          unsigned long long* es, unsigned long long* im,
                                          unsigned long long* sa, unsigned long long* se,
                                          unsigned long long* es2 = nullptr,
                                          unsigned long long* se2 = nullptr) {
  __shared__ unsigned long long part[1024 / kWave][5];
  const unsigned long long v0 = wave_sum64(a.fe), v1 = wave_sum64(a.es), v2 = wave_sum64(a.im);
  const unsigned long long v3 = wave_sum64(a.sa), v4 = wave_sum64(a.se);
  const int w = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
  __syncthreads();  // an earlier call's readers of `part` are done
  if (lane_id() == 0) {
    part[w][0] = v0;
    part[w][1] = v1;
    part[w][2] = v2;
    part[w][3] = v3;
    part[w][4] = v4;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int c = threadIdx.x == 5 ? 1 : threadIdx.x == 6 ? 4 : threadIdx.x;
    unsigned long long s = 0;
    for (int i = 0; i < nw; ++i) s += part[i][c];
    unsigned long long* dst = threadIdx.x == 0 ? fe
                              : threadIdx.x == 1 ? es
                              : threadIdx.x == 2 ? im
                              : threadIdx.x == 3 ? sa
                              : threadIdx.x == 4 ? se
                              : threadIdx.x == 5 ? es2
                                                 : se2;
    if (dst && s) atomicAdd(dst, s);
  }
}

// A control word read once per workgroup (thread 0, agent scope) and shared
// through LDS: an agent-scope load misses in the L2, and one per wavefront
// from a large grid queues on a single address.  Every thread must call it.
__device__ __forceinline__ uint32_t ld_agent_block(const uint32_t* p) {
  __shared__ uint32_t s_val;
  __syncthreads();  // an earlier call's readers are done
  if (threadIdx.x == 0) s_val = ld_agent(p);
  __syncthreads();
  return s_val;
}

// Sum of one counter over the stripes, in every lane (all lanes must be active).
template <typename Stripe>
__device__ __forceinline__ unsigned long long ctr_sum(const Stripe* ctr, size_t offset) {
  const int lane = lane_id();
  unsigned long long x = 0;
  if (lane < kCtrStripes)
    x = ld_agent64(reinterpret_cast<const unsigned long long*>(
        reinterpret_cast<const char*>(ctr + lane) + offset));
  return wave_sum64(x);
}

}  // namespace dawn

namespace dawn {

// The reverse graph for pull steps (built by tgraph_build): in-edge lists per
// target, cut into chunks of at most kPullChunk in-edges.
constexpr int kPullChunk = 1024;
struct TGraphHeader {
  uint32_t nchunks, pad;
};
struct TGraph {
  const TGraphHeader* hdr;
  const int32_t* rowptr;   // [n+1]
  const int32_t* colidx;   // [m] source vertex of each in-edge
  const uint32_t* w;       // [m]
  const int4* chunks;      // {target, first in-edge, count, split (target has several chunks)}
  int64_t cap_chunks;
};

// Kernel arguments of a single-source (or many-seed) GOVM run.
struct SsArgs {
  const int32_t* rowptr;
  const int32_t* colidx;
  const uint32_t* w;      // uint32 weights, or fp32 weights as bits
  uint32_t* dist;         // alpha
  int32_t n, m;
  int32_t src;            // the "index != source" guard; -1 with many seeds
  int32_t skip;           // skip expanding a row already lowered again in this step
  TGraph T;               // reverse graph for pull steps, or hdr == nullptr
  long long pull_min;     // pull when the frontier has >= this many out-edges; < 0: never
  int32_t t_lane, t_wave, t_chunk;
  int32_t* qlane[2];      // delta of one-workgroup runs [step % 2]
  int32_t* qwave[2];      // delta, wave tier
  int4* qwg[2];           // delta, workgroup tier: {row, first edge, edges, first chunk?}
  uint32_t* bm[2];        // beta dedup bitmaps [step % 2]
  uint32_t* hv;           // rows with more than t_lane edges (queued; shorter rows are scanned)
  uint32_t cap_v, cap_wg;
  SsCtl* ctl;
  unsigned long long bar_ticks;  // grid-barrier wait bound (persistent launches)
  uint32_t* latch;               // run-status latch of the device (runs without run info)
};


// Kernel arguments of a batched [n x K] distance-tile run (K = 64 * nseg).
struct TileArgs {
  const int32_t* rowptr;
  const int32_t* colidx;
  const uint32_t* w;
  uint32_t* D;            // [n][K] vertex-major: the K sources of a vertex are contiguous
  int32_t n, m, K, nseg;
  int32_t t_group, t_wave, t_chunk;
  int32_t skip;               // skip (row, source) pairs already lowered again this step
  int32_t sparse;             // rows with at most this many active sources: one edge per lane
  unsigned long long* mk[3];  // per-vertex active-source masks [step % 3][n][nseg]
  int32_t* qgrp[3];           // union frontier, 16-lane-group tier [step % 3]
  int32_t* qwave[3];          // union frontier, wave tier
  int4* qwg[3];               // union frontier, workgroup-chunk records
  uint32_t* fbm[2];           // union frontier as a bitmap [step % 2] (for pull steps)
  uint32_t cap_v, cap_wg;
  TileCtl* ctl;
  TGraph T;                   // reverse graph, or hdr == nullptr
  long long pull_min;         // pull steps when the frontier has >= this many out-edges; < 0: never
  long long pull_src;         // ... and >= this many active sources per frontier edge on average
  unsigned long long* vis;    // hop-count tiles: reached (vertex, source) pairs [n][nseg]; else null
  // hop-count tiles: the distances as bit planes, plane b = bit b of the step
  // that reached each pair, [nplanes][n][nseg]; D is null there
  unsigned long long* planes;
  int32_t nplanes;
  unsigned long long bar_ticks;  // grid-barrier wait bound (persistent launches)
  uint32_t* latch;               // run-status latch of the device (runs without run info)
};

}  // namespace dawn
