// govm_host.hpp -- host-side interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/dawn.h"
#include "govm_device.hpp"

namespace dawn {

struct Tuning {
  int32_t t_lane = 256;
  int32_t t_wave = 2048;
  int32_t t_chunk = 8192;
  int32_t wg_threads = 0;
  int32_t grid = 0;
  int32_t mode = 0;
  int32_t step_launches = 20;
  int32_t tile_k = 256;
  int32_t tile_t_wave = 64;
  int32_t tile_t_chunk = 256;
  int32_t validate = 0;
  int32_t coop = 0;
  int32_t tile_t_group = 8;
  int32_t tile_skip = 0;
  int32_t small_m = 131072;
  int32_t step_min_m = 1 << 25;
  int32_t tile_sparse = 8;
  int32_t tile_pull = 400;
  int32_t tile_pull_src = 16;
  int32_t ss_skip = 1;
  int32_t ss_pull = 1001;
  int32_t tile_step_launches = 16;
  int32_t barrier_ms = 4000;
  int32_t ss_tail_grid = 0;
};

Tuning& tuning();

struct DevInfo {
  int device = -1;
  int cus = 0;
  bool coop = false;
  uint32_t* latch = nullptr;  // this device's run-status latch (device address)
  void* noalloc = nullptr;    // this device's copy of the no-allocation scratch array
};
const DevInfo& dev_info();

// Run-status latch of the current device: runs that are given no
// dawn_run_info record here a status other than 1 (converged), for
// dawn_run_status.  latch[0] counts such runs, latch[1] holds the last status.
__device__ __forceinline__ void latch_status(uint32_t* latch, int32_t conv) {
  if (conv != 1 && latch) {
    atomicAdd(&latch[0], 1u);
    atomicExch(&latch[1], (uint32_t)conv);
  }
}

// Status of a run from its control words: 1 converged, 0 step cap, -1 failed
// validation or a bad source, -2 a persistent launch gave up at a grid
// barrier, -3 a frontier queue overflowed (cannot happen on a valid CSR).
__device__ __forceinline__ int32_t run_status(int32_t converged, uint32_t abort,
                                              uint32_t overflow) {
  if (abort) return -2;
  if (overflow) return -3;
  return converged;
}

// Workgroups of `threads` threads one compute unit holds at once for a kernel
// with these compiled resources (see resident_per_cu in dawn_api.hip).
int resident_per_cu(int vgprs, size_t lds_bytes, int threads);

// Persistent-grid sizing of a kernel: the smaller of the residency derived from
// its compiled resources and the runtime's occupancy figure, times the CUs.
struct Residency {
  int vgprs = 0, lds = 0, api_per_cu = 0, rule_per_cu = 0, per_cu = 0, grid = 0;
};
Residency residency_compute(const void* kernel, int threads, int api_per_cu);
// Cached per (kernel, threads, device): the queries run once, outside any
// graph capture that a later call may be part of.
const Residency& residency_cached(const void* kernel, int threads, int api_per_cu);
template <typename K>
Residency residency_of(K kernel, int threads) {
  const void* key = reinterpret_cast<const void*>(kernel);
  int api = -1;  // queried only on a cache miss
  const Residency* r = &residency_cached(key, threads, api);
  if (r->grid > 0) return *r;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&api, kernel, threads, 0) != hipSuccess)
    api = 0;
  return residency_cached(key, threads, api);
}

// Carves a workspace into 256-byte aligned pieces.
struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  }
};

// ----- single source ---------------------------------------------------------
struct SsLayout {
  size_t ctl, qlane[2], qwave[2], qwg[2], bm[2], hv, total;
  uint32_t cap_v, cap_wg;
  int64_t nwords;
};
SsLayout ss_layout(int64_t n, int64_t m);

// Seeds: either sources_dev[count] (+ voff_dev[count] if non-null) or the
// single host-side `source`.
struct SsSeeds {
  const int32_t* sources_dev = nullptr;
  const int64_t* voff_dev = nullptr;
  int32_t count = 1;
  int32_t source = 0;
};

// Enqueue a full single-source (or many-seed) GOVM run on `stream`; nothing
// waits on the host.  capture=true: never use a cooperative launch (HIP graph
// capture).  Without `info` the run's status goes to the run-status latch.
dawn_status ss_run(const int32_t* rowptr, const int32_t* colidx, const void* w, int wt,
                   int32_t n, int32_t m, const SsSeeds& seeds, bool guard_source, void* dist,
                   void* ws, dawn_run_info* info, hipStream_t stream, bool capture,
                   const void* tgraph = nullptr);

// ----- distance tile ---------------------------------------------------------
struct TileLayout {
  size_t ctl, info, D, mk[3], qgrp[3], qwave[3], qwg[3], fbm[2], vis, planes, total;
  bool unweighted;
  int32_t nplanes;
  uint32_t cap_v, cap_wg;
  int32_t K, nseg;
};
// unweighted: with the reached-pairs bitset of the hop-count tiles
TileLayout tile_layout(int64_t n, int64_t m, int32_t k, bool unweighted = false);

TileArgs tile_args(const int32_t* rowptr, const int32_t* colidx, const void* w, int32_t n,
                   int32_t m, const TileLayout& L, void* ws);
// Reset the whole tile (INF distances, empty masks and queues, zero control).
dawn_status tile_reset(const TileArgs& a, bool f32, hipStream_t stream);
// Seed columns [0, count) with sources_dev (msssp), on a freshly reset tile.
dawn_status tile_seed_all(const TileArgs& a, const int32_t* sources_dev, int32_t count,
                          bool validate, bool f32, hipStream_t stream);
// Admit one query into column col (between steps).
dawn_status tile_admit(const TileArgs& a, bool f32, int32_t col, int32_t source,
                       hipStream_t stream);
dawn_status tile_evict(const TileArgs& a, bool f32, int32_t col, hipStream_t stream);
// Run steps: persistent (all until done) or `max_steps` step launches.
dawn_status tile_steps(const TileArgs& a, bool f32, bool persistent, int32_t max_steps,
                       hipStream_t stream);
dawn_status tile_done_bits(const TileArgs& a, int32_t k, uint32_t* done_bits, hipStream_t stream);
dawn_status tile_store(const TileArgs& a, int32_t col0, int32_t count, void* out, int64_t ld,
                       hipStream_t stream);
dawn_status tile_read_col(const TileArgs& a, int32_t col, void* out, hipStream_t stream);
// The run summary into `info`, or, with info == NULL, the run's status into the
// run-status latch (when it is not 1).
dawn_status tile_info(const TileArgs& a, dawn_run_info* info, hipStream_t stream);
dawn_status tile_col_steps(const TileArgs& a, int32_t k, int32_t* out, hipStream_t stream);
// Hop-count tiles (unit weights): `max_steps` step launches; distances out
// of the bit planes into out[j * ld + v] for columns [col0, col0 + count).
dawn_status utile_steps(const TileArgs& a, int32_t max_steps, hipStream_t stream);
dawn_status utile_store(const TileArgs& a, int32_t col0, int32_t count, uint32_t* out, int64_t ld,
                        hipStream_t stream);

// Persistent grid sizing of the single-source, tile and hop-count-tile
// persistent kernels at `threads` per workgroup (0: the default).
Residency ss_persistent_residency(int threads);
Residency tile_persistent_residency(int threads);
Residency utile_persistent_residency(int threads);
// Hop-count tiles: the rest of the run (until no column is active, at most n
// steps) in one persistent launch (returns at once when the run has ended).
dawn_status utile_persistent(const TileArgs& a, hipStream_t stream);

// ----- measurement -------------------------------------------------------------
// Bracket a main launch with events when the kernel timer is on.
void* ktimer_begin(hipStream_t stream);
void ktimer_end(void* token, hipStream_t stream, int32_t launches);

// ----- reverse graph for pull steps ------------------------------------------
size_t tgraph_bytes(int64_t n, int64_t m);
size_t tgraph_build_bytes(int64_t n, int64_t m);
dawn_status tgraph_build(const int32_t* rowptr, const int32_t* colidx, const void* w, int64_t n,
                         int64_t m, void* buf, void* scratch, hipStream_t stream);
TGraph tgraph_view(const void* buf, int64_t n, int64_t m);

// ----- misc ------------------------------------------------------------------
// Host-side checks of a call's graph arguments and of the current tuning.
dawn_status check_graph(const int32_t* rowptr, const int32_t* colidx, const void* w,
                        dawn_wtype wt, int32_t n, int32_t m, bool need_w = true,
                        bool allow_i32 = false);
dawn_status set_error(dawn_status s, const char* fmt, ...);
dawn_status hip_check(hipError_t e, const char* what);

}  // namespace dawn
