// govm_host.hpp -- host-side interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/dawn.h"
#include "govm_device.hpp"

namespace dawn {

struct Tuning {
  int32_t t_lane = 16;
  int32_t t_wave = 2048;
  int32_t t_chunk = 8192;
  int32_t wg_threads = 0;
  int32_t grid = 0;
  int32_t mode = 0;
  int32_t host_check = 32;
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
};

Tuning& tuning();

struct DevInfo {
  int device = -1;
  int cus = 0;
  bool coop = false;
};
const DevInfo& dev_info();

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
  size_t ctl, qlane[2], qwave[2], qwg[2], bm[2], total;
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

// Enqueue a full single-source (or many-seed) GOVM run on `stream`.
// capture=true: never use a cooperative launch (HIP graph capture).
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
dawn_status tile_info(const TileArgs& a, dawn_run_info* info, hipStream_t stream);
dawn_status tile_col_steps(const TileArgs& a, int32_t k, int32_t* out, hipStream_t stream);
// Hop-count tiles (unit weights): `max_steps` step launches; distances out
// of the bit planes into out[j * ld + v] for columns [col0, col0 + count).
dawn_status utile_steps(const TileArgs& a, int32_t max_steps, hipStream_t stream);
dawn_status utile_store(const TileArgs& a, int32_t col0, int32_t count, uint32_t* out, int64_t ld,
                        hipStream_t stream);

// Persistent grid sizes (workgroups per CU, total) at `threads` per workgroup.
void ss_persistent_occupancy(int threads, int* per_cu, int* grid);
void tile_persistent_occupancy(int threads, int* per_cu, int* grid);

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

// ----- host polling -----------------------------------------------------------
// A pinned host word for reading a device flag after a stream synchronisation.
// Pinned allocations cost far more than a step, so words come from a
// process-wide pool and go back to it (the pool lives until the process ends).
struct PinnedWord {
  uint32_t* p = nullptr;
  PinnedWord();
  ~PinnedWord();
  PinnedWord(const PinnedWord&) = delete;
  PinnedWord& operator=(const PinnedWord&) = delete;
};

// ----- misc ------------------------------------------------------------------
dawn_status set_error(dawn_status s, const char* fmt, ...);
dawn_status hip_check(hipError_t e, const char* what);

}  // namespace dawn
