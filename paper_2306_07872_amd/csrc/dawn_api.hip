// dawn_api.hip -- the C ABI declared in include/dawn.h.
//
// Host-side work only: argument checks, workspace carving, launch sequencing,
// batch and tile-session bookkeeping.  Every distance is computed by the
// kernels in govm_sssp.hip and govm_tile.hip.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "govm_host.hpp"

namespace dawn {

// ---------------------------------------------------------------------------
// process state
// ---------------------------------------------------------------------------
static Tuning g_tuning;
Tuning& tuning() { return g_tuning; }

static thread_local char g_err[512] = "";

dawn_status set_error(dawn_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

dawn_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return DAWN_OK;
  return set_error(DAWN_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

static std::mutex g_dev_mu;
static DevInfo g_dev[64];

// Per-device run-status latch: [0] runs given no run info that ended with a
// status other than 1, [1] the last such status.  Each device holds its own
// copy of this array; host code reaches it only through the device address
// hipGetSymbolAddress returns with that device current (DevInfo::latch).
__device__ __align__(256) uint32_t g_run_latch[64];

// Workspace of dawn_sssp_noalloc: one copy per device, held by the loaded code
// object until the process ends.  Host code never names the array in a launch
// or copy; it uses the device address that hipGetSymbolAddress returned with
// that device current (DevInfo::noalloc).
static __device__ __align__(256) unsigned char g_noalloc_scratch[DAWN_NOALLOC_SCRATCH_BYTES];

const DevInfo& dev_info() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) d = 0;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  DevInfo& di = g_dev[d];
  if (di.device != d) {
    int cus = 0, coop = 0;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d);
    hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, d);
    di.cus = cus > 0 ? cus : 1;
    di.coop = coop != 0;
    void* p = nullptr;
    di.latch = hipGetSymbolAddress(&p, HIP_SYMBOL(g_run_latch)) == hipSuccess
                   ? static_cast<uint32_t*>(p) : nullptr;
    // The array's name is a host-side stand-in: kernels get this address.
    void* q = nullptr;
    di.noalloc = hipGetSymbolAddress(&q, HIP_SYMBOL(g_noalloc_scratch)) == hipSuccess ? q : nullptr;
    di.device = d;
  }
  return di;
}

// Residency rule of a gfx950 compute unit: 4 SIMDs, each with 512 VGPRs per
// lane for wave64 (allocated in granules of 8) and at most 8 waves, and 160 KiB
// of LDS shared by the CU's workgroups; a workgroup's waves are spread evenly
// over the 4 SIMDs.  At most 16 workgroups per CU are assumed.  SGPRs are not
// counted: every persistent kernel here is limited by its VGPRs first (the
// compiler's own occupancy figure for each is checked against this rule).
int resident_per_cu(int vgprs, size_t lds_bytes, int threads) {
  if (vgprs <= 0 || threads <= 0) return 0;
  const int waves = (threads + kWave - 1) / kWave;
  const int per_simd = (waves + 3) / 4;
  const int alloc = std::max(8, (vgprs + 7) / 8 * 8);
  const int waves_per_simd = std::min(8, 512 / alloc);
  const int by_regs = waves_per_simd / per_simd;
  const int by_lds = lds_bytes > 0 ? (int)((size_t)160 * 1024 / lds_bytes) : 16;
  return std::max(0, std::min(std::min(by_regs, by_lds), 16));
}

Residency residency_compute(const void* kernel, int threads, int api_per_cu) {
  Residency r;
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, kernel) == hipSuccess) {
    r.vgprs = fa.numRegs;
    r.lds = (int)fa.sharedSizeBytes;
  }
  r.api_per_cu = api_per_cu;
  r.rule_per_cu = resident_per_cu(r.vgprs, (size_t)r.lds, threads);
  int pc = r.rule_per_cu;
  if (api_per_cu > 0 && api_per_cu < pc) pc = api_per_cu;
  r.per_cu = pc < 1 ? 1 : pc;
  r.grid = r.per_cu * dev_info().cus;
  return r;
}

static std::mutex g_res_mu;
static std::map<std::tuple<const void*, int, int>, Residency> g_res;

// api_per_cu < 0: look up only (a miss returns an entry with grid 0).
const Residency& residency_cached(const void* kernel, int threads, int api_per_cu) {
  static const Residency miss{};
  const int dev = dev_info().device;
  std::lock_guard<std::mutex> lk(g_res_mu);
  auto key = std::make_tuple(kernel, threads, dev);
  auto it = g_res.find(key);
  if (it != g_res.end()) return it->second;
  if (api_per_cu < 0) return miss;
  return g_res.emplace(key, residency_compute(kernel, threads, api_per_cu)).first->second;
}

static bool tuning_ok(const Tuning& t) {
  return t.t_lane >= 1 && t.t_lane <= 4096 && t.t_wave >= std::max(64, t.t_lane) &&
         t.t_wave <= 65536 && t.t_chunk >= 256 && t.t_chunk <= (1 << 20) &&
         (t.wg_threads == 0 || t.wg_threads == 256 || t.wg_threads == 512 || t.wg_threads == 1024) && t.grid >= 0 &&
         t.grid <= (1 << 20) && t.mode >= 0 && t.mode <= 2 && t.step_launches >= 0 &&
         t.step_launches <= 4096 && t.tile_k >= 64 && t.tile_k <= DAWN_TILE_K_MAX &&
         t.tile_k % 64 == 0 && t.tile_t_wave >= 32 && t.tile_t_wave <= 65536 &&
         t.tile_t_chunk >= 64 && t.tile_t_chunk <= 65536 && (t.validate == 0 || t.validate == 1) &&
         (t.coop == 0 || t.coop == 1) && t.tile_t_group >= 0 && t.tile_t_group <= 64 &&
         t.tile_t_group < t.tile_t_wave && (t.tile_skip == 0 || t.tile_skip == 1) &&
         t.small_m >= 0 && t.step_min_m >= 0 && t.tile_sparse >= 0 && t.tile_sparse <= 512 &&
         t.tile_pull >= 0 && t.tile_pull <= 1001 && t.tile_pull_src >= 0 &&
         t.tile_pull_src <= 512 && (t.ss_skip == 0 || t.ss_skip == 1) && t.ss_pull >= 0 &&
         t.ss_pull <= 1001 && t.tile_step_launches >= 0 && t.tile_step_launches <= 4096 &&
         t.ss_tail_grid >= 0 && t.ss_tail_grid <= (1 << 20) &&
         t.barrier_ms >= 0 && t.barrier_ms <= 600000;
}

dawn_status check_graph(const int32_t* rowptr, const int32_t* colidx, const void* w,
                        dawn_wtype wt, int32_t n, int32_t m, bool need_w, bool allow_i32) {
  if (n < 1) return set_error(DAWN_E_INVALID, "n must be >= 1 (got %d)", n);
  if (n == INT32_MAX) return set_error(DAWN_E_INVALID, "n too large");
  if (m < 0) return set_error(DAWN_E_INVALID, "m must be >= 0 (got %d)", m);
  if (!rowptr) return set_error(DAWN_E_INVALID, "rowptr is null");
  if (m > 0 && !colidx) return set_error(DAWN_E_INVALID, "colidx is null");
  if (wt != DAWN_W_U32 && wt != DAWN_W_F32 && wt != DAWN_W_I32 && wt != DAWN_W_UNIT)
    return set_error(DAWN_E_INVALID, "unknown wtype");
  if (m > 0 && need_w && wt != DAWN_W_UNIT && !w) return set_error(DAWN_E_INVALID, "weights are null");
  if (wt == DAWN_W_I32 && !allow_i32)
    return set_error(DAWN_E_UNSUPPORTED, "int32 weights: single-source calls only");
  if (!tuning_ok(g_tuning)) return set_error(DAWN_E_INVALID, "tuning out of range");
  return DAWN_OK;
}

// Scratch owned for the duration of one call: hipMallocAsync / hipFreeAsync
// on the call's stream.
struct StreamScratch {
  void* p = nullptr;
  hipStream_t s;
  explicit StreamScratch(hipStream_t st) : s(st) {}
  dawn_status alloc(size_t bytes) {
    return hip_check(hipMallocAsync(&p, std::max<size_t>(bytes, 256), s), "hipMallocAsync");
  }
  ~StreamScratch() {
    if (p) hipFreeAsync(p, s);
  }
};

// ---------------------------------------------------------------------------
// kernel timer
// ---------------------------------------------------------------------------
struct TimedLaunch {
  hipEvent_t a, b;
  int32_t launches;
};
static std::mutex g_timer_mu;
static bool g_timer_on = false;
static std::vector<TimedLaunch> g_timed;

void* ktimer_begin(hipStream_t stream) {
  {
    std::lock_guard<std::mutex> lk(g_timer_mu);
    if (!g_timer_on) return nullptr;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return nullptr;  // a captured launch sequence carries no timing events
  TimedLaunch* t = new TimedLaunch();
  if (hipEventCreate(&t->a) != hipSuccess || hipEventCreate(&t->b) != hipSuccess) {
    delete t;
    return nullptr;
  }
  hipEventRecord(t->a, stream);
  return t;
}

void ktimer_end(void* token, hipStream_t stream, int32_t launches) {
  if (!token) return;
  TimedLaunch* t = static_cast<TimedLaunch*>(token);
  hipEventRecord(t->b, stream);
  t->launches = launches;
  std::lock_guard<std::mutex> lk(g_timer_mu);
  g_timed.push_back(*t);
  delete t;
}

}  // namespace dawn

using namespace dawn;

extern "C" dawn_status dawn_kernel_timer(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_timer_mu);
  if (enable) {
    for (auto& t : g_timed) {
      hipEventDestroy(t.a);
      hipEventDestroy(t.b);
    }
    g_timed.clear();
  }
  g_timer_on = enable != 0;
  return DAWN_OK;
}

extern "C" dawn_status dawn_kernel_time(double* total_ms, int32_t* launches) {
  if (!total_ms || !launches) return set_error(DAWN_E_INVALID, "null output");
  std::lock_guard<std::mutex> lk(g_timer_mu);
  double sum = 0.0;
  int32_t cnt = 0;
  for (auto& t : g_timed) {
    dawn_status st = hip_check(hipEventSynchronize(t.b), "timer sync");
    if (st != DAWN_OK) return st;
    float ms = 0.f;
    if ((st = hip_check(hipEventElapsedTime(&ms, t.a, t.b), "timer elapsed")) != DAWN_OK) return st;
    sum += ms;
    cnt += t.launches;
  }
  *total_ms = sum;
  *launches = cnt;
  return DAWN_OK;
}

// ---------------------------------------------------------------------------
// misc
// ---------------------------------------------------------------------------
extern "C" const char* dawn_status_str(dawn_status s) {
  switch (s) {
    case DAWN_OK: return "ok";
    case DAWN_E_INVALID: return "invalid argument";
    case DAWN_E_UNSUPPORTED: return "unsupported";
    case DAWN_E_WORKSPACE: return "workspace too small";
    case DAWN_E_HIP: return "HIP error";
    case DAWN_E_INCOMPLETE: return "run did not converge";
  }
  return "unknown status";
}

extern "C" const char* dawn_last_error(void) { return g_err; }

extern "C" dawn_status dawn_device_query(int32_t* out) {
  if (!out) return set_error(DAWN_E_INVALID, "null output");
  const DevInfo& di = dev_info();
  const Residency ss = ss_persistent_residency(g_tuning.wg_threads);
  const Residency tl = tile_persistent_residency(g_tuning.wg_threads);
  const Residency ut = utile_persistent_residency(g_tuning.wg_threads);
  const int32_t v[DAWN_DEVICE_QUERY_LEN] = {
      di.cus,        di.coop ? 1 : 0, ss.per_cu,    tl.per_cu,    ss.grid,      tl.grid,
      di.device,     g_tuning.wg_threads, ss.vgprs, ss.lds,       ss.api_per_cu, tl.vgprs,
      tl.lds,        tl.api_per_cu,   ut.per_cu,    ut.vgprs};
  memcpy(out, v, sizeof(v));
  return DAWN_OK;
}

extern "C" dawn_status dawn_run_status(int32_t* incomplete_runs, int32_t* last_status) {
  const DevInfo& di = dev_info();
  if (!di.latch) return set_error(DAWN_E_HIP, "run-status latch unavailable");
  uint32_t w[2] = {0u, 0u};
  dawn_status st = hip_check(hipMemcpy(w, di.latch, sizeof(w), hipMemcpyDeviceToHost),
                             "read run status");
  if (st != DAWN_OK) return st;
  if (w[0] != 0u) {
    const uint32_t z[2] = {0u, 0u};
    if ((st = hip_check(hipMemcpy(di.latch, z, sizeof(z), hipMemcpyHostToDevice),
                        "clear run status")) != DAWN_OK)
      return st;
  }
  if (incomplete_runs) *incomplete_runs = (int32_t)w[0];
  if (last_status) *last_status = w[0] ? (int32_t)w[1] : 1;
  if (w[0] == 0u) return DAWN_OK;
  return set_error(DAWN_E_INCOMPLETE, "%u run(s) ended without converging (last status %d)", w[0],
                   (int32_t)w[1]);
}

extern "C" const char* dawn_build_info(void) {
  return "gfx950 hipcc -O3 (IEEE fp32 adds, no denormal flush, no packed-fp32)";
}

extern "C" dawn_status dawn_get_tuning(dawn_tuning* out) {
  if (!out) return set_error(DAWN_E_INVALID, "null output");
  const Tuning& t = g_tuning;
  out->t_lane = t.t_lane;
  out->t_wave = t.t_wave;
  out->t_chunk = t.t_chunk;
  out->wg_threads = t.wg_threads;
  out->grid = t.grid;
  out->mode = t.mode;
  out->step_launches = t.step_launches;
  out->tile_k = t.tile_k;
  out->tile_t_wave = t.tile_t_wave;
  out->tile_t_chunk = t.tile_t_chunk;
  out->validate = t.validate;
  out->coop = t.coop;
  out->tile_t_group = t.tile_t_group;
  out->tile_skip = t.tile_skip;
  out->small_m = t.small_m;
  out->step_min_m = t.step_min_m;
  out->tile_sparse = t.tile_sparse;
  out->tile_pull = t.tile_pull;
  out->tile_pull_src = t.tile_pull_src;
  out->ss_skip = t.ss_skip;
  out->ss_pull = t.ss_pull;
  out->tile_step_launches = t.tile_step_launches;
  out->barrier_ms = t.barrier_ms;
  out->ss_tail_grid = t.ss_tail_grid;
  return DAWN_OK;
}

extern "C" dawn_status dawn_set_tuning(const dawn_tuning* in) {
  Tuning t;
  if (in) {
    t.t_lane = in->t_lane;
    t.t_wave = in->t_wave;
    t.t_chunk = in->t_chunk;
    t.wg_threads = in->wg_threads;
    t.grid = in->grid;
    t.mode = in->mode;
    t.step_launches = in->step_launches;
    t.tile_k = in->tile_k;
    t.tile_t_wave = in->tile_t_wave;
    t.tile_t_chunk = in->tile_t_chunk;
    t.validate = in->validate;
    t.coop = in->coop;
    t.tile_t_group = in->tile_t_group;
    t.tile_skip = in->tile_skip;
    t.small_m = in->small_m;
    t.step_min_m = in->step_min_m;
    t.tile_sparse = in->tile_sparse;
    t.tile_pull = in->tile_pull;
    t.tile_pull_src = in->tile_pull_src;
    t.ss_skip = in->ss_skip;
    t.ss_pull = in->ss_pull;
    t.tile_step_launches = in->tile_step_launches;
    t.barrier_ms = in->barrier_ms;
    t.ss_tail_grid = in->ss_tail_grid;
  }
  if (!tuning_ok(t)) return set_error(DAWN_E_INVALID, "tuning out of range");
  g_tuning = t;
  return DAWN_OK;
}

// ---------------------------------------------------------------------------
// single source
// ---------------------------------------------------------------------------
extern "C" size_t dawn_sssp_workspace_bytes(int32_t n, int32_t m) {
  if (n < 1 || m < 0) return 0;
  return ss_layout(n, m).total;
}

extern "C" dawn_status dawn_sssp_ws(const int32_t* rowptr, const int32_t* colidx,
                                    const void* weights, dawn_wtype wt, int32_t n, int32_t m,
                                    int32_t source, void* dist_out, void* ws, size_t ws_bytes,
                                    dawn_run_info* info, hipStream_t stream) {
  dawn_status st = check_graph(rowptr, colidx, weights, wt, n, m, true, true);
  if (st != DAWN_OK) return st;
  if (source < 0 || source >= n) return set_error(DAWN_E_INVALID, "source %d out of range", source);
  if (!dist_out) return set_error(DAWN_E_INVALID, "dist_out is null");
  if (!ws) return set_error(DAWN_E_INVALID, "workspace is null");
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0)
    return set_error(DAWN_E_INVALID, "workspace must be 256-byte aligned");
  if (ws_bytes < ss_layout(n, m).total)
    return set_error(DAWN_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, ss_layout(n, m).total);
  SsSeeds seeds;
  seeds.source = source;
  return ss_run(rowptr, colidx, weights, (int)wt, n, m, seeds, true, dist_out, ws, info, stream,
                false);
}

extern "C" dawn_status dawn_sssp_tg_ws(const int32_t* rowptr, const int32_t* colidx,
                                       const void* weights, dawn_wtype wt, int32_t n, int32_t m,
                                       const void* tgraph, int32_t source, void* dist_out,
                                       void* ws, size_t ws_bytes, dawn_run_info* info,
                                       hipStream_t stream) {
  dawn_status st = check_graph(rowptr, colidx, weights, wt, n, m, true, true);
  if (st != DAWN_OK) return st;
  if (!tgraph) return set_error(DAWN_E_INVALID, "null reverse graph");
  if (source < 0 || source >= n) return set_error(DAWN_E_INVALID, "source %d out of range", source);
  if (!dist_out || !ws) return set_error(DAWN_E_INVALID, "null pointer");
  if (((reinterpret_cast<uintptr_t>(ws) | reinterpret_cast<uintptr_t>(tgraph)) & 255u) != 0)
    return set_error(DAWN_E_INVALID, "workspace and reverse graph must be 256-byte aligned");
  if (ws_bytes < ss_layout(n, m).total)
    return set_error(DAWN_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, ss_layout(n, m).total);
  SsSeeds seeds;
  seeds.source = source;
  return ss_run(rowptr, colidx, weights, (int)wt, n, m, seeds, true, dist_out, ws, info, stream,
                false, tgraph);
}

extern "C" dawn_status dawn_sssp(const int32_t* rowptr, const int32_t* colidx, const void* weights,
                                 dawn_wtype wt, int32_t n, int32_t m, int32_t source,
                                 void* dist_out, hipStream_t stream) {
  dawn_status st = check_graph(rowptr, colidx, weights, wt, n, m, true, true);
  if (st != DAWN_OK) return st;
  if (source < 0 || source >= n) return set_error(DAWN_E_INVALID, "source %d out of range", source);
  if (!dist_out) return set_error(DAWN_E_INVALID, "dist_out is null");
  const size_t bytes = ss_layout(n, m).total;
  StreamScratch ws(stream);
  if ((st = ws.alloc(bytes)) != DAWN_OK) return st;
  return dawn_sssp_ws(rowptr, colidx, weights, wt, n, m, source, dist_out, ws.p, bytes, nullptr,
                      stream);
}

extern "C" dawn_status dawn_sssp_noalloc(const int32_t* rowptr, const int32_t* colidx,
                                         const void* weights, dawn_wtype wt, int32_t n,
                                         int32_t m, int32_t source, void* dist_out,
                                         hipStream_t stream) {
  dawn_status st = check_graph(rowptr, colidx, weights, wt, n, m, true, true);
  if (st != DAWN_OK) return st;
  if (source < 0 || source >= n) return set_error(DAWN_E_INVALID, "source %d out of range", source);
  if (!dist_out) return set_error(DAWN_E_INVALID, "dist_out is null");
  const size_t bytes = ss_layout(n, m).total;
  if (bytes > (size_t)DAWN_NOALLOC_SCRATCH_BYTES)
    return set_error(DAWN_E_WORKSPACE,
                     "graph needs %zu bytes of scratch; dawn_sssp_noalloc holds %zu (use dawn_sssp_ws)",
                     bytes, (size_t)DAWN_NOALLOC_SCRATCH_BYTES);
  const DevInfo& di = dev_info();
  if (!di.noalloc) return set_error(DAWN_E_HIP, "no-allocation scratch unavailable on this device");
  SsSeeds seeds;
  seeds.source = source;
  // capture = true: no timing events (creating them may allocate) and no
  // cooperative launch; the launch sequence is the same as dawn_sssp's.
  return ss_run(rowptr, colidx, weights, (int)wt, n, m, seeds, true, dist_out, di.noalloc,
                nullptr, stream, true);
}

// ---------------------------------------------------------------------------
// multi source / all pairs
// ---------------------------------------------------------------------------
extern "C" size_t dawn_msssp_workspace_bytes(int32_t n, int32_t m, int32_t k) {
  if (n < 1 || m < 0 || k < 1) return 0;
  return tile_layout(n, m, std::min(k, g_tuning.tile_k)).total;
}

__global__ void dawn_info_zero_kernel(dawn_run_info* info) {
  if (threadIdx.x == 0) *info = dawn_run_info{};
}

__global__ void dawn_info_add_kernel(dawn_run_info* acc, const dawn_run_info* part, int first) {
  if (threadIdx.x != 0) return;
  if (first) {
    *acc = *part;
    return;
  }
  acc->steps = max(acc->steps, part->steps);
  if (part->converged < acc->converged) acc->converged = part->converged;
  acc->frontier_entries += part->frontier_entries;
  acc->edges_scanned += part->edges_scanned;
  acc->improvements += part->improvements;
  acc->union_rows += part->union_rows;
  acc->union_edges += part->union_edges;
}

// A multi-source run, tile by tile.  Each tile: reset, seeding,
// `tile_step_launches` step launches (a step launch returns at once once the
// tile's run has ended), then one persistent launch for whatever steps remain
// (tuning mode 2: the persistent launch alone), the transposed store and the
// run summary.  Nothing waits on the host, so the whole call is a fixed launch
// sequence on `stream` that a HIP graph can capture.
static dawn_status msssp_impl(const int32_t* rowptr, const int32_t* colidx, const void* weights,
                              dawn_wtype wt, int32_t n, int32_t m, const int32_t* sources,
                              int32_t k, void* dist_out, void* ws, dawn_run_info* info,
                              hipStream_t stream, const void* tgraph = nullptr,
                              bool unweighted = false) {
  unweighted = unweighted || wt == DAWN_W_UNIT;  // unit weights: the hop-count tiles
  const bool f32 = wt == DAWN_W_F32;
  const int32_t kt = std::min(k, g_tuning.tile_k);
  const TileLayout L = tile_layout(n, m, kt, unweighted);
  TileArgs A = tile_args(rowptr, colidx, weights, n, m, L, ws);
  if (tgraph && g_tuning.tile_pull <= 1000) {
    A.T = tgraph_view(tgraph, n, m);
    A.pull_min = (long long)m * g_tuning.tile_pull / 1000;
    A.pull_src = g_tuning.tile_pull_src;
  }
  // per-tile summary, inside the workspace (no allocation on this path)
  dawn_run_info* part = reinterpret_cast<dawn_run_info*>(static_cast<char*>(ws) + L.info);
  dawn_status st;
  const int32_t launches =
      g_tuning.mode == 2 ? 0 : (int32_t)std::min<int64_t>(g_tuning.tile_step_launches, (int64_t)n + 1);
  for (int32_t j0 = 0; j0 < k; j0 += kt) {
    const int32_t cnt = std::min(kt, k - j0);
    if ((st = tile_reset(A, f32, stream)) != DAWN_OK) return st;
    if ((st = tile_seed_all(A, sources + j0, cnt, g_tuning.validate != 0, f32, stream)) != DAWN_OK)
      return st;
    if (launches > 0) {
      st = unweighted ? utile_steps(A, launches, stream) : tile_steps(A, f32, false, launches, stream);
      if (st != DAWN_OK) return st;
    }
    st = unweighted ? utile_persistent(A, stream) : tile_steps(A, f32, true, INT32_MAX, stream);
    if (st != DAWN_OK) return st;
    char* out = static_cast<char*>(dist_out) + (size_t)j0 * (size_t)n * 4;
    st = unweighted ? utile_store(A, 0, cnt, reinterpret_cast<uint32_t*>(out), n, stream)
                    : tile_store(A, 0, cnt, out, n, stream);
    if (st != DAWN_OK) return st;
    // with run info: this tile's summary, summed into the caller's; without:
    // the tile's status into the run-status latch
    if ((st = tile_info(A, info ? part : nullptr, stream)) != DAWN_OK) return st;
    if (info) {
      hipLaunchKernelGGL(dawn_info_add_kernel, dim3(1), dim3(64), 0, stream, info, part,
                         (int)(j0 == 0));
      if ((st = hip_check(hipGetLastError(), "info")) != DAWN_OK) return st;
    }
  }
  return DAWN_OK;
}

extern "C" dawn_status dawn_msssp_ws(const int32_t* rowptr, const int32_t* colidx,
                                     const void* weights, dawn_wtype wt, int32_t n, int32_t m,
                                     const int32_t* sources, int32_t k, void* dist_out, void* ws,
                                     size_t ws_bytes, dawn_run_info* info, hipStream_t stream) {
  dawn_status st = check_graph(rowptr, colidx, weights, wt, n, m);
  if (st != DAWN_OK) return st;
  if (k < 1) return set_error(DAWN_E_INVALID, "k must be >= 1");
  if (!sources || !dist_out || !ws) return set_error(DAWN_E_INVALID, "null pointer");
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0)
    return set_error(DAWN_E_INVALID, "workspace must be 256-byte aligned");
  const size_t need = tile_layout(n, m, std::min(k, g_tuning.tile_k)).total;
  if (ws_bytes < need) return set_error(DAWN_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  return msssp_impl(rowptr, colidx, weights, wt, n, m, sources, k, dist_out, ws, info, stream);
}

extern "C" size_t dawn_tgraph_bytes(int32_t n, int32_t m) {
  if (n < 1 || m < 0) return 0;
  return tgraph_bytes(n, m);
}

extern "C" size_t dawn_tgraph_build_bytes(int32_t n, int32_t m) {
  if (n < 1 || m < 0) return 0;
  return tgraph_build_bytes(n, m);
}

extern "C" dawn_status dawn_tgraph_build(const int32_t* rowptr, const int32_t* colidx,
                                         const void* weights, int32_t n, int32_t m,
                                         void* tgraph, size_t tgraph_bytes_, void* scratch,
                                         size_t scratch_bytes, hipStream_t stream) {
  dawn_status st = check_graph(rowptr, colidx, weights, DAWN_W_U32, n, m, false);
  if (st != DAWN_OK) return st;
  if (!tgraph || !scratch) return set_error(DAWN_E_INVALID, "null buffer");
  if (((reinterpret_cast<uintptr_t>(tgraph) | reinterpret_cast<uintptr_t>(scratch)) & 255u) != 0)
    return set_error(DAWN_E_INVALID, "buffers must be 256-byte aligned");
  if (tgraph_bytes_ < tgraph_bytes(n, m))
    return set_error(DAWN_E_WORKSPACE, "reverse-graph buffer too small (%zu < %zu)", tgraph_bytes_,
                     tgraph_bytes(n, m));
  if (scratch_bytes < tgraph_build_bytes(n, m))
    return set_error(DAWN_E_WORKSPACE, "scratch too small (%zu < %zu)", scratch_bytes,
                     tgraph_build_bytes(n, m));
  return tgraph_build(rowptr, colidx, weights, n, m, tgraph, scratch, stream);
}

extern "C" dawn_status dawn_msssp_tg_ws(const int32_t* rowptr, const int32_t* colidx,
                                        const void* weights, dawn_wtype wt, int32_t n, int32_t m,
                                        const void* tgraph, const int32_t* sources, int32_t k,
                                        void* dist_out, void* ws, size_t ws_bytes,
                                        dawn_run_info* info, hipStream_t stream) {
  dawn_status st = check_graph(rowptr, colidx, weights, wt, n, m);
  if (st != DAWN_OK) return st;
  if (!tgraph) return set_error(DAWN_E_INVALID, "null reverse graph");
  if (!sources || !dist_out || !ws) return set_error(DAWN_E_INVALID, "null pointer");
  if (k < 1) return set_error(DAWN_E_INVALID, "k must be >= 1 (got %d)", k);
  if (((reinterpret_cast<uintptr_t>(ws) | reinterpret_cast<uintptr_t>(tgraph)) & 255u) != 0)
    return set_error(DAWN_E_INVALID, "workspace and reverse graph must be 256-byte aligned");
  const size_t need = tile_layout(n, m, std::min(k, g_tuning.tile_k)).total;
  if (ws_bytes < need)
    return set_error(DAWN_E_WORKSPACE, "workspace too small (%zu < %zu)", ws_bytes, need);
  return msssp_impl(rowptr, colidx, weights, wt, n, m, sources, k, dist_out, ws, info, stream,
                    tgraph);
}

extern "C" size_t dawn_umsssp_workspace_bytes(int32_t n, int32_t m, int32_t k) {
  if (n < 1 || m < 0 || k < 1) return 0;
  return tile_layout(n, m, std::min(k, g_tuning.tile_k), true).total;
}

extern "C" size_t dawn_workspace_bytes(int32_t n, int32_t m, int32_t k, dawn_wtype wt) {
  if (n < 1 || m < 0 || k < 1) return 0;
  if (wt != DAWN_W_U32 && wt != DAWN_W_F32 && wt != DAWN_W_I32 && wt != DAWN_W_UNIT) return 0;
  if (k == 1) return dawn_sssp_workspace_bytes(n, m);
  if (wt == DAWN_W_I32) return 0;
  return wt == DAWN_W_UNIT ? dawn_umsssp_workspace_bytes(n, m, k)
                           : dawn_msssp_workspace_bytes(n, m, k);
}

extern "C" dawn_status dawn_umsssp_ws(const int32_t* rowptr, const int32_t* colidx, int32_t n,
                                      int32_t m, const void* tgraph, const int32_t* sources,
                                      int32_t k, uint32_t* dist_out, void* ws, size_t ws_bytes,
                                      dawn_run_info* info, hipStream_t stream) {
  dawn_status st = check_graph(rowptr, colidx, nullptr, DAWN_W_U32, n, m, false);
  if (st != DAWN_OK) return st;
  if (!sources || !dist_out || !ws) return set_error(DAWN_E_INVALID, "null pointer");
  if (k < 1) return set_error(DAWN_E_INVALID, "k must be >= 1 (got %d)", k);
  if (((reinterpret_cast<uintptr_t>(ws) | reinterpret_cast<uintptr_t>(tgraph)) & 255u) != 0)
    return set_error(DAWN_E_INVALID, "workspace and reverse graph must be 256-byte aligned");
  const size_t need = tile_layout(n, m, std::min(k, g_tuning.tile_k), true).total;
  if (ws_bytes < need)
    return set_error(DAWN_E_WORKSPACE, "workspace too small (%zu < %zu)", ws_bytes, need);
  return msssp_impl(rowptr, colidx, nullptr, DAWN_W_U32, n, m, sources, k, dist_out, ws, info,
                    stream, tgraph, true);
}

extern "C" dawn_status dawn_msssp(const int32_t* rowptr, const int32_t* colidx,
                                  const void* weights, dawn_wtype wt, int32_t n, int32_t m,
                                  const int32_t* sources, int32_t k, void* dist_out,
                                  hipStream_t stream) {
  dawn_status st = check_graph(rowptr, colidx, weights, wt, n, m);
  if (st != DAWN_OK) return st;
  if (k < 1) return set_error(DAWN_E_INVALID, "k must be >= 1");
  if (!sources || !dist_out) return set_error(DAWN_E_INVALID, "null pointer");
  const size_t need = tile_layout(n, m, std::min(k, g_tuning.tile_k)).total;
  StreamScratch ws(stream);
  if ((st = ws.alloc(need)) != DAWN_OK) return st;
  return msssp_impl(rowptr, colidx, weights, wt, n, m, sources, k, dist_out, ws.p, nullptr, stream);
}

__global__ void dawn_iota_kernel(int32_t* out, int32_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = (int32_t)i;
}

extern "C" dawn_status dawn_apsp(const int32_t* rowptr, const int32_t* colidx, const void* weights,
                                 dawn_wtype wt, int32_t n, int32_t m, void* dist_out,
                                 hipStream_t stream) {
  dawn_status st = check_graph(rowptr, colidx, weights, wt, n, m);
  if (st != DAWN_OK) return st;
  if (!dist_out) return set_error(DAWN_E_INVALID, "dist_out is null");
  const unsigned __int128 nn = (unsigned __int128)(uint64_t)n * (uint64_t)n * 4u;
  if (nn > (unsigned __int128)SIZE_MAX) return set_error(DAWN_E_INVALID, "n*n overflows");
  StreamScratch ids(stream);
  if ((st = ids.alloc((size_t)n * 4)) != DAWN_OK) return st;
  hipLaunchKernelGGL(dawn_iota_kernel, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)),
                     dim3(256), 0, stream, static_cast<int32_t*>(ids.p), n);
  if ((st = hip_check(hipGetLastError(), "iota")) != DAWN_OK) return st;
  return dawn_msssp(rowptr, colidx, weights, wt, n, m, static_cast<int32_t*>(ids.p), n, dist_out,
                    stream);
}

// ---------------------------------------------------------------------------
// many graphs, one launch
// ---------------------------------------------------------------------------
struct dawn_batch {
  int32_t count = 0;
  dawn_wtype wt = DAWN_W_U32;
  int64_t total_n = 0, total_m = 0;
  std::vector<int64_t> voff_h;
  int64_t* voff = nullptr;  // device copy
  int32_t* rowptr = nullptr;
  int32_t* colidx = nullptr;
  uint32_t* w = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
};

__global__ void batch_rows_kernel(const int32_t* rp, int32_t n, int64_t voff, int64_t eoff,
                                  int32_t* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    out[voff + v] = (int32_t)(rp[v] + eoff);
}

__global__ void batch_cols_kernel(const int32_t* ci, int32_t m, int64_t voff, int32_t* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride)
    out[e] = (int32_t)(ci[e] + voff);
}

__global__ void batch_last_row_kernel(int32_t* rowptr, int64_t total_n, int64_t total_m) {
  if (threadIdx.x == 0) rowptr[total_n] = (int32_t)total_m;
}

static void batch_free(dawn_batch* b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  hipFree(b->voff);
  hipFree(b->rowptr);
  hipFree(b->colidx);
  hipFree(b->w);
  hipFree(b->ws);
  delete b;
}

extern "C" dawn_status dawn_batch_create(dawn_batch** out, int32_t count,
                                         const int32_t* const* rowptrs,
                                         const int32_t* const* colidxs,
                                         const void* const* weights, const int32_t* ns,
                                         const int32_t* ms, dawn_wtype wt, hipStream_t stream) {
  if (!out || count < 1 || !rowptrs || !colidxs || !weights || !ns || !ms)
    return set_error(DAWN_E_INVALID, "bad batch arguments");
  if (wt == DAWN_W_I32) return set_error(DAWN_E_UNSUPPORTED, "int32 weights: single-source calls only");
  if (wt == DAWN_W_UNIT) return set_error(DAWN_E_UNSUPPORTED, "unit weights: not in a batch");
  if (wt != DAWN_W_U32 && wt != DAWN_W_F32) return set_error(DAWN_E_INVALID, "unknown wtype");
  *out = nullptr;
  dawn_batch* b = new dawn_batch();
  b->count = count;
  b->wt = wt;
  b->voff_h.resize(count);
  for (int32_t i = 0; i < count; i++) {
    if (ns[i] < 1 || ms[i] < 0 || !rowptrs[i] || (ms[i] > 0 && (!colidxs[i] || !weights[i]))) {
      delete b;
      return set_error(DAWN_E_INVALID, "graph %d: bad size or pointer", i);
    }
    b->voff_h[i] = b->total_n;
    b->total_n += ns[i];
    b->total_m += ms[i];
  }
  if (b->total_n >= INT32_MAX || b->total_m >= INT32_MAX) {
    delete b;
    return set_error(DAWN_E_UNSUPPORTED, "union too large for int32 ids");
  }
  dawn_status st = DAWN_OK;
  auto fail = [&](dawn_status s) {
    batch_free(b);
    return s;
  };
  if ((st = hip_check(hipMalloc(&b->voff, count * 8), "hipMalloc")) != DAWN_OK) return fail(st);
  if ((st = hip_check(hipMalloc(&b->rowptr, (b->total_n + 1) * 4), "hipMalloc")) != DAWN_OK)
    return fail(st);
  if ((st = hip_check(hipMalloc(&b->colidx, std::max<int64_t>(b->total_m, 1) * 4), "hipMalloc")) !=
      DAWN_OK)
    return fail(st);
  if ((st = hip_check(hipMalloc(&b->w, std::max<int64_t>(b->total_m, 1) * 4), "hipMalloc")) != DAWN_OK)
    return fail(st);
  b->ws_bytes = ss_layout(b->total_n, b->total_m).total;
  if ((st = hip_check(hipMalloc(&b->ws, b->ws_bytes), "hipMalloc")) != DAWN_OK) return fail(st);
  hipMemcpyAsync(b->voff, b->voff_h.data(), count * 8, hipMemcpyHostToDevice, stream);
  int64_t eoff = 0;
  for (int32_t i = 0; i < count; i++) {
    const unsigned gr = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, (ns[i] + 255) / 256));
    hipLaunchKernelGGL(batch_rows_kernel, dim3(gr), dim3(256), 0, stream, rowptrs[i], ns[i],
                       b->voff_h[i], eoff, b->rowptr);
    if (ms[i] > 0) {
      const unsigned ge = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (ms[i] + 255) / 256));
      hipLaunchKernelGGL(batch_cols_kernel, dim3(ge), dim3(256), 0, stream, colidxs[i], ms[i],
                         b->voff_h[i], b->colidx + eoff);
      hipMemcpyAsync(b->w + eoff, weights[i], (size_t)ms[i] * 4, hipMemcpyDeviceToDevice, stream);
    }
    eoff += ms[i];
  }
  hipLaunchKernelGGL(batch_last_row_kernel, dim3(1), dim3(64), 0, stream, b->rowptr, b->total_n,
                     b->total_m);
  if ((st = hip_check(hipGetLastError(), "batch build")) != DAWN_OK) return fail(st);
  // the caller's host arrays (voff_h) are read by the async copy: finish it here
  if ((st = hip_check(hipStreamSynchronize(stream), "batch build sync")) != DAWN_OK) return fail(st);
  *out = b;
  return DAWN_OK;
}

extern "C" dawn_status dawn_batch_sizes(const dawn_batch* b, int64_t* total_n, int64_t* total_m) {
  if (!b) return set_error(DAWN_E_INVALID, "null batch");
  if (total_n) *total_n = b->total_n;
  if (total_m) *total_m = b->total_m;
  return DAWN_OK;
}

extern "C" int64_t dawn_batch_vertex_offset(const dawn_batch* b, int32_t i) {
  if (!b || i < 0 || i >= b->count) return -1;
  return b->voff_h[i];
}

static dawn_status batch_enqueue(dawn_batch* b, const int32_t* sources, void* dist_out,
                                 dawn_run_info* info, hipStream_t stream, bool capture) {
  if (!tuning_ok(g_tuning)) return set_error(DAWN_E_INVALID, "tuning out of range");
  SsSeeds seeds;
  seeds.sources_dev = sources;
  seeds.voff_dev = b->voff;
  seeds.count = b->count;
  seeds.source = 0;
  return ss_run(b->rowptr, b->colidx, b->w, (int)b->wt, (int32_t)b->total_n,
                (int32_t)b->total_m, seeds, false, dist_out, b->ws, info, stream, capture);
}

extern "C" dawn_status dawn_batch_run(dawn_batch* b, const int32_t* sources, void* dist_out,
                                      dawn_run_info* info, hipStream_t stream) {
  if (!b || !sources || !dist_out) return set_error(DAWN_E_INVALID, "null pointer");
  return batch_enqueue(b, sources, dist_out, info, stream, false);
}

extern "C" dawn_status dawn_batch_capture(dawn_batch* b, const int32_t* sources, void* dist_out,
                                          dawn_run_info* info, hipStream_t stream) {
  if (!b || !sources || !dist_out) return set_error(DAWN_E_INVALID, "null pointer");
  dawn_status st;
  if (b->exec) {
    hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  if (!b->cap_stream &&
      (st = hip_check(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking),
                      "hipStreamCreate")) != DAWN_OK)
    return st;
  // make the capture stream wait for the caller's prior work (batch build etc)
  hipEvent_t ev;
  if ((st = hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event")) != DAWN_OK)
    return st;
  hipEventRecord(ev, stream);
  hipStreamWaitEvent(b->cap_stream, ev, 0);
  hipStreamSynchronize(b->cap_stream);
  hipEventDestroy(ev);
  if ((st = hip_check(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal),
                      "begin capture")) != DAWN_OK)
    return st;
  dawn_status rs = batch_enqueue(b, sources, dist_out, info, b->cap_stream, true);
  hipGraph_t g = nullptr;
  st = hip_check(hipStreamEndCapture(b->cap_stream, &g), "end capture");
  if (rs != DAWN_OK) {
    if (g) hipGraphDestroy(g);
    return rs;
  }
  if (st != DAWN_OK) return st;
  b->graph = g;
  return hip_check(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "graph instantiate");
}

extern "C" dawn_status dawn_batch_replay(dawn_batch* b, hipStream_t stream) {
  if (!b || !b->exec) return set_error(DAWN_E_INVALID, "batch has no captured graph");
  return hip_check(hipGraphLaunch(b->exec, stream), "graph launch");
}

extern "C" void dawn_batch_destroy(dawn_batch* b) { batch_free(b); }

// ---------------------------------------------------------------------------
// tile sessions
// ---------------------------------------------------------------------------
struct dawn_tile {
  TileLayout L;
  TileArgs A;
  void* ws = nullptr;            // the caller's workspace (not owned)
  bool f32 = false;
  int32_t k = 0;
  const void* tgraph = nullptr;  // reverse graph for pull steps, or null
  // a captured run (dawn_tile_capture)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void tile_graph_free(dawn_tile* t) {
  if (t->exec) hipGraphExecDestroy(t->exec);
  if (t->graph) hipGraphDestroy(t->graph);
  t->exec = nullptr;
  t->graph = nullptr;
}

extern "C" size_t dawn_tile_bytes(int32_t n, int32_t m, int32_t k) {
  if (n < 1 || m < 0 || k < 1 || k > DAWN_TILE_K_MAX) return 0;
  return tile_layout(n, m, k).total;
}

extern "C" dawn_status dawn_tile_create(dawn_tile** out, const int32_t* rowptr,
                                        const int32_t* colidx, const void* weights, dawn_wtype wt,
                                        int32_t n, int32_t m, int32_t k, void* ws, size_t ws_bytes,
                                        hipStream_t stream) {
  if (!out) return set_error(DAWN_E_INVALID, "null output");
  *out = nullptr;
  dawn_status st = check_graph(rowptr, colidx, weights, wt, n, m);
  if (st != DAWN_OK) return st;
  if (wt == DAWN_W_UNIT) return set_error(DAWN_E_UNSUPPORTED, "unit weights: not in a tile session");
  if (k < 1) return set_error(DAWN_E_INVALID, "k must be >= 1");
  if (k > DAWN_TILE_K_MAX) return set_error(DAWN_E_UNSUPPORTED, "k above %d", DAWN_TILE_K_MAX);
  if (!ws) return set_error(DAWN_E_INVALID, "workspace is null");
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0)
    return set_error(DAWN_E_INVALID, "workspace must be 256-byte aligned");
  const TileLayout L = tile_layout(n, m, k);
  if (ws_bytes < L.total)
    return set_error(DAWN_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
  dawn_tile* t = new dawn_tile();
  t->L = L;
  t->f32 = wt == DAWN_W_F32;
  t->k = k;
  t->ws = ws;
  t->A = tile_args(rowptr, colidx, weights, n, m, t->L, t->ws);
  if ((st = tile_reset(t->A, t->f32, stream)) != DAWN_OK) {
    delete t;
    return st;
  }
  *out = t;
  return DAWN_OK;
}

extern "C" dawn_status dawn_tile_admit(dawn_tile* t, int32_t col, int32_t source,
                                       hipStream_t stream) {
  if (!t) return set_error(DAWN_E_INVALID, "null tile");
  if (col < 0 || col >= t->k) return set_error(DAWN_E_INVALID, "column %d out of range", col);
  if (source < 0 || source >= t->A.n) return set_error(DAWN_E_INVALID, "source out of range");
  return tile_admit(t->A, t->f32, col, source, stream);
}

// The launches of one run: max_steps step launches, then the done bits.
static dawn_status tile_run_enqueue(dawn_tile* t, int32_t max_steps, uint32_t* done_bits,
                                    hipStream_t stream) {
  TileArgs a = t->A;
  if (t->tgraph && g_tuning.tile_pull <= 1000) {
    a.T = tgraph_view(t->tgraph, a.n, a.m);
    a.pull_min = (long long)a.m * g_tuning.tile_pull / 1000;
    a.pull_src = g_tuning.tile_pull_src;
  }
  dawn_status st = tile_steps(a, t->f32, false, max_steps, stream);
  if (st != DAWN_OK) return st;
  if (done_bits) st = tile_done_bits(t->A, t->k, done_bits, stream);
  return st;
}

extern "C" dawn_status dawn_tile_run(dawn_tile* t, int32_t max_steps, uint32_t* done_bits,
                                     hipStream_t stream) {
  if (!t) return set_error(DAWN_E_INVALID, "null tile");
  if (max_steps < 1) return set_error(DAWN_E_INVALID, "max_steps must be >= 1");
  return tile_run_enqueue(t, max_steps, done_bits, stream);
}

// The run's launch sequence holds only kernel launches that read the run's
// state from device memory (step, done flag, masks, column words), so one
// captured sequence serves every later run of the session, whatever columns
// were admitted or evicted in between.
extern "C" dawn_status dawn_tile_capture(dawn_tile* t, int32_t max_steps, uint32_t* done_bits) {
  if (!t) return set_error(DAWN_E_INVALID, "null tile");
  if (max_steps < 1) return set_error(DAWN_E_INVALID, "max_steps must be >= 1");
  tile_graph_free(t);
  dawn_status st;
  if (!t->cap_stream &&
      (st = hip_check(hipStreamCreateWithFlags(&t->cap_stream, hipStreamNonBlocking),
                      "hipStreamCreate")) != DAWN_OK)
    return st;
  if ((st = hip_check(hipStreamBeginCapture(t->cap_stream, hipStreamCaptureModeThreadLocal),
                      "begin capture")) != DAWN_OK)
    return st;
  const dawn_status rs = tile_run_enqueue(t, max_steps, done_bits, t->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(t->cap_stream, &g);
  if (rs != DAWN_OK) {
    if (g) hipGraphDestroy(g);
    return rs;
  }
  if ((st = hip_check(e, "end capture")) != DAWN_OK) return st;
  t->graph = g;
  st = hip_check(hipGraphInstantiate(&t->exec, g, nullptr, nullptr, 0), "graph instantiate");
  if (st != DAWN_OK) tile_graph_free(t);
  return st;
}

extern "C" dawn_status dawn_tile_replay(dawn_tile* t, hipStream_t stream) {
  if (!t || !t->exec) return set_error(DAWN_E_INVALID, "tile has no captured run");
  return hip_check(hipGraphLaunch(t->exec, stream), "graph launch");
}

extern "C" dawn_status dawn_tile_set_tgraph(dawn_tile* t, const void* tgraph) {
  if (!t) return set_error(DAWN_E_INVALID, "null tile");
  if ((reinterpret_cast<uintptr_t>(tgraph) & 255u) != 0)
    return set_error(DAWN_E_INVALID, "reverse graph must be 256-byte aligned");
  t->tgraph = tgraph;
  return DAWN_OK;
}

extern "C" dawn_status dawn_tile_read(dawn_tile* t, int32_t col, void* dist_out,
                                      hipStream_t stream) {
  if (!t || !dist_out) return set_error(DAWN_E_INVALID, "null pointer");
  if (col < 0 || col >= t->k) return set_error(DAWN_E_INVALID, "column %d out of range", col);
  return tile_read_col(t->A, col, dist_out, stream);
}

extern "C" dawn_status dawn_tile_steps(dawn_tile* t, int32_t* steps_out, hipStream_t stream) {
  if (!t || !steps_out) return set_error(DAWN_E_INVALID, "null pointer");
  return tile_col_steps(t->A, t->k, steps_out, stream);
}

extern "C" dawn_status dawn_tile_evict(dawn_tile* t, int32_t col, hipStream_t stream) {
  if (!t) return set_error(DAWN_E_INVALID, "null tile");
  if (col < 0 || col >= t->k) return set_error(DAWN_E_INVALID, "column %d out of range", col);
  return tile_evict(t->A, t->f32, col, stream);
}

extern "C" void dawn_tile_destroy(dawn_tile* t) {
  if (!t) return;
  tile_graph_free(t);
  if (t->cap_stream) hipStreamDestroy(t->cap_stream);
  delete t;
}
