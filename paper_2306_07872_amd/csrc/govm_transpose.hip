// govm_transpose.hip -- the reverse graph that pull steps read.
//
// A pull step relaxes every edge (u, v) whose source u is in the frontier by
// walking the in-edges of each target v, so it needs the graph transposed:
// for each v the list of (u, w(u, v)).  The lists are cut into chunks of at
// most kPullChunk in-edges; a target with several chunks ("split") is
// combined with atomics, every other target is written by the one wavefront
// that owns it.  Built once per graph into an opaque buffer:
//
//   header            {nchunks}
//   t_rowptr int32[n+1], t_colidx int32[m] (the sources u), t_w uint32[m]
//   chunks   int4[n + m / kPullChunk + 1]   {v, first in-edge, count, split}
//
// Construction: in-degree histogram (atomics), exclusive scan (per-block
// sums, a one-workgroup scan of the block sums, then offsets), scatter of the
// edges (each thread walks a fixed range of edges, finding its first row by
// binary search), and the chunk list (wave-aggregated reservations).
#include <algorithm>

#include "govm_host.hpp"

namespace dawn {

constexpr int kScanBlock = 1024;
constexpr int kScanItems = 4;  // per thread
constexpr int kScanTile = kScanBlock * kScanItems;
constexpr int kEdgesPerThread = 16;

struct TGraphLayout {
  size_t hdr, rowptr, colidx, w, chunks, total;
  int64_t cap_chunks;
};

static TGraphLayout tgraph_layout(int64_t n, int64_t m) {
  TGraphLayout L{};
  Carver c;
  L.cap_chunks = n + m / kPullChunk + 1;
  L.hdr = c.take(sizeof(TGraphHeader));
  L.rowptr = c.take((size_t)(n + 1) * 4);
  L.colidx = c.take((size_t)std::max<int64_t>(m, 1) * 4);
  L.w = c.take((size_t)std::max<int64_t>(m, 1) * 4);
  L.chunks = c.take((size_t)L.cap_chunks * 16);
  L.total = c.off;
  return L;
}

size_t tgraph_bytes(int64_t n, int64_t m) { return tgraph_layout(n, m).total; }

TGraph tgraph_view(const void* buf, int64_t n, int64_t m) {
  const TGraphLayout L = tgraph_layout(n, m);
  const char* b = static_cast<const char*>(buf);
  TGraph T{};
  T.hdr = reinterpret_cast<const TGraphHeader*>(b + L.hdr);
  T.rowptr = reinterpret_cast<const int32_t*>(b + L.rowptr);
  T.colidx = reinterpret_cast<const int32_t*>(b + L.colidx);
  T.w = reinterpret_cast<const uint32_t*>(b + L.w);
  T.chunks = reinterpret_cast<const int4*>(b + L.chunks);
  T.cap_chunks = L.cap_chunks;
  return T;
}

// scratch of a build: counts / cursors int32[n], block sums int32[nblocks]
size_t tgraph_build_bytes(int64_t n, int64_t m) {
  (void)m;
  Carver c;
  c.take((size_t)std::max<int64_t>(n, 1) * 4);
  c.take((size_t)((n + kScanTile - 1) / kScanTile + 1) * 4);
  return c.off;
}

__global__ void tg_zero_kernel(int32_t* a, int64_t n, TGraphHeader* hdr) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hdr->nchunks = 0;
  }
}

__global__ void tg_hist_kernel(const int32_t* colidx, int64_t m, int32_t* counts) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride)
    atomicAdd(&counts[colidx[e]], 1);
}

// Inclusive prefix sum over the 1024 threads of a workgroup (LDS).
__device__ __forceinline__ int64_t block_incl_scan(int64_t x, int64_t* sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const int64_t y = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += y;
    __syncthreads();
  }
  return sh[threadIdx.x];
}

// Sum of each tile of kScanTile counts.
__global__ void __launch_bounds__(kScanBlock) tg_tile_sums_kernel(const int32_t* counts, int64_t n,
                                                                  int32_t* sums) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
  for (int i = 0; i < kScanItems; i++) {
    const int64_t j = base + (int64_t)threadIdx.x * kScanItems + i;
    if (j < n) s += counts[j];
  }
  const int64_t tot = block_incl_scan(s, sh);
  if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = (int32_t)tot;
}

// Exclusive scan of the tile sums in place, in one workgroup (any count).
__global__ void __launch_bounds__(kScanBlock) tg_scan_sums_kernel(int32_t* sums, int64_t nt) {
  __shared__ int64_t sh[kScanBlock];
  int64_t carry = 0;
  for (int64_t t0 = 0; t0 < nt; t0 += kScanBlock) {
    const int64_t i = t0 + threadIdx.x;
    const int64_t x = i < nt ? sums[i] : 0;
    const int64_t incl = block_incl_scan(x, sh);
    if (i < nt) sums[i] = (int32_t)(carry + incl - x);
    const int64_t total = sh[kScanBlock - 1];
    __syncthreads();
    carry += total;
  }
}

// t_rowptr[j] = exclusive prefix of counts; counts becomes the scatter cursor.
__global__ void __launch_bounds__(kScanBlock) tg_offsets_kernel(int32_t* counts, int64_t n,
                                                                const int32_t* sums,
                                                                int32_t* t_rowptr, int64_t m) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t v[kScanItems], s = 0;
  for (int i = 0; i < kScanItems; i++) {
    const int64_t j = base + (int64_t)threadIdx.x * kScanItems + i;
    v[i] = j < n ? counts[j] : 0;
    s += v[i];
  }
  const int64_t incl = block_incl_scan(s, sh);
  int64_t run = sums[blockIdx.x] + incl - s;
  for (int i = 0; i < kScanItems; i++) {
    const int64_t j = base + (int64_t)threadIdx.x * kScanItems + i;
    if (j < n) {
      t_rowptr[j] = (int32_t)run;
      counts[j] = (int32_t)run;
    }
    run += v[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) t_rowptr[n] = (int32_t)m;
}

// Thread t scatters edges [t*E, (t+1)*E): its first row comes from a binary
// search of rowptr, later rows by walking forward.
__global__ void tg_scatter_kernel(const int32_t* rowptr, const int32_t* colidx, const uint32_t* w,
                                  int64_t n, int64_t m, int32_t* cursor, int32_t* t_colidx,
                                  uint32_t* t_w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t e0 = t * kEdgesPerThread;
  if (e0 >= m) return;
  const int64_t e1 = e0 + kEdgesPerThread < m ? e0 + kEdgesPerThread : m;
  // last row u with rowptr[u] <= e0
  int64_t lo = 0, hi = n;  // invariant: rowptr[lo] <= e0 < rowptr[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (rowptr[mid] <= e0) lo = mid;
    else hi = mid;
  }
  int64_t u = lo;
  for (int64_t e = e0; e < e1; e++) {
    while (rowptr[u + 1] <= e) u++;
    const int32_t v = colidx[e];
    const int32_t p = atomicAdd(&cursor[v], 1);
    t_colidx[p] = (int32_t)u;
    if (w) t_w[p] = w[e];
  }
}

// One chunk record per kPullChunk in-edges of each target with in-edges.
__global__ void tg_chunks_kernel(const int32_t* t_rowptr, int64_t n, int4* chunks, int64_t cap,
                                 TGraphHeader* hdr) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < n; v0 += stride) {
    const int64_t v = v0 + threadIdx.x;
    int32_t start = 0, deg = 0;
    if (v < n) {
      start = t_rowptr[v];
      deg = t_rowptr[v + 1] - start;
    }
    const uint32_t nch = deg > 0 ? (uint32_t)((deg + kPullChunk - 1) / kPullChunk) : 0u;
    // wave-aggregated reservation
    uint32_t incl = nch;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t y = __shfl_up(incl, off, kWave);
      if (lane_id() >= off) incl += y;
    }
    const uint32_t total = __shfl(incl, kWave - 1, kWave);
    uint32_t base = 0;
    if (lane_id() == 0 && total) base = atomicAdd(&hdr->nchunks, total);
    base = __shfl(base, 0, kWave);
    const uint32_t mine = base + incl - nch;
    for (uint32_t c = 0; c < nch; c++) {
      const int64_t p = (int64_t)mine + c;
      const int32_t off = (int32_t)c * kPullChunk;
      if (p < cap) chunks[p] = make_int4((int32_t)v, start + off, min(kPullChunk, deg - off), nch > 1);
    }
  }
}

dawn_status tgraph_build(const int32_t* rowptr, const int32_t* colidx, const void* w, int64_t n,
                         int64_t m, void* buf, void* scratch, hipStream_t stream) {
  const TGraphLayout L = tgraph_layout(n, m);
  char* b = static_cast<char*>(buf);
  TGraphHeader* hdr = reinterpret_cast<TGraphHeader*>(b + L.hdr);
  int32_t* t_rowptr = reinterpret_cast<int32_t*>(b + L.rowptr);
  int32_t* t_colidx = reinterpret_cast<int32_t*>(b + L.colidx);
  uint32_t* t_w = reinterpret_cast<uint32_t*>(b + L.w);
  int4* chunks = reinterpret_cast<int4*>(b + L.chunks);
  Carver c;
  int32_t* counts = reinterpret_cast<int32_t*>(static_cast<char*>(scratch) + c.take((size_t)std::max<int64_t>(n, 1) * 4));
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  int32_t* sums = reinterpret_cast<int32_t*>(static_cast<char*>(scratch) + c.take((size_t)(ntiles + 1) * 4));
  auto grid = [](int64_t work, int threads) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(65536, (work + threads - 1) / threads));
  };
  hipLaunchKernelGGL(tg_zero_kernel, dim3(grid(n, 256)), dim3(256), 0, stream, counts, n, hdr);
  hipLaunchKernelGGL(tg_hist_kernel, dim3(grid(m, 256)), dim3(256), 0, stream, colidx, m, counts);
  hipLaunchKernelGGL(tg_tile_sums_kernel, dim3((unsigned)std::max<int64_t>(ntiles, 1)),
                     dim3(kScanBlock), 0, stream, counts, n, sums);
  hipLaunchKernelGGL(tg_scan_sums_kernel, dim3(1), dim3(kScanBlock), 0, stream, sums, ntiles);
  hipLaunchKernelGGL(tg_offsets_kernel, dim3((unsigned)std::max<int64_t>(ntiles, 1)),
                     dim3(kScanBlock), 0, stream, counts, n, sums, t_rowptr, m);
  const int64_t nthreads = (m + kEdgesPerThread - 1) / kEdgesPerThread;
  if (m > 0)
    hipLaunchKernelGGL(tg_scatter_kernel, dim3((unsigned)((nthreads + 255) / 256)), dim3(256), 0,
                       stream, rowptr, colidx, static_cast<const uint32_t*>(w), n, m, counts,
                       t_colidx, t_w);
  hipLaunchKernelGGL(tg_chunks_kernel, dim3(grid(n, 256)), dim3(256), 0, stream, t_rowptr, n,
                     chunks, L.cap_chunks, hdr);
  return hip_check(hipGetLastError(), "transpose");
}

}  // namespace dawn
