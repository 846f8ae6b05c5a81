/*
 * dawn.h -- C ABI of the MI355X (gfx950) GOVM library.
 *
 * GOVM ("General Optimized Vector-Matrix operation", Section 3.4, Algorithm 2
 * of Feng, "Expanding the Scope of DAWN: A Novel Version for Weighted Shortest
 * Path Problem", arXiv 2306.07872) computes single-source shortest paths on a
 * weighted directed graph stored as CSR.  Each step applies the (min,+)
 * vector-matrix product  p_j = min_k (p_k + a_kj)  but only over the rows k
 * whose distance changed in the previous step; it stops after a step with no
 * change (the paper's "ptr" flag) or after n steps.  Section 3.1 shows the
 * fixed point is the Floyd-Warshall recurrence's, so for non-negative weights
 * the output is exactly the shortest-path distance vector:
 *
 *   d(v) = min over directed source->v paths of the path weight,
 *   d(source) = 0, d(v) = INF when v is unreachable.
 *
 * Multi-source (MSSP) and all-pairs (APSP) repeat this per source (Section 1,
 * Section 3.4 "APSP" cost); the library batches sources into a distance tile
 * because different sources never update the same path (Section 3.5).
 *
 * Conventions for every call
 * --------------------------
 * - Graph: rowptr int32[n+1] (rowptr[0] = 0, non-decreasing, rowptr[n] = m),
 *   colidx int32[m] in [0,n), weights[m] of type `wt`.  Rows need not be
 *   sorted; self-loops and parallel edges are allowed.
 * - Weights: DAWN_W_U32 = uint32 (any value; sums saturate at 0xFFFFFFFF, so a
 *   path of total weight >= 2^32-1 reads as unreachable), or DAWN_W_F32 =
 *   float32, finite with the sign bit clear (no negatives, no -0.0, no NaN).
 *   fp32 sums are IEEE round-to-nearest-even, no flush to zero.
 *   DAWN_W_I32 = int32 of either sign (single-source calls only: dawn_sssp,
 *   dawn_sssp_ws; every other call returns DAWN_E_UNSUPPORTED).  The paper
 *   claims negative weights without giving the mechanism; here it is the
 *   same GOVM iteration on int32 sums, ordered through keys (the int32 with
 *   its sign bit flipped, so the unsigned atomicMin orders them), with
 *   Algorithm 2's guard: the source's own distance is never lowered.  Result:
 *   the shortest-path distances of the graph without the edges into the
 *   source.  A reachable negative cycle keeps the iteration going to the
 *   n-step cap: info.converged = 0, distances meaningless (Bellman-Ford's
 *   criterion).  Finite distances must lie strictly between INT32_MIN and
 *   INT32_MAX: a sum at or above INT32_MAX reads as unreachable, a sum at or
 *   below INT32_MIN also makes the run report converged = 0.
 *   DAWN_W_UNIT = every edge weight 1, weights_dev not read (may be NULL):
 *   uint32 hop counts, the unweighted case (each vertex reached once, at its
 *   level, so a level is stored without atomicMin); dawn_msssp / dawn_apsp
 *   run the hop-count tiles of dawn_umsssp_ws; batches and tile sessions
 *   return DAWN_E_UNSUPPORTED.
 * - Distances: uint32 (INF = 0xFFFFFFFF), float32 (INF = +inf) or int32
 *   (INF = INT32_MAX), matching the weight type (uint32 for unit weights).
 * - Pointers named *_dev are DEVICE pointers (hipMalloc'd or torch CUDA
 *   tensors) owned by the caller.  The library never frees them and keeps no
 *   pointer after the call's stream work completes, except tile and batch
 *   sessions, which keep their graph pointers until destroyed.
 * - Every call is stream-ordered and asynchronous: it validates its scalar
 *   arguments on the host, enqueues a fixed sequence of launches on `stream`
 *   and returns; no call waits on the host for device work, so every run can
 *   be captured into a HIP graph.  The return code reports host-side
 *   validation and launch errors only; a device fault surfaces at the
 *   caller's next synchronisation.
 * - A run that ends without reaching its fixed point (dawn_run_info.converged
 *   other than 1) is never silent: with a dawn_run_info the caller reads the
 *   status there; without one (every plain call) the status is recorded on the
 *   device and dawn_run_status reports it once the stream has been
 *   synchronised.
 * - Without a caller workspace, scratch memory is taken with hipMallocAsync
 *   and released with hipFreeAsync on the same stream.
 * - With tuning fields out of range a call returns DAWN_E_INVALID.  Tuning
 *   never changes results: the distances are unique (see above).
 */
#ifndef DAWN_H_
#define DAWN_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DAWN_OK = 0,
  DAWN_E_INVALID = 1,     /* bad argument: n < 1, m < 0, source out of range, k < 1,
                             null pointer, unknown weight type, tuning out of range */
  DAWN_E_UNSUPPORTED = 2, /* valid request this build does not handle (mixed weight
                             types in one batch, k above the tile maximum, ...) */
  DAWN_E_WORKSPACE = 3,   /* caller workspace smaller than dawn_*_workspace_bytes() */
  DAWN_E_HIP = 4,         /* a HIP runtime call failed (allocation, launch) */
  DAWN_E_INCOMPLETE = 5   /* dawn_run_status: a run ended without converging */
} dawn_status;

typedef enum { DAWN_W_U32 = 0, DAWN_W_F32 = 1, DAWN_W_I32 = 2, DAWN_W_UNIT = 3 } dawn_wtype;

/* Device-written run summary (optional output of the *_ws calls).  Counters
 * follow the paper's cost model (Section 3.4: T = mu(s) * E_wcc(s)):
 *   steps            iterations of the step loop, including the final step
 *                    that changes nothing (Algorithm 2's loop count);
 *   converged        1 = stopped after a step with no change; 0 = stopped at
 *                    the n-step cap; -1 = input validation failed on the
 *                    device, or a source id outside [0, n) reached a batched
 *                    run; -2 = a persistent launch gave up waiting at a grid
 *                    barrier (tuning field barrier_ms); -3 = a frontier queue
 *                    overflowed (cannot happen on a valid CSR).  Anything but
 *                    1 means the distances are incomplete;
 *   frontier_entries sum over steps of the frontier rows (changed in the
 *                    previous step and having out-edges);
 *   edges_scanned    sum over steps of the out-degrees of the rows expanded
 *                    (single source with ss_skip: a row lowered again within
 *                    its step is expanded, and counted, in the next step only);
 *   improvements     per step, the vertices whose distance the step lowered
 *                    (two decreases of one vertex in one step count once).
 * For a batched call the counters are summed over its sources and `steps` is
 * the largest per-source step count; union_rows / union_edges count the rows
 * and edges the tile actually read (each serving every source active there);
 * improvements counts, per step, the (vertex, source) pairs whose distance
 * the step lowered (two decreases of one pair in one step count once).  The
 * row and edge counters are taken from the frontier of each step (the same
 * for push and pull steps); with tile_skip = 1 a (row, source) pair lowered
 * again within the step it was to be expanded in is expanded only in the next
 * step, but counted in both.
 * For single-source calls union_rows / union_edges equal frontier_entries /
 * edges_scanned. */
typedef struct {
  int32_t steps;
  int32_t converged;
  int64_t frontier_entries;
  int64_t edges_scanned;
  int64_t improvements;
  int64_t union_rows;   /* batched calls: rows expanded once for all sources */
  int64_t union_edges;  /* batched calls: edges read once for all sources */
} dawn_run_info;

/* Launch tuning, process-wide (set before concurrent use; not thread-safe).
 * Frontier rows are binned by out-degree d into three tiers:
 *   lane tier      d <= t_lane   rows packed 64 per wavefront, one edge per lane
 *                                (single source: taken from a scan of the
 *                                frontier bitmap rather than from a queue);
 *   wave tier      d <= t_wave   one wavefront per row (t_wave >= 64);
 *   workgroup tier d >  t_wave   the row is cut into chunks of t_chunk edges,
 *                                one workgroup per chunk.
 * mode: how the step loop (Algorithm 2's `while`) is launched.  No mode waits
 * on the host: a run is a fixed launch sequence, and a launch that finds the
 * run already ended returns at once.
 *   0 auto: single source and batches of graphs run in one workgroup when
 *     m <= small_m, as mode 1 when m >= step_min_m, else as mode 2; tiles
 *     (dawn_msssp, dawn_apsp, dawn_umsssp_ws) as mode 1;
 *   1 `step_launches` (tiles: `tile_step_launches`) launches of one step
 *     each, then one persistent launch for the steps that remain;
 *   2 one persistent launch for all steps, with a grid barrier between steps.
 * A persistent launch's grid is what the compute units hold at once, by the
 * kernel's compiled VGPR and LDS use (dawn_device_query); a grid barrier that
 * waits longer than barrier_ms ends the run with converged = -2, never a hang.
 * Tile sessions always take step launches.
 * wg_threads: 256, 512 or 1024, or 0 = auto (single source: 512 for step launches,
 * 1024 for persistent launches; tiles: 256 for step launches, 1024 for
 * persistent launches).  One-workgroup single-source runs
 * of graphs held whole in LDS (n <= 6144 and m <= 16384) always take 1024
 * threads: each thread keeps its share of the edges in registers.
 * grid: workgroups per launch, 0 = auto (persistent: what the device holds at
 * once; tile step launches: 4 per compute unit for the push relaxation (the
 * pull relaxation always takes 16); single-source step launches:
 * 4 per compute unit).
 * tile_k: sources per tile for dawn_msssp / dawn_apsp, a multiple of 64,
 * at most DAWN_TILE_K_MAX. */
typedef struct {
  int32_t t_lane;     /* 1..4096, default 256 */
  int32_t t_wave;     /* max(64,t_lane)..65536, default 2048 */
  int32_t t_chunk;    /* 256..1<<20, default 8192 */
  int32_t wg_threads; /* default 0 (auto) */
  int32_t grid;       /* default 0 (auto) */
  int32_t mode;       /* default 0 (auto) */
  int32_t step_launches; /* single source, mode 1: step launches before the persistent
                            launch, 0..4096, default 20 */
  int32_t tile_k;     /* default 256 */
  int32_t tile_t_wave;  /* workgroup-tier threshold of the tile kernel, 32..65536, default 64 */
  int32_t tile_t_chunk; /* edges per workgroup chunk in the tile kernel, 64..65536, default 256 */
  int32_t validate;     /* 1 = check the CSR on the device before running */
  int32_t coop;         /* 1 = launch persistent kernels with hipLaunchCooperativeKernel
                           (not under graph capture); 0 (default) = an ordinary launch of
                           the same grid */
  int32_t tile_t_group; /* tile rows of out-degree <= this go one per 16-lane group,
                           0..64, default 8 (0: none) */
  int32_t tile_skip;    /* 1: in a tile step, a (row, source) pair whose distance was
                           already lowered again in the same step is not expanded (it is
                           expanded next step with the lower value); 0 (default): every
                           pair of the frontier is expanded, as Algorithm 2 states */
  int32_t small_m;      /* single-source and batch runs with mode 0 and m <= small_m run in
                           one workgroup, one launch (no grid barrier); default 131072,
                           0 = never */
  int32_t step_min_m;   /* mode 0: graphs with at least this many edges start with step
                           launches (see mode); default 1 << 25 */
  int32_t tile_sparse;  /* tile rows (and workgroup chunks) with at most this many active
                           sources are relaxed one edge per lane, 4 bytes per source,
                           instead of 16 lanes per 64-source segment; 0..512, default 8 */
  int32_t tile_pull;    /* with a reverse graph (dawn_msssp_tg_ws), a tile step whose
                           frontier rows hold at least tile_pull / 1000 of the m edges, and
                           whose frontier edges carry on average at least tile_pull_src
                           active sources, is run as a pull step over the in-edges of every
                           vertex; 0 = every step, 1001 = never; default 400 */
  int32_t tile_pull_src; /* see tile_pull: a pull step reads a frontier in-neighbour's whole
                           64-source segments, a push step only its active sources, so tiles
                           holding few queries stay with push; 0..512, default 16 */
  int32_t ss_skip;      /* single source, multi-workgroup launches: 1 = a frontier row that
                           another row lowered again within the step is expanded only in the
                           next step (once, with the lower value); 0 or 1 (default: on
                           R-MAT scale 22 it scans 43 % fewer edges, 16 % faster) */
  int32_t ss_pull;      /* single source with a reverse graph (dawn_sssp_tg_ws), step
                           launches: a step whose frontier rows hold at least ss_pull / 1000
                           of the m edges pulls over the in-edges of every vertex; 1001 =
                           never (default) */
  int32_t tile_step_launches; /* tiles, mode 0 or 1: step launches (each one step, with pull
                           steps on dense frontiers) before the persistent launch that
                           finishes the run, 0..4096, default 16 (R-MAT scale 20 with 256
                           sources takes 15 steps) */
  int32_t barrier_ms;   /* persistent launches: a grid barrier that waits longer than this
                           gives up and ends the run with converged = -2; 0..600000,
                           default 4000 (0: give up at the first wait, for tests) */
  int32_t ss_tail_grid; /* single-source and batch runs: at most this many workgroups in the
                           persistent launch (0 = what the device holds at once).  A persistent
                           launch waits at grid barriers for all of its workgroups; when kernels
                           of other streams may hold compute units meanwhile, 1 keeps it from
                           waiting on workgroups that cannot start (a server's lone queries run
                           with mode 1 and ss_tail_grid 1); default 0 */
} dawn_tuning;

#define DAWN_TILE_K_MAX 512

dawn_status dawn_get_tuning(dawn_tuning* out);
dawn_status dawn_set_tuning(const dawn_tuning* in); /* NULL restores the defaults */

const char* dawn_status_str(dawn_status s);
/* Last error text of this thread (HIP error string or validation message). */
const char* dawn_last_error(void);

/* Status of the runs launched on the current device without a dawn_run_info
 * (every dawn_sssp / dawn_msssp / dawn_apsp call, and the *_ws calls given
 * info = NULL) whose stream work has completed: call it after synchronising
 * those streams.  Returns DAWN_OK when each of them converged (status 1), else
 * DAWN_E_INCOMPLETE with *incomplete_runs = how many did not and
 * *last_status = the dawn_run_info.converged code of the last one; the record
 * is cleared by the call.  Either output pointer may be NULL.  Blocking (it
 * copies two words from the device). */
dawn_status dawn_run_status(int32_t* incomplete_runs, int32_t* last_status);

/* ---------------------------------------------------------------------------
 * Single source (Algorithm 2).  dist_out_dev: n elements (uint32 or float32
 * per wt), fully written.
 * ------------------------------------------------------------------------- */
dawn_status dawn_sssp(const int32_t* rowptr_dev, const int32_t* colidx_dev,
                      const void* weights_dev, dawn_wtype wt, int32_t n, int32_t m,
                      int32_t source, void* dist_out_dev, hipStream_t stream);

/* Bytes of scratch a single-source call needs for this graph. */
size_t dawn_sssp_workspace_bytes(int32_t n, int32_t m);


/* Same, with caller scratch (>= dawn_sssp_workspace_bytes, 256-byte aligned
 * device memory, contents ignored) and an optional DEVICE pointer to a
 * dawn_run_info the device fills. */
dawn_status dawn_sssp_ws(const int32_t* rowptr_dev, const int32_t* colidx_dev,
                         const void* weights_dev, dawn_wtype wt, int32_t n, int32_t m,
                         int32_t source, void* dist_out_dev, void* ws_dev, size_t ws_bytes,
                         dawn_run_info* info_dev, hipStream_t stream);

/* dawn_sssp_ws with the reverse graph of the same CSR (dawn_tgraph_build):
 * step launches whose frontier is dense (tuning field ss_pull) run as pull
 * steps over the in-edges of every vertex, with the same results. */
dawn_status dawn_sssp_tg_ws(const int32_t* rowptr_dev, const int32_t* colidx_dev,
                            const void* weights_dev, dawn_wtype wt, int32_t n, int32_t m,
                            const void* tgraph_dev, int32_t source, void* dist_out_dev,
                            void* ws_dev, size_t ws_bytes, dawn_run_info* info_dev,
                            hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dawn_sssp
 * with its workspace taken from a fixed array of DAWN_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device it runs on until the process ends.
 * The call allocates nothing (no hipMalloc, hipMallocAsync or hipFree, no
 * timing events) and launches the same kernels as dawn_sssp; the kernels clear
 * what must start at zero, so the array's contents from earlier calls do not
 * matter.  Graphs whose dawn_sssp_workspace_bytes exceeds the array return
 * DAWN_E_WORKSPACE before anything is launched (about 8.4 bytes per vertex plus
 * 0.62 bytes per edge: R-MAT scale 22 with 33.5M edges fits).  Every call on a
 * device shares that device's array: calls that overlap on one device (two
 * streams, two threads) race and give wrong distances; order them on one
 * stream.  A run that does not converge is reported by dawn_run_status, as for
 * dawn_sssp. */
#define DAWN_NOALLOC_SCRATCH_BYTES (64u << 20)
dawn_status dawn_sssp_noalloc(const int32_t* rowptr_dev, const int32_t* colidx_dev,
                              const void* weights_dev, dawn_wtype wt, int32_t n, int32_t m,
                              int32_t source, void* dist_out_dev, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Multi source.  sources_dev: int32[k] on the device (duplicates allowed).
 * dist_out_dev: k x n row-major, row j = distances from sources[j].  Sources
 * are processed in tiles of tile_k columns of an [n x tile_k] distance tile,
 * so every edge read from memory serves up to tile_k relaxations.
 * ------------------------------------------------------------------------- */
dawn_status dawn_msssp(const int32_t* rowptr_dev, const int32_t* colidx_dev,
                       const void* weights_dev, dawn_wtype wt, int32_t n, int32_t m,
                       const int32_t* sources_dev, int32_t k, void* dist_out_dev,
                       hipStream_t stream);

size_t dawn_msssp_workspace_bytes(int32_t n, int32_t m, int32_t k);

dawn_status dawn_msssp_ws(const int32_t* rowptr_dev, const int32_t* colidx_dev,
                          const void* weights_dev, dawn_wtype wt, int32_t n, int32_t m,
                          const int32_t* sources_dev, int32_t k, void* dist_out_dev,
                          void* ws_dev, size_t ws_bytes, dawn_run_info* info_dev,
                          hipStream_t stream);

/* All pairs: dist_out_dev is n x n row-major (row s = distances from s).
 * DAWN_E_INVALID if n*n elements overflow size_t. */
dawn_status dawn_apsp(const int32_t* rowptr_dev, const int32_t* colidx_dev,
                      const void* weights_dev, dawn_wtype wt, int32_t n, int32_t m,
                      void* dist_out_dev, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Reverse graph and pull steps (direction-optimising tile steps).
 *
 * Algorithm 2 expands the rows of the frontier (push).  When the frontier's
 * rows hold a large share of the edges, the same relaxations -- every edge
 * (u, v) with u active for a source -- can be done per target v over its
 * in-edges (pull): each v is then written by one wavefront with plain stores,
 * with no atomics.  A pull step needs the reverse graph, built once per graph
 * into an opaque device buffer owned by the caller (layout private to the
 * library; valid while the CSR it was built from is unchanged).  Results are
 * identical with and without pull steps.
 * ------------------------------------------------------------------------- */
size_t dawn_tgraph_bytes(int32_t n, int32_t m);
/* Scratch (device, caller-owned, 256-byte aligned) for one build. */
size_t dawn_tgraph_build_bytes(int32_t n, int32_t m);
/* Build the reverse graph of a valid CSR (rowptr non-decreasing, column ids in
 * [0,n)) into tgraph_dev (256-byte aligned, >= dawn_tgraph_bytes).  Weights
 * are copied as 32-bit patterns, so one reverse graph serves u32 and f32;
 * weights_dev = NULL builds one without weights, for dawn_umsssp_ws only.
 * Stream-ordered; nothing is kept after the call. */
dawn_status dawn_tgraph_build(const int32_t* rowptr_dev, const int32_t* colidx_dev,
                              const void* weights_dev, int32_t n, int32_t m, void* tgraph_dev,
                              size_t tgraph_bytes, void* scratch_dev, size_t scratch_bytes,
                              hipStream_t stream);
/* dawn_msssp_ws with the reverse graph of the same CSR: tile steps whose
 * frontier is dense (see tuning field tile_pull) run as pull steps. */
dawn_status dawn_msssp_tg_ws(const int32_t* rowptr_dev, const int32_t* colidx_dev,
                             const void* weights_dev, dawn_wtype wt, int32_t n, int32_t m,
                             const void* tgraph_dev, const int32_t* sources_dev, int32_t k,
                             void* dist_out_dev, void* ws_dev, size_t ws_bytes,
                             dawn_run_info* info_dev, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Hop counts (every edge weight 1): the unweighted case of the method.  With
 * unit weights each step finds exactly the vertices one hop further, so each
 * shortest path is found once and never changes (mu = 1, Introduction) and a
 * step is the boolean vector-matrix product of Section 3.1 ("Principle") over
 * per-vertex source masks: no distances are read and no atomicMin is needed.
 * dist_out_dev: uint32 [k][n], row j = hop counts from sources[j]
 * (0xFFFFFFFF = unreachable); the values equal dawn_msssp's with all weights
 * 1.  No weights are read.  tgraph_dev: NULL, or the reverse graph of the
 * same CSR (dawn_tgraph_build; weights_dev may be NULL there), with which
 * dense steps run as pull steps that stop reading a vertex's in-edges once
 * all its missing sources are found.  Sources are tiled as in dawn_msssp.
 * A source outside [0, n) ends the call with info.converged = -1 and no
 * distances beyond the initial INF.
 * ------------------------------------------------------------------------- */
size_t dawn_umsssp_workspace_bytes(int32_t n, int32_t m, int32_t k);

/* Bytes of caller scratch the workspace-taking call for this graph, k sources
 * and weight type needs: k = 1, dawn_sssp_ws (= dawn_sssp_workspace_bytes);
 * k > 1, dawn_msssp_ws (= dawn_msssp_workspace_bytes), or for DAWN_W_UNIT the
 * hop-count tiles (= dawn_umsssp_workspace_bytes).  0 for arguments no such
 * call accepts: n < 1, m < 0, k < 1, an unknown weight type, or DAWN_W_I32
 * with k > 1 (signed weights are single-source only).  Host-only. */
size_t dawn_workspace_bytes(int32_t n, int32_t m, int32_t k, dawn_wtype wt);
dawn_status dawn_umsssp_ws(const int32_t* rowptr_dev, const int32_t* colidx_dev, int32_t n,
                           int32_t m, const void* tgraph_dev, const int32_t* sources_dev,
                           int32_t k, uint32_t* dist_out_dev, void* ws_dev, size_t ws_bytes,
                           dawn_run_info* info_dev, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Many graphs in one launch.  A batch concatenates `count` CSR graphs of one
 * weight type into a single disjoint union held in library-owned device memory
 * (vertex ids and edge positions offset by a graph-offset table), so one GOVM
 * run seeded with one source per graph solves all of them at once.  The run
 * can be captured once into a HIP graph and replayed with new sources.
 * ------------------------------------------------------------------------- */
typedef struct dawn_batch dawn_batch;

/* Arrays of `count` device pointers / sizes, read on the host during the
 * call; the graph data is copied, so the caller may free it afterwards. */
dawn_status dawn_batch_create(dawn_batch** out, int32_t count, const int32_t* const* rowptr_devs,
                              const int32_t* const* colidx_devs, const void* const* weight_devs,
                              const int32_t* ns, const int32_t* ms, dawn_wtype wt,
                              hipStream_t stream);
/* Totals of the union: sum of n and of m. */
dawn_status dawn_batch_sizes(const dawn_batch* b, int64_t* total_n, int64_t* total_m);
/* Vertex offset of graph i inside the union (host value). */
int64_t dawn_batch_vertex_offset(const dawn_batch* b, int32_t i);
/* sources_dev: int32[count], LOCAL vertex id of each graph's source.
 * dist_out_dev: total_n elements; graph i's distances start at its vertex
 * offset.  info_dev optional (summed over graphs). */
dawn_status dawn_batch_run(dawn_batch* b, const int32_t* sources_dev, void* dist_out_dev,
                           dawn_run_info* info_dev, hipStream_t stream);
/* Capture dawn_batch_run(b, sources_dev, dist_out_dev, info_dev) into a HIP
 * graph once; dawn_batch_replay launches it again (the device buffers named
 * at capture are re-read, so new source ids written there take effect). */
dawn_status dawn_batch_capture(dawn_batch* b, const int32_t* sources_dev, void* dist_out_dev,
                               dawn_run_info* info_dev, hipStream_t stream);
dawn_status dawn_batch_replay(dawn_batch* b, hipStream_t stream);
void dawn_batch_destroy(dawn_batch* b);

/* ---------------------------------------------------------------------------
 * Tile sessions (continuous batching).  A tile holds per-query distance state
 * for up to k queries on one resident graph as an [n x k] column tile.  Queries
 * are admitted into free columns between runs, advance together one GOVM step
 * at a time, and are read out when done; each column's arithmetic is the same
 * as a lone query's, so results do not depend on what else shares the tile.
 * ------------------------------------------------------------------------- */
typedef struct dawn_tile dawn_tile;

/* Device bytes a tile of k columns needs (its workspace). */
size_t dawn_tile_bytes(int32_t n, int32_t m, int32_t k);
/* k: 1..DAWN_TILE_K_MAX (rounded up to a multiple of 64 internally).
 * ws_dev: the session's device memory, owned by the caller, 256-byte aligned,
 * at least dawn_tile_bytes(n, m, k) bytes; the session keeps it (and the CSR
 * arrays) until dawn_tile_destroy, which frees neither.  The library allocates
 * no device memory for a session.  The tile is reset on `stream`. */
dawn_status dawn_tile_create(dawn_tile** out, const int32_t* rowptr_dev, const int32_t* colidx_dev,
                             const void* weights_dev, dawn_wtype wt, int32_t n, int32_t m,
                             int32_t k, void* ws_dev, size_t ws_bytes, hipStream_t stream);
/* Start query `source` in free column col (0..k-1). */
dawn_status dawn_tile_admit(dawn_tile* t, int32_t col, int32_t source, hipStream_t stream);
/* Attach the reverse graph of the session's CSR (dawn_tgraph_build, with
 * weights), or detach it with NULL: later runs take pull steps on dense
 * frontiers (tuning field tile_pull), with identical results.  The caller
 * keeps the buffer alive while it is attached. */
dawn_status dawn_tile_set_tgraph(dawn_tile* t, const void* tgraph_dev);
/* Run up to max_steps GOVM steps for every admitted column (steps stop early
 * on the device once no column is active).  If done_bits_dev is non-NULL it
 * receives ceil(k/32) uint32 words (bit j of word j/32) with the bits of
 * admitted columns that have finished set. */
dawn_status dawn_tile_run(dawn_tile* t, int32_t max_steps, uint32_t* done_bits_dev,
                          hipStream_t stream);
/* Capture the launches of dawn_tile_run(t, max_steps, done_bits_dev) once into
 * a HIP graph held by the session; dawn_tile_replay enqueues that graph on
 * `stream`, doing what the same dawn_tile_run call does (one graph launch
 * instead of 3 * max_steps + 1 kernel launches, for a server that runs the
 * same step chunk of a tile every tick).  Every run reads its state from
 * device memory, so admissions, evictions and reads between replays are
 * fine.  The graph keeps the tuning, the attached reverse graph and
 * done_bits_dev as they were at capture: capture again after changing them.
 * A new capture replaces the previous one and dawn_tile_destroy frees it:
 * call either only once the replays already enqueued have finished.
 * Replay without a capture: DAWN_E_INVALID. */
dawn_status dawn_tile_capture(dawn_tile* t, int32_t max_steps, uint32_t* done_bits_dev);
dawn_status dawn_tile_replay(dawn_tile* t, hipStream_t stream);
/* Copy column col (n distances) to dist_out_dev; valid once the column is done. */
dawn_status dawn_tile_read(dawn_tile* t, int32_t col, void* dist_out_dev, hipStream_t stream);
/* Per-column step counts (int32[k], k as given to dawn_tile_create) to steps_out_dev. */
dawn_status dawn_tile_steps(dawn_tile* t, int32_t* steps_out_dev, hipStream_t stream);
/* Cancel the query in column col (its column becomes free). */
dawn_status dawn_tile_evict(dawn_tile* t, int32_t col, hipStream_t stream);
void dawn_tile_destroy(dawn_tile* t);

/* Kernel timer for measurement.  While enabled, every main GOVM launch (the
 * persistent kernel, or a run of step launches) is bracketed by HIP events on
 * the stream it runs on.  dawn_kernel_timer(1) clears and starts recording,
 * dawn_kernel_timer(0) stops; dawn_kernel_time waits for the recorded events
 * and returns their summed elapsed milliseconds and how many launches they
 * cover.  Not recorded under HIP graph capture. */
dawn_status dawn_kernel_timer(int32_t enable);
dawn_status dawn_kernel_time(double* total_ms, int32_t* launches);

/* Device query for tuning, about the current device.  `out` is a host array
 * of DAWN_DEVICE_QUERY_LEN:
 *   [0] compute units, [1] cooperative launch supported (0/1),
 *   [2] / [3] workgroups per compute unit the single-source / tile persistent
 *   kernels are launched with at the current wg_threads, [4] / [5] their
 *   persistent grids, [6] device id, [7] wg_threads,
 *   [8] / [9] VGPRs and LDS bytes of the single-source persistent kernel as
 *   compiled, [10] the runtime occupancy API's workgroups per CU for it,
 *   [11] / [12] / [13] the same for the tile persistent kernel,
 *   [14] / [15] workgroups per CU and VGPRs of the hop-count-tile persistent
 *   kernel.
 * The per-CU figure is the smaller of the residency rule applied to the
 * compiled VGPRs and LDS (512 VGPRs per SIMD lane in granules of 8, at most 8
 * waves per SIMD, 4 SIMDs, 160 KiB LDS) and the occupancy API's figure. */
#define DAWN_DEVICE_QUERY_LEN 16
dawn_status dawn_device_query(int32_t* out);

/* Build information: "gfx950 <compile options>". */
const char* dawn_build_info(void);

#ifdef __cplusplus
}
#endif

#endif /* DAWN_H_ */
