/*
 * mapcheck.h -- C ABI of the MI355X (gfx950) MAP accepting-cycle detector.
 *
 * Method (Barnat, Brim, Ceska: "DiVinE-CUDA -- A Tool for GPU Accelerated LTL
 * Model Checking", PDMC 2009, Section 2 "DiVinE CUDA Algorithmics"): detect
 * whether a directed graph with accepting vertices has a cycle through an
 * accepting vertex.  Accepting vertices are ordered; for every vertex the
 * maximal accepting predecessor map(v) is computed by propagating values to
 * a fixpoint, posed as a repeated sparse matrix-vector product.  An accepting
 * vertex that is its own maximal accepting predecessor lies on an accepting
 * cycle; otherwise every accepting vertex that is some vertex's map value loses
 * its accepting flag and the computation restarts, until a cycle is found or no
 * accepting vertex is left.  The paper runs MAP on the transposed graph, so on
 * the generated graph G that callers pass here:
 *
 *   map(v) = max { a accepting : v reaches a along >= 1 edge of G },  0 if none.
 *
 * Conventions shared by every entry point
 *   - Vertex ids are int32 1..n; 0 means "none".  Edge lists, map vectors and
 *     the witness use ids; CSR column arrays hold 0-based vertex indices.
 *   - The order on accepting vertices is numeric id (larger wins).
 *   - Accepting flags are uint8[n]; entry i (nonzero = accepting) is id i+1.
 *   - 1 <= n <= 2^31 - 2 and 0 <= m <= 2^31 - 1, else MAP_ERANGE.
 *   - Pointers marked "device" must be device memory (hipMalloc or a torch
 *     CUDA tensor) of the stated length, owned by the caller.  Apart from the
 *     serving engine (map_engine_create allocates its own queue and control
 *     state, map_engine_destroy frees them) the library never allocates or
 *     frees memory; scratch comes from the caller's workspace `ws` of at least
 *     map_workspace_bytes(n, m, flags) bytes, 256-byte aligned.  Its contents
 *     need no initialisation; one word of it (the iteration-tag epoch of the
 *     packed values) carries over from one map_propagate / map_detect call to
 *     the next on the same workspace, so that values left by an earlier call
 *     never carry a tag of the new call's first iterations.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every
 *     call only enqueues work on it and returns; nothing synchronizes.  Device
 *     outputs are valid once the stream has been synchronized.
 *   - Host-detectable errors (null pointers, sizes, workspace too small) are
 *     returned before anything is enqueued.  Errors found on the device are
 *     written to the device status word and the call itself returns MAP_OK.
 *     A failure of the HIP runtime to launch returns MAP_EDEVICE.
 *   - Calls on different streams with disjoint outputs and workspaces may
 *     run concurrently; the library holds no mutable state besides a per-
 *     device cache of launch limits.
 *   - map_propagate, map_detect, map_lasso, map_trim, map_engine_create and
 *     map_detect_batch (when given a gang array) start their kernels with a
 *     cooperative launch (the workgroups wait for one another).  The HIP runtime may hold such a launch until an earlier one
 *     on the device has ended; and while one process makes cooperative
 *     launches, another process's cooperative launch on the same device has
 *     been refused, which the call reports as MAP_EDEVICE.
 */
#ifndef MAPCHECK_H
#define MAPCHECK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define MAP_OK 0
#define MAP_EINVAL (-1)        /* null pointer or unknown flag bits */
#define MAP_ERANGE (-2)        /* n or m outside the supported range */
#define MAP_ENOSPC (-3)        /* workspace smaller than map_workspace_bytes */
#define MAP_EDEVICE (-4)       /* the HIP runtime refused a launch */
#define MAP_ENOTCONVERGED (-5) /* device: iteration or sweep cap reached */
#define MAP_ERANGE_DEV (-6)    /* device: an edge endpoint outside 1..n */
#define MAP_EBUSY (-7)         /* engine: no free job slot or ticket space */
#define MAP_ENOPATH (-8)       /* lasso: no path from the initial vertex, or no cycle through the witness */
#define MAP_PENDING 1          /* engine: the job has not finished yet */

/* Flags (bitwise or; 0 = automatic choice). */
#define MAP_FLAG_DENSE_ONLY 0x1u /* pull sweeps only: overrides MAP_FLAG_PUSH */
#define MAP_FLAG_NO_TRACE_DIGEST 0x2u /* leave the digest column of the trace 0 */
#define MAP_FLAG_STREAM 0x4u /* never stage the CSR in on-chip memory: stream it every sweep */
#define MAP_FLAG_SYNC_SWEEPS 0x8u /* a grid-wide barrier after every sweep (no asynchronous sweeps) */
#define MAP_FLAG_PUSH 0x10u /* frontier sweeps over the transposed CSR (needs rrow_ptr, rcol) */
/* map_detect, map_detect_batch, engine jobs: stop as soon as some vertex's
 * value equals its own id during a propagation, not only at its fixpoint.
 * Values during a propagation are genuine maximal accepting successors of
 * subsets of the paths, so such a vertex lies on an accepting cycle: the
 * verdict is the same as without the flag, but K can be smaller and the
 * witness (a vertex on an accepting cycle, accepting in A_1) depends on the
 * schedule.  Runs with a grid-wide barrier after every sweep, as if
 * MAP_FLAG_SYNC_SWEEPS were set.  Ignored by map_propagate; MAP_EINVAL together
 * with MAP_FLAG_PUSH (unless MAP_FLAG_DENSE_ONLY is set as well). */
#define MAP_FLAG_EARLY 0x20u
/* map_propagate, map_detect: when every workgroup streams its rows (the graph
 * is too large for the rows to be staged on chip, or MAP_FLAG_STREAM is set)
 * and frontier sweeps and MAP_FLAG_EARLY are not used, the sweeps run with a
 * grid barrier after each and gather a successor's value only if it grew in
 * the previous sweep (bitmaps of one bit per vertex in the workspace); the
 * results are the same.  This flag turns that filter off (the previous
 * control applies: asynchronous unless MAP_FLAG_SYNC_SWEEPS). */
#define MAP_FLAG_NO_FILTER 0x40u
/* map_propagate, map_detect: direction switch of the filtered sweeps above
 * (push or pull by frontier size, after direction-optimizing breadth-first
 * search).  A sweep whose previous sweep grew fewer than n/16 rows runs as a
 * push round instead: each row that grew raises its predecessors, read from
 * the transposed CSR, with an atomic max; larger frontiers keep the pull over
 * every row.  The results are the same.  A push round costs a chain of
 * dependent device-scope atomics (tens of microseconds), so it pays on large
 * graphs (config 3, 134M edges: detect twice as fast) and not on small ones
 * (a 4M-edge graph forced to stream: 1.6x slower).  Needs rrow_ptr and rcol
 * (else MAP_EINVAL); MAP_EINVAL with MAP_FLAG_PUSH; ignored with
 * MAP_FLAG_DENSE_ONLY and wherever the filtered sweeps do not run. */
#define MAP_FLAG_DIRECTION 0x80u

/* Result of map_propagate / map_detect, written to device memory (32 bytes). */
typedef struct map_result {
  int32_t found;          /* 1 if an accepting cycle was detected, else 0 */
  int32_t witness;        /* largest id v with map(v) == v in the last iteration, else 0 */
  int32_t iterations;     /* K: number of fixpoint computations made */
  int32_t status;         /* MAP_OK, MAP_ENOTCONVERGED */
  int64_t sweeps;         /* whole-graph propagation sweeps, summed over the iterations; those
                             of one iteration are the sum of every workgroup's sweeps over the
                             number of workgroups, rounded (schedule dependent; in barrier mode
                             every workgroup's count) */
  int32_t accepting_left; /* number of accepting vertices at exit */
  int32_t reserved;
} map_result;

/*
 * Bytes of device workspace that map_build_csr, map_propagate and map_detect
 * need for a graph with n vertices and m edges (host only, no side effects).
 * Returns 0 when n or m is out of range.
 */
size_t map_workspace_bytes(int32_t n, int64_t m, uint32_t flags);

/*
 * CSR of the graph from its edge list (the paper's adjacency matrix in
 * compressed sparse row form, built by the tool before propagation; Section 2).
 *   src, dst   device int32[m]: edge src[i] -> dst[i] of G, ids 1..n.
 *   row_ptr    device int32[n+1] out: row v (0-based) of the pull CSR lists the
 *              successors of vertex v+1 in col[row_ptr[v] .. row_ptr[v+1]).
 *   col        device int32[m] out: 0-based successor indices.
 *   rrow_ptr,  device int32[n+1] / int32[m] out, or both NULL: the transposed
 *   rcol       CSR (row v lists the predecessors of vertex v+1), used by the
 *              frontier sweeps (MAP_FLAG_PUSH).
 *   status     device int32 out: MAP_OK, or MAP_ERANGE_DEV if an id lies
 *              outside 1..n (the CSR contents are then unspecified).
 * Duplicate edges and self-loops are kept.  The columns of each row follow
 * the order of their edges in src/dst, so the CSR is the same on every run.
 * Each orientation is built by one of two paths, chosen on the device from a
 * sample of neighbouring edges: per-row cursors (one atomic per run of equal
 * keys) with a pass that orders the rows, when the list is mostly grouped by
 * key; otherwise a stable radix sort by key (from 2^20 edges).  The workspace
 * holds four per-edge int32 arrays (16m bytes) beside the per-vertex arrays.
 */
int map_build_csr(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t *row_ptr,
                  int32_t *col, int32_t *rrow_ptr, int32_t *rcol, int32_t *status, void *ws,
                  size_t ws_bytes, void *stream);

/*
 * One fixpoint of the value propagation (Section 2: every vertex keeps the
 * largest accepting value that reached it through a successor; repeat until no
 * value improves), for a given accepting set.
 *   row_ptr, col    device pull CSR from map_build_csr.
 *   rrow_ptr, rcol  device transposed CSR, or NULL.  With MAP_FLAG_PUSH the
 *                   fixpoint runs in frontier rounds over it (each vertex
 *                   whose value grew raises its predecessors with an atomic
 *                   max; one grid barrier per round) instead of pull sweeps;
 *                   MAP_EINVAL if the flag is given without it.
 *   accepting       device uint8[n], not modified.
 *   map_out         device int32[n] out: map(v) for id v at index v-1.
 *   result          device map_result out: sweeps and status (found, witness
 *                   and iterations are 0).
 */
int map_propagate(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *rrow_ptr,
                  const int32_t *rcol, const uint8_t *accepting, int32_t *map_out, map_result *result,
                  uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/*
 * The MAP outer loop (Section 2), entirely on the device: for k = 1, 2, ...
 * compute map_k for the accepting set A_k; if some v has map_k(v) == v report a
 * cycle (witness = the largest such v); otherwise remove the accepting flag of
 * every nonzero map_k value and continue.  The loop stops when a cycle is
 * found, when no accepting vertex is left, or when no flag was removed (every
 * map value is 0, so no accepting cycle exists).
 *   accepting0     device uint8[n]: A_1, not modified.
 *   result         device map_result out.
 *   trace          device uint64[trace_cap][3] out, or NULL: row k-1 holds
 *                  { |Del_k| (flags removed after iteration k; 0 when it found a
 *                  cycle or removed none), whole-graph sweeps of iteration k
 *                  (counted as in map_result.sweeps), digest of
 *                  map_k = sum over v of mix64((v << 32) | map_k(v)) mod 2^64,
 *                  mix64 the SplitMix64 finalizer }.  Rows beyond trace_cap are
 *                  dropped.
 *   accepting_out  device uint8[n] out, or NULL: the accepting set at exit.
 *   max_iterations >= 1 caps K (status MAP_ENOTCONVERGED when reached);
 *                  <= 0 means no cap (K <= |A_1| always holds).
 */
int map_detect(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *rrow_ptr,
               const int32_t *rcol, const uint8_t *accepting0, map_result *result, uint64_t *trace,
               int32_t trace_cap, uint8_t *accepting_out, int32_t max_iterations, uint32_t flags, void *ws,
               size_t ws_bytes, void *stream);

/* map_detect without a workspace and without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * errors as map_detect, except:
 *   - scratch is a fixed array in the library's device memory (about 21 MB on
 *     every device that calls this, held until the process ends) instead of a
 *     workspace; n above MAP_NOALLOC_MAX_N is MAP_ERANGE;
 *   - frontier sweeps are not available (no transposed CSR argument):
 *     MAP_FLAG_PUSH without MAP_FLAG_DENSE_ONLY is MAP_EINVAL;
 *   - every call on one device shares that device's array, which keeps the
 *     last call's contents (each call starts from what it initialises): calls
 *     that overlap on one device race, so the caller serializes them (one
 *     stream, or synchronization between streams).
 * The first call on a device looks up the array's device address
 * (hipGetSymbolAddress); no call allocates or frees memory. */
#define MAP_NOALLOC_MAX_N (1 << 22)
int map_detect_noalloc(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint8_t *accepting0,
                       map_result *result, uint64_t *trace, int32_t trace_cap, uint8_t *accepting_out,
                       int32_t max_iterations, uint32_t flags, void *stream);

/* Result of map_lasso (device memory, 32 bytes). */
typedef struct map_lasso_result {
  int32_t status;        /* MAP_OK, MAP_ENOPATH, MAP_ENOSPC (path_cap too small), MAP_ERANGE_DEV, MAP_EDEVICE */
  int32_t stem_len;      /* edges of the path from init to the witness (0 without init); -1 if none */
  int32_t cycle_len;     /* edges of the cycle through the witness; -1 if none or not searched */
  int32_t path_len;      /* ids written to path: stem_len + cycle_len + 1 on MAP_OK, else 0 */
  int64_t edges_scanned; /* edges examined by both searches */
  int32_t levels;        /* breadth-first rounds of both searches */
  int32_t reserved;
} map_lasso_result;

/*
 * Counterexample for a reported cycle, which the paper lists as missing from
 * its tool (Section 5): a lasso made of a shortest path in G from an initial
 * vertex to the witness and a shortest cycle in G through the witness.  Both
 * are found by breadth-first search over the successor rows of the pull CSR
 * that map_detect uses, in one cooperative launch (a grid barrier per round).
 * The two lengths are unique.  Where several shortest paths exist, the one
 * returned is fixed by the edge set alone (not by column order or schedule):
 * walking back from the end of the stem and of the cycle, each step goes to
 * the smallest vertex one breadth-first level closer to the start that has an
 * edge to the current one; of all shortest paths, the one whose vertices read
 * backwards are lexicographically smallest.
 *   row_ptr, col  device pull CSR of G from map_build_csr (row v = successors).
 *   witness       1..n, typically map_result.witness of a found cycle.
 *   init          1..n: the stem starts there; 0 (or == witness): no stem.
 *   path          device int32[path_cap] out, ids: init = s_0, ..., s_S = witness,
 *                 c_1, ..., c_L = witness.  Contents unspecified unless
 *                 result->status == MAP_OK.  May be NULL when path_cap == 0.
 *   result        device map_lasso_result out.  MAP_ENOPATH: init does not
 *                 reach the witness (both lengths -1) or the witness lies on no
 *                 cycle (cycle_len -1); MAP_ENOSPC: path_cap < stem_len +
 *                 cycle_len + 1 (both lengths set, nothing written).
 *   ws            workspace of at least map_workspace_bytes(n, m, 0) bytes; its
 *                 contents from another call are not needed.
 * Host errors: MAP_ERANGE (n), MAP_EINVAL (null pointer, witness or init out
 * of range, path_cap < 0), MAP_ENOSPC (workspace).
 */
int map_lasso(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t witness, int32_t init,
              int32_t *path, int32_t path_cap, map_lasso_result *result, void *ws, size_t ws_bytes,
              void *stream);

/* Result of map_trim (device memory, 16 bytes). */
typedef struct map_trim_result {
  int32_t status;         /* MAP_OK, MAP_ERANGE_DEV (a CSR entry outside 0..n-1), MAP_EDEVICE */
  int32_t kept;           /* vertices kept */
  int32_t accepting_kept; /* accepting vertices kept (0 without accepting flags) */
  int32_t rounds;         /* peeling rounds after the first frontier */
} map_trim_result;

/*
 * Relevance pruning before detection.  The paper's tool keeps in its matrix
 * only the states of components that contain accepting states and runs the
 * detection repeatedly on the part of the graph built so far (Section 2); that
 * reduction needs the property automaton.  Its stand-in on a bare graph:
 * remove, while one exists, a vertex with no remaining predecessor or no
 * remaining successor.  The vertices left form the largest set in which every
 * vertex has a predecessor and a successor inside the set; every cycle lies in
 * it, so MAP on accepting & keep gives the same verdict as on accepting (K and
 * the witness follow the reduced accepting set).  One cooperative launch,
 * peeling in rounds with a grid barrier each.
 *   row_ptr, col      device pull CSR of G (row v = successors), from map_build_csr.
 *   rrow_ptr, rcol    device transposed CSR (row v = predecessors), from map_build_csr.
 *   accepting         device uint8[n] or NULL; accepting_out device uint8[n] out
 *                     (accepting & keep), NULL exactly when accepting is.
 *   keep_out          device uint8[n] out: 1 if the vertex is kept.
 *   result            device map_trim_result out.
 *   ws                workspace of at least map_workspace_bytes(n, m, 0) bytes.
 * Host errors: MAP_ERANGE (n), MAP_EINVAL (null pointer, or only one of
 * accepting / accepting_out), MAP_ENOSPC (workspace).
 */
int map_trim(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *rrow_ptr, const int32_t *rcol,
             const uint8_t *accepting, uint8_t *keep_out, uint8_t *accepting_out, map_trim_result *result,
             void *ws, size_t ws_bytes, void *stream);

/* One graph of a batch (device memory; see map_detect_batch). */
typedef struct map_graph_desc {
  int32_t n;                  /* vertices, ids 1..n */
  int32_t options;            /* 0 = defaults, else an or of the MAP_GRAPH_* bits below */
  int64_t m;                  /* edges */
  const int32_t *row_ptr;     /* device pull CSR from map_build_csr: int32[n+1] */
  const int32_t *col;         /* device int32[m] */
  const uint8_t *accepting0;  /* device uint8[n]: A_1, not modified */
  const int32_t *rrow_ptr;    /* device transposed CSR (row v: predecessors of v) from map_build_csr, or NULL: int32[n+1] */
  const int32_t *rcol;        /* device int32[m], or NULL; read only with MAP_GRAPH_DIRECTION */
} map_graph_desc;

/* map_graph_desc.options.  Low 16 bits: a row with more edges than this in a
 * staged chunk of a streamed tile (512 edges) is folded by the whole wave
 * instead of its own lane (0 = the default, 64).  MAP_GRAPH_SYNC_SWEEPS and
 * MAP_GRAPH_STREAM apply MAP_FLAG_SYNC_SWEEPS / MAP_FLAG_STREAM to this graph
 * alone.  MAP_GRAPH_FILTER runs this graph's gang with filtered stream sweeps
 * (a barrier after every sweep; a sweep gathers only from rows that grew in
 * the one before, as map_detect does when no workgroup can stage its rows on
 * chip); ignored with MAP_FLAG_EARLY.  MAP_GRAPH_DIRECTION, with
 * MAP_GRAPH_FILTER and the graph's transposed CSR in rrow_ptr / rcol, adds the
 * direction switch of MAP_FLAG_DIRECTION (a sweep after one that grew fewer
 * than n / 16 rows runs as push rounds over the transposed CSR); without them
 * it is ignored.  None of them changes a result. */
#define MAP_GRAPH_HUB_MASK 0xffff
#define MAP_GRAPH_SYNC_SWEEPS 0x10000
#define MAP_GRAPH_STREAM 0x20000
#define MAP_GRAPH_FILTER 0x40000
#define MAP_GRAPH_DIRECTION 0x80000

/*
 * Bytes of device workspace for map_detect_batch over `count` graphs whose
 * vertex counts sum to total_n (host only; 0 when out of range).  It holds
 * every graph's scratch with the room MAP_GRAPH_FILTER needs, whatever the
 * options.
 */
size_t map_batch_workspace_bytes(int32_t count, int64_t total_n, uint32_t flags);

/*
 * The MAP outer loop (as map_detect) for many independent graphs in one
 * persistent launch: a device work queue hands each graph to a gang of
 * gang[g] workgroups (clamped to 1..min(256, workgroups in the launch, i.e.
 * one per compute unit); NULL = 1 for every graph), in the order given
 * (put the largest graphs first).  With gang == NULL no workgroup ever waits
 * on another, so the launch is an ordinary one and can be captured in a HIP
 * graph; otherwise it is a cooperative launch.
 *   graphs   device map_graph_desc[count].
 *   gang     device int32[count] or NULL.
 *   results  device map_result[count] out (as map_detect, one per graph).
 *   total_n  sum of graphs[g].n (sizes the scratch; checked on the device,
 *            every result gets MAP_ENOSPC if it does not fit).
 */
int map_detect_batch(int32_t count, const map_graph_desc *graphs, const int32_t *gang, map_result *results,
                     int64_t total_n, uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/*
 * Serving engine: one persistent launch that takes jobs while it runs.
 *
 * The MAP outer loop of map_detect, for graphs that arrive while others are
 * being checked (continuous batching).  map_engine_create launches a
 * cooperative kernel that stays on the device until map_engine_stop; the host
 * posts jobs into fine-grained host memory and the kernel's workgroups pick
 * them up as they free up, so a job submitted while others run starts on the
 * workgroups the earlier jobs release, with no new launch.  Each job is an edge
 * list: its gang of workgroups builds the pull CSR (as map_build_csr, up to the
 * order of the columns inside a row) and runs
 * the MAP loop on it (as map_detect, without trace, accepting_out or iteration
 * cap); the result is written to host memory.  The edge list and flags may stay
 * in pinned host memory (hipHostMalloc, torch pin_memory): the engine reads
 * them over the bus itself, so no copy has to run beside it.
 *
 * While the engine runs it occupies all but `cus / 32` compute units (by
 * default): other kernels on the device run on the rest, or wait for the
 * engine to stop.  Calls on one engine must come from one host thread.
 */
typedef struct map_engine map_engine;

/* One job of the engine; the engine reads it when the job starts. */
typedef struct map_job {
  int32_t n;                  /* vertices, ids 1..n */
  int32_t gang;               /* workgroups for this graph; clamped to 1..min(256, engine workgroups) */
  int64_t m;                  /* edges */
  const int32_t *src;         /* int32[m]: edge src[i] -> dst[i], ids 1..n (device or pinned host) */
  const int32_t *dst;         /* int32[m] (device or pinned host) */
  int32_t *row_ptr;           /* device int32[n+1] out: pull CSR (as map_build_csr) */
  int32_t *col;               /* device int32[m] out (column order inside a row unspecified) */
  const uint8_t *accepting0;  /* uint8[n]: A_1, not modified (device or pinned host) */
  void *scratch;              /* device, map_job_scratch_bytes(n, m) bytes, 256-byte aligned */
  uint64_t tag;               /* free for the caller; not read by the engine */
} map_job;

/* Bytes of device scratch one job needs (0 when n or m is out of range): the
 * packed values and working flags (5n), the filtered sweeps' four bitmaps
 * (n / 2), scan partials, a staged copy of a host edge list (8m) and the
 * transposed CSR (4n + 4m) that MAP_FLAG_DIRECTION builds. */
size_t map_job_scratch_bytes(int32_t n, int64_t m);

/*
 * Start an engine on the current device.
 *   max_jobs      1..65536 jobs in flight (submitted, not yet polled as done).
 *   workgroups    0 = all but one compute unit in 32; else at most that many.
 *   idle_seconds  the kernel exits by itself after this long without a job
 *                 (every later submit returns MAP_EDEVICE); (0, 86400].
 *   flags         MAP_FLAG_STREAM / MAP_FLAG_SYNC_SWEEPS as for map_detect;
 *                 MAP_FLAG_DIRECTION: each job also builds the transposed CSR
 *                 of its graph in its scratch and runs filtered stream sweeps
 *                 with the direction switch (MAP_GRAPH_FILTER |
 *                 MAP_GRAPH_DIRECTION of a batch); no result changes.
 *   stream        the engine kernel's stream; keep other work off it.
 *   out           the engine handle.
 * Returns MAP_EDEVICE when allocation or the launch fails.
 */
int map_engine_create(int32_t max_jobs, int32_t workgroups, double idle_seconds, uint32_t flags, void *stream,
                      map_engine **out);

/* Workgroups of the engine launch (0 for NULL). */
int map_engine_workgroups(const map_engine *e);

/*
 * Post a job.  Every buffer it names must hold its final contents (copies into
 * src, dst and accepting0 complete) and stay allocated until the job is polled
 * as done.  src, dst and accepting0 must be device memory or pinned host
 * memory; row_ptr, col and scratch device memory; anything else (pageable
 * host memory, unknown pointers) is rejected with MAP_EINVAL before the engine
 * sees the job.  *slot identifies the job for map_engine_poll.  Returns
 * MAP_EBUSY when max_jobs jobs are in flight or the ticket ring is full (poll
 * finished jobs, then retry), MAP_EDEVICE when the engine has exited,
 * MAP_EINVAL / MAP_ERANGE for bad arguments or after map_engine_stop.
 */
int map_engine_submit(map_engine *e, const map_job *job, int32_t *slot);

/*
 * Non-blocking completion check.  MAP_PENDING while the job runs; MAP_OK when
 * it has finished, with its map_result copied to *out (status MAP_OK, or
 * MAP_ERANGE_DEV for an edge outside 1..n, or MAP_EDEVICE) and the slot freed;
 * MAP_EDEVICE (slot freed) when the engine exited without running it.
 */
int map_engine_poll(map_engine *e, int32_t slot, map_result *out);

/* Ask the engine to exit once every submitted job has started (returns at once). */
int map_engine_stop(map_engine *e);

/* Stop, wait until the kernel has exited, and free the engine. */
int map_engine_destroy(map_engine *e);

/* Measurement build only (libmapcheck_phases.so, compiled with
 * -DMAPCHECK_PHASES): per-workgroup phase clocks of the last map_propagate /
 * map_detect launch, 16 uint64 per workgroup in workgroup order: device
 * wall-clock ticks (100 MHz) spent in set-up, remote passes, LDS passes,
 * streamed tiles, change reports (barriers in barrier mode), waiting for work,
 * detect and strip (with its barrier), and the rest; then the counts of sweeps,
 * LDS passes, quiet sweeps and iterations; then the ticks spent waiting, after
 * a resident remote pass, for the workgroup's other waves to finish theirs;
 * the ticks of the gather part of asynchronous resident remote passes (the
 * rest of those passes, clearing and row updates, stays in the second word);
 * 2 words unused.  Copies
 * min(*blocks, max_blocks) workgroups to host memory `out` (synchronous, after
 * the launch has finished) and sets *blocks to the launch's workgroup count.
 * MAP_EINVAL in the normal build. */
int map_phase_counters(uint64_t *out, int32_t max_blocks, int32_t *blocks);

/* Static description of a status code. */
const char *map_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* MAPCHECK_H */
