// MAP accepting-cycle detection for MI355X (gfx950, CDNA4): HIP kernels and
// the C ABI declared in include/mapcheck.h.
//
// Method: Barnat, Brim, Ceska, "DiVinE-CUDA", PDMC 2009, Section 2.  MAP runs on
// the transposed state graph, so on the generated graph G a vertex v keeps
//   map(v) = max{ a accepting : v reaches a along >= 1 edge },
// the least fixpoint of  map(v) = max over edges v->w of max(map(w), [w in A]*w),
// computed by repeated sparse (max, id) matrix-vector products ("sweeps") over
// the pull CSR of G (row v = successors of v).  The fixpoint is unique, so any
// monotone schedule -- in place, stale reads across workgroups, any order --
// reaches the same vector; only the sweep count depends on the schedule.
//
// Device data layout (workspace):
//   ctrl   control block: grid-barrier counters, per-epoch reduction slots,
//          the asynchronous change counter and quiet reports, and the
//          iteration-tag epoch kept across calls;
//   pv     uint32[n]: bit 31 = vertex is accepting in the current iteration,
//          low bits (the bit length of n) = current map value (id, 0 = none),
//          the bits between = tag of the iteration that wrote the word;
//   accw   uint8[n]: working accepting flags, stripped between iterations;
//   frontier lists, change bitmaps and the CSR build's scratch (see layout()).
//
// One cooperative persistent kernel runs the whole outer loop (reset, sweeps
// to the fixpoint, detect, strip, next iteration) with grid barriers between
// phases; the host enqueues one launch per call and never synchronizes.
// Sweeps pull over the CSR (staged in LDS where a workgroup's slice fits,
// streamed otherwise); on large graphs the streamed sweeps can switch to
// pushing from the rows that grew over the transposed CSR.  The CSR itself is
// built on the device, by per-row cursors or a radix sort.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "mapcheck.h"

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 1024;  // threads per workgroup of the loop kernel (one per CU)
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kTileRows = 128;    // rows per wave tile
constexpr int kTileEdges = 512;   // stream mode: edges staged in LDS per wave (2 KiB)
constexpr int kRowsPerLane = kTileRows / kWave;
constexpr int kEdgesPerLane = kTileEdges / kWave;
constexpr int kResRowsPerLane = 4;                     // resident mode: rows per lane
constexpr int kResWaveRows = kWave * kResRowsPerLane;  // resident mode: rows per wave
constexpr int kResEdges = 24576;                        // resident mode: CSR edges per block in LDS
constexpr int kGatherBatch = 6;                         // resident mode: gathers in flight per lane
constexpr int kLocalPasses = 4;                         // resident mode: LDS-only passes after a sweep
constexpr int kSortSlots = 1024;                        // resident mode: bitonic sort width (>= 64 * kGatherBatch)
constexpr int kSortPerLane = kSortSlots / kWave;
static_assert(kSortSlots >= kWave * kGatherBatch, "sort must cover a gather batch");
constexpr uint32_t kAllFlags =
    MAP_FLAG_DENSE_ONLY | MAP_FLAG_NO_TRACE_DIGEST | MAP_FLAG_STREAM | MAP_FLAG_SYNC_SWEEPS | MAP_FLAG_PUSH |
    MAP_FLAG_EARLY | MAP_FLAG_NO_FILTER |
    MAP_FLAG_DIRECTION;
constexpr uint32_t kAccBit = 0x80000000u;
#ifndef MAPCHECK_PUSH_DIV
#define MAPCHECK_PUSH_DIV 16
#endif
constexpr int kPushDiv = MAPCHECK_PUSH_DIV;  // direction switch: push rounds while the previous sweep grew fewer than n / kPushDiv rows
constexpr int kHubEdges = 64;  // stream tiles: default edges of a row in a staged chunk above which a wave folds it

// Global-memory views of device pointers, for out-of-line functions where the
// address space of a pointer loaded from an argument struct is not inferred.
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) const int32_t g_ci32;
typedef __attribute__((address_space(1))) const uint8_t g_cu8;
constexpr uint32_t kValMask = 0x7fffffffu;
constexpr int kStripes = 16;
constexpr int kSets = 3;
constexpr int kMaxGroups = 8;  // barrier arrival groups (one per XCD)
constexpr int kMaxBlocks = 2048;  // upper bound on the loop kernel's grid
constexpr int kMaxGang = 256;     // upper bound on the blocks that share one graph of a batch
// Bound on one barrier wait, in ticks of the 100 MHz device wall clock (10 s):
// far beyond any legitimate phase, so a broken launch exits instead of hanging.
constexpr uint64_t kWaitTicks = 1000000000ull;
// Bound on the asynchronous sweeping of one fixpoint computation (60 s of
// device wall clock): a sweep loop that has not settled by then (a livelock)
// ends the launch with MAP_EDEVICE instead of running on.
constexpr uint64_t kIterTicks = 6000000000ull;

// ------------------------------------------------------------------ ctrl --

struct alignas(128) Stripe {
  unsigned long long digest;
  unsigned long long sweeps;  // sweeps of the blocks of this stripe in the iteration
  uint32_t count;
  int32_t witness;
  uint32_t nonzero;
  uint32_t pad[25];
};

struct alignas(128) Line64 {
  unsigned long long v;
  unsigned long long pad[15];
};

// Control block of one set of cooperating blocks: the whole grid for a single
// graph, or the gang of blocks that solves one graph of a batch.  Q bounds the
// number of blocks in the set.
template <int Q>
struct alignas(256) CtrlT {
  Line64 grp[kMaxGroups];  // barrier arrivals per group: high 32 = arrivals, low 32 = payload sum
  Line64 top;              // arrivals of the group leaders
  alignas(128) uint32_t gen;       // barrier generation
  uint32_t payload;                // payload sum of the last completed barrier
  int32_t abort;                   // set when a barrier wait exceeded its bound
  uint32_t pad0[29];
  Stripe sets[kSets][kStripes];    // per-epoch reductions
  // Asynchronous fixpoint: change counter, per-block quiet reports
  // {iteration, counter + 1} and the iteration whose fixpoint is established.
  alignas(128) uint32_t dirty;
  uint32_t pad1[31];
  alignas(128) uint32_t done;
  uint32_t pad2[31];
  alignas(128) uint32_t fcount[2];  // push and lasso: entries appended to frontier 0 / 1
  uint32_t hit;                     // lasso: smallest vertex whose edge reached the target, or kNoHit
  uint32_t bad;                     // lasso and trim: an edge endpoint outside 0..n-1 was read
  unsigned long long scanned;       // lasso: edges examined
  uint32_t kept;                    // trim: vertices kept
  uint32_t acc_kept;                // trim: accepting vertices kept
  uint32_t early;                   // MAP_FLAG_EARLY: largest id seen equal to its own value (0: none)
  uint32_t pad3[23];
  unsigned long long quiet[Q];
};
using Ctrl = CtrlT<kMaxBlocks>;
using GangCtrl = CtrlT<kMaxGang>;
constexpr size_t kCtrlBytes = 32768;
// The last line of a single graph's control region holds the tag epoch, which
// outlives the call (the per-call clear stops before it): the first iteration
// tag of a call follows the last one of the previous call on the workspace.
constexpr size_t kEpochOff = kCtrlBytes - 256;
static_assert(sizeof(Ctrl) <= kEpochOff, "ctrl block too large");
constexpr size_t kGangCtrlBytes = sizeof(GangCtrl);
// Arrays of control blocks are indexed with GangCtrl pointers and cleared in
// kGangCtrlBytes units: the two strides must agree.
static_assert(kGangCtrlBytes % 256 == 0, "control blocks are 256-byte multiples");

// Completes this wave's global writes before a workgroup barrier after which
// the workgroup's leader publishes them to other workgroups (an agent-scope
// release, then an atomic).  On gfx950 a workgroup-scope release waits only
// for LDS operations (the waves of a workgroup share one CU's L1), and the
// leader's agent-scope release -- an L2 write-back (`buffer_wbl2 sc1`) and a
// wait on the leader's own wave's memory operations -- is documented to order
// only that wave's operations.  Waiting here for every vector memory operation
// of every wave (`s_waitcnt vmcnt(0)`: each store acknowledged by L2) puts all
// of them in L2 before the barrier, so the leader's write-back that follows the
// barrier covers them.
__device__ __forceinline__ void wave_writes_done() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0x0F70);  // gfx9 encoding of vmcnt(0), expcnt and lgkmcnt left at their maxima
}

__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------- wave reductions --

// Max over the 64 lanes with DPP row operations (GFX9 row_bcast), result in
// every lane.
__device__ __forceinline__ int wave_max_i32(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x141, 0xF, 0xF, false));  // row_half_mirror
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x140, 0xF, 0xF, false));  // row_mirror
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x142, 0xA, 0xF, false));  // row_bcast:15
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(x, 63);
}

// Max over the 64 lanes of values below 2^31 (map values and ids), result in
// every lane: the same DPP row operations as wave_max_i32.
__device__ __forceinline__ uint32_t wave_max_u31(uint32_t x) { return (uint32_t)wave_max_i32((int)x); }

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// SplitMix64 finalizer (Steele, Lea & Flood, OOPSLA 2014), the per-vertex term
// of the order-independent map digest.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ------------------------------------------------------------ grid barrier --

template <typename C>
struct Grid {
  C* c;
  uint32_t gen;      // generation this block expects to complete next
  int nblocks;
  int group;         // arrival group of this block
  int group_size;    // blocks in this group
  int ngroups;
  int rank;          // index of this block in the set
};

// Grid-wide barrier with a summed 32-bit payload.  Every thread must call it.
// Returns false if the wait exceeded its bound (the kernel must then exit).
//
// Ordering: every wave completes its global writes (wave_writes_done) before
// the workgroup barrier; the block's leader then issues one agent-scope release
// fence before its arrival; the last arrival of a group and the last group
// leader acquire before forwarding; waiters poll with relaxed loads (no cache
// invalidation per poll) and acquire once when the generation moves.
template <typename C>
__device__ bool grid_sync(Grid<C>& g, uint32_t payload, uint32_t* total) {
  __shared__ uint32_t s_total;
  __shared__ int s_ok;
  if (g.nblocks == 1) {
    // A single block: a workgroup barrier orders everything it shares.
    __syncthreads();
    if (threadIdx.x < kStripes) {
      Stripe& s = g.c->sets[(g.gen + 2) % kSets][threadIdx.x];
      __hip_atomic_store(&s.digest, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&s.sweeps, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      st_agent(&s.count, 0u);
      __hip_atomic_store(&s.witness, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      st_agent(&s.nonzero, 0u);
    }
    __syncthreads();
    g.gen++;
    if (total) *total = payload;
    return true;
  }
  wave_writes_done();
  __syncthreads();
  if (threadIdx.x == 0) {
    C* c = g.c;
    int ok = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned long long inc = (1ull << 32) | payload;
    unsigned long long old = __hip_atomic_fetch_add(&c->grp[g.group].v, inc, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    if ((int)(old >> 32) == g.group_size - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const uint32_t gsum = (uint32_t)old + payload;
      __hip_atomic_store(&c->grp[g.group].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      unsigned long long old2 = __hip_atomic_fetch_add(&c->top.v, (1ull << 32) | gsum, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
      if ((int)(old2 >> 32) == g.ngroups - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(&c->top.v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st_agent(&c->payload, (uint32_t)old2 + gsum);
        __hip_atomic_store(&c->gen, g.gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    const uint64_t t0 = wall_clock64();
    while (ld_agent(&c->gen) == g.gen) {
      __builtin_amdgcn_s_sleep(1);
      if (wall_clock64() - t0 > kWaitTicks || ld_agent((const uint32_t*)&c->abort)) {
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (!ok) st_agent((uint32_t*)&c->abort, 1u);
    if (total) s_total = ok ? ld_agent(&c->payload) : 0u;
    s_ok = ok;
  }
  __syncthreads();
  // Epoch E+1 writes set (E+1)%3 and reads set E%3; set (E-1)%3 was last read
  // during epoch E, so block 0 clears it now for epoch E+2.
  if (g.rank == 0 && threadIdx.x < kStripes) {
    Stripe& s = g.c->sets[(g.gen + 2) % kSets][threadIdx.x];
    __hip_atomic_store(&s.digest, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&s.sweeps, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    st_agent(&s.count, 0u);
    __hip_atomic_store(&s.witness, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    st_agent(&s.nonzero, 0u);
  }
  g.gen++;
  if (total) *total = s_total;
  return s_ok != 0;
}

// ------------------------------------------------------------- the kernel --

struct LoopArgs {
  int32_t n;
  int32_t ntiles;
  const int32_t* row_ptr;
  const int32_t* col;
  const uint8_t* acc_in;  // A_1 (detect) or the accepting set (propagate)
  uint32_t* pv;
  uint8_t* accw;
  Ctrl* ctrl;
  map_result* result;
  uint64_t* trace;
  int32_t trace_cap;
  uint8_t* acc_out;
  int32_t* map_out;
  int32_t max_iter;
  int32_t propagate;  // 1: one fixpoint of acc_in, write map_out
  int32_t digest;     // 1: compute the trace digest
  int32_t force_stream;  // 1: never stage the CSR in LDS
  int32_t sync_sweeps;   // 1: a grid barrier after every sweep instead of the asynchronous fixpoint
  uint32_t val_mask;     // bits of a packed word holding the map value
  uint32_t tag_mask;     // bits holding the iteration tag (0: untagged, n >= 2^30)
  uint32_t tag_shift;    // lowest bit of the tag
  uint32_t* epoch;       // single graph: the workspace's tag epoch word (else null)
  int32_t push;          // 1: frontier sweeps over the transposed CSR (barrier per round)
  int32_t early;         // 1: stop once a value equals its own row's id (MAP_FLAG_EARLY)
  const int32_t* rrow_ptr;  // push: transposed CSR (row w = predecessors of w)
  const int32_t* rcol;
  int32_t* front[2];     // push: frontier lists, int32[n] each
  uint32_t* mark;        // push: round in which a vertex last joined a frontier
  // Filtered stream sweeps (every block streams, barrier per sweep): three
  // change bitmaps of one bit per vertex (the rows that grew in a sweep) and
  // the bitmap of the current accepting set; null where no workspace holds them.
  uint32_t* chg;         // [3][words]
  uint32_t* accb;        // [words]
  int64_t words;         // 32-bit words per bitmap
  int32_t filt;          // 1: run the filtered stream kernel
  int32_t dopt;          // filtered stream kernel: small frontiers run as push rounds (transposed CSR, front[])
  int32_t hub;           // stream tiles: rows with more edges in a staged chunk are folded by the whole wave
};

// Row ownership: the rows are cut into one contiguous range per block and,
// inside it, one contiguous range per wave.  A wave is the only writer of the
// packed values of its rows for the whole launch.
//
// Two sweep modes, chosen per block at launch:
//   resident  the block's slice of the CSR (column indices plus, per edge, the
//             row's offset inside its wave) is staged in LDS once; the wave's
//             packed values live in registers; a sweep is one batch of gathers
//             per lane, reduced per row with LDS atomic max.
//   stream    row offsets and column indices are streamed from HBM in tiles of
//             kTileRows rows, gathered values staged in LDS, reduced per row.
struct TileLds {
  int32_t rp[kTileRows + 1];
  uint32_t val[kTileEdges];
};

struct ResLds {
  // Staged edges of each wave: first those to rows of other blocks, as
  // (successor << 8) | row offset in the wave, sorted by successor in gather
  // batches; then those to rows of this block, as successor - block base,
  // grouped by row in row order.
  uint32_t e[kResEdges];
  uint16_t lrow[kWavesPerBlock * kResWaveRows];  // first in-block edge of each row of the block
  uint32_t best[kWavesPerBlock][kResWaveRows];
  uint32_t pv[kWavesPerBlock * kResWaveRows];  // the block's own packed values (row - block base)
};

union BlockLds {
  TileLds tile[kWavesPerBlock];
  ResLds res;
};

struct WaveRows {
  int64_t rb0, rb1;  // rows of this block
  int64_t r0, r1;  // rows of this wave
  int32_t we0, we1;  // resident: edge range of the wave inside the block's LDS slice
  int32_t wr;        // resident: [we0, wr) edges to rows of other blocks, [wr, we1) to rows of this block
  bool resident;
  bool ascending;    // stream: sweep tiles in increasing row order (most edges point to lower rows)
};

// The block's LDS, at namespace scope so that out-of-line sweep functions
// address it directly (LDS instructions, not generic pointers).  In resident
// mode g_lds.res.pv holds the block's own packed values, the only copy a wave
// reads its rows from.
__shared__ BlockLds g_lds;
// MAP_FLAG_EARLY: the largest id of a row of this block whose value equals
// its own id (0: none), found by a scan of the block's rows after each sweep.
__shared__ uint32_t g_early;
// Resident asynchronous bodies: where each wave's edges to other blocks' rows
// start in the staged slice, and the prefix sums of their counts, so that the
// block's remote edges can be shared evenly over its waves.
__shared__ int32_t g_rseg[kWavesPerBlock];
__shared__ int32_t g_rpre[kWavesPerBlock + 1];

#ifdef MAPCHECK_PHASES
// Phase clocks of the loop kernel, in a build made only to measure where the
// time goes (libmapcheck_phases.so): thread 0 of each block adds the device
// wall-clock ticks since its previous mark to the phase a mark names, and counts
// events; the block writes its totals to g_phase_out when it finishes.
enum PhaseSlot {
  kPhSetup, kPhRemote, kPhLocal, kPhStream, kPhReport, kPhWait, kPhDetect, kPhOther,
  kPhSweeps, kPhLocalPasses, kPhQuiet, kPhIters, kPhRemoteWait, kPhGather, kPhSlots = 16
};
__shared__ uint64_t g_ph[kPhSlots];
__shared__ uint64_t g_ph_t;
__device__ uint64_t g_phase_out[kMaxBlocks * kPhSlots];
__device__ __forceinline__ void ph_start() {
  if (threadIdx.x == 0) {
    for (int i = 0; i < kPhSlots; ++i) g_ph[i] = 0;
    g_ph_t = wall_clock64();
  }
}
__device__ __forceinline__ void ph_mark(int slot) {
  if (threadIdx.x == 0) {
    const uint64_t t = wall_clock64();
    g_ph[slot] += t - g_ph_t;
    g_ph_t = t;
  }
}
__device__ __forceinline__ void ph_count(int slot, uint64_t d) {
  if (threadIdx.x == 0) g_ph[slot] += d;
}
__device__ __forceinline__ void ph_store(int b) {
  if (threadIdx.x == 0 && b < kMaxBlocks)
    for (int i = 0; i < kPhSlots; ++i) g_phase_out[(size_t)b * kPhSlots + i] = g_ph[i];
}
#define PH_START() ph_start()
#define PH_MARK(slot) ph_mark(slot)
#define PH_COUNT(slot, d) ph_count((slot), (d))
#define PH_STORE(b) ph_store(b)
#else
#define PH_START() ((void)0)
#define PH_MARK(slot) ((void)0)
#define PH_COUNT(slot, d) ((void)0)
#define PH_STORE(b) ((void)0)
#endif

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Layout of a packed value word for ids 1..n: the value takes the bit length
// of n, the accepting flag bit 31, and the iteration tag the bits between
// (none when n >= 2^30, one bit -- the iteration parity -- when n >= 2^29).
__host__ __device__ inline void word_layout(int32_t n, uint32_t* vmask, uint32_t* tmask, uint32_t* tshift) {
  int vbits = 0;
  while (vbits < 31 && ((uint32_t)n >> vbits) != 0u) ++vbits;
  if (vbits >= 31) {
    *vmask = kValMask;
    *tmask = 0u;
    *tshift = 31u;
    return;
  }
  *vmask = (1u << vbits) - 1u;
  *tmask = kValMask & ~*vmask;
  *tshift = (uint32_t)vbits;
}

// Tag of the words written in iteration k (k >= 1) of a call whose epoch is
// `base`.  With two or more tag bits the tags run through 1 .. 2^T - 1 (tag 0,
// the launch-start clear, is never current), consecutive iterations differ,
// and a call starts right after the tags its predecessor on the workspace
// used; with one bit the tag is the parity of k.
__device__ __forceinline__ uint32_t iter_tag(uint32_t tmask, uint32_t tshift, uint32_t base, int32_t k) {
  if (tmask == 0u) return 0u;
  const uint32_t span = tmask >> tshift;
  if (span == 1u) return (k & 1) ? tmask : 0u;
  return (1u + (base + (uint32_t)k - 1u) % span) << tshift;
}

// Fold of one staged chunk of a stream tile into the maxima of the rows a lane
// owns: a row with at most `hub` edges in the chunk is folded by its own lane;
// each longer row is folded by the whole wave -- every lane takes every 64th of
// its edges, then a DPP max gives the row's maximum to its lane.
template <int kRows>
__device__ __forceinline__ void fold_chunk(const uint32_t* val, const int32_t* lo, const int32_t* hi, int32_t c0,
                                          int cnt, int hub, int lane, uint32_t* best) {
#pragma unroll
  for (int j = 0; j < kRows; ++j) {
    const int b = max(lo[j] - c0, 0), e = min(hi[j] - c0, cnt);
    const bool longrow = e - b > hub;
    uint32_t m = best[j];
    if (!longrow)
      for (int k = b; k < e; ++k) m = max(m, val[k]);
    unsigned long long lr = __ballot(longrow);
    while (lr) {
      const int src = __ffsll(lr) - 1;
      lr &= lr - 1;
      const int bb = __shfl(b, src, kWave), ee = __shfl(e, src, kWave);
      uint32_t x = 0;
      for (int k = bb + lane; k < ee; k += kWave) x = max(x, val[k]);
      x = wave_max_u31(x);
      if (lane == src) m = max(m, x);
    }
    best[j] = m;
  }
}

// Value that successor w (0-based) sends along an edge: its map value, or its
// own id if it is accepting and larger.  A word tagged with another iteration
// has not been reset in this iteration yet and sends 0, a valid lower bound
// (its owner's reset sweep then counts as a change, so the reader sweeps again
// once the true value is there).
__device__ __forceinline__ uint32_t sent_word(uint32_t x, int32_t w, uint32_t cur, uint32_t vmask, uint32_t tmask) {
  const uint32_t id = (uint32_t)w + 1u;
  if ((x & tmask) != cur) return 0u;
  const uint32_t m = x & vmask;
  return (x & kAccBit) ? (m > id ? m : id) : m;
}

// What successor w sends in the first sweep of an iteration (map = 0 everywhere).
__device__ __forceinline__ uint32_t sent_first(const uint8_t* acc, int32_t w) {
  return ((g_cu8*)acc)[w] ? (uint32_t)w + 1u : 0u;
}

// Stream mode, rows [r0, r1) with r1 - r0 <= kTileRows, processed by one wave.
// kFirst: the sweep that starts an iteration from map = 0 (successors send their
// id if accepting, every row is written).  Otherwise a row is written only when
// its value grows.  Returns nonzero (wave-uniform) if some row changed.
template <bool kFirst, bool kHub>
__device__ uint32_t sweep_tile(const LoopArgs& a, const uint8_t* acc, int64_t r0, int64_t r1, TileLds& L, int lane,
                               uint32_t cur, uint32_t* acc_count) {
  const int nr = (int)(r1 - r0);
  g_ci32* row_ptr = (g_ci32*)a.row_ptr;
  g_ci32* colp = (g_ci32*)a.col;
  g_u32* pv = (g_u32*)a.pv;
  g_cu8* gacc = (g_cu8*)acc;
  const uint32_t n = (uint32_t)a.n, vmask = a.val_mask, tmask = a.tag_mask;
  for (int i = lane; i <= nr; i += kWave) L.rp[i] = __builtin_nontemporal_load(row_ptr + r0 + i);
  wave_lds_sync();
  const int32_t e0 = L.rp[0], e1 = L.rp[nr];
  int32_t lo[kRowsPerLane], hi[kRowsPerLane];
  uint32_t best[kRowsPerLane], old[kRowsPerLane];
#pragma unroll
  for (int j = 0; j < kRowsPerLane; ++j) {
    int r = lane + j * kWave;
    lo[j] = r < nr ? L.rp[r] : 0;
    hi[j] = r < nr ? L.rp[r + 1] : 0;
    best[j] = 0;
    old[j] = (!kFirst && r < nr) ? pv[r0 + r] : 0u;
  }
  for (int32_t c0 = e0; c0 < e1; c0 += kTileEdges) {
    const int cnt = (int)min((int64_t)kTileEdges, (int64_t)e1 - c0);
    int32_t w[kEdgesPerLane];
#pragma unroll
    for (int u = 0; u < kEdgesPerLane; ++u) {
      int i = lane + u * kWave;
      w[u] = i < cnt ? __builtin_nontemporal_load(colp + c0 + i) : -1;
    }
#pragma unroll
    for (int u = 0; u < kEdgesPerLane; ++u) {
      int i = lane + u * kWave;
      uint32_t x = 0;
      if ((uint32_t)w[u] < n) x = kFirst ? sent_first(acc, w[u]) : sent_word(pv[w[u]], w[u], cur, vmask, tmask);
      if (i < cnt) L.val[i] = x;
    }
    wave_lds_sync();
    if (kHub) {
      fold_chunk<kRowsPerLane>(L.val, lo, hi, c0, cnt, a.hub, lane, best);
    } else {
#pragma unroll
      for (int j = 0; j < kRowsPerLane; ++j) {
        int b = max(lo[j] - c0, 0), e = min(hi[j] - c0, cnt);
        uint32_t m = best[j];
        for (int k = b; k < e; ++k) m = max(m, L.val[k]);
        best[j] = m;
      }
    }
    wave_lds_sync();
  }
  uint32_t changed = 0, nacc = 0;
#pragma unroll
  for (int j = 0; j < kRowsPerLane; ++j) {
    int r = lane + j * kWave;
    if (r < nr) {
      int64_t v = r0 + r;
      if (kFirst) {
        uint32_t isacc = gacc[v] ? 1u : 0u;
        nacc += isacc;
        pv[v] = (isacc << 31) | cur | best[j];
        changed |= (best[j] | isacc) != 0;
      } else if (best[j] > (old[j] & vmask)) {
        pv[v] = (old[j] & ~vmask) | best[j];
        changed = 1;
      }
    }
  }
  if (acc_count) *acc_count += nacc;
  return __ballot(changed) != 0;
}

// Resident mode: one pass over the wave's staged edges to rows of other
// blocks, folding what each successor sends into best[row] with LDS atomic
// max.  kSrc 0: first sweep of an iteration (successors send their id if
// accepting); 1: the successors' packed values, gathered from memory.
template <int kSrc>
__device__ __forceinline__ void gather_range(const uint8_t* acc, int32_t e0, int32_t e1, uint32_t* best,
                                             const LoopArgs& a, int lane, uint32_t cur) {
  ResLds& R = g_lds.res;
  g_u32* pv = (g_u32*)a.pv;
  const uint32_t n = (uint32_t)a.n, vmask = a.val_mask, tmask = a.tag_mask;
  for (int32_t k0 = e0; k0 < e1; k0 += kWave * kGatherBatch) {
    uint32_t e[kGatherBatch];
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u) {
      const int32_t k = k0 + lane + u * kWave;
      e[u] = k < e1 ? R.e[k] : 0xffffffffu;
    }
    uint32_t x[kGatherBatch];
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u) {
      x[u] = 0;
      const uint32_t w = e[u] >> 8;
      if (e[u] != 0xffffffffu && w < n) {
        if (kSrc == 0) x[u] = sent_first(acc, (int32_t)w);
        else x[u] = sent_word(pv[w], (int32_t)w, cur, vmask, tmask);
      }
    }
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u) {
      if (x[u] != 0) atomicMax(&best[e[u] & 0xffu], x[u]);
    }
  }
}

// Resident mode, kBal: the pass over the block's edges to other blocks' rows,
// shared evenly over the block's waves (the waves' staged lists taken as one
// list of g_rpre[16] edges), each value folded with an LDS atomic max into the
// maxima of its row's wave.  Every wave must have cleared its maxima before
// (block barrier), and the rows are updated after another block barrier.
template <int kSrc>
__device__ __forceinline__ void gather_block(const uint8_t* acc, uint32_t* best_all, const LoopArgs& a, int wib,
                                             int lane, uint32_t cur) {
  ResLds& R = g_lds.res;
  g_u32* pv = (g_u32*)a.pv;
  const uint32_t n = (uint32_t)a.n, vmask = a.val_mask, tmask = a.tag_mask;
  const int32_t total = g_rpre[kWavesPerBlock];
  const int32_t share = (total + kWavesPerBlock - 1) / kWavesPerBlock;
  const int32_t lo = min(total, wib * share), hi = min(total, lo + share);
  // The list that holds the wave's first edge (the last one whose prefix sum
  // does not exceed it), found once: a lane's later edges only move forward.
  int w_lo = 0;
  while (w_lo + 1 < kWavesPerBlock && lo >= g_rpre[w_lo + 1]) ++w_lo;
  for (int32_t g0 = lo; g0 < hi; g0 += kWave * kGatherBatch) {
    uint32_t e[kGatherBatch];
    int32_t seg[kGatherBatch];
    int w = w_lo;  // the list a lane's next edge lies in (its edges increase)
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u) {
      const int32_t gi = g0 + lane + u * kWave;
      e[u] = 0xffffffffu;
      seg[u] = 0;
      if (gi < hi) {
        while (gi >= g_rpre[w + 1]) ++w;
        e[u] = R.e[g_rseg[w] + (gi - g_rpre[w])];
        seg[u] = w;
      }
    }
    uint32_t x[kGatherBatch];
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u) {
      x[u] = 0;
      const uint32_t wv = e[u] >> 8;
      if (e[u] != 0xffffffffu && wv < n) {
        if (kSrc == 0) x[u] = sent_first(acc, (int32_t)wv);
        else x[u] = sent_word(pv[wv], (int32_t)wv, cur, vmask, tmask);
      }
    }
#pragma unroll
    for (int u = 0; u < kGatherBatch; ++u) {
      if (x[u] != 0) atomicMax(&best_all[seg[u] * kResWaveRows + (e[u] & 0xffu)], x[u]);
    }
  }
}

// Rows of the wave in the order values travel: a row takes values from its
// successors, so when the block's edges mostly point to higher rows values
// flow downwards and the rows go from high to low.
__device__ __forceinline__ int row_step(const WaveRows& W, int jj) {
  return W.ascending ? jj : kResRowsPerLane - 1 - jj;
}

// Resident mode, edges to rows of this block: every lane folds the successors
// of its own rows from the block's LDS values, row by row in the order values
// travel, so rows raised earlier in the pass are seen later in it.  No
// atomics: a row's in-block edges are contiguous.  Returns nonzero
// (wave-uniform) if some row grew.
__device__ uint32_t local_pass(const LoopArgs& a, const WaveRows& W, int lane, uint32_t cur) {
  ResLds& R = g_lds.res;
  g_u32* pv = (g_u32*)a.pv;
  const uint32_t vmask = a.val_mask, tmask = a.tag_mask, base = (uint32_t)W.rb0;
  const int32_t nrow = (int32_t)(W.r1 - W.r0), r0 = (int32_t)(W.r0 - W.rb0);
  uint32_t changed = 0;
#pragma unroll
  for (int jj = 0; jj < kResRowsPerLane; ++jj) {
    const int32_t i = lane + row_step(W, jj) * kWave;
    if (i < nrow) {
      const int32_t li = r0 + i;
      const int32_t k1 = i + 1 < nrow ? (int32_t)R.lrow[li + 1] : W.we1;
      uint32_t b = 0;
      for (int32_t k = R.lrow[li]; k < k1; ++k) {
        const uint32_t t = R.e[k];
        b = max(b, sent_word(R.pv[t], (int32_t)(base + t), cur, vmask, tmask));
      }
      const uint32_t old = R.pv[li];
      if (b > (old & vmask)) {
        const uint32_t x = (old & ~vmask) | b;
        pv[(int64_t)base + li] = x;
        R.pv[li] = x;
        changed = 1;
      }
    }
  }
  return __ballot(changed) != 0;
}

// kBal: the balanced layout of the resident slice, used by the asynchronous
// bodies.  Its in-block edge entries carry the successor's row offset in the
// block (low 16 bits) and the edge's own row offset in the wave (high 16 bits);
// otherwise an entry is the successor's row offset alone.
__device__ __forceinline__ uint32_t in_succ(uint32_t e) { return e & 0xffffu; }
__device__ __forceinline__ uint32_t in_row(uint32_t e) { return e >> 16; }

// Resident mode, edges to rows of this block, balanced over the lanes (kBal).
// The wave's rows are taken in groups of 64 in the order values travel, so a
// group sees the rows the groups before it raised in the same pass.  A group's
// in-block edges are contiguous (grouped by row) and the lanes share them
// evenly: lane l folds edges l, l + 64, ... into the group's per-row maxima
// with an LDS atomic max, so a row of high degree costs its group a few more
// edges per lane instead of holding up one lane for all of them.  Every
// in-block row carries the current iteration's tag here (the reset sweep wrote
// them all before the first pass), so no tag is compared.  Returns nonzero
// (wave-uniform) if some row grew.
__device__ uint32_t local_pass_bal(const LoopArgs& a, const WaveRows& W, int wib, int lane) {
  ResLds& R = g_lds.res;
  uint32_t* best = R.best[wib];
  g_u32* pv = (g_u32*)a.pv;
  const uint32_t vmask = a.val_mask, base = (uint32_t)W.rb0;
  const int32_t nrow = (int32_t)(W.r1 - W.r0), r0 = (int32_t)(W.r0 - W.rb0);
  uint32_t changed = 0;
  for (int jj = 0; jj < kResRowsPerLane; ++jj) {
    const int32_t g0 = row_step(W, jj) * kWave;  // first row of the group in the wave
    if (g0 >= nrow) continue;                    // wave-uniform
    const int32_t g1 = min(g0 + kWave, nrow);
    const int32_t k0 = R.lrow[r0 + g0];
    const int32_t k1 = g1 < nrow ? (int32_t)R.lrow[r0 + g1] : W.we1;
    best[g0 + lane] = 0;
    wave_lds_sync();
    for (int32_t k = k0 + lane; k < k1; k += kWave) {
      const uint32_t e = R.e[k];
      const uint32_t t = in_succ(e);
      const uint32_t x = R.pv[t];
      const uint32_t m = x & vmask, id = base + t + 1u;
      const uint32_t sv = (x & kAccBit) ? max(m, id) : m;
      if (sv) atomicMax(&best[in_row(e)], sv);
    }
    wave_lds_sync();
    const int32_t i = g0 + lane;
    if (i < g1) {
      const int32_t li = r0 + i;
      const uint32_t b = best[i];
      const uint32_t old = R.pv[li];
      if (b > (old & vmask)) {
        const uint32_t x = (old & ~vmask) | b;
        pv[(int64_t)base + li] = x;
        R.pv[li] = x;
        changed = 1;
      }
    }
    wave_lds_sync();
  }
  return __ballot(changed) != 0;
}

// Resident mode: the pass over the wave's edges to other blocks' rows.
// kFirst: the reset sweep, which also folds the in-block edges (successors
// send their id if accepting) and writes every row.  Otherwise a row is
// written only when its value grows.  Returns nonzero (wave-uniform) if some
// row changed.
template <bool kFirst, bool kBal>
__device__ uint32_t sweep_resident(const LoopArgs& a, const uint8_t* acc, const WaveRows& W, int wib, int lane,
                                   uint32_t cur, uint32_t* acc_count) {
  ResLds& R = g_lds.res;
  uint32_t* best = R.best[wib];
  g_u32* pv = (g_u32*)a.pv;
  g_cu8* gacc = (g_cu8*)acc;
  const uint32_t vmask = a.val_mask, base = (uint32_t)W.rb0;
  const int32_t nrow = (int32_t)(W.r1 - W.r0), r0 = (int32_t)(W.r0 - W.rb0);
#pragma unroll
  for (int j = 0; j < kResRowsPerLane; ++j) best[lane + j * kWave] = 0;
  if (kBal) {
    __syncthreads();  // every wave's maxima cleared before any wave folds into them
    gather_block<kFirst ? 0 : 1>(acc, &R.best[0][0], a, wib, lane, cur);
    if (!kFirst) PH_MARK(kPhGather);
  } else {
    wave_lds_sync();
    gather_range<kFirst ? 0 : 1>(acc, W.we0, W.wr, best, a, lane, cur);
  }
  if (kFirst && kBal) {
    // In-block successors send their id if accepting: folded like the remote
    // edges, shared evenly over the lanes.
    for (int32_t k = W.wr + lane; k < W.we1; k += kWave) {
      const uint32_t e = R.e[k];
      const uint32_t x = sent_first(acc, (int32_t)(base + in_succ(e)));
      if (x) atomicMax(&best[in_row(e)], x);
    }
  }
  if (kBal) __syncthreads();  // every wave's folds into these maxima are done
  else wave_lds_sync();
  uint32_t changed = 0, nacc = 0;
#pragma unroll
  for (int j = 0; j < kResRowsPerLane; ++j) {
    const int32_t i = lane + j * kWave;
    if (i < nrow) {
      const int32_t li = r0 + i;
      const int64_t v = (int64_t)base + li;
      uint32_t b = best[i];
      if (kFirst) {
        if (!kBal) {
          const int32_t k1 = i + 1 < nrow ? (int32_t)R.lrow[li + 1] : W.we1;
          for (int32_t k = R.lrow[li]; k < k1; ++k) b = max(b, sent_first(acc, (int32_t)(base + R.e[k])));
        }
        uint32_t isacc = gacc[v] ? 1u : 0u;
        nacc += isacc;
        const uint32_t x = (isacc << 31) | cur | b;
        pv[v] = x;
        R.pv[li] = x;
        changed |= (b | isacc) != 0;
      } else {
        const uint32_t old = R.pv[li];
        if (b > (old & vmask)) {
          const uint32_t x = (old & ~vmask) | b;
          pv[v] = x;
          R.pv[li] = x;
          changed = 1;
        }
      }
    }
  }
  if (acc_count) *acc_count += nacc;
  return __ballot(changed) != 0;
}

// One sweep of the block's rows.  Every thread of the block calls it.
// Resident mode: the pass over edges to other blocks' rows (every edge in the
// reset sweep), then up to kLocalPasses LDS passes over in-block edges, which
// stop once a pass changes nothing in the block.  *local_fix (block-uniform)
// records that the last LDS pass changed nothing: while it holds and the first
// pass changes nothing, the block's values are at the fixpoint of the values
// gathered, and the LDS passes are skipped.
template <bool kFirst, bool kBal>
__device__ uint32_t sweep_rows(const LoopArgs& a, const uint8_t* acc, const WaveRows W, int wib, int lane,
                               uint32_t cur, uint32_t* acc_count, bool* local_fix) {
  __shared__ uint32_t s_any;
  if (W.resident) {
    uint32_t ch = sweep_resident<kFirst, kBal>(a, acc, W, wib, lane, cur, acc_count);
    PH_MARK(kPhRemote);
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    if (ch && lane == 0) atomicOr(&s_any, 1u);
    __syncthreads();
    const bool run = kFirst || s_any != 0 || !*local_fix;
    *local_fix = false;
    PH_MARK(kPhRemoteWait);
    if (run) {
      for (int p = 0; p < kLocalPasses; ++p) {
        __syncthreads();  // every thread has read s_any; the previous pass's LDS values are complete
        if (threadIdx.x == 0) s_any = 0;
        __syncthreads();
        const uint32_t lc = kBal ? local_pass_bal(a, W, wib, lane) : local_pass(a, W, lane, cur);
        if (lc && lane == 0) atomicOr(&s_any, 1u);
        ch |= lc;
        __syncthreads();
        PH_COUNT(kPhLocalPasses, 1);
        if (s_any == 0) {
          *local_fix = true;
          break;
        }
      }
    } else {
      *local_fix = true;
    }
    __syncthreads();  // every thread has read s_any
    PH_MARK(kPhLocal);
    return ch;
  }
  uint32_t ch = 0;
  if (W.r1 > W.r0) {
    // Tiles in the order values travel: a row takes values from its
    // successors, so when most edges point to higher rows values flow from
    // high ids to low and the tiles go downwards, otherwise upwards; a tile
    // then sees the values its neighbours produced earlier in the same sweep.
    const int64_t last = W.r0 + ((W.r1 - W.r0 - 1) / kTileRows) * kTileRows;
    if (W.ascending) {
      for (int64_t t0 = W.r0; t0 <= last; t0 += kTileRows)
        ch |= sweep_tile<kFirst, kBal>(a, acc, t0, min(W.r1, t0 + kTileRows), g_lds.tile[wib], lane, cur, acc_count);
    } else {
      for (int64_t t0 = last; t0 >= W.r0; t0 -= kTileRows)
        ch |= sweep_tile<kFirst, kBal>(a, acc, t0, min(W.r1, t0 + kTileRows), g_lds.tile[wib], lane, cur, acc_count);
    }
  }
  PH_MARK(kPhStream);
  return ch;
}

// Appends v (where take) to frontier F with one counter update per wave;
// returns the number appended by the wave (wave-uniform).
__device__ __forceinline__ uint32_t frontier_append(int32_t* F, uint32_t* cnt, bool take, int32_t v, int lane) {
  const uint64_t m = __ballot(take);
  if (m == 0) return 0;
  const int first = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if (lane == first) base = __hip_atomic_fetch_add(cnt, (uint32_t)__popcll(m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  base = (uint32_t)__shfl((int)base, first, kWave);
  const uint64_t below = lane ? (~0ull >> (kWave - lane)) : 0ull;
  if (take) F[base + (uint32_t)__popcll(m & below)] = v;
  return (uint32_t)__popcll(m);
}

// Sets, with one atomic per 32-bit word, the bits of bitmap `mark` for the
// rows v0 + l (l = 0..63) whose lane l is set in m (wave-uniform m).
__device__ __forceinline__ void mark_rows(uint32_t* mark, int64_t v0, unsigned long long m, int lane) {
  if (m == 0) return;
  const uint32_t sh = (uint32_t)(v0 & 31);
  const int64_t w0 = v0 >> 5;
  const unsigned long long lo = m << sh;
  uint32_t part = 0;
  if (lane == 0) part = (uint32_t)lo;
  else if (lane == 1) part = (uint32_t)(lo >> 32);
  else if (lane == 2) part = sh ? (uint32_t)(m >> (64 - sh)) : 0u;
  if (part) atomicOr(&mark[w0 + lane], part);
}

__device__ __forceinline__ bool bit_set(const uint32_t* b, uint32_t v) { return (b[v >> 5] >> (v & 31)) & 1u; }

// Filtered stream mode (every block streams its rows, a grid barrier after
// every sweep): like sweep_tile, but an edge's successor w is gathered only if
// its bit is set in `keep` -- in the reset sweep the accepting set (w sends its
// id), later the rows that grew in the previous sweep (w sends its value).  A
// successor left out either sends nothing new (not accepting) or has not grown
// since the previous sweep, whose rows already folded in its value: the
// fixpoint is unchanged.  The rows that grow (in the reset sweep: that get a
// nonzero value) are set in `mark` for the next sweep.  Returns the rows that
// grew (the wave's count).
template <bool kFirst>
__device__ uint32_t sweep_tile_filt(const LoopArgs& a, const uint8_t* acc, int64_t r0, int64_t r1, TileLds& L,
                                    int lane, uint32_t cur, uint32_t* acc_count, const uint32_t* keep,
                                    uint32_t* mark) {
  const int nr = (int)(r1 - r0);
  g_ci32* row_ptr = (g_ci32*)a.row_ptr;
  g_ci32* colp = (g_ci32*)a.col;
  g_u32* pv = (g_u32*)a.pv;
  g_cu8* gacc = (g_cu8*)acc;
  const uint32_t n = (uint32_t)a.n, vmask = a.val_mask, tmask = a.tag_mask;
  for (int i = lane; i <= nr; i += kWave) L.rp[i] = __builtin_nontemporal_load(row_ptr + r0 + i);
  wave_lds_sync();
  const int32_t e0 = L.rp[0], e1 = L.rp[nr];
  int32_t lo[kRowsPerLane], hi[kRowsPerLane];
  uint32_t best[kRowsPerLane], old[kRowsPerLane];
#pragma unroll
  for (int j = 0; j < kRowsPerLane; ++j) {
    int r = lane + j * kWave;
    lo[j] = r < nr ? L.rp[r] : 0;
    hi[j] = r < nr ? L.rp[r + 1] : 0;
    best[j] = 0;
    old[j] = (!kFirst && r < nr) ? pv[r0 + r] : 0u;
  }
  for (int32_t c0 = e0; c0 < e1; c0 += kTileEdges) {
    const int cnt = (int)min((int64_t)kTileEdges, (int64_t)e1 - c0);
    uint32_t w[kEdgesPerLane];
#pragma unroll
    for (int u = 0; u < kEdgesPerLane; ++u) {
      int i = lane + u * kWave;
      w[u] = i < cnt ? (uint32_t)__builtin_nontemporal_load(colp + c0 + i) : 0xffffffffu;
    }
#pragma unroll
    for (int u = 0; u < kEdgesPerLane; ++u) {
      int i = lane + u * kWave;
      uint32_t x = 0;
      if (w[u] < n && bit_set(keep, w[u])) x = kFirst ? w[u] + 1u : sent_word(pv[w[u]], (int32_t)w[u], cur, vmask, tmask);
      if (i < cnt) L.val[i] = x;
    }
    wave_lds_sync();
    fold_chunk<kRowsPerLane>(L.val, lo, hi, c0, cnt, a.hub, lane, best);
    wave_lds_sync();
  }
  uint32_t grown = 0, nacc = 0;
#pragma unroll
  for (int j = 0; j < kRowsPerLane; ++j) {
    int r = lane + j * kWave;
    bool grew = false;
    if (r < nr) {
      int64_t v = r0 + r;
      if (kFirst) {
        uint32_t isacc = gacc[v] ? 1u : 0u;
        nacc += isacc;
        pv[v] = (isacc << 31) | cur | best[j];
        grew = best[j] != 0;
      } else if (best[j] > (old[j] & vmask)) {
        pv[v] = (old[j] & ~vmask) | best[j];
        grew = true;
      }
    }
    const unsigned long long gm = __ballot(grew);
    mark_rows(mark, r0 + j * kWave, gm, lane);
    grown += (uint32_t)__popcll(gm);
  }
  if (acc_count) *acc_count += nacc;
  return grown;
}

// Lane of this wave whose slice of the combined list holds slot q: the last
// lane whose first slot is <= q (binary search over the lanes with shuffles;
// every lane of the wave must call it).
__device__ __forceinline__ int slot_owner(uint32_t q, uint32_t first) {
  int lo = 0;
#pragma unroll
  for (int step = kWave / 2; step > 0; step >>= 1) {
    const uint32_t f = (uint32_t)__shfl((int)first, lo + step, kWave);
    if (f <= q) lo += step;
  }
  return lo;
}

// Filtered stream mode, direction switch (dopt): a sweep whose frontier (the
// rows that grew in the previous sweep, set in `keep`) is small runs as a
// push round over the transposed CSR instead of a pull over every row.  A
// wave takes 64 words of `keep` at a time and deals their set rows out to its
// lanes; a lane raises each predecessor v of its row w with an atomic max of
// what w sends, behind v's
// own accepting bit and the iteration tag (the reset sweep wrote every row
// with both, so the words compare by value); a predecessor that grows is set
// in `mark`.  A row with more than kPushHub predecessors is queued in LDS and
// pushed by the whole wave after the step (64 predecessors at a time), so it
// does not hold up its wave.  The result is that of the filtered pull: both
// fold, into each row, what its grown successors send.  Returns the wave's
// count of raises that grew a row (a row raised twice counts twice: an upper
// bound on the next frontier, zero exactly when nothing grew).
constexpr int32_t kPushHub = 64;
__shared__ int32_t g_hubq[kWavesPerBlock][kWave];
__shared__ uint32_t g_hubn[kWavesPerBlock];

__device__ __forceinline__ bool push_raise(const LoopArgs& a, uint32_t* mark, int32_t v, uint32_t x, uint32_t cur) {
  if ((uint32_t)v >= (uint32_t)a.n) return false;
  const uint32_t word = (bit_set(a.accb, (uint32_t)v) ? kAccBit : 0u) | cur | x;
  const uint32_t old = __hip_atomic_fetch_max(&a.pv[v], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((old & a.val_mask) >= x) return false;
  atomicOr(&mark[v >> 5], 1u << (v & 31));
  return true;
}

__device__ __forceinline__ uint32_t push_round_filt(const LoopArgs& a, const uint32_t* keep, uint32_t* mark,
                                                    uint32_t cur, int64_t gw, int64_t nw, int wib, int lane) {
  g_u32* pvg = (g_u32*)a.pv;
  g_ci32* rrow = (g_ci32*)a.rrow_ptr;
  g_ci32* rcol = (g_ci32*)a.rcol;
  const uint32_t n = (uint32_t)a.n;
  uint32_t grew = 0;
  for (int64_t w0 = gw * kWave; w0 < a.words; w0 += nw * kWave) {
    if (lane == 0) g_hubn[wib] = 0;
    wave_lds_sync();
    // The rows set in the wave's 64 words, dealt out one per lane per step
    // (rows that grow together sit in the same words).
    const int64_t wi = w0 + lane;
    const uint32_t bits = wi < a.words ? keep[wi] : 0u;
    const uint32_t c = (uint32_t)__popc(bits);
    uint32_t incl = c;
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)incl, off, kWave);
      if (lane >= off) incl += y;
    }
    const uint32_t first = incl - c;
    const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
    for (uint32_t s0 = 0; s0 < total; s0 += kWave) {
      const uint32_t q = s0 + (uint32_t)lane;
      const int o = slot_owner(q, first);
      const uint32_t ob = (uint32_t)__shfl((int)bits, o, kWave);
      const uint32_t of = (uint32_t)__shfl((int)first, o, kWave);
      if (q >= total) continue;
      uint32_t b = ob;
      for (uint32_t t = of; t < q; ++t) b &= b - 1u;  // drop the owner's set bits before this slot's
      const uint32_t w = (uint32_t)((w0 + o) << 5) + (uint32_t)__builtin_ctz(b);
      if (w >= n) continue;
      const int32_t k0 = rrow[w], k1 = rrow[w + 1];
      if (k1 - k0 > kPushHub) {
        const uint32_t hq = atomicAdd(&g_hubn[wib], 1u);
        if (hq < (uint32_t)kWave) {
          g_hubq[wib][hq] = (int32_t)w;
          continue;
        }
      }
      const uint32_t x = sent_word(pvg[w], (int32_t)w, cur, a.val_mask, a.tag_mask);
      if (!x) continue;
      for (int32_t k = k0; k < k1; ++k) grew += push_raise(a, mark, rcol[k], x, cur) ? 1u : 0u;
    }
    wave_lds_sync();
    const uint32_t hubs = min(g_hubn[wib], (uint32_t)kWave);
    for (uint32_t h = 0; h < hubs; ++h) {  // wave-uniform: the whole wave pushes each queued row
      const uint32_t w = (uint32_t)g_hubq[wib][h];
      const uint32_t x = sent_word(pvg[w], (int32_t)w, cur, a.val_mask, a.tag_mask);
      if (!x) continue;
      const int32_t k1 = rrow[w + 1];
      for (int32_t k = rrow[w] + lane; k < k1; k += kWave) grew += push_raise(a, mark, rcol[k], x, cur) ? 1u : 0u;
    }
    wave_lds_sync();  // the queue is read before the next step clears it
  }
  return wave_sum_u32(grew);
}

// One filtered stream sweep of the wave's rows, in tiles in the order values
// travel (see sweep_rows).
template <bool kFirst>
__device__ uint32_t sweep_stream_filt(const LoopArgs& a, const uint8_t* acc, const WaveRows& W, int wib, int lane,
                                      uint32_t cur, uint32_t* acc_count, const uint32_t* keep, uint32_t* mark) {
  uint32_t ch = 0;
  if (W.r1 > W.r0) {
    const int64_t last = W.r0 + ((W.r1 - W.r0 - 1) / kTileRows) * kTileRows;
    if (W.ascending) {
      for (int64_t t0 = W.r0; t0 <= last; t0 += kTileRows)
        ch += sweep_tile_filt<kFirst>(a, acc, t0, min(W.r1, t0 + kTileRows), g_lds.tile[wib], lane, cur, acc_count,
                                      keep, mark);
    } else {
      for (int64_t t0 = last; t0 >= W.r0; t0 -= kTileRows)
        ch += sweep_tile_filt<kFirst>(a, acc, t0, min(W.r1, t0 + kTileRows), g_lds.tile[wib], lane, cur, acc_count,
                                      keep, mark);
    }
  }
  PH_MARK(kPhStream);
  return ch;
}

// Clears this block's share of the words of bitmap b (word-striped over the grid).
__device__ __forceinline__ void clear_share(uint32_t* b, int64_t words, int blk, int nb) {
  for (int64_t i = (int64_t)blk * kBlock + threadIdx.x; i < words; i += (int64_t)nb * kBlock) b[i] = 0u;
}

// Calls f(v, packed value of v) for every row v of the wave (lane-strided).
template <typename F>
__device__ __forceinline__ void for_own_rows(const LoopArgs& a, const WaveRows& W, int lane, F f) {
  if (W.resident) {
#pragma unroll
    for (int j = 0; j < kResRowsPerLane; ++j) {
      int64_t v = W.r0 + lane + j * kWave;
      if (v < W.r1) f(v, g_lds.res.pv[v - W.rb0]);
    }
  } else {
    for (int64_t v = W.r0 + lane; v < W.r1; v += kWave) f(v, a.pv[v]);
  }
}

// Resident mode set-up: sort each gather batch of the wave's edges by target
// (key = target << 8 | row offset), so that the 64 lanes of one gather
// instruction read neighbouring addresses and touch few cache lines.  Bitonic
// network over kSortSlots keys held kSortSlots / 64 per lane (element i lives
// in lane i % 64, slot i / 64); padding keys are 0xffffffff and sort last.
__device__ void sort_gather_batches(int32_t we0, int32_t we1, int lane) {
  ResLds& R = g_lds.res;
  for (int32_t k0 = we0; k0 < we1; k0 += kWave * kGatherBatch) {
    const int cnt = (int)min((int32_t)(kWave * kGatherBatch), we1 - k0);
    uint32_t key[kSortPerLane];
#pragma unroll
    for (int u = 0; u < kSortPerLane; ++u) {
      const int i = lane + u * kWave;
      key[u] = i < cnt ? R.e[k0 + i] : 0xffffffffu;
    }
#pragma unroll
    for (int k = 2; k <= kSortSlots; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        if (j >= kWave) {
          const int ju = j / kWave;
#pragma unroll
          for (int u = 0; u < kSortPerLane; ++u) {
            if (u & ju) continue;
            const int i = lane + u * kWave;
            const bool asc = (i & k) == 0;
            const uint32_t x = key[u], y = key[u | ju];
            const bool sw = asc ? (x > y) : (x < y);
            key[u] = sw ? y : x;
            key[u | ju] = sw ? x : y;
          }
        } else {
#pragma unroll
          for (int u = 0; u < kSortPerLane; ++u) {
            const int i = lane + u * kWave;
            const uint32_t y = (uint32_t)__shfl_xor((int)key[u], j, kWave);
            const bool asc = (i & k) == 0;
            const bool lower = (i & j) == 0;
            const uint32_t lo = min(key[u], y), hi = max(key[u], y);
            key[u] = (lower == asc) ? lo : hi;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kSortPerLane; ++u) {
      const int i = lane + u * kWave;
      if (i < cnt) R.e[k0 + i] = key[u];
    }
  }
}

// The whole MAP computation for one graph, run by `nb` cooperating blocks of
// which this is block `b`; `logical` is the block's position in row order.
// Every block of the set must call it; c is the set's zeroed control block.
// kAsync selects the fixpoint control at compile time: asynchronous sweeps with
// quiescence detection, or a grid barrier after every sweep (required for a
// single block, for untagged values, and with MAP_FLAG_SYNC_SWEEPS).
template <typename C, bool kAsync, bool kEarly, bool kFilt = false>
__device__ void map_body(const LoopArgs& a, C* c, const int nb, const int b, const int logical) {
  BlockLds& S = g_lds;
  __shared__ uint32_t s_red[kWavesPerBlock];
  __shared__ unsigned long long s_red64[kWavesPerBlock];
  __shared__ int32_t s_wit[kWavesPerBlock];

  const int lane = threadIdx.x & (kWave - 1);
  const int wib = threadIdx.x / kWave;
  // The asynchronous bodies use the balanced layout of the resident slice and
  // LDS pass; the barrier-mode bodies keep the per-lane row fold.
  constexpr bool kBal = kAsync;
  PH_START();
  if (kEarly && threadIdx.x == 0) g_early = 0;  // ordered before its first use by the set-up's barriers
  // Tag epoch of this call: left by the previous call on the workspace (an
  // earlier kernel); block 0 writes the next one only after the first grid
  // barrier, which every block reaches after this read.
  const uint32_t tbase = a.epoch ? *a.epoch : 0u;

  // Row ranges of this block and wave.
  const int64_t rows_per_block = ((int64_t)a.n + nb - 1) / nb;
  const int64_t rb0 = min((int64_t)a.n, (int64_t)logical * rows_per_block);
  const int64_t rb1 = min((int64_t)a.n, rb0 + rows_per_block);
  const int64_t rows_per_wave = (rows_per_block + kWavesPerBlock - 1) / kWavesPerBlock;
  WaveRows W;
  W.rb0 = rb0;
  W.rb1 = rb1;
  W.r0 = min(rb1, rb0 + (int64_t)wib * rows_per_wave);
  W.r1 = min(rb1, W.r0 + rows_per_wave);
  W.we0 = W.we1 = 0;
  {
    const int32_t eb0 = a.row_ptr[rb0], eb1 = a.row_ptr[rb1];
    // n < 2^24 keeps every staged remote key (successor << 8 | row offset)
    // below 0xffffffff, the padding key of the sort and the gather.
    W.resident = !kFilt && !a.force_stream && a.n < (1 << 24) && rows_per_wave <= kResWaveRows &&
                 (int64_t)eb1 - eb0 <= kResEdges;
    W.wr = 0;
    {
      // Direction of the block's edges, from up to 8 rows per thread.
      __shared__ uint32_t s_dir[2];
      if (threadIdx.x < 2) s_dir[threadIdx.x] = 0;
      __syncthreads();
      uint32_t down = 0, up = 0;
      for (int64_t r = rb0 + threadIdx.x, i = 0; r < rb1 && i < 8; r += kBlock, ++i) {
        const int32_t k1 = a.row_ptr[r + 1];
        for (int32_t k = a.row_ptr[r]; k < k1; ++k) {
          if ((int64_t)a.col[k] < r) ++down;
          else if ((int64_t)a.col[k] > r) ++up;
        }
      }
      down = wave_sum_u32(down);
      up = wave_sum_u32(up);
      if (lane == 0) {
        atomicAdd(&s_dir[0], down);
        atomicAdd(&s_dir[1], up);
      }
      __syncthreads();
      W.ascending = s_dir[0] > s_dir[1];
      __syncthreads();
    }
    if (W.resident) {
      // Each wave stages its rows' edges in its part of the block's slice:
      // first the edges to rows of other blocks (gathered from memory each
      // sweep), then the edges to rows of this block grouped by row (folded
      // from LDS by the row's lane).
      W.we0 = a.row_ptr[W.r0] - eb0;
      W.we1 = a.row_ptr[W.r1] - eb0;
      const uint32_t base = (uint32_t)rb0, span = (uint32_t)(rb1 - rb0);
      const uint64_t below = lane ? (~0ull >> (kWave - lane)) : 0ull;
      uint32_t nr = 0;
      for (int64_t r = W.r0 + lane; r < W.r1; r += kWave) {
        const int32_t k1 = a.row_ptr[r + 1];
        for (int32_t k = a.row_ptr[r]; k < k1; ++k) nr += (uint32_t)a.col[k] - base >= span ? 1u : 0u;
      }
      W.wr = W.we0 + (int32_t)wave_sum_u32(nr);
      int32_t nrem = 0, lrun = W.wr;
      for (int64_t rc = W.r0; rc < W.r1; rc += kWave) {
        const int64_t r = rc + lane;
        int32_t k = 0, k1 = 0;
        if (r < W.r1) {
          k = a.row_ptr[r];
          k1 = a.row_ptr[r + 1];
        }
        uint32_t dl = 0;
        for (int32_t kk = k; kk < k1; ++kk) dl += (uint32_t)a.col[kk] - base < span ? 1u : 0u;
        uint32_t incl = dl;
        for (int off = 1; off < kWave; off <<= 1) {
          const uint32_t y = (uint32_t)__shfl_up((int)incl, off, kWave);
          if (lane >= off) incl += y;
        }
        int32_t lpos = lrun + (int32_t)(incl - dl);
        if (r < W.r1) S.res.lrow[r - rb0] = (uint16_t)lpos;
        lrun += (int32_t)__shfl((int)incl, kWave - 1, kWave);
        const uint32_t off = (uint32_t)(r - W.r0);
        for (;;) {
          const bool act = k < k1;
          if (__ballot(act) == 0) break;
          const int32_t t = act ? a.col[k] : 0;
          const bool rem = act && (uint32_t)t - base >= span;
          const uint64_t mr = __ballot(rem);
          if (rem) S.res.e[W.we0 + nrem + __popcll(mr & below)] = ((uint32_t)t << 8) | off;
          nrem += __popcll(mr);
          if (act && !rem) S.res.e[lpos++] = (kBal ? (off << 16) : 0u) | ((uint32_t)t - base);
          k += act ? 1 : 0;
        }
      }
      wave_lds_sync();
      sort_gather_batches(W.we0, W.wr, lane);
    }
    __syncthreads();
    if (kBal && W.resident) {  // block-uniform
      if (lane == 0) {
        g_rseg[wib] = W.we0;
        g_rpre[wib + 1] = W.wr - W.we0;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        g_rpre[0] = 0;
        for (int i = 1; i <= kWavesPerBlock; ++i) g_rpre[i] += g_rpre[i - 1];
      }
      __syncthreads();
    }
  }

  Grid<C> g;
  g.c = c;
  g.gen = 0;
  g.nblocks = nb;
  g.ngroups = min(nb, kMaxGroups);
  g.group = b % g.ngroups;
  g.group_size = nb / g.ngroups + ((b % g.ngroups) < (nb % g.ngroups) ? 1 : 0);
  g.rank = b;
  uint8_t* acc = a.propagate ? const_cast<uint8_t*>(a.acc_in) : a.accw;

  // Block-level sum of per-wave u32 values followed by one striped atomic.
  auto block_add_count = [&](uint32_t x, int set) {
    x = wave_sum_u32(x);
    if (lane == 0) s_red[wib] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int i = 0; i < kWavesPerBlock; ++i) t += s_red[i];
      if (t) __hip_atomic_fetch_add(&c->sets[set][b % kStripes].count, t, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  };
  // Reads of a completed set (after the barrier that closed it).
  auto read_count = [&](int set) {
    uint32_t t = lane < kStripes ? ld_agent(&c->sets[set][lane].count) : 0u;
    return wave_sum_u32(t);
  };
  // Any wave of the block changed a row: one flag per block.  Each wave first
  // completes its writes, so that the leader's release after this barrier
  // (change report, or grid barrier) covers every wave's new values.
  auto block_any = [&](uint32_t ch) {
    if (lane == 0) s_red[wib] = ch;
    wave_writes_done();
    __syncthreads();
    uint32_t any = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) any |= s_red[i];
    __syncthreads();
    return any ? 1u : 0u;
  };
  // Filtered stream sweeps report how many rows grew (the barrier sums them):
  // the next sweep's frontier size.
  auto block_count = [&](uint32_t x) {
    if (lane == 0) s_red[wib] = x;
    wave_writes_done();
    __syncthreads();
    uint32_t t = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) t += s_red[i];
    __syncthreads();
    return t;
  };

  uint32_t count_prev = 0;  // |A_k| of the last completed iteration
  uint32_t rtag = 0;        // push: frontier round, the same in every block
  uint32_t gsw = 0;         // filtered stream sweeps: sweeps so far, the same in every block
  int32_t k = 0;
  int64_t total_sweeps = 0;  // whole-graph sweeps, summed over the iterations
  int32_t status = MAP_OK, found = 0, witness = 0;
  int32_t left = 0;
  bool acc_from_pv = false;  // acc_out comes from the accepting bits of the packed values
  bool ok = true;
  uint32_t tot = 0;
  // Asynchronous sweeps need the iteration tag; without it (n >= 2^30) every
  // sweep ends with a grid barrier.
  constexpr bool sync = !kAsync;

  {
    // Own packed values start in iteration 0 (tag 0), so no value left in the
    // workspace by an earlier call is mistaken for one of this call; A_1 is
    // copied to the working flags and counted.
    uint32_t cnt = 0;
    for (int64_t v = W.r0 + lane; v < W.r1; v += kWave) {
      a.pv[v] = 0u;
      if (a.push) a.mark[v] = 0u;
      if (!a.propagate) {
        uint8_t x = a.acc_in[v] ? 1 : 0;
        a.accw[v] = x;
        cnt += x;
      }
    }
    if (kFilt) clear_share(a.chg, 3 * a.words, b, nb);
    block_add_count(cnt, g.gen % kSets);
    ok = grid_sync(g, 0, nullptr);
    if (!ok) goto aborted;
    count_prev = read_count((g.gen - 1) % kSets);
    PH_MARK(kPhSetup);
    if (!a.propagate && count_prev == 0) { left = 0; goto done; }
  }

  for (;;) {
    k++;
    // Iteration tag: values written in iteration k carry the tag of k; a
    // reader that finds another tag takes the reset value instead.
    const uint32_t cur = iter_tag(a.tag_mask, a.tag_shift, tbase, k);
    if (kFilt) {
      // The accepting set of this iteration as a bitmap (64 vertices per wave
      // step), complete in every block before the reset sweep reads it.
      const int64_t gw = (int64_t)b * kWavesPerBlock + wib, nw = (int64_t)nb * kWavesPerBlock;
      for (int64_t v0 = gw * kWave; v0 < (int64_t)a.n; v0 += nw * kWave) {
        const int64_t v = v0 + lane;
        const unsigned long long am = __ballot(v < (int64_t)a.n && acc[v] != 0);
        const int64_t wi = (v0 >> 5) + lane;
        if (lane < 2 && wi < a.words) a.accb[wi] = lane ? (uint32_t)(am >> 32) : (uint32_t)am;
      }
      if (!grid_sync(g, 0, nullptr)) goto aborted;
    }
    uint32_t nacc = 0;       // accepting rows of this block in A_k (reset sweep)
    uint32_t cnt_k = 0;      // |A_k|
    int64_t s = 0;           // sweeps of this block in iteration k
    bool local_fix = false;  // resident: the block's values are at the fixpoint of its in-block edges
    // One loop for both fixpoint controls, so that each sweep variant is
    // inlined once.
    //  - sync: a grid barrier after every sweep carries the changed count.
    //  - asynchronous (the reset is each block's first sweep): blocks sweep
    //    their rows without waiting for one another; values only grow, so
    //    reads of stale remote values are safe.  A sweep that changed
    //    something releases its writes and bumps `dirty`; a sweep that changed
    //    nothing, started after reading dirty == d (then an acquire), reports
    //    quiet {k, d+1}.  When every block reports quiet for the current value
    //    of `dirty`, no change happened while any of those sweeps ran and every
    //    change before them was visible to them, so all rows are at the
    //    fixpoint: block 0 then publishes done = k.
    const uint32_t tag = (uint32_t)k;
    uint32_t d_seen = 0xffffffffu;  // async: counter value of this block's last quiet sweep (wave 0)
    // Async: start of this fixpoint computation on the device wall clock
    // (wave 0), against which kIterTicks bounds the sweeping.
    const uint64_t t_iter = wall_clock64();
    // After a sweep: the barrier (sync) or the change / quiet report (async).
    // Returns false when the launch must stop.
    auto report = [&](uint32_t any, uint32_t d0) -> bool {
      // A row that reached its own id in this sweep (block_any's barrier has
      // ordered every wave's record before this read); published before the
      // barrier or the release below.
      if (kEarly && threadIdx.x == 0 && g_early)
        __hip_atomic_fetch_max(&c->early, g_early, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (sync) {
        if (s == 1 && !a.propagate) block_add_count(nacc, g.gen % kSets);
        if (!grid_sync(g, any, &tot)) return false;
        if (s == 1 && !a.propagate) cnt_k = read_count((g.gen - 1) % kSets);
        return true;
      }
      if (threadIdx.x == 0) {
        if (any) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_fetch_add(&c->dirty, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          __hip_atomic_store(&c->quiet[b], ((unsigned long long)tag << 32) | (uint32_t)(d0 + 1u),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      if (wib == 0) d_seen = any ? 0xffffffffu : d0;
      return true;
    };
    // MAP_FLAG_EARLY: after a sweep, the block's rows whose value is their
    // own id (kept out of the sweep code, whose register allocation it would
    // otherwise share); block_any's barrier orders the records before report
    // reads them.
    auto early_scan = [&]() {
      if (!kEarly) return;
      for_own_rows(a, W, lane, [&](int64_t v, uint32_t x) {
        if ((x & a.val_mask) == (uint32_t)v + 1u) atomicMax(&g_early, (uint32_t)v + 1u);
      });
    };
    // Sum over the block of a per-wave count (every thread gets it).
    auto block_sum_waves = [&](uint32_t x) {
      if (lane == 0) s_red[wib] = x;
      __syncthreads();
      uint32_t t = 0;
      for (int i = 0; i < kWavesPerBlock; ++i) t += s_red[i];
      __syncthreads();
      return t;
    };
    if (sync && a.push) {
      // Frontier rounds over the transposed CSR: every vertex whose value grew
      // sends its new value to each predecessor with an atomic max on the
      // packed word (same accepting bit and tag, so the words compare by
      // value); the predecessors that grew form the next frontier.  A grid
      // barrier ends each round and carries the size of the next frontier.
      // The reset gives every row map 0 and puts the accepting rows in the
      // first frontier (they send their own id).
      g_u32* pvg = (g_u32*)a.pv;
      g_cu8* gacc = (g_cu8*)acc;
      ++rtag;
      if (b == 0 && threadIdx.x == 0) st_agent(&c->fcount[1], 0u);
      uint32_t napp = 0;
      for (int64_t v0 = W.r0; v0 < W.r1; v0 += kWave) {
        const int64_t v = v0 + lane;
        uint32_t isacc = 0;
        if (v < W.r1) {
          isacc = gacc[v] ? 1u : 0u;
          pvg[v] = (isacc << 31) | cur;
          if (isacc) a.mark[v] = rtag;
        }
        nacc += isacc;
        napp += frontier_append(a.front[0], &c->fcount[0], isacc != 0, (int32_t)v, lane);
      }
      if (!a.propagate) block_add_count(nacc, g.gen % kSets);
      uint32_t bapp = block_sum_waves(napp);
      if (!grid_sync(g, bapp, &tot)) goto aborted;
      if (!a.propagate) cnt_k = read_count((g.gen - 1) % kSets);
      s = 1;
      int fc = 0;
      uint32_t S = tot;
      const int64_t gw = (int64_t)b * kWavesPerBlock + wib, nw = (int64_t)nb * kWavesPerBlock;
      while (S > 0) {
        if (s > (int64_t)a.n + 1) { status = MAP_ENOTCONVERGED; break; }
        ++rtag;
        // This round reads frontier fc; its counter is next written in the
        // round after (the barrier ending this round orders the clear).
        if (b == 0 && threadIdx.x == 0) st_agent(&c->fcount[fc], 0u);
        const int32_t* F = a.front[fc];
        int32_t* Fn = a.front[fc ^ 1];
        uint32_t* cn = &c->fcount[fc ^ 1];
        napp = 0;
        for (int64_t i0 = gw * kWave; i0 < (int64_t)S; i0 += nw * kWave) {
          const int64_t i = i0 + lane;
          int32_t k = 0, k1 = 0;
          uint32_t x = 0;
          if (i < (int64_t)S) {
            const int32_t w = F[i];
            x = sent_word(pvg[w], w, cur, a.val_mask, a.tag_mask);
            if (x) {
              k = a.rrow_ptr[w];
              k1 = a.rrow_ptr[w + 1];
            }
          }
          for (;;) {
            const bool act = k < k1;
            if (__ballot(act) == 0) break;
            bool grew = false;
            int32_t v = 0;
            if (act) {
              v = a.rcol[k++];
              const uint32_t word = ((gacc[v] ? 1u : 0u) << 31) | cur | x;
              const uint32_t old = __hip_atomic_fetch_max(&a.pv[v], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              grew = (old & a.val_mask) < x &&
                     __hip_atomic_exchange(&a.mark[v], rtag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != rtag;
            }
            napp += frontier_append(Fn, cn, grew, v, lane);
          }
        }
        bapp = block_sum_waves(napp);
        if (!grid_sync(g, bapp, &tot)) goto aborted;
        S = tot;
        fc ^= 1;
        s++;
      }
    } else {
    {
      // The reset sweep of iteration k.
      uint32_t d0 = 0;
      if (!sync) {
        if (threadIdx.x == 0) {
          s_red[1] = ld_agent(&c->dirty);
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        d0 = s_red[1];
        __syncthreads();
      }
      PH_MARK(kPhOther);
      uint32_t c1;
      if (kFilt) {
        // Sweep gsw reads the rows that grew in sweep gsw - 1 (the reset sweep:
        // the accepting set), marks its own in bitmap gsw % 3 and clears
        // bitmap (gsw + 1) % 3 for the next sweep.
        clear_share(a.chg + ((gsw + 1) % 3) * a.words, a.words, b, nb);
        c1 = sweep_stream_filt<true>(a, acc, W, wib, lane, cur, &nacc, a.accb, a.chg + (gsw % 3) * a.words);
        ++gsw;
      } else {
        c1 = sweep_rows<true, kBal>(a, acc, W, wib, lane, cur, &nacc, &local_fix);
      }
      s = 1;
      early_scan();
      const uint32_t any1 = kFilt ? block_count(c1) : block_any(c1);
      if (!report(any1, d0)) goto aborted;
      PH_MARK(kPhReport);
      PH_COUNT(kPhSweeps, 1);
      PH_COUNT(kPhQuiet, any1 ? 0 : 1);
    }
    for (;;) {
      uint32_t d0 = 0;
      if (sync) {
        if (tot == 0) break;
        if (kEarly && ld_agent(&c->early)) break;  // read after the barrier: the same in every block
        if (s > (int64_t)a.n + 1) { status = MAP_ENOTCONVERGED; break; }
      } else {
        if (wib == 0) {
          uint32_t cmd = 0;  // 0 sweep, 1 done, 2 abort
          const uint64_t t0 = wall_clock64();
          for (;;) {
            if (ld_agent(&c->done) == tag) { cmd = 1; break; }
            if (kEarly && ld_agent(&c->early)) { cmd = 1; break; }
            // Sweeping that has not settled within kIterTicks ends the launch,
            // however often the counter moves.
            if (wall_clock64() - t_iter > kIterTicks) { cmd = 2; break; }
            const uint32_t d = ld_agent(&c->dirty);
            if (d != d_seen) { cmd = 0; d0 = d; break; }
            if (b == 0) {
              const unsigned long long want = ((unsigned long long)tag << 32) | (uint32_t)(d + 1u);
              bool mine = true;
              for (int i = lane; i < nb; i += kWave)
                mine &= __hip_atomic_load(&c->quiet[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == want;
              if (__ballot(!mine) == 0 && ld_agent(&c->dirty) == d) {
                if (lane == 0) __hip_atomic_store(&c->done, tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                cmd = 1;
                break;
              }
            }
            if (wall_clock64() - t0 > kWaitTicks || ld_agent((const uint32_t*)&c->abort)) { cmd = 2; break; }
            __builtin_amdgcn_s_sleep(1);
          }
          if (lane == 0) {
            if (cmd == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (cmd == 2) st_agent((uint32_t*)&c->abort, 1u);
            s_red[0] = cmd;
            s_red[1] = d0;
          }
        }
        __syncthreads();
        const uint32_t cmd = s_red[0];
        d0 = s_red[1];
        __syncthreads();
        PH_MARK(kPhWait);
        if (cmd == 2) goto aborted;
        if (cmd == 1) break;
      }
      uint32_t c2;
      if (kFilt) {
        clear_share(a.chg + ((gsw + 1) % 3) * a.words, a.words, b, nb);
        uint32_t* markb = a.chg + (gsw % 3) * a.words;
        const uint32_t* keepb = a.chg + ((gsw + 2) % 3) * a.words;
        // tot: the rows that grew in the previous sweep (an upper bound after a
        // push round), the same in every block
        if (a.dopt && (int64_t)tot * kPushDiv < (int64_t)a.n) {
          const int64_t gw = (int64_t)b * kWavesPerBlock + wib, nw = (int64_t)nb * kWavesPerBlock;
          c2 = push_round_filt(a, keepb, markb, cur, gw, nw, wib, lane);
          PH_MARK(kPhStream);
        } else {
          c2 = sweep_stream_filt<false>(a, acc, W, wib, lane, cur, nullptr, keepb, markb);
        }
        ++gsw;
      } else {
        c2 = sweep_rows<false, kBal>(a, acc, W, wib, lane, cur, nullptr, &local_fix);
      }
      s++;
      early_scan();
      const uint32_t any2 = kFilt ? block_count(c2) : block_any(c2);
      if (!report(any2, d0)) goto aborted;
      PH_MARK(kPhReport);
      PH_COUNT(kPhSweeps, 1);
      PH_COUNT(kPhQuiet, any2 ? 0 : 1);
    }
    }
    // Asynchronous mode: |A_k| is reduced together with the detect pass (same
    // barrier epoch).
    if (!sync && !a.propagate) block_add_count(nacc, g.gen % kSets);
    if (status != MAP_OK) { total_sweeps += s; left = (int32_t)count_prev; acc_from_pv = !a.propagate; break; }
    if (a.propagate) {
      // The blocks' sweep counts, summed at one more barrier.
      if (threadIdx.x == 0 && s)
        __hip_atomic_fetch_add(&c->sets[g.gen % kSets][b % kStripes].sweeps, (unsigned long long)s,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ok = grid_sync(g, 0, nullptr);
      if (!ok) goto aborted;
      unsigned long long sw = lane < kStripes ? __hip_atomic_load(&c->sets[(g.gen - 1) % kSets][lane].sweeps,
                                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
      total_sweeps += ((int64_t)wave_sum_u64(sw) + nb / 2) / nb;
      break;
    }

    // Detect and strip: witness = max v with map(v) == v; every nonzero map
    // value loses its accepting flag (the flags of this iteration stay in the
    // packed values).
    {
      int32_t wit = 0;
      unsigned long long dig = 0;
      uint32_t nz = 0;
      const bool want_digest = a.digest != 0;
      auto note = [&](int64_t v, uint32_t mv) {
        const uint32_t id = (uint32_t)v + 1u;
        if (mv == id) wit = max(wit, (int32_t)id);
        if (want_digest) dig += mix64(((unsigned long long)id << 32) | mv);
        nz |= mv;
      };
      if (W.resident) {
        // The flag of every map value is cleared without reading it first: no
        // load waits here, and the stores complete before the barrier below
        // (rows that share a map value clear it more than once, harmlessly).
#pragma unroll
        for (int j = 0; j < kResRowsPerLane; ++j) {
          const int64_t v = W.r0 + lane + j * kWave;
          const uint32_t mv = v < W.r1 ? g_lds.res.pv[v - W.rb0] & a.val_mask : 0u;
          if (v < W.r1) note(v, mv);
          if (mv) acc[mv - 1] = 0;
        }
      } else {
        for_own_rows(a, W, lane, [&](int64_t v, uint32_t x) {
          const uint32_t mv = x & a.val_mask;
          note(v, mv);
          // Many vertices share a map value: read before writing.
          if (mv != 0 && acc[mv - 1]) acc[mv - 1] = 0;
        });
      }
      wit = wave_max_i32(wit);
      if (want_digest) dig = wave_sum_u64(dig);
      const uint32_t wnz = __ballot(nz != 0) != 0 ? 1u : 0u;
      if (lane == 0) { s_wit[wib] = wit; s_red64[wib] = dig; s_red[wib] = wnz; }
      __syncthreads();
      if (threadIdx.x == 0) {
        int32_t bw = 0;
        unsigned long long bd = 0;
        uint32_t bn = 0;
        for (int i = 0; i < kWavesPerBlock; ++i) { bw = max(bw, s_wit[i]); bd += s_red64[i]; bn |= s_red[i]; }
        Stripe& st = c->sets[g.gen % kSets][b % kStripes];
        if (bw) __hip_atomic_fetch_max(&st.witness, bw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (bd) __hip_atomic_fetch_add(&st.digest, bd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (s) __hip_atomic_fetch_add(&st.sweeps, (unsigned long long)s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (bn) __hip_atomic_fetch_add(&st.nonzero, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
      ok = grid_sync(g, 0, nullptr);
      if (!ok) goto aborted;
      const int set = (g.gen - 1) % kSets;
      // Lane i of every wave reads stripe i; the wave combines them.
      int32_t w2 = 0;
      unsigned long long d2 = 0, sw2 = 0;
      uint32_t nz2 = 0, cnt2 = 0;
      if (lane < kStripes) {
        Stripe& st = c->sets[set][lane];
        w2 = __hip_atomic_load(&st.witness, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        d2 = __hip_atomic_load(&st.digest, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sw2 = __hip_atomic_load(&st.sweeps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        nz2 = ld_agent(&st.nonzero);
        cnt2 = ld_agent(&st.count);
      }
      w2 = wave_max_i32(w2);
      d2 = wave_sum_u64(d2);
      sw2 = wave_sum_u64(sw2);
      nz2 = wave_sum_u32(nz2);
      cnt2 = wave_sum_u32(cnt2);
      if (!sync) cnt_k = cnt2;
      PH_MARK(kPhDetect);
      PH_COUNT(kPhIters, 1);
      // MAP_FLAG_EARLY: a published early hit (every block's publication
      // precedes its arrival at the barrier above) is a cycle vertex too.
      if (kEarly) w2 = max(w2, (int32_t)ld_agent(&c->early));
      const bool leader = b == 0 && threadIdx.x == 0;
      if (k >= 2 && cnt_k == 0) {
        // No accepting vertex was left after iteration k-1: iteration k did not happen.
        if (leader && a.trace && k - 1 <= a.trace_cap) a.trace[(int64_t)(k - 2) * 3 + 0] = (uint64_t)count_prev;
        k--;
        left = 0;
        break;
      }
      // Whole-graph sweeps of iteration k: the blocks' sweeps over their
      // count, rounded (in barrier mode every block's count).
      const int64_t sweeps_k = ((int64_t)sw2 + nb / 2) / nb;
      total_sweeps += sweeps_k;
      if (leader && a.trace) {
        if (k >= 2 && k - 1 <= a.trace_cap) a.trace[(int64_t)(k - 2) * 3 + 0] = (uint64_t)(count_prev - cnt_k);
        if (k <= a.trace_cap) {
          uint64_t* row = a.trace + (int64_t)(k - 1) * 3;
          row[0] = 0;
          row[1] = (uint64_t)sweeps_k;
          row[2] = want_digest ? d2 : 0ull;
        }
      }
      if (w2 > 0) {  // some vertex is its own maximal accepting predecessor
        found = 1;
        witness = w2;
        left = (int32_t)cnt_k;
        acc_from_pv = true;
        break;
      }
      if (nz2 == 0) { left = (int32_t)cnt_k; break; }  // every map value is 0: nothing to strip
      if (a.max_iter > 0 && k >= a.max_iter) {
        // Cap reached: count the accepting set left after this strip.
        uint32_t cnt = 0;
        for (int64_t v = W.r0 + lane; v < W.r1; v += kWave) cnt += a.accw[v];
        block_add_count(cnt, g.gen % kSets);
        ok = grid_sync(g, 0, nullptr);
        if (!ok) goto aborted;
        const uint32_t nxt = read_count((g.gen - 1) % kSets);
        if (leader && a.trace && k <= a.trace_cap) a.trace[(int64_t)(k - 1) * 3 + 0] = (uint64_t)(cnt_k - nxt);
        left = (int32_t)nxt;
        if (nxt != 0) status = MAP_ENOTCONVERGED;
        break;
      }
      count_prev = cnt_k;
    }
  }

done:
  // Outputs: map vector (propagate) or the accepting set at exit (detect).
  if (a.propagate && a.map_out) {
    for_own_rows(a, W, lane, [&](int64_t v, uint32_t x) { a.map_out[v] = (int32_t)(x & a.val_mask); });
  }
  if (!a.propagate && a.acc_out) {
    for_own_rows(a, W, lane, [&](int64_t v, uint32_t x) {
      a.acc_out[v] = acc_from_pv ? (uint8_t)(x >> 31) : a.accw[v];
    });
  }
  if (b == 0 && threadIdx.x == 0) {
    // Words now carry the tags of iterations k and, where a reset was cut
    // short, k - 1: the next call's first tag is past both.
    if (a.epoch) *a.epoch = tbase + (uint32_t)k + 1u;
    a.result->found = found;
    a.result->witness = witness;
    a.result->iterations = a.propagate ? 0 : k;
    a.result->status = status;
    a.result->sweeps = total_sweeps;
    a.result->accepting_left = a.propagate ? 0 : left;
    a.result->reserved = 0;
  }
  PH_MARK(kPhOther);
  PH_STORE(b);
  return;

aborted:
  if (threadIdx.x == 0) {
    __hip_atomic_store(&a.result->status, (int32_t)MAP_EDEVICE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

// kEarly: MAP_FLAG_EARLY (a separate instantiation, so that the plain loop
// carries none of its code).
template <bool kAsync, bool kEarly, bool kFilt = false>
__global__ void __launch_bounds__(kBlock) map_loop_kernel(LoopArgs a) {
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  // XCD-aware numbering: consecutive hardware block ids land on different
  // XCDs; give each XCD a contiguous range of logical blocks (and rows).
  const int logical = (nb % kMaxGroups == 0) ? (b % kMaxGroups) * (nb / kMaxGroups) + b / kMaxGroups : b;
  map_body<Ctrl, kAsync, kEarly, kFilt>(a, a.ctrl, nb, b, logical);
}

// ------------------------------------------------------------------ batch --

struct BatchArgs {
  int32_t count;
  const map_graph_desc* graphs;
  map_result* results;
  const int32_t* item_start;  // [count + 1]: first work item of each graph
  const int64_t* scratch_off;  // [count]: byte offset of each graph's scratch
  GangCtrl* gctrl;             // [count]
  char* scratch;
  uint32_t* next_item;
  int32_t* status;             // MAP_ENOSPC when the scratch does not fit
  uint32_t flags;
};

// One graph of a batch, out of line so that its register allocation is not
// shared with the work-queue loop around it.
__device__ __noinline__ void map_body_gang_async(const LoopArgs& a, GangCtrl* c, int nb, int rank) {
  map_body<GangCtrl, true, false>(a, c, nb, rank, rank);
}
__device__ __noinline__ void map_body_gang_sync(const LoopArgs& a, GangCtrl* c, int nb, int rank) {
  map_body<GangCtrl, false, false>(a, c, nb, rank, rank);
}
__device__ __noinline__ void map_body_gang_sync_early(const LoopArgs& a, GangCtrl* c, int nb, int rank) {
  map_body<GangCtrl, false, true>(a, c, nb, rank, rank);
}
__device__ __noinline__ void map_body_gang_filt(const LoopArgs& a, GangCtrl* c, int nb, int rank) {
  map_body<GangCtrl, false, false, true>(a, c, nb, rank, rank);
}
// One graph solved by a gang, in the fixpoint control and mode its arguments ask
// for.  MAP_FLAG_EARLY always runs with a grid barrier after every sweep: the
// asynchronous early body is not built (its builds hung on the device).
__device__ __forceinline__ void map_body_gang(const LoopArgs& a, GangCtrl* c, int nb, int rank) {
  const bool async = nb > 1 && !a.sync_sweeps && a.tag_mask;
  if (a.early) {
    map_body_gang_sync_early(a, c, nb, rank);
  } else if (a.filt) {
    map_body_gang_filt(a, c, nb, rank);
  } else {
    if (async) map_body_gang_async(a, c, nb, rank);
    else map_body_gang_sync(a, c, nb, rank);
  }
}

// --------------------------------------------------------- counterexample --

// Barrier state of a launch whose blocks all cooperate on one control block,
// in hardware block order.
__device__ __forceinline__ Grid<Ctrl> whole_grid(Ctrl* c) {
  Grid<Ctrl> g;
  g.c = c;
  g.gen = 0;
  g.nblocks = gridDim.x;
  g.ngroups = min((int)gridDim.x, kMaxGroups);
  g.group = blockIdx.x % g.ngroups;
  g.group_size = gridDim.x / g.ngroups + ((blockIdx.x % g.ngroups) < (gridDim.x % g.ngroups) ? 1 : 0);
  g.rank = blockIdx.x;
  return g;
}

// Arguments of the lasso search: a shortest path from `init` to the witness
// and a shortest cycle through it, by breadth-first search over successors.
struct LassoArgs {
  int32_t n;
  const int32_t* row_ptr;  // pull CSR of G: row v = successors of v
  const int32_t* col;
  int32_t w;               // witness, 0-based
  int32_t init;            // initial vertex, 0-based, or -1
  int32_t* path;           // ids out
  int32_t cap;
  map_lasso_result* result;
  uint64_t* parent;        // [n]: level << 32 | (1 + the vertex it was reached from); the start
                           // level 0 with low word -1; unreached kUnreached
  int32_t* front[2];       // frontiers [n]
  Ctrl* ctrl;
};

// Sum over the block of a per-wave u32 (every thread gets it).
__device__ uint32_t lasso_block_sum(uint32_t x) {
  __shared__ uint32_t s_part[kWavesPerBlock];
  const int lane = threadIdx.x & (kWave - 1), wib = threadIdx.x / kWave;
  if (lane == 0) s_part[wib] = x;
  __syncthreads();
  uint32_t t = 0;
  for (int i = 0; i < kWavesPerBlock; ++i) t += s_part[i];
  __syncthreads();
  return t;
}

// Flattened frontier expansion, shared by the counterexample search and the
// pruning.  A wave takes 64 frontier vertices at a time; an inclusive scan of
// their degrees across the wave gives each vertex the first slot of its edges
// in the wave's combined list, and lane l examines slots q0 + l + 64 s (s <
// kExpandPerLane) of that list.  The wave thus issues the reads and atomics of
// up to 64 * kExpandPerLane edges together, instead of one edge per lane per
// step, and appends what it claimed with one counter update per chunk.
constexpr int kExpandPerLane = 4;
constexpr uint64_t kUnreached = ~0ull;    // lasso parent word of a vertex not reached
constexpr uint32_t kNoHit = 0xffffffffu;  // lasso: no edge has entered the target yet

// Appends x[s] for every s with take[s] to frontier F with one counter update
// for the whole wave; returns the number appended by the wave (wave-uniform).
template <int N>
__device__ __forceinline__ uint32_t frontier_append_n(int32_t* F, uint32_t* cnt, const bool* take, const int32_t* x,
                                                      int lane) {
  uint32_t c = 0;
#pragma unroll
  for (int s = 0; s < N; ++s) c += take[s] ? 1u : 0u;
  uint32_t incl = c;
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)incl, off, kWave);
    if (lane >= off) incl += y;
  }
  const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
  if (total == 0) return 0;
  uint32_t base = 0;
  if (lane == 0) base = __hip_atomic_fetch_add(cnt, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  base = (uint32_t)__shfl((int)base, 0, kWave) + (incl - c);
#pragma unroll
  for (int s = 0; s < N; ++s)
    if (take[s]) F[base++] = x[s];
  return total;
}

// Breadth-first search from `from` until an edge enters `to`, run by every
// thread of the grid.  The start is marked reached (level 0) but an edge into
// `to` is taken before that mark is looked at, so from == to finds a shortest
// cycle.  Each round expands one frontier: a wave takes 64 frontier vertices
// and a lane walks its vertex's successors.  A successor not reached in an
// earlier round takes, by an atomic minimum on its 64-bit parent word (round
// in the high half), the smallest frontier vertex with an edge to it; the
// lane whose minimum found the word unreached appends it to the next
// frontier.  An edge into `to` takes the minimum of its source into c->hit.
// The parents, the last vertex and so the path therefore depend only on the
// edge set, not on the column order or the schedule: walking back from `to`,
// each step goes to the smallest vertex of the level before.  A grid barrier
// ends each round and carries the size of the next frontier.  Returns the
// length of a shortest path of >= 1 edge, 0 if `to` is not reached, -1 if a
// barrier wait gave up (the launch must stop); *last (every block) is the
// vertex whose edge entered `to`.
__device__ int32_t lasso_bfs(const LassoArgs& a, Grid<Ctrl>& g, int32_t from, int32_t to, int32_t* last,
                             unsigned long long* scanned, int32_t* levels) {
  Ctrl* c = a.ctrl;
  const int lane = threadIdx.x & (kWave - 1), wib = threadIdx.x / kWave;
  const int64_t gw = (int64_t)g.rank * kWavesPerBlock + wib, nw = (int64_t)g.nblocks * kWavesPerBlock;
  for (int64_t v = (int64_t)g.rank * kBlock + threadIdx.x; v < a.n; v += (int64_t)g.nblocks * kBlock)
    a.parent[v] = kUnreached;
  if (g.rank == 0 && threadIdx.x == 0) {
    st_agent(&c->hit, kNoHit);
    st_agent(&c->fcount[0], 0u);
    st_agent(&c->fcount[1], 0u);
  }
  if (!grid_sync(g, 0, nullptr)) return -1;
  if (g.rank == 0 && threadIdx.x == 0) {
    a.front[0][0] = from;
    a.parent[from] = 0xffffffffull;  // level 0, low word -1
  }
  if (!grid_sync(g, 0, nullptr)) return -1;
  uint64_t* parent = a.parent;
  uint32_t size = 1;
  int fc = 0;
  for (int32_t level = 1;; ++level) {
    // This round reads frontier fc and appends to fc ^ 1, whose counter was
    // cleared before the barrier that opened the round; fc's counter is
    // appended to in the next round, after the barrier that closes this one.
    if (g.rank == 0 && threadIdx.x == 0) st_agent(&c->fcount[fc], 0u);
    const int32_t* F = a.front[fc];
    int32_t* Fn = a.front[fc ^ 1];
    uint32_t* cn = &c->fcount[fc ^ 1];
    uint32_t napp = 0;
    for (int64_t i0 = gw * kWave; i0 < (int64_t)size; i0 += nw * kWave) {
      const int64_t i = i0 + lane;
      int32_t u = 0, k = 0;
      uint32_t deg = 0;
      if (i < (int64_t)size) {
        u = F[i];
        if ((uint32_t)u < (uint32_t)a.n) {
          k = a.row_ptr[u];
          deg = (uint32_t)(a.row_ptr[u + 1] - k);
        } else {
          st_agent(&c->bad, 1u);
        }
      }
      uint32_t incl = deg;
      for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, off, kWave);
        if (lane >= off) incl += y;
      }
      const uint32_t first = incl - deg;
      const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
      for (uint32_t q0 = 0; q0 < total; q0 += kWave * kExpandPerLane) {
        int32_t v[kExpandPerLane], src[kExpandPerLane];
        bool ok[kExpandPerLane], take[kExpandPerLane];
        uint32_t pw[kExpandPerLane];
#pragma unroll
        for (int s = 0; s < kExpandPerLane; ++s) {
          const uint32_t q = q0 + (uint32_t)(s * kWave + lane);
          const int o = slot_owner(q, first);
          const int32_t ko = __shfl(k, o, kWave);
          const uint32_t fo = (uint32_t)__shfl((int)first, o, kWave);
          src[s] = __shfl(u, o, kWave);
          ok[s] = q < total;
          v[s] = ok[s] ? a.col[ko + (int32_t)(q - fo)] : 0;
        }
        // Plain reads of the round in a parent word: words set in an earlier
        // round are final (they precede a barrier) and are skipped; an
        // unreached word or one of this round takes the atomic minimum.
#pragma unroll
        for (int s = 0; s < kExpandPerLane; ++s) {
          pw[s] = 0u;
          if (!ok[s]) continue;
          ++*scanned;
          if ((uint32_t)v[s] >= (uint32_t)a.n) {
            st_agent(&c->bad, 1u);
            ok[s] = false;
          } else if (v[s] == to) {
            __hip_atomic_fetch_min(&c->hit, (uint32_t)src[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok[s] = false;
          } else {
            pw[s] = (uint32_t)(parent[v[s]] >> 32);
          }
        }
#pragma unroll
        for (int s = 0; s < kExpandPerLane; ++s) {
          take[s] = false;
          if (ok[s] && pw[s] >= (uint32_t)level) {
            const uint64_t claim = ((uint64_t)(uint32_t)level << 32) | (uint32_t)(src[s] + 1);
            take[s] = __hip_atomic_fetch_min(&parent[v[s]], claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                      kUnreached;
          }
        }
        napp += frontier_append_n<kExpandPerLane>(Fn, cn, take, v, lane);
      }
    }
    uint32_t tot = 0;
    if (!grid_sync(g, lasso_block_sum(napp), &tot)) return -1;
    *levels += 1;
    if (ld_agent(&c->bad)) return 0;
    const uint32_t h = ld_agent(&c->hit);
    if (h != kNoHit) {
      *last = (int32_t)h;
      return level;
    }
    if (tot == 0) return 0;
    size = tot;
    fc ^= 1;
  }
}

// Walks parent words back from `x` and writes path[hi], path[hi-1], ...,
// path[lo] (ids); the word of the vertex written at path[lo] must name `root`.
// Single thread.  Returns false if the chain does not end there.
__device__ bool lasso_walk(const LassoArgs& a, int32_t x, int32_t hi, int32_t lo, int32_t root) {
  for (int32_t i = hi; i >= lo; --i) {
    if ((uint32_t)x >= (uint32_t)a.n) return false;
    a.path[i] = x + 1;
    const int32_t p = (int32_t)(uint32_t)__hip_atomic_load(&a.parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (i == lo) return p == root + 1 || (p == -1 && x == root);
    if (p <= 0) return false;
    x = p - 1;
  }
  return true;
}

__global__ void __launch_bounds__(kBlock) map_lasso_kernel(LassoArgs a) {
  Grid<Ctrl> g = whole_grid(a.ctrl);
  const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
  unsigned long long scanned = 0;
  int32_t levels = 0, S = 0, L = -1, last = 0;
  int32_t status = MAP_OK;
  bool written = false;
  if (a.init >= 0 && a.init != a.w) {
    S = lasso_bfs(a, g, a.init, a.w, &last, &scanned, &levels);
    if (S < 0) goto aborted;
    if (S == 0) {
      S = -1;
      status = MAP_ENOPATH;
    } else if (leader && (int64_t)S + 1 <= a.cap) {
      // s_S = w, s_{S-1} = last, ..., s_0 = init (parent word -1)
      a.path[S] = a.w + 1;
      if (!lasso_walk(a, last, S - 1, 0, a.init)) status = MAP_EDEVICE;
    }
    // The stem's parent words are read above before the next search clears them.
    if (!grid_sync(g, 0, nullptr)) goto aborted;
  }
  if (status == MAP_OK) {
    L = lasso_bfs(a, g, a.w, a.w, &last, &scanned, &levels);
    if (L < 0) goto aborted;
    if (L == 0) {
      L = -1;
      status = MAP_ENOPATH;
    } else if ((int64_t)S + L + 1 > a.cap) {
      status = MAP_ENOSPC;
    } else if (leader) {
      // c_L = w, c_{L-1} = last, ..., c_1 (parent word names w)
      a.path[S + L] = a.w + 1;
      if (S == 0) a.path[0] = a.w + 1;
      if (L > 1 && !lasso_walk(a, last, S + L - 1, S + 1, a.w)) status = MAP_EDEVICE;
      if (L == 1 && last != a.w) status = MAP_EDEVICE;
      written = status == MAP_OK;
    }
  }
  {
    // Edges examined: one atomic per wave, read after a last barrier.
    const unsigned long long ws = wave_sum_u64(scanned);
    if ((threadIdx.x & (kWave - 1)) == 0 && ws)
      __hip_atomic_fetch_add(&a.ctrl->scanned, ws, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!grid_sync(g, 0, nullptr)) goto aborted;
  }
  if (leader) {
    if (ld_agent(&a.ctrl->bad)) status = MAP_ERANGE_DEV;
    map_lasso_result* r = a.result;
    r->status = status;
    r->stem_len = status == MAP_ENOPATH && S < 0 ? -1 : S;
    r->cycle_len = L;
    r->path_len = written && status == MAP_OK ? S + L + 1 : 0;
    r->edges_scanned = (int64_t)__hip_atomic_load(&a.ctrl->scanned, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    r->levels = levels;
    r->reserved = 0;
  }
  return;
aborted:
  if (leader) {
    a.result->status = MAP_EDEVICE;
    a.result->path_len = 0;
  }
}

// ---------------------------------------------------------------- pruning --

// Arguments of the trim of cycle-free vertices.
struct TrimArgs {
  int32_t n;
  const int32_t* row_ptr;  // pull CSR of G: row v = successors
  const int32_t* col;
  const int32_t* rrow_ptr; // transposed CSR: row v = predecessors
  const int32_t* rcol;
  const uint8_t* acc_in;   // or nullptr
  uint8_t* keep_out;
  uint8_t* acc_out;        // or nullptr
  map_trim_result* result;
  uint32_t* indeg;         // [n] in-edges from vertices not removed
  uint32_t* outdeg;        // [n] out-edges to vertices not removed
  uint32_t* removed;       // [n] 1 once removed (claimed by compare-and-swap)
  int32_t* front[2];
  Ctrl* ctrl;
};

// Removes, while one exists, a vertex with no remaining predecessor or no
// remaining successor (parallel edges counted with multiplicity), in rounds:
// the first frontier is every vertex with no in-edge or no out-edge; a round
// takes a frontier of removed vertices, subtracts each one's out-edges from
// its successors' in-counts and its in-edges from its predecessors'
// out-counts, and a vertex whose count reaches 0 is claimed (compare-and-swap
// on its removed word) and appended to the next frontier.  A grid barrier
// ends each round and carries the next frontier's size.  A vertex on a cycle
// always keeps an in-edge and an out-edge from the cycle, so it is never
// removed.
__global__ void __launch_bounds__(kBlock) map_trim_kernel(TrimArgs a) {
  Grid<Ctrl> g = whole_grid(a.ctrl);
  Ctrl* c = a.ctrl;
  const int lane = threadIdx.x & (kWave - 1), wib = threadIdx.x / kWave;
  const int64_t gw = (int64_t)g.rank * kWavesPerBlock + wib, nw = (int64_t)g.nblocks * kWavesPerBlock;
  const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
  int32_t rounds = 0;
  uint32_t napp = 0, size = 0, kept = 0, acc_kept = 0;
  int fc = 0;
  // Counts, and the first frontier into front[0] (counter fcount[0], zero).
  for (int64_t v0 = gw * kWave; v0 < a.n; v0 += nw * kWave) {
    const int64_t v = v0 + lane;
    bool take = false;
    if (v < a.n) {
      const uint32_t in = (uint32_t)(a.rrow_ptr[v + 1] - a.rrow_ptr[v]);
      const uint32_t out = (uint32_t)(a.row_ptr[v + 1] - a.row_ptr[v]);
      a.indeg[v] = in;
      a.outdeg[v] = out;
      take = in == 0 || out == 0;
      a.removed[v] = take ? 1u : 0u;
    }
    napp += frontier_append(a.front[0], &c->fcount[0], take, (int32_t)v, lane);
  }
  if (!grid_sync(g, lasso_block_sum(napp), &size)) goto aborted;
  while (size > 0) {
    // Frontier fc is read and fc ^ 1 appended to (its counter is zero: it was
    // cleared in the round that read it, before the barrier that closed it).
    if (g.rank == 0 && threadIdx.x == 0) st_agent(&c->fcount[fc], 0u);
    const int32_t* F = a.front[fc];
    int32_t* Fn = a.front[fc ^ 1];
    uint32_t* cn = &c->fcount[fc ^ 1];
    napp = 0;
    for (int64_t i0 = gw * kWave; i0 < (int64_t)size; i0 += nw * kWave) {
      const int64_t i = i0 + lane;
      // A removed vertex's out-edges then its in-edges, flattened across the
      // wave (slots [0, dout) of a vertex are col entries, the rest rcol).
      int32_t k = 0, r = 0;
      uint32_t dout = 0, deg = 0;
      if (i < (int64_t)size) {
        const int32_t v = F[i];
        if ((uint32_t)v < (uint32_t)a.n) {
          k = a.row_ptr[v];
          r = a.rrow_ptr[v];
          dout = (uint32_t)(a.row_ptr[v + 1] - k);
          deg = dout + (uint32_t)(a.rrow_ptr[v + 1] - r);
        } else {
          st_agent(&c->bad, 1u);
        }
      }
      uint32_t incl = deg;
      for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, off, kWave);
        if (lane >= off) incl += y;
      }
      const uint32_t first = incl - deg;
      const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
      for (uint32_t q0 = 0; q0 < total; q0 += kWave * kExpandPerLane) {
        int32_t x[kExpandPerLane];
        bool ok[kExpandPerLane], out_e[kExpandPerLane], take[kExpandPerLane];
        uint32_t old[kExpandPerLane];
#pragma unroll
        for (int s = 0; s < kExpandPerLane; ++s) {
          const uint32_t q = q0 + (uint32_t)(s * kWave + lane);
          const int o = slot_owner(q, first);
          const int32_t ko = __shfl(k, o, kWave), ro = __shfl(r, o, kWave);
          const uint32_t fo = (uint32_t)__shfl((int)first, o, kWave);
          const uint32_t dout_o = (uint32_t)__shfl((int)dout, o, kWave);
          const uint32_t j = q - fo;
          ok[s] = q < total;
          out_e[s] = j < dout_o;
          x[s] = ok[s] ? (out_e[s] ? a.col[ko + (int32_t)j] : a.rcol[ro + (int32_t)(j - dout_o)]) : 0;
        }
#pragma unroll
        for (int s = 0; s < kExpandPerLane; ++s) {
          old[s] = 0u;
          if (!ok[s]) continue;
          if ((uint32_t)x[s] >= (uint32_t)a.n) {
            st_agent(&c->bad, 1u);
            ok[s] = false;
            continue;
          }
          uint32_t* cnt = out_e[s] ? &a.indeg[x[s]] : &a.outdeg[x[s]];
          old[s] = __hip_atomic_fetch_sub(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (int s = 0; s < kExpandPerLane; ++s) {
          take[s] = false;
          if (ok[s] && old[s] == 1u) {
            uint32_t zero = 0;
            take[s] = __hip_atomic_compare_exchange_strong(&a.removed[x[s]], &zero, 1u, __ATOMIC_RELAXED,
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
        napp += frontier_append_n<kExpandPerLane>(Fn, cn, take, x, lane);
      }
    }
    if (!grid_sync(g, lasso_block_sum(napp), &size)) goto aborted;
    ++rounds;
    fc ^= 1;
  }
  // Outputs and counts.
  for (int64_t v = (int64_t)g.rank * kBlock + threadIdx.x; v < a.n; v += (int64_t)g.nblocks * kBlock) {
    const uint32_t keep = ld_agent(&a.removed[v]) ? 0u : 1u;
    a.keep_out[v] = (uint8_t)keep;
    kept += keep;
    if (a.acc_out) {
      const uint32_t ak = keep && a.acc_in[v] ? 1u : 0u;
      a.acc_out[v] = (uint8_t)ak;
      acc_kept += ak;
    }
  }
  kept = wave_sum_u32(kept);
  acc_kept = wave_sum_u32(acc_kept);
  if (lane == 0) {
    if (kept) __hip_atomic_fetch_add(&c->kept, kept, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (acc_kept) __hip_atomic_fetch_add(&c->acc_kept, acc_kept, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!grid_sync(g, 0, nullptr)) goto aborted;
  if (leader) {
    a.result->status = ld_agent(&c->bad) ? MAP_ERANGE_DEV : MAP_OK;
    a.result->kept = (int32_t)ld_agent(&c->kept);
    a.result->accepting_kept = (int32_t)ld_agent(&c->acc_kept);
    a.result->rounds = rounds;
  }
  return;
aborted:
  if (leader) a.result->status = MAP_EDEVICE;
}

// Scratch of one graph of a batch: the packed values (4n bytes), the working
// accepting flags (n), and with MAP_GRAPH_FILTER the three change bitmaps and
// the accepting bitmap of the filtered sweeps (ceil(n / 32) words each); every
// part 256-aligned.
__host__ __device__ inline int64_t gang_bitmap_bytes(int64_t n) { return ((((n + 31) / 32) * 4) + 255) & ~(int64_t)255; }
__host__ __device__ inline int64_t gang_scratch_bytes(int64_t n, int32_t options) {
  n = n < 1 ? 1 : n;
  const int64_t base = ((n * 4 + 255) & ~(int64_t)255) + ((n + 255) & ~(int64_t)255);
  return base + ((options & MAP_GRAPH_FILTER) ? 4 * gang_bitmap_bytes(n) : 0);
}

// Loop arguments of one graph solved by a gang, on its scratch.
__device__ LoopArgs gang_args(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* rrow_ptr,
                              const int32_t* rcol, const uint8_t* acc0, char* scratch, map_result* result,
                              uint32_t flags, int32_t options) {
  LoopArgs a;
  a.n = n;
  a.ntiles = (int32_t)(((int64_t)n + kTileRows - 1) / kTileRows);
  a.row_ptr = row_ptr;
  a.col = col;
  a.acc_in = acc0;
  a.pv = reinterpret_cast<uint32_t*>(scratch);
  a.accw = reinterpret_cast<uint8_t*>(scratch + (((size_t)n * 4 + 255) & ~(size_t)255));
  a.ctrl = nullptr;
  a.result = result;
  a.trace = nullptr;
  a.trace_cap = 0;
  a.acc_out = nullptr;
  a.map_out = nullptr;
  a.max_iter = 0;
  a.propagate = 0;
  a.digest = 0;
  a.force_stream = (flags & MAP_FLAG_STREAM) ? 1 : 0;
  a.sync_sweeps = (flags & MAP_FLAG_SYNC_SWEEPS) ? 1 : 0;
  word_layout(n, &a.val_mask, &a.tag_mask, &a.tag_shift);
  a.epoch = nullptr;
  a.push = 0;
  a.early = (flags & MAP_FLAG_EARLY) ? 1 : 0;
  a.rrow_ptr = nullptr;
  a.rcol = nullptr;
  a.front[0] = a.front[1] = nullptr;
  a.mark = nullptr;
  a.chg = nullptr;
  a.accb = nullptr;
  a.words = 0;
  a.filt = 0;
  a.dopt = 0;
  if ((options & MAP_GRAPH_FILTER) && !a.early) {
    // Filtered stream sweeps, a barrier after each (the change bitmaps follow
    // the working flags).
    const int64_t off = (((int64_t)n * 4 + 255) & ~(int64_t)255) + (((int64_t)n + 255) & ~(int64_t)255);
    const int64_t bb = gang_bitmap_bytes(n);
    a.chg = reinterpret_cast<uint32_t*>(scratch + off);
    a.accb = reinterpret_cast<uint32_t*>(scratch + off + 3 * bb);
    a.words = ((int64_t)n + 31) / 32;
    a.filt = 1;
    if ((options & MAP_GRAPH_DIRECTION) && rrow_ptr && rcol) {
      // Direction switch: small frontiers run as push rounds.
      a.dopt = 1;
      a.rrow_ptr = rrow_ptr;
      a.rcol = rcol;
    }
  }
  // Per-graph options of a batch (map_graph_desc.options): long-row threshold,
  // barrier per sweep, streamed CSR (filtered sweeps and the direction switch
  // above).
  a.hub = (options & MAP_GRAPH_HUB_MASK) ? (options & MAP_GRAPH_HUB_MASK) : kHubEdges;
  if (options & MAP_GRAPH_SYNC_SWEEPS) a.sync_sweeps = 1;
  if (options & MAP_GRAPH_STREAM) a.force_stream = 1;
  return a;
}

// Persistent work queue over the graphs of a batch.  Graph g is solved by
// item_start[g+1] - item_start[g] blocks (its gang); each block pops one item
// (graph, rank) at a time.  Items of a gang are consecutive in the queue, so a
// gang is always completed by blocks that free up, and it never waits on a
// later one.
__global__ void __launch_bounds__(kBlock) map_batch_kernel(BatchArgs ba) {
  __shared__ int32_t s_item;
  const int32_t total = ba.item_start[ba.count];
  if (__hip_atomic_load(ba.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != MAP_OK) {
    for (int32_t gi = blockIdx.x * blockDim.x + threadIdx.x; gi < ba.count; gi += gridDim.x * blockDim.x)
      ba.results[gi].status = MAP_ENOSPC;
    return;
  }
  for (;;) {
    if (threadIdx.x == 0) s_item = (int32_t)__hip_atomic_fetch_add(ba.next_item, 1u, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int32_t item = s_item;
    __syncthreads();
    if (item >= total) break;
    int32_t lo = 0, hi = ba.count;  // largest gi with item_start[gi] <= item
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (ba.item_start[mid] <= item) lo = mid; else hi = mid;
    }
    const int32_t gi = lo;
    const int nb = ba.item_start[gi + 1] - ba.item_start[gi];
    const int rank = item - ba.item_start[gi];
    const map_graph_desc d = ba.graphs[gi];
    if (d.n < 1 || d.n > 0x7ffffffe || !d.row_ptr || !d.col || !d.accepting0) {
      if (rank == 0 && threadIdx.x == 0) {
        ba.results[gi].status = MAP_EINVAL;
        ba.results[gi].found = ba.results[gi].witness = ba.results[gi].iterations = 0;
      }
      continue;
    }
    char* base = ba.scratch + ba.scratch_off[gi];
    const LoopArgs a = gang_args(d.n, d.row_ptr, d.col, d.rrow_ptr, d.rcol, d.accepting0, base, ba.results + gi,
                                 ba.flags, d.options);
    map_body_gang(a, ba.gctrl + gi, nb, rank);
  }
}

// ----------------------------------------------------------------- engine --
//
// A persistent server kernel: one cooperative launch that runs until the host
// asks it to stop.  The host posts jobs (an edge list to turn into a CSR and
// check) into fine-grained host memory; a job whose gang has g workgroups
// takes g consecutive tickets, each naming (job slot, rank).  Workgroups take
// tickets in order from a device counter, so, as in the batch queue, every gang
// is completed by workgroups that free up and never waits on a later ticket.
// Only the workgroup holding the first unpublished ticket polls host memory; it
// mirrors the host's ticket count into device memory for the other waiters.

struct EngineShared {          // fine-grained host memory, shared with the host
  unsigned long long tail;     // tickets published by the host
  uint32_t stop;               // host: exit once every published ticket is taken
  uint32_t expired;            // device: the idle bound elapsed and the engine exited
  uint32_t pad[28];
};
static_assert(sizeof(EngineShared) == 128, "shared block is one 128-byte line");

struct alignas(128) EngineDev {  // device memory
  unsigned long long head;       // next ticket to hand out
  unsigned long long pad0[15];
  unsigned long long mirror;     // the host's ticket count as last seen by the polling workgroup
  unsigned long long pad1[15];
  uint32_t quit;                 // 1: no further ticket will be published
  uint32_t pad2[31];
};

// A job as the engine reads it: the caller's map_job with its inputs resolved
// to device addresses, and whether the edge list lies in host memory.
struct EngineJob {
  map_job j;
  uint64_t host_edges;
};
static_assert(sizeof(EngineJob) % 8 == 0, "jobs are read as 64-bit words");

struct EngineArgs {
  EngineShared* sh;                // device address of the shared host block
  const unsigned long long* ring;  // [ring_cap] host: (slot << 32) | rank
  const EngineJob* jobs;           // [slots] host
  map_result* hres;                // [slots] host: status MAP_PENDING until the job is done
  EngineDev* dev;
  GangCtrl* bctrl;                 // [slots] barriers of the CSR build
  GangCtrl* mctrl;                 // [slots] barriers of the MAP loop
  map_result* dres;                // [slots] device results
  unsigned long long* ready;       // [slots] first ticket + 1 of the job whose control blocks are zeroed
  int32_t ring_cap;
  int32_t slots;
  uint64_t idle_ticks;             // idle bound in device wall-clock ticks
  uint32_t flags;
};


__device__ uint32_t block_sum_u32(uint32_t x) {
  __shared__ uint32_t s_bs[kWavesPerBlock];
  x = wave_sum_u32(x);
  if ((threadIdx.x & (kWave - 1)) == 0) s_bs[threadIdx.x / kWave] = x;
  __syncthreads();
  uint32_t t = 0;
  for (int i = 0; i < kWavesPerBlock; ++i) t += s_bs[i];
  __syncthreads();
  return t;
}

// Inclusive scan of one value per thread over the block; *total = block sum.
__device__ uint32_t block_scan_u32(uint32_t x, uint32_t* total) {
  __shared__ uint32_t s_ws[kWavesPerBlock];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, off, kWave);
    if (lane >= off) x += y;
  }
  if (lane == kWave - 1) s_ws[w] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int i = 0; i < kWavesPerBlock; ++i) {
    const uint32_t v = s_ws[i];
    pre += i < w ? v : 0u;
    tot += v;
  }
  __syncthreads();
  *total = tot;
  return x + pre;
}

template <typename C>
__device__ Grid<C> make_grid(C* c, int nb, int b) {
  Grid<C> g;
  g.c = c;
  g.gen = 0;
  g.nblocks = nb;
  g.ngroups = min(nb, kMaxGroups);
  g.group = b % g.ngroups;
  g.group_size = nb / g.ngroups + ((b % g.ngroups) < (nb % g.ngroups) ? 1 : 0);
  g.rank = b;
  return g;
}

// Calls f(src[e], dst[e]) for the edges e = gt, gt + gs, ... of [0, m), and
// copies them to copy_src / copy_dst when those are given.  The arrays may
// live in host memory, where every load is a bus round trip, so when both are
// 16-byte aligned they are read four edges at a time with two such loads per
// array in flight.
template <typename F>
__device__ __forceinline__ void for_edges(const int32_t* src, const int32_t* dst, int64_t m, int64_t gt,
                                          int64_t gs, int32_t* copy_src, int32_t* copy_dst, F f) {
  int64_t e0 = 0;
  if (((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0) {
    const int64_t q = m / 4;
    const int4* s4 = reinterpret_cast<const int4*>(src);
    const int4* d4 = reinterpret_cast<const int4*>(dst);
    int64_t i = gt;
    for (; i + gs < q; i += 2 * gs) {
      const int4 a = s4[i], b = d4[i], c = s4[i + gs], d = d4[i + gs];
      if (copy_src) {
        reinterpret_cast<int4*>(copy_src)[i] = a;
        reinterpret_cast<int4*>(copy_dst)[i] = b;
        reinterpret_cast<int4*>(copy_src)[i + gs] = c;
        reinterpret_cast<int4*>(copy_dst)[i + gs] = d;
      }
      f(a.x, b.x);
      f(a.y, b.y);
      f(a.z, b.z);
      f(a.w, b.w);
      f(c.x, d.x);
      f(c.y, d.y);
      f(c.z, d.z);
      f(c.w, d.w);
    }
    if (i < q) {
      const int4 a = s4[i], b = d4[i];
      if (copy_src) {
        reinterpret_cast<int4*>(copy_src)[i] = a;
        reinterpret_cast<int4*>(copy_dst)[i] = b;
      }
      f(a.x, b.x);
      f(a.y, b.y);
      f(a.z, b.z);
      f(a.w, b.w);
    }
    e0 = q * 4;
  }
  for (int64_t e = e0 + gt; e < m; e += gs) {
    const int32_t a = src[e], b = dst[e];
    if (copy_src) {
      copy_src[e] = a;
      copy_dst[e] = b;
    }
    f(a, b);
  }
}

// Pull CSR of a job's edge list, built by its gang: the same arrays that
// map_build_csr produces, up to the order of columns inside a row.  cursor is
// int32[n] and part uint32[nb] of scratch.  With stage_src / stage_dst (edge
// list in host memory) the histogram pass also copies the edges there, so the
// bus is crossed once and the scatter reads device memory.  Returns false if a
// gang barrier timed out; *bad = edges with an endpoint outside 1..n (the CSR
// is then unspecified and the gang stops after the histogram).
__device__ bool gang_build_csr(const map_job& j, int32_t* cursor, uint32_t* part, int32_t* stage_src,
                               int32_t* stage_dst, Grid<GangCtrl>& g, int nb, int rank, uint32_t* bad,
                               int32_t* rp, int32_t* col, const int32_t* esrc, const int32_t* edst, bool swap) {
  const int32_t n = j.n;
  const int64_t m = j.m;
  const int64_t gt = (int64_t)rank * kBlock + threadIdx.x, gs = (int64_t)nb * kBlock;
  for (int64_t i = gt; i <= n; i += gs) rp[i] = 0;
  if (!grid_sync(g, 0u, nullptr)) return false;
  // Degree histogram: the count of row v (vertex v+1) lands at rp[v+1].
  uint32_t nbad = 0;
  for_edges(esrc, edst, m, gt, gs, stage_src, stage_dst, [&](int32_t s, int32_t d) {
    if (s < 1 || s > n || d < 1 || d > n) {
      ++nbad;
      return;
    }
    __hip_atomic_fetch_add(&rp[swap ? d : s], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  });
  nbad = block_sum_u32(nbad);
  uint32_t tot = 0;
  if (!grid_sync(g, nbad, &tot)) return false;
  *bad = tot;
  if (tot) return true;
  // Inclusive scan of rp[0..n]: chunk totals, then each block scans its chunk
  // from the sum of the chunks before it.
  const int64_t len = (int64_t)n + 1, chunk = (len + nb - 1) / nb;
  const int64_t lo = min(len, (int64_t)rank * chunk), hi = min(len, lo + chunk);
  uint32_t sum = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) sum += (uint32_t)rp[i];
  sum = block_sum_u32(sum);
  if (threadIdx.x == 0) st_agent(&part[rank], sum);
  if (!grid_sync(g, 0u, nullptr)) return false;
  uint32_t off = 0;
  for (int i = threadIdx.x; i < rank; i += kBlock) off += ld_agent(&part[i]);
  off = block_sum_u32(off);
  for (int64_t base = lo; base < hi; base += kBlock) {
    const int64_t i = base + threadIdx.x;
    uint32_t piece = 0;
    const uint32_t incl = block_scan_u32(i < hi ? (uint32_t)rp[i] : 0u, &piece);
    if (i < hi) rp[i] = (int32_t)(off + incl);
    off += piece;
  }
  if (!grid_sync(g, 0u, nullptr)) return false;
  for (int64_t r = gt; r < n; r += gs) cursor[r] = rp[r];
  if (!grid_sync(g, 0u, nullptr)) return false;
  const int32_t* src = stage_src ? stage_src : esrc;
  const int32_t* dst = stage_src ? stage_dst : edst;
  for_edges(src, dst, m, gt, gs, nullptr, nullptr, [&](int32_t s, int32_t d) {
    const int32_t r = swap ? d : s, c = swap ? s : d;
    const int32_t pos = __hip_atomic_fetch_add(&cursor[r - 1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    col[pos] = c - 1;
  });
  return grid_sync(g, 0u, nullptr);
}

// One ticket of a job: rank `rank` of its gang.  Rank 0 zeroes the job's
// control blocks before any rank uses them, and publishes the result to host
// memory after every other rank has left the job.
__device__ __noinline__ void engine_job(const EngineArgs& ea, int slot, int rank, unsigned long long start) {
  constexpr int kJobWords = (int)(sizeof(EngineJob) / 8);
  __shared__ unsigned long long s_job[kJobWords];
  __shared__ int s_ready;
  if (threadIdx.x < kJobWords)
    s_job[threadIdx.x] = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(ea.jobs + slot) + threadIdx.x,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __syncthreads();
  EngineJob ej;
  memcpy(&ej, s_job, sizeof(ej));
  const map_job& j = ej.j;
  const int nb = max(1, min(j.gang, min((int)gridDim.x, kMaxGang)));
  GangCtrl* bc = ea.bctrl + slot;
  GangCtrl* mcx = ea.mctrl + slot;
  map_result* res = ea.dres + slot;
  char* sc = static_cast<char*>(j.scratch);
  // Scratch: packed values | working flags | bitmaps of the filtered sweeps |
  // scan partials | staged edge list (src, dst) | transposed CSR.
  const size_t pv_bytes = ((size_t)j.n * 4 + 255) & ~(size_t)255;
  const size_t acc_bytes = ((size_t)j.n + 255) & ~(size_t)255;
  const size_t bm_bytes = 4 * (size_t)gang_bitmap_bytes(j.n);
  const size_t edge_bytes = ((size_t)j.m * 4 + 255) & ~(size_t)255;
  char* part = sc + pv_bytes + acc_bytes + bm_bytes;
  char* stage = part + (size_t)kMaxGang * 4;
  int32_t* rrow = reinterpret_cast<int32_t*>(stage + 2 * edge_bytes);
  int32_t* rcol = reinterpret_cast<int32_t*>(stage + 2 * edge_bytes + (((size_t)j.n * 4 + 4 + 255) & ~(size_t)255));
  const bool dir = (ea.flags & MAP_FLAG_DIRECTION) != 0;

  if (rank == 0) {
    uint32_t* pb = reinterpret_cast<uint32_t*>(bc);
    uint32_t* pm = reinterpret_cast<uint32_t*>(mcx);
    for (int i = threadIdx.x; i < (int)(kGangCtrlBytes / 4); i += kBlock) {
      pb[i] = 0u;
      pm[i] = 0u;
    }
    if (threadIdx.x < 8) reinterpret_cast<uint32_t*>(res)[threadIdx.x] = 0u;
    wave_writes_done();
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(ea.ready + slot, start + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_ready = 1;
    }
  } else if (threadIdx.x == 0) {
    int ok = 1;
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(ea.ready + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != start + 1) {
      __builtin_amdgcn_s_sleep(2);
      if (wall_clock64() - t0 > kWaitTicks) {
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ready = ok;
  }
  __syncthreads();
  bool ok = s_ready != 0;
  uint32_t bad = 0;
  if (ok) {
    Grid<GangCtrl> g = make_grid(bc, nb, rank);
    int32_t* ss = ej.host_edges ? reinterpret_cast<int32_t*>(stage) : nullptr;
    int32_t* sd = ej.host_edges ? reinterpret_cast<int32_t*>(stage + edge_bytes) : nullptr;
    ok = gang_build_csr(j, reinterpret_cast<int32_t*>(sc), reinterpret_cast<uint32_t*>(part), ss, sd, g, nb, rank,
                        &bad, j.row_ptr, j.col, j.src, j.dst, false);
    // MAP_FLAG_DIRECTION: the transposed CSR too, from the staged copy of a
    // host edge list.
    if (ok && bad == 0 && dir)
      ok = gang_build_csr(j, reinterpret_cast<int32_t*>(sc), reinterpret_cast<uint32_t*>(part), nullptr, nullptr, g,
                          nb, rank, &bad, rrow, rcol, ss ? ss : j.src, ss ? sd : j.dst, true);
  }
  if (ok && bad == 0) {
    const LoopArgs a = gang_args(j.n, j.row_ptr, j.col, dir ? rrow : nullptr, dir ? rcol : nullptr, j.accepting0, sc,
                                 res, ea.flags, dir ? (MAP_GRAPH_FILTER | MAP_GRAPH_DIRECTION) : 0);
    map_body_gang(a, mcx, nb, rank);
  }
  // Leave the job: release this block's writes, then report (ranks > 0) or
  // wait for the others and publish the result (rank 0).
  wave_writes_done();
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (rank != 0) {
      __hip_atomic_fetch_add(&bc->dirty, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      int waited = 1;
      const uint64_t t0 = wall_clock64();
      while (ld_agent(&bc->dirty) != (uint32_t)(nb - 1)) {
        __builtin_amdgcn_s_sleep(2);
        if (wall_clock64() - t0 > kWaitTicks) {
          waited = 0;
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const int32_t* d = reinterpret_cast<const int32_t*>(res);
      int32_t r[8];
      for (int i = 0; i < 8; ++i) r[i] = __hip_atomic_load(d + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const bool broken = !ok || !waited || ld_agent((const uint32_t*)&bc->abort) ||
                          ld_agent((const uint32_t*)&mcx->abort);
      if (broken || bad) {
        for (int i = 0; i < 8; ++i) r[i] = 0;
        r[3] = broken ? MAP_EDEVICE : MAP_ERANGE_DEV;
      }
      int32_t* h = reinterpret_cast<int32_t*>(ea.hres + slot);
      for (int i = 0; i < 8; ++i)
        if (i != 3) __hip_atomic_store(h + i, r[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
      __hip_atomic_store(h + 3, r[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kBlock) map_engine_kernel(EngineArgs ea) {
  __shared__ int32_t s_slot, s_rank, s_quit;
  __shared__ unsigned long long s_start;
  for (;;) {
    if (threadIdx.x == 0) {
      const unsigned long long t =
          __hip_atomic_fetch_add(&ea.dev->head, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int quit = 0;
      uint64_t t0 = wall_clock64();
      unsigned long long seen = ~0ull;
      for (;;) {
        const unsigned long long mir = __hip_atomic_load(&ea.dev->mirror, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t < mir) break;
        if (ld_agent(&ea.dev->quit)) {
          quit = 1;
          break;
        }
        if (mir != seen) {  // progress: restart the idle clock
          seen = mir;
          t0 = wall_clock64();
        }
        if (t == mir) {
          // This block holds the first unpublished ticket: it polls the host.
          unsigned long long tail = __hip_atomic_load(&ea.sh->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          if (tail == mir && __hip_atomic_load(&ea.sh->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
            // The host publishes before it stops: read the count once more.
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            tail = __hip_atomic_load(&ea.sh->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (tail == mir) {
              st_agent(&ea.dev->quit, 1u);
              quit = 1;
              break;
            }
          }
          if (tail > mir) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            __hip_atomic_store(&ea.dev->mirror, tail, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            continue;
          }
        }
        if (wall_clock64() - t0 > ea.idle_ticks) {
          st_agent(&ea.dev->quit, 1u);
          __hip_atomic_store(&ea.sh->expired, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          quit = 1;
          break;
        }
        if (t == mir) __builtin_amdgcn_s_sleep(1);
        else __builtin_amdgcn_s_sleep(8);
      }
      s_quit = quit;
      if (!quit) {
        // Acquire the host's writes of the ticket, its job and the job's device
        // buffers (filled by copies the host waited for before publishing).
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        const unsigned long long e = __hip_atomic_load(ea.ring + (t % (unsigned long long)ea.ring_cap),
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        s_slot = (int32_t)(e >> 32);
        s_rank = (int32_t)(e & 0xffffffffu);
        s_start = t - (e & 0xffffffffu);
      }
    }
    __syncthreads();
    const int quit = s_quit, slot = s_slot, rank = s_rank;
    const unsigned long long start = s_start;
    __syncthreads();
    if (quit) break;
    if (slot >= 0 && slot < ea.slots) engine_job(ea, slot, rank, start);
  }
}

// Batch set-up (one block): gang sizes -> work item offsets, scratch offsets,
// and the scratch size check.
__global__ void __launch_bounds__(1024) batch_plan(int32_t count, const map_graph_desc* graphs,
                                                   const int32_t* gang, int32_t* item_start, int64_t* scratch_off,
                                                   size_t scratch_bytes, int32_t max_gang, int32_t* status,
                                                   uint32_t* next_item) {
  __shared__ int64_t part_i[1024];
  __shared__ int64_t part_b[1024];
  const int64_t per = ((int64_t)count + 1023) / 1024;
  const int64_t lo = (int64_t)threadIdx.x * per, hi = min((int64_t)count, lo + per);
  int64_t si = 0, sb = 0;
  for (int64_t i = lo; i < hi; ++i) {
    int32_t gsz = gang ? gang[i] : 1;
    gsz = max(1, min(gsz, max_gang));
    si += gsz;
    sb += gang_scratch_bytes(graphs[i].n, graphs[i].options);
  }
  part_i[threadIdx.x] = si;
  part_b[threadIdx.x] = sb;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t yi = threadIdx.x >= off ? part_i[threadIdx.x - off] : 0;
    const int64_t yb = threadIdx.x >= off ? part_b[threadIdx.x - off] : 0;
    __syncthreads();
    part_i[threadIdx.x] += yi;
    part_b[threadIdx.x] += yb;
    __syncthreads();
  }
  int64_t pi = threadIdx.x ? part_i[threadIdx.x - 1] : 0;
  int64_t pb = threadIdx.x ? part_b[threadIdx.x - 1] : 0;
  for (int64_t i = lo; i < hi; ++i) {
    item_start[i] = (int32_t)pi;
    scratch_off[i] = pb;
    int32_t gsz = gang ? gang[i] : 1;
    pi += max(1, min(gsz, max_gang));
    pb += gang_scratch_bytes(graphs[i].n, graphs[i].options);
  }
  if (threadIdx.x == 1023) {
    item_start[count] = (int32_t)part_i[1023];
    *status = (size_t)part_b[1023] <= scratch_bytes ? MAP_OK : MAP_ENOSPC;
    *next_item = 0;
  }
}

// --------------------------------------------------------------- CSR build --

// CSR build: the path a build takes, chosen on the device (csr_pick) and read
// by every kernel of both paths, which return at once when it is not theirs.
constexpr int32_t kBuildAtomic = 1;  // per-row cursors, one atomic per run of equal keys, then row ordering
constexpr int32_t kBuildRadix = 2;   // stable radix sort by key (keys mostly differ from their neighbour's)
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;

__global__ void fill_i32(int32_t* p, int64_t count, int32_t val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

__global__ void fill_u32(uint32_t* p, int64_t count, uint32_t val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

// Runs of equal keys among a wave's 64 consecutive edges.  Edge lists in
// generation order come grouped by source, so one atomic per run instead of
// one per edge takes most of the atomic traffic out of the build; on lists in
// random order nearly every run has length 1 and nothing changes.  A run
// starts at a valid lane whose key differs from the previous lane's (or whose
// previous lane is invalid, or at lane 0) and ends before the next start or
// invalid lane.  All 64 lanes must call it (the wave walks the edges in
// wave-aligned steps).
struct KeyRun {
  bool head;  // this lane starts a run
  int len;    // head: lanes in the run
  int first;  // valid lane: the lane that starts its run
};

__device__ __forceinline__ KeyRun key_run(bool valid, int32_t k, int lane) {
  const int32_t pk = __shfl_up(k, 1, kWave);
  const int pv = __shfl_up(valid ? 1 : 0, 1, kWave);
  const bool head = valid && (lane == 0 || pv == 0 || pk != k);
  const unsigned long long heads = __ballot(head);
  const unsigned long long stops = heads | ~__ballot(valid);
  const unsigned long long upto = (2ull << lane) - 1ull;  // lanes 0..lane (all 64 for lane 63)
  const unsigned long long after = stops & ~upto;
  KeyRun r;
  r.head = head;
  r.len = (after ? __builtin_ctzll(after) : kWave) - lane;
  const unsigned long long before = heads & upto;
  r.first = before ? 63 - __builtin_clzll(before) : lane;
  return r;
}

// Degree histogram of the key endpoint: cnt[key] += (edges with that key)
// (cnt = row_ptr, so row v's count lands at index v+1 for 1-based key v+1).
__global__ void csr_hist(const int32_t* gate, int32_t n, int64_t m, const int32_t* __restrict__ key,
                         const int32_t* __restrict__ other, int32_t* cnt, int32_t* status) {
  if (*gate != kBuildAtomic) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1)); w0 < m; w0 += stride) {
    const int64_t i = w0 + lane;
    int32_t k = 0;
    bool valid = false;
    if (i < m) {
      const int32_t o = other[i];
      k = key[i];
      valid = k >= 1 && k <= n && o >= 1 && o <= n;
      if (!valid) __hip_atomic_store(status, (int32_t)MAP_ERANGE_DEV, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const KeyRun r = key_run(valid, k, lane);
    if (r.head) atomicAdd(&cnt[k], r.len);
  }
}

// In-place inclusive scan of each tile of kScanTile elements; tile totals to sums.
__global__ void __launch_bounds__(kScanThreads) scan_tiles(const int32_t* gate, int32_t want, int32_t* a, int64_t len,
                                                          int32_t* sums) {
  if (*gate != want) return;
  __shared__ int32_t part[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  int32_t x[kScanPer];
  int32_t run = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    int64_t i = base + j;
    run += (i < len) ? a[i] : 0;
    x[j] = run;
  }
  part[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int32_t y = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += y;
    __syncthreads();
  }
  int32_t pre = threadIdx.x ? part[threadIdx.x - 1] : 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    int64_t i = base + j;
    if (i < len) a[i] = x[j] + pre;
  }
  if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = part[kScanThreads - 1];
}

// Exclusive scan of the tile totals by one workgroup.
__global__ void __launch_bounds__(1024) scan_sums(const int32_t* gate, int32_t want, int32_t* sums, int64_t count) {
  if (*gate != want) return;
  __shared__ int32_t part[1024];
  const int64_t per = (count + 1023) / 1024;
  const int64_t lo = (int64_t)threadIdx.x * per, hi = min(count, lo + per);
  int32_t run = 0;
  for (int64_t i = lo; i < hi; ++i) run += sums[i];
  part[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int32_t y = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += y;
    __syncthreads();
  }
  int32_t pre = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (int64_t i = lo; i < hi; ++i) {
    int32_t v = sums[i];
    sums[i] = pre;
    pre += v;
  }
}

__global__ void scan_add(const int32_t* gate, int32_t want, int32_t* a, int64_t len, const int32_t* sums) {
  if (*gate != want) return;
  const int64_t tile = blockIdx.x;
  const int32_t pre = sums[tile];
  if (pre == 0) return;
  for (int64_t i = tile * kScanTile + threadIdx.x; i < min(len, (tile + 1) * kScanTile); i += blockDim.x) a[i] += pre;
}

__global__ void copy_i32(const int32_t* gate, int32_t* dst, const int32_t* src, int64_t count) {
  if (*gate != kBuildAtomic) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// col[cursor[key-1]++] = other-1 and ids[same slot] = edge index for every
// in-range edge; a run of equal keys reserves its slots with one atomic and
// fills them in edge order.  The order of the runs inside a row depends on the
// schedule; the csr_order_* kernels then put every row whose edge indices are
// out of order in edge order.
__global__ void csr_scatter(const int32_t* gate, int32_t n, int64_t m, const int32_t* __restrict__ key,
                            const int32_t* __restrict__ other, int32_t* cursor, int32_t* col, int32_t* ids) {
  if (*gate != kBuildAtomic) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1)); w0 < m; w0 += stride) {
    const int64_t i = w0 + lane;
    int32_t k = 0, o = 0;
    bool valid = false;
    if (i < m) {
      k = key[i];
      o = other[i];
      valid = k >= 1 && k <= n && o >= 1 && o <= n;
    }
    const KeyRun r = key_run(valid, k, lane);
    int32_t pos = 0;
    if (r.head) pos = atomicAdd(&cursor[k - 1], r.len);
    pos = __shfl(pos, r.first, kWave) + (lane - r.first);
    if (valid) {
      col[pos] = o - 1;
      ids[pos] = (int32_t)i;
    }
  }
}

// Putting each row in edge order: rows of at most kOrderShort edges by one
// lane, rows of at most 64 by one wave, longer rows by one workgroup.  A row
// whose edge indices already ascend (the usual case for edge lists grouped by
// source, where one wave's run fills most rows) is only read.
constexpr int kOrderShort = 16;
constexpr int kOrderChunk = 4096;   // long rows: entries sorted in LDS at a time
constexpr int kOrderThreads = 1024;
constexpr int kOrderLongGrid = 256;
constexpr int kOrderMidGrid = 1024;

// Appends `val` for every lane with `take` to list[count...] (from the back,
// list[back - 1 - index], when back > 0).  All 64 lanes must call it.
__device__ void wave_list_append(bool take, int32_t val, int32_t* list, int32_t* count, int64_t back, int lane) {
  const unsigned long long mask = __ballot(take);
  if (!mask) return;
  const int leader = __builtin_ctzll(mask);
  int32_t base = 0;
  if (lane == leader) base = atomicAdd(count, __popcll(mask));
  base = __shfl(base, leader, kWave);
  const int64_t idx = base + __popcll(mask & ((1ull << lane) - 1ull));
  if (take) list[back > 0 ? back - 1 - idx : idx] = val;
}

// A row of 2..W edges in one lane: its edge indices are loaded together (no
// branch between the loads, so their latencies overlap) and, unless they
// ascend, each column is written at the rank of its edge index in the row.
template <int W>
__device__ __forceinline__ void order_short_row(int32_t b, int32_t d, int32_t* col, const int32_t* __restrict__ ids) {
  int32_t e[W];
#pragma unroll
  for (int k = 0; k < W; ++k) e[k] = k < d ? ids[b + k] : INT32_MAX;
  bool sorted = true;
#pragma unroll
  for (int k = 1; k < W; ++k) sorted = sorted && e[k - 1] < e[k];
  if (sorted) return;
  int32_t o[W];
#pragma unroll
  for (int k = 0; k < W; ++k) o[k] = k < d ? col[b + k] : 0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    int rank = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) rank += e[q] < e[k] ? 1 : 0;
    if (k < d) col[b + rank] = o[k];
  }
}

// One lane per row of 2..kOrderShort edges (order_short_row, at the width of
// the wave's longest such row).  Rows of kOrderShort+1..64 edges go to the
// front of `lists` (count counts[0]), longer ones to its back (n entries,
// count counts[1]); both counts start at zero.  Waves step over the rows in
// grid strides (the launch grid is capped).
__global__ void csr_order_rows(const int32_t* gate, int32_t n, const int32_t* __restrict__ row_ptr, int32_t* col,
                               const int32_t* __restrict__ ids, int32_t* lists, int32_t* counts) {
  if (*gate != kBuildAtomic) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1)); r0 < n; r0 += stride) {
    const int64_t r = r0 + lane;
    int32_t b = 0, d = 0;
    if (r < n) {
      b = row_ptr[r];
      d = row_ptr[r + 1] - b;
    }
    wave_list_append(d > kOrderShort && d <= kWave, (int32_t)r, lists, &counts[0], 0, lane);
    wave_list_append(d > kWave, (int32_t)r, lists, &counts[1], n, lane);
    const bool mine = d >= 2 && d <= kOrderShort;
    int dm = mine ? d : 0;  // longest short row of the wave
    for (int off = kWave / 2; off > 0; off >>= 1) dm = max(dm, __shfl_xor(dm, off, kWave));
    if (!mine) continue;
    if (dm <= 4)
      order_short_row<4>(b, d, col, ids);
    else if (dm <= 8)
      order_short_row<8>(b, d, col, ids);
    else
      order_short_row<kOrderShort>(b, d, col, ids);
  }
}

// One wave per listed row of kOrderShort+1..64 edges: lane l holds entry l;
// unless the edge indices ascend, each lane counts the lanes with a smaller
// one and writes its column there.
__global__ void csr_order_mid(const int32_t* gate, const int32_t* __restrict__ row_ptr, int32_t* col,
                              const int32_t* __restrict__ ids, const int32_t* __restrict__ lists,
                              const int32_t* __restrict__ counts) {
  if (*gate != kBuildAtomic) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  const int32_t cnt = counts[0];
  for (int64_t li = gw; li < cnt; li += nw) {
    const int32_t r = lists[li];
    const int32_t b = row_ptr[r], d = row_ptr[r + 1] - b;
    const int32_t e = lane < d ? ids[b + lane] : INT32_MAX;
    const int32_t prev = __shfl_up(e, 1, kWave);
    if (!__ballot(lane > 0 && lane < d && prev > e)) continue;
    const int32_t o = lane < d ? col[b + lane] : 0;
    int rank = 0;
#pragma unroll
    for (int q = 0; q < kWave; ++q) rank += __builtin_amdgcn_readlane(e, q) < e ? 1 : 0;
    if (lane < d) col[b + rank] = o;  // every lane's read precedes (the ranks depend on all of them)
  }
}

// Compare-exchange step of an ascending bitonic sort over se/so[0, S): pairs
// (i, i ^ (k - 1)) on the first step of merge size k, else (i, i + j); the
// smaller edge index goes to the lower position.
__device__ void order_lds_step(int32_t* se, int32_t* so, int S, int k, int j, bool first) {
  for (int t = threadIdx.x; t < S / 2; t += blockDim.x) {
    const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
    const int p = first ? (i ^ (k - 1)) : (i + j);
    const int32_t x = se[i], y = se[p];
    if (x > y) {
      se[i] = y;
      se[p] = x;
      const int32_t z = so[i];
      so[i] = so[p];
      so[p] = z;
    }
  }
  __syncthreads();
}

// The same step over a whole row in global memory (E edge indices, O columns,
// d entries, P the power of two the network spans).  Positions d and beyond
// stand for +infinity: a pair that reaches one never exchanges.
__device__ void order_global_step(int32_t* E, int32_t* O, int64_t d, int64_t P, int64_t k, int64_t j, bool first) {
  for (int64_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
    const int64_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
    const int64_t p = first ? (i ^ (k - 1)) : (i + j);
    if (p >= d) continue;
    const int32_t x = E[i], y = E[p];
    if (x > y) {
      E[i] = y;
      E[p] = x;
      const int32_t z = O[i];
      O[i] = O[p];
      O[p] = z;
    }
  }
  __syncthreads();
}

// Entries [c0, c0 + S) of a row through LDS: either a whole bitonic sort of
// the chunk (k == 0) or the steps j = S/2 .. 1 of merge size k.  The entries
// below d go back to E and O, or only to O on the chunk's last pass.
__device__ void order_lds_chunk(int32_t* se, int32_t* so, int32_t* E, int32_t* O, int64_t d, int64_t c0, int S,
                                int64_t k, bool last) {
  for (int i = threadIdx.x; i < S; i += blockDim.x) {
    const int64_t g = c0 + i;
    se[i] = g < d ? E[g] : INT32_MAX;
    so[i] = g < d ? O[g] : 0;
  }
  __syncthreads();
  if (k == 0) {
    for (int kk = 2; kk <= S; kk <<= 1) {
      order_lds_step(se, so, S, kk, kk >> 1, true);
      for (int j = kk >> 2; j > 0; j >>= 1) order_lds_step(se, so, S, kk, j, false);
    }
  } else {
    for (int j = S >> 1; j > 0; j >>= 1) order_lds_step(se, so, S, 0, j, false);
  }
  for (int i = threadIdx.x; i < S; i += blockDim.x) {
    const int64_t g = c0 + i;
    if (g >= d) break;
    if (!last) E[g] = se[i];
    O[g] = so[i];
  }
  __syncthreads();
}

// One workgroup per listed row of more than 64 edges (from the back of
// `lists`, count counts[1]) whose edge indices do not ascend: an ascending
// bitonic sort of (edge index, column) pairs, in LDS for rows of up to
// kOrderChunk entries, else chunks sorted in LDS and merged by steps over the
// row in global memory (the row's edge indices are scratch).
__global__ void __launch_bounds__(kOrderThreads)
    csr_order_long(const int32_t* gate, int32_t n, const int32_t* __restrict__ row_ptr, int32_t* col, int32_t* ids,
                   const int32_t* __restrict__ lists, const int32_t* __restrict__ counts) {
  if (*gate != kBuildAtomic) return;
  __shared__ int32_t se[kOrderChunk];
  __shared__ int32_t so[kOrderChunk];
  const int32_t cnt = counts[1];
  for (int32_t li = blockIdx.x; li < cnt; li += gridDim.x) {
    const int32_t r = lists[(int64_t)n - 1 - li];
    const int64_t b = row_ptr[r];
    const int64_t d = (int64_t)row_ptr[r + 1] - b;
    int32_t* E = ids + b;
    int32_t* O = col + b;
    int descents = 0;
    for (int64_t i = 1 + threadIdx.x; i < d; i += blockDim.x) descents |= E[i - 1] > E[i] ? 1 : 0;
    if (!__syncthreads_or(descents)) continue;
    if (d <= kOrderChunk) {
      int S = 2 * kWave;
      while (S < d) S <<= 1;
      order_lds_chunk(se, so, E, O, d, 0, S, 0, true);
      continue;
    }
    int64_t P = kOrderChunk;
    while (P < d) P <<= 1;
    for (int64_t c0 = 0; c0 < d; c0 += kOrderChunk) order_lds_chunk(se, so, E, O, d, c0, kOrderChunk, 0, false);
    for (int64_t k = 2 * (int64_t)kOrderChunk; k <= P; k <<= 1) {
      order_global_step(E, O, d, P, k, k >> 1, true);
      for (int64_t j = k >> 2; j >= kOrderChunk; j >>= 1) order_global_step(E, O, d, P, k, j, false);
      for (int64_t c0 = 0; c0 < d; c0 += kOrderChunk) order_lds_chunk(se, so, E, O, d, c0, kOrderChunk, k, k == P);
    }
  }
}

// Picks the build path from 1024 evenly spaced pairs of neighbouring edges:
// when most pairs differ in key, runs of equal keys are short and every edge
// would take its own atomic, so the radix sort (bandwidth-bound) is taken.
// Below kRadixMinEdges edges the radix kernels are not even launched: their
// twenty-odd launches cost more than the atomics they would save.
constexpr int64_t kRadixMinEdges = 1 << 20;
__global__ void __launch_bounds__(1024) csr_pick(int64_t m, const int32_t* __restrict__ key, int32_t* mode) {
  __shared__ uint32_t s_diff;
  if (threadIdx.x == 0) s_diff = 0;
  __syncthreads();
  uint32_t d = 0;
  if (m >= kRadixMinEdges) {
    const int64_t i = (m - 1) * (int64_t)threadIdx.x / 1024;
    d = key[i] != key[i + 1] ? 1u : 0u;
  }
  d = wave_sum_u32(d);
  if ((threadIdx.x & (kWave - 1)) == 0 && d) atomicAdd(&s_diff, d);
  __syncthreads();
  if (threadIdx.x == 0) *mode = 2 * s_diff > 1024 ? kBuildRadix : kBuildAtomic;
}

// Radix path: a least-significant-digit radix sort of (key - 1, other - 1)
// pairs by key, stable in every pass, so each row lists its columns in edge
// order; an edge with an endpoint outside 1..n gets key n and sorts last.
// Digits of up to kRadixMaxBits bits; a tile of kRadixTile edges per
// workgroup, kRadixSub consecutive ones per wave.
constexpr int kRadixMaxBits = 7;
constexpr int kRadixBins = 1 << kRadixMaxBits;
constexpr int kRadixWaves = 8;
constexpr int kRadixThreads = kRadixWaves * kWave;
constexpr int kRadixSub = 1024;
constexpr int kRadixTile = kRadixWaves * kRadixSub;

// Key of edge i (0-based; n for an edge outside 1..n, which also marks status).
__device__ __forceinline__ int32_t radix_key_in(int32_t n, int64_t i, const int32_t* key, const int32_t* other,
                                                const int32_t* kin, int32_t* status) {
  if (kin) return kin[i];
  const int32_t k = key[i], o = other[i];
  const bool ok = k >= 1 && k <= n && o >= 1 && o <= n;
  if (!ok && status) __hip_atomic_store(status, (int32_t)MAP_ERANGE_DEV, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return ok ? k - 1 : n;
}

// Per tile, the count of each digit value: hist[digit * tiles + tile].
__global__ void __launch_bounds__(kRadixThreads)
    radix_count(const int32_t* gate, int32_t n, int64_t m, const int32_t* __restrict__ key,
                const int32_t* __restrict__ other, const int32_t* __restrict__ kin, int shift, int bits, int64_t tiles,
                int32_t* hist, int32_t* status) {
  if (*gate != kBuildRadix) return;
  __shared__ uint32_t h[kRadixBins];
  const uint32_t mask = (1u << bits) - 1u;
  for (int i = threadIdx.x; i <= (int)mask; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kRadixTile, t1 = min(m, t0 + kRadixTile);
  constexpr int kPer = kRadixTile / kRadixThreads;
  int32_t kk[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {  // every load of the thread in flight together
    const int64_t i = t0 + threadIdx.x + (int64_t)u * kRadixThreads;
    kk[u] = i < t1 ? radix_key_in(n, i, key, other, kin, status) : -1;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u)
    if (kk[u] >= 0) atomicAdd(&h[((uint32_t)kk[u] >> shift) & mask], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d <= (int)mask; d += blockDim.x) hist[(int64_t)d * tiles + blockIdx.x] = (int32_t)h[d];
}

// Stable scatter of one pass.  hist holds the inclusive scan of the counts
// (digit-major), so a tile's first slot for digit d is hist[d][tile] minus
// the tile's own count of d.  The tile is first sorted by digit in LDS, then
// written out a digit run at a time (consecutive threads, consecutive slots).
// Inside the tile the waves take their sub-ranges in order (per-wave counts,
// summed over the waves before), and a wave walks its sub-range 64 edges at a
// time: the lanes that share a digit (found bit by bit with ballots) take
// consecutive places in lane order, and the lowest of them advances the
// wave's cursor for that digit.
__global__ void __launch_bounds__(kRadixThreads)
    radix_scatter(const int32_t* gate, int32_t n, int64_t m, const int32_t* __restrict__ key,
                  const int32_t* __restrict__ other, const int32_t* __restrict__ kin, const int32_t* __restrict__ vin,
                  int shift, int bits, int64_t tiles, const int32_t* __restrict__ hist, int32_t* kout,
                  int32_t* vout) {
  if (*gate != kBuildRadix) return;
  __shared__ uint32_t off[kRadixWaves][kRadixBins];
  __shared__ uint32_t loc[kRadixBins];   // first place of each digit in the sorted tile
  __shared__ uint32_t gpos[kRadixBins];  // its first slot in the output
  __shared__ int32_t sk[kRadixTile];
  __shared__ int32_t sv[kRadixTile];
  const int lane = threadIdx.x & (kWave - 1), wib = threadIdx.x / kWave;
  const uint32_t mask = (1u << bits) - 1u;
  for (int i = threadIdx.x; i < kRadixWaves * kRadixBins; i += blockDim.x) off[i / kRadixBins][i % kRadixBins] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kRadixTile;
  const int32_t cnt = (int32_t)min((int64_t)kRadixTile, m - t0);
  const int64_t s0 = min(m, t0 + (int64_t)wib * kRadixSub);
  const int64_t s1 = min(m, s0 + kRadixSub);
  // The wave's sub-range in registers, every load in flight together: step u
  // holds edges s0 + 64u + lane.
  constexpr int kSteps = kRadixSub / kWave;
  int32_t kr[kSteps], vr[kSteps];
#pragma unroll
  for (int u = 0; u < kSteps; ++u) {
    const int64_t i = s0 + (int64_t)u * kWave + lane;
    kr[u] = vr[u] = 0;
    if (i < s1) {
      kr[u] = radix_key_in(n, i, key, other, kin, nullptr);
      vr[u] = vin ? vin[i] : other[i] - 1;
    }
  }
#pragma unroll
  for (int u = 0; u < kSteps; ++u)
    if (s0 + (int64_t)u * kWave + lane < s1) atomicAdd(&off[wib][((uint32_t)kr[u] >> shift) & mask], 1u);
  __syncthreads();
  // Per digit: the tile's total (into loc) and each wave's place before the
  // scan over digits.
  for (int d = threadIdx.x; d < kRadixBins; d += blockDim.x) {
    uint32_t run = 0;
    if (d <= (int)mask) {
      for (int w = 0; w < kRadixWaves; ++w) {
        const uint32_t c = off[w][d];
        off[w][d] = run;
        run += c;
      }
      gpos[d] = (uint32_t)hist[(int64_t)d * tiles + blockIdx.x] - run;
    }
    loc[d] = run;
  }
  __syncthreads();
  if (wib == 0) {
    // Exclusive scan of the digit totals, kRadixBins / 64 digits per lane.
    uint32_t v[kRadixBins / kWave], sum = 0;
#pragma unroll
    for (int j = 0; j < kRadixBins / kWave; ++j) {
      v[j] = loc[lane * (kRadixBins / kWave) + j];
      sum += v[j];
    }
    uint32_t incl = sum;
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)incl, o, kWave);
      if (lane >= o) incl += y;
    }
    uint32_t run = incl - sum;
#pragma unroll
    for (int j = 0; j < kRadixBins / kWave; ++j) {
      loc[lane * (kRadixBins / kWave) + j] = run;
      run += v[j];
    }
  }
  __syncthreads();
  const unsigned long long below = lane ? (~0ull >> (kWave - lane)) : 0ull;
#pragma unroll
  for (int u = 0; u < kSteps; ++u) {
    const bool ok = s0 + (int64_t)u * kWave + lane < s1;
    const int32_t kk = kr[u], vv = vr[u];
    const uint32_t d = ((uint32_t)kk >> shift) & mask;
    unsigned long long peers = __ballot(ok);
    for (int bit = 0; bit < bits; ++bit) {
      const unsigned long long one = __ballot(ok && ((d >> bit) & 1u));
      peers &= ((d >> bit) & 1u) ? one : ~one;
    }
    const uint32_t r = (uint32_t)__popcll(peers & below);
    if (ok) {
      const uint32_t lp = loc[d] + off[wib][d] + r;
      sk[lp] = kk;
      sv[lp] = vv;
    }
    // Every lane has read off[wib][d] above (the wave's LDS operations
    // complete in order) before the group's lowest lane advances it.
    if (ok && r == 0) off[wib][d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
    const int32_t kk = sk[j];
    const uint32_t d = ((uint32_t)kk >> shift) & mask;
    const uint32_t pos = gpos[d] + ((uint32_t)j - loc[d]);
    kout[pos] = kk;
    vout[pos] = sv[j];
  }
}

// Row pointers from the sorted keys: the rows (key of edge i-1, key of edge
// i] start at edge i (before the first edge: -1; after the last: n).
__global__ void radix_row_ptr(const int32_t* gate, int32_t n, int64_t m, const int32_t* __restrict__ ks,
                              int32_t* row_ptr) {
  if (*gate != kBuildRadix) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= m; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t prev = i == 0 ? -1 : (int64_t)ks[i - 1];
    const int64_t cur = i == m ? (int64_t)n : min((int64_t)ks[i], (int64_t)n);
    for (int64_t r = prev + 1; r <= cur; ++r) row_ptr[r] = (int32_t)i;
  }
}

// ------------------------------------------------------------------- host --

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool sizes_ok(int32_t n, int64_t m) { return n >= 1 && n <= 0x7ffffffe && m >= 0 && m <= 0x7fffffff; }

struct Layout {
  size_t ctrl, pv, accw, front0, front1, mark, aux, chg, accb, parent, cursor, sums, counts, ids, total;
  size_t rk[2], rv[2], rhist, rsums;  // CSR build, radix path (rk[0] shares the atomic path's ids)
  int64_t words;  // 32-bit words of one vertex bitmap
};

// m > 0 adds the CSR build's per-edge scratch.
Layout layout(int32_t n, int64_t m = 0) {
  Layout L;
  size_t off = 0;
  L.ctrl = off;
  off += align256(kCtrlBytes);
  const size_t region = off;
  // propagation / detection
  L.pv = off;
  off += align256((size_t)n * 4);
  L.accw = off;
  off += align256((size_t)n);
  // frontier sweeps
  L.front0 = off;
  off += align256((size_t)n * 4);
  L.front1 = off;
  off += align256((size_t)n * 4);
  L.mark = off;
  off += align256((size_t)n * 4);
  // pruning: removed flags
  L.aux = off;
  off += align256((size_t)n * 4);
  // lasso: 64-bit parent words over the mark and removed-flag arrays
  L.parent = L.mark;
  // filtered stream sweeps: three change bitmaps and the accepting bitmap
  L.words = ((int64_t)n + 31) / 32;
  L.chg = off;
  off += align256((size_t)L.words * 4 * 3);
  L.accb = off;
  off += align256((size_t)L.words * 4);
  size_t end_loop = off;
  // CSR build (shares the region after ctrl)
  off = region;
  L.cursor = off;
  off += align256(((size_t)n + 1) * 4);
  L.sums = off;
  off += align256((((size_t)n + 1 + kScanTile - 1) / kScanTile + 1) * 4);
  L.counts = off;  // two list counts, then the build path
  off += 256;
  const size_t per_edge = align256((size_t)(m > 0 ? m : 0) * 4);
  L.ids = off;  // edge index of every CSR slot (atomic path)
  L.rk[0] = off;
  off += per_edge;
  L.rv[0] = off;
  off += per_edge;
  L.rk[1] = off;
  off += per_edge;
  L.rv[1] = off;
  off += per_edge;
  const int64_t rtiles = ((m > 0 ? m : 0) + kRadixTile - 1) / kRadixTile;
  const int64_t rlen = (int64_t)kRadixBins * rtiles;
  L.rhist = off;
  off += align256((size_t)rlen * 4);
  L.rsums = off;
  off += align256(((size_t)(rlen + kScanTile - 1) / kScanTile + 1) * 4);
  size_t end_build = off;
  L.total = end_loop > end_build ? end_loop : end_build;
  return L;
}

struct DeviceInfo {
  int cus = 0;
  int blocks_per_cu = 0;
  int coop = 0;
};

std::mutex g_dev_mu;
DeviceInfo g_dev[64];

int device_info(DeviceInfo* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return MAP_EDEVICE;
  std::lock_guard<std::mutex> lock(g_dev_mu);
  DeviceInfo& d = g_dev[dev];
  if (d.cus == 0) {
    int cus = 0, coop = 0, nb = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return MAP_EDEVICE;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess) return MAP_EDEVICE;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(map_loop_kernel<true, false>), kBlock,
                                                     0) != hipSuccess)
      return MAP_EDEVICE;
    if (cus <= 0 || nb <= 0) return MAP_EDEVICE;
    d.cus = cus;
    d.coop = coop;
    d.blocks_per_cu = nb;
  }
  *out = d;
  return MAP_OK;
}

// Grid of the last loop-kernel launch (read by map_phase_counters).
std::atomic<int> g_last_grid{0};

int launch_loop(LoopArgs& a, hipStream_t stream) {
  DeviceInfo di;
  int rc = device_info(&di);
  if (rc) return rc;
  if (!di.coop) return MAP_EDEVICE;
  const int64_t need = ((int64_t)a.n + (int64_t)kWavesPerBlock * kTileRows - 1) / ((int64_t)kWavesPerBlock * kTileRows);
  int64_t grid = (int64_t)di.cus * di.blocks_per_cu;
  if (grid > need) grid = need;
  if (grid > kMaxBlocks) grid = kMaxBlocks;
  if (grid >= kMaxGroups) grid -= grid % kMaxGroups;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(fill_u32, dim3(8), dim3(256), 0, stream, reinterpret_cast<uint32_t*>(a.ctrl),
                     (int64_t)(kEpochOff / 4), 0u);
  if (hipGetLastError() != hipSuccess) return MAP_EDEVICE;
  void* args[] = {&a};
  // MAP_FLAG_EARLY runs with a grid barrier after every sweep (no asynchronous
  // early instantiation exists).
  // When no block can stage its slice on chip (or staging is refused) and the
  // workspace holds the change bitmaps, the filtered stream kernel runs: a
  // barrier after every sweep, gathers only from rows that grew.
  const int64_t rpb = ((int64_t)a.n + grid - 1) / grid;
  const int64_t rpw = (rpb + kWavesPerBlock - 1) / kWavesPerBlock;
  const bool all_stream = a.force_stream || a.n >= (1 << 24) || rpw > kResWaveRows;
  a.filt = (a.chg != nullptr && !a.early && !a.push && all_stream) ? 1 : 0;
  if (!a.filt) a.dopt = 0;
  const bool async = !a.filt && grid > 1 && !a.sync_sweeps && a.tag_mask != 0 && !a.early;
  const void* kernel =
      a.early ? reinterpret_cast<const void*>(map_loop_kernel<false, true>)
      : a.filt ? reinterpret_cast<const void*>(map_loop_kernel<false, false, true>)
               : (async ? reinterpret_cast<const void*>(map_loop_kernel<true, false>)
                        : reinterpret_cast<const void*>(map_loop_kernel<false, false>));
  if (hipLaunchCooperativeKernel(kernel, dim3((unsigned)grid), dim3(kBlock), args, 0, stream) != hipSuccess)
    return MAP_EDEVICE;
  g_last_grid.store((int)grid);
  return MAP_OK;
}

inline unsigned grid_for(int64_t work, int threads) {
  int64_t g = (work + threads - 1) / threads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Digit width and pass count of the radix path: keys 0..n (n: an edge outside
// 1..n) in passes of at most kRadixMaxBits bits.
static void radix_plan(int32_t n, int* passes, int* bits) {
  int k = 1;
  while (k < 31 && (1ll << k) <= (int64_t)n) ++k;
  *passes = (k + kRadixMaxBits - 1) / kRadixMaxBits;
  *bits = (k + *passes - 1) / *passes;
}

int build_one(int32_t n, int64_t m, const int32_t* key, const int32_t* other, int32_t* row_ptr, int32_t* col,
              int32_t* status, char* ws, const Layout& L, hipStream_t stream) {
  int32_t* cursor = reinterpret_cast<int32_t*>(ws + L.cursor);
  int32_t* sums = reinterpret_cast<int32_t*>(ws + L.sums);
  int32_t* counts = reinterpret_cast<int32_t*>(ws + L.counts);
  int32_t* mode = counts + 2;
  int32_t* ids = reinterpret_cast<int32_t*>(ws + L.ids);
  const int64_t len = (int64_t)n + 1;
  // Path choice (a device word: the host never waits for the device here).
  hipLaunchKernelGGL(csr_pick, dim3(1), dim3(1024), 0, stream, m, key, mode);
  // Atomic path: degree histogram, scan, per-row cursors, then row ordering.
  hipLaunchKernelGGL(fill_i32, dim3(grid_for(len, 256)), dim3(256), 0, stream, row_ptr, len, 0);
  if (m > 0)
    hipLaunchKernelGGL(csr_hist, dim3(grid_for(m, 256)), dim3(256), 0, stream, mode, n, m, key, other, row_ptr,
                       status);
  const int64_t tiles = (len + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, stream, mode, kBuildAtomic, row_ptr,
                     len, sums);
  hipLaunchKernelGGL(scan_sums, dim3(1), dim3(1024), 0, stream, mode, kBuildAtomic, sums, tiles);
  hipLaunchKernelGGL(scan_add, dim3((unsigned)tiles), dim3(256), 0, stream, mode, kBuildAtomic, row_ptr, len, sums);
  if (m > 0) {
    hipLaunchKernelGGL(copy_i32, dim3(grid_for(n, 256)), dim3(256), 0, stream, mode, cursor, row_ptr, (int64_t)n);
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, stream, counts, (int64_t)2, 0);
    hipLaunchKernelGGL(csr_scatter, dim3(grid_for(m, 256)), dim3(256), 0, stream, mode, n, m, key, other, cursor, col,
                       ids);
    // the cursors are spent: their array holds the lists of longer rows
    hipLaunchKernelGGL(csr_order_rows, dim3(grid_for(n, 256)), dim3(256), 0, stream, mode, n, row_ptr, col, ids,
                       cursor, counts);
    hipLaunchKernelGGL(csr_order_mid, dim3(kOrderMidGrid), dim3(256), 0, stream, mode, row_ptr, col, ids, cursor,
                       counts);
    hipLaunchKernelGGL(csr_order_long, dim3(kOrderLongGrid), dim3(kOrderThreads), 0, stream, mode, n, row_ptr, col,
                       ids, cursor, counts);
  }
  // Radix path (m >= kRadixMinEdges only): passes from the edge list through
  // the two scratch pairs; the last pass writes the columns into col.
  if (m >= kRadixMinEdges) {
    int passes = 0, bits = 0;
    radix_plan(n, &passes, &bits);
    const int64_t rtiles = (m + kRadixTile - 1) / kRadixTile;
    const int64_t hlen = (int64_t)(1 << bits) * rtiles;
    const int64_t htiles = (hlen + kScanTile - 1) / kScanTile;
    int32_t* hist = reinterpret_cast<int32_t*>(ws + L.rhist);
    int32_t* hsums = reinterpret_cast<int32_t*>(ws + L.rsums);
    const int32_t* kin = nullptr;
    const int32_t* vin = nullptr;
    int32_t* ks = nullptr;
    for (int p = 0; p < passes; ++p) {
      const int shift = p * bits;
      int32_t* kout = reinterpret_cast<int32_t*>(ws + L.rk[p & 1]);
      int32_t* vout = p + 1 == passes ? col : reinterpret_cast<int32_t*>(ws + L.rv[p & 1]);
      hipLaunchKernelGGL(radix_count, dim3((unsigned)rtiles), dim3(kRadixThreads), 0, stream, mode, n, m, key, other,
                         kin, shift, bits, rtiles, hist, status);
      hipLaunchKernelGGL(scan_tiles, dim3((unsigned)htiles), dim3(kScanThreads), 0, stream, mode, kBuildRadix, hist,
                         hlen, hsums);
      hipLaunchKernelGGL(scan_sums, dim3(1), dim3(1024), 0, stream, mode, kBuildRadix, hsums, htiles);
      hipLaunchKernelGGL(scan_add, dim3((unsigned)htiles), dim3(256), 0, stream, mode, kBuildRadix, hist, hlen,
                         hsums);
      hipLaunchKernelGGL(radix_scatter, dim3((unsigned)rtiles), dim3(kRadixThreads), 0, stream, mode, n, m, key,
                         other, kin, vin, shift, bits, rtiles, hist, kout, vout);
      kin = kout;
      vin = vout;
      ks = kout;
    }
    hipLaunchKernelGGL(radix_row_ptr, dim3(grid_for(m + 1, 256)), dim3(256), 0, stream, mode, n, m, ks, row_ptr);
  }
  return hipGetLastError() == hipSuccess ? MAP_OK : MAP_EDEVICE;
}

struct BatchLayout {
  size_t header, item_start, scratch_off, gctrl, scratch, total;
};

BatchLayout batch_layout(int32_t count, int64_t total_n) {
  BatchLayout L;
  size_t off = 0;
  L.header = off;
  off += 256;
  L.item_start = off;
  off += align256(((size_t)count + 1) * 4);
  L.scratch_off = off;
  off += align256((size_t)count * 8);
  L.gctrl = off;
  off += (size_t)count * kGangCtrlBytes;
  L.scratch = off;
  // Per graph at most gang_scratch_bytes with MAP_GRAPH_FILTER: 5n + 4 ceil(n / 32)
  // words plus six 256-byte alignments.
  off += (size_t)total_n * 5 + (size_t)(total_n / 2) + (size_t)count * (2 * 256 + 4 * (4 + 256));
  L.total = off;
  return L;
}

int batch_device_info(int* cus, int* per_cu) {
  static std::mutex mu;
  static int cache_cus[64], cache_per[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return MAP_EDEVICE;
  std::lock_guard<std::mutex> lock(mu);
  if (cache_cus[dev] == 0) {
    int c = 0, nb = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return MAP_EDEVICE;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(map_batch_kernel), kBlock,
                                                     0) != hipSuccess)
      return MAP_EDEVICE;
    if (c <= 0 || nb <= 0) return MAP_EDEVICE;
    cache_cus[dev] = c;
    cache_per[dev] = nb;
  }
  *cus = cache_cus[dev];
  *per_cu = cache_per[dev];
  return MAP_OK;
}

int engine_device_info(int* cus, int* per_cu, int* wall_khz) {
  static std::mutex mu;
  static int cache_cus[64], cache_per[64], cache_khz[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return MAP_EDEVICE;
  std::lock_guard<std::mutex> lock(mu);
  if (cache_cus[dev] == 0) {
    int c = 0, nb = 0, khz = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return MAP_EDEVICE;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return MAP_EDEVICE;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(map_engine_kernel), kBlock,
                                                     0) != hipSuccess)
      return MAP_EDEVICE;
    if (c <= 0 || nb <= 0 || khz <= 0) return MAP_EDEVICE;
    cache_cus[dev] = c;
    cache_per[dev] = nb;
    cache_khz[dev] = khz;
  }
  *cus = cache_cus[dev];
  *per_cu = cache_per[dev];
  *wall_khz = cache_khz[dev];
  return MAP_OK;
}

// Grid of a cooperative frontier launch (counterexample search, pruning):
// about one workgroup per 4096 vertices and at most one per CU — a round's
// frontier is usually far smaller than the graph, and fewer workgroups make the
// per-round barrier cheaper.  Limits are cached per device and kernel.
int frontier_grid(const void* kernel, int32_t n, int64_t* grid_out) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, std::pair<int, int>> cache;  // -> (CUs, blocks per CU)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MAP_EDEVICE;
  int cus = 0, per = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({dev, kernel});
    if (it == cache.end()) {
      int co = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return MAP_EDEVICE;
      if (hipDeviceGetAttribute(&co, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess) return MAP_EDEVICE;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0) != hipSuccess) return MAP_EDEVICE;
      if (cus <= 0 || per <= 0 || !co) return MAP_EDEVICE;
      it = cache.emplace(std::make_pair(dev, kernel), std::make_pair(cus, per)).first;
    }
    cus = it->second.first;
    per = it->second.second;
  }
  int64_t grid = ((int64_t)n + 4095) / 4096;
  if (grid > (int64_t)cus * per) grid = (int64_t)cus * per;
  if (grid > cus) grid = cus;
  if (grid > kMaxBlocks) grid = kMaxBlocks;
  if (grid >= kMaxGroups) grid -= grid % kMaxGroups;
  if (grid < 1) grid = 1;
  *grid_out = grid;
  return MAP_OK;
}

constexpr int32_t kEngineRing = 1 << 17;  // ticket ring entries (1 MiB of host memory)

// Fixed device scratch of map_detect_noalloc, for callers that cannot allocate:
// the control block, packed values and working accepting flags of one graph of
// at most MAP_NOALLOC_MAX_N vertices, laid out as in a map_detect workspace.
// Each device that runs the library holds its own copy until the process ends.
constexpr size_t kNoAllocBytes = kCtrlBytes + (size_t)MAP_NOALLOC_MAX_N * 4 + (size_t)MAP_NOALLOC_MAX_N;
static_assert(kCtrlBytes % 256 == 0 && ((size_t)MAP_NOALLOC_MAX_N * 4) % 256 == 0,
              "no-alloc scratch regions are 256-byte aligned");
static __device__ __align__(256) char noalloc_scratch[kNoAllocBytes];

// Device address of noalloc_scratch on each device, taken once per device with
// that device current (the array's name in host code is only a stand-in).
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[64];

int noalloc_scratch_ptr(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return MAP_EDEVICE;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)) != hipSuccess || !p) return MAP_EDEVICE;
    g_noalloc_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_noalloc_ptr[dev]);
  return MAP_OK;
}

}  // namespace

// Host state of a serving engine (one per map_engine_create).
struct map_engine {
  hipStream_t stream;
  hipEvent_t exited;             // recorded after the engine launch
  int grid;                      // workgroups of the launch
  int32_t slots;
  char* host;                    // fine-grained host block: shared line, ring, jobs, results
  EngineShared* sh;
  unsigned long long* ring;
  EngineJob* jobs;
  map_result* res;
  char* dmem;                    // device state
  std::vector<int32_t> free_slots;
  std::vector<unsigned long long> start;  // first ticket of the job in each busy slot
  std::vector<uint8_t> busy;
  unsigned long long tail;       // tickets published
  bool stopped;
};

extern "C" {

size_t map_workspace_bytes(int32_t n, int64_t m, uint32_t flags) {
  (void)flags;
  if (!sizes_ok(n, m)) return 0;
  return layout(n, m).total;
}

int map_build_csr(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, int32_t* row_ptr, int32_t* col,
                  int32_t* rrow_ptr, int32_t* rcol, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  if (!sizes_ok(n, m)) return MAP_ERANGE;
  if (!row_ptr || !status || !ws || (m > 0 && (!src || !dst || !col))) return MAP_EINVAL;
  if ((rrow_ptr == nullptr) != (rcol == nullptr)) return MAP_EINVAL;
  if (rrow_ptr && m > 0 && !rcol) return MAP_EINVAL;
  const Layout L = layout(n, m);
  if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MAP_ENOSPC;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, status, (int64_t)1, (int32_t)MAP_OK);
  int rc = build_one(n, m, src, dst, row_ptr, col, status, static_cast<char*>(ws), L, s);
  if (rc == MAP_OK && rrow_ptr) rc = build_one(n, m, dst, src, rrow_ptr, rcol, status, static_cast<char*>(ws), L, s);
  return rc;
}

// Loop arguments over scratch at w laid out by L (control block, packed values,
// working flags).
static void loop_args(int32_t n, const int32_t* row_ptr, const int32_t* col, const uint8_t* acc, map_result* result,
                      char* w, const Layout& L, LoopArgs& a) {
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.ntiles = (int32_t)(((int64_t)n + kTileRows - 1) / kTileRows);
  a.row_ptr = row_ptr;
  a.col = col;
  a.acc_in = acc;
  a.pv = reinterpret_cast<uint32_t*>(w + L.pv);
  a.accw = reinterpret_cast<uint8_t*>(w + L.accw);
  a.ctrl = reinterpret_cast<Ctrl*>(w + L.ctrl);
  a.result = result;
  word_layout(n, &a.val_mask, &a.tag_mask, &a.tag_shift);
  a.epoch = reinterpret_cast<uint32_t*>(w + L.ctrl + kEpochOff);
  a.chg = reinterpret_cast<uint32_t*>(w + L.chg);
  a.accb = reinterpret_cast<uint32_t*>(w + L.accb);
  a.words = L.words;
  a.hub = kHubEdges;
}

static int loop_common(int32_t n, const int32_t* row_ptr, const int32_t* col, const uint8_t* acc, map_result* result,
                       void* ws, size_t ws_bytes, LoopArgs& a) {
  if (n < 1 || n > 0x7ffffffe) return MAP_ERANGE;
  if (!row_ptr || !col || !acc || !result || !ws) return MAP_EINVAL;
  const Layout L = layout(n);
  if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MAP_ENOSPC;
  loop_args(n, row_ptr, col, acc, result, static_cast<char*>(ws), L, a);
  return MAP_OK;
}

// Frontier sweeps (MAP_FLAG_PUSH, not with MAP_FLAG_DENSE_ONLY) need the
// transposed CSR; they run with a barrier per round and read the values from
// memory (no LDS-resident rows).
static int push_setup(LoopArgs& a, const int32_t* rrow_ptr, const int32_t* rcol, uint32_t flags, void* ws) {
  if (!(flags & MAP_FLAG_PUSH) || (flags & MAP_FLAG_DENSE_ONLY)) return MAP_OK;
  if (!rrow_ptr || !rcol) return MAP_EINVAL;
  const Layout L = layout(a.n);
  char* w = static_cast<char*>(ws);
  a.push = 1;
  a.rrow_ptr = rrow_ptr;
  a.rcol = rcol;
  a.front[0] = reinterpret_cast<int32_t*>(w + L.front0);
  a.front[1] = reinterpret_cast<int32_t*>(w + L.front1);
  a.mark = reinterpret_cast<uint32_t*>(w + L.mark);
  a.force_stream = 1;
  a.sync_sweeps = 1;
  return MAP_OK;
}

// Direction switch of the filtered stream sweeps (MAP_FLAG_DIRECTION, not with
// MAP_FLAG_DENSE_ONLY): needs the transposed CSR; the frontier is the change
// bitmap the sweeps keep anyway.  It takes effect only where the filtered
// stream kernel runs (launch_loop).
static int dir_setup(LoopArgs& a, const int32_t* rrow_ptr, const int32_t* rcol, uint32_t flags) {
  if (!(flags & MAP_FLAG_DIRECTION) || (flags & MAP_FLAG_DENSE_ONLY)) return MAP_OK;
  if (flags & MAP_FLAG_PUSH) return MAP_EINVAL;
  if (!rrow_ptr || !rcol) return MAP_EINVAL;
  a.dopt = 1;
  a.rrow_ptr = rrow_ptr;
  a.rcol = rcol;
  return MAP_OK;
}

int map_propagate(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* rrow_ptr, const int32_t* rcol,
                  const uint8_t* accepting, int32_t* map_out, map_result* result, uint32_t flags, void* ws,
                  size_t ws_bytes, void* stream) {
  if (flags & ~kAllFlags) return MAP_EINVAL;
  if (!map_out) return MAP_EINVAL;
  LoopArgs a;
  int rc = loop_common(n, row_ptr, col, accepting, result, ws, ws_bytes, a);
  if (rc) return rc;
  a.propagate = 1;
  a.force_stream = (flags & MAP_FLAG_STREAM) ? 1 : 0;
  a.sync_sweeps = (flags & MAP_FLAG_SYNC_SWEEPS) ? 1 : 0;
  if (flags & MAP_FLAG_NO_FILTER) a.chg = nullptr;
  a.map_out = map_out;
  rc = push_setup(a, rrow_ptr, rcol, flags, ws);
  if (rc) return rc;
  rc = dir_setup(a, rrow_ptr, rcol, flags);
  if (rc) return rc;
  return launch_loop(a, reinterpret_cast<hipStream_t>(stream));
}

int map_detect(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* rrow_ptr, const int32_t* rcol,
               const uint8_t* accepting0, map_result* result, uint64_t* trace, int32_t trace_cap,
               uint8_t* accepting_out, int32_t max_iterations, uint32_t flags, void* ws, size_t ws_bytes,
               void* stream) {
  if (flags & ~kAllFlags) return MAP_EINVAL;
  if (trace && trace_cap < 0) return MAP_EINVAL;
  LoopArgs a;
  int rc = loop_common(n, row_ptr, col, accepting0, result, ws, ws_bytes, a);
  if (rc) return rc;
  a.propagate = 0;
  a.trace = trace;
  a.trace_cap = trace ? trace_cap : 0;
  a.acc_out = accepting_out;
  a.max_iter = max_iterations;
  a.digest = (trace && !(flags & MAP_FLAG_NO_TRACE_DIGEST)) ? 1 : 0;
  a.force_stream = (flags & MAP_FLAG_STREAM) ? 1 : 0;
  a.sync_sweeps = (flags & MAP_FLAG_SYNC_SWEEPS) ? 1 : 0;
  if (flags & MAP_FLAG_NO_FILTER) a.chg = nullptr;
  rc = push_setup(a, rrow_ptr, rcol, flags, ws);
  if (rc) return rc;
  rc = dir_setup(a, rrow_ptr, rcol, flags);
  if (rc) return rc;
  if (flags & MAP_FLAG_EARLY) {
    if (a.push) return MAP_EINVAL;
    a.early = 1;
  }
  return launch_loop(a, reinterpret_cast<hipStream_t>(stream));
}

int map_detect_noalloc(int32_t n, const int32_t* row_ptr, const int32_t* col, const uint8_t* accepting0,
                       map_result* result, uint64_t* trace, int32_t trace_cap, uint8_t* accepting_out,
                       int32_t max_iterations, uint32_t flags, void* stream) {
  if (flags & ~kAllFlags) return MAP_EINVAL;
  if ((flags & (MAP_FLAG_PUSH | MAP_FLAG_DIRECTION)) && !(flags & MAP_FLAG_DENSE_ONLY)) return MAP_EINVAL;
  if (trace && trace_cap < 0) return MAP_EINVAL;
  if (n < 1 || n > MAP_NOALLOC_MAX_N) return MAP_ERANGE;
  if (!row_ptr || !col || !accepting0 || !result) return MAP_EINVAL;
  const Layout L = layout(n);
  // Only the control block, packed values and working flags are used.
  if (L.accw + (size_t)n > kNoAllocBytes) return MAP_ERANGE;
  char* w = nullptr;
  int rc = noalloc_scratch_ptr(&w);
  if (rc) return rc;
  LoopArgs a;
  loop_args(n, row_ptr, col, accepting0, result, w, L, a);
  a.chg = nullptr;  // the fixed scratch holds no change bitmaps: unfiltered sweeps
  a.accb = nullptr;
  a.propagate = 0;
  a.trace = trace;
  a.trace_cap = trace ? trace_cap : 0;
  a.acc_out = accepting_out;
  a.max_iter = max_iterations;
  a.digest = (trace && !(flags & MAP_FLAG_NO_TRACE_DIGEST)) ? 1 : 0;
  a.force_stream = (flags & MAP_FLAG_STREAM) ? 1 : 0;
  a.sync_sweeps = (flags & MAP_FLAG_SYNC_SWEEPS) ? 1 : 0;
  a.early = (flags & MAP_FLAG_EARLY) ? 1 : 0;
  return launch_loop(a, reinterpret_cast<hipStream_t>(stream));
}

int map_lasso(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t witness, int32_t init, int32_t* path,
              int32_t path_cap, map_lasso_result* result, void* ws, size_t ws_bytes, void* stream) {
  if (n < 1 || n > 0x7ffffffe) return MAP_ERANGE;
  if (!row_ptr || !col || !result || !ws || path_cap < 0 || (path_cap > 0 && !path)) return MAP_EINVAL;
  if (witness < 1 || witness > n || init < 0 || init > n) return MAP_EINVAL;
  const Layout L = layout(n);
  if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MAP_ENOSPC;
  int64_t grid = 0;
  int rc = frontier_grid(reinterpret_cast<const void*>(map_lasso_kernel), n, &grid);
  if (rc) return rc;
  char* w = static_cast<char*>(ws);
  LassoArgs a;
  a.n = n;
  a.row_ptr = row_ptr;
  a.col = col;
  a.w = witness - 1;
  a.init = init - 1;
  a.path = path;
  a.cap = path_cap;
  a.result = result;
  a.parent = reinterpret_cast<uint64_t*>(w + L.parent);
  a.front[0] = reinterpret_cast<int32_t*>(w + L.front0);
  a.front[1] = reinterpret_cast<int32_t*>(w + L.front1);
  a.ctrl = reinterpret_cast<Ctrl*>(w + L.ctrl);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(fill_u32, dim3(8), dim3(256), 0, st, reinterpret_cast<uint32_t*>(a.ctrl),
                     (int64_t)(kEpochOff / 4), 0u);
  if (hipGetLastError() != hipSuccess) return MAP_EDEVICE;
  void* args[] = {&a};
  if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(map_lasso_kernel), dim3((unsigned)grid), dim3(kBlock),
                                 args, 0, st) != hipSuccess)
    return MAP_EDEVICE;
  return MAP_OK;
}

int map_trim(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* rrow_ptr, const int32_t* rcol,
             const uint8_t* accepting, uint8_t* keep_out, uint8_t* accepting_out, map_trim_result* result, void* ws,
             size_t ws_bytes, void* stream) {
  if (n < 1 || n > 0x7ffffffe) return MAP_ERANGE;
  if (!row_ptr || !col || !rrow_ptr || !rcol || !keep_out || !result || !ws) return MAP_EINVAL;
  if ((accepting == nullptr) != (accepting_out == nullptr)) return MAP_EINVAL;
  const Layout L = layout(n);
  if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MAP_ENOSPC;
  int64_t grid = 0;
  int rc = frontier_grid(reinterpret_cast<const void*>(map_trim_kernel), n, &grid);
  if (rc) return rc;
  char* w = static_cast<char*>(ws);
  TrimArgs a;
  a.n = n;
  a.row_ptr = row_ptr;
  a.col = col;
  a.rrow_ptr = rrow_ptr;
  a.rcol = rcol;
  a.acc_in = accepting;
  a.keep_out = keep_out;
  a.acc_out = accepting_out;
  a.result = result;
  a.indeg = reinterpret_cast<uint32_t*>(w + L.pv);
  a.outdeg = reinterpret_cast<uint32_t*>(w + L.mark);
  a.removed = reinterpret_cast<uint32_t*>(w + L.aux);
  a.front[0] = reinterpret_cast<int32_t*>(w + L.front0);
  a.front[1] = reinterpret_cast<int32_t*>(w + L.front1);
  a.ctrl = reinterpret_cast<Ctrl*>(w + L.ctrl);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(fill_u32, dim3(8), dim3(256), 0, st, reinterpret_cast<uint32_t*>(a.ctrl),
                     (int64_t)(kEpochOff / 4), 0u);
  if (hipGetLastError() != hipSuccess) return MAP_EDEVICE;
  void* args[] = {&a};
  if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(map_trim_kernel), dim3((unsigned)grid), dim3(kBlock),
                                 args, 0, st) != hipSuccess)
    return MAP_EDEVICE;
  return MAP_OK;
}

size_t map_batch_workspace_bytes(int32_t count, int64_t total_n, uint32_t flags) {
  (void)flags;
  if (count < 1 || count > (1 << 24) || total_n < count || total_n > ((int64_t)1 << 40)) return 0;
  return batch_layout(count, total_n).total;
}

int map_detect_batch(int32_t count, const map_graph_desc* graphs, const int32_t* gang, map_result* results,
                     int64_t total_n, uint32_t flags, void* ws, size_t ws_bytes, void* stream) {
  if (count < 1 || count > (1 << 24) || total_n < count || total_n > ((int64_t)1 << 40)) return MAP_ERANGE;
  if (!graphs || !results || !ws) return MAP_EINVAL;
  if (flags & ~kAllFlags) return MAP_EINVAL;
  const BatchLayout L = batch_layout(count, total_n);
  if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MAP_ENOSPC;
  int cus = 0, per_cu = 0;
  int rc = batch_device_info(&cus, &per_cu);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  BatchArgs ba;
  ba.count = count;
  ba.graphs = graphs;
  ba.results = results;
  ba.item_start = reinterpret_cast<int32_t*>(w + L.item_start);
  ba.scratch_off = reinterpret_cast<int64_t*>(w + L.scratch_off);
  ba.gctrl = reinterpret_cast<GangCtrl*>(w + L.gctrl);
  ba.scratch = w + L.scratch;
  ba.next_item = reinterpret_cast<uint32_t*>(w + L.header);
  ba.status = reinterpret_cast<int32_t*>(w + L.header + 128);
  ba.flags = flags;
  const int64_t ctrl_words = (int64_t)((size_t)count * kGangCtrlBytes / 4);
  hipLaunchKernelGGL(fill_u32, dim3(grid_for(ctrl_words, 256)), dim3(256), 0, st,
                     reinterpret_cast<uint32_t*>(ba.gctrl), ctrl_words, 0u);
  // A gang must fit in the grid at once: its blocks wait for each other.
  const int grid = cus * per_cu;
  hipLaunchKernelGGL(batch_plan, dim3(1), dim3(1024), 0, st, count, graphs, gang,
                     const_cast<int32_t*>(ba.item_start), const_cast<int64_t*>(ba.scratch_off),
                     (size_t)(L.total - L.scratch), (int32_t)std::min(kMaxGang, grid), ba.status, ba.next_item);
  if (hipGetLastError() != hipSuccess) return MAP_EDEVICE;
  if (gang == nullptr) {
    hipLaunchKernelGGL(map_batch_kernel, dim3(grid), dim3(kBlock), 0, st, ba);
    if (hipGetLastError() != hipSuccess) return MAP_EDEVICE;
  } else {
    void* args[] = {&ba};
    if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(map_batch_kernel), dim3(grid), dim3(kBlock), args,
                                   0, st) != hipSuccess)
      return MAP_EDEVICE;
  }
  return MAP_OK;
}

size_t map_job_scratch_bytes(int32_t n, int64_t m) {
  if (!sizes_ok(n, m)) return 0;
  // packed values | working flags | bitmaps of the filtered sweeps | scan
  // partials | staged edge list (src, dst) | transposed CSR (the last three
  // parts used with MAP_FLAG_DIRECTION only)
  return align256((size_t)n * 4) + align256((size_t)n) + 4 * (size_t)gang_bitmap_bytes(n) + (size_t)kMaxGang * 4 +
         2 * align256((size_t)m * 4) + align256((size_t)n * 4 + 4) + align256((size_t)m * 4);
}

static void engine_free(map_engine* e) {
  if (e->dmem) (void)hipFree(e->dmem);
  if (e->host) (void)hipHostFree(e->host);
  if (e->exited) (void)hipEventDestroy(e->exited);
  delete e;
}

int map_engine_create(int32_t max_jobs, int32_t workgroups, double idle_seconds, uint32_t flags, void* stream,
                      map_engine** out) {
  if (!out) return MAP_EINVAL;
  *out = nullptr;
  if (flags & ~kAllFlags) return MAP_EINVAL;
  if (max_jobs < 1 || max_jobs > (1 << 16) || workgroups < 0 || !(idle_seconds > 0.0) || idle_seconds > 86400.0)
    return MAP_ERANGE;
  int cus = 0, per_cu = 0, khz = 0;
  int rc = engine_device_info(&cus, &per_cu, &khz);
  if (rc) return rc;
  const int full = cus * per_cu;
  // By default one compute unit per 32 is left to other work (copy kernels of
  // the runtime, the caller's own launches) while the engine runs.
  const int grid = workgroups > 0 ? std::min(workgroups, full) : std::max(1, full - cus / 32);
  map_engine* e = new map_engine();
  e->stream = reinterpret_cast<hipStream_t>(stream);
  e->grid = grid;
  e->slots = max_jobs;
  const size_t off_ring = sizeof(EngineShared);
  const size_t off_jobs = off_ring + (size_t)kEngineRing * 8;
  const size_t off_res = off_jobs + align256((size_t)max_jobs * sizeof(EngineJob));
  const size_t host_bytes = off_res + (size_t)max_jobs * sizeof(map_result);
  void* h = nullptr;
  if (hipHostMalloc(&h, host_bytes, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess || !h) {
    delete e;
    return MAP_EDEVICE;
  }
  e->host = static_cast<char*>(h);
  std::memset(e->host, 0, host_bytes);
  e->sh = reinterpret_cast<EngineShared*>(e->host);
  e->ring = reinterpret_cast<unsigned long long*>(e->host + off_ring);
  e->jobs = reinterpret_cast<EngineJob*>(e->host + off_jobs);
  e->res = reinterpret_cast<map_result*>(e->host + off_res);
  void* hd = nullptr;
  if (hipHostGetDevicePointer(&hd, h, 0) != hipSuccess || !hd) {
    engine_free(e);
    return MAP_EDEVICE;
  }
  char* hdev = static_cast<char*>(hd);
  const size_t off_b = align256(sizeof(EngineDev));
  const size_t off_m = off_b + (size_t)max_jobs * kGangCtrlBytes;
  const size_t off_d = off_m + (size_t)max_jobs * kGangCtrlBytes;
  const size_t off_r = off_d + align256((size_t)max_jobs * sizeof(map_result));
  const size_t dev_bytes = off_r + align256((size_t)max_jobs * 8);
  void* dm = nullptr;
  if (hipMalloc(&dm, dev_bytes) != hipSuccess || !dm) {
    engine_free(e);
    return MAP_EDEVICE;
  }
  e->dmem = static_cast<char*>(dm);
  if (hipEventCreateWithFlags(&e->exited, hipEventDisableTiming) != hipSuccess) {
    e->exited = nullptr;
    engine_free(e);
    return MAP_EDEVICE;
  }
  e->free_slots.reserve(max_jobs);
  for (int32_t i = max_jobs - 1; i >= 0; --i) e->free_slots.push_back(i);
  e->start.assign(max_jobs, 0ull);
  e->busy.assign(max_jobs, 0);
  e->tail = 0;
  e->stopped = false;

  EngineArgs ea;
  ea.sh = reinterpret_cast<EngineShared*>(hdev);
  ea.ring = reinterpret_cast<const unsigned long long*>(hdev + off_ring);
  ea.jobs = reinterpret_cast<const EngineJob*>(hdev + off_jobs);
  ea.hres = reinterpret_cast<map_result*>(hdev + off_res);
  ea.dev = reinterpret_cast<EngineDev*>(e->dmem);
  ea.bctrl = reinterpret_cast<GangCtrl*>(e->dmem + off_b);
  ea.mctrl = reinterpret_cast<GangCtrl*>(e->dmem + off_m);
  ea.dres = reinterpret_cast<map_result*>(e->dmem + off_d);
  ea.ready = reinterpret_cast<unsigned long long*>(e->dmem + off_r);
  ea.ring_cap = kEngineRing;
  ea.slots = max_jobs;
  ea.idle_ticks = (uint64_t)(idle_seconds * (double)khz * 1000.0);
  ea.flags = flags;
  hipLaunchKernelGGL(fill_u32, dim3(grid_for((int64_t)(dev_bytes / 4), 256)), dim3(256), 0, e->stream,
                     reinterpret_cast<uint32_t*>(e->dmem), (int64_t)(dev_bytes / 4), 0u);
  void* args[] = {&ea};
  if (hipGetLastError() != hipSuccess ||
      hipLaunchCooperativeKernel(reinterpret_cast<const void*>(map_engine_kernel), dim3(grid), dim3(kBlock), args, 0,
                                 e->stream) != hipSuccess ||
      hipEventRecord(e->exited, e->stream) != hipSuccess) {
    // Nothing was launched, or the launch failed: no kernel can be using the memory.
    (void)hipStreamSynchronize(e->stream);
    engine_free(e);
    return MAP_EDEVICE;
  }
  *out = e;
  return MAP_OK;
}

int map_engine_workgroups(const map_engine* e) { return e ? e->grid : 0; }

// Device address through which the engine reads a job input: device memory
// as is, pinned host memory through its device mapping; anything else (pageable
// host memory, unknown pointers) is rejected so the kernel never touches it.
static int engine_input(const void* p, const void** out, bool* host = nullptr) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return MAP_EINVAL;
  }
  if (at.type == hipMemoryTypeDevice) {
    *out = p;
    return MAP_OK;
  }
  if (at.type == hipMemoryTypeHost) {
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, const_cast<void*>(p), 0) != hipSuccess || !d) {
      (void)hipGetLastError();
      return MAP_EINVAL;
    }
    *out = d;
    if (host) *host = true;
    return MAP_OK;
  }
  return MAP_EINVAL;
}

static bool engine_output(const void* p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice;
}

int map_engine_submit(map_engine* e, const map_job* job, int32_t* slot) {
  if (!e || !job || !slot) return MAP_EINVAL;
  if (e->stopped) return MAP_EINVAL;
  if (__atomic_load_n(&e->sh->expired, __ATOMIC_ACQUIRE)) return MAP_EDEVICE;
  if (!sizes_ok(job->n, job->m)) return MAP_ERANGE;
  if (!job->row_ptr || !job->accepting0 || !job->scratch) return MAP_EINVAL;
  if (job->m > 0 && (!job->src || !job->dst || !job->col)) return MAP_EINVAL;
  if (reinterpret_cast<uintptr_t>(job->scratch) & 255) return MAP_EINVAL;
  EngineJob ej;
  std::memset(&ej, 0, sizeof(ej));
  map_job& jj = ej.j;
  jj = *job;
  bool host_src = false, host_dst = false;
  if (engine_input(job->accepting0, reinterpret_cast<const void**>(&jj.accepting0)) ||
      !engine_output(job->row_ptr) || !engine_output(job->scratch))
    return MAP_EINVAL;
  if (job->m > 0 && (engine_input(job->src, reinterpret_cast<const void**>(&jj.src), &host_src) ||
                     engine_input(job->dst, reinterpret_cast<const void**>(&jj.dst), &host_dst) ||
                     !engine_output(job->col)))
    return MAP_EINVAL;
  ej.host_edges = (host_src || host_dst) ? 1u : 0u;
  const int32_t gang = std::max(1, std::min(job->gang, std::min(kMaxGang, e->grid)));
  if (e->free_slots.empty()) return MAP_EBUSY;
  // The new tickets reuse ring entries of tickets [tail + gang - ring, ...),
  // which must all have been taken: every ticket below the first one of the
  // oldest unfinished job has been.
  unsigned long long oldest = e->tail;
  for (int32_t i = 0; i < e->slots; ++i)
    if (e->busy[i] && e->start[i] < oldest) oldest = e->start[i];
  if (e->tail + (unsigned long long)gang > oldest + (unsigned long long)kEngineRing) return MAP_EBUSY;
  const int32_t s = e->free_slots.back();
  e->free_slots.pop_back();
  jj.gang = gang;
  e->jobs[s] = ej;
  map_result r0;
  std::memset(&r0, 0, sizeof(r0));
  r0.status = MAP_PENDING;
  e->res[s] = r0;
  for (int32_t r = 0; r < gang; ++r)
    e->ring[(e->tail + (unsigned long long)r) % kEngineRing] = ((unsigned long long)s << 32) | (unsigned)r;
  e->start[s] = e->tail;
  e->busy[s] = 1;
  e->tail += (unsigned long long)gang;
  __atomic_store_n(&e->sh->tail, e->tail, __ATOMIC_RELEASE);
  *slot = s;
  return MAP_OK;
}

int map_engine_poll(map_engine* e, int32_t slot, map_result* out) {
  if (!e || slot < 0 || slot >= e->slots || !e->busy[slot]) return MAP_EINVAL;
  const int32_t st = __atomic_load_n(&e->res[slot].status, __ATOMIC_ACQUIRE);
  if (st == MAP_PENDING) {
    // A job still pending after the engine exited (idle bound) never completes.
    if (hipEventQuery(e->exited) != hipSuccess) return MAP_PENDING;
    if (__atomic_load_n(&e->res[slot].status, __ATOMIC_ACQUIRE) == MAP_PENDING) {
      e->busy[slot] = 0;
      e->free_slots.push_back(slot);
      return MAP_EDEVICE;
    }
  }
  if (out) std::memcpy(out, &e->res[slot], sizeof(map_result));
  e->busy[slot] = 0;
  e->free_slots.push_back(slot);
  return MAP_OK;
}

int map_engine_stop(map_engine* e) {
  if (!e) return MAP_EINVAL;
  __atomic_store_n(&e->sh->stop, 1u, __ATOMIC_RELEASE);
  e->stopped = true;
  return MAP_OK;
}

int map_engine_destroy(map_engine* e) {
  if (!e) return MAP_EINVAL;
  map_engine_stop(e);
  const int rc = hipEventSynchronize(e->exited) == hipSuccess ? MAP_OK : MAP_EDEVICE;
  engine_free(e);
  return rc;
}

int map_phase_counters(uint64_t* out, int32_t max_blocks, int32_t* blocks) {
#ifdef MAPCHECK_PHASES
  if (!out || !blocks || max_blocks < 0) return MAP_EINVAL;
  const int nb = g_last_grid.load();
  *blocks = nb;
  const int k = nb < max_blocks ? nb : max_blocks;
  if (k > 0 && hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase_out), (size_t)k * kPhSlots * sizeof(uint64_t), 0,
                                   hipMemcpyDeviceToHost) != hipSuccess)
    return MAP_EDEVICE;
  return MAP_OK;
#else
  (void)out;
  (void)max_blocks;
  (void)blocks;
  return MAP_EINVAL;
#endif
}

const char* map_strerror(int status) {
  switch (status) {
    case MAP_OK: return "ok";
    case MAP_EINVAL: return "invalid argument (null pointer or unknown flag)";
    case MAP_ERANGE: return "n or m out of the supported range";
    case MAP_ENOSPC: return "workspace too small or not 256-byte aligned";
    case MAP_EDEVICE: return "HIP runtime error or device-side barrier timeout";
    case MAP_ENOTCONVERGED: return "iteration or sweep cap reached";
    case MAP_ERANGE_DEV: return "edge endpoint outside 1..n";
    case MAP_EBUSY: return "engine has no free job slot or ticket space; poll finished jobs first";
    case MAP_ENOPATH: return "no path from the initial vertex to the witness, or no cycle through the witness";
    case MAP_PENDING: return "job not finished yet";
    default: return "unknown status";
  }
}

}  // extern "C"
