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
//   ctrl   control block: grid-barrier counters and per-epoch reduction slots;
//   pv     uint32[n]: bit 31 = vertex is accepting in the current iteration,
//          bits 0..30 = current map value (id, 0 = none);
//   accw   uint8[n]: working accepting flags, stripped between iterations.
//
// One cooperative persistent kernel runs the whole outer loop (reset, sweeps
// to the fixpoint, detect, strip, next iteration) with grid barriers between
// phases; the host enqueues one launch per call and never synchronizes.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "mapcheck.h"

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 512;  // threads per workgroup of the loop kernel
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kTileRows = 128;    // rows per wave tile
constexpr int kTileEdges = 1024;  // edges staged in LDS per wave (4 KiB)
constexpr int kRowsPerLane = kTileRows / kWave;
constexpr int kEdgesPerLane = kTileEdges / kWave;
constexpr uint32_t kAccBit = 0x80000000u;
constexpr uint32_t kValMask = 0x7fffffffu;
constexpr int kStripes = 16;
constexpr int kSets = 3;
constexpr int kMaxGroups = 8;  // barrier arrival groups (one per XCD)
// Bound on one barrier wait, in ticks of the 100 MHz device wall clock (10 s):
// far beyond any legitimate phase, so a broken launch exits instead of hanging.
constexpr uint64_t kWaitTicks = 1000000000ull;

// ------------------------------------------------------------------ ctrl --

struct alignas(128) Stripe {
  unsigned long long digest;
  uint32_t count;
  int32_t witness;
  uint32_t nonzero;
  uint32_t pad[27];
};

struct alignas(128) Line64 {
  unsigned long long v;
  unsigned long long pad[15];
};

struct Ctrl {
  Line64 grp[kMaxGroups];  // barrier arrivals per group: high 32 = arrivals, low 32 = payload sum
  Line64 top;              // arrivals of the group leaders
  alignas(128) uint32_t gen;       // barrier generation
  uint32_t payload;                // payload sum of the last completed barrier
  int32_t abort;                   // set when a barrier wait exceeded its bound
  uint32_t pad0[29];
  Stripe sets[kSets][kStripes];    // per-epoch reductions
};
static_assert(sizeof(Ctrl) <= 16384, "ctrl block too large");
constexpr size_t kCtrlBytes = 16384;

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

struct Grid {
  Ctrl* c;
  uint32_t gen;      // generation this block expects to complete next
  int nblocks;
  int group;         // arrival group of this block
  int group_size;    // blocks in this group
  int ngroups;
};

// Grid-wide barrier with a summed 32-bit payload.  Every thread must call it.
// Returns false if the wait exceeded its bound (the kernel must then exit).
//
// Ordering: each block's leader issues one agent-scope release fence before
// its arrival (cumulative over the block's waves through the workgroup
// barrier); the last arrival of a group and the last group leader acquire
// before forwarding; waiters poll with relaxed loads (no cache invalidation
// per poll) and acquire once when the generation moves.
__device__ bool grid_sync(Grid& g, uint32_t payload, uint32_t* total) {
  __shared__ uint32_t s_total;
  __shared__ int s_ok;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  if (threadIdx.x == 0) {
    Ctrl* c = g.c;
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
    s_total = ok ? ld_agent(&c->payload) : 0u;
    s_ok = ok;
  }
  __syncthreads();
  // Epoch E+1 writes set (E+1)%3 and reads set E%3; set (E-1)%3 was last read
  // during epoch E, so block 0 clears it now for epoch E+2.
  if (blockIdx.x == 0 && threadIdx.x < kStripes) {
    Stripe& s = g.c->sets[(g.gen + 2) % kSets][threadIdx.x];
    __hip_atomic_store(&s.digest, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
};

struct TileLds {
  int32_t rp[kTileRows + 1];
  uint32_t val[kTileEdges];
};

// Value that successor w (0-based) sends along an edge: its map value, or its
// own id if it is accepting and larger.
__device__ __forceinline__ uint32_t sent_packed(uint32_t x, int32_t w) {
  uint32_t m = x & kValMask;
  uint32_t id = (uint32_t)w + 1u;
  return (x & kAccBit) ? (m > id ? m : id) : m;
}

// One tile of a sweep, processed by one wave.  first != 0: the sweep that
// starts an iteration from map = 0; successors send their id if accepting
// (read from acc) and every row's packed value is written.  Otherwise rows
// pull the packed values of their successors and a row is written only when
// its value grows.  Returns nonzero (wave-uniform) if some row changed.
template <bool kFirst>
__device__ uint32_t sweep_tile(const LoopArgs& a, const uint8_t* acc, int tile, TileLds& L, int lane,
                               uint32_t* acc_count) {
  const int64_t r0 = (int64_t)tile * kTileRows;
  const int64_t r1 = min((int64_t)a.n, r0 + kTileRows);
  const int nr = (int)(r1 - r0);
  for (int i = lane; i <= nr; i += kWave) L.rp[i] = __builtin_nontemporal_load(a.row_ptr + r0 + i);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int32_t e0 = L.rp[0], e1 = L.rp[nr];
  int32_t lo[kRowsPerLane], hi[kRowsPerLane];
  uint32_t best[kRowsPerLane];
#pragma unroll
  for (int j = 0; j < kRowsPerLane; ++j) {
    int r = lane + j * kWave;
    lo[j] = r < nr ? L.rp[r] : 0;
    hi[j] = r < nr ? L.rp[r + 1] : 0;
    best[j] = 0;
  }
  for (int32_t c0 = e0; c0 < e1; c0 += kTileEdges) {
    const int cnt = (int)min((int64_t)kTileEdges, (int64_t)e1 - c0);
    int32_t w[kEdgesPerLane];
#pragma unroll
    for (int u = 0; u < kEdgesPerLane; ++u) {
      int i = lane + u * kWave;
      w[u] = i < cnt ? __builtin_nontemporal_load(a.col + c0 + i) : -1;
    }
#pragma unroll
    for (int u = 0; u < kEdgesPerLane; ++u) {
      int i = lane + u * kWave;
      uint32_t s = 0;
      if ((uint32_t)w[u] < (uint32_t)a.n) {
        if (kFirst) s = acc[w[u]] ? (uint32_t)w[u] + 1u : 0u;
        else s = sent_packed(a.pv[w[u]], w[u]);
      }
      if (i < cnt) L.val[i] = s;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int j = 0; j < kRowsPerLane; ++j) {
      int b = max(lo[j] - c0, 0), e = min(hi[j] - c0, cnt);
      uint32_t m = best[j];
      for (int k = b; k < e; ++k) m = max(m, L.val[k]);
      best[j] = m;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  uint32_t changed = 0, nacc = 0;
#pragma unroll
  for (int j = 0; j < kRowsPerLane; ++j) {
    int r = lane + j * kWave;
    if (r < nr) {
      int64_t v = r0 + r;
      if (kFirst) {
        uint32_t isacc = acc[v] ? 1u : 0u;
        nacc += isacc;
        a.pv[v] = (isacc << 31) | best[j];
        changed |= best[j] != 0;
      } else {
        uint32_t old = a.pv[v];
        if (best[j] > (old & kValMask)) {
          a.pv[v] = (old & kAccBit) | best[j];
          changed = 1;
        }
      }
    }
  }
  if (acc_count) *acc_count += nacc;
  return __ballot(changed) != 0;
}

__global__ void __launch_bounds__(kBlock) map_loop_kernel(LoopArgs a) {
  __shared__ TileLds lds[kWavesPerBlock];
  __shared__ uint32_t s_red[kWavesPerBlock];
  __shared__ unsigned long long s_red64[kWavesPerBlock];
  __shared__ int32_t s_wit[kWavesPerBlock];

  const int lane = threadIdx.x & (kWave - 1);
  const int wib = threadIdx.x / kWave;
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  // XCD-aware numbering: consecutive hardware block ids land on different
  // XCDs; give each XCD a contiguous range of logical blocks (and rows).
  const int logical = (nb % kMaxGroups == 0) ? (b % kMaxGroups) * (nb / kMaxGroups) + b / kMaxGroups : b;
  const int nwaves = nb * kWavesPerBlock;
  const int gw = logical * kWavesPerBlock + wib;
  const int per = (a.ntiles + nwaves - 1) / nwaves;
  const int t_begin = min(a.ntiles, gw * per);
  const int t_end = min(a.ntiles, t_begin + per);
  TileLds& L = lds[wib];

  Grid g;
  g.c = a.ctrl;
  g.gen = 0;
  g.nblocks = nb;
  g.ngroups = min(nb, kMaxGroups);
  g.group = b % g.ngroups;
  g.group_size = nb / g.ngroups + ((b % g.ngroups) < (nb % g.ngroups) ? 1 : 0);

  Ctrl* c = a.ctrl;
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
    uint32_t t = 0;
    for (int i = 0; i < kStripes; ++i) t += ld_agent(&c->sets[set][i].count);
    return t;
  };

  uint32_t count_prev = 0;  // |A_k| of the current iteration
  int32_t k = 0;
  int64_t total_sweeps = 0;
  int32_t status = MAP_OK, found = 0, witness = 0;
  int32_t left = 0;
  bool acc_from_pv = false;  // acc_out comes from the accepting bits of pv
  bool ok = true;
  uint32_t tot = 0;

  if (!a.propagate) {
    // A_1 -> working flags; count |A_1|.
    uint32_t cnt = 0;
    for (int t = t_begin; t < t_end; ++t) {
      int64_t r0 = (int64_t)t * kTileRows, r1 = min((int64_t)a.n, r0 + kTileRows);
      for (int64_t v = r0 + lane; v < r1; v += kWave) {
        uint8_t x = a.acc_in[v] ? 1 : 0;
        a.accw[v] = x;
        cnt += x;
      }
    }
    block_add_count(cnt, g.gen % kSets);
    ok = grid_sync(g, 0, nullptr);
    if (!ok) goto aborted;
    count_prev = read_count((g.gen - 1) % kSets);
    if (count_prev == 0) { left = 0; goto done; }
  }

  for (;;) {
    // First sweep of an iteration: map from 0, accepting flags from acc.
    uint32_t nacc = 0, ch = 0;
    for (int t = t_end - 1; t >= t_begin; --t) ch |= sweep_tile<true>(a, acc, t, L, lane, &nacc);
    if (!a.propagate) block_add_count(nacc, g.gen % kSets);
    if (lane == 0) s_red[wib] = ch;
    __syncthreads();
    uint32_t bch = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) bch |= s_red[i];
    ok = grid_sync(g, bch ? 1u : 0u, &tot);
    if (!ok) goto aborted;
    if (!a.propagate) {
      uint32_t cnt = read_count((g.gen - 1) % kSets);
      if (k > 0) {
        // Iteration k is complete: |Del_k| = |A_k| - |A_{k+1}|.
        if (b == 0 && threadIdx.x == 0 && a.trace && k <= a.trace_cap)
          a.trace[(int64_t)(k - 1) * 3 + 0] = (uint64_t)(count_prev - cnt);
        if (cnt == 0 || cnt == count_prev) { left = (int32_t)cnt; break; }  // no accepting left / none removed
        if (a.max_iter > 0 && k >= a.max_iter) { status = MAP_ENOTCONVERGED; left = (int32_t)cnt; break; }
      }
      count_prev = cnt;
    }
    k++;
    int64_t s = 1;
    while (tot != 0) {
      if (s > (int64_t)a.n + 1) { status = MAP_ENOTCONVERGED; break; }
      uint32_t c2 = 0;
      for (int t = t_end - 1; t >= t_begin; --t) c2 |= sweep_tile<false>(a, acc, t, L, lane, nullptr);
      if (lane == 0) s_red[wib] = c2;
      __syncthreads();
      bch = 0;
      for (int i = 0; i < kWavesPerBlock; ++i) bch |= s_red[i];
      s++;
      ok = grid_sync(g, bch ? 1u : 0u, &tot);
      if (!ok) goto aborted;
    }
    total_sweeps += s;
    if (status != MAP_OK) { left = (int32_t)count_prev; acc_from_pv = !a.propagate; break; }
    if (a.propagate) break;

    // Detect and strip: witness = max v with map(v) == v; every nonzero map
    // value loses its accepting flag (the flags of this iteration stay in pv).
    {
      int32_t wit = 0;
      unsigned long long dig = 0;
        for (int t = t_begin; t < t_end; ++t) {
        int64_t r0 = (int64_t)t * kTileRows, r1 = min((int64_t)a.n, r0 + kTileRows);
        for (int64_t v = r0 + lane; v < r1; v += kWave) {
          uint32_t mv = a.pv[v] & kValMask;
          uint32_t id = (uint32_t)v + 1u;
          if (mv == id) wit = max(wit, (int32_t)id);
          if (a.digest) dig += mix64(((unsigned long long)id << 32) | mv);
          if (mv != 0) {
            // Many vertices share a map value: read before writing.
            if (acc[mv - 1]) acc[mv - 1] = 0;
          }
        }
      }
      wit = wave_max_i32(wit);
      if (a.digest) dig = wave_sum_u64(dig);
      if (lane == 0) { s_wit[wib] = wit; s_red64[wib] = dig; }
      __syncthreads();
      if (threadIdx.x == 0) {
        int32_t bw = 0;
        unsigned long long bd = 0;
        for (int i = 0; i < kWavesPerBlock; ++i) { bw = max(bw, s_wit[i]); bd += s_red64[i]; }
        Stripe& st = c->sets[g.gen % kSets][b % kStripes];
        if (bw) __hip_atomic_fetch_max(&st.witness, bw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (bd) __hip_atomic_fetch_add(&st.digest, bd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      ok = grid_sync(g, 0, nullptr);
      if (!ok) goto aborted;
      int set = (g.gen - 1) % kSets;
      int32_t w2 = 0;
      unsigned long long d2 = 0;
      for (int i = 0; i < kStripes; ++i) {
        w2 = max(w2, __hip_atomic_load(&c->sets[set][i].witness, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        d2 += __hip_atomic_load(&c->sets[set][i].digest, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (b == 0 && threadIdx.x == 0 && a.trace && k <= a.trace_cap) {
        uint64_t* row = a.trace + (int64_t)(k - 1) * 3;
        row[0] = 0;
        row[1] = (uint64_t)s;
        row[2] = a.digest ? d2 : 0ull;
      }
      if (w2 > 0) {
        found = 1;
        witness = w2;
        left = (int32_t)count_prev;
        acc_from_pv = true;
        break;
      }
    }
  }

done:
  // Outputs: map vector (propagate) or the accepting set at exit (detect).
  if (a.propagate && a.map_out) {
    for (int t = t_begin; t < t_end; ++t) {
      int64_t r0 = (int64_t)t * kTileRows, r1 = min((int64_t)a.n, r0 + kTileRows);
      for (int64_t v = r0 + lane; v < r1; v += kWave) a.map_out[v] = (int32_t)(a.pv[v] & kValMask);
    }
  }
  if (!a.propagate && a.acc_out) {
    for (int t = t_begin; t < t_end; ++t) {
      int64_t r0 = (int64_t)t * kTileRows, r1 = min((int64_t)a.n, r0 + kTileRows);
      for (int64_t v = r0 + lane; v < r1; v += kWave)
        a.acc_out[v] = acc_from_pv ? (uint8_t)(a.pv[v] >> 31) : a.accw[v];
    }
  }
  if (b == 0 && threadIdx.x == 0) {
    a.result->found = found;
    a.result->witness = witness;
    a.result->iterations = a.propagate ? 0 : k;
    a.result->status = status;
    a.result->sweeps = total_sweeps;
    a.result->accepting_left = a.propagate ? 0 : left;
    a.result->reserved = 0;
  }
  return;

aborted:
  if (threadIdx.x == 0) {
    __hip_atomic_store(&a.result->status, (int32_t)MAP_EDEVICE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// --------------------------------------------------------------- CSR build --

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

// Degree histogram of the key endpoint: cnt[key] += 1 (cnt = row_ptr, so row
// v's count lands at index v+1 for 1-based key v+1).
__global__ void csr_hist(int32_t n, int64_t m, const int32_t* __restrict__ key, const int32_t* __restrict__ other,
                         int32_t* cnt, int32_t* status) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t k = key[i], o = other[i];
    if (k < 1 || k > n || o < 1 || o > n) {
      __hip_atomic_store(status, (int32_t)MAP_ERANGE_DEV, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      continue;
    }
    atomicAdd(&cnt[k], 1);
  }
}

// In-place inclusive scan of each tile of kScanTile elements; tile totals to sums.
__global__ void __launch_bounds__(kScanThreads) scan_tiles(int32_t* a, int64_t len, int32_t* sums) {
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
__global__ void __launch_bounds__(1024) scan_sums(int32_t* sums, int64_t count) {
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

__global__ void scan_add(int32_t* a, int64_t len, const int32_t* sums) {
  const int64_t tile = blockIdx.x;
  const int32_t pre = sums[tile];
  if (pre == 0) return;
  for (int64_t i = tile * kScanTile + threadIdx.x; i < min(len, (tile + 1) * kScanTile); i += blockDim.x) a[i] += pre;
}

__global__ void copy_i32(int32_t* dst, const int32_t* src, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// col[cursor[key-1]++] = other-1 for every in-range edge.
__global__ void csr_scatter(int32_t n, int64_t m, const int32_t* __restrict__ key, const int32_t* __restrict__ other,
                            int32_t* cursor, int32_t* col) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t k = key[i], o = other[i];
    if (k < 1 || k > n || o < 1 || o > n) continue;
    int32_t pos = atomicAdd(&cursor[k - 1], 1);
    col[pos] = o - 1;
  }
}

// ------------------------------------------------------------------- host --

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool sizes_ok(int32_t n, int64_t m) { return n >= 1 && n <= 0x7ffffffe && m >= 0 && m <= 0x7fffffff; }

struct Layout {
  size_t ctrl, pv, accw, cursor, sums, total;
};

Layout layout(int32_t n) {
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
  size_t end_loop = off;
  // CSR build (shares the region after ctrl)
  off = region;
  L.cursor = off;
  off += align256(((size_t)n + 1) * 4);
  L.sums = off;
  off += align256((((size_t)n + 1 + kScanTile - 1) / kScanTile + 1) * 4);
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
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(map_loop_kernel), kBlock,
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

int launch_loop(LoopArgs& a, hipStream_t stream) {
  DeviceInfo di;
  int rc = device_info(&di);
  if (rc) return rc;
  if (!di.coop) return MAP_EDEVICE;
  const int64_t need = ((int64_t)a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  int64_t grid = (int64_t)di.cus * di.blocks_per_cu;
  if (grid > need) grid = need;
  if (grid >= kMaxGroups) grid -= grid % kMaxGroups;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(fill_u32, dim3(8), dim3(256), 0, stream, reinterpret_cast<uint32_t*>(a.ctrl),
                     (int64_t)(kCtrlBytes / 4), 0u);
  if (hipGetLastError() != hipSuccess) return MAP_EDEVICE;
  void* args[] = {&a};
  if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(map_loop_kernel), dim3((unsigned)grid),
                                 dim3(kBlock), args, 0, stream) != hipSuccess)
    return MAP_EDEVICE;
  return MAP_OK;
}

inline unsigned grid_for(int64_t work, int threads) {
  int64_t g = (work + threads - 1) / threads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

int build_one(int32_t n, int64_t m, const int32_t* key, const int32_t* other, int32_t* row_ptr, int32_t* col,
              int32_t* status, char* ws, const Layout& L, hipStream_t stream) {
  int32_t* cursor = reinterpret_cast<int32_t*>(ws + L.cursor);
  int32_t* sums = reinterpret_cast<int32_t*>(ws + L.sums);
  const int64_t len = (int64_t)n + 1;
  hipLaunchKernelGGL(fill_i32, dim3(grid_for(len, 256)), dim3(256), 0, stream, row_ptr, len, 0);
  if (m > 0)
    hipLaunchKernelGGL(csr_hist, dim3(grid_for(m, 256)), dim3(256), 0, stream, n, m, key, other, row_ptr, status);
  const int64_t tiles = (len + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, stream, row_ptr, len, sums);
  hipLaunchKernelGGL(scan_sums, dim3(1), dim3(1024), 0, stream, sums, tiles);
  hipLaunchKernelGGL(scan_add, dim3((unsigned)tiles), dim3(256), 0, stream, row_ptr, len, sums);
  hipLaunchKernelGGL(copy_i32, dim3(grid_for(n, 256)), dim3(256), 0, stream, cursor, row_ptr, (int64_t)n);
  if (m > 0)
    hipLaunchKernelGGL(csr_scatter, dim3(grid_for(m, 256)), dim3(256), 0, stream, n, m, key, other, cursor, col);
  return hipGetLastError() == hipSuccess ? MAP_OK : MAP_EDEVICE;
}

}  // namespace

extern "C" {

size_t map_workspace_bytes(int32_t n, int64_t m, uint32_t flags) {
  (void)flags;
  if (!sizes_ok(n, m)) return 0;
  return layout(n).total;
}

int map_build_csr(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, int32_t* row_ptr, int32_t* col,
                  int32_t* rrow_ptr, int32_t* rcol, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  if (!sizes_ok(n, m)) return MAP_ERANGE;
  if (!row_ptr || !status || !ws || (m > 0 && (!src || !dst || !col))) return MAP_EINVAL;
  if ((rrow_ptr == nullptr) != (rcol == nullptr)) return MAP_EINVAL;
  if (rrow_ptr && m > 0 && !rcol) return MAP_EINVAL;
  const Layout L = layout(n);
  if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MAP_ENOSPC;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, status, (int64_t)1, (int32_t)MAP_OK);
  int rc = build_one(n, m, src, dst, row_ptr, col, status, static_cast<char*>(ws), L, s);
  if (rc == MAP_OK && rrow_ptr) rc = build_one(n, m, dst, src, rrow_ptr, rcol, status, static_cast<char*>(ws), L, s);
  return rc;
}

static int loop_common(int32_t n, const int32_t* row_ptr, const int32_t* col, const uint8_t* acc, map_result* result,
                       void* ws, size_t ws_bytes, LoopArgs& a) {
  if (n < 1 || n > 0x7ffffffe) return MAP_ERANGE;
  if (!row_ptr || !col || !acc || !result || !ws) return MAP_EINVAL;
  const Layout L = layout(n);
  if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MAP_ENOSPC;
  char* w = static_cast<char*>(ws);
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
  return MAP_OK;
}

int map_propagate(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* rrow_ptr, const int32_t* rcol,
                  const uint8_t* accepting, int32_t* map_out, map_result* result, uint32_t flags, void* ws,
                  size_t ws_bytes, void* stream) {
  (void)rrow_ptr;
  (void)rcol;
  if (flags & ~(MAP_FLAG_DENSE_ONLY | MAP_FLAG_NO_TRACE_DIGEST)) return MAP_EINVAL;
  if (!map_out) return MAP_EINVAL;
  LoopArgs a;
  int rc = loop_common(n, row_ptr, col, accepting, result, ws, ws_bytes, a);
  if (rc) return rc;
  a.propagate = 1;
  a.map_out = map_out;
  return launch_loop(a, reinterpret_cast<hipStream_t>(stream));
}

int map_detect(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* rrow_ptr, const int32_t* rcol,
               const uint8_t* accepting0, map_result* result, uint64_t* trace, int32_t trace_cap,
               uint8_t* accepting_out, int32_t max_iterations, uint32_t flags, void* ws, size_t ws_bytes,
               void* stream) {
  (void)rrow_ptr;
  (void)rcol;
  if (flags & ~(MAP_FLAG_DENSE_ONLY | MAP_FLAG_NO_TRACE_DIGEST)) return MAP_EINVAL;
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
  return launch_loop(a, reinterpret_cast<hipStream_t>(stream));
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
    default: return "unknown status";
  }
}

}  // extern "C"
