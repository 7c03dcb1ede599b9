// Batched decoding: several jobs (each a code, a batch of frames and an
// iteration budget) in one HIP graph, run either as one persistent launch or
// as one launch per phase (MET_BATCH_PHASE_LAUNCHES); the autotuner picks.
//
// The iterations of every job (Methods, Steps 3-5) run inside one kernel as a
// sequence of phases separated by a grid-wide barrier.  A job's check update
// and variable update alternate phase by phase; jobs are staggered by one
// phase, so the same phase holds check work of some jobs (ALU-heavy) and
// variable work of others (memory-heavy) and the two kinds share the machine.
// Blocks claim the phase's tiles dynamically, one job after the other, so each
// compute unit runs a mix of both kinds.  A job whose budget is spent stops
// contributing tiles; frames that converged are retired exactly as in
// met_decode (the same device code runs here, so the results are identical).
//
// The grid is sized so that all blocks are resident at once (occupancy query,
// at most 6 blocks per compute unit), which the barrier needs.  The barrier's
// wait is bounded: if it ever expires (blocks not co-resident), an error flag is
// set, every block returns at its next barrier, and met_batched_check reports it.
//
// With one launch per phase the same tile bodies run in ordinary launches, one
// per phase with the tiles of every job in that phase; the kernel boundary is
// the barrier and the hardware dispatcher hands out the tiles.  Where every
// phase fills the GPU (the three codes at N = 10^6) this is the faster
// schedule: the persistent launch pays a grid barrier and a tail per phase,
// and its resident blocks keep one fixed order of preference in the compute
// units' issue arbitration for the whole phase (the oldest block of a compute
// unit completes 2.3 times the check tiles of the youngest), while short
// ordinary blocks rotate it.  The persistent launch wins where phases are
// short and frames converge: it stops at the first barrier after every frame
// has stopped, while a graph of launches runs to the end.  The launches of a
// phase can also run on parallel streams (by kind of tile, or each job's
// launches as a chain of its own); where every launch fills the GPU that only
// splits the same memory path between them.
#include "met_gpu.h"

namespace met {
namespace {

// Frames per group (interleave width) of a launch: 64 by default; 32 and 16
// (one check step per wave, as in met_decode) for batches of few frames.
constexpr int kBatchWidths[] = {64, 32, 16};

struct BatchJob {
  CheckParams cp;  // per-iteration fields are set in the kernel
  VarParams vp;
  ClassArgs cls[kMaxClasses];
  int32_t cls_blocks[kMaxClasses];  // tiles of each class per frame group
  int32_t cls_wide[kMaxClasses];    // 1 for classes outside the (3,1) / (2,1) shapes
  int32_t cn_tiles_k[2];            // tiles per frame group of narrow / wide classes
  int32_t n_classes, cn_tiles, vn_blocks, G;
  int32_t max_iter, early, offset, pad;
  float *P, *L2;
  uint64_t *B1, *unsat;
  int64_t leaf_words;
};

// Control block at the start of the workspace: grid-barrier state, the
// barrier's group counters and the per-phase tile counters.  Every counter
// sits on its own 128-byte line.
struct BarrierState {
  uint32_t count;  // top-level arrivals (read-modify-written by group leaders)
  uint32_t pad0[31];
  uint32_t gen;    // generation, polled by every block (its own line)
  int32_t err;     // set when a wait expired
  uint32_t stop;   // set with a generation flip when every job has finished
  uint32_t pad1[29];
};
static_assert(sizeof(BarrierState) == 256, "barrier state fills the first 256 bytes");

constexpr int kLine = 32;                     // uint32 words per 128-byte line
constexpr int kMaxBarrierGroups = 64;         // groups of at most 32 blocks of one XCD
constexpr int kMaxJobs = 64;
constexpr int kCounterSets = 3;               // tile counters rotate over phases
constexpr size_t kOffGroups = 256;
constexpr size_t kOffTiles = kOffGroups + (size_t)kMaxBarrierGroups * kLine * 4;
constexpr size_t kOffCursor = kOffTiles + (size_t)kCounterSets * kMaxJobs * kXcds * kLine * 4;
constexpr size_t kControlBytes = kOffCursor + (size_t)kMaxJobs * 4;  // + per job: first group maybe running
constexpr int kMaxGrid = 32 * kXcds * (kMaxBarrierGroups / kXcds);  // 2048 blocks

constexpr uint32_t kSpinLimit = 1u << 21;  // polls of about 1 us each (load + sleep)

__device__ __forceinline__ uint32_t *group_counter(char *ctl, int g) {
  return reinterpret_cast<uint32_t *>(ctl + kOffGroups) + (size_t)g * kLine;
}

__device__ __forceinline__ uint32_t *tile_counter(char *ctl, int set, int job, int xcd) {
  return reinterpret_cast<uint32_t *>(ctl + kOffTiles) + ((size_t)(set * kMaxJobs + job) * kXcds + xcd) * kLine;
}

// Grid-wide barrier in two levels: the blocks of one XCD count in groups of
// at most 32 on their own line, and the last arriver of each group counts at
// the top; the last group flips the generation that everyone polls.  Cache
// maintenance is kept to what the hand-over needs: each wave waits for its own
// stores, one thread per block writes the compute unit's stores back to
// device scope (release) and, after the flip, invalidates its caches
// (acquire), which the block's other waves, held at the block barrier, share.
// The wait is bounded; on expiry the error flag is set, every later barrier
// returns at once and the caller stops.  The last arrival also evaluates
// done() (with every block's writes visible) and publishes the result with the
// flip, so every block takes the same decision.  Returns non-zero when the
// caller must stop (a wait expired, or done() held).
template <class Done>
__device__ int grid_barrier(char *ctl, uint32_t nblocks, Done done) {
  __shared__ int s_err;
  BarrierState *b = reinterpret_cast<BarrierState *>(ctl);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t xcd = blockIdx.x % kXcds, k = blockIdx.x / kXcds;
    const uint32_t nx = (nblocks - xcd + kXcds - 1) / kXcds;  // blocks on this XCD
    const uint32_t gsz = min(32u, nx - (k & ~31u));
    uint32_t ngroups = 0;
    for (uint32_t x = 0; x < kXcds && x < nblocks; ++x) ngroups += ((nblocks - x + kXcds - 1) / kXcds + 31) / 32;
    uint32_t *gc = group_counter(ctl, (int)((k / 32) * kXcds + xcd));
    const uint32_t gen0 = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    bool last = false;
    if (__hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gsz - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == ngroups - 1;
    }
    if (last) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&b->stop, done() ? 1u : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t spins = 0;
      // polls are spaced out so that the waiting blocks do not crowd the
      // memory path of the blocks still working
      while (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen0) {
        if ((++spins & 63) == 0 && __hip_atomic_load(&b->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        if (spins == kSpinLimit) {
          __hip_atomic_store(&b->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(10);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_err = __hip_atomic_load(&b->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) |
            (int)__hip_atomic_load(&b->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  return s_err;
}

// The job table is read through the constant address space: it is written
// before the launch and never during it, so its fields come in as wide scalar
// loads into scalar registers.
#if defined(__HIP_DEVICE_COMPILE__)
using CJob = const __attribute__((address_space(4))) BatchJob;
#else
using CJob = const BatchJob;  // the host pass only parses device code
#endif

// Check tile t of job j at iteration l, among all of its check tiles (KF = -1)
// or among the tiles of its narrow (KF = 0: the (3,1) and (2,1) shapes) or
// wide (KF = 1: every other shape) classes.
// PERSIST: inside the persistent launch (words written by earlier phases of the
// same launch are read with vector loads); false in the phase launches, where
// every earlier phase is an earlier launch and such words are constant.
// Frame group and tile within it of tile t of a job's phase, n tiles per
// group: in 32 bits when the phase has fewer than 2^32 tiles (always, at the
// sizes a workspace can hold), with no division for the first group (a 64-bit
// division is a long sequence of scalar instructions per wave).
__device__ __forceinline__ void split_tile(int64_t t, int32_t n, int G, int64_t *g, int64_t *r) {
  if ((int64_t)n * G <= (int64_t)UINT32_MAX) {
    const uint32_t u = (uint32_t)t, m = (uint32_t)n;
    const uint32_t q = u < m ? 0u : u / m;
    *g = q;
    *r = u - q * m;
  } else {
    *g = t / n;
    *r = t % n;
  }
}

template <int IPW, bool GEN, int W, int KF = -1, bool PERSIST = true>
__device__ __forceinline__ void check_tile(CJob *jobs, int j, int l, int64_t t) {
  const int32_t cn_tiles = KF < 0 ? jobs[j].cn_tiles : jobs[j].cn_tiles_k[KF < 0 ? 0 : KF];
  int64_t g = 0, r = 0;
  split_tile(t, cn_tiles, jobs[j].G, &g, &r);
  int c = 0;
  if constexpr (KF < 0) {
    while (r >= jobs[j].cls_blocks[c]) r -= jobs[j].cls_blocks[c++];
  } else {
    while (jobs[j].cls_wide[c] != KF || r >= jobs[j].cls_blocks[c]) {
      if (jobs[j].cls_wide[c] == KF) r -= jobs[j].cls_blocks[c];
      ++c;
    }
  }
  CheckParams p = jobs[j].cp;
  const int64_t lw = jobs[j].leaf_words;
  uint64_t *B1 = jobs[j].B1, *unsat = jobs[j].unsat;
  const int32_t G = jobs[j].G;
  p.it = l;
  p.flags = jobs[j].early && l >= 2 ? F_TEST : 0;
  p.Pin = l == 1 ? jobs[j].L2 : jobs[j].P;
  p.B1in = B1 + (size_t)((l - 1) & 1) * lw;
  p.B1out = B1 + (size_t)(l & 1) * lw;
  p.unsat = unsat + (size_t)((l - 1) & 1) * G;
  p.unsat_clear = c == 0 ? unsat + (size_t)(l & 1) * G : nullptr;
  const ClassArgs a = jobs[j].cls[c];
  constexpr int I2 = 1;  // degree-11/12 checks: one step (keeps the union of the shapes' registers small)
  const int gi = (int)g;
  // One compiled mode: c2v starts zero-filled, so iteration 1 needs no variant.
  constexpr bool narrow = KF != 1, wide = KF != 0;
  switch (a.shape) {
    case 0: if constexpr (narrow) check_fixed_body<W, 3, 1, M_MAIN, IPW, PERSIST>(p, a, r, gi); break;
    case 1: if constexpr (narrow) check_fixed_body<W, 2, 1, M_MAIN, IPW, PERSIST>(p, a, r, gi); break;
    case 2: if constexpr (wide) check_fixed_body<W, 12, 0, M_MAIN, I2, PERSIST>(p, a, r, gi); break;
    case 3: if constexpr (wide) check_fixed_body<W, 11, 0, M_MAIN, I2, PERSIST>(p, a, r, gi); break;
    case 4: if constexpr (wide) check_fixed_body<W, 6, 0, M_MAIN, IPW, PERSIST>(p, a, r, gi); break;
    case 5: if constexpr (wide) check_fixed_body<W, 5, 0, M_MAIN, IPW, PERSIST>(p, a, r, gi); break;
    case 6: if constexpr (wide) check_fixed_body<W, 4, 0, M_MAIN, IPW, PERSIST>(p, a, r, gi); break;
    default:
      if constexpr (wide && GEN) check_generic_body<W, PERSIST>(p, a, r, gi);
      break;
  }
}

template <int W, bool PERSIST = true>
__device__ __forceinline__ void variable_tile(CJob *jobs, int j, int l, int64_t t) {
  VarParams vp = jobs[j].vp;
  const int32_t vb = jobs[j].vn_blocks;
  vp.it = l;
  vp.retire = jobs[j].early && l >= 2;
  vp.unsat = jobs[j].unsat + (size_t)((l - 1) & 1) * jobs[j].G;
  int64_t g = 0, r = 0;
  split_tile(t, vb, jobs[j].G, &g, &r);
  variable_body<W, 16, PERSIST>(vp, r, (int)g);
}

// Phase step of job j: s = phase - offset; even s: check update of iteration
// s/2 + 1, odd s: its variable update; nothing outside [0, 2 max_iter).
__device__ __forceinline__ int64_t job_tiles(CJob *jobs, int j, int phase, int *l, int *kind) {
  const int s = phase - jobs[j].offset;
  if (s < 0 || s >= 2 * jobs[j].max_iter) return 0;
  *l = s / 2 + 1;
  *kind = s & 1;
  return (int64_t)(*kind == 0 ? jobs[j].cn_tiles : jobs[j].vn_blocks) * jobs[j].G;
}

// Next job (from *cur, round-robin) that has tiles this phase and is not yet
// exhausted on this XCD; *cnt = its number of tiles on this XCD.  XCD x takes
// the tiles x, x + 8, x + 16, ... of a job's phase (as the hardware deals out
// blocks), so every XCD gets the same mix of check classes.  (Contiguous
// ranges per XCD, faster in the plain kernels, were 3 % slower here, also
// when split per check class.)
__device__ bool next_range(CJob *jobs, int n_jobs, int phase, int xcd, int *cur, uint64_t *done, int *j,
                           int64_t *cnt) {
  for (int k = 0; k < n_jobs; ++k) {
    int jj = *cur + k;
    if (jj >= n_jobs) jj -= n_jobs;
    if ((*done >> jj) & 1ull) continue;
    int l = 0, kind = 0;
    const int64_t n = job_tiles(jobs, jj, phase, &l, &kind);
    const int64_t c = n > xcd ? (n - xcd + kXcds - 1) / kXcds : 0;
    if (c > 0) {
      *j = jj;
      *cnt = c;
      *cur = jj + 1 == n_jobs ? 0 : jj + 1;
      return true;
    }
    *done |= 1ull << jj;
  }
  return false;
}

// Atomic add by lane 0 of the calling wave, result broadcast to the wave.
__device__ __forceinline__ uint32_t wave_fetch_inc(uint32_t *c) {
  uint32_t v = 0;
  if ((threadIdx.x & 63) == 0) v = __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Claims the next tile for the block (wave 0 of the block, wave-uniformly):
// -1 when every job's range on this XCD is exhausted for the phase.
__device__ int64_t claim(CJob *jobs, int n_jobs, int phase, int xcd, char *ctl, int *cur, uint64_t *done, int *j) {
  int64_t cnt = 0;
  while (next_range(jobs, n_jobs, phase, xcd, cur, done, j, &cnt)) {
    const uint32_t v = wave_fetch_inc(tile_counter(ctl, phase % kCounterSets, *j, xcd));
    if ((int64_t)v < cnt) return xcd + (int64_t)v * kXcds;
    *done |= 1ull << *j;
  }
  return -1;
}

// One launch runs every phase of every job.  Within a phase, blocks claim
// tiles dynamically from per-(job, XCD) counters, alternating between jobs, so
// blocks that the hardware schedules faster take more tiles and all finish
// together; the claim for the next tile is issued before the current tile's
// loads.  The register budget is capped for 6 resident waves per SIMD.
// Run-time-degree checks (GEN) are compiled only into the variant used by
// batches that hold such classes, which keeps their register arrays out of
// the common one.
template <int IPW, bool GEN, int W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_persistent(
    const BatchJob *table, int n_jobs, int n_phases, char *ctl) {
  CJob *jobs = (CJob *)table;
  __shared__ int s_job[2];
  __shared__ int64_t s_tile[2];
  const int xcd = (int)(blockIdx.x % kXcds);
  int cur = (int)((blockIdx.x / kXcds) % n_jobs);  // claim state of wave 0
  for (int phase = 0; phase < n_phases; ++phase) {
    if (blockIdx.x == 0) {  // counters of the phase after this one (last used two phases ago)
      const int nxt = (phase + 1) % kCounterSets;
      for (int i = threadIdx.x; i < n_jobs * kXcds; i += kBlock)
        __hip_atomic_store(tile_counter(ctl, nxt, i / kXcds, i % kXcds), 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    uint64_t done = 0;
    const bool leader = wave_id() == 0;  // wave 0 claims tiles for the block
    if (leader) {
      int j = -1;
      const int64_t t = claim(jobs, n_jobs, phase, xcd, ctl, &cur, &done, &j);
      if ((threadIdx.x & 63) == 0) {
        s_job[0] = t >= 0 ? j : -1;
        s_tile[0] = t;
      }
    }
    __syncthreads();
    for (int k = 0;; k ^= 1) {
      const int j = __builtin_amdgcn_readfirstlane(s_job[k]);
      if (j < 0) break;
      const int64_t t = uniform64(s_tile[k]);
      int pj = -1;
      int64_t pcnt = 0;
      uint32_t pv = 0;
      if (leader && next_range(jobs, n_jobs, phase, xcd, &cur, &done, &pj, &pcnt))
        pv = wave_fetch_inc(tile_counter(ctl, phase % kCounterSets, pj, xcd));
      int l = 0, kind = 0;
      (void)job_tiles(jobs, j, phase, &l, &kind);
      if (kind == 0)
        check_tile<IPW, GEN, W>(jobs, j, l, t);
      else
        variable_tile<W>(jobs, j, l, t);
      if (leader) {
        int64_t nt = -1;
        if (pj >= 0) {
          if ((int64_t)pv < pcnt) {
            nt = xcd + (int64_t)pv * kXcds;
          } else {
            done |= 1ull << pj;
            nt = claim(jobs, n_jobs, phase, xcd, ctl, &cur, &done, &pj);
          }
        }
        if ((threadIdx.x & 63) == 0) {
          s_job[k ^ 1] = nt >= 0 ? pj : -1;
          s_tile[k ^ 1] = nt;
        }
      }
      __syncthreads();
    }
    // Every job finished: its phases are over, or (early exit) all its frames
    // have retired, after which its tiles would change nothing (masks only
    // shrink, and the output kernels skip retired frames).  Groups below a
    // job's cursor are known to be empty.
    auto all_done = [&]() {
      int32_t *first = reinterpret_cast<int32_t *>(ctl + kOffCursor);
      for (int j = 0; j < n_jobs; ++j) {
        if (phase + 1 - jobs[j].offset >= 2 * jobs[j].max_iter) continue;
        if (!jobs[j].early) return false;
        const uint64_t *act = jobs[j].vp.active;
        int g = __hip_atomic_load(first + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (g < jobs[j].G && __hip_atomic_load(act + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0ull) ++g;
        __hip_atomic_store(first + j, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (g < jobs[j].G) return false;
      }
      return true;
    };
    // a wait expired (results invalid), or every job finished
    if (grid_barrier(ctl, gridDim.x, all_done)) return;
  }
}

// The same phases as separate launches (MET_BATCH_PHASE_LAUNCHES): block b
// takes the b-th tile of the phase, the jobs' tiles one job after the other;
// the kernel boundary replaces the grid barrier and the hardware dispatcher
// the tile claims.  Blocks are short-lived, so the hardware's preference for
// older waves rotates over the blocks instead of fixing the order of the
// resident ones for a whole phase.
// KIND 0 holds every tile of the phase (check and variable tiles when the jobs
// are staggered); without stagger a phase holds one kind, run as up to two
// launches each compiled without the other bodies, so that every launch has
// its own register budget: KIND 1 the check tiles of the (3,1) / (2,1) shapes
// (the bulk of the work, as lean as the plain decoder's check kernel), KIND 3
// the check tiles of every other shape, KIND 2 the variable tiles.
template <int IPW, bool GEN, int W, int KIND>
__device__ __forceinline__ void phase_body(const BatchJob *table, int n_jobs, int phase) {
  CJob *jobs = (CJob *)table;
  int64_t t = blockIdx.x;
  for (int j = 0; j < n_jobs; ++j) {
    int l = 0, kind = 0;
    int64_t cnt = job_tiles(jobs, j, phase, &l, &kind);  // 0 (kind unset) outside the job's phases
    if constexpr (KIND == 1 || KIND == 3)
      cnt = cnt > 0 && kind == 0 ? (int64_t)jobs[j].cn_tiles_k[KIND == 3] * jobs[j].G : 0;
    if constexpr (KIND == 2) cnt = kind == 1 ? cnt : 0;
    if (t < cnt) {
      if constexpr (KIND == 0) {
        if (kind == 0)
          check_tile<IPW, GEN, W, -1, false>(jobs, j, l, t);
        else
          variable_tile<W, false>(jobs, j, l, t);
      } else if constexpr (KIND == 1) {
        check_tile<IPW, false, W, 0, false>(jobs, j, l, t);
      } else if constexpr (KIND == 3) {
        check_tile<IPW, GEN, W, 1, false>(jobs, j, l, t);
      } else {
        variable_tile<W, false>(jobs, j, l, t);
      }
      return;
    }
    t -= cnt;
  }
}

template <int IPW, bool GEN, int W, int KIND>
__global__ __launch_bounds__(kBlock) void k_phase(const BatchJob *table, int n_jobs, int phase) {
  phase_body<IPW, GEN, W, KIND>(table, n_jobs, phase);
}

// The (3,1) / (2,1) check launches and the variable launches, compiled for
// eight resident waves per SIMD: the job table's parameters otherwise take
// more than a hundred scalar registers, which leaves room for seven.
template <int IPW, int W, int KIND>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_phase_lean(
    const BatchJob *table, int n_jobs, int phase) {
  static_assert(KIND == 1 || KIND == 2, "lean launches hold no run-time-degree body");
  phase_body<IPW, false, W, KIND>(table, n_jobs, phase);
}

__global__ __launch_bounds__(kBlock) void k_zero_floats(float *x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) x[i] = 0.0f;
}

__global__ __launch_bounds__(kBlock) void k_control_init(uint32_t *ctl) {
  for (size_t i = threadIdx.x; i < kControlBytes / 4; i += kBlock) ctl[i] = 0u;
}

// ----------------------------------------------------------------------------

struct BatchLayout {
  size_t off_barrier = 0, off_table = 0;
  std::vector<size_t> off_job;
  std::vector<Plan> plans;
  size_t total = 0;
};

BatchLayout make_batch_layout(const met_job *jobs, int n, int W) {
  BatchLayout L;
  size_t o = 0;
  L.off_barrier = o;
  o += align256(kControlBytes);
  L.off_table = o;
  o += align256(sizeof(BatchJob) * (size_t)n);
  for (int j = 0; j < n; ++j) {
    Plan p = make_plan(jobs[j].code, jobs[j].B, false, false, W);
    L.off_job.push_back(o);
    o += p.total;
    L.plans.push_back(p);
  }
  L.total = o;
  return L;
}

int shape_ipw(int shape, int ipw) {
  if (shape == kShapeGeneric) return 1;
  if (kShapeMsg[shape] >= 11) return 1;  // as check_tile compiles them
  return ipw;
}

struct GraphEntry {
  std::vector<uint8_t> key;
  hipGraphExec_t exec = nullptr;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;  // small cache of instantiated graphs
constexpr size_t kGraphCache = 8;

// Graphs are captured on a library-owned stream per device (the caller's may
// be the null stream, which cannot be captured) and launched on the caller's.
std::mutex g_cap_mu;
hipStream_t g_cap_stream[64] = {};

int capture_stream(hipStream_t *out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MET_EHIP, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_cap_mu);
  if (!g_cap_stream[dev]) HIP_TRY(hipStreamCreateWithFlags(&g_cap_stream[dev], hipStreamNonBlocking));
  *out = g_cap_stream[dev];
  return MET_OK;
}

// Side streams of the phase schedule's parallel modes (default priority), with
// the events that fork them from and join them to the launching stream; per
// device, created on first use and kept until the process ends.
constexpr int kSideStreams = 3;
struct SideStreams {
  hipStream_t s[kSideStreams] = {};
  hipEvent_t fork = nullptr, join[kSideStreams] = {};
};
std::mutex g_side_mu;
SideStreams g_side[64];

int side_streams(SideStreams **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MET_EHIP, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_side_mu);
  SideStreams &ss = g_side[dev];
  if (!ss.fork) {
    for (int i = 0; i < kSideStreams; ++i) {
      if (!ss.s[i]) HIP_TRY(hipStreamCreateWithFlags(&ss.s[i], hipStreamNonBlocking));
      if (!ss.join[i]) HIP_TRY(hipEventCreateWithFlags(&ss.join[i], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming));
  }
  *out = &ss;
  return MET_OK;
}

template <typename T>
void append_bytes(std::vector<uint8_t> &k, const T &v) {
  const uint8_t *p = reinterpret_cast<const uint8_t *>(&v);
  k.insert(k.end(), p, p + sizeof(T));
}

// Narrow check classes with at least this many tiles (about eight blocks per
// compute unit) fill the GPU in a launch of their own.
constexpr int64_t kOwnLaunchTiles = 2048;

// Per-launch timer names of the phase launches, by kind of tile.
const char *phase_timer_name(int kind) {
  switch (kind) {
    case 1: return "k_phase:checks(3,1)(2,1)";
    case 2: return "k_phase:variables";
    case 3: return "k_phase:checks(other)";
    default: return "k_phase:mixed";
  }
}

struct Batched {
  const met_job *jobs;
  int n;
  char *ws;
  hipStream_t st;
  int ipw = 4, blocks_per_cu = 0, stagger = 1, use_graph = 1, W = 64, phases = 0;
  int ipw_narrow = 4;  // steps per wave of the (3,1) / (2,1) check tiles
  // phase launches: 0 all on the launching stream; 1 the kinds of a phase
  // (narrow checks, wide checks, variables) on parallel streams, joined at the
  // end of the phase; 2 every job's phases as a chain of its own on one of up
  // to 1 + kSideStreams parallel streams, joined once at the end; 3 the same
  // chains one job after the other on the launching stream
  int streams = 0;
  SideStreams *side = nullptr;
  BatchLayout L;
  std::vector<BatchJob> table;
  std::vector<const DeviceCode *> dev;
  int n_phases = 0;
  unsigned grid = 0;
  bool gen = false;  // some class has no compiled shape

  template <int KIND>
  const void *phase_kernel_k() const {
    // the narrow-check and variable launches hold no run-time-degree body
    if constexpr (KIND == 1 || KIND == 2) {
      if (W == 32) return (const void *)k_phase_lean<1, 32, KIND>;
      if (W == 16) return (const void *)k_phase_lean<1, 16, KIND>;
      const int s = KIND == 1 ? ipw_narrow : 1;  // variable tiles have no steps
      return s == 4 ? (const void *)k_phase_lean<4, 64, KIND>
                    : s == 2 ? (const void *)k_phase_lean<2, 64, KIND> : (const void *)k_phase_lean<1, 64, KIND>;
    } else {
      if (W == 32) return gen ? (const void *)k_phase<1, true, 32, KIND> : (const void *)k_phase<1, false, 32, KIND>;
      if (W == 16) return gen ? (const void *)k_phase<1, true, 16, KIND> : (const void *)k_phase<1, false, 16, KIND>;
      if (gen) return (const void *)k_phase<1, true, 64, KIND>;
      return ipw == 4 ? (const void *)k_phase<4, false, 64, KIND>
                      : ipw == 2 ? (const void *)k_phase<2, false, 64, KIND> : (const void *)k_phase<1, false, 64, KIND>;
    }
  }
  const void *phase_kernel(int kind) const {
    switch (kind) {
      case 1: return phase_kernel_k<1>();
      case 2: return phase_kernel_k<2>();
      case 3: return phase_kernel_k<3>();
      default: return phase_kernel_k<0>();
    }
  }

  const void *kernel() const {
    if (W == 32) return gen ? (const void *)k_persistent<1, true, 32> : (const void *)k_persistent<1, false, 32>;
    if (W == 16) return gen ? (const void *)k_persistent<1, true, 16> : (const void *)k_persistent<1, false, 16>;
    if (gen) return (const void *)k_persistent<1, true, 64>;
    return ipw == 4 ? (const void *)k_persistent<4, false, 64>
                    : ipw == 2 ? (const void *)k_persistent<2, false, 64> : (const void *)k_persistent<1, false, 64>;
  }

  int prepare() {
    if (W != 64) ipw = 1;  // several steps per wave are compiled for groups of 64 only
    L = make_batch_layout(jobs, n, W);
    dev.resize(n);
    table.resize(n);
    int max_end = 0;
    for (int j = 0; j < n; ++j) {
      const met_job &jb = jobs[j];
      int rc = device_code(jb.code, &dev[j]);
      if (rc) return rc;
      const met_code *c = jb.code;
      const DeviceCode *d = dev[j];
      const Plan &pl = L.plans[j];
      char *base = ws + L.off_job[j];
      auto at = [&](size_t off) { return base + off; };
      BatchJob &b = table[j];
      std::memset(&b, 0, sizeof b);
      b.G = pl.G;
      b.max_iter = jb.max_iter;
      b.early = !(jb.flags & MET_FIXED_ITERS);
      b.offset = stagger ? (j & 1) : 0;
      b.P = reinterpret_cast<float *>(at(pl.off_P));
      b.L2 = reinterpret_cast<float *>(at(pl.off_L2));
      b.B1 = reinterpret_cast<uint64_t *>(at(pl.off_B1));
      b.unsat = reinterpret_cast<uint64_t *>(at(pl.off_unsat));
      b.leaf_words = (int64_t)pl.G * c->EL;
      CheckParams &cp = b.cp;
      cp.edge_msgvn = d->edge_msgvn;
      cp.edge_type = d->edge_type;
      cp.leaf_type = d->leaf_type;
      cp.chk_msg_ptr = d->chk_msg_ptr;
      cp.chk_leaf_ptr = d->chk_leaf_ptr;
      cp.M = c->M;
      cp.N2 = c->N2;
      cp.E12 = c->E12;
      cp.EL = c->EL;
      cp.c2v = reinterpret_cast<float *>(at(pl.off_c2v));
      cp.c2v_in = cp.c2v;
      cp.Lphi = reinterpret_cast<float *>(at(pl.off_Lphi));
      cp.Lraw = pl.lraw ? reinterpret_cast<float *>(at(pl.off_Lraw)) : nullptr;
      cp.synw = reinterpret_cast<uint64_t *>(at(pl.off_synw));
      cp.active = reinterpret_cast<uint64_t *>(at(pl.off_active));
      cp.G = pl.G;
      VarParams &vp = b.vp;
      vp.vn_ptr = d->vn_ptr;
      vp.vn_edges = d->vn_edges;
      vp.N2 = c->N2;
      vp.E12 = c->E12;
      vp.L2 = b.L2;
      vp.c2v = cp.c2v;
      vp.P = b.P;
      vp.active = reinterpret_cast<uint64_t *>(at(pl.off_active));
      vp.iters = jb.iters;
      vp.converged = jb.converged;
      vp.G = pl.G;
      const std::vector<ClassArgs> cls = class_args(c);
      b.n_classes = (int)cls.size();
      const int64_t vn_per = (int64_t)kWavesPerBlock * (64 / W);  // variable nodes per tile
      b.vn_blocks = (int32_t)((c->N2 + vn_per - 1) / vn_per);
      max_end = std::max(max_end, b.offset + 2 * jb.max_iter);
      for (size_t k = 0; k < cls.size(); ++k) {
        b.cls[k] = cls[k];
        if (cls[k].shape == kShapeGeneric) gen = true;
      }
    }
    // Run-time-degree classes: check tiles take one step per wave in every
    // launch that holds their body (the persistent launch, the wide-check
    // launches, a phase launch that holds every body); the (3,1) / (2,1)
    // checks keep the requested steps where they have launches of their own.
    ipw_narrow = ipw;
    if (gen) {
      ipw = 1;
      const bool own_narrow = phases && (streams != 0 || !stagger);
      if (!own_narrow) ipw_narrow = 1;
    }
    for (int j = 0; j < n; ++j) {
      BatchJob &b = table[j];
      b.cn_tiles = 0;
      b.cn_tiles_k[0] = b.cn_tiles_k[1] = 0;
      for (int k = 0; k < b.n_classes; ++k) {
        const ClassArgs &ck = b.cls[k];
        const int wide = (ck.shape == 0 || ck.shape == 1) ? 0 : 1;
        const int ip = shape_ipw(ck.shape, wide ? ipw : ipw_narrow);
        const int64_t per = (int64_t)kWavesPerBlock * ip * (64 / W);  // checks per tile
        b.cls_blocks[k] = (int32_t)((ck.n_checks + per - 1) / per);
        b.cn_tiles += b.cls_blocks[k];
        b.cls_wide[k] = wide;
        b.cn_tiles_k[wide] += b.cls_blocks[k];
      }
    }
    n_phases = max_end;
    int dev_id = 0, cus = 0, occ = 0;
    HIP_TRY(hipGetDevice(&dev_id));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id));
    const void *kfn = kernel();
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kfn, kBlock, 0));
    if (occ < 1) return fail(MET_EHIP, "persistent kernel cannot be resident");
    const int per_cu = blocks_per_cu > 0 ? std::min(blocks_per_cu, occ) : std::min(occ, 6);
    grid = (unsigned)std::min(per_cu * cus, kMaxGrid);
    return MET_OK;
  }

  // Everything after the job table copy: set-up, persistent iterations, outputs.
  void enqueue() {
    if (W == 32)
      enqueue_w<32>();
    else if (W == 16)
      enqueue_w<16>();
    else
      enqueue_w<64>();
  }

  template <int kBatchW>
  void enqueue_w() {
    for (int j = 0; j < n; ++j) {
      const met_job &jb = jobs[j];
      const met_code *c = jb.code;
      const DeviceCode *d = dev[j];
      const Plan &pl = L.plans[j];
      char *base = ws + L.off_job[j];
      InitParams ip{};
      ip.llr = jb.llr;
      ip.syn = jb.syn;
      ip.msg_vn_user = d->msg_vn_user;
      ip.leaf_vn = d->leaf_vn;
      ip.chk_pos = d->chk_pos;
      ip.N = c->N;
      ip.M = c->M;
      ip.N2 = c->N2;
      ip.EL = c->EL;
      ip.B = jb.B;
      ip.G = pl.G;
      ip.Lt = reinterpret_cast<float *>(base + pl.off_c2v);
      ip.L2 = reinterpret_cast<float *>(base + pl.off_L2);
      ip.Lphi = reinterpret_cast<float *>(base + pl.off_Lphi);
      ip.Lraw = pl.lraw ? reinterpret_cast<float *>(base + pl.off_Lraw) : nullptr;
      ip.synw = reinterpret_cast<uint64_t *>(base + pl.off_synw);
      ip.active = reinterpret_cast<uint64_t *>(base + pl.off_active);
      ip.unsat = reinterpret_cast<uint64_t *>(base + pl.off_unsat);
      ip.iters = jb.iters;
      ip.converged = jb.converged;
      const int G = pl.G;
      hipLaunchKernelGGL(k_transpose<kBatchW>, dim3((unsigned)((c->N + 63) / 64), G), dim3(kBlock), 0, st, ip);
      const int64_t ni = (c->N2 + c->EL) * kBatchW;
      if (ni > 0)
        hipLaunchKernelGGL(k_init_items<kBatchW>, dim3((unsigned)((ni + kBlock - 1) / kBlock), G), dim3(kBlock), 0,
                           st, ip);
      hipLaunchKernelGGL(k_pack_syndrome<kBatchW>,
                         dim3((unsigned)std::max<int64_t>(1, (c->M + kBlock - 1) / kBlock), G), dim3(kBlock), 0, st,
                         ip);
    }
    for (int j = 0; j < n; ++j) {
      const Plan &pl = L.plans[j];
      const int64_t nc = (int64_t)pl.G * jobs[j].code->E12 * kBatchW;
      if (nc > 0)
        hipLaunchKernelGGL(k_zero_floats, dim3((unsigned)std::min<int64_t>(8192, (nc + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, st, reinterpret_cast<float *>(ws + L.off_job[j] + pl.off_c2v), nc);
    }
    char *ctl = ws + L.off_barrier;
    const BatchJob *tab = reinterpret_cast<const BatchJob *>(ws + L.off_table);
    hipLaunchKernelGGL(k_control_init, dim3(1), dim3(kBlock), 0, st, reinterpret_cast<uint32_t *>(ctl));
    if (phases) {
      // streams 0..k-1: the launching stream and k - 1 side streams
      auto stream_of = [&](int i) { return i == 0 ? st : side->s[i - 1]; };
      auto fork = [&](int k) {
        if (k < 2) return;
        (void)hipEventRecord(side->fork, st);
        for (int i = 1; i < k; ++i) (void)hipStreamWaitEvent(side->s[i - 1], side->fork, 0);
      };
      auto join = [&](int k) {
        for (int i = 1; i < k; ++i) {
          (void)hipEventRecord(side->join[i - 1], side->s[i - 1]);
          (void)hipStreamWaitEvent(st, side->join[i - 1], 0);
        }
      };
      // per-job chains (streams 2: on up to 1 + kSideStreams parallel streams;
      // streams 3: one job after the other on the launching stream)
      const bool chains = streams >= 2;
      const int n_chains = streams == 2 ? std::min(n, kSideStreams + 1) : 1;
      if (chains) fork(n_chains);
      for (int j = 0; j < n && chains; ++j) {
        const BatchJob &b = table[j];
        const BatchJob *tj = tab + j;  // a table of one job: the kernel sees job j alone
        const hipStream_t hs = stream_of(j % n_chains);
        const int64_t cnt[4] = {0, (int64_t)b.cn_tiles_k[0] * b.G, (int64_t)b.vn_blocks * b.G,
                                (int64_t)b.cn_tiles_k[1] * b.G};
        for (int ph = b.offset; ph < b.offset + 2 * b.max_iter; ++ph) {
          int phv = ph, one = 1;
          void *args[] = {(void *)&tj, (void *)&one, (void *)&phv};
          for (int kind : {1, 3, 2}) {
            if ((kind == 2) != (((ph - b.offset) & 1) == 1) || cnt[kind] == 0) continue;
            if (kind == 1 && narrow_fills(j)) {
              launch_narrow_plain<kBatchW>(ph, j, hs);
              continue;
            }
            ScopedTimer t(hs, phase_timer_name(kind));
            (void)hipLaunchKernel(phase_kernel(kind), dim3((unsigned)cnt[kind]), dim3(kBlock), args, 0, hs);
          }
        }
      }
      if (chains) join(n_chains);
      for (int ph = 0; ph < n_phases && !chains; ++ph) {
        // tiles of the phase: [0] all, [1] narrow checks, [2] variables, [3] wide checks
        int64_t tiles[4] = {0, 0, 0, 0};
        std::vector<int> narrow_jobs;  // jobs with (3,1) / (2,1) tiles in this phase
        for (int j = 0; j < n; ++j) {
          const BatchJob &b = table[j];
          const int s = ph - b.offset;
          if (s < 0 || s >= 2 * b.max_iter) continue;
          if ((s & 1) == 0) {
            if (b.cn_tiles_k[0] > 0) narrow_jobs.push_back(j);
            tiles[1] += (int64_t)b.cn_tiles_k[0] * b.G;
            tiles[3] += (int64_t)b.cn_tiles_k[1] * b.G;
          } else {
            tiles[2] += (int64_t)b.vn_blocks * b.G;
          }
        }
        tiles[0] = tiles[1] + tiles[2] + tiles[3];
        if (tiles[0] == 0) continue;
        int phv = ph;
        void *args[] = {(void *)&tab, (void *)&n, (void *)&phv};
        const bool mixed = streams == 0 && tiles[2] > 0 && tiles[1] + tiles[3] > 0;
        int n_kinds = 0;
        for (int kind : {1, 3, 2}) n_kinds += tiles[kind] > 0;
        const int k_streams = streams == 1 ? n_kinds : 1;
        fork(k_streams);
        int i = 0;
        for (int kind : {0, 1, 3, 2}) {
          if (mixed ? kind != 0 : (kind == 0 || tiles[kind] == 0)) continue;
          const hipStream_t hs = stream_of(k_streams > 1 ? i++ : 0);
          if (kind == 1) {
            // jobs whose narrow classes fill the GPU on their own take the
            // plain decoder's launches; the others share one launch
            bool own = true;
            for (int j : narrow_jobs) own = own && narrow_fills(j);
            if (own) {
              for (int j : narrow_jobs) launch_narrow_plain<kBatchW>(ph, j, hs);
              continue;
            }
          }
          ScopedTimer t(hs, phase_timer_name(kind));
          (void)hipLaunchKernel(phase_kernel(kind), dim3((unsigned)tiles[kind]), dim3(kBlock), args, 0, hs);
        }
        join(k_streams);
      }
    } else {
      ScopedTimer t(st, "k_persistent");
      void *args[] = {(void *)&tab, (void *)&n, (void *)&n_phases, (void *)&ctl};
      (void)hipLaunchKernel(kernel(), dim3(grid), dim3(kBlock), args, 0, st);
    }
    for (int j = 0; j < n; ++j) {
      const met_job &jb = jobs[j];
      const met_code *c = jb.code;
      const DeviceCode *d = dev[j];
      const Plan &pl = L.plans[j];
      char *base = ws + L.off_job[j];
      const int G = pl.G;
      const size_t leaf_words = (size_t)G * c->EL, leaf_floats = leaf_words * kBatchW;
      uint64_t *B1 = reinterpret_cast<uint64_t *>(base + pl.off_B1);
      uint64_t *unsat = reinterpret_cast<uint64_t *>(base + pl.off_unsat);
      float *P1 = nullptr;
      TestParams tp{};
      tp.edge_msgvn = d->edge_msgvn;
      tp.chk_msg_ptr = d->chk_msg_ptr;
      tp.chk_leaf_ptr = d->chk_leaf_ptr;
      tp.M = c->M;
      tp.N2 = c->N2;
      tp.E12 = c->E12;
      tp.EL = c->EL;
      tp.P = reinterpret_cast<float *>(base + pl.off_P);
      tp.synw = reinterpret_cast<uint64_t *>(base + pl.off_synw);
      tp.B1 = B1 + (size_t)(jb.max_iter & 1) * leaf_words;
      tp.active = reinterpret_cast<uint64_t *>(base + pl.off_active);
      tp.unsat = unsat + (size_t)(jb.max_iter & 1) * G;
      const int64_t per = (int64_t)kWavesPerBlock * (64 / kBatchW);
      hipLaunchKernelGGL(k_test<kBatchW>, dim3((unsigned)((c->M + per - 1) / per), G), dim3(kBlock), 0, st, tp);
      FinalParams fp{};
      fp.vn_slot = d->vn_slot;
      fp.N = c->N;
      fp.N2 = c->N2;
      fp.EL = c->EL;
      fp.B = jb.B;
      fp.max_iter = jb.max_iter;
      fp.P = tp.P;
      fp.P1a = P1;
      fp.P1b = P1 ? P1 + leaf_floats : nullptr;
      fp.B1a = B1;
      fp.B1b = B1 + leaf_words;
      fp.active = tp.active;
      fp.unsat_last = tp.unsat;
      fp.iters = jb.iters;
      fp.converged = jb.converged;
      fp.bits = jb.bits;
      fp.posterior = jb.posterior;
      fp.G = G;
      hipLaunchKernelGGL(k_final_status<kBatchW>, dim3((jb.B + kBlock - 1) / kBlock), dim3(kBlock), 0, st, fp);
      hipLaunchKernelGGL(k_finalize<kBatchW>, dim3((unsigned)((c->N + 63) / 64), G), dim3(kBlock), 0, st, fp);
    }
  }

  std::vector<uint8_t> key() const {
    std::vector<uint8_t> k;
    append_bytes(k, ws);
    int dev = 0;
    (void)hipGetDevice(&dev);
    append_bytes(k, dev);
    append_bytes(k, ipw);
    append_bytes(k, ipw_narrow);
    append_bytes(k, phases);
    append_bytes(k, stagger);  // the phase schedule bakes each phase's tile count into the graph
    append_bytes(k, streams);
    append_bytes(k, W);
    append_bytes(k, gen);
    append_bytes(k, grid);
    append_bytes(k, n_phases);
    for (int j = 0; j < n; ++j) {
      append_bytes(k, jobs[j]);
      append_bytes(k, jobs[j].code->uid);  // a new code at a freed code's address must not match
    }
    return k;
  }

  // Every (3,1) / (2,1) class of job j fills the GPU in a launch of its own.
  bool narrow_fills(int j) const {
    const BatchJob &b = table[j];
    for (int c = 0; c < b.n_classes; ++c)
      if (!b.cls_wide[c] && (int64_t)b.cls_blocks[c] * b.G < kOwnLaunchTiles) return false;
    return true;
  }

  // The (3,1) / (2,1) checks of job j at phase ph as the plain decoder
  // launches them: one launch per class, parameters by value.
  template <int kBatchW>
  void launch_narrow_plain(int ph, int j, hipStream_t hs) {
    const BatchJob &b = table[j];
    const int l = (ph - b.offset) / 2 + 1;
    CheckParams p = b.cp;
    p.it = l;
    p.flags = b.early && l >= 2 ? F_TEST : 0;
    p.Pin = l == 1 ? b.L2 : b.P;
    p.B1in = b.B1 + (size_t)((l - 1) & 1) * b.leaf_words;
    p.B1out = b.B1 + (size_t)(l & 1) * b.leaf_words;
    p.unsat = b.unsat + (size_t)((l - 1) & 1) * b.G;
    for (int c = 0; c < b.n_classes; ++c) {
      if (b.cls_wide[c]) continue;
      p.unsat_clear = c == 0 ? b.unsat + (size_t)(l & 1) * b.G : nullptr;
      ScopedTimer t(hs, phase_timer_name(1));
      launch_check<kBatchW, float>(p, b.cls[c], M_MAIN, ipw_narrow, b.G, hs);
    }
  }

  int run() {
    int rc = prepare();
    if (rc) return rc;
    if (phases && streams) {
      rc = side_streams(&side);
      if (rc) return rc;
    }
    // the job table is stream-ordered before the graph (or the plain launches)
    HIP_TRY(hipMemcpyAsync(ws + L.off_table, table.data(), sizeof(BatchJob) * table.size(), hipMemcpyHostToDevice,
                           st));
    if (!use_graph || g_timing.on) {
      enqueue();
      HIP_TRY(hipGetLastError());
      return MET_OK;
    }
    const std::vector<uint8_t> k = key();
    hipGraphExec_t exec = nullptr;
    {
      std::lock_guard<std::mutex> lock(g_graph_mu);
      for (const GraphEntry &e : g_graphs)
        if (e.key == k) exec = e.exec;
    }
    if (!exec) {
      hipStream_t cap = nullptr;
      rc = capture_stream(&cap);
      if (rc) return rc;
      const hipStream_t user = st;
      st = cap;
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
      enqueue();
      const hipError_t le = hipGetLastError();
      const hipError_t ce = hipStreamEndCapture(cap, &graph);
      st = user;
      if (le != hipSuccess) return fail(MET_EHIP, "launch during capture: %s", hipGetErrorString(le));
      if (ce != hipSuccess) return fail(MET_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ce));
      const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) return fail(MET_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
      std::lock_guard<std::mutex> lock(g_graph_mu);
      if (g_graphs.size() == kGraphCache) {
        (void)hipGraphExecDestroy(g_graphs.front().exec);
        g_graphs.erase(g_graphs.begin());
      }
      g_graphs.push_back({k, exec});
    }
    HIP_TRY(hipGraphLaunch(exec, st));
    return MET_OK;
  }
};

}  // namespace
}  // namespace met

using met::fail;

static int validate_jobs(const met_job *jobs, int32_t n) {
  if (!jobs || n < 1 || n > 64) return fail(MET_EINVAL, "n_jobs = %d outside 1..64", n);
  for (int j = 0; j < n; ++j) {
    const met_job &b = jobs[j];
    if (!b.code) return fail(MET_EINVAL, "job %d: NULL code", j);
    if (b.B < 1 || b.B > 65535) return fail(MET_EINVAL, "job %d: B = %d outside 1..65535", j, b.B);
    if (b.max_iter < 1 || b.max_iter > 1000000) return fail(MET_EINVAL, "job %d: bad max_iter", j);
    if (b.flags & ~(uint32_t)MET_FIXED_ITERS) return fail(MET_EINVAL, "job %d: unknown flags", j);
    if (!b.llr || !b.syn || !b.bits || !b.iters || !b.converged) return fail(MET_EINVAL, "job %d: NULL buffer", j);
    if (b.posterior) return fail(MET_EINVAL, "job %d: posterior output is not available in batched mode", j);
    if (((uintptr_t)b.llr & 3) || ((uintptr_t)b.posterior & 3) || ((uintptr_t)b.iters & 3))
      return fail(MET_EINVAL, "job %d: misaligned buffer", j);
  }
  return MET_OK;
}

// Enough for every interleave width a launch (or the autotuner) may use.
static size_t batched_bytes(const met_job *jobs, int32_t n_jobs) {
  size_t most = 0;
  for (int w : met::kBatchWidths) most = std::max(most, met::make_batch_layout(jobs, n_jobs, w).total);
  return most;
}

extern "C" int met_batched_workspace_bytes(const met_job *jobs, int32_t n_jobs, size_t *bytes) { return met::guarded("met_batched_workspace_bytes", [&]() -> int {
  met::clear_error();
  int rc = validate_jobs(jobs, n_jobs);
  if (rc) return rc;
  if (!bytes) return fail(MET_EINVAL, "NULL bytes");
  *bytes = batched_bytes(jobs, n_jobs);
  return MET_OK;
  });
}

extern "C" int met_decode_batched(const met_job *jobs, int32_t n_jobs, void *workspace, size_t ws_bytes,
                                  const met_tuning *tuning, void *stream) { return met::guarded("met_decode_batched", [&]() -> int {
  met::clear_error();
  int rc = validate_jobs(jobs, n_jobs);
  if (rc) return rc;
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(MET_EINVAL, "workspace NULL or not 256-byte aligned");
  const size_t need = batched_bytes(jobs, n_jobs);
  if (ws_bytes < need) return fail(MET_EINVAL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  met::Batched b{jobs, n_jobs, static_cast<char *>(workspace), (hipStream_t)stream};
  if (tuning) {
    const int s = tuning->check_steps_per_wave;
    if (s != 0 && s != 1 && s != 2 && s != 4) return fail(MET_EINVAL, "check_steps_per_wave must be 0, 1, 2 or 4");
    if (s) b.ipw = s;
    if (tuning->blocks_per_cu < 0 || tuning->blocks_per_cu > 64) return fail(MET_EINVAL, "bad blocks_per_cu");
    b.blocks_per_cu = tuning->blocks_per_cu;
    const uint32_t bf = tuning->batch_flags;
    if (bf & ~63u) return fail(MET_EINVAL, "unknown batch_flags");
    const uint32_t order = bf & (MET_BATCH_KIND_STREAMS | MET_BATCH_JOB_STREAMS | MET_BATCH_JOBS_IN_TURN);
    if (order & (order - 1))
      return fail(MET_EINVAL, "MET_BATCH_KIND_STREAMS, MET_BATCH_JOB_STREAMS and MET_BATCH_JOBS_IN_TURN exclude each other");
    b.stagger = !(bf & MET_BATCH_NO_STAGGER);
    b.use_graph = !(bf & MET_BATCH_NO_GRAPH);
    b.streams = (bf & MET_BATCH_KIND_STREAMS) ? 1 : (bf & MET_BATCH_JOB_STREAMS) ? 2 : (bf & MET_BATCH_JOBS_IN_TURN) ? 3 : 0;
    b.phases = (bf & MET_BATCH_PHASE_LAUNCHES) || b.streams ? 1 : 0;
    const int w = tuning->interleave;
    if (w != 0 && w != 16 && w != 32 && w != 64) return fail(MET_EINVAL, "interleave must be 0, 16, 32 or 64");
    if (w) b.W = w;
    for (int r = 0; r < 3; ++r)
      if (tuning->reserved[r]) return fail(MET_EINVAL, "reserved tuning fields must be 0");
  }
  return b.run();
  });
}

// ---- Autotuning -------------------------------------------------------------
// Launch shapes are ranked on a short run of the same jobs (each budget capped
// at probe_iters iterations): the per-phase cost of a shape is the same in
// every phase, so a few iterations rank the shapes as the full run would.
// Results are cached per (device, jobs) signature for the life of the process.

namespace met {
namespace {

struct TuneEntry {
  std::vector<uint8_t> key;
  met_tuning best;
  float ms;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

std::vector<uint8_t> tune_key(const met_job *jobs, int n, int probe_iters) {
  std::vector<uint8_t> k;
  int dev = 0;
  (void)hipGetDevice(&dev);
  append_bytes(k, dev);
  append_bytes(k, probe_iters);
  for (int j = 0; j < n; ++j) {
    const met_code *c = jobs[j].code;
    append_bytes(k, c->uid);
    append_bytes(k, c->N);
    append_bytes(k, c->M);
    append_bytes(k, c->E12);
    append_bytes(k, jobs[j].B);
    append_bytes(k, jobs[j].max_iter);
    append_bytes(k, jobs[j].flags);
  }
  return k;
}

// Time one launch shape: one untimed run, then `reps` runs between events.
// Returns a negative time if the barrier expired.
int time_shape(const std::vector<met_job> &probe, char *ws, hipStream_t st, const met_tuning &t, int reps,
               float *ms) {
  met_tuning u = t;
  u.batch_flags |= MET_BATCH_NO_GRAPH;
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  int rc = MET_OK;
  for (int r = 0; r <= reps && rc == MET_OK; ++r) {
    if (r == 1) rc = hipEventRecord(a, st) == hipSuccess ? MET_OK : fail(MET_EHIP, "hipEventRecord");
    if (rc == MET_OK) rc = met_decode_batched(probe.data(), (int32_t)probe.size(), ws, SIZE_MAX, &u, st);
  }
  if (rc == MET_OK && hipEventRecord(b, st) != hipSuccess) rc = fail(MET_EHIP, "hipEventRecord");
  if (rc == MET_OK && hipEventSynchronize(b) != hipSuccess) rc = fail(MET_EHIP, "hipEventSynchronize");
  float t_ms = 0.0f;
  if (rc == MET_OK && hipEventElapsedTime(&t_ms, a, b) != hipSuccess) rc = fail(MET_EHIP, "hipEventElapsedTime");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  int32_t expired = 0;
  rc = met_batched_check(ws, &expired);
  if (rc) return rc;
  *ms = expired ? -1.0f : t_ms / (float)reps;
  return MET_OK;
}

}  // namespace
}  // namespace met

extern "C" int met_batched_autotune(const met_job *jobs, int32_t n_jobs, void *workspace, size_t ws_bytes,
                                    int32_t probe_iters, met_tuning *best, float *best_ms, void *stream) { return met::guarded("met_batched_autotune", [&]() -> int {
  met::clear_error();
  int rc = validate_jobs(jobs, n_jobs);
  if (rc) return rc;
  if (!best) return fail(MET_EINVAL, "NULL best");
  if (probe_iters < 0 || probe_iters > 1000) return fail(MET_EINVAL, "probe_iters = %d outside 0..1000", probe_iters);
  if (probe_iters == 0) probe_iters = 6;
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(MET_EINVAL, "workspace NULL or not 256-byte aligned");
  const size_t need = batched_bytes(jobs, n_jobs);
  if (ws_bytes < need) return fail(MET_EINVAL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  const std::vector<uint8_t> key = met::tune_key(jobs, n_jobs, probe_iters);
  {
    std::lock_guard<std::mutex> lock(met::g_tune_mu);
    for (const met::TuneEntry &e : met::g_tune)
      if (e.key == key) {
        *best = e.best;
        if (best_ms) *best_ms = e.ms;
        return MET_OK;
      }
  }
  std::vector<met_job> probe(jobs, jobs + n_jobs);
  for (met_job &j : probe) j.max_iter = std::min(j.max_iter, probe_iters);
  char *ws = static_cast<char *>(workspace);
  const hipStream_t st = (hipStream_t)stream;
  met_tuning cur{};
  float cur_ms = -1.0f;
  // interleave width x steps per wave x resident blocks per CU, then the
  // stagger of the best (widths below 64 take one step per wave)
  for (int w : met::kBatchWidths)
    for (int ipw : {4, 2, 1})
      for (int bpc : {6, 5, 4, 3, 2}) {
      if (w != 64 && (ipw != 1 || bpc == 5 || bpc == 3)) continue;
      met_tuning t{};
      t.interleave = w;
      t.check_steps_per_wave = ipw;
      t.blocks_per_cu = bpc;
      float ms = 0.0f;
      rc = met::time_shape(probe, ws, st, t, 2, &ms);
      if (rc) return rc;
      if (ms > 0.0f && (cur_ms < 0.0f || ms < cur_ms)) {
        cur = t;
        cur_ms = ms;
      }
    }
  if (cur_ms < 0.0f) return fail(MET_EHIP, "no launch shape kept its blocks resident");
  {
    met_tuning t = cur;
    t.batch_flags = MET_BATCH_NO_STAGGER;
    float ms = 0.0f;
    rc = met::time_shape(probe, ws, st, t, 2, &ms);
    if (rc) return rc;
    if (ms > 0.0f && ms < cur_ms) {
      cur = t;
      cur_ms = ms;
    }
  }
  // one launch per phase: interleave width x steps per wave x stagger x streams
  for (int w : met::kBatchWidths)
    for (int ipw : {4, 2, 1})
      for (uint32_t stag : {0u, (uint32_t)MET_BATCH_NO_STAGGER})
        for (uint32_t par : {0u, (uint32_t)MET_BATCH_KIND_STREAMS, (uint32_t)MET_BATCH_JOB_STREAMS,
                             (uint32_t)MET_BATCH_JOBS_IN_TURN}) {
        if (w != 64 && ipw != 1) continue;
        met_tuning t{};
        t.interleave = w;
        t.check_steps_per_wave = ipw;
        t.batch_flags = MET_BATCH_PHASE_LAUNCHES | stag | par;
        float ms = 0.0f;
        rc = met::time_shape(probe, ws, st, t, 2, &ms);
        if (rc) return rc;
        if (ms > 0.0f && ms < cur_ms) {
          cur = t;
          cur_ms = ms;
        }
      }
  {
    std::lock_guard<std::mutex> lock(met::g_tune_mu);
    met::g_tune.push_back({key, cur, cur_ms});
  }
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return MET_OK;
  });
}

extern "C" int met_batched_check(const void *workspace, int32_t *barrier_expired) { return met::guarded("met_batched_check", [&]() -> int {
  met::clear_error();
  if (!workspace || !barrier_expired) return fail(MET_EINVAL, "NULL argument");
  met::BarrierState s{};
  const hipError_t e = hipMemcpy(&s, workspace, sizeof s, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(MET_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
  *barrier_expired = s.err;
  return MET_OK;
  });
}
