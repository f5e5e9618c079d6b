// driver.h -- device-side pieces shared by the adaptive solver kernels:
// precision traits, compensated time, save-time bookkeeping and the two
// work-assignment forms (one lane per trajectory; persistent atomic queue).
//
// A "Lane" type provides
//   init(a, i)    load trajectory i and prepare its first step
//   attempt(a, i) one step attempt (accept or reject), sets `done`
//   finish(a, i)  write status / step counts, NaN-fill unreached saves
// and is run unchanged by both forms, so their outputs are bit-identical.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ens_internal.h"

namespace ens {

// Precision traits: FP32 uses the hardware reciprocal/log2/exp2 (error
// control only needs a few correct bits); FP64 uses the libm functions.
template <class R>
struct Num;

template <>
struct Num<float> {
  __device__ static inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  __device__ static inline float log2(float x) { return __builtin_amdgcn_logf(x); }
  __device__ static inline float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
  __device__ static inline float sqrt(float x) { return __builtin_sqrtf(x); }
  __device__ static inline float nan() { return __builtin_nanf(""); }
  // max, min and clamp as one v_med3_f32 (operands not NaN).  fmax / fmin of
  // a value computed in another basic block (a loop-carried step size, state
  // or error) first quiets it with an extra v_max, because the selector sees
  // one block at a time; the median against +-inf needs no quieting.  The
  // infinity goes through an opaque scalar move so that the median is not
  // folded back into fmax / fmin.
  __device__ static inline float inf() {
    float v;
    asm("s_mov_b32 %0, 0x7f800000" : "=s"(v));
    return v;
  }
  __device__ static inline float max(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, inf()); }
  __device__ static inline float min(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, -inf()); }
  __device__ static inline float clamp(float x, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(x, lo, hi);
  }
  // max(x, floor) for x >= 0 and a positive floor: non-negative floats order
  // as their bit patterns do, so an integer maximum (no quieting) suffices
  __device__ static inline float max_nonneg(float x, float floor) {
    return __builtin_bit_cast(float, ::max(__builtin_bit_cast(int, x), __builtin_bit_cast(int, floor)));
  }
};

template <>
struct Num<double> {
  __device__ static inline double rcp(double x) { return 1.0 / x; }
  __device__ static inline double log2(double x) { return ::log2(x); }
  __device__ static inline double exp2(double x) { return ::exp2(x); }
  __device__ static inline double sqrt(double x) { return ::sqrt(x); }
  __device__ static inline double nan() { return __builtin_nan(""); }
  __device__ static inline double max(double a, double b) { return fmax(a, b); }
  __device__ static inline double min(double a, double b) { return fmin(a, b); }
  __device__ static inline double clamp(double x, double lo, double hi) {
    return fmin(hi, fmax(lo, x));
  }
  __device__ static inline double max_nonneg(double x, double floor) { return fmax(x, floor); }
};

// Save-time landing: a step whose proposal reaches within this factor of
// the remaining distance to the next save time is set to exactly that
// distance (cut when longer, stretched when up to 10% shorter).
constexpr double kStretch = 1.1;

// t_hi + t_lo carries the time exactly enough that N steps of size h lose no
// more than one rounding of the final sum (Knuth's TwoSum on every add).
struct CompTime {
  double hi, lo;
  __device__ inline void set(double v) { hi = v; lo = 0.0; }
  __device__ inline void add(double h) {
    const double s = hi + h;
    const double bp = s - hi;
    const double err = (hi - (s - bp)) + (h - bp);
    hi = s;
    lo += err;
  }
  // distance from the current time to `target`
  __device__ inline double to(double target) const { return (target - hi) - lo; }
  __device__ inline double value() const { return hi + lo; }
  // the current time has reached save time v
  __device__ inline bool reached(double v) const { return v <= hi + lo; }
};

// Number of work items of a launch: `n`, or the device-side count when the
// launch was sized on the host for an upper bound.
__device__ inline int64_t work_items(const LaunchArgs& a) {
  if (!a.n_dev) return a.n;
  const int64_t d = (int64_t)*a.n_dev;
  return d < a.n ? d : a.n;
}

// Column of work item k in the input arrays, and in `out`.
__device__ inline int64_t in_col(const LaunchArgs& a, int64_t k) {
  return a.idx ? a.idx[k] : k;
}
__device__ inline int64_t out_col(const LaunchArgs& a, int64_t k, int64_t i) {
  return a.scatter ? i : k;
}

// The save fractions, copied into LDS once per block (stage_theta).  Each
// lane indexes them with its own save counter; read from the kernel
// arguments that would be a global load per save, and its wait would also
// wait for every older store and load of the wave.
static __shared__ double lds_theta[kMaxSave];

__device__ inline void stage_theta(const LaunchArgs& a) {
  for (int j = (int)threadIdx.x; j < a.n_save; j += (int)blockDim.x) lds_theta[j] = a.theta[j];
  __syncthreads();
}

__device__ inline double save_time(const LaunchArgs&, double t0, double tf, int j) {
  return t0 + lds_theta[j] * (tf - t0);
}

__device__ inline double tspan_at(const LaunchArgs& a, int row, int64_t i) {
  return a.tspan_bcast ? a.tspan[row] : a.tspan[row * a.in_stride + i];
}

template <class R>
__device__ inline R load_col(const LaunchArgs& a, const void* base, int row, int64_t i) {
  return static_cast<const R*>(base)[row * a.in_stride + i];
}


// Inputs of one trajectory, loaded ahead of its integration so that the
// persistent form can fetch a lane's next trajectory while the lane is still
// busy with the current one.
template <class R, int M, int N>
struct LaneInput {
  R p[M], u[N];
  double t0, tf;
  int64_t i;  // input column
  __device__ inline void load(const LaunchArgs& a, int64_t k) {
    i = in_col(a, k);
#pragma unroll
    for (int r = 0; r < M; ++r) p[r] = load_col<R>(a, a.params, r, i);
#pragma unroll
    for (int c = 0; c < N; ++c) u[c] = load_col<R>(a, a.u0, c, i);
    t0 = tspan_at(a, 0, i);
    tf = tspan_at(a, 1, i);
  }
};

// ---------------------------------------------------------------------------
// Form 2 (cost-sorted lanes): each block of B threads takes R*B consecutive
// trajectories (R = tpl rounds), initialises each one to learn its expected
// amount of work -- the span divided by the first step, (tf - t0) / h --
// sorts the R*B items by that key (bitonic network in LDS), and integrates
// them in sorted order, 64 consecutive sorted items per wave and round, so
// that the lanes of a wave hold trajectories of similar cost and finish at
// similar times.  Rounds alternate direction (round 0: wave w takes sorted
// group w, round 1: group 2W-1-w, ...), so every wave of the block gets a
// similar total and the block does not idle behind one expensive wave.  The
// first initialisation is thrown away; the second, on the lane the item was
// sorted to, is the same computation, so results are bit-identical to the
// other forms.
//
// Staged variant (one round): a wave's lanes hold items scattered over the
// block's window and, with dense output, each writes a save in whichever
// step covers it, so every 128-byte output line would be filled by several
// waves at different times and leave L2 partially written again and again.
// Instead the saves go to LDS rows [j][c][item] (n_save N B values) and the
// block copies them out, one full row at a time, once all its lanes are done.

// Ascending bitonic sort of v[0..NE) in LDS by the B threads of the block.
template <int NE, int B>
__device__ inline void block_sort(uint64_t* v, int tid) {
  static_assert((NE & (NE - 1)) == 0 && NE >= 2, "sort size must be a power of two");
  for (int k = 2; k <= NE; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int p = tid; p < NE / 2; p += B) {
        const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));  // lower index of the pair
        const int m = i | j;
        const uint64_t x = v[i], y = v[m];
        const bool up = (i & k) == 0;
        if ((x > y) == up) {
          v[i] = y;
          v[m] = x;
        }
      }
      __syncthreads();
    }
  }
}

// Expected work of an initialised lane: attempts scale with span / step.
template <class Lane>
__device__ inline float work_key(const Lane& L) {
  if (L.done) return 0.0f;
  const float r = (float)((L.tf - L.t0) / (double)L.h);
  return (r >= 0.0f && r <= 3.0e38f) ? r : 3.0e38f;  // NaN or inf: last
}

template <class Lane, int B, int R, bool Staged = false>
__device__ inline void run_sorted(const LaunchArgs& a) {
  constexpr int NE = B * R, W = B / kWave;
  static_assert(!Staged || R == 1, "the staged form holds one round's saves");
  __shared__ uint64_t keys[NE];
  extern __shared__ __align__(16) unsigned char lds_stage_bytes[];
  using Real = typename Lane::Real;
  Real* const stage = reinterpret_cast<Real*>(lds_stage_bytes);
  stage_theta(a);
  const int tid = (int)threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int64_t base = (int64_t)blockIdx.x * NE;
  const int64_t n = work_items(a);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = r * B + tid;
    float key = __builtin_inff();  // items past the end sort last
    if (base + e < n) {
      typename Lane::Input in;
      in.load(a, base + e);
      Lane L;
      L.init(a, base + e, in);
      key = work_key(L);
    }
    keys[e] = ((uint64_t)__float_as_uint(key) << 32) | (uint32_t)e;
  }
  __syncthreads();
  block_sort<NE, B>(keys, tid);
  for (int r = 0; r < R; ++r) {
    const int grp = r * W + ((r & 1) ? (W - 1 - wave) : wave);
    const int item = (int)(uint32_t)keys[grp * kWave + lane];
    const int64_t k = base + item;
    if (k >= n) continue;
    typename Lane::Input in;
    in.load(a, k);
    Lane L;
    if constexpr (Staged)
      L.init_to(a, in, stage + item, B);
    else
      L.init(a, k, in);
    while (!L.done) L.attempt(a, k);
    L.finish(a, k);
  }
  if constexpr (Staged) {
    __syncthreads();
    const int64_t k = base + tid;
    if (k < n) {
      Real* const dst = static_cast<Real*>(a.out) + out_col(a, k, in_col(a, k));
      const int rows = a.n_save * Lane::N;
      for (int r = 0; r < rows; ++r) dst[r * a.out_stride] = stage[r * B + tid];
    }
  }
}

// ---------------------------------------------------------------------------
// Form 3 (persistent queue of cost-sorted chunks): a resident grid of blocks
// of B threads, each claiming chunks of B consecutive trajectories from the
// atomic work counter (one atomic per chunk), until the queue is empty.  A
// chunk is handled as the sorted form handles its block: every thread
// initialises one item to learn its expected work, the block sorts the chunk
// by it in LDS, and wave w integrates the w-th group of 64 sorted items, so
// a wave's lanes finish together.  The block then claims the next chunk:
// blocks that drew cheap chunks take more of them.  Each item runs the same
// lane code as in the other forms, so results are bit-identical.
// One chunk of B items starting at work item `base`: every thread
// initialises one item for its key, the block sorts, wave w integrates sorted
// group w.  Ends with a barrier, so keys may be reused at once.
template <class Lane, int B>
__device__ inline void sorted_chunk(const LaunchArgs& a, int64_t base, int64_t n, int tid,
                                    uint64_t* keys) {
  float key = __builtin_inff();  // items past the end sort last
  if (base + tid < n) {
    typename Lane::Input in;
    in.load(a, base + tid);
    Lane L;
    L.init(a, base + tid, in);
    key = work_key(L);
  }
  keys[tid] = ((uint64_t)__float_as_uint(key) << 32) | (uint32_t)tid;
  __syncthreads();
  block_sort<B, B>(keys, tid);
  const int64_t k = base + (int)(uint32_t)keys[tid];
  if (k < n) {
    typename Lane::Input in;
    in.load(a, k);
    Lane L;
    L.init(a, k, in);
    while (!L.done) L.attempt(a, k);
    L.finish(a, k);
  }
  __syncthreads();  // keys (and the claimed chunk) are reused by the next chunk
}

template <class Lane, int B>
__device__ inline void run_chunked(const LaunchArgs& a) {
  __shared__ uint64_t keys[B];
  __shared__ unsigned int chunk;
  stage_theta(a);
  const int tid = (int)threadIdx.x;
  const int64_t n = work_items(a);
  while (true) {
    if (tid == 0) chunk = (unsigned int)atomicAdd(a.queue, 1ull);
    __syncthreads();
    const int64_t base =
        (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)chunk) * (int64_t)B;
    if (base >= n) break;  // the same for the whole block
    sorted_chunk<Lane, B>(a, base, n, tid, keys);
  }
}

// ---------------------------------------------------------------------------
// Mixed systems: one persistent launch over several groups of trajectories,
// each group an ensemble of its own system in its own arrays.  Every group is
// cut into chunks of B trajectories (a group's last chunk may be short, so no
// chunk holds two systems and no wave mixes them); the chunks of all groups
// form one work queue, drained by a persistent grid through an atomic
// counter as in form 3, or handed out one chunk per block of a grid of
// chunk-count blocks.  A block that finishes a chunk of one system takes the
// next chunk whatever its system, so the groups' uneven work is balanced
// across the whole GPU in a single launch instead of running one launch's
// tail after the other's.  Queue position c belongs to the group g with
// chunk0[g] <= c < chunk0[g + 1] (the host orders the groups).
// `body(sys, a, base, n, tid, keys)` runs one chunk of system `sys` with the
// launch arguments of its group.
// Persistent = false: block b takes queue position b.
template <int B, bool Persistent, class Body>
__device__ inline void run_mixed(const MixedArgs& m, Body&& body) {
  __shared__ uint64_t keys[B];
  __shared__ unsigned int chunk;
  stage_theta(m.c);
  const int tid = (int)threadIdx.x;
  while (true) {
    int64_t c;
    if constexpr (Persistent) {
      if (tid == 0) chunk = (unsigned int)atomicAdd(m.c.queue, 1ull);
      __syncthreads();
      c = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)chunk);
    } else {
      c = (int64_t)blockIdx.x;
    }
    if (c >= m.n_chunks) break;  // the same for the whole block
    int g = 0;
    for (int h = 1; h < m.n_groups; ++h)
      if (c >= m.g[h].chunk0) g = h;
    const int64_t j = c - m.g[g].chunk0;
    const GroupArgs& G = m.g[g];
    LaunchArgs a = m.c;
    a.n = G.n;
    a.in_stride = G.n;
    a.out_stride = G.n;
    a.params = G.params;
    a.u0 = G.u0;
    a.tspan = G.tspan;
    a.tspan_bcast = G.tspan_bcast;
    a.out = G.out;
    a.status = G.status;
    a.stats = G.stats;
    body(G.sys, a, j * B, G.n, tid, keys);
    if constexpr (!Persistent) break;
  }
}

// ---------------------------------------------------------------------------
// Form 0: lane g of G integrates trajectories g, g + G, ... (tpl of them),
// one after another.  A wave stays resident until its slowest lane is done;
// idle lanes are masked off by the SIMT loop.
template <class Lane>
__device__ inline void run_plain(const LaunchArgs& a) {
  stage_theta(a);
  const int64_t G = (int64_t)gridDim.x * blockDim.x;
  const int64_t n = work_items(a);
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int r = 0; r < a.tpl; ++r, k += G) {
    if (k >= n) return;
    typename Lane::Input in;
    in.load(a, k);
    Lane L;
    L.init(a, k, in);
    while (!L.done) L.attempt(a, k);
    L.finish(a, k);
  }
}

// Form 1: a resident grid.  Thread g starts on work item g (< first_queued).
// Each wave keeps a pocket of consecutive ids claimed from the global queue
// kChunk at a time with one atomicAdd (so the one counter sees a few atomics
// per kChunk trajectories, not one per refill).  Whenever at least `refill`
// lanes of a wave are idle, the wave hands them ids from its pocket (ballot +
// popcount + prefix count give each idle lane its rank), claiming a new
// chunk when the pocket runs short.  A wave leaves the loop once the queue
// and its pocket are empty and all its lanes are idle; each lane's work is
// bounded by maxiters attempts, so the grid always drains.
constexpr int64_t kChunk = 128;

template <class Lane>
__device__ inline void run_persistent(const LaunchArgs& a) {
  stage_theta(a);
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  const int64_t n = work_items(a);
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool active = k < n;
  bool queue_empty = a.first_queued >= n;
  int64_t pk_next = 0, pk_end = 0;  // the wave's pocket [pk_next, pk_end)
  Lane L;
  if (active) {
    typename Lane::Input in;
    in.load(a, k);
    L.init(a, k, in);
  }
  while (true) {
    if (active) {
      if (!L.done) L.attempt(a, k);
      if (L.done) {
        L.finish(a, k);
        active = false;
      }
    }
    if (!queue_empty || pk_next < pk_end) {
      const unsigned long long idle = __ballot(!active);
      const int nidle = __popcll(idle);
      if (nidle >= a.refill) {
        const int64_t left = pk_end - pk_next;
        int64_t c0 = 0, c1 = 0;  // newly claimed chunk
        if (left < nidle && !queue_empty) {
          const int leader = __ffsll((long long)idle) - 1;
          unsigned long long got = 0;
          if (lane == leader) got = atomicAdd(a.queue, (unsigned long long)kChunk);
          // read back from the leader lane as a scalar, so that the pocket
          // bounds derived from it stay in scalar registers
          const unsigned long long base =
              ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(got >> 32), leader)
               << 32) |
              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)got, leader);
          c0 = a.first_queued + (int64_t)base;
          c1 = c0 + kChunk < n ? c0 + kChunk : n;
          if (c0 >= n) {
            queue_empty = true;
            c0 = c1 = 0;
          }
        }
        if (!active) {
          const int64_t r = __popcll(idle & below);
          int64_t id = -1;
          if (r < left)
            id = pk_next + r;
          else if (r - left < c1 - c0)
            id = c0 + (r - left);
          if (id >= 0) {
            k = id;
            typename Lane::Input in;
            in.load(a, k);
            L.init(a, k, in);
            active = true;
          }
        }
        if (c1 > c0) {  // leftovers were used up first; keep the rest of the chunk
          const int64_t used = nidle - left;
          pk_next = c0 + (used < c1 - c0 ? used : c1 - c0);
          pk_end = c1;
        } else {
          pk_next += (nidle < left ? nidle : left);
        }
      }
    }
    if (__ballot(active) == 0ull) break;
  }
}

}  // namespace ens
