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
};

template <>
struct Num<double> {
  __device__ static inline double rcp(double x) { return 1.0 / x; }
  __device__ static inline double log2(double x) { return ::log2(x); }
  __device__ static inline double exp2(double x) { return ::exp2(x); }
  __device__ static inline double sqrt(double x) { return ::sqrt(x); }
  __device__ static inline double nan() { return __builtin_nan(""); }
};

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
};

__device__ inline double save_time(const LaunchArgs& a, double t0, double tf, int j) {
  return t0 + a.theta[j] * (tf - t0);
}

__device__ inline double tspan_at(const LaunchArgs& a, int row, int64_t i) {
  return a.tspan_bcast ? a.tspan[row] : a.tspan[row * a.n + i];
}

template <class R>
__device__ inline R load_col(const void* base, int row, int64_t n, int64_t i) {
  return static_cast<const R*>(base)[row * n + i];
}

template <class R>
__device__ inline void store_out(const LaunchArgs& a, int j, int c, int ncomp,
                                 int64_t i, R v) {
  static_cast<R*>(a.out)[((int64_t)j * ncomp + c) * a.n + i] = v;
}

// ---------------------------------------------------------------------------
// Form 0: lane g of G integrates trajectories g, g + G, ... (tpl of them),
// one after another.  A wave stays resident until its slowest lane is done;
// idle lanes are masked off by the SIMT loop.
template <class Lane>
__device__ inline void run_plain(const LaunchArgs& a) {
  const int64_t G = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = 0; k < a.tpl; ++k, i += G) {
    if (i >= a.n) return;
    Lane L;
    L.init(a, i);
    while (!L.done) L.attempt(a, i);
    L.finish(a, i);
  }
}

// Form 1: a resident grid.  Thread g starts on trajectory g (< first_queued);
// whenever at least `refill` lanes of a wave are idle, the wave takes that
// many consecutive ids from the queue with one atomicAdd (ballot + popcount
// + prefix count give each idle lane its id).  Every wave leaves the loop once
// the queue is drained and all its lanes are idle; each lane's work is
// bounded by maxiters attempts, so the grid always drains.
template <class Lane>
__device__ inline void run_persistent(const LaunchArgs& a) {
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool active = i < a.n;
  bool drained = a.first_queued >= a.n;
  Lane L;
  if (active) L.init(a, i);
  while (true) {
    if (active) {
      if (!L.done) L.attempt(a, i);
      if (L.done) {
        L.finish(a, i);
        active = false;
      }
    }
    if (!drained) {
      const unsigned long long idle = __ballot(!active);
      const int nidle = __popcll(idle);
      if (nidle >= a.refill) {
        const int leader = __ffsll((long long)idle) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(a.queue, (unsigned long long)nidle);
        base = __shfl(base, leader);
        const int64_t first = a.first_queued + (int64_t)base;
        if (!active) {
          const int64_t mine = first + __popcll(idle & below);
          if (mine < a.n) {
            i = mine;
            L.init(a, i);
            active = true;
          }
        }
        if (first + nidle >= a.n) drained = true;
      }
    }
    if (__ballot(active) == 0ull) break;
  }
}

}  // namespace ens
