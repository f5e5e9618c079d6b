// rosenbrock.h -- what the adaptive Rosenbrock kernels share (section 3.2.1,
// eqs. 5-8; GPURodas4 and GPURosenbrock23 of section 5.2.1): the in-register
// FP64 LU of W (the per-system block of the block-diagonal LU of section
// 5.1.3, eq. 16) and one lane type that runs a whole trajectory -- save-time
// landing, scaled error norm, PI control, status -- around a method's step.
//
// A method M provides
//   kK      the PI exponent k (embedded order + 1)
//   kP      the order used by the starting-step heuristic
//   kFsal   true when the step returns f(u_new) for the next step's f(u)
//   step<R, S>(p, u, f0, h, unew, err, fnew)
//           one step of size h from u (f0 = f(u) when kFsal); writes the
//           propagated solution, the error estimate and (kFsal) f(unew).
#pragma once
#include <float.h>

#include <type_traits>

#include "../../include/ens.h"
#include "driver.h"

namespace ens {

// 1/x from the hardware estimate and two Newton-Raphson steps
// r <- r + r (1 - x r): each step squares the relative error, so the result
// is within an ulp or two of the rounded quotient -- a third of the
// instructions of the IEEE-correct division, whose last-bit rounding an LU
// pivot does not need.  x = 0 or a non-finite x gives a non-finite result.
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// In-register LU with partial pivoting of an N x N FP64 matrix.  Column k
// is pivoted by comparing row k with each row r > k in turn and swapping
// the two (in columns k..N-1) when row r has the larger entry, so row k ends
// up holding the largest.  The swaps are selects (no per-lane branches) recorded in `swp`
// for solve() to replay on the right-hand side.  A swap no lane of the wave
// makes is skipped as a whole (wave-uniform branch on a ballot), and when no
// lane swapped at all (`any` false) the solves take
// their swap-free form -- for the column-diagonally-dominant W of many
// stiff systems (Robertson's among them) that is every factorisation.
template <int N>
struct LU {
  double a[N][N];
  double inv_piv[N];
  bool swp[N][N];
  bool any;  // some lane of the wave swapped rows (wave-uniform)

  __device__ inline void factor() {
    any = false;
#pragma unroll
    for (int k = 0; k < N; ++k) {
#pragma unroll
      for (int r = k + 1; r < N; ++r) {
        const bool s = fabs(a[r][k]) > fabs(a[k][k]);
        swp[k][r] = s;
        if (__ballot(s) != 0ull) {
          any = true;
          // columns < k hold the multipliers of earlier columns, which stay
          // with the row they were computed on: solve() replays this
          // column's swaps on the right-hand side just before eliminating
          // with column k (LINPACK's storage), so they must not move
#pragma unroll
          for (int c = k; c < N; ++c) {
            const double x = a[k][c], y = a[r][c];
            a[k][c] = s ? y : x;
            a[r][c] = s ? x : y;
          }
        }
      }
      inv_piv[k] = recip(a[k][k]);
#pragma unroll
      for (int r = k + 1; r < N; ++r) {
        const double l = a[r][k] * inv_piv[k];
        a[r][k] = l;
#pragma unroll
        for (int c = k + 1; c < N; ++c) a[r][c] = fma(-l, a[k][c], a[r][c]);
      }
    }
  }

  // Solve (LU) x = b in place.  Pivoted = false skips the row swaps: valid
  // only when `any` is 0 (no lane of the wave swapped), which callers test
  // once per factorisation to pick the swap-free copy of their stage code.
  template <bool Pivoted = true>
  __device__ inline void solve(double* x) const {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      if constexpr (Pivoted) {
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
          const double p = x[k], q = x[r];
          x[k] = swp[k][r] ? q : p;
          x[r] = swp[k][r] ? p : q;
        }
      }
#pragma unroll
      for (int r = k + 1; r < N; ++r) x[r] = fma(-a[r][k], x[k], x[r]);
    }
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
      double s = x[k];
#pragma unroll
      for (int c = k + 1; c < N; ++c) s = fma(-a[k][c], x[c], s);
      x[k] = s * inv_piv[k];
    }
  }
};

// W = alpha I - beta J of a system held whole by each lane: analytic FP64
// Jacobian, LU in registers.  Methods build it through this interface
// (build, then solve<Pivoted>), so a system can substitute its own
// (cooperative) matrix type with WOf.
template <class S>
struct LaneW {
  static constexpr int N = S::N;
  LU<N> lu;
  template <class R>
  __device__ inline void build(const R* p, const R* u, double alpha, double beta) {
    double J[N * N];
    S::jac(p, u, J);
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int c = 0; c < N; ++c) lu.a[r][c] = (r == c ? alpha : 0.0) - beta * J[r * N + c];
    lu.factor();
  }
  __device__ inline bool pivoted() const { return lu.any; }
  template <bool Pivoted>
  __device__ inline void solve(double* x) const {
    lu.template solve<Pivoted>(x);
  }
};

// The matrix type a method builds for system S (LaneW unless S names one).
template <class S, class = void>
struct WOf {
  using type = LaneW<S>;
};
template <class S>
struct WOf<S, std::void_t<typename S::Matrix>> {
  using type = typename S::Matrix;
};

// Runs body(std::true_type) when some lane of the wave pivoted, else
// body(std::false_type) -- a wave-uniform choice between two copies of a
// method's stage code, with and without the row swaps in its solves.
template <class WT, class Body>
__device__ inline void with_pivoting(const WT& W, Body&& body) {
  if (W.pivoted())
    body(std::true_type{});
  else
    body(std::false_type{});
}

// How a lane sees its system.  By default a lane holds a whole trajectory
// (all N components).  A grouped system (kGrouped) spreads one trajectory
// over a group of lanes, one component per lane (comp() of them, kDim real
// components, the rest padding): its sums over components are group
// reductions, each lane stores its own component, and one lane of the group
// writes status and counters.
template <class S, class = void>
struct View {
  static constexpr int kDim = S::N;
  template <class R>
  using Input = LaneInput<R, S::M, S::N>;
  __device__ static inline int comp() { return 0; }
  __device__ static inline bool writes() { return true; }
  __device__ static inline bool leader() { return true; }
  template <class T>
  __device__ static inline T sum(T x) { return x; }
};
template <class S>
struct View<S, std::enable_if_t<S::kGrouped>> {
  static constexpr int kDim = S::kDim;
  template <class R>
  using Input = typename S::template Input<R>;
  __device__ static inline int comp() { return S::comp(); }
  __device__ static inline bool writes() { return S::comp() < S::kDim; }
  __device__ static inline bool leader() { return S::comp() == 0; }
  template <class T>
  __device__ static inline T sum(T x) { return S::sum(x); }
};

// PI control (section 3.1, eq. 4) with Hairer & Wanner's constants.
constexpr double kRosEta = 0.9, kRosFacMin = 0.2, kRosFacMax = 10.0;
constexpr double kLog2QFloor = -13.287712379549449;  // log2(1e-4)

template <class R, class S, class M>
struct RosLane {
  using Real = R;
  static constexpr int N = S::N, NP = S::M;
  using V = View<S>;
  using Input = typename V::template Input<R>;
  R p[NP], u[N];
  R f0[M::kFsal ? N : 1];  // f(u), carried from step to step by FSAL methods
  // FP64 time with a compensation term in both precisions (a TwoSum pair of
  // floats measured no faster for Rodas4 and 12% slower for Rosenbrock23's
  // 512-thread sorted form)
  using Time = CompTime;
  Time t;
  double t0, tf;
  double ts;  // next save time
  R h;
  R hmax;    // tf - t0: no step is longer
  R hfloor;  // 16 eps64 |t|: steps at or below it stop the trajectory (status 2)
  R lqold;
  R* sp;        // out[j][0][col]: where the next save goes
  int j, nacc, nrej, status;
  bool done;

  // Store u at every save time reached; sp walks the [n_save][n][stride]
  // output one save at a time, so a save costs N stores and an add.
  __device__ inline void save_reached(const LaunchArgs& a) {
    while (j < a.n_save && t.reached(ts)) {
      if (V::writes()) {
#pragma unroll
        for (int c = 0; c < N; ++c) sp[c * a.out_stride] = u[c];
      }
      sp += V::kDim * a.out_stride;
      ++j;
      if (j < a.n_save) ts = save_time(a, t0, tf, j);
    }
    if (j >= a.n_save) done = true;
  }

  // Starting step when none is given: Hairer-Norsett-Wanner I, II.4 with
  // the method's order (two f calls), capped by the interval length.
  __device__ inline R initial_step(const LaunchArgs& a) {
    double sc[N], d0 = 0, d1 = 0, f0d[N], y1[N], f1[N], uu[N];
    R fr[N];
    S::f(p, u, fr);
#pragma unroll
    for (int c = 0; c < N; ++c) {
      uu[c] = (double)u[c];
      f0d[c] = (double)fr[c];
      sc[c] = a.atol + a.rtol * fabs(uu[c]);
      d0 += (uu[c] / sc[c]) * (uu[c] / sc[c]);
      d1 += (f0d[c] / sc[c]) * (f0d[c] / sc[c]);
    }
    d0 = ::sqrt(V::sum(d0) / V::kDim);
    d1 = ::sqrt(V::sum(d1) / V::kDim);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    h0 = fmin(h0, hmax);
    R yr[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      y1[c] = uu[c] + h0 * f0d[c];
      yr[c] = (R)y1[c];
    }
    S::f(p, yr, fr);
    double d2 = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      f1[c] = (double)fr[c];
      const double z = (f1[c] - f0d[c]) / sc[c];
      d2 += z * z;
    }
    d2 = ::sqrt(V::sum(d2) / V::kDim) / h0;
    const double dm = fmax(d1, d2);
    double h1;
    if (dm <= 1e-15) {
      h1 = fmax(1e-6, h0 * 1e-3);
    } else if constexpr (std::is_same_v<R, float>) {
      // an FP32 lane keeps an FP32 step: the hardware log2 / exp2 suffice, and
      // unlike the FP64 library routines they bring no table of polynomial
      // constants that a loop around the lane would keep in registers
      h1 = (double)Num<float>::exp2(Num<float>::log2((float)(0.01 / dm)) *
                                    (float)(1.0 / (M::kP + 1.0)));
    } else {
      h1 = ::exp2(::log2(0.01 / dm) / (M::kP + 1.0));
    }
    return (R)fmin(fmin(100.0 * h0, h1), hmax);
  }

  __device__ inline void init(const LaunchArgs& a, int64_t k, const Input& in) {
    sp = static_cast<R*>(a.out) + out_col(a, k, in.i) +
         (V::writes() ? (int64_t)V::comp() * a.out_stride : 0);
#pragma unroll
    for (int r = 0; r < NP; ++r) p[r] = in.p[r];
#pragma unroll
    for (int c = 0; c < N; ++c) u[c] = in.u[c];
    t0 = in.t0;
    tf = in.tf;
    t.set(t0);
    j = 0;
    nacc = nrej = 0;
    status = ENS_ST_OK;
    done = false;
    if (!(tf >= t0) || !isfinite(t0) || !isfinite(tf)) {  // invalid span
      status = ENS_ST_NONFINITE;
      done = true;
      return;
    }
    ts = save_time(a, t0, tf, 0);
    save_reached(a);
    if (done) return;
    hmax = (R)(tf - t0);
    h = (a.h0 > 0.0) ? (R)a.h0 : initial_step(a);
    h = fmin(h, hmax);
    hfloor = (R)(16.0 * DBL_EPSILON) * (R)fabs(t.hi);
    lqold = (R)kLog2QFloor;
    if constexpr (M::kFsal) S::f(p, u, f0);
  }

  __device__ inline void attempt(const LaunchArgs& a, int64_t) {
    using F = Num<R>;
    if (nacc + nrej >= (int)a.maxiters) {  // maxiters <= 2e9 (ens_set_option)
      status = ENS_ST_MAXITERS;
      done = true;
      return;
    }
    // distance to the next save time: a longer step is cut to land on it,
    // and one ending within 10% short of it is stretched onto it (after a
    // rejected stretched step h <= 0.9 rem, so the stretch cannot repeat)
    const R rem = (R)t.to(ts);
    const bool clamped = h * (R)kStretch >= rem;
    const R he = clamped ? rem : h;

    R unew[N], err[N], fnew[M::kFsal ? N : 1];
    M::template step<R, S>(p, u, f0, he, unew, err, fnew);

    R q2 = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const R sc = fma((R)a.rtol, F::max(fabs(u[c]), fabs(unew[c])), (R)a.atol);
      const R r = err[c] * F::rcp(sc);
      q2 = fma(r, r, q2);
    }
    q2 = V::sum(q2) * (R)(1.0 / V::kDim);
    if (!(q2 <= (R)3.0e38)) {
      status = ENS_ST_NONFINITE;
      done = true;
      return;
    }
    const R lq = (R)0.5 * F::log2(F::max_nonneg(q2, (R)1e-20));  // q2 >= 0
    if (q2 <= (R)1) {
      ++nacc;
      if (clamped)
        t.set(ts);
      else
        t.add((double)he);
#pragma unroll
      for (int c = 0; c < N; ++c) u[c] = unew[c];
      if constexpr (M::kFsal) {
#pragma unroll
        for (int c = 0; c < N; ++c) f0[c] = fnew[c];
      }
      R fac = (R)kRosEta * F::exp2(fma((R)(-0.7 / M::kK), lq, (R)(0.4 / M::kK) * lqold));
      fac = fmin((R)kRosFacMax, fmax((R)kRosFacMin, fac));
      lqold = fmax(lq, (R)kLog2QFloor);
      R hn = he * fac;
      if (clamped) hn = F::max(hn, h);  // keep the proposal made before the clamp
      h = F::min(hn, hmax);
      hfloor = (R)(16.0 * DBL_EPSILON) * (R)fabs(t.hi);
      if (clamped) {  // only a cut step lands on a save time
        save_reached(a);
        if (done) return;
      }
    } else {
      ++nrej;
      const R fac = fmax((R)kRosFacMin, (R)kRosEta * F::exp2((R)(-1.0 / M::kK) * lq));
      h = he * fac;
    }
    if (!(h > hfloor)) {
      status = ENS_ST_DTMIN;
      done = true;
    }
  }

  __device__ inline void finish(const LaunchArgs& a, int64_t k) {
    if (V::writes())
      for (int jj = j; jj < a.n_save; ++jj, sp += V::kDim * a.out_stride)
#pragma unroll
        for (int c = 0; c < N; ++c) sp[c * a.out_stride] = Num<R>::nan();
    if (!V::leader()) return;
    if (a.status) a.status[k] = (uint8_t)status;
    if (a.stats) {
      a.stats[k] = nacc;
      a.stats[a.n + k] = nrej;
    }
  }
};

// The three work-assignment forms for a Rosenbrock method; a translation
// unit instantiates them with ENS_ROS_LAUNCHERS(M, name).
template <class R, class S, class M>
__global__ void __launch_bounds__(kMaxBlock) ros_plain(const LaunchArgs a) {
  run_plain<RosLane<R, S, M>>(a);
}

template <class R, class S, class M>
__global__ void __launch_bounds__(kMaxBlock) ros_persistent(const LaunchArgs a) {
  run_persistent<RosLane<R, S, M>>(a);
}

template <class R, class S, class M, int B>
__global__ void __launch_bounds__(B) ros_chunked(const LaunchArgs a) {
  run_chunked<RosLane<R, S, M>, B>(a);
}

template <class R, class S, class M, int B, int RR>
__global__ void __launch_bounds__(B) ros_sorted(const LaunchArgs a) {
  run_sorted<RosLane<R, S, M>, B, RR>(a);
}

// Sorted form: block in {256, 512, 1024} x rounds (tpl) in {1, 2, 4}.
template <class R, class S, class M>
void ros_launch_sorted(const LaunchCfg& cfg, const LaunchArgs& a, hipStream_t s) {
  const int rr = a.tpl >= 4 ? 4 : (a.tpl >= 2 ? 2 : 1);
  const int64_t per = (int64_t)cfg.block * rr;
  const dim3 grid((unsigned)((a.n + per - 1) / per)), blk((unsigned)cfg.block);
#define ENS_SORTED(BB, RRR)                                                      \
  if (cfg.block == BB && rr == RRR) {                                            \
    hipLaunchKernelGGL((ros_sorted<R, S, M, BB, RRR>), grid, blk, 0, s, a);      \
    return;                                                                      \
  }
  ENS_SORTED(256, 1) ENS_SORTED(256, 2) ENS_SORTED(256, 4)
  ENS_SORTED(512, 1) ENS_SORTED(512, 2) ENS_SORTED(512, 4)
  ENS_SORTED(1024, 1) ENS_SORTED(1024, 2) ENS_SORTED(1024, 4)
#undef ENS_SORTED
}

template <class R, class S, class M>
hipError_t ros_launch_typed(const LaunchCfg& cfg, LaunchArgs a, hipStream_t s) {
  if (cfg.form == 0) {
    const int64_t per_block = (int64_t)cfg.block * a.tpl;
    const int64_t grid = (a.n + per_block - 1) / per_block;
    hipLaunchKernelGGL((ros_plain<R, S, M>), dim3((unsigned)grid), dim3(cfg.block), 0, s, a);
  } else if (cfg.form == 1) {
    hipLaunchKernelGGL((ros_persistent<R, S, M>), dim3((unsigned)cfg.grid), dim3(cfg.block), 0,
                       s, a);
  } else if (cfg.form == 3) {
    if (cfg.block == 64)
      hipLaunchKernelGGL((ros_chunked<R, S, M, 64>), dim3((unsigned)cfg.grid), dim3(64), 0, s, a);
    else if (cfg.block == 128)
      hipLaunchKernelGGL((ros_chunked<R, S, M, 128>), dim3((unsigned)cfg.grid), dim3(128), 0, s, a);
    else
      hipLaunchKernelGGL((ros_chunked<R, S, M, 256>), dim3((unsigned)cfg.grid), dim3(256), 0, s, a);
  } else {
    ros_launch_sorted<R, S, M>(cfg, a, s);
  }
  return hipGetLastError();
}

template <class R, class S, class M>
int ros_occupancy_typed(int block, int form, int tpl) {
  int nb = 0;
  hipError_t e;
  if (form == 3)
    e = block == 64    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ros_chunked<R, S, M, 64>, 64, 0)
        : block == 128 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ros_chunked<R, S, M, 128>, 128, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ros_chunked<R, S, M, 256>, 256, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ros_persistent<R, S, M>, block, 0);
  if (e != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

// Mixed-system launch (ens_solve_mixed) for a method M over the systems
// whose lanes hold a whole trajectory in three components -- Robertson,
// OREGO, Lorenz, Linear: one kernel holds all four lane types, so its
// registers are the largest of theirs (the eight-component HIRES and the
// grouped POLLU would take them for everyone and are left out).
constexpr int kMixedBlock = 256;

template <class R, class M, class S>
__device__ inline bool mixed_chunk(int sys, int id, const LaunchArgs& a, int64_t base, int64_t n,
                                   int tid, uint64_t* keys) {
  if (sys != id) return false;
  sorted_chunk<RosLane<R, S, M>, kMixedBlock>(a, base, n, tid, keys);
  return true;
}

template <class R, class M, bool P, class S0, class S1, class S2, class S3>
__global__ void __launch_bounds__(kMixedBlock) ros_mixed(const MixedArgs m) {
  run_mixed<kMixedBlock, P>(m, [&](int sys, const LaunchArgs& a, int64_t base, int64_t n, int tid,
                                   uint64_t* keys) {
    mixed_chunk<R, M, S0>(sys, S0::kId, a, base, n, tid, keys) ||
        mixed_chunk<R, M, S1>(sys, S1::kId, a, base, n, tid, keys) ||
        mixed_chunk<R, M, S2>(sys, S2::kId, a, base, n, tid, keys) ||
        mixed_chunk<R, M, S3>(sys, S3::kId, a, base, n, tid, keys);
  });
}

// grid 0: one block per chunk, no queue; otherwise a persistent grid.
template <class M, class S0, class S1, class S2, class S3>
hipError_t ros_launch_mixed(int prec, int grid, const MixedArgs& m, hipStream_t s) {
  const dim3 g((unsigned)(grid > 0 ? grid : m.n_chunks)), b(kMixedBlock);
  if (prec == 64) {
    if (grid > 0)
      hipLaunchKernelGGL((ros_mixed<double, M, true, S0, S1, S2, S3>), g, b, 0, s, m);
    else
      hipLaunchKernelGGL((ros_mixed<double, M, false, S0, S1, S2, S3>), g, b, 0, s, m);
  } else {
    if (grid > 0)
      hipLaunchKernelGGL((ros_mixed<float, M, true, S0, S1, S2, S3>), g, b, 0, s, m);
    else
      hipLaunchKernelGGL((ros_mixed<float, M, false, S0, S1, S2, S3>), g, b, 0, s, m);
  }
  return hipGetLastError();
}

template <class M, class S0, class S1, class S2, class S3>
int ros_mixed_blocks(int prec) {
  int nb = 0;
  const hipError_t e =
      prec == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                       &nb, ros_mixed<double, M, true, S0, S1, S2, S3>, kMixedBlock, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                       &nb, ros_mixed<float, M, true, S0, S1, S2, S3>, kMixedBlock, 0);
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

template <class S, class M>
hipError_t ros_launch_prec(int prec, const LaunchCfg& cfg, LaunchArgs a, hipStream_t s) {
  return prec == 64 ? ros_launch_typed<double, S, M>(cfg, a, s)
                    : ros_launch_typed<float, S, M>(cfg, a, s);
}

template <class S, class M>
int ros_occ_prec(int prec, int block, int form, int tpl) {
  return prec == 64 ? ros_occupancy_typed<double, S, M>(block, form, tpl)
                    : ros_occupancy_typed<float, S, M>(block, form, tpl);
}

}  // namespace ens
