// rodas4.hip -- adaptive Rosenbrock ensemble kernels (GPURodas4 of the paper,
// section 5.2.1), one whole trajectory per lane.
//
// Rosenbrock step (section 3.2.1, eqs. 5-8) in the transformed variables
// U_i = sum_j gamma_ij k_j of Hairer & Wanner (Solving ODEs II, IV.7):
//   W = I/(gamma h) - J   (one analytic Jacobian and one LU per step),
//   W U_i = f(u + sum_{j<i} a_ij U_j) + (1/h) sum_{j<i} C_ij U_j,  i = 1..6,
// stiffly accurate: the 6th stage point is the embedded 3rd-order solution,
// u_new = that point + U_6, and U_6 is the error estimate.
//
// Precision split: FP32 (or FP64) state and stage vectors; the Jacobian, W,
// its LU factorisation with partial pivoting (select-based, no branches) and
// the six triangular solves run in FP64 -- the per-system block-diagonal LU
// of section 5.1.3 (eq. 16), held in registers.
#include <float.h>

#include "../../include/ens.h"
#include "driver.h"
#include "systems.h"

namespace ens {
namespace {

constexpr double kGamma = 0.25;
constexpr double RA[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.544, 0, 0, 0, 0, 0},
    {0.9466785280815826, 0.2557011698983284, 0, 0, 0, 0},
    {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0, 0}};
constexpr double RC[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {-5.6688, 0, 0, 0, 0, 0},
    {-2.430093356833875, -0.2063599157091915, 0, 0, 0, 0},
    {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0, 0},
    {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160, 0, 0},
    {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
     -6.058818238834054, 0}};

// PI control as for Tsit5 with k = 4 (embedded order 3 + 1).
constexpr double kK = 4.0;
constexpr double kEta = 0.9, kFacMin = 0.2, kFacMax = 10.0;
constexpr double kLog2QFloor = -13.287712379549449;  // log2(1e-4)

// In-register LU with partial pivoting of an N x N FP64 matrix.  The row
// interchanges are decided by compares and applied with selects; `swp`
// records them so that solve() replays them on the right-hand side.
template <int N>
struct LU {
  double a[N][N];
  double inv_piv[N];
  bool swp[N][N];

  __device__ inline void factor() {
#pragma unroll
    for (int k = 0; k < N; ++k) {
#pragma unroll
      for (int r = k + 1; r < N; ++r) {
        const bool s = fabs(a[r][k]) > fabs(a[k][k]);
        swp[k][r] = s;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          const double x = a[k][c], y = a[r][c];
          a[k][c] = s ? y : x;
          a[r][c] = s ? x : y;
        }
      }
      inv_piv[k] = 1.0 / a[k][k];
#pragma unroll
      for (int r = k + 1; r < N; ++r) {
        const double l = a[r][k] * inv_piv[k];
        a[r][k] = l;
#pragma unroll
        for (int c = k + 1; c < N; ++c) a[r][c] = fma(-l, a[k][c], a[r][c]);
      }
    }
  }

  __device__ inline void solve(double* x) const {
#pragma unroll
    for (int k = 0; k < N; ++k) {
#pragma unroll
      for (int r = k + 1; r < N; ++r) {
        const double p = x[k], q = x[r];
        x[k] = swp[k][r] ? q : p;
        x[r] = swp[k][r] ? p : q;
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

template <class R, class S>
struct Rodas4Lane {
  static constexpr int N = S::N, M = S::M;
  using Input = LaneInput<R, M, N>;
  R p[M], u[N];
  CompTime t;
  double t0, tf;
  double ts;  // next save time
  R h;
  R hmax;    // tf - t0: no step is longer
  R hfloor;  // 16 eps64 |t|: steps at or below it stop the trajectory (status 2)
  R lqold;
  R* sp;        // out[j][0][col]: where the next save goes
  int j, nacc, nrej, status;
  bool done;

  // Store u at every save time reached; sp walks the [n_save][N][stride]
  // output one save at a time, so a save costs N stores and an add.
  __device__ inline void save_reached(const LaunchArgs& a) {
    while (j < a.n_save && ts <= t.hi + t.lo) {
#pragma unroll
      for (int c = 0; c < N; ++c) sp[c * a.out_stride] = u[c];
      sp += N * a.out_stride;
      ++j;
      if (j < a.n_save) ts = save_time(a, t0, tf, j);
    }
    if (j >= a.n_save) done = true;
  }

  // Starting step when none is given: Hairer-Norsett-Wanner I, II.4 with
  // the order p = 4 (two f calls), capped by the interval length.
  __device__ inline R initial_step(const LaunchArgs& a) {
    double sc[N], d0 = 0, d1 = 0, f0[N], y1[N], f1[N], uu[N];
    R fr[N];
    S::f(p, u, fr);
#pragma unroll
    for (int c = 0; c < N; ++c) {
      uu[c] = (double)u[c];
      f0[c] = (double)fr[c];
      sc[c] = a.atol + a.rtol * fabs(uu[c]);
      d0 += (uu[c] / sc[c]) * (uu[c] / sc[c]);
      d1 += (f0[c] / sc[c]) * (f0[c] / sc[c]);
    }
    d0 = ::sqrt(d0 / N);
    d1 = ::sqrt(d1 / N);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    h0 = fmin(h0, hmax);
    R yr[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      y1[c] = uu[c] + h0 * f0[c];
      yr[c] = (R)y1[c];
    }
    S::f(p, yr, fr);
    double d2 = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      f1[c] = (double)fr[c];
      const double z = (f1[c] - f0[c]) / sc[c];
      d2 += z * z;
    }
    d2 = ::sqrt(d2 / N) / h0;
    const double dm = fmax(d1, d2);
    const double h1 = (dm <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : ::exp2(::log2(0.01 / dm) / 5.0);
    return (R)fmin(fmin(100.0 * h0, h1), hmax);
  }

  __device__ inline void init(const LaunchArgs& a, int64_t k, const Input& in) {
    sp = static_cast<R*>(a.out) + out_col(a, k, in.i);
#pragma unroll
    for (int r = 0; r < M; ++r) p[r] = in.p[r];
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
    h = (a.h0 > 0.0) ? (R)a.h0 : initial_step(a);
    hmax = (R)(tf - t0);
    h = fmin(h, hmax);
    hfloor = (R)(16.0 * DBL_EPSILON) * (R)fabs(t.hi);
    lqold = (R)kLog2QFloor;
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

    // W = I/(gamma h) - J, factored in FP64
    LU<N> W;
    {
      double J[N * N];
      S::jac(p, u, J);
      const double d = 1.0 / (kGamma * (double)he);
#pragma unroll
      for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) W.a[r][c] = (r == c ? d : 0.0) - J[r * N + c];
    }
    W.factor();

    const R inv_h = (R)1 / he;
    R U[6][N], y[N], fy[N];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
#pragma unroll
      for (int c = 0; c < N; ++c) {
        R acc = u[c];
#pragma unroll
        for (int q = 0; q < s; ++q) acc = fma((R)RA[s][q], U[q][c], acc);
        y[c] = acc;
      }
      S::f(p, y, fy);
      double x[N];
#pragma unroll
      for (int c = 0; c < N; ++c) {
        R cs = 0;
#pragma unroll
        for (int q = 0; q < s; ++q) cs = fma((R)RC[s][q], U[q][c], cs);
        x[c] = (double)fma(cs, inv_h, fy[c]);
      }
      W.solve(x);
#pragma unroll
      for (int c = 0; c < N; ++c) U[s][c] = (R)x[c];
    }

    // u_new = 6th stage point + U_6; error estimate U_6
    R unew[N], q2 = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      unew[c] = y[c] + U[5][c];
      const R sc = fma((R)a.rtol, fmax(fabs(u[c]), fabs(unew[c])), (R)a.atol);
      const R r = U[5][c] * F::rcp(sc);
      q2 = fma(r, r, q2);
    }
    q2 = q2 * (R)(1.0 / N);
    if (!(q2 <= (R)3.0e38)) {
      status = ENS_ST_NONFINITE;
      done = true;
      return;
    }
    const R lq = (R)0.5 * F::log2(fmax(q2, (R)1e-20));
    if (q2 <= (R)1) {
      ++nacc;
      if (clamped)
        t.set(ts);
      else
        t.add((double)he);
#pragma unroll
      for (int c = 0; c < N; ++c) u[c] = unew[c];
      R fac = (R)kEta * F::exp2(fma((R)(-0.7 / kK), lq, (R)(0.4 / kK) * lqold));
      fac = fmin((R)kFacMax, fmax((R)kFacMin, fac));
      lqold = fmax(lq, (R)kLog2QFloor);
      R hn = he * fac;
      if (clamped) hn = fmax(hn, h);  // keep the proposal made before the clamp
      h = fmin(hn, hmax);
      hfloor = (R)(16.0 * DBL_EPSILON) * (R)fabs(t.hi);
      if (clamped) {  // only a cut step lands on a save time
        save_reached(a);
        if (done) return;
      }
    } else {
      ++nrej;
      const R fac = fmax((R)kFacMin, (R)kEta * F::exp2((R)(-1.0 / kK) * lq));
      h = he * fac;
    }
    if (!(h > hfloor)) {
      status = ENS_ST_DTMIN;
      done = true;
    }
  }

  __device__ inline void finish(const LaunchArgs& a, int64_t k) {
    for (int jj = j; jj < a.n_save; ++jj, sp += N * a.out_stride)
#pragma unroll
      for (int c = 0; c < N; ++c) sp[c * a.out_stride] = Num<R>::nan();
    if (a.status) a.status[k] = (uint8_t)status;
    if (a.stats) {
      a.stats[k] = nacc;
      a.stats[a.n + k] = nrej;
    }
  }
};

template <class R, class S>
__global__ void __launch_bounds__(kMaxBlock) rodas4_plain(const LaunchArgs a) {
  run_plain<Rodas4Lane<R, S>>(a);
}

template <class R, class S>
__global__ void __launch_bounds__(kMaxBlock) rodas4_persistent(const LaunchArgs a) {
  run_persistent<Rodas4Lane<R, S>>(a);
}

template <class R, class S, int B, int RR>
__global__ void __launch_bounds__(B) rodas4_sorted(const LaunchArgs a) {
  run_sorted<Rodas4Lane<R, S>, B, RR>(a);
}

// Sorted form: block in {256, 512, 1024} x rounds (tpl) in {1, 2, 4}.
template <class R, class S>
void launch_sorted(const LaunchCfg& cfg, const LaunchArgs& a, hipStream_t s) {
  const int rr = a.tpl >= 4 ? 4 : (a.tpl >= 2 ? 2 : 1);
  const int64_t per = (int64_t)cfg.block * rr;
  const dim3 grid((unsigned)((a.n + per - 1) / per)), blk((unsigned)cfg.block);
#define ENS_SORTED(BB, RRR) \
  if (cfg.block == BB && rr == RRR) { hipLaunchKernelGGL((rodas4_sorted<R, S, BB, RRR>), grid, blk, 0, s, a); return; }
  ENS_SORTED(256, 1) ENS_SORTED(256, 2) ENS_SORTED(256, 4)
  ENS_SORTED(512, 1) ENS_SORTED(512, 2) ENS_SORTED(512, 4)
  ENS_SORTED(1024, 1) ENS_SORTED(1024, 2) ENS_SORTED(1024, 4)
#undef ENS_SORTED
}

template <class R, class S>
hipError_t launch_typed(const LaunchCfg& cfg, LaunchArgs a, hipStream_t s) {
  if (cfg.form == 0) {
    const int64_t per_block = (int64_t)cfg.block * a.tpl;
    const int64_t grid = (a.n + per_block - 1) / per_block;
    hipLaunchKernelGGL((rodas4_plain<R, S>), dim3((unsigned)grid), dim3(cfg.block), 0, s, a);
  } else if (cfg.form == 1) {
    hipLaunchKernelGGL((rodas4_persistent<R, S>), dim3((unsigned)cfg.grid), dim3(cfg.block),
                       0, s, a);
  } else {
    launch_sorted<R, S>(cfg, a, s);
  }
  return hipGetLastError();
}

template <class R, class S>
int occupancy_typed(int block) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, rodas4_persistent<R, S>, block, 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <class S>
hipError_t launch_prec(int prec, const LaunchCfg& cfg, LaunchArgs a, hipStream_t s) {
  return prec == 64 ? launch_typed<double, S>(cfg, a, s) : launch_typed<float, S>(cfg, a, s);
}

template <class S>
int occ_prec(int prec, int block) {
  return prec == 64 ? occupancy_typed<double, S>(block) : occupancy_typed<float, S>(block);
}

}  // namespace

hipError_t launch_rodas4(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a, hipStream_t s) {
  switch (sys) {
    case ENS_SYS_ROBERTSON: return launch_prec<Robertson>(prec, cfg, a, s);
    case ENS_SYS_LORENZ: return launch_prec<Lorenz>(prec, cfg, a, s);
    case ENS_SYS_LINEAR: return launch_prec<Linear>(prec, cfg, a, s);
  }
  return hipErrorInvalidValue;
}

int rodas4_blocks_per_cu(int sys, int prec, int block) {
  switch (sys) {
    case ENS_SYS_ROBERTSON: return occ_prec<Robertson>(prec, block);
    case ENS_SYS_LORENZ: return occ_prec<Lorenz>(prec, block);
    default: return occ_prec<Linear>(prec, block);
  }
}

}  // namespace ens
