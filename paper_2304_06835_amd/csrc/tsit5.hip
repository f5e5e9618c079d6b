// tsit5.hip -- adaptive Tsitouras 5(4) ensemble kernels (GPUTsit5 of the
// paper, section 5.2.1), one whole trajectory per lane.
//
// Step (section 3.1, eqs. 2-3): k1 = f(u) (first-same-as-last), stage points
// y_i = u + h sum_{j<i} a_ij k_j, k_i = f(y_i) for i = 2..7; the 7th stage
// point is the new solution and k7 its derivative.  Embedded estimate
// E = h sum_j btilde_j k_j, scaled error q = RMS(E / (atol + rtol max(|u|,
// |u_new|))) (eq. 4), accept iff q <= 1, PI control of the step size.
//
// State lives in registers (u, k1..k7, stage point: 27 values for n = 3);
// parameters, initial values and outputs are structure-of-arrays, so a
// wave's 64 lanes read and write 64 consecutive elements.  FP32 variant:
// FP32 state and stages, FP64 time with a TwoSum compensation term, so save
// times are hit exactly however many steps are taken.
#include <float.h>

#include "../../include/ens.h"
#include "driver.h"
#include "systems.h"

namespace ens {
namespace {

// Tsitouras (2011) 5(4) pair.  A is strictly lower triangular; row 7 holds b
// (FSAL).  BT = b - bhat weights the embedded error estimate.
constexpr double TA[7][7] = {
    {0, 0, 0, 0, 0, 0, 0},
    {0.161, 0, 0, 0, 0, 0, 0},
    {-0.008480655492356989, 0.335480655492357, 0, 0, 0, 0, 0},
    {2.897153057105493, -6.359448489975075, 4.3622954328695815, 0, 0, 0, 0},
    {5.325864828439257, -11.748883564062828, 7.4955393428898365,
     -0.09249506636175525, 0, 0, 0},
    {5.86145544294642, -12.92096931784711, 8.159367898576159,
     -0.071584973281401, -0.028269050394068383, 0, 0},
    {0.09646076681806523, 0.01, 0.4798896504144996, 1.379008574103742,
     -3.290069515436081, 2.324710524099774, 0}};
constexpr double BT[7] = {-0.00178001105222577714, -0.0008164344596567469,
                          0.007880878010261995,    -0.1447110071732629,
                          0.5823571654525552,      -0.45808210592918697,
                          0.015151515151515152};

// Dense output, u(t + theta h) = u + h sum_i b_i(theta) k_i with
// b_i(theta) = sum_m TD[i][m] theta^(m+1): the 4th-order C1 continuous
// extension of the pair (every order-<=4 condition for every theta,
// b(1) = b, b'(0) = e_1, b'(1) = e_7), the member of that one-parameter family
// with the least integrated squared order-5 defect.  Section 5.2.1 names this
// "free" interpolation without printing it.
constexpr double TD[7][4] = {
    {1.0, -2.7697190860447156, 2.925281239361705, -1.059101386498926},
    {0.0, 0.12894207915150258, -0.2178841583029839, 0.09894207915151598},
    {0.0, 3.95691789344045, -5.994277185222965, 2.517248942196988},
    {0.0, -12.89991187880857, 31.315858054031978, -17.036937601119686},
    {0.0, 39.47651966255469, -92.1133173868537, 49.346728208862906},
    {0.0, -29.443930585810573, 68.18670326802032, -36.41806215810994},
    {0.0, 1.5511819155171473, -4.102363831034384, 2.55118191551721}};

// PI controller (section 3.1: h_new = eta q_{n-1}^beta2 q_n^beta1 h) with
// Gustafsson's exponents beta1 = -0.7/k, beta2 = 0.4/k, k = 5 (embedded
// order + 1), eta = 0.9, growth clamped to [0.2, 10]; q_{n-1} starts at 1e-4
// and is floored there.  Reject: h *= max(0.2, eta q^(-1/k)).
constexpr double kK = 5.0;
constexpr double kEta = 0.9, kFacMin = 0.2, kFacMax = 10.0, kQFloor = 1e-4;

template <class R, class S>
struct Tsit5Lane {
  using Real = R;
  static constexpr int N = S::N, M = S::M;
  using Input = LaneInput<R, M, N>;
  // FP64 time with a TwoSum compensation term in both precisions (a pair of
  // floats measured no faster for the FP32 lanes: 4.84 against 4.86 ms on
  // the 2^24 headline in the sorted form)
  using Time = CompTime;
  R p[M], u[N], k1[N];
  Time t;
  double t0, tf;
  double ts;     // next save time
  double tland;  // the time steps land on: the next save time, or with dense
                 // output (a.dense) the last one
  R h;
  R hmax;    // tf - t0: no step is longer
  R hfloor;  // 16 eps64 |t|: steps at or below it stop the trajectory (status 2)
  R lqold;  // log2 of the last accepted error proportion
  R* sp;        // out[j][0][col]: where the next save goes
  int64_t os;   // row stride of the save destination
  int j;        // next save index
  int nacc, nrej;
  int status;
  bool done;

  // Store u at every save time reached; sp walks the [n_save][N][os]
  // destination one save at a time, so a save costs N stores and an add.
  __device__ inline void save_reached(const LaunchArgs& a) {
    while (j < a.n_save && t.reached(ts)) {
#pragma unroll
      for (int c = 0; c < N; ++c) sp[c * os] = u[c];
      sp += N * os;
      ++j;
      if (j < a.n_save) ts = save_time(a, t0, tf, j);
    }
    if (j >= a.n_save) done = true;
  }

  // Hairer-Norsett-Wanner I, section II.4 starting step (two f calls, order
  // p = 5), capped by the interval length.  Written on squared norms:
  // d0 = ||u0/sc||, d1 = ||f0/sc||, h0 = 0.01 d0/d1 (1e-6 if either is below
  // 1e-5), d2 = ||(f(u0 + h0 f0) - f0)/sc|| / h0,
  // h1 = (0.01 / max(d1, d2))^(1/6), h = min(100 h0, h1).
  __device__ inline R initial_step(const LaunchArgs& a) {
    using F = Num<R>;
    const R atol = (R)a.atol, rtol = (R)a.rtol;
    const R span = (R)(tf - t0);
    R isc[N], s0 = 0, s1 = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      isc[c] = F::rcp(fma(rtol, fabs(u[c]), atol));
      const R x = u[c] * isc[c], y = k1[c] * isc[c];
      s0 = fma(x, x, s0);
      s1 = fma(y, y, s1);
    }
    const R small = (R)(1e-10 * N);  // d < 1e-5  <=>  s / N < 1e-10
    R h0 = (s0 < small || s1 < small) ? (R)1e-6 : (R)0.01 * F::sqrt(s0 * F::rcp(s1));
    h0 = fmin(h0, span);
    R y1[N], f1[N];
#pragma unroll
    for (int c = 0; c < N; ++c) y1[c] = fma(h0, k1[c], u[c]);
    S::f(p, y1, f1);
    R s2 = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const R z = (f1[c] - k1[c]) * isc[c];
      s2 = fma(z, z, s2);
    }
    const R dm2 = fmax(s1, s2 * F::rcp(h0 * h0)) * (R)(1.0 / N);  // max(d1, d2)^2
    const R h1 = (dm2 <= (R)1e-30)
                     ? fmax((R)1e-6, h0 * (R)1e-3)
                     : F::exp2(((R)-6.643856189774724 - (R)0.5 * F::log2(dm2)) * (R)(1.0 / 6.0));
    return fmin(fmin((R)100 * h0, h1), span);
  }

  __device__ inline void init(const LaunchArgs& a, int64_t k, const Input& in) {
    init_to(a, in, static_cast<R*>(a.out) + out_col(a, k, in.i), a.out_stride);
  }

  // Saves go to dst[(j N + c) stride] instead of the output column (the
  // staged sorted form points dst at the block's LDS rows).
  __device__ inline void init_to(const LaunchArgs& a, const Input& in, R* dst, int64_t stride) {
    sp = dst;
    os = stride;
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
    save_reached(a);  // saves that coincide with t0 (tf == t0)
    tland = a.dense ? save_time(a, t0, tf, a.n_save - 1) : ts;
    if (done) return;
    S::f(p, u, k1);
    h = (a.h0 > 0.0) ? (R)a.h0 : initial_step(a);
    hmax = (R)(tf - t0);
    h = fmin(h, hmax);
    hfloor = (R)(16.0 * DBL_EPSILON) * (R)fabs(t.hi);
    lqold = (R)-13.287712379549449;  // log2(1e-4)
  }

  // Dense output: every save time before the landing time that the accepted
  // step [t, t + he] covers is read off the continuous extension (t, u still
  // hold the step's start).
  __device__ inline void dense_saves(const LaunchArgs& a, R he, const R (&k)[7][N]) {
    using F = Num<R>;
    const R ih = F::rcp(he);
    while (j < a.n_save - 1) {
      const R d = (R)((ts - (double)t.hi) - (double)t.lo);  // FP64: once per save
      if (!(d <= he)) break;
      const R th = d * ih;
      // b_0 = th (1 + th (B01 + th (B02 + th B03))); every other weight has
      // no linear term, b_i = th^2 q_i with q_i = B_i1 + th (B_i2 + th B_i3),
      // so u + he sum b_i k_i = u + (he b_0) k_0 + (he th^2) sum_{i>0} q_i k_i
      static_assert(TD[1][0] == 0.0 && TD[2][0] == 0.0 && TD[3][0] == 0.0 && TD[4][0] == 0.0 &&
                        TD[5][0] == 0.0 && TD[6][0] == 0.0,
                    "the factored form needs b_i(0)' = 0 for i > 0");
      const R hb0 =
          he * (fma(fma(fma((R)TD[0][3], th, (R)TD[0][2]), th, (R)TD[0][1]), th, (R)TD[0][0]) * th);
      const R hth2 = he * (th * th);
      R q[7];
#pragma unroll
      for (int i = 1; i < 7; ++i) q[i] = fma(fma((R)TD[i][3], th, (R)TD[i][2]), th, (R)TD[i][1]);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        R acc = q[1] * k[1][c];
#pragma unroll
        for (int i = 2; i < 7; ++i) acc = fma(q[i], k[i][c], acc);
        sp[c * os] = fma(hth2, acc, fma(hb0, k[0][c], u[c]));
      }
      sp += N * os;
      ++j;
      ts = save_time(a, t0, tf, j);
    }
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
    const R rem = (R)t.to(tland);
    const bool clamped = h * (R)kStretch >= rem;
    const R he = clamped ? rem : h;

    R k[7][N], y[N];
#pragma unroll
    for (int c = 0; c < N; ++c) k[0][c] = k1[c];
#pragma unroll
    for (int s = 1; s < 7; ++s) {
      if (s <= 2) {  // one or two terms: he a_sq once per lane, then one FMA per term
        R ha[2];
#pragma unroll
        for (int q = 0; q < s; ++q) ha[q] = he * (R)TA[s][q];
#pragma unroll
        for (int c = 0; c < N; ++c) {
          y[c] = fma(ha[0], k[0][c], u[c]);
#pragma unroll
          for (int q = 1; q < s; ++q) y[c] = fma(ha[q], k[q][c], y[c]);
        }
      } else {
#pragma unroll
        for (int c = 0; c < N; ++c) {
          R acc = (R)TA[s][0] * k[0][c];
#pragma unroll
          for (int q = 1; q < s; ++q) acc = fma((R)TA[s][q], k[q][c], acc);
          y[c] = fma(he, acc, u[c]);
        }
      }
      S::f(p, y, k[s]);
    }

    // scaled error proportion, squared (avoids a square root); the step size
    // and the mean's 1/N scale the sum once
    R q2 = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      R e = (R)BT[0] * k[0][c];
#pragma unroll
      for (int q = 1; q < 7; ++q) e = fma((R)BT[q], k[q][c], e);
      const R sc = fma((R)a.rtol, F::max(fabs(u[c]), fabs(y[c])), (R)a.atol);
      const R r = e * F::rcp(sc);
      q2 = fma(r, r, q2);
    }
    q2 = q2 * (he * (he * (R)(1.0 / N)));
    if (!(q2 <= (R)3.0e38)) {  // NaN or inf
      status = ENS_ST_NONFINITE;
      done = true;
      return;
    }
    const R lq = (R)0.5 * F::log2(F::max_nonneg(q2, (R)1e-20));  // log2 q (q2 >= 0)
    if (q2 <= (R)1) {
      ++nacc;
      if (a.dense) dense_saves(a, he, k);  // save times inside this step
      if (clamped)
        t.set(tland);
      else
        t.add(he);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        u[c] = y[c];
        k1[c] = k[6][c];
      }
      R fac = (R)kEta * F::exp2(fma((R)(-0.7 / kK), lq, (R)(0.4 / kK) * lqold));
      fac = fmin((R)kFacMax, fmax((R)kFacMin, fac));
      lqold = fmax(lq, (R)-13.287712379549449);
      R hn = he * fac;
      if (clamped) hn = F::max(hn, h);  // keep the proposal made before the clamp
      h = F::min(hn, hmax);
      hfloor = (R)(16.0 * DBL_EPSILON) * (R)fabs(t.hi);
      if (clamped) {  // only a cut step lands on a save time
        save_reached(a);
        if (done) return;
        if (!a.dense) tland = ts;
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
    for (int jj = j; jj < a.n_save; ++jj, sp += N * os)
#pragma unroll
      for (int c = 0; c < N; ++c) sp[c * os] = Num<R>::nan();
    if (a.status) a.status[k] = (uint8_t)status;
    if (a.stats) {
      a.stats[k] = nacc;
      a.stats[a.n + k] = nrej;
    }
  }
};

template <class R, class S>
__global__ void __launch_bounds__(kMaxBlock) tsit5_plain(const LaunchArgs a) {
  run_plain<Tsit5Lane<R, S>>(a);
}

template <class R, class S>
__global__ void __launch_bounds__(kMaxBlock) tsit5_persistent(const LaunchArgs a) {
  run_persistent<Tsit5Lane<R, S>>(a);
}

// FP32 lanes of the chunked form held to five waves per SIMD (96 registers;
// left alone the compiler takes 101, four waves): measured faster than
// holding them to six or seven, where the stage chains lose their overlap
template <class R>
constexpr int kChunkWaves = sizeof(R) == 4 ? 5 : 1;

template <class R, class S, int B>
__global__ void __launch_bounds__(B, kChunkWaves<R>) tsit5_chunked(const LaunchArgs a) {
  run_chunked<Tsit5Lane<R, S>, B>(a);
}

template <class R, class S, int B, int RR, bool Staged>
__global__ void __launch_bounds__(B) tsit5_sorted(const LaunchArgs a) {
  run_sorted<Tsit5Lane<R, S>, B, RR, Staged>(a);
}

// LDS the staged sorted form may take for one block's saves.
constexpr size_t kStageBytes = 64 * 1024;

// Sorted form: block in {256, 512, 1024} x rounds (tpl) in {1, 2, 4}; on
// request (a.stage), block 256 with one round stages its saves in LDS when
// they fit.
template <class R, class S>
void launch_sorted(const LaunchCfg& cfg, const LaunchArgs& a, hipStream_t s) {
  const int rr = a.tpl >= 4 ? 4 : (a.tpl >= 2 ? 2 : 1);
  const int64_t per = (int64_t)cfg.block * rr;
  const dim3 grid((unsigned)((a.n + per - 1) / per)), blk((unsigned)cfg.block);
  const size_t stage = (size_t)a.n_save * S::N * 256 * sizeof(R);
  if (a.stage && cfg.block == 256 && rr == 1 && stage <= kStageBytes) {
    hipLaunchKernelGGL((tsit5_sorted<R, S, 256, 1, true>), grid, blk, stage, s, a);
    return;
  }
#define ENS_SORTED(BB, RRR) \
  if (cfg.block == BB && rr == RRR) { hipLaunchKernelGGL((tsit5_sorted<R, S, BB, RRR, false>), grid, blk, 0, s, a); return; }
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
    hipLaunchKernelGGL((tsit5_plain<R, S>), dim3((unsigned)grid), dim3(cfg.block), 0, s, a);
  } else if (cfg.form == 1) {
    hipLaunchKernelGGL((tsit5_persistent<R, S>), dim3((unsigned)cfg.grid), dim3(cfg.block),
                       0, s, a);
  } else if (cfg.form == 3) {
    if (cfg.block == 64)
      hipLaunchKernelGGL((tsit5_chunked<R, S, 64>), dim3((unsigned)cfg.grid), dim3(64), 0, s, a);
    else if (cfg.block == 128)
      hipLaunchKernelGGL((tsit5_chunked<R, S, 128>), dim3((unsigned)cfg.grid), dim3(128), 0, s, a);
    else
      hipLaunchKernelGGL((tsit5_chunked<R, S, 256>), dim3((unsigned)cfg.grid), dim3(256), 0, s, a);
  } else {
    launch_sorted<R, S>(cfg, a, s);
  }
  return hipGetLastError();
}

template <class R, class S>
int occupancy_typed(int block, int form, int tpl) {
  int nb = 0;
  hipError_t e;
  if (form == 3)
    e = block == 64    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tsit5_chunked<R, S, 64>, 64, 0)
        : block == 128 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tsit5_chunked<R, S, 128>, 128, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tsit5_chunked<R, S, 256>, 256, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tsit5_persistent<R, S>, block, 0);
  if (e != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

// Mixed-system launch (ens_solve_mixed) over the Tsit5 systems.
constexpr int kMixedBlock = 256;

template <class R, bool P>
__global__ void __launch_bounds__(kMixedBlock) tsit5_mixed(const MixedArgs m) {
  run_mixed<kMixedBlock, P>(m, [&](int sys, const LaunchArgs& a, int64_t base, int64_t n, int tid,
                                   uint64_t* keys) {
    if (sys == Lorenz::kId)
      sorted_chunk<Tsit5Lane<R, Lorenz>, kMixedBlock>(a, base, n, tid, keys);
    else
      sorted_chunk<Tsit5Lane<R, Linear>, kMixedBlock>(a, base, n, tid, keys);
  });
}

}  // namespace

// grid 0: one block per chunk, no queue; otherwise a persistent grid.
hipError_t launch_tsit5_mixed(int prec, int grid, const MixedArgs& m, hipStream_t s) {
  const dim3 g((unsigned)(grid > 0 ? grid : m.n_chunks)), b(kMixedBlock);
  if (prec == 64) {
    if (grid > 0)
      hipLaunchKernelGGL((tsit5_mixed<double, true>), g, b, 0, s, m);
    else
      hipLaunchKernelGGL((tsit5_mixed<double, false>), g, b, 0, s, m);
  } else {
    if (grid > 0)
      hipLaunchKernelGGL((tsit5_mixed<float, true>), g, b, 0, s, m);
    else
      hipLaunchKernelGGL((tsit5_mixed<float, false>), g, b, 0, s, m);
  }
  return hipGetLastError();
}

int tsit5_mixed_blocks(int prec) {
  int nb = 0;
  const hipError_t e =
      prec == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tsit5_mixed<double, true>,
                                                                kMixedBlock, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tsit5_mixed<float, true>,
                                                                kMixedBlock, 0);
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_tsit5(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a, hipStream_t s) {
  if (sys == ENS_SYS_LORENZ)
    return prec == 64 ? launch_typed<double, Lorenz>(cfg, a, s)
                      : launch_typed<float, Lorenz>(cfg, a, s);
  if (sys == ENS_SYS_LINEAR)
    return prec == 64 ? launch_typed<double, Linear>(cfg, a, s)
                      : launch_typed<float, Linear>(cfg, a, s);
  return hipErrorInvalidValue;
}

int tsit5_blocks_per_cu(int sys, int prec, int block, int form, int tpl) {
  if (sys == ENS_SYS_LORENZ)
    return prec == 64 ? occupancy_typed<double, Lorenz>(block, form, tpl)
                      : occupancy_typed<float, Lorenz>(block, form, tpl);
  return prec == 64 ? occupancy_typed<double, Linear>(block, form, tpl)
                    : occupancy_typed<float, Linear>(block, form, tpl);
}

}  // namespace ens
