// pollu.h -- POLLU (appendix B.1: the 20-species, 25-reaction air-pollution
// model of Verwer 1994) as a grouped system: one trajectory per group of 32
// lanes, one component per lane, so the 20 x 20 FP64 matrix W of a
// Rosenbrock step is spread over the group by rows (20 doubles per lane)
// instead of needing 400 doubles in one lane.  At the paper's 8192
// trajectories this also fills the chip: 4096 waves instead of 128.
//
// The right-hand side is the mass-action network read off the paper's
// equations (u_9 and u_16 there read as y9 and y16): reaction j runs at
// r_j = k_j y_a (y_b), and dy_i = sum_j s_ij r_j with s_ij in {-1, 0, 1, 2}
// stored as three species bit masks per reaction.  Every lane gathers the
// group's state through an LDS row, evaluates the 25 rates
// and forms its own component; its row of J follows the same table.
//
// W is inverted cooperatively (section 5.1.3, eq. 16's per-system block,
// here per group) by Gauss-Jordan elimination in place with partial
// pivoting: at step k the group's largest |W_rk| among the rows not yet used
// (lowest lane on ties) is the pivot row; its lane scales it and broadcasts
// it through LDS, and every other row eliminates column k against it and
// keeps the new column in place.  Lane r ends with the row of (P W)^-1 that
// belongs to the step at which it was the pivot, so each of a step's solves
// is one LDS exchange of the right-hand side in pivot order, a 20-term dot
// product per lane and one exchange of the result -- instead of forward and
// back substitutions whose 40 broadcasts each wait for the previous one.
#pragma once
#include <type_traits>

#include "driver.h"
#include "rosenbrock.h"

namespace ens {

constexpr int kGroup = 32;  // lanes per trajectory of a grouped system
constexpr int kGroupMaxDim = 20;

// Per-group LDS rows of the cooperative inverse: the current pivot row, and
// a solve's right-hand side (in pivot order) and result (block of at most
// kMaxBlock threads).
static __shared__ double lds_prow[kMaxBlock / kGroup][kGroupMaxDim];
static __shared__ double lds_rhs[kMaxBlock / kGroup][kGroupMaxDim];
static __shared__ double lds_sol[kMaxBlock / kGroup][kGroupMaxDim];
// Per-group LDS copy of the state, for gathering it in every lane, and the
// trajectory's parameters (lane j holds parameter j and writes it here).
static __shared__ double lds_state[kMaxBlock / kGroup][kGroup];
static __shared__ double lds_param[kMaxBlock / kGroup][kGroup];

// Orders LDS writes of one lane before reads of them by the other lanes of
// the wave (LDS operations of a wave execute in issue order; this keeps the
// compiler from moving them).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ inline int group_slot() { return (int)(threadIdx.x / kGroup); }

// Group reductions and broadcasts within the 32-lane half of a wave.
template <class T>
__device__ inline T group_sum(T x) {
#pragma unroll
  for (int m = kGroup / 2; m >= 1; m >>= 1) x += __shfl_xor(x, m, kGroup);
  return x;  // every lane ends with the same bits (addition commutes)
}
template <class T>
__device__ inline T group_max(T x) {
#pragma unroll
  for (int m = kGroup / 2; m >= 1; m >>= 1) x = fmax(x, __shfl_xor(x, m, kGroup));
  return x;
}
// The same for FP32 values that are not NaN: one shuffle and one median per
// level (an fmax of a shuffled value would first quiet it)
__device__ inline float group_max_f(float x) {
#pragma unroll
  for (int m = kGroup / 2; m >= 1; m >>= 1) x = Num<float>::max(x, __shfl_xor(x, m, kGroup));
  return x;
}
__device__ inline int group_lane() { return (int)(threadIdx.x & (kGroup - 1)); }
// The group's bits of a wave-wide ballot.
__device__ inline uint32_t group_bits(unsigned long long ballot) {
  return (uint32_t)(ballot >> (threadIdx.x & (kWave - kGroup)));
}

// Inputs of a grouped trajectory: lane j loads parameter j (j < NP) into its
// own register and the group's LDS parameter row, and its own component of u0.
template <class R, int NP, int D>
struct GroupInput {
  R p[1], u[1];
  double t0, tf;
  int64_t i;
  __device__ inline void load(const LaunchArgs& a, int64_t k) {
    i = in_col(a, k);
    const int c = group_lane();
    p[0] = c < NP ? load_col<R>(a, a.params, c, i) : (R)0;
    u[0] = c < D ? load_col<R>(a, a.u0, c, i) : (R)0;
    wave_lds_sync();
    lds_param[group_slot()][c] = (double)p[0];
    wave_lds_sync();
    t0 = tspan_at(a, 0, i);
    tf = tspan_at(a, 1, i);
  }
};

// W = alpha I - beta J of a grouped system, inverted cooperatively.
template <class S>
struct GroupW {
  static constexpr int D = S::kDim;
  static_assert(D <= kGroupMaxDim, "group LDS rows hold kGroupMaxDim entries");
  double a[D];  // this lane's row: W, then the row kr of (P W)^-1
  int kr;       // elimination step at which this lane's row was the pivot (D: never)

  template <class R>
  __device__ inline void build(const R* p, const R* u, double alpha, double beta) {
    double row[D];
    S::jac_row(p, u, row);
    const int r = group_lane();
#pragma unroll
    for (int c = 0; c < D; ++c) a[c] = (c == r ? alpha : 0.0) - beta * row[c];
    factor();
  }

  // In-place Gauss-Jordan: with p_k the pivot lane of step k and P the
  // permutation taking row p_k to position k, lane p_k ends holding row k of
  // (P W)^-1, whose entry c is (W^-1)[k][p_c].
  __device__ inline void factor() {
    const int r = group_lane(), g = group_slot();
    bool used = r >= D;  // padding lanes never hold a pivot
    kr = D;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      // a NaN entry counts as the largest, so every step pivots on a row not
      // yet used (kr is a permutation of 0..D-1) and the NaN reaches x
      const double v = fabs(a[k]);
      const double cand = used ? -1.0 : (v == v ? v : __builtin_inf());
      // the maximum of the candidates rounded to FP32 first: rounding keeps
      // order, so the lane of the exact maximum holds it, and when no other
      // lane does, that lane is the pivot; otherwise (ties after rounding)
      // the exact FP64 reduction decides, lowest lane first as before
      const float cf = (float)cand;
      const uint32_t top = group_bits(__ballot(cf == group_max_f(cf)));
      int pk;
      if (__popc(top) == 1) {
        pk = __ffs(top) - 1;
      } else {
        const double m = group_max(cand);
        pk = __ffs(group_bits(__ballot(cand == m))) - 1;
      }
      const bool piv = r == pk;
      if (piv) {  // the pivot row goes to the group's LDS row unscaled
#pragma unroll
        for (int c = 0; c < D; ++c) lds_prow[g][c] = a[c];
        used = true;
        kr = k;
      }
      wave_lds_sync();
      // pivot row: scaled by ip, its column k becomes ip; every other row
      // (above and below, padding rows stay 0): row -= (a_k ip) pivot row,
      // its column k becomes -a_k ip.  Selects, not branches, so the row is
      // not held twice across a divergent update.
      const double ip = recip(lds_prow[g][k]);
      const double l = piv ? 0.0 : a[k] * ip;
      const double sc = piv ? ip : 1.0;
#pragma unroll
      for (int c = 0; c < D; ++c)
        a[c] = c == k ? (piv ? ip : -l) : fma(-l, lds_prow[g][c], a[c] * sc);
      wave_lds_sync();
    }
  }

  __device__ inline bool pivoted() const { return true; }

  // x[0]: this lane's component of the right-hand side in, of the solution
  // out (padding lanes: 0).  x = W^-1 b: slot c of the exchange row gets
  // b_{p_c} (lane r writes b_r at kr), lane r forms x_{kr} from its row, and
  // lane j reads x_j back.
  template <bool>
  __device__ inline void solve(double* x) const {
    const int r = group_lane(), g = group_slot();
    wave_lds_sync();  // earlier readers of the rows have read them
    if (kr < D) lds_rhs[g][kr] = x[0];
    wave_lds_sync();
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) s = fma(a[c], lds_rhs[g][c], s);
    if (kr < D) lds_sol[g][kr] = s;
    wave_lds_sync();
    x[0] = r < D ? lds_sol[g][r] : 0.0;
  }
};

// One POLLU reaction: rate constant k_j, reactants y_a (and y_b when b >= 0),
// and the species it consumes (coefficient -1), produces once (+1) and twice
// (+2), as bit masks over species 0..19.
struct MassAction {
  int a, b;
  uint32_t neg, pos1, pos2;
};

constexpr MassAction kPollu[25] = {
    { 0, -1, 0x00001u, 0x00006u, 0x00000u},  // r1  = k1 y1
    { 1,  3, 0x0000au, 0x00001u, 0x00000u},  // r2  = k2 y2 y4
    { 4,  1, 0x00012u, 0x00021u, 0x00000u},  // r3  = k3 y5 y2
    { 6, -1, 0x00040u, 0x00080u, 0x00010u},  // r4  = k4 y7
    { 6, -1, 0x00040u, 0x00080u, 0x00000u},  // r5  = k5 y7
    { 6,  5, 0x00060u, 0x00090u, 0x00000u},  // r6  = k6 y7 y6
    { 8, -1, 0x00100u, 0x00290u, 0x00000u},  // r7  = k7 y9
    { 8,  5, 0x00120u, 0x00400u, 0x00000u},  // r8  = k8 y9 y6
    {10,  1, 0x00402u, 0x00a01u, 0x00000u},  // r9  = k9 y11 y2
    {10,  0, 0x00401u, 0x01000u, 0x00000u},  // r10 = k10 y11 y1
    {12, -1, 0x01000u, 0x00401u, 0x00000u},  // r11 = k11 y13
    { 9,  1, 0x00202u, 0x02001u, 0x00000u},  // r12 = k12 y10 y2
    {13, -1, 0x02000u, 0x00050u, 0x00000u},  // r13 = k13 y14
    { 0,  5, 0x00021u, 0x04000u, 0x00000u},  // r14 = k14 y1 y6
    { 2, -1, 0x00004u, 0x00008u, 0x00000u},  // r15 = k15 y3
    { 3, -1, 0x00008u, 0x08000u, 0x00000u},  // r16 = k16 y4
    { 3, -1, 0x00008u, 0x00004u, 0x00000u},  // r17 = k17 y4
    {15, -1, 0x08000u, 0x00000u, 0x00020u},  // r18 = k18 y16
    {15, -1, 0x08000u, 0x00004u, 0x00000u},  // r19 = k19 y16
    {16,  5, 0x10020u, 0x20010u, 0x00000u},  // r20 = k20 y17 y6
    {18, -1, 0x40000u, 0x00002u, 0x00000u},  // r21 = k21 y19
    {18, -1, 0x40000u, 0x00005u, 0x00000u},  // r22 = k22 y19
    { 0,  3, 0x00009u, 0x40000u, 0x00000u},  // r23 = k23 y1 y4
    {18,  0, 0x40001u, 0x80000u, 0x00000u},  // r24 = k24 y19 y1
    {19, -1, 0x80000u, 0x40001u, 0x00000u},  // r25 = k25 y20
};

struct Pollu {
  static constexpr bool kGrouped = true;
  // N = 1 component and M = 1 parameter per lane; the 25 rate constants sit
  // in the group's LDS parameter row
  static constexpr int kDim = 20, kParams = 25, N = 1, M = 1;
  template <class R>
  using Input = GroupInput<R, kParams, kDim>;
  template <class R>
  __device__ static inline R rate_constant(int j) {
    return (R)lds_param[group_slot()][j];
  }
  using Matrix = GroupW<Pollu>;
  static constexpr int kFlopsF = 140;  // 25 rates (13 two-factor) + 63 stoichiometric terms x 2

  __device__ static inline int comp() { return group_lane(); }
  template <class T>
  __device__ static inline T sum(T x) { return group_sum(x); }

  // stoichiometric coefficient of this lane's species in reaction j
  template <class T>
  __device__ static inline T coef(int j, int i) {
    const MassAction& r = kPollu[j];
    return (T)(int)(((r.pos1 >> i) & 1u) + 2u * ((r.pos2 >> i) & 1u)) - (T)(int)((r.neg >> i) & 1u);
  }

  // every lane gets the group's whole state (through the group's LDS row:
  // one write per lane, broadcast reads at fixed offsets)
  template <class R>
  __device__ static inline void gather(const R* u, R* y) {
    const int g = group_slot();
    wave_lds_sync();  // earlier readers of the row have read it
    lds_state[g][group_lane()] = (double)u[0];
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < kDim; ++c) y[c] = (R)lds_state[g][c];
  }

  // Every lane forms the whole right-hand side (the stoichiometric table is
  // compile-time, so every term lands in a fixed register) and keeps its own
  // component: no per-lane coefficients to hold.
  template <class R>
  __device__ static inline void f(const R*, const R* u, R* du) {
    R y[kDim], d[kDim];
    gather(u, y);
#pragma unroll
    for (int c = 0; c < kDim; ++c) d[c] = (R)0;
#pragma unroll
    for (int j = 0; j < 25; ++j) {
      R r = rate_constant<R>(j) * y[kPollu[j].a];
      if (kPollu[j].b >= 0) r = r * y[kPollu[j].b];
#pragma unroll
      for (int c = 0; c < kDim; ++c) {
        const int s = (int)((kPollu[j].pos1 >> c) & 1u) + 2 * (int)((kPollu[j].pos2 >> c) & 1u) -
                      (int)((kPollu[j].neg >> c) & 1u);
        if (s != 0) d[c] = fma((R)s, r, d[c]);
      }
    }
    const int i = group_lane();
    R own = (R)0;
#pragma unroll
    for (int c = 0; c < kDim; ++c) own = i == c ? d[c] : own;
    du[0] = own;
  }

  // this lane's row of J = S dr/dy (padding lanes: 0)
  template <class R>
  __device__ static inline void jac_row(const R* k, const R* u, double* row) {
    R yr[kDim];
    gather(u, yr);
    const int i = group_lane();
#pragma unroll
    for (int c = 0; c < kDim; ++c) row[c] = 0.0;
#pragma unroll
    for (int j = 0; j < 25; ++j) {
      const double s = coef<double>(j, i);
      const int ra = kPollu[j].a, rb = kPollu[j].b;
      const double kj = (double)rate_constant<R>(j);
      if (rb >= 0) {
        row[ra] = fma(s, kj * (double)yr[rb], row[ra]);
        row[rb] = fma(s, kj * (double)yr[ra], row[rb]);
      } else {
        row[ra] = fma(s, kj, row[ra]);
      }
    }
  }
};

// Plain form for grouped systems: group g of the grid (kGroup consecutive
// threads) integrates trajectory g.  All lanes of a group take the same
// branches: every decision comes from group-reduced values.
template <class Lane>
__device__ inline void run_grouped(const LaunchArgs& a) {
  stage_theta(a);
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kGroup;
  if (k >= work_items(a)) return;
  typename Lane::Input in;
  in.load(a, k);
  Lane L;
  L.init(a, k, in);
  while (!L.done) L.attempt(a, k);
  L.finish(a, k);
}

// At least two waves per SIMD (256 registers a lane): the step's latency
// chains (group reductions, LDS exchanges) need a second wave to hide them;
// left to itself the compiler takes 268 (FP32) and 308 (FP64) registers
// and one wave.  The cap costs a 32-byte (FP32) and 200-byte (FP64)
// scratch spill, and runs POLLU 1.2-1.4x faster.
template <class R, class S, class M>
__global__ void __launch_bounds__(kMaxBlock, 2) ros_grouped(const LaunchArgs a) {
  run_grouped<RosLane<R, S, M>>(a);
}

// Grouped systems run the plain form only (block of 64, 128 or 256 threads:
// 2, 4 or 8 trajectories).
template <class S, class M>
hipError_t ros_launch_grouped(int prec, const LaunchCfg& cfg, LaunchArgs a, hipStream_t s) {
  const int64_t per_block = cfg.block / kGroup;
  const dim3 grid((unsigned)((a.n + per_block - 1) / per_block)), blk((unsigned)cfg.block);
  if (prec == 64)
    hipLaunchKernelGGL((ros_grouped<double, S, M>), grid, blk, 0, s, a);
  else
    hipLaunchKernelGGL((ros_grouped<float, S, M>), grid, blk, 0, s, a);
  return hipGetLastError();
}

}  // namespace ens
