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
// group's state with cross-lane reads (ds_bpermute), evaluates the 25 rates
// and forms its own component; its row of J follows the same table.
//
// The cooperative LU (section 5.1.3, eq. 16's per-system block, here per
// group) keeps partial pivoting: at step k the group's largest remaining
// |W_rk| (lowest lane on ties) becomes the pivot row, which is broadcast
// from its lane; the other rows eliminate against it and keep their
// multiplier in place.  Solves run the same order: forward through the
// pivots, back through them in reverse, each value broadcast from the lane
// that finalises it.
#pragma once
#include <type_traits>

#include "driver.h"
#include "rosenbrock.h"

namespace ens {

constexpr int kGroup = 32;  // lanes per trajectory of a grouped system

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
__device__ inline int group_lane() { return (int)(threadIdx.x & (kGroup - 1)); }
// The group's bits of a wave-wide ballot.
__device__ inline uint32_t group_bits(unsigned long long ballot) {
  return (uint32_t)(ballot >> (threadIdx.x & (kWave - kGroup)));
}

// Inputs of a grouped trajectory: every lane loads all parameters (each
// evaluates all rates) and its own component of u0.
template <class R, int M, int D>
struct GroupInput {
  R p[M], u[1];
  double t0, tf;
  int64_t i;
  __device__ inline void load(const LaunchArgs& a, int64_t k) {
    i = in_col(a, k);
#pragma unroll
    for (int r = 0; r < M; ++r) p[r] = load_col<R>(a, a.params, r, i);
    const int c = group_lane();
    u[0] = c < D ? load_col<R>(a, a.u0, c, i) : (R)0;
    t0 = tspan_at(a, 0, i);
    tf = tspan_at(a, 1, i);
  }
};

// W = alpha I - beta J of a grouped system, factored cooperatively.
template <class S>
struct GroupW {
  static constexpr int D = S::kDim;
  double a[D];  // this lane's row: W, then its multipliers and U entries
  double inv;   // 1 / pivot of this lane's row
  int kr;       // elimination step at which this lane's row was the pivot (D: never)
  int piv[D];   // group lane holding the pivot row of each step (same in all lanes)

  template <class R>
  __device__ inline void build(const R* p, const R* u, double alpha, double beta) {
    double row[D];
    S::jac_row(p, u, row);
    const int r = group_lane();
#pragma unroll
    for (int c = 0; c < D; ++c) a[c] = (c == r ? alpha : 0.0) - beta * row[c];
    factor();
  }

  __device__ inline void factor() {
    const int r = group_lane();
    bool used = r >= D;  // padding lanes never hold a pivot
    kr = D;
    inv = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double cand = used ? -1.0 : fabs(a[k]);
      const double m = group_max(cand);
      const int pk = __ffs(group_bits(__ballot(cand == m))) - 1;
      piv[k] = pk;
      double prow[D];
#pragma unroll
      for (int c = k; c < D; ++c) prow[c] = __shfl(a[c], pk, kGroup);
      const double ip = recip(prow[k]);
      if (r == pk) {
        used = true;
        kr = k;
        inv = ip;
      } else if (!used) {
        const double l = a[k] * ip;
        a[k] = l;
#pragma unroll
        for (int c = k + 1; c < D; ++c) a[c] = fma(-l, prow[c], a[c]);
      }
    }
  }

  __device__ inline bool pivoted() const { return true; }

  // x[0]: this lane's component of the right-hand side in, of the solution
  // out (padding lanes: 0).
  template <bool>
  __device__ inline void solve(double* x) const {
    const int r = group_lane();
    double b = x[0];
#pragma unroll
    for (int k = 0; k < D; ++k) {  // L z = P b
      const double z = __shfl(b, piv[k], kGroup);
      if (kr > k) b = fma(-a[k], z, b);
    }
    double res = 0.0;
#pragma unroll
    for (int c = D - 1; c >= 0; --c) {  // U x = z, pivot c finalises x_c
      const double v = __shfl(b * inv, piv[c], kGroup);
      if (kr < c) b = fma(-a[c], v, b);
      if (r == c) res = v;
    }
    x[0] = res;
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
  static constexpr int kDim = 20, N = 1, M = 25;
  template <class R>
  using Input = GroupInput<R, M, kDim>;
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

  template <class R>
  __device__ static inline void gather(const R* u, R* y) {
#pragma unroll
    for (int c = 0; c < kDim; ++c) y[c] = __shfl(u[0], c, kGroup);
  }

  template <class R>
  __device__ static inline void f(const R* k, const R* u, R* du) {
    R y[kDim];
    gather(u, y);
    const int i = group_lane();
    R acc = (R)0;
#pragma unroll
    for (int j = 0; j < 25; ++j) {
      R r = k[j] * y[kPollu[j].a];
      if (kPollu[j].b >= 0) r = r * y[kPollu[j].b];
      acc = fma(coef<R>(j, i), r, acc);
    }
    du[0] = acc;
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
      const double kj = (double)k[j];
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

template <class R, class S, class M>
__global__ void __launch_bounds__(kMaxBlock) ros_grouped(const LaunchArgs a) {
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
