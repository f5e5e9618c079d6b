// rodas.h -- one step of a stiffly accurate Rosenbrock method of the RODAS
// family (section 3.2.1, eqs. 5-8; GPURodas4 and GPURodas5P of section
// 5.2.1) in the transformed variables U_i = sum_j gamma_ij k_j of Hairer &
// Wanner (Solving ODEs II, IV.7):
//   W = I/(gamma h) - J   (one analytic Jacobian and one LU per step),
//   W U_i = f(u + sum_{j<i} a_ij U_j) + (1/h) sum_{j<i} C_ij U_j,
// where the last stage point is the embedded solution: u_new = that point +
// U_s, and U_s is the error estimate.
//
// A tableau T provides kStages, kGamma, a(i, j), c(i, j) (strictly lower),
// the PI exponent kK (embedded order + 1) and the order kP of the solution.
//
// Precision split: FP32 (or FP64) state and stage vectors; the Jacobian, W,
// its LU factorisation with partial pivoting and the triangular solves run in
// FP64 -- the per-system block-diagonal LU of section 5.1.3 (eq. 16), held in
// registers.
#pragma once
#include "rosenbrock.h"

namespace ens {

template <class T>
struct StifflyAccurateRosenbrock {
  static constexpr double kK = T::kK;
  static constexpr double kP = T::kP;
  static constexpr bool kFsal = false;

  template <class R, class S>
  __device__ static inline void step(const R* p, const R* u, const R*, R he, R* unew, R* err,
                                     R*) {
    constexpr int N = S::N, NS = T::kStages;
    // W = I/(gamma h) - J, factored in FP64
    typename WOf<S>::type W;
    W.build(p, u, recip(T::kGamma * (double)he), 1.0);

    const R inv_h = Num<R>::rcp(he);  // FP32: the hardware reciprocal (1 ulp)
    with_pivoting(W, [&](auto piv) {
      constexpr bool P = decltype(piv)::value;
      R U[NS][N], y[N], fy[N];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int c = 0; c < N; ++c) {
          R acc = u[c];
#pragma unroll
          for (int q = 0; q < s; ++q) acc = fma((R)T::a(s, q), U[q][c], acc);
          y[c] = acc;
        }
        S::f(p, y, fy);
        double x[N];
#pragma unroll
        for (int c = 0; c < N; ++c) {
          R cs = 0;
#pragma unroll
          for (int q = 0; q < s; ++q) cs = fma((R)T::c(s, q), U[q][c], cs);
          x[c] = (double)fma(cs, inv_h, fy[c]);
        }
        W.template solve<P>(x);
#pragma unroll
        for (int c = 0; c < N; ++c) U[s][c] = (R)x[c];
      }
      // u_new = last stage point + U_s; error estimate U_s
#pragma unroll
      for (int c = 0; c < N; ++c) {
        unew[c] = y[c] + U[NS - 1][c];
        err[c] = U[NS - 1][c];
      }
    });
  }
};

}  // namespace ens
