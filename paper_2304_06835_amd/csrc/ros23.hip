// ros23.hip -- adaptive Rosenbrock23 ensemble kernels (GPURosenbrock23 of the
// paper, section 5.2.1), one whole trajectory per lane.
//
// The 2(3) modified Rosenbrock pair of Shampine & Reichelt (SIAM J. Sci.
// Comput. 18, 1997), d = 1/(2 + sqrt 2), e32 = 6 + sqrt 2, W = I - h d J:
//   k1 = W^-1 f(u)
//   F1 = f(u + h k1 / 2),  k2 = W^-1 (F1 - k1) + k1
//   u_new = u + h k2                                     (order 2, L-stable)
//   F2 = f(u_new),         k3 = W^-1 (F2 - e32 (k2 - F1) - 2 (k1 - f(u)))
//   error estimate h (k1 - 2 k2 + k3) / 6                (order-3 companion)
// F2 is the next step's f(u) (first same as last): two f calls, one
// analytic Jacobian, one LU and three solves per step.
//
// Precision split: FP32 (or FP64) state and stage points; the Jacobian, W,
// its LU (partial pivoting, select-based), the three solves, the stage
// vectors k_i and the error combination run in FP64 (k1 - 2 k2 + k3 cancels
// to O(h^2) of |k|, which FP32 stage vectors would swamp at tight rtol).
#include "pollu.h"
#include "rosenbrock.h"
#include "systems.h"

namespace ens {
namespace {

struct Ros23 {
  static constexpr double kK = 3.0;  // PI exponent: embedded order 2 + 1
  static constexpr double kP = 2.0;
  static constexpr bool kFsal = true;
  static constexpr double kD = 0.29289321881345247560;    // 1 / (2 + sqrt 2)
  static constexpr double kE32 = 7.41421356237309504880;  // 6 + sqrt 2

  template <class R, class S>
  __device__ static inline void step(const R* p, const R* u, const R* f0, R he, R* unew, R* err,
                                     R* fnew) {
    constexpr int N = S::N;
    const double hd = (double)he;
    typename WOf<S>::type W;  // I - h d J
    W.build(p, u, 1.0, hd * kD);

    with_pivoting(W, [&](auto piv) {
      constexpr bool P = decltype(piv)::value;
      double k1[N], k2[N], k3[N];
      R y[N], f1[N];
#pragma unroll
      for (int c = 0; c < N; ++c) k1[c] = (double)f0[c];
      W.template solve<P>(k1);
      const R hh = (R)0.5 * he;
#pragma unroll
      for (int c = 0; c < N; ++c) y[c] = fma(hh, (R)k1[c], u[c]);
      S::f(p, y, f1);
#pragma unroll
      for (int c = 0; c < N; ++c) k2[c] = (double)f1[c] - k1[c];
      W.template solve<P>(k2);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        k2[c] += k1[c];
        unew[c] = (R)fma(hd, k2[c], (double)u[c]);
      }
      S::f(p, unew, fnew);
#pragma unroll
      for (int c = 0; c < N; ++c)
        k3[c] = fma(-2.0, k1[c] - (double)f0[c],
                    fma(-kE32, k2[c] - (double)f1[c], (double)fnew[c]));
      W.template solve<P>(k3);
      const double h6 = hd * (1.0 / 6.0);
#pragma unroll
      for (int c = 0; c < N; ++c) err[c] = (R)(h6 * (fma(-2.0, k2[c], k1[c]) + k3[c]));
    });
  }
};

}  // namespace

hipError_t launch_ros23(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a, hipStream_t s) {
  switch (sys) {
    case ENS_SYS_ROBERTSON: return ros_launch_prec<Robertson, Ros23>(prec, cfg, a, s);
    case ENS_SYS_LORENZ: return ros_launch_prec<Lorenz, Ros23>(prec, cfg, a, s);
    case ENS_SYS_LINEAR: return ros_launch_prec<Linear, Ros23>(prec, cfg, a, s);
    case ENS_SYS_OREGO: return ros_launch_prec<Orego, Ros23>(prec, cfg, a, s);
    case ENS_SYS_HIRES: return ros_launch_prec<Hires, Ros23>(prec, cfg, a, s);
    case ENS_SYS_POLLU: return ros_launch_grouped<Pollu, Ros23>(prec, cfg, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_ros23_mixed(int prec, int grid, const MixedArgs& m, hipStream_t s) {
  return ros_launch_mixed<Ros23, Robertson, Orego, Lorenz, Linear>(prec, grid, m, s);
}

int ros23_mixed_blocks(int prec) {
  return ros_mixed_blocks<Ros23, Robertson, Orego, Lorenz, Linear>(prec);
}

int ros23_blocks_per_cu(int sys, int prec, int block, int form, int tpl) {
  switch (sys) {
    case ENS_SYS_ROBERTSON: return ros_occ_prec<Robertson, Ros23>(prec, block, form, tpl);
    case ENS_SYS_LORENZ: return ros_occ_prec<Lorenz, Ros23>(prec, block, form, tpl);
    case ENS_SYS_OREGO: return ros_occ_prec<Orego, Ros23>(prec, block, form, tpl);
    case ENS_SYS_HIRES: return ros_occ_prec<Hires, Ros23>(prec, block, form, tpl);
    default: return ros_occ_prec<Linear, Ros23>(prec, block, form, tpl);
  }
}

}  // namespace ens
