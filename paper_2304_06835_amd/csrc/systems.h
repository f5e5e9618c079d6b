// systems.h -- compile-time right-hand sides and analytic Jacobians of the
// built-in ODE/SDE systems, device side.
//
// Each system is a struct with N (states), M (parameters), f(p, u, du) and
// jac(p, u, J) (J row-major, FP64: the Rosenbrock path factors W in FP64).
// All systems are autonomous, so the df/dt term of the Rosenbrock formula
// (section 3.2.1, eq. 5) vanishes.  Models: appendix of the paper (Lorenz
// problem; Robertson equation; linear SDE; the stiff test problems OREGO and
// HIRES of appendix B.1 -- POLLU, n = 20, lives in pollu.h with its
// cooperative matrix).  Arithmetic uses explicit fma()
// calls and the library is built with -ffp-contract=off, so every launch
// configuration performs bit-identical operations.
#pragma once
#include <hip/hip_runtime.h>
#include "../../include/ens.h"
#include "driver.h"  // Num<R>

namespace ens {

// du = A u, A row-major in p[0..8].
struct Linear {
  static constexpr int kId = ENS_SYS_LINEAR;
  static constexpr int N = 3, M = 9;
  template <class R>
  __device__ static inline void f(const R* p, const R* u, R* du) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
      du[i] = fma(p[3 * i + 2], u[2], fma(p[3 * i + 1], u[1], p[3 * i] * u[0]));
  }
  template <class R>
  __device__ static inline void jac(const R* p, const R*, double* J) {
#pragma unroll
    for (int i = 0; i < 9; ++i) J[i] = (double)p[i];
  }
  static constexpr int kFlopsF = 15;  // 3 x (mul + 2 fma)
};

// Lorenz: (sigma (y - x), x (rho - z) - y, x y - beta z), p = (sigma, rho, beta).
struct Lorenz {
  static constexpr int kId = ENS_SYS_LORENZ;
  static constexpr int N = 3, M = 3;
  template <class R>
  __device__ static inline void f(const R* p, const R* u, R* du) {
    du[0] = p[0] * (u[1] - u[0]);
    du[1] = fma(u[0], p[1] - u[2], -u[1]);
    du[2] = fma(u[0], u[1], -(p[2] * u[2]));
  }
  template <class R>
  __device__ static inline void jac(const R* p, const R* u, double* J) {
    const double s = p[0], r = p[1], b = p[2];
    const double x = u[0], y = u[1], z = u[2];
    J[0] = -s;    J[1] = s;   J[2] = 0.0;
    J[3] = r - z; J[4] = -1;  J[5] = -x;
    J[6] = y;     J[7] = x;   J[8] = -b;
  }
  static constexpr int kFlopsF = 8;
};

// Robertson kinetics, p = (k1, k2, k3):
// (-k1 y1 + k3 y2 y3, k1 y1 - k3 y2 y3 - k2 y2^2, k2 y2^2).
struct Robertson {
  static constexpr int kId = ENS_SYS_ROBERTSON;
  static constexpr int N = 3, M = 3;
  template <class R>
  __device__ static inline void f(const R* p, const R* u, R* du) {
    const R a = p[0] * u[0];          // k1 y1
    const R b = p[2] * u[1] * u[2];   // k3 y2 y3
    const R c = p[1] * u[1] * u[1];   // k2 y2^2
    du[0] = b - a;
    du[1] = (a - b) - c;
    du[2] = c;
  }
  template <class R>
  __device__ static inline void jac(const R* p, const R* u, double* J) {
    const double k1 = p[0], k2 = p[1], k3 = p[2];
    const double y2 = u[1], y3 = u[2];
    J[0] = -k1; J[1] = k3 * y3;                    J[2] = k3 * y2;
    J[3] = k1;  J[4] = -k3 * y3 - 2.0 * k2 * y2;   J[5] = -k3 * y2;
    J[6] = 0.0; J[7] = 2.0 * k2 * y2;              J[8] = 0.0;
  }
  static constexpr int kFlopsF = 10;
};

// Oregonator (appendix B.1, OREGO), p = (k1, k2, k3), with the textbook sign
// of dy1 (the leading minus printed there makes the solution from the printed
// y0 blow up): (k1 (y2 + y1 (1 - k2 y1 - y2)), (y3 - (1 + y1) y2) / k1,
// k3 (y1 - y3)).
struct Orego {
  static constexpr int kId = ENS_SYS_OREGO;
  static constexpr int N = 3, M = 3;
  template <class R>
  __device__ static inline void f(const R* p, const R* u, R* du) {
    const R one = (R)1;
    du[0] = p[0] * (u[1] + u[0] * ((one - p[1] * u[0]) - u[1]));
    // one reciprocal of the lane-constant k1 (shared by the step's inlined
    // calls) instead of a division per call
    du[1] = (u[2] - (one + u[0]) * u[1]) * Num<R>::rcp(p[0]);
    du[2] = p[2] * (u[0] - u[2]);
  }
  template <class R>
  __device__ static inline void jac(const R* p, const R* u, double* J) {
    const double k1 = p[0], k2 = p[1], k3 = p[2];
    const double y1 = u[0], y2 = u[1];
    J[0] = k1 * ((1.0 - 2.0 * k2 * y1) - y2); J[1] = k1 * (1.0 - y1); J[2] = 0.0;
    const double ik1 = 1.0 / k1;
    J[3] = -y2 * ik1;                         J[4] = -(1.0 + y1) * ik1; J[5] = ik1;
    J[6] = k3;                                J[7] = 0.0;              J[8] = -k3;
  }
  static constexpr int kFlopsF = 14;
};

// HIRES (appendix B.1), n = 8, p = its 12 distinct rate constants
// (1.71, 0.43, 8.32, 0.0007, 8.75, 10.03, 0.035, 1.12, 1.745, 280, 0.69,
// 1.81), each standing for every occurrence of its value.
struct Hires {
  static constexpr int kId = ENS_SYS_HIRES;
  static constexpr int N = 8, M = 12;
  template <class R>
  __device__ static inline void f(const R* k, const R* y, R* d) {
    const R r = k[9] * y[5] * y[7];  // 280 y6 y8
    d[0] = fma(k[2], y[2], fma(k[1], y[1], -k[0] * y[0])) + k[3];
    d[1] = fma(k[0], y[0], -k[4] * y[1]);
    d[2] = fma(k[6], y[4], fma(k[1], y[3], -k[5] * y[2]));
    d[3] = fma(k[0], y[2], fma(k[2], y[1], -k[7] * y[3]));
    d[4] = fma(k[1], y[6], fma(k[1], y[5], -k[8] * y[4]));
    d[5] = fma(k[10], y[6], fma(-k[1], y[5], fma(k[0], y[4], fma(k[10], y[3], -r))));
    d[6] = fma(-k[11], y[6], r);
    d[7] = fma(k[11], y[6], -r);
  }
  template <class R>
  __device__ static inline void jac(const R* kr, const R* yr, double* J) {
    double k[12], y6 = yr[5], y8 = yr[7];
#pragma unroll
    for (int i = 0; i < 12; ++i) k[i] = kr[i];
#pragma unroll
    for (int i = 0; i < 64; ++i) J[i] = 0.0;
    J[0] = -k[0];  J[1] = k[1];   J[2] = k[2];
    J[8] = k[0];   J[9] = -k[4];
    J[18] = -k[5]; J[19] = k[1];  J[20] = k[6];
    J[25] = k[2];  J[26] = k[0];  J[27] = -k[7];
    J[36] = -k[8]; J[37] = k[1];  J[38] = k[1];
    J[43] = k[10]; J[44] = k[0];  J[45] = -k[9] * y8 - k[1]; J[46] = k[10]; J[47] = -k[9] * y6;
    J[53] = k[9] * y8;  J[54] = -k[11]; J[55] = k[9] * y6;
    J[61] = -k[9] * y8; J[62] = k[11];  J[63] = -k[9] * y6;
  }
  static constexpr int kFlopsF = 35;
};

}  // namespace ens
