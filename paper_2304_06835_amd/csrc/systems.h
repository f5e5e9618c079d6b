// systems.h -- compile-time right-hand sides and analytic Jacobians of the
// built-in ODE/SDE systems, device side.
//
// Each system is a struct with N (states), M (parameters), f(p, u, du) and
// jac(p, u, J) (J row-major, FP64: the Rosenbrock path factors W in FP64).
// All systems are autonomous, so the df/dt term of the Rosenbrock formula
// (section 3.2.1, eq. 5) vanishes.  Models: appendix of the paper (Lorenz
// problem; Robertson equation; linear SDE).  Arithmetic uses explicit fma()
// calls and the library is built with -ffp-contract=off, so every launch
// configuration performs bit-identical operations.
#pragma once
#include <hip/hip_runtime.h>

namespace ens {

// du = A u, A row-major in p[0..8].
struct Linear {
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

}  // namespace ens
