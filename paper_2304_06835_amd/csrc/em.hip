// em.hip -- fixed-step SDE ensemble kernels for dX = a(X) dt + b(X) dW,
// dW ~ N(0, dt) (section 3.3, eq. 11): Euler-Maruyama (GPUEM of section
// 5.2.2) for four independent geometric Brownian motions dX_c = mu X_c dt +
// sigma X_c dW_c (appendix, linear SDE, p = (mu, sigma)) and for the
// sigma-factor CRN (appendix, non-diagonal noise, 8 Wiener processes), and
// a weak order-2 scheme (GPUSIEA) for the GBMs.
//
// Randomness: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), counter
// (step, trajectory low word, trajectory high word, 0) and key = the 64-bit
// seed, so every (trajectory, step) has its own four words whatever the
// launch shape.  Each word's top 23 bits map to the open-interval midpoint
// (2k + 1) 2^-24 (exact in FP32) and Box-Muller turns pairs into N(0,1).
// One lane per trajectory; no divergence: every lane takes the same steps.
#include "../../include/ens.h"
#include "driver.h"
#include "philox.h"

namespace ens {
namespace {

__device__ inline float unit_open(uint32_t x) {
  return (float)(2u * (x >> 9) + 1u) * 0x1p-24f;
}

// (r cos 2 pi v, r sin 2 pi v), r = sqrt(-2 ln u).  The angle is in
// revolutions, which is what the hardware sine and cosine take: one
// instruction each instead of a range-reduced library sincos (measured on
// 2^22 points of (0, 1): max absolute error 1.3e-7 against FP64).  The
// radius also uses the bare hardware log2 and square root,
// r = sqrt(-2 ln 2 log2 u): u lies in [2^-24, 1) and -2 ln u in (0, 33.3],
// never zero, denormal, negative or infinite, so the library functions'
// special-case handling (compares, selects and rescaling) has nothing to do.
__device__ inline void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
  const float r =
      __builtin_amdgcn_sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(unit_open(a)));
  const float v = unit_open(b);
  z0 = r * __builtin_amdgcn_cosf(v);
  z1 = r * __builtin_amdgcn_sinf(v);
}

__global__ void __launch_bounds__(kMaxBlock) em_gbm4(const LaunchArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const float* P = static_cast<const float*>(a.params);
  const float* U0 = static_cast<const float*>(a.u0);
  float* out = static_cast<float*>(a.out);
  const float mu = P[i], sigma = P[a.in_stride + i];
  float X[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) X[c] = U0[c * a.in_stride + i];
  const double t0 = tspan_at(a, 0, i), tf = tspan_at(a, 1, i);
  if (!(tf >= t0) || !isfinite(t0) || !isfinite(tf)) {  // invalid span
    for (int j = 0; j < a.n_save; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) out[((int64_t)j * 4 + c) * a.out_stride + i] = __builtin_nanf("");
    if (a.status) a.status[i] = ENS_ST_NONFINITE;
    return;
  }
  const int64_t nsteps = llround((tf - t0) / a.dt);
  const float h = (float)a.dt;
  const float sqh = (float)::sqrt(a.dt);
  const float muh = mu * h;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const uint32_t ilo = (uint32_t)i, ihi = (uint32_t)((uint64_t)i >> 32);
  int j = 0;
  int64_t next = llround(a.theta[0] * (double)nsteps);
  while (j < a.n_save && next <= 0) {  // saves at t0
#pragma unroll
    for (int c = 0; c < 4; ++c) out[((int64_t)j * 4 + c) * a.out_stride + i] = X[c];
    ++j;
    next = j < a.n_save ? llround(a.theta[j] * (double)nsteps) : -1;
  }
  for (int64_t s = 0; s < nsteps && j < a.n_save; ++s) {
    const Philox4 r = philox4x32_10((uint32_t)s, ilo, ihi, 0u, k0, k1);
    float z[4];
    box_muller(r.x0, r.x1, z[0], z[1]);
    box_muller(r.x2, r.x3, z[2], z[3]);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // X + mu X h + sigma X dW,  dW = sqrt(h) Z
      const float g = fma(sigma * sqh, z[c], muh);
      X[c] = fma(X[c], g, X[c]);
    }
    while (j < a.n_save && s + 1 == next) {
#pragma unroll
      for (int c = 0; c < 4; ++c) out[((int64_t)j * 4 + c) * a.out_stride + i] = X[c];
      ++j;
      next = j < a.n_save ? llround(a.theta[j] * (double)nsteps) : -1;
    }
  }
  if (a.status) a.status[i] = ENS_ST_OK;
  if (a.stats) {
    a.stats[i] = (int32_t)nsteps;
    a.stats[a.n + i] = 0;
  }
}

// ---------------------------------------------------------------------------
// General fixed-step SDE kernel: one lane per trajectory, state in FP32, the
// M Wiener increments of step s drawn from Philox counters (s, id_lo, id_hi,
// c) for c = 0, 1, ... (four normals per call).

// The sigma-factor CRN of the appendix (chemical Langevin equation), state
// (s, A1, A2, A3), p = (S, D, tau, nu0, n, eta), 8 Wiener processes:
//   ds  = (nu0 + H - s) dt + eta sqrt(nu0 + H) dW1 - eta sqrt(s) dW2,
//   dAk = (A(k-1) - Ak)/tau dt + eta sqrt(A(k-1)/tau) dW(2k+1) - eta sqrt(Ak/tau) dW(2k+2)
// with A0 = s and H = (S s)^n / ((S s)^n + (D A3)^n + 1).  A concentration an
// increment drives below zero enters H and the square roots as 0.
struct Crn {
  static constexpr int N = 4, P = 6, NW = 8;
  float S, D, itau, nu0, n, eta;
  __device__ inline void load(const float* p) {
    S = p[0];
    D = p[1];
    itau = 1.0f / p[2];
    nu0 = p[3];
    n = p[4];
    eta = p[5];
  }
  // (x)^n for x >= 0 as 2^(n log2 x); x = 0 gives 0
  __device__ inline float powc(float x) const {
    return __builtin_amdgcn_exp2f(n * __builtin_amdgcn_logf(x));
  }
  // square root of a clamped (>= 0) rate: the bare hardware instruction; the
  // library version's rescaling only matters below 2^-96, where the term it
  // feeds is below 1e-14 of the unit-order drift
  __device__ static inline float rt(float x) { return __builtin_amdgcn_sqrtf(x); }
  // X += a(X) h + b(X) dW, dW = sqrt(h) z
  __device__ inline void em_step(float* X, float h, float sqh, const float* z) const {
    using F = Num<float>;  // the loop-carried state is clamped without quieting
    const float s = F::max(X[0], 0.0f), a1 = F::max(X[1], 0.0f), a2 = F::max(X[2], 0.0f),
                a3 = F::max(X[3], 0.0f);
    const float hs = powc(S * s), hd = powc(D * a3);
    const float H = hs * __builtin_amdgcn_rcpf(hs + hd + 1.0f);  // denominator >= 1
    const float prod = nu0 + H;
    const float es = eta * sqh;
    const float d0 = fma(rt(prod), z[0], -rt(s) * z[1]);
    const float d1 = fma(rt(s * itau), z[2], -rt(a1 * itau) * z[3]);
    const float d2 = fma(rt(a1 * itau), z[4], -rt(a2 * itau) * z[5]);
    const float d3 = fma(rt(a2 * itau), z[6], -rt(a3 * itau) * z[7]);
    const float x0 = X[0], x1 = X[1], x2 = X[2], x3 = X[3];
    X[0] = fma(es, d0, fma(prod - x0, h, x0));
    X[1] = fma(es, d1, fma((x0 - x1) * itau, h, x1));
    X[2] = fma(es, d2, fma((x1 - x2) * itau, h, x2));
    X[3] = fma(es, d3, fma((x2 - x3) * itau, h, x3));
  }
};

// Four GBMs under the weak order-2 scheme (GPUSIEA of section 5.2.2, read
// as Kloeden & Platen's explicit order-2.0 weak scheme, eq. 15.1.1), per
// component with a = mu X, b = sigma X:
//   Ybar = X + a h + b dW,  Y+- = X + a h +- b sqrt(h)
//   X' = X + (a(Ybar) + a) h/2 + (b(Y+) + b(Y-) + 2 b) dW/4
//          + (b(Y+) - b(Y-)) (dW^2 - h) / (4 sqrt h)
struct Gbm4Siea {
  static constexpr int N = 4, P = 2, NW = 4;
  float mu, sigma;
  __device__ inline void load(const float* p) {
    mu = p[0];
    sigma = p[1];
  }
  __device__ inline void em_step(float* X, float h, float sqh, const float* z) const {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float x = X[c], dW = sqh * z[c];
      const float a = mu * x, b = sigma * x;
      const float base = fma(a, h, x);
      const float yb = fma(b, dW, base);
      const float yp = fma(b, sqh, base), ym = fma(-b, sqh, base);
      const float bp = sigma * yp, bm = sigma * ym;
      const float drift = 0.5f * h * (mu * yb + a);
      const float diff = 0.25f * dW * (bp + bm + 2.0f * b);
      // (dW^2 - h) / sqrt(h) = sqrt(h) (z^2 - 1) with dW = sqrt(h) z: no division
      const float fit = 0.25f * (bp - bm) * (sqh * fma(z[c], z[c], -1.0f));
      X[c] = x + drift + diff + fit;
    }
  }
};

template <class Sys>
__global__ void __launch_bounds__(kMaxBlock) sde_fixed(const LaunchArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  constexpr int N = Sys::N;
  const float* P = static_cast<const float*>(a.params);
  const float* U0 = static_cast<const float*>(a.u0);
  float* out = static_cast<float*>(a.out);
  float pv[Sys::P];
#pragma unroll
  for (int r = 0; r < Sys::P; ++r) pv[r] = P[r * a.in_stride + i];
  Sys sys;
  sys.load(pv);
  float X[N];
#pragma unroll
  for (int c = 0; c < N; ++c) X[c] = U0[c * a.in_stride + i];
  const double t0 = tspan_at(a, 0, i), tf = tspan_at(a, 1, i);
  if (!(tf >= t0) || !isfinite(t0) || !isfinite(tf)) {  // invalid span
    for (int j = 0; j < a.n_save; ++j)
#pragma unroll
      for (int c = 0; c < N; ++c) out[((int64_t)j * N + c) * a.out_stride + i] = __builtin_nanf("");
    if (a.status) a.status[i] = ENS_ST_NONFINITE;
    return;
  }
  const int64_t nsteps = llround((tf - t0) / a.dt);
  const float h = (float)a.dt;
  const float sqh = (float)::sqrt(a.dt);
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const uint32_t ilo = (uint32_t)i, ihi = (uint32_t)((uint64_t)i >> 32);
  int j = 0;
  int64_t next = llround(a.theta[0] * (double)nsteps);
  while (j < a.n_save && next <= 0) {  // saves at t0
#pragma unroll
    for (int c = 0; c < N; ++c) out[((int64_t)j * N + c) * a.out_stride + i] = X[c];
    ++j;
    next = j < a.n_save ? llround(a.theta[j] * (double)nsteps) : -1;
  }
  for (int64_t s = 0; s < nsteps && j < a.n_save; ++s) {
    float z[Sys::NW];
#pragma unroll
    for (int call = 0; call < Sys::NW / 4; ++call) {
      const Philox4 r = philox4x32_10((uint32_t)s, ilo, ihi, (uint32_t)call, k0, k1);
      box_muller(r.x0, r.x1, z[4 * call + 0], z[4 * call + 1]);
      box_muller(r.x2, r.x3, z[4 * call + 2], z[4 * call + 3]);
    }
    sys.em_step(X, h, sqh, z);
    while (j < a.n_save && s + 1 == next) {
#pragma unroll
      for (int c = 0; c < N; ++c) out[((int64_t)j * N + c) * a.out_stride + i] = X[c];
      ++j;
      next = j < a.n_save ? llround(a.theta[j] * (double)nsteps) : -1;
    }
  }
  if (a.status) a.status[i] = ENS_ST_OK;
  if (a.stats) {
    a.stats[i] = (int32_t)nsteps;
    a.stats[a.n + i] = 0;
  }
}

__global__ void __launch_bounds__(kMaxBlock)
    philox_fill(uint64_t seed, int64_t n, uint32_t step, uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Philox4 r = philox4x32_10(step, (uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u,
                                  (uint32_t)seed, (uint32_t)(seed >> 32));
  out[i] = r.x0;
  out[n + i] = r.x1;
  out[2 * n + i] = r.x2;
  out[3 * n + i] = r.x3;
}

}  // namespace

hipError_t launch_philox_fill(uint64_t seed, int64_t n, uint32_t step, uint32_t* out,
                              hipStream_t s) {
  const int64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(philox_fill, dim3((unsigned)grid), dim3(256), 0, s, seed, n, step, out);
  return hipGetLastError();
}

hipError_t launch_em(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a, hipStream_t s) {
  if (prec != 32) return hipErrorInvalidValue;
  const int64_t grid = (a.n + cfg.block - 1) / cfg.block;
  if (sys == ENS_SYS_GBM4)
    hipLaunchKernelGGL(em_gbm4, dim3((unsigned)grid), dim3(cfg.block), 0, s, a);
  else if (sys == ENS_SYS_CRN)
    hipLaunchKernelGGL(sde_fixed<Crn>, dim3((unsigned)grid), dim3(cfg.block), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_siea(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a, hipStream_t s) {
  if (prec != 32 || sys != ENS_SYS_GBM4) return hipErrorInvalidValue;
  const int64_t grid = (a.n + cfg.block - 1) / cfg.block;
  hipLaunchKernelGGL(sde_fixed<Gbm4Siea>, dim3((unsigned)grid), dim3(cfg.block), 0, s, a);
  return hipGetLastError();
}

}  // namespace ens
