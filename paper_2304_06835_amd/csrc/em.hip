// em.hip -- fixed-step Euler-Maruyama ensemble kernel (GPUEM of the paper,
// section 5.2.2) for SDEs dX = a(X) dt + b(X) dW with diagonal noise,
// dW ~ N(0, dt) (section 3.3, eq. 11).  Built-in system: four independent
// geometric Brownian motions dX_c = mu X_c dt + sigma X_c dW_c (appendix,
// linear SDE), p = (mu, sigma).
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
// 2^22 points of (0, 1): max absolute error 1.3e-7 against FP64).
__device__ inline void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
  const float r = sqrtf(-2.0f * logf(unit_open(a)));
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
  if (sys != ENS_SYS_GBM4 || prec != 32) return hipErrorInvalidValue;
  const int64_t grid = (a.n + cfg.block - 1) / cfg.block;
  hipLaunchKernelGGL(em_gbm4, dim3((unsigned)grid), dim3(cfg.block), 0, s, a);
  return hipGetLastError();
}

}  // namespace ens
