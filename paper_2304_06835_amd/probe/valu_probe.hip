// valu_probe.hip -- issue-rate probe of the vector ALU, the ceiling against
// which the measurement reports the integrators' instruction streams.
//
// Each lane runs 16 independent dependency chains of one instruction class
// (vector-register operands, except the two kinds that measure a literal and
// a scalar-register operand; no memory traffic inside the loop), so the
// measured rate is the issue limit of that class, not its latency.  The
// result is lane-operations per second over the whole device, timed with
// HIP events around one launch after a warm-up launch.  Not part of the
// solver library (libens.so): a separate shared object loaded by the
// benchmark only.
//
// A second probe measures the matrix cores beside the vector unit, the
// ceiling of the fused surrogate kernel's instruction stream: bf16 matrix
// products (v_mfma_f32_16x16x32_bf16 on registers) and SiLU rows (one
// activation per lane: multiply, exp2, add, reciprocal, multiply, and a bf16
// pack per two), alone and one block after the other in the same wave, with
// two waves per SIMD as that kernel runs.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

enum Kind {
  kFmaF32 = 0,   // v_fma_f32
  kAddF32 = 1,   // v_add_f32
  kMulF32 = 2,   // v_mul_f32
  kFmaF64 = 3,   // v_fma_f64
  kExpF32 = 4,   // v_exp_f32 (transcendental unit)
  kMadU64 = 5,   // v_mad_u64_u32 (the Philox multiply)
  kXorB32 = 6,   // v_xor_b32, register operands (integer / logic)
  kFmaLit = 7,   // v_fmac_f32 / v_fmamk_f32 with a 32-bit literal operand
  kFmaSgpr = 8,  // v_fma_f32 with a scalar-register operand
  kKinds = 9
};

constexpr int kChains = 16;

template <int K>
__global__ void __launch_bounds__(256) probe(float* fo, double* dout, uint32_t* uo, int iters,
                                             float s) {
  float x[kChains];
  double xd[kChains / 2];
  uint32_t xu[kChains];
  const float y = s * 1.0001f, z = s * 0.9999f;
  const double yd = (double)s, zd = 0.5 * (double)s;
  const uint32_t ku = 0xD2511F53u ^ (uint32_t)(s * 7.0f), cu = threadIdx.x;
  const uint32_t kv = ku ^ (threadIdx.x * 0x9E3779B9u);  // per lane: a vector register
#pragma unroll
  for (int i = 0; i < kChains; ++i) {
    x[i] = s * (float)(threadIdx.x + i) * 1e-3f;
    xu[i] = threadIdx.x * 2654435761u + i;
  }
#pragma unroll
  for (int i = 0; i < kChains / 2; ++i) xd[i] = (double)x[i];
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
      if (K == kFmaF32) x[i] = __builtin_fmaf(x[i], y, z);
      if (K == kAddF32) x[i] = x[i] + y;
      if (K == kMulF32) x[i] = x[i] * y;
      if (K == kFmaF64 && i < kChains / 2) xd[i] = __builtin_fma(xd[i], yd, zd);
      if (K == kExpF32) x[i] = __builtin_amdgcn_exp2f(x[i]);
      if (K == kMadU64) {
        const uint64_t p = (uint64_t)xu[i] * ku + cu;
        xu[i] = (uint32_t)(p >> 32);
      }
      if (K == kXorB32) xu[i] = xu[i] ^ (kv + (uint32_t)i);
      if (K == kFmaLit) x[i] = __builtin_fmaf(x[i], 1.00013f, z);
      if (K == kFmaSgpr) x[i] = __builtin_fmaf(x[i], s, z);
    }
  }
  float t = 0.0f;
  uint32_t tu = 0u;
  double td = 0.0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) {
    t += x[i];
    tu += xu[i];
  }
#pragma unroll
  for (int i = 0; i < kChains / 2; ++i) td += xd[i];
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  fo[g] = t;
  dout[g] = td;
  uo[g] = tu;
}

template <int K>
hipError_t launch(int blocks, float* f, double* d, uint32_t* u, int iters, hipStream_t st) {
  hipLaunchKernelGGL(probe<K>, dim3((unsigned)blocks), dim3(256), 0, st, f, d, u, iters, 1.0f);
  return hipGetLastError();
}

hipError_t launch_kind(int kind, int blocks, float* f, double* d, uint32_t* u, int iters,
                       hipStream_t st) {
  switch (kind) {
    case kFmaF32: return launch<kFmaF32>(blocks, f, d, u, iters, st);
    case kAddF32: return launch<kAddF32>(blocks, f, d, u, iters, st);
    case kMulF32: return launch<kMulF32>(blocks, f, d, u, iters, st);
    case kFmaF64: return launch<kFmaF64>(blocks, f, d, u, iters, st);
    case kExpF32: return launch<kExpF32>(blocks, f, d, u, iters, st);
    case kMadU64: return launch<kMadU64>(blocks, f, d, u, iters, st);
    case kXorB32: return launch<kXorB32>(blocks, f, d, u, iters, st);
    case kFmaLit: return launch<kFmaLit>(blocks, f, d, u, iters, st);
    case kFmaSgpr: return launch<kFmaSgpr>(blocks, f, d, u, iters, st);
  }
  return hipErrorInvalidValue;
}

// ---- matrix cores beside the vector unit ----------------------------------
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

enum MixKind {
  kMixMfma = 0,  // 24 products per wave-iteration
  kMixSilu = 1,  // 12 SiLU rows per wave-iteration
  kMixBoth = 2,  // 24 products, then 12 SiLU rows (a hidden layer's 2 : 1)
  kMixKinds = 3
};
constexpr int kMixProducts = 24, kMixRows = 12, kMixAcc = 6, kMixBlock = 512;

__device__ inline float mix_silu(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// Products use the packed bf16 activations of the previous iteration as
// their B operand, as a layer consumes the one before; the SiLU chains feed
// themselves.
template <int K>
__global__ void __launch_bounds__(kMixBlock) mix_probe(float* fo, int iters, float s) {
  bf16x8_t w;
  uint32_t pk[4];
#pragma unroll
  for (int i = 0; i < 8; ++i) w[i] = (__bf16)(s * (float)((threadIdx.x * 7 + i * 13) % 97) * 1e-2f);
  f32x4_t acc[kMixAcc];
#pragma unroll
  for (int j = 0; j < kMixAcc; ++j) acc[j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  float x[kMixRows];
#pragma unroll
  for (int i = 0; i < kMixRows; ++i) x[i] = s * (float)(threadIdx.x + 3 * i) * 1e-2f - 2.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) pk[i] = threadIdx.x * 0x9E3779B9u + i;
  uint32_t sink = 0u;
  for (int it = 0; it < iters; ++it) {
    if (K != kMixSilu) {
      bf16x8_t b;
      __builtin_memcpy(&b, pk, sizeof(b));
#pragma unroll
      for (int m = 0; m < kMixProducts; ++m)
        acc[m % kMixAcc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, b, acc[m % kMixAcc], 0, 0, 0);
    }
    if (K != kMixMfma) {
#pragma unroll
      for (int e = 0; e < kMixRows; ++e) x[e] = mix_silu(x[e]);
#pragma unroll
      for (int e = 0; e < kMixRows; e += 2) {
        typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
        const bf16x2_t v = {(__bf16)x[e], (__bf16)x[e + 1]};
        uint32_t u;
        __builtin_memcpy(&u, &v, 4);
        if (K == kMixBoth && e < 8)
          pk[e / 2] = u;
        else
          sink ^= u;
      }
    }
  }
  float t = (float)sink;
#pragma unroll
  for (int j = 0; j < kMixAcc; ++j) t += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
#pragma unroll
  for (int i = 0; i < kMixRows; ++i) t += x[i];
#pragma unroll
  for (int i = 0; i < 4; ++i) t += (float)pk[i];
  fo[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = t;
}

hipError_t launch_mix(int kind, int blocks, float* f, int iters, hipStream_t st) {
  switch (kind) {
    case kMixMfma: hipLaunchKernelGGL(mix_probe<kMixMfma>, dim3((unsigned)blocks), dim3(kMixBlock), 0, st, f, iters, 1.0f); break;
    case kMixSilu: hipLaunchKernelGGL(mix_probe<kMixSilu>, dim3((unsigned)blocks), dim3(kMixBlock), 0, st, f, iters, 1.0f); break;
    case kMixBoth: hipLaunchKernelGGL(mix_probe<kMixBoth>, dim3((unsigned)blocks), dim3(kMixBlock), 0, st, f, iters, 1.0f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

extern "C" {

// Wave-iterations per second, summed over the device, of mix kind `kind`
// (0: 24 bf16 products; 1: 12 SiLU rows; 2: both, the products first) with
// one 512-lane block (two waves per SIMD) per compute unit, written to
// *rate.  Allocates and frees its own buffer and synchronises the device.
// Returns 0, or -1 for a bad argument, -3 for a HIP error.
int mfma_mix_rate(int device, int kind, int iters, double* rate) {
  if (!rate || kind < 0 || kind >= kMixKinds || iters < 1) return -1;
  if (hipSetDevice(device) != hipSuccess) return -3;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      cus < 1)
    return -3;
  const int blocks = cus;
  float* f = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  bool ok = hipMalloc(&f, (size_t)blocks * kMixBlock * sizeof(float)) == hipSuccess &&
            hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
  float ms = 0.0f;
  ok = ok && launch_mix(kind, blocks, f, iters, nullptr) == hipSuccess &&
       hipDeviceSynchronize() == hipSuccess && hipEventRecord(a, nullptr) == hipSuccess &&
       launch_mix(kind, blocks, f, iters, nullptr) == hipSuccess &&
       hipEventRecord(b, nullptr) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
       hipEventElapsedTime(&ms, a, b) == hipSuccess;
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (f) (void)hipFree(f);
  if (!ok || !(ms > 0.0f)) return -3;
  *rate = (double)blocks * (kMixBlock / 64) * (double)iters / ((double)ms * 1e-3);
  return 0;
}

// Lane-operations per second of instruction class `kind` (0 fma_f32, 1
// add_f32, 2 mul_f32, 3 fma_f64, 4 exp_f32, 5 mad_u64_u32, 6 xor_b32, 7
// fma_f32 with a literal, 8 fma_f32 with a scalar register operand) on
// HIP device `device`, written to *rate.  Allocates and frees its own
// buffers (2048 blocks x 256 lanes) and synchronises the device.  Returns 0,
// or -1 for a bad argument, -3 for a HIP error.
int valu_probe_rate(int device, int kind, int iters, double* rate) {
  if (!rate || kind < 0 || kind >= kKinds || iters < 1) return -1;
  if (hipSetDevice(device) != hipSuccess) return -3;
  const int blocks = 2048;
  const size_t lanes = (size_t)blocks * 256;
  float* f = nullptr;
  double* d = nullptr;
  uint32_t* u = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  bool ok = hipMalloc(&f, lanes * sizeof(float)) == hipSuccess &&
            hipMalloc(&d, lanes * sizeof(double)) == hipSuccess &&
            hipMalloc(&u, lanes * sizeof(uint32_t)) == hipSuccess &&
            hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
  float ms = 0.0f;
  ok = ok && launch_kind(kind, blocks, f, d, u, iters, nullptr) == hipSuccess &&
       hipDeviceSynchronize() == hipSuccess && hipEventRecord(a, nullptr) == hipSuccess &&
       launch_kind(kind, blocks, f, d, u, iters, nullptr) == hipSuccess &&
       hipEventRecord(b, nullptr) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
       hipEventElapsedTime(&ms, a, b) == hipSuccess;
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (f) (void)hipFree(f);
  if (d) (void)hipFree(d);
  if (u) (void)hipFree(u);
  if (!ok || !(ms > 0.0f)) return -3;
  const double per_lane = (double)iters * (kind == kFmaF64 ? kChains / 2 : kChains);
  *rate = (double)lanes * per_lane / ((double)ms * 1e-3);
  return 0;
}

}  // extern "C"
