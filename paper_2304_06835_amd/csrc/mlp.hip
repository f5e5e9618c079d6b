// mlp.hip -- kernels of the learned surrogate: a multilayer perceptron
// (rho, x0, y0, z0) -> 256 -> 256 -> 256 -> 48 with SiLU hidden activations,
// bfloat16 weights and activations, FP32 accumulation on the matrix cores.
//
//   forward   A0 = bf16(X);  Z_l = A_{l-1} W_l^T + b_l;  A_l = bf16(silu(Z_l));
//             Y = A_3 W_4^T + b_4                              (FP32 out)
//   loss      mean over batch and outputs of (Y - T)^2
//   backward  G_4 = 2 (Y - T) / (B 48);  dW_l = bf16(G_l)^T A_{l-1};
//             db_l = sum_batch G_l;  G_{l-1} = (bf16(G_l) W_l) * silu'(Z_{l-1})
//   Adam      Kingma & Ba (2015), Algorithm 1, on FP32 master weights, then
//             a bfloat16 copy of the weights for the next forward pass.
//
// Every matrix product goes through one tiled kernel: 64 x 64 output tile per
// 256-thread block, K in steps of 32 staged through LDS (either operand may
// be stored K-contiguous or K-strided; the staging transposes), and each of
// the four waves issues 2 x 2 v_mfma_f32_16x16x32_bf16 per K step.  Layer
// epilogues (bias, SiLU, bf16 rounding, SiLU', de-normalisation into the
// structure-of-arrays output) are fused into the tile's store.
#include "../../include/ens.h"
#include "ens_internal.h"
#include "mlp.h"
#include "philox.h"

namespace ens {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline float sigmoid(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ inline float silu(float z) { return z * sigmoid(z); }
__device__ inline float dsilu(float z) {
  const float s = sigmoid(z);
  return s * (1.0f + z * (1.0f - s));
}

constexpr int BM = 64, BN = 64, BK = 32, LDW = BK + 8;  // LDS row: 40 bf16 = 80 B

// Stage rows [r0, r0+64) x K [k0, k0+32) of an operand into LDS as [row][k].
// kRowK: element (r, k) at src[r * ld + k]; kKRow: at src[k * ld + r].
template <int LAY>
__device__ inline void stage(uint16_t (*dst)[LDW], const uint16_t* __restrict__ src, int64_t ld,
                             int64_t rows, int64_t K, int64_t r0, int64_t k0, int tid) {
  uint16_t t[8];
  if (LAY == kRowK) {
    const int r = tid >> 2, kk = (tid & 3) * 8;
    const int64_t gr = r0 + r, gk = k0 + kk;
    const uint16_t* p = src + gr * ld + gk;
    if (gr < rows && gk + 8 <= K && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
      *reinterpret_cast<uint4*>(&dst[r][kk]) = *reinterpret_cast<const uint4*>(p);
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] = (gr < rows && gk + e < K) ? p[e] : (uint16_t)0;
#pragma unroll
    for (int e = 0; e < 8; ++e) dst[r][kk + e] = t[e];
  } else {
    const int kk = tid >> 3, r = (tid & 7) * 8;
    const int64_t gk = k0 + kk, gr = r0 + r;
    const uint16_t* p = src + gk * ld + gr;
    if (gk < K && gr + 8 <= rows && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
      const uint4 v = *reinterpret_cast<const uint4*>(p);
      const uint16_t* q = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int e = 0; e < 8; ++e) t[e] = q[e];
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) t[e] = (gk < K && gr + e < rows) ? p[e] : (uint16_t)0;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) dst[r + e][kk] = t[e];
  }
}

// C[M x N] = A[M x K] B[K x N]; A stored per LA, B per LB (with "rows" = N).
// blockIdx.z selects the K range [z kc, min(K, (z+1) kc)) of a split-K
// product; the epilogue sees blockIdx.z and writes that split's partial.
template <int LA, int LB, class Epi>
__global__ void __launch_bounds__(256) gemm_bf16(const uint16_t* __restrict__ A, int64_t lda,
                                                 const uint16_t* __restrict__ B, int64_t ldb,
                                                 int64_t M, int64_t N, int64_t K, int64_t kc,
                                                 Epi epi) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM][LDW];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][LDW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  f32x4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const int64_t kbeg = (int64_t)blockIdx.z * kc;
  const int64_t kend = kbeg + kc < K ? kbeg + kc : K;
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    stage<LA>(As, A, lda, M, kend, m0, k0, tid);
    stage<LB>(Bs, B, ldb, N, kend, n0, k0, tid);
    __syncthreads();
    bf16x8_t af[2], bfr[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      af[t] = *reinterpret_cast<const bf16x8_t*>(&As[wm * 32 + t * 16 + (lane & 15)][(lane >> 4) * 8]);
      bfr[t] = *reinterpret_cast<const bf16x8_t*>(&Bs[wn * 32 + t * 16 + (lane & 15)][(lane >> 4) * 8]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }
  // lane holds D[4*(lane/16) + r][lane % 16] of each 16 x 16 tile
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 32 + a * 16 + (lane >> 4) * 4 + r;
        const int64_t n = n0 + wn * 32 + b * 16 + (lane & 15);
        if (m < M && n < N) epi(m, n, acc[a][b][r]);
      }
}

// ---- epilogues -------------------------------------------------------------
struct EpiHidden {  // Z = acc + b (kept for the backward pass), A = bf16(silu(Z))
  const float* bias;
  float* z;
  uint16_t* act;
  int64_t ld;
  __device__ void operator()(int64_t m, int64_t n, float v) const {
    const float zz = v + bias[n];
    if (z) z[m * ld + n] = zz;
    act[m * ld + n] = f2bf(silu(zz));
  }
};
struct EpiLinear {  // Y = acc + b
  const float* bias;
  float* y;
  int64_t ld;
  __device__ void operator()(int64_t m, int64_t n, float v) const { y[m * ld + n] = v + bias[n]; }
};
struct EpiSoA {  // de-normalised output into out[n][q0 + m] (structure of arrays)
  const float* bias;
  const float* mean;
  const float* stdv;
  float* out;
  int64_t stride, q0;
  __device__ void operator()(int64_t m, int64_t n, float v) const {
    out[n * stride + q0 + m] = fmaf(v + bias[n], stdv[n], mean[n]);
  }
};
struct EpiBack {  // G = acc * silu'(Z), kept in FP32 (bias gradient) and bf16
  const float* z;
  float* g;
  uint16_t* gb;
  int64_t ld;
  __device__ void operator()(int64_t m, int64_t n, float v) const {
    const float gg = v * dsilu(z[m * ld + n]);
    g[m * ld + n] = gg;
    gb[m * ld + n] = f2bf(gg);
  }
};
struct EpiStore {  // partial product of split blockIdx.z at c + z * zstride
  float* c;
  int64_t ld, zstride;
  __device__ void operator()(int64_t m, int64_t n, float v) const {
    c[(int64_t)blockIdx.z * zstride + m * ld + n] = v;
  }
};

// `splits` > 1: K is cut into that many ranges of a multiple of BK each.
template <int LA, int LB, class Epi>
hipError_t gemm(const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, int64_t M,
                int64_t N, int64_t K, Epi epi, hipStream_t s, int splits = 1) {
  if (M <= 0 || N <= 0) return hipSuccess;
  int64_t kc = (K + splits - 1) / splits;
  kc = (kc + BK - 1) / BK * BK;
  const dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)splits);
  hipLaunchKernelGGL((gemm_bf16<LA, LB, Epi>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K,
                     kc, epi);
  return hipGetLastError();
}

// ---- element-wise and reduction kernels ------------------------------------

// He-uniform weights (bound sqrt(6 / fan_in)) from Philox4x32-10 keyed by the
// seed, counter = parameter index; zero biases; then the bf16 copy.
__global__ void init_params(float* w, uint16_t* wb, MlpLayout L, uint64_t seed) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= L.total) return;
  float v = 0.0f;
  for (int l = 0; l < L.layers; ++l) {
    const int64_t wo = L.w_off[l], nw = (int64_t)L.dims[l] * L.dims[l + 1];
    if (p >= wo && p < wo + nw) {
      const Philox4 r = philox4x32_10((uint32_t)p, (uint32_t)((uint64_t)p >> 32), 0u, 0u,
                                      (uint32_t)seed, (uint32_t)(seed >> 32));
      const float u = (float)(r.x0 >> 8) * 0x1p-24f;  // [0, 1)
      v = (2.0f * u - 1.0f) * sqrtf(6.0f / (float)L.dims[l]);
    }
  }
  w[p] = v;
  wb[p] = f2bf(v);
}

__global__ void to_bf16(const float* w, uint16_t* wb, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) wb[p] = f2bf(w[p]);
}

// Adam with bias correction c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t).
__global__ void adam_step(float* w, float* m, float* v, const float* g, uint16_t* wb, int64_t n,
                          float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float gg = g[p];
  const float mm = b1 * m[p] + (1.0f - b1) * gg;
  const float vv = b2 * v[p] + (1.0f - b2) * gg * gg;
  m[p] = mm;
  v[p] = vv;
  const float ww = w[p] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
  w[p] = ww;
  wb[p] = f2bf(ww);
}

// Normalised network inputs of work items [q0, q0 + count): item b is
// trajectory (q0 + b) or, for training, the affine permutation
// (mult * (q0 + b) + add) mod n.  Writes A0 [count][4] bf16 and, when y is
// given, the normalised targets T [count][48].
__global__ void gather_batch(const float* params, const float* u0, const float* y, int64_t n,
                             int64_t q0, int64_t count, uint64_t mult, uint64_t add,
                             const float* norm, uint16_t* a0, float* T, int nout) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= count) return;
  const int64_t i = (int64_t)(((unsigned __int128)mult * (uint64_t)(q0 + b) + add) % (uint64_t)n);
  const float x[4] = {params[n + i], u0[i], u0[n + i], u0[2 * n + i]};  // rho, x0, y0, z0
#pragma unroll
  for (int f = 0; f < 4; ++f) a0[b * 4 + f] = f2bf((x[f] - norm[kInMean + f]) * norm[kInIStd + f]);
  if (y)
    for (int o = 0; o < nout; ++o)
      T[b * nout + o] = (y[(int64_t)o * n + i] - norm[kOutMean + o]) * norm[kOutIStd + o];
}

// G = scale (Y - T) in FP32 and bf16; per-block partial sums of (Y - T)^2.
__global__ void loss_grad(const float* Y, const float* T, float* g, uint16_t* gb, int64_t cnt,
                          float scale, double* partial) {
  __shared__ double red[256];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0.0;
  if (p < cnt) {
    const float d = Y[p] - T[p];
    const float gg = scale * d;
    g[p] = gg;
    gb[p] = f2bf(gg);
    e2 = (double)d * d;
  }
  red[threadIdx.x] = e2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out[0] = factor * sum(partial[0..count)), one block, fixed order.
__global__ void finish_sum(const double* partial, int64_t count, double factor, float* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < count; k += blockDim.x) s += partial[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(factor * red[0]);
}

// part[y][c] = sum of G[r][c] over the y-th range of rows: 64 columns per
// block, four row lanes per column (strided), combined in LDS in a fixed
// order.
__global__ void col_sums(const float* G, int64_t rows, int64_t cols, int64_t rows_per,
                         float* part) {
  __shared__ float red[4][64];
  const int cl = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * 64 + cl;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per;
  const int64_t r1 = r0 + rows_per < rows ? r0 + rows_per : rows;
  float s = 0.0f;
  if (c < cols)
    for (int64_t r = r0 + rl; r < r1; r += 4) s += G[r * cols + c];
  red[rl][cl] = s;
  __syncthreads();
  if (rl == 0 && c < cols)
    part[(int64_t)blockIdx.y * cols + c] = (red[0][cl] + red[1][cl]) + (red[2][cl] + red[3][cl]);
}

// out[i] = sum over z of part[z][i] in increasing z (deterministic).
__global__ void sum_splits(const float* part, int splits, int64_t count, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float s = part[i];
  for (int z = 1; z < splits; ++z) s += part[(int64_t)z * count + i];
  out[i] = s;
}

// Mean, 1/std and std (population, std floored at 1e-6) of `nrows` rows of
// length n, and their min / max; one block per row, FP64 sums in a fixed order.
__global__ void row_stats(RowSet rows, int64_t n, float* mean, float* istd, float* sd, float* lo,
                          float* hi) {
  __shared__ double s1[256], s2[256];
  __shared__ float mn[256], mx[256];
  const int r = blockIdx.x;
  const float* x = rows.ptr[r];
  double a = 0.0, b = 0.0;
  float l = 3.0e38f, h = -3.0e38f;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = x[i];
    a += v;
    b += v * v;
    l = fminf(l, x[i]);
    h = fmaxf(h, x[i]);
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  mn[threadIdx.x] = l;
  mx[threadIdx.x] = h;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      s1[threadIdx.x] += s1[threadIdx.x + st];
      s2[threadIdx.x] += s2[threadIdx.x + st];
      mn[threadIdx.x] = fminf(mn[threadIdx.x], mn[threadIdx.x + st]);
      mx[threadIdx.x] = fmaxf(mx[threadIdx.x], mx[threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mu = s1[0] / (double)n;
    const double var = fmax(s2[0] / (double)n - mu * mu, 0.0);
    mean[r] = (float)mu;
    const double sdev = fmax(sqrt(var), 1e-6);
    istd[r] = (float)(1.0 / sdev);
    if (sd) sd[r] = (float)sdev;
    if (lo) lo[r] = mn[0];
    if (hi) hi[r] = mx[0];
  }
}

}  // namespace

// ---- host launchers --------------------------------------------------------

hipError_t mlp_init(float* w, uint16_t* wb, const MlpLayout& L, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(init_params, dim3((unsigned)((L.total + 255) / 256)), dim3(256), 0, s, w, wb,
                     L, seed);
  return hipGetLastError();
}

hipError_t mlp_to_bf16(const float* w, uint16_t* wb, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, wb, n);
  return hipGetLastError();
}

hipError_t mlp_adam(float* w, float* m, float* v, const float* g, uint16_t* wb, int64_t n,
                    float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(adam_step, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, m, v, g,
                     wb, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_gather(const float* params, const float* u0, const float* y, int64_t n, int64_t q0,
                      int64_t count, uint64_t mult, uint64_t add, const float* norm, uint16_t* a0,
                      float* T, int nout, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_batch, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, params,
                     u0, y, n, q0, count, mult, add, norm, a0, T, nout);
  return hipGetLastError();
}

hipError_t mlp_row_stats(const RowSet& rows, int nrows, int64_t n, float* mean, float* istd,
                         float* sd, float* lo, float* hi, hipStream_t s) {
  hipLaunchKernelGGL(row_stats, dim3((unsigned)nrows), dim3(256), 0, s, rows, n, mean, istd, sd,
                     lo, hi);
  return hipGetLastError();
}

// Forward through all layers for `count` rows already gathered into a0.
// Training (z != null): keeps Z_l and A_l of every hidden layer and writes Y
// [count][48]; inference (soa_out != null): writes the de-normalised outputs
// into soa_out[o][q0 + row] and keeps only two activation buffers.
hipError_t mlp_forward(const MlpLayout& L, const uint16_t* wb, const float* w, const float* norm,
                       const uint16_t* a0, int64_t count, MlpActs& acts, float* Y,
                       float* soa_out, int64_t soa_stride, int64_t q0, hipStream_t s) {
  hipError_t e = hipSuccess;
  const uint16_t* x = a0;
  int64_t ldx = L.dims[0];
  for (int l = 0; l < L.layers; ++l) {
    const int nin = L.dims[l], nout = L.dims[l + 1];
    const uint16_t* W = wb + L.w_off[l];
    const float* b = w + L.b_off[l];
    if (l + 1 < L.layers) {
      uint16_t* a = acts.act[acts.keep_all ? l : (l & 1)];
      float* z = acts.keep_all ? acts.z[l] : nullptr;
      e = gemm<kRowK, kRowK>(x, ldx, W, nin, count, nout, nin, EpiHidden{b, z, a, nout}, s);
      x = a;
      ldx = nout;
    } else if (soa_out) {
      e = gemm<kRowK, kRowK>(x, ldx, W, nin, count, nout, nin,
                             EpiSoA{b, norm + kOutMean, norm + kOutStd, soa_out, soa_stride, q0}, s);
    } else {
      e = gemm<kRowK, kRowK>(x, ldx, W, nin, count, nout, nin, EpiLinear{b, Y, nout}, s);
    }
    if (e != hipSuccess) return e;
  }
  return e;
}

// Loss and gradient of a training batch whose forward pass is in acts / Y.
hipError_t mlp_backward(const MlpLayout& L, const uint16_t* wb, const uint16_t* a0, int64_t B,
                        MlpActs& acts, const float* Y, const float* T, float* grad,
                        double* partial, float* loss, hipStream_t s) {
  const int nl = L.layers;
  const int nout = L.dims[nl];
  const int64_t cnt = B * nout;
  const unsigned nb = (unsigned)((cnt + 255) / 256);
  hipLaunchKernelGGL(loss_grad, dim3(nb), dim3(256), 0, s, Y, T, acts.g[0], acts.gb[0], cnt,
                     (float)(2.0 / (double)cnt), partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (loss) {
    hipLaunchKernelGGL(finish_sum, dim3(1), dim3(256), 0, s, partial, (int64_t)nb,
                       1.0 / (double)cnt, loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  int cur = 0;
  for (int l = nl - 1; l >= 0; --l) {
    const int nin = L.dims[l], no = L.dims[l + 1];
    const uint16_t* prev = l > 0 ? acts.act[l - 1] : a0;
    // dW_l [no][nin] = G^T [no x B] . A_{l-1} [B x nin], K = B cut into
    // kSplits ranges (partials summed in a fixed order)
    const int64_t cnt_w = (int64_t)no * nin;
    e = gemm<kKRow, kKRow>(acts.gb[cur], no, prev, nin, no, nin, B,
                           EpiStore{acts.split, nin, cnt_w}, s, kSplits);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_splits, dim3((unsigned)((cnt_w + 255) / 256)), dim3(256), 0, s,
                       acts.split, kSplits, cnt_w, grad + L.w_off[l]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // db_l = column sums of G
    const int64_t rows_per = (B + kSplits - 1) / kSplits;
    hipLaunchKernelGGL(col_sums, dim3((unsigned)((no + 63) / 64), (unsigned)kSplits), dim3(256), 0,
                       s, acts.g[cur], B, (int64_t)no, rows_per, acts.split);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(sum_splits, dim3((unsigned)((no + 255) / 256)), dim3(256), 0, s, acts.split,
                       kSplits, (int64_t)no, grad + L.b_off[l]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (l > 0) {
      // G_{l-1} [B x nin] = (G [B x no] . W_l [no x nin]) * silu'(Z_{l-1})
      e = gemm<kRowK, kKRow>(acts.gb[cur], no, wb + L.w_off[l], nin, B, nin, no,
                             EpiBack{acts.z[l - 1], acts.g[cur ^ 1], acts.gb[cur ^ 1], nin}, s);
      if (e != hipSuccess) return e;
      cur ^= 1;
    }
  }
  return hipSuccess;
}

}  // namespace ens
