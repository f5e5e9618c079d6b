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
// structure-of-arrays output, the bias gradient's column sums) are fused into
// the tile's store; the weight gradients' split-K partials and the bias
// partials are summed inside the Adam kernel, so a training step on this
// layer-by-layer path is eleven products and three small kernels (gather,
// loss, Adam).  The default training path is the fused one in
// mlp_fused.hip, which shares the Adam kernel.
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

constexpr int BM = 64, BN = 64;
constexpr int KB = 32, LDW = KB + 8;  // K per LDS round; LDS row: 40 bf16 = 80 B
constexpr int kChunks = KB / 32;       // 8-element fragments per thread per operand per round

// One round of an operand tile, rows [r0, r0+64) x K [k0, k0+KB), is 64 x KB
// bf16 = kChunks fragments of 8 per thread.  Fragment c of thread tid:
// kRowK (element (r, k) at src[r * ld + k]): row tid/4, k 8 (tid%4) + 32 c;
// kKRow (element (r, k) at src[k * ld + r]): k tid/8 + 32 c, rows
// 8 (tid%8) .. 8 (tid%8) + 7, so eight consecutive lanes read 128 contiguous
// bytes of one k row.  The load is one 16-byte access where the fragment is
// whole and aligned, element loads with zero fill at the edges.
template <int LAY>
__device__ inline uint4 load_frag(const uint16_t* __restrict__ src, int64_t ld, int64_t rows,
                                  int64_t K, int64_t r0, int64_t k0, int tid, int c) {
  int64_t gr, gk;
  const uint16_t* p;
  bool whole;
  if (LAY == kRowK) {
    gr = r0 + (tid >> 2);
    gk = k0 + (tid & 3) * 8 + 32 * c;
    p = src + gr * ld + gk;
    whole = gr < rows && gk + 8 <= K;
  } else {
    gk = k0 + (tid >> 3) + 32 * c;
    gr = r0 + (tid & 7) * 8;
    p = src + gk * ld + gr;
    whole = gk < K && gr + 8 <= rows;
  }
  if (whole && (reinterpret_cast<uintptr_t>(p) & 15) == 0) return *reinterpret_cast<const uint4*>(p);
  uint16_t t[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const bool in = LAY == kRowK ? (gr < rows && gk + e < K) : (gk < K && gr + e < rows);
    t[e] = in ? p[e] : (uint16_t)0;
  }
  uint4 v;
  uint16_t* q = reinterpret_cast<uint16_t*>(&v);
#pragma unroll
  for (int e = 0; e < 8; ++e) q[e] = t[e];
  return v;
}

// Fragment c of thread tid into the LDS tile dst[row][k] (row stride LDW).
template <int LAY>
__device__ inline void store_frag(uint16_t (*dst)[LDW], uint4 v, int tid, int c) {
  if (LAY == kRowK) {
    *reinterpret_cast<uint4*>(&dst[tid >> 2][(tid & 3) * 8 + 32 * c]) = v;
  } else {
    const uint16_t* q = reinterpret_cast<const uint16_t*>(&v);
    const int kk = (tid >> 3) + 32 * c, r = (tid & 7) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) dst[r + e][kk] = q[e];
  }
}

// One 64 x 64 tile of C[M x N] = A[M x K] B[K x N] over the K range
// [kbeg, kend), rows from m0 and columns from n0; A stored per LA, B per LB
// (with "rows" = N).  K is consumed in rounds of KB through LDS; the next
// round's global loads are issued before the current round's products, so
// they overlap them.  An epilogue with kColSums also receives, per output
// column, the sum over the tile's 64 rows of the values it returned (fixed
// order: rows within a lane, then the four row groups of a wave, then the
// two waves), tagged with the tile's row index `tile_m`.
template <int LA, int LB, class Epi>
__device__ inline void gemm_tile(const uint16_t* __restrict__ A, int64_t lda,
                                 const uint16_t* __restrict__ B, int64_t ldb, int64_t M, int64_t N,
                                 int64_t kbeg, int64_t kend, int64_t m0, int64_t n0, int64_t tile_m,
                                 const Epi& epi) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM][LDW];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][LDW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  f32x4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  uint4 fa[kChunks], fb[kChunks];
  if (kbeg < kend) {
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      fa[c] = load_frag<LA>(A, lda, M, kend, m0, kbeg, tid, c);
      fb[c] = load_frag<LB>(B, ldb, N, kend, n0, kbeg, tid, c);
    }
  }
  for (int64_t k0 = kbeg; k0 < kend; k0 += KB) {
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      store_frag<LA>(As, fa[c], tid, c);
      store_frag<LB>(Bs, fb[c], tid, c);
    }
    __syncthreads();
    if (k0 + KB < kend) {
#pragma unroll
      for (int c = 0; c < kChunks; ++c) {
        fa[c] = load_frag<LA>(A, lda, M, kend, m0, k0 + KB, tid, c);
        fb[c] = load_frag<LB>(B, ldb, N, kend, n0, k0 + KB, tid, c);
      }
    }
#pragma unroll
    for (int ks = 0; ks < KB; ks += 32) {
      bf16x8_t af[2], bfr[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        af[t] = *reinterpret_cast<const bf16x8_t*>(
            &As[wm * 32 + t * 16 + (lane & 15)][ks + (lane >> 4) * 8]);
        bfr[t] = *reinterpret_cast<const bf16x8_t*>(
            &Bs[wn * 32 + t * 16 + (lane & 15)][ks + (lane >> 4) * 8]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // lane holds D[4*(lane/16) + r][lane % 16] of each 16 x 16 tile
  float cs[2] = {0.0f, 0.0f};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 32 + a * 16 + (lane >> 4) * 4 + r;
        const int64_t n = n0 + wn * 32 + b * 16 + (lane & 15);
        if (m < M && n < N) cs[b] += epi(m, n, acc[a][b][r]);
      }
  if constexpr (Epi::kColSums) {
    __shared__ float red[2][BN];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      float v = cs[b];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (lane < 16) red[wm][wn * 32 + b * 16 + lane] = v;
    }
    __syncthreads();
    if (tid < BN && n0 + tid < N) epi.colsum(tile_m, n0 + tid, red[0][tid] + red[1][tid]);
  }
}

// Grid-mapped product: blockIdx.x / .y pick the column / row tile, and
// blockIdx.z the K range [z kc, min(K, (z+1) kc)) of a split-K product.
template <int LA, int LB, class Epi>
__global__ void __launch_bounds__(256) gemm_bf16(const uint16_t* __restrict__ A, int64_t lda,
                                                 const uint16_t* __restrict__ B, int64_t ldb,
                                                 int64_t M, int64_t N, int64_t K, int64_t kc,
                                                 Epi epi) {
  const int64_t kbeg = (int64_t)blockIdx.z * kc;
  const int64_t kend = kbeg + kc < K ? kbeg + kc : K;
  epi.split = blockIdx.z;
  gemm_tile<LA, LB>(A, lda, B, ldb, M, N, kbeg, kend, (int64_t)blockIdx.y * BM,
                    (int64_t)blockIdx.x * BN, blockIdx.y, epi);
}

// ---- epilogues -------------------------------------------------------------
// operator() stores one output element and returns the value whose column
// sums an epilogue with kColSums receives through colsum().
struct EpiHidden {  // Z = acc + b (kept for the backward pass), A = bf16(silu(Z))
  static constexpr bool kColSums = false;
  const float* bias;
  float* z;
  uint16_t* act;
  int64_t ld;
  int split = 0;  // K range of a split-K product (set by the kernel)
  __device__ float operator()(int64_t m, int64_t n, float v) const {
    const float zz = v + bias[n];
    if (z) z[m * ld + n] = zz;
    act[m * ld + n] = f2bf(silu(zz));
    return 0.0f;
  }
  __device__ void colsum(int64_t, int64_t, float) const {}
};
struct EpiLinear {  // Y = acc + b
  static constexpr bool kColSums = false;
  const float* bias;
  float* y;
  int64_t ld;
  int split = 0;  // K range of a split-K product (set by the kernel)
  __device__ float operator()(int64_t m, int64_t n, float v) const {
    y[m * ld + n] = v + bias[n];
    return 0.0f;
  }
  __device__ void colsum(int64_t, int64_t, float) const {}
};
struct EpiSoA {  // de-normalised output into out[n][q0 + m] (structure of arrays)
  static constexpr bool kColSums = false;
  const float* bias;
  const float* mean;
  const float* stdv;
  float* out;
  int64_t stride, q0;
  int split = 0;  // K range of a split-K product (set by the kernel)
  __device__ float operator()(int64_t m, int64_t n, float v) const {
    out[n * stride + q0 + m] = fmaf(v + bias[n], stdv[n], mean[n]);
    return 0.0f;
  }
  __device__ void colsum(int64_t, int64_t, float) const {}
};
// G = acc * silu'(Z), stored in bf16; the FP32 column sums of each 64-row
// block are that block's partial of the layer's bias gradient, stored at
// colpart[row tile][n].
struct EpiBack {
  static constexpr bool kColSums = true;
  const float* z;
  uint16_t* gb;
  int64_t ld;
  float* colpart;
  int split = 0;  // K range of a split-K product (set by the kernel)
  __device__ float operator()(int64_t m, int64_t n, float v) const {
    const float gg = v * dsilu(z[m * ld + n]);
    gb[m * ld + n] = f2bf(gg);
    return gg;
  }
  __device__ void colsum(int64_t by, int64_t n, float s) const { colpart[by * ld + n] = s; }
};
struct EpiStore {  // partial product of K range `split` at c + split * zstride
  static constexpr bool kColSums = false;
  float* c;
  int64_t ld, zstride;
  int split = 0;  // K range of a split-K product (set by the kernel)
  __device__ float operator()(int64_t m, int64_t n, float v) const {
    c[(int64_t)split * zstride + m * ld + n] = v;
    return 0.0f;
  }
  __device__ void colsum(int64_t, int64_t, float) const {}
};

// The split-K weight-gradient products of every layer in one launch.  Block
// b belongs to the last problem whose block0 <= b; its index within the
// problem picks the K range (split), then the row tile, then the column tile.
struct GemmProblem {
  const uint16_t* A;  // kKRow: element (r, k) at A[k * lda + r]
  const uint16_t* B;  // kKRow
  float* C;           // [splits][M][N] partials
  int64_t lda, ldb, M, N, K, kc, block0;
  int tiles_m, tiles_n;
};
struct GemmGroup {
  GemmProblem p[kMlpMaxLayers];
  int count;
};

__global__ void __launch_bounds__(256) gemm_grouped_store(GemmGroup G) {
  int q = 0;
  for (int i = 1; i < G.count; ++i)
    if ((int64_t)blockIdx.x >= G.p[i].block0) q = i;
  const GemmProblem& P = G.p[q];
  const int64_t local = (int64_t)blockIdx.x - P.block0;
  const int64_t per_split = (int64_t)P.tiles_m * P.tiles_n;
  const int split = (int)(local / per_split);
  const int64_t rem = local - split * per_split;
  const int64_t tm = rem / P.tiles_n, tn = rem - tm * P.tiles_n;
  const int64_t kbeg = split * P.kc;
  const int64_t kend = kbeg + P.kc < P.K ? kbeg + P.kc : P.K;
  EpiStore epi{P.C, P.N, P.M * P.N};
  epi.split = split;
  gemm_tile<kKRow, kKRow>(P.A, P.lda, P.B, P.ldb, P.M, P.N, kbeg, kend, tm * BM, tn * BN, tm, epi);
}

// `splits` > 1: K is cut into that many ranges of a multiple of 32 each.
template <int LA, int LB, class Epi>
hipError_t gemm(const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, int64_t M,
                int64_t N, int64_t K, Epi epi, hipStream_t s, int splits = 1) {
  if (M <= 0 || N <= 0) return hipSuccess;
  int64_t kc = (K + splits - 1) / splits;
  kc = (kc + 31) / 32 * 32;
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

// Adam with bias correction c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t), on the
// gradient summed here from the partials a backward pass left (fixed order:
// split 0, 1, ... of a weight; row block 0, 1, ... of a bias); the sum is
// also stored in g.  A weight's new bf16 value also goes to its place in the
// fused kernels' packed copy when `packed` is given.
__global__ void adam_step(float* w, float* m, float* v, float* g, uint16_t* wb,
                          uint16_t* packed, int64_t n, GradParts P, MlpLayout L, float lr,
                          float b1, float b2, float eps, float c1, float c2) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  float gg = 0.0f;
  int64_t pk = -1, pt = -1;
  for (int l = 0; l < L.layers; ++l) {
    const int64_t nw = (int64_t)L.dims[l] * L.dims[l + 1], nb = L.dims[l + 1];
    if (p >= L.w_off[l] && p < L.w_off[l] + nw) {
      const int e = (int)(p - L.w_off[l]);  // < dims[l] * dims[l+1]: 32-bit division
      const int row = e / L.dims[l], col = e - row * L.dims[l];
      pk = packed_pos(l, row, col);
      if (l > 0) pt = packed_pos_t(l, row, col);
      const float* q = P.w[l] + (p - L.w_off[l]);
      float t[16];  // 16 loads in flight per round, summed in split order
#pragma unroll
      for (int z = 0; z < 16; ++z) t[z] = z < P.splits ? q[(int64_t)z * nw] : 0.0f;
      gg = t[0];
#pragma unroll
      for (int z = 1; z < 16; ++z)
        if (z < P.splits) gg += t[z];
      for (int z0 = 16; z0 < P.splits; z0 += 16) {
#pragma unroll
        for (int z = 0; z < 16; ++z) t[z] = z0 + z < P.splits ? q[(int64_t)(z0 + z) * nw] : 0.0f;
#pragma unroll
        for (int z = 0; z < 16; ++z)
          if (z0 + z < P.splits) gg += t[z];
      }
    } else if (p >= L.b_off[l] && p < L.b_off[l] + nb) {
      const float* q = P.b[l] + (p - L.b_off[l]);
      int t = 0;
      for (; t + 64 <= P.tiles; t += 64) {  // 64 loads in flight per round, summed in order
        float u[64];
#pragma unroll
        for (int j = 0; j < 64; ++j) u[j] = q[(int64_t)(t + j) * nb];
#pragma unroll
        for (int j = 0; j < 64; ++j) gg += u[j];
      }
      for (; t + 16 <= P.tiles; t += 16) {
        float u[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) u[j] = q[(int64_t)(t + j) * nb];
#pragma unroll
        for (int j = 0; j < 16; ++j) gg += u[j];
      }
      for (; t < P.tiles; ++t) gg += q[(int64_t)t * nb];
    }
  }
  g[p] = gg;
  const float mm = b1 * m[p] + (1.0f - b1) * gg;
  const float vv = b2 * v[p] + (1.0f - b2) * gg * gg;
  m[p] = mm;
  v[p] = vv;
  const float ww = w[p] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
  w[p] = ww;
  const uint16_t h = f2bf(ww);
  wb[p] = h;
  if (packed && pk >= 0) packed[pk] = h;
  if (packed && pt >= 0) packed[pt] = h;
}

// Normalised network inputs of work items [q0, q0 + count): item b is
// trajectory (q0 + b) or, for training, the affine permutation
// (mult * (q0 + b) + add) mod n.  One wave per item, one lane per value:
// lanes 0-3 write A0 [count][4] bf16 (rho, x0, y0, z0), lanes 4 .. 3 + nout
// (nout <= 60) the normalised targets T [count][nout] when y is given.
__global__ void gather_batch(const float* params, const float* u0, const float* y, int64_t n,
                             int64_t q0, int64_t count, uint64_t mult, uint64_t add,
                             const float* norm, uint16_t* a0, float* T, int nout) {
  const int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int r = threadIdx.x & 63;
  if (b >= count) return;
  const int64_t i = (int64_t)(((unsigned __int128)mult * (uint64_t)(q0 + b) + add) % (uint64_t)n);
  if (r < 4) {
    const float x = r == 0 ? params[n + i] : u0[(int64_t)(r - 1) * n + i];
    a0[b * 4 + r] = f2bf((x - norm[kInMean + r]) * norm[kInIStd + r]);
  } else if (y && r - 4 < nout) {
    const int o = r - 4;
    T[b * nout + o] = (y[(int64_t)o * n + i] - norm[kOutMean + o]) * norm[kOutIStd + o];
  }
}

// G = scale (Y - T), stored in bf16, for rows [64 t, 64 t + 64) of block t
// (cols <= 64 outputs per row); the block's sum of (Y - T)^2 goes to
// partial[t] and its FP32 column sums of G, the output layer's bias-gradient
// partial, to colpart[t][c].  Fixed summation order.
__global__ void loss_grad(const float* Y, const float* T, uint16_t* gb, int64_t rows, int cols,
                          float scale, double* partial, float* colpart) {
  __shared__ double red[256];
  __shared__ float cred[4][64];
  const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  double e2 = 0.0;
  float cs = 0.0f;
  if (c < cols) {
    for (int k = rg; k < 64; k += 4) {
      const int64_t r = r0 + k;
      if (r >= rows) break;
      const int64_t p = r * cols + c;
      const float d = Y[p] - T[p];
      const float gg = scale * d;
      gb[p] = f2bf(gg);
      e2 += (double)d * d;
      cs += gg;
    }
  }
  red[threadIdx.x] = e2;
  cred[rg][c] = cs;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
  if (rg == 0 && c < cols)
    colpart[(int64_t)blockIdx.x * cols + c] = (cred[0][c] + cred[1][c]) + (cred[2][c] + cred[3][c]);
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

hipError_t mlp_adam(float* w, float* m, float* v, float* g, uint16_t* wb, uint16_t* packed,
                    const MlpLayout& L, const GradParts& parts, float lr, float b1, float b2,
                    float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(adam_step, dim3((unsigned)((L.total + 255) / 256)), dim3(256), 0, s, w, m, v,
                     g, wb, packed, L.total, parts, L, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_gather(const float* params, const float* u0, const float* y, int64_t n, int64_t q0,
                      int64_t count, uint64_t mult, uint64_t add, const float* norm, uint16_t* a0,
                      float* T, int nout, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (nout > 60) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gather_batch, dim3((unsigned)((count + 3) / 4)), dim3(256), 0, s, params, u0,
                     y, n, q0, count, mult, add, norm, a0, T, nout);
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

// Loss and gradient partials of a training batch whose forward pass is in
// acts / Y: the output gradient and the input gradients of layers 3..1 in
// sequence (each product's epilogue leaving the bias-gradient partials of
// its layer in parts.b), then the kSplits split-K partials of every
// layer's dW in one grouped launch into parts.w (the Adam kernel sums both).
// Needs the output layer's width <= 64.
hipError_t mlp_backward(const MlpLayout& L, const uint16_t* wb, const uint16_t* a0, int64_t B,
                        MlpActs& acts, const float* Y, const float* T, GradParts& parts,
                        double* partial, float* loss, hipStream_t s) {
  const int nl = L.layers;
  const int nout = L.dims[nl];
  if (nout > 64 || nl > kMlpMaxLayers) return hipErrorInvalidValue;
  const unsigned tiles = (unsigned)((B + 63) / 64);
  parts.tiles = (int)tiles;
  hipLaunchKernelGGL(loss_grad, dim3(tiles), dim3(256), 0, s, Y, T, acts.gb[nl - 1], B, nout,
                     (float)(2.0 / (double)(B * nout)), partial, parts.b[nl - 1]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (loss) {
    hipLaunchKernelGGL(finish_sum, dim3(1), dim3(256), 0, s, partial, (int64_t)tiles,
                       1.0 / (double)(B * nout), loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // G_{l-1} [B x nin] = (G_l [B x no] . W_l [no x nin]) * silu'(Z_{l-1})
  for (int l = nl - 1; l > 0; --l) {
    const int nin = L.dims[l], no = L.dims[l + 1];
    e = gemm<kRowK, kKRow>(acts.gb[l], no, wb + L.w_off[l], nin, B, nin, no,
                           EpiBack{acts.z[l - 1], acts.gb[l - 1], nin, parts.b[l - 1]}, s);
    if (e != hipSuccess) return e;
  }
  return mlp_weight_grads(L, a0, B, acts, parts, s);
}

hipError_t mlp_loss_sum(const double* partial, int64_t count, double factor, float* loss,
                        hipStream_t s) {
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(256), 0, s, partial, count, factor, loss);
  return hipGetLastError();
}

// dW_l [no][nin] = G_l^T [no x B] . A_{l-1} [B x nin], K = B in kSplits
// ranges, every layer in one grouped launch.
hipError_t mlp_weight_grads(const MlpLayout& L, const uint16_t* a0, int64_t B, MlpActs& acts,
                            GradParts& parts, hipStream_t s) {
  const int nl = L.layers;
  parts.splits = kSplits;
  GemmGroup G{};
  G.count = nl;
  int64_t blocks = 0;
  int64_t kc = (B + kSplits - 1) / kSplits;
  kc = (kc + 31) / 32 * 32;
  for (int l = 0; l < nl; ++l) {
    const int nin = L.dims[l], no = L.dims[l + 1];
    GemmProblem& P = G.p[l];
    P.A = acts.gb[l];
    P.lda = no;
    P.B = l > 0 ? acts.act[l - 1] : a0;
    P.ldb = nin;
    P.C = parts.w[l];
    P.M = no;
    P.N = nin;
    P.K = B;
    P.kc = kc;
    P.tiles_m = (no + BM - 1) / BM;
    P.tiles_n = (nin + BN - 1) / BN;
    P.block0 = blocks;
    blocks += (int64_t)P.tiles_m * P.tiles_n * kSplits;
  }
  hipLaunchKernelGGL(gemm_grouped_store, dim3((unsigned)blocks), dim3(256), 0, s, G);
  return hipGetLastError();
}

}  // namespace ens
