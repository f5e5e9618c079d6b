// mlp_fused.hip -- the fused kernels of the surrogate MLP (rho, x0, y0, z0)
// -> 256 -> 256 -> 256 -> 48: inference in one persistent kernel (below), and
// the training step (forward, loss and input gradients of a minibatch in one
// kernel, the weight gradients in another; see "training step").
//
// Layer l computes Z_l = W_l A_{l-1} + b_l for a tile of queries on the
// matrix cores (v_mfma_f32_16x16x32_bf16: bf16 operands, FP32 accumulation)
// and A_l = bf16(silu(Z_l)).  The activations never leave registers: a
// 16 x 16 accumulator tile leaves each lane with four consecutive output
// features of one query, and two such tiles (32 features) are exactly the
// eight k-values one lane feeds into the next layer's product -- provided
// the next layer's weights are read with the matching permutation of k
// inside every 32-wide block.  `pack_weights` stores the weights in that
// permuted, fragment-major order (one 1 KiB fragment = one wave-wide
// 16-byte-per-lane load), so the kernel streams them into LDS with direct
// global->LDS loads and each lane reads its fragment with one ds_read_b128.
//
// Per block (4 waves, one per SIMD) and tile of 64*NS queries: layer 1 (K = 4,
// zero-padded to 32) and layer 4 (48 outputs) read their fragments from LDS
// copies made once per block; the two 256 x 256 layers stream through a
// double-buffered ring of 32 KiB chunks (64 output rows each), the next
// chunk loading while the current one is used.  Each fragment read from LDS
// feeds NS products (one per 16-query subtile), which keeps LDS traffic at
// 1/NS of the matrix-core operand rate.
#include "../../include/ens.h"
#include "ens_internal.h"
#include "mlp.h"

namespace ens {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kH = 256, kNO = 48;
constexpr int kFrag = kPackFrag;  // bf16 elements of one fragment (64 lanes x 8)
// packed fragment-major weights (bf16 elements), the layout of mlp.h
constexpr int64_t kP1 = kPackL1;  // layer 1: 16 row blocks
constexpr int64_t kP2 = kPackL2;  // layer 2: 16 row blocks x 8 k-blocks
constexpr int64_t kP3 = kPackL3;  // layer 3: same
constexpr int64_t kP4 = kPackL4;  // layer 4: 3 row blocks x 8 k-blocks
constexpr int kChunkBytes = 32 * kFrag * 2;  // 4 row blocks x 8 k-blocks

// LDS map (bytes).  The ring comes first so that every fragment of either
// slot is a 16-bit immediate offset (< 64 KiB) from one per-lane address;
// the per-block copies follow, reached from a second one.
constexpr int kLdsRing = 0;
constexpr int kLdsW1 = kLdsRing + 2 * kChunkBytes;
constexpr int kLdsW4 = kLdsW1 + 16 * kFrag * 2;
constexpr int kLdsBias = kLdsW4 + 24 * kFrag * 2;
static_assert(2 * kChunkBytes <= 65536, "ring fragments must be immediate offsets");
// floats at kLdsBias: b1 [256], b2 [256], b3 [256], b4 [48], out mean [48],
// out std [48], in mean [4], in 1/std [4]
constexpr int kBB1 = 0, kBB2 = 256, kBB3 = 512, kBB4 = 768, kBMean = 816, kBStd = 864,
              kBInMean = 912, kBInIStd = 916, kBCount = 920;
constexpr int kLdsBytes = kLdsBias + kBCount * 4;

__global__ void pack_weights(const uint16_t* __restrict__ wb, MlpLayout L,
                             uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kPackAll) return;
  const int e = (int)(i & 7), lane = (int)((i >> 3) & 63);
  const int64_t f = i >> 9;
  const int r16 = lane & 15, g = lane >> 4;
  uint16_t v = 0;
  if (i >= kPackT2) {  // W_l^T of layers 2..4: row = input 16 rb + r16, k = output
    const int layer = i < kPackT3 ? 1 : (i < kPackT4 ? 2 : 3);
    const int nkb = layer == 3 ? 2 : 8;
    const int64_t ff = f - (layer == 1 ? kPackT2 : (layer == 2 ? kPackT3 : kPackT4)) / kFrag;
    const int rb = (int)(ff / nkb), kb = (int)(ff % nkb);
    const int in = 16 * rb + r16, o = 32 * kb + perm32(8 * g + e);
    if (o < L.dims[layer + 1]) v = wb[L.w_off[layer] + (int64_t)o * kH + in];
  } else if (i < kP2) {  // A operand of layer 1: row 16f + r16, k = 8g + e (< 4 real)
    const int row = 16 * (int)f + r16, k = 8 * g + e;
    if (k < 4) v = wb[L.w_off[0] + row * 4 + k];
  } else {
    int layer;
    int64_t ff;
    if (i < kP3) {
      layer = 1;
      ff = f - kP2 / kFrag;
    } else if (i < kP4) {
      layer = 2;
      ff = f - kP3 / kFrag;
    } else {
      layer = 3;
      ff = f - kP4 / kFrag;
    }
    const int rb = (int)(ff >> 3), kb = (int)(ff & 7);
    const int row = 16 * rb + r16, col = 32 * kb + perm32(8 * g + e);
    v = wb[L.w_off[layer] + (int64_t)row * kH + col];
  }
  out[i] = v;
}

struct FusedArgs {
  const uint16_t* packed;
  const float* w;  // FP32 master parameters (biases)
  const float* norm;
  const float* params;  // [3][in_stride]: sigma, rho, beta
  const float* u0;      // [3][in_stride]
  float* out;           // [48][stride]
  int64_t n, stride, in_stride;
  // optional query list: work item q reads row idx[q * idx_step] of params /
  // u0 and writes that column of out (or column q with out_compact); the
  // item count is then *n_dev (at most n) when n_dev is given
  const int64_t* idx;
  int64_t idx_step;
  const unsigned long long* n_dev;
  int out_compact;
  int64_t b_off[4];
};

__device__ inline float silu(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

__device__ inline bf16x8_t silu_pack(f32x4_t lo, f32x4_t hi) {
  bf16x8_t r;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    r[e] = (__bf16)silu(lo[e]);
    r[4 + e] = (__bf16)silu(hi[e]);
  }
  return r;
}

__device__ inline bf16x8_t frag(const uint8_t* lds, int byte_off, int lane) {
  return *reinterpret_cast<const bf16x8_t*>(lds + byte_off + lane * 16);
}

__device__ inline f32x4_t bias4(const uint8_t* lds, int idx) {
  return *reinterpret_cast<const f32x4_t*>(lds + kLdsBias + idx * 4);
}

// This wave's share of one 32 KiB chunk (32 fragments over NW waves),
// global -> LDS.
// The per-lane byte offset goes through an empty asm statement so that the
// compiler rebuilds each address from the (scalar) chunk base inside the
// loop instead of hoisting 64-bit addresses of every chunk out of the tile
// loop, where they would occupy a hundred registers.
template <int NW>
__device__ inline void load_chunk(const uint16_t* src, uint8_t* slot, int wave, int lane) {
  uint32_t voff = (uint32_t)lane * 16u;
  asm volatile("" : "+v"(voff));
  const int w = __builtin_amdgcn_readfirstlane(wave);
  const char* base = reinterpret_cast<const char*>(src);
#pragma unroll
  for (int j = 0; j < 32 / NW; ++j) {
    const int fi = w * (32 / NW) + j;
    __builtin_amdgcn_global_load_lds(
        reinterpret_cast<const void*>(base + (size_t)fi * (kFrag * 2) + voff),
        (__attribute__((address_space(3))) void*)(slot + fi * kFrag * 2), 16, 0, 0);
  }
}

// The per-block copies of the layer-1 and layer-4 fragments (40, contiguous
// in LDS from kLdsW1), this wave's share, as direct global -> LDS loads: all
// in flight at once rather than a register round trip each.
template <int NW>
__device__ inline void load_fixed(const uint16_t* packed, uint8_t* lds, int wave, int lane) {
  static_assert(40 % NW == 0, "fragments per wave");
  uint32_t voff = (uint32_t)lane * 16u;
  asm volatile("" : "+v"(voff));
  const int w = __builtin_amdgcn_readfirstlane(wave);
  const char* base = reinterpret_cast<const char*>(packed);
#pragma unroll
  for (int j = 0; j < 40 / NW; ++j) {
    const int fi = w * (40 / NW) + j;
    const int64_t src = fi < 16 ? kP1 + (int64_t)fi * kFrag : kP4 + (int64_t)(fi - 16) * kFrag;
    __builtin_amdgcn_global_load_lds(
        reinterpret_cast<const void*>(base + src * 2 + voff),
        (__attribute__((address_space(3))) void*)(lds + kLdsW1 + fi * kFrag * 2), 16, 0, 0);
  }
}

__device__ inline void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// Row of minibatch item b, (mult * b + add) mod n, for mult, add < n (the
// host reduces them): 64-bit arithmetic while n <= 2^32, else 128-bit.
__device__ inline int64_t affine_row(uint64_t mult, uint64_t add, uint64_t b, uint64_t n) {
  if (n <= (1ull << 32)) return (int64_t)((mult * (b % n) + add) % n);
  return (int64_t)(((unsigned __int128)mult * b + add) % n);
}

// Products of one pair of 16-row output blocks (rb, rb+1) of a 256 x 256
// layer for every subtile, the accumulators starting from the bias.
template <int NS>
__device__ inline void pair_mfma(const uint8_t* lds, int slot_off, int pp, int rb, int bias0,
                                 int g, int lane, const bf16x8_t (&x)[NS][8],
                                 f32x4_t (&acc)[2][NS]) {
  const f32x4_t b0 = bias4(lds, bias0 + 16 * rb + 4 * g);
  const f32x4_t b1 = bias4(lds, bias0 + 16 * (rb + 1) + 4 * g);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    acc[0][s] = b0;
    acc[1][s] = b1;
  }
#pragma unroll
  for (int kb = 0; kb < 8; ++kb) {
    const bf16x8_t a0 = frag(lds, slot_off + ((2 * pp) * 8 + kb) * kFrag * 2, lane);
    const bf16x8_t a1 = frag(lds, slot_off + ((2 * pp + 1) * 8 + kb) * kFrag * 2, lane);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      acc[0][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, x[s][kb], acc[0][s], 0, 0, 0);
      acc[1][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, x[s][kb], acc[1][s], 0, 0, 0);
    }
  }
}

// The activation epilogue of a pair: y[s][k] = bf16(silu(acc)).
template <int NS>
__device__ inline void pair_silu(const f32x4_t (&acc)[2][NS], bf16x8_t (&y)[NS][8], int k) {
#pragma unroll
  for (int s = 0; s < NS; ++s) y[s][k] = silu_pack(acc[0][s], acc[1][s]);
}

// One 64-row chunk (pairs 2c and 2c+1) of a 256 x 256 layer.  Fences keep
// each pair's products and its epilogue in program order: left free, the
// scheduler merges neighbouring pairs and runs out of registers.  Matrix-core
// and vector work overlap across the two waves that share a SIMD.  (Running
// those two waves deliberately out of phase -- one deferring each chunk's
// last epilogue past the block barrier -- measured 2-5% slower.)
template <int NS>
__device__ inline void chunk_layer(const uint8_t* lds, int slot_off, int c, int bias0, int g,
                                   int lane, const bf16x8_t (&x)[NS][8], bf16x8_t (&y)[NS][8]) {
#pragma unroll
  for (int pp = 0; pp < 2; ++pp) {
    f32x4_t acc[2][NS];
    __builtin_amdgcn_sched_barrier(0);
    pair_mfma<NS>(lds, slot_off, pp, 4 * c + 2 * pp, bias0, g, lane, x, acc);
    __builtin_amdgcn_sched_barrier(0);
    pair_silu<NS>(acc, y, 2 * c + pp);
  }
}

template <int NS, int NW>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW / 4, NW / 4)))
mlp_fused_fwd(const FusedArgs a) {
  constexpr int NT = 64 * NW;
  __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsBytes];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, col = lane & 15;

  {  // per-block copies: layer-1 and layer-4 fragments, biases, normalisation
    const uint4* s1 = reinterpret_cast<const uint4*>(a.packed + kP1);
    const uint4* s4 = reinterpret_cast<const uint4*>(a.packed + kP4);
    uint4* d1 = reinterpret_cast<uint4*>(lds + kLdsW1);
    uint4* d4 = reinterpret_cast<uint4*>(lds + kLdsW4);
    for (int i = tid; i < 16 * kFrag / 8; i += NT) d1[i] = s1[i];
    for (int i = tid; i < 24 * kFrag / 8; i += NT) d4[i] = s4[i];
    float* bs = reinterpret_cast<float*>(lds + kLdsBias);
    for (int i = tid; i < kH; i += NT) {
      bs[kBB1 + i] = a.w[a.b_off[0] + i];
      bs[kBB2 + i] = a.w[a.b_off[1] + i];
      bs[kBB3 + i] = a.w[a.b_off[2] + i];
    }
    if (tid < kNO) {
      bs[kBB4 + tid] = a.w[a.b_off[3] + tid];
      bs[kBMean + tid] = a.norm[kOutMean + tid];
      bs[kBStd + tid] = a.norm[kOutStd + tid];
    }
    if (tid < 4) {
      bs[kBInMean + tid] = a.norm[kInMean + tid];
      bs[kBInIStd + tid] = a.norm[kInIStd + tid];
    }
  }
  load_chunk<NW>(a.packed + kP2, lds + kLdsRing, wave, lane);  // layer 2, chunk 0 -> slot 0
  __syncthreads();

  const float* bs = reinterpret_cast<const float*>(lds + kLdsBias);
  const int64_t n = a.n_dev ? (int64_t)(*a.n_dev < (unsigned long long)a.n ? *a.n_dev
                                                                           : (unsigned long long)a.n)
                            : a.n;
  const int64_t tq = 16 * NS * NW, ns = a.in_stride;
  const int64_t ntiles = (n + tq - 1) / tq;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t qw = tile * tq + (int64_t)wave * 16 * NS;  // this wave's first query
    bf16x8_t xa[NS][8], xb[NS][8];

    // ---- layer 1: normalised (rho, x0, y0, z0) in k = 0..3 of lane group 0
    {
      bf16x8_t xin[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int64_t q = qw + 16 * s + col;
        float f[4] = {0.f, 0.f, 0.f, 0.f};
        if (g == 0 && q < n) {
          const int64_t i = a.idx ? a.idx[q * a.idx_step] : q;
          f[0] = a.params[ns + i];
          f[1] = a.u0[i];
          f[2] = a.u0[ns + i];
          f[3] = a.u0[2 * ns + i];
#pragma unroll
          for (int k = 0; k < 4; ++k) f[k] = (f[k] - bs[kBInMean + k]) * bs[kBInIStd + k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          xin[s][k] = (__bf16)f[k];
          xin[s][4 + k] = (__bf16)0.0f;
        }
      }
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const bf16x8_t a0 = frag(lds, kLdsW1 + (2 * p) * kFrag * 2, lane);
        const bf16x8_t a1 = frag(lds, kLdsW1 + (2 * p + 1) * kFrag * 2, lane);
        const f32x4_t b0 = bias4(lds, kBB1 + 32 * p + 4 * g);
        const f32x4_t b1 = bias4(lds, kBB1 + 32 * p + 16 + 4 * g);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const f32x4_t z0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, xin[s], b0, 0, 0, 0);
          const f32x4_t z1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, xin[s], b1, 0, 0, 0);
          xa[s][p] = silu_pack(z0, z1);
        }
      }
    }

    // ---- layers 2 and 3: four chunks each through the LDS ring
    // eight chunks per tile, so chunk c of a tile always sits in slot c & 1
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      wait_vm();
      __syncthreads();
      load_chunk<NW>(a.packed + (c < 3 ? kP2 + (c + 1) * 32 * kFrag : kP3),
                     lds + kLdsRing + ((c + 1) & 1) * kChunkBytes, wave, lane);
      chunk_layer<NS>(lds, kLdsRing + (c & 1) * kChunkBytes, c, kBB2, g, lane, xa, xb);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      wait_vm();
      __syncthreads();
      load_chunk<NW>(a.packed + (c < 3 ? kP3 + (c + 1) * 32 * kFrag : kP2),
                     lds + kLdsRing + ((c + 1) & 1) * kChunkBytes, wave, lane);
      chunk_layer<NS>(lds, kLdsRing + (c & 1) * kChunkBytes, c, kBB3, g, lane, xb, xa);
    }

    // ---- layer 4: 48 outputs, de-normalised into out[o][q]
#pragma unroll
    for (int rb = 0; rb < 3; ++rb) {
      f32x4_t acc[NS];
      const f32x4_t b = bias4(lds, kBB4 + 16 * rb + 4 * g);
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[s] = b;
#pragma unroll
      for (int kb = 0; kb < 8; ++kb) {
        const bf16x8_t w = frag(lds, kLdsW4 + (rb * 8 + kb) * kFrag * 2, lane);
#pragma unroll
        for (int s = 0; s < NS; ++s)
          acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, xa[s][kb], acc[s], 0, 0, 0);
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int64_t q = qw + 16 * s + col;
        if (q < n) {
          const int64_t oc = (a.idx && !a.out_compact) ? a.idx[q * a.idx_step] : q;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int o = 16 * rb + 4 * g + r;
            a.out[(int64_t)o * a.stride + oc] = fmaf(acc[s][r], bs[kBStd + o], bs[kBMean + o]);
          }
        }
      }
    }
  }
  wait_vm();  // no global->LDS load may land after the block has left
}

// ---- training step ---------------------------------------------------------
// A training minibatch is small (a few thousand items), so the inference
// kernel's decomposition -- each wave takes whole queries through all 256
// features, the weights staged once per block in LDS -- would leave most
// CUs idle and each busy wave with a long serial chain of SiLU evaluations
// (transcendentals at a quarter of the vector rate, one wave per SIMD).
// Here a block takes 16 items through the forward pass, the loss and the
// backward pass, and its four waves split every layer's features: wave w
// computes rows 64 w .. 64 w + 63 (row blocks 4w .. 4w+3) of each hidden
// layer, and of each input gradient, reading exactly those fragments of W_l
// (or W_l^T, from the transposed packed copy) -- 32 KiB of a hidden layer,
// contiguous -- straight from global memory into registers, each used once.
// The activations and gradients are exchanged through LDS, one barrier per
// layer: lane (g, col) writes the pair of accumulator tiles it produced and
// reads back the eight pairs that are its next operands.  A 4096-item batch
// makes 256 blocks.  The pre-activations Z_l of the wave's features stay in
// registers for SiLU' in the backward pass; each layer's A_l and G_l leave
// through a transposition tile in the item-fragment layout of the weight-
// gradient product, and every G_l's sum over the block's items goes to the
// block's bias-gradient partial row.

// A block takes NS subtiles of 16 items (NS = 1 below a batch of 8192 items,
// else 2: each weight fragment then feeds two products).  LDS, per NS: two
// pair buffers [subtile][pair K][lane] of 16 bytes (layer outputs alternate
// between them); two transposition tiles [feature][16 NS items] of bf16; a
// small tile [48][16 NS] for the inputs / the output gradient; the output
// gradient's operand pieces [subtile][3][64 lanes] of 8 bytes; three loss
// partials; the biases and normalisation.
constexpr int kTB1 = 0, kTB2 = 256, kTB3 = 512, kTB4 = 768, kTOutMean = 816, kTOutIStd = 864,
              kTInMean = 912, kTInIStd = 916, kTBCount = 920;
template <int NS>
struct TLds {
  static constexpr int kItems = 16 * NS;
  static constexpr int kAct = NS * 8 * 64 * 16;
  static constexpr int kTile = 256 * kItems * 2;
  static constexpr int kTiles = 2 * kAct;
  static constexpr int kSmall = kTiles + 2 * kTile;
  static constexpr int kG4 = kSmall + 48 * kItems * 2;
  static constexpr int kLoss = kG4 + NS * 3 * 64 * 8;
  static constexpr int kBias = kLoss + 4 * 8;
  static constexpr int kBytes = kBias + kTBCount * 4;
};

struct StepArgs {
  const uint16_t* packed;  // forward and transposed fragments
  const float* w;          // FP32 master parameters (biases)
  const float* norm;
  const float* params;  // [3][in_stride]
  const float* u0;      // [3][in_stride]
  const float* y;       // [48][in_stride]
  const float* staged;  // or the set staged item-major ([in_stride][kStageW]), null
  int64_t n, in_stride, first;
  uint64_t mult, add;   // item q is row (mult (first + q) + add) mod in_stride
  int64_t b_off[4];
  uint16_t* a0;         // item-fragment outputs: inputs, A_1..A_3, G_1..G_4
  uint16_t* act[3];
  uint16_t* gb[4];
  float* bpart[4];      // [blocks][width] bias-gradient partials
  double* partial;      // [blocks] sums of (Y - T)^2
  float scale;          // dLoss / dY = scale (Y - T)
};

template <int NS>
__device__ inline bf16x8_t* act_slot(uint8_t* lds, int buf, int s, int K, int lane) {
  return reinterpret_cast<bf16x8_t*>(lds + buf * TLds<NS>::kAct + ((s * 8 + K) * 64 + lane) * 16);
}

template <int NS>
__device__ inline __bf16* ttile(uint8_t* lds, int t) {
  return reinterpret_cast<__bf16*>(lds + TLds<NS>::kTiles + t * TLds<NS>::kTile);
}

// A block's 16 NS items, from item `first`, of a [feature][16 NS items]
// transposition tile with nfb 16-feature blocks (`real` features, the rest
// zero) into the item-fragment layout of mlp.h: entry (fb, g', r16) of item
// block first / 32 holds 8 consecutive items of one feature, 16 contiguous
// bytes in the tile; the block fills lane groups g' = g0 .. g0 + 2 NS - 1.
// Non-temporal stores: the next kernel reads these from other XCDs anyway,
// and lines left dirty in this XCD's L2 would have to be written back when
// the kernel ends (measured: the step kernel 18.9 -> 16.4 us, the weight-
// gradient kernel that reads them 9.3 -> 10.3 us).
template <int NS>
__device__ inline void if_store(const __bf16* tile, uint16_t* dst, int64_t first, int nfb,
                                int real, int tid) {
  typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
  const int64_t kb = first >> 5;
  const int g0 = (int)((first & 31) >> 3);
  for (int E = tid; E < 32 * NS * nfb; E += 256) {
    const int fb = E / (32 * NS), w = E % (32 * NS), r16 = w & 15, gi = w >> 4;
    const int f = 16 * fb + r16;
    u32x4_t v = u32x4_t{0u, 0u, 0u, 0u};
    if (f < real) v = *reinterpret_cast<const u32x4_t*>(tile + f * (16 * NS) + 8 * gi);
    __builtin_nontemporal_store(
        v, reinterpret_cast<u32x4_t*>(
               dst + ((kb * nfb + fb) * kPackFrag + (16 * (g0 + gi) + r16) * 8)));
  }
}

// One fragment of the packed weights, straight from global memory.
__device__ inline bf16x8_t gfrag(const uint16_t* packed, int64_t frag_index, int lane) {
  return *reinterpret_cast<const bf16x8_t*>(packed + frag_index * kFrag + lane * 8);
}

// Forward: this wave's 64 rows of a layer for subtile s, their SiLU into
// the pair buffer (pairs K = 2w, 2w+1: features 32 K + 4 g + {0..3} and
// 32 K + 16 + 4 g + {0..3}) and into the transposition tile.
template <int NS>
__device__ inline void train_rows(const f32x4_t (&acc)[4], uint8_t* lds, int out_buf,
                                  __bf16* tile, int s, int wave, int g, int col, int lane) {
#pragma unroll
  for (int pp = 0; pp < 2; ++pp) {
    const int K = 2 * wave + pp;
    const bf16x8_t v = silu_pack(acc[2 * pp], acc[2 * pp + 1]);
    *act_slot<NS>(lds, out_buf, s, K, lane) = v;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      tile[(32 * K + 4 * g + r) * (16 * NS) + 16 * s + col] = v[r];
      tile[(32 * K + 16 + 4 * g + r) * (16 * NS) + 16 * s + col] = v[4 + r];
    }
  }
}

__device__ inline float dsilu(float z) {
  const float s = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
  return s * (1.0f + z * (1.0f - s));
}

// Sum over the 16 lanes of a lane group (a subtile's 16 items): rotations
// by 8, 4, 2, 1 within each 16-lane DPP row, plain vector adds (a lane-
// crossbar shuffle would cost an LDS round trip per step).  Every lane ends
// with the group's total; callers take lane 0 of the group, whose order of
// additions is fixed.
__device__ inline float ror16(float v, int ctrl_sel) {
  const int x = __builtin_bit_cast(int, v);
  int r;
  switch (ctrl_sel) {  // row_ror:8 / :4 / :2 / :1
    case 8: r = __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false); break;
    case 4: r = __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false); break;
    case 2: r = __builtin_amdgcn_update_dpp(0, x, 0x122, 0xF, 0xF, false); break;
    default: r = __builtin_amdgcn_update_dpp(0, x, 0x121, 0xF, 0xF, false); break;
  }
  return __builtin_bit_cast(float, r);
}
__device__ inline float sum16(float v) {
  v += ror16(v, 8);
  v += ror16(v, 4);
  v += ror16(v, 2);
  v += ror16(v, 1);
  return v;
}

// Backward: G = acc * silu'(Z) for this wave's 64 features (row blocks
// 4w + j) of subtile s: bf16 pairs into the pair buffer (out_buf >= 0) and
// the transposition tile; each value's sum over the subtile's 16 items is
// added to bs (lane 0 of a group holds the group's sums).
template <int NS>
__device__ inline void bwd_rows(const f32x4_t (&acc)[4], const f32x4_t (&zv)[4], uint8_t* lds,
                                int out_buf, __bf16* tile, int s, int wave, int g, int col,
                                int lane, int r0, float (&bs)[16]) {
  f32x4_t G[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) G[j][r] = acc[j][r] * dsilu(zv[j][r]);
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) tile[(r0 + 16 * j + r) * (16 * NS) + 16 * s + col] = (__bf16)G[j][r];
  if (out_buf >= 0) {
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
      bf16x8_t v;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v[r] = (__bf16)G[2 * pp][r];
        v[4 + r] = (__bf16)G[2 * pp + 1][r];
      }
      *act_slot<NS>(lds, out_buf, s, 2 * wave + pp, lane) = v;
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) bs[4 * j + r] = s == 0 ? sum16(G[j][r]) : bs[4 * j + r] + sum16(G[j][r]);
}

// The block's bias-gradient partial row: lane 0 of each group writes its 16.
__device__ inline void write_bias_row(const float (&bs)[16], int col, int r0, float* bp) {
  if (col == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) bp[r0 + 16 * j + r] = bs[4 * j + r];
  }
}

// A hidden layer's products for this wave's four row blocks over the eight
// k-blocks of the pair buffer in_buf, every subtile; accumulators start
// from acc.
template <int NS>
__device__ inline void rows_mfma(f32x4_t (&acc)[NS][4], const bf16x8_t (&w)[4][8], uint8_t* lds,
                                 int in_buf, int lane) {
  bf16x8_t x[NS][8];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) x[s][kb] = *act_slot<NS>(lds, in_buf, s, kb, lane);
#pragma unroll
  for (int kb = 0; kb < 8; ++kb)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int s = 0; s < NS; ++s)
        acc[s][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[j][kb], x[s][kb], acc[s][j], 0, 0, 0);
}

__device__ inline void load_rows(bf16x8_t (&w)[4][8], const uint16_t* packed, int64_t base_frag,
                                 int wave, int lane) {
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) w[j][kb] = gfrag(packed, base_frag + (4 * wave + j) * 8 + kb, lane);
}

template <int NS>
__global__ void __launch_bounds__(256) mlp_train_step(const StepArgs a) {
  using T = TLds<NS>;
  constexpr int IT = 16 * NS;  // items per block
  __shared__ __attribute__((aligned(16))) uint8_t lds[T::kBytes];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, col = lane & 15;
  const int64_t ns = a.in_stride;
  const int64_t first = (int64_t)blockIdx.x * IT;  // the block's first item
  const int r0 = 64 * wave + 4 * g;  // this lane's first feature of its row blocks
  float* bw = reinterpret_cast<float*>(lds + T::kBias);
  __bf16* small = reinterpret_cast<__bf16*>(lds + T::kSmall);

  // biases and normalisation first, so that their wait before the LDS
  // stores does not wait for the loads issued after them
  const float bh0 = a.w[a.b_off[0] + tid], bh1 = a.w[a.b_off[1] + tid],
              bh2 = a.w[a.b_off[2] + tid];
  float b4 = 0.f, om = 0.f, ois = 0.f, im = 0.f, iis = 0.f;
  if (tid < kNO) {
    b4 = a.w[a.b_off[3] + tid];
    om = a.norm[kOutMean + tid];
    ois = a.norm[kOutIStd + tid];
  }
  if (tid < 4) {
    im = a.norm[kInMean + tid];
    iis = a.norm[kInIStd + tid];
  }
  // each subtile's item (lane col), its row, inputs (lane group 0) and, in
  // waves 0..2, the four targets of outputs 16 w + 4 g + r its output
  // gradient uses
  bool live[NS];
  float f[NS][4], yt[NS][4];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int64_t q = first + 16 * s + col;
    live[s] = q < a.n;
#pragma unroll
    for (int k = 0; k < 4; ++k) f[s][k] = yt[s][k] = 0.f;
    if (live[s]) {
      const int64_t row = affine_row(a.mult, a.add, (uint64_t)(a.first + q), (uint64_t)ns);
      if (a.staged) {  // normalised already, one 208-byte record per item
        const float* rec = a.staged + row * kStageW;
        if (g == 0) {
          const f32x4_t v = *reinterpret_cast<const f32x4_t*>(rec);
#pragma unroll
          for (int k = 0; k < 4; ++k) f[s][k] = v[k];
        }
        if (wave < 3) {
          const f32x4_t v = *reinterpret_cast<const f32x4_t*>(rec + 4 + 16 * wave + 4 * g);
#pragma unroll
          for (int r = 0; r < 4; ++r) yt[s][r] = v[r];
        }
      } else {
        if (g == 0) {
          f[s][0] = a.params[ns + row];
          f[s][1] = a.u0[row];
          f[s][2] = a.u0[ns + row];
          f[s][3] = a.u0[2 * ns + row];
        }
        if (wave < 3) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            yt[s][r] = a.y[(int64_t)(16 * wave + 4 * g + r) * ns + row];
        }
      }
    }
  }
  // this wave's weights of layers 1 and 2
  bf16x8_t w1[4], w[4][8];
#pragma unroll
  for (int j = 0; j < 4; ++j) w1[j] = gfrag(a.packed, kP1 / kFrag + 4 * wave + j, lane);
  load_rows(w, a.packed, kP2 / kFrag, wave, lane);
  bw[kTB1 + tid] = bh0;
  bw[kTB2 + tid] = bh1;
  bw[kTB3 + tid] = bh2;
  if (tid < kNO) {
    bw[kTB4 + tid] = b4;
    bw[kTOutMean + tid] = om;
    bw[kTOutIStd + tid] = ois;
  }
  if (tid < 4) {
    bw[kTInMean + tid] = im;
    bw[kTInIStd + tid] = iis;
  }
  __syncthreads();
  f32x4_t z[3][NS][4];  // pre-activations of this wave's features, kept for SiLU'
  f32x4_t acc[NS][4];

  // ---- forward, layer 1: normalised (rho, x0, y0, z0) in k = 0..3 of lane
  // group 0
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    bf16x8_t xin;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float v = !(g == 0 && live[s]) ? 0.f
                      : a.staged          ? f[s][k]
                                          : (f[s][k] - bw[kTInMean + k]) * bw[kTInIStd + k];
      xin[k] = (__bf16)v;
      xin[4 + k] = (__bf16)0.0f;
    }
    if (wave == 0 && g == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) small[k * IT + 16 * s + col] = xin[k];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      z[0][s][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          w1[j], xin, *reinterpret_cast<const f32x4_t*>(bw + kTB1 + r0 + 16 * j), 0, 0, 0);
    train_rows<NS>(z[0][s], lds, 0, ttile<NS>(lds, 0), s, wave, g, col, lane);
  }
  __syncthreads();
  if_store<NS>(small, a.a0, first, 1, 4, tid);
  if_store<NS>(ttile<NS>(lds, 0), a.act[0], first, 16, kH, tid);

  // ---- layer 2
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      z[1][s][j] = *reinterpret_cast<const f32x4_t*>(bw + kTB2 + r0 + 16 * j);
  rows_mfma<NS>(z[1], w, lds, 0, lane);
  load_rows(w, a.packed, kP3 / kFrag, wave, lane);  // layer 3, in flight meanwhile
#pragma unroll
  for (int s = 0; s < NS; ++s) train_rows<NS>(z[1][s], lds, 1, ttile<NS>(lds, 1), s, wave, g, col, lane);
  __syncthreads();
  if_store<NS>(ttile<NS>(lds, 1), a.act[1], first, 16, kH, tid);

  // ---- layer 3
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      z[2][s][j] = *reinterpret_cast<const f32x4_t*>(bw + kTB3 + r0 + 16 * j);
  rows_mfma<NS>(z[2], w, lds, 1, lane);
  bf16x8_t w4[8], w4t[4][2];  // layer 4's row block `wave` (waves 0..2), W_4^T rows
  if (wave < 3) {
#pragma unroll
    for (int kb4 = 0; kb4 < 8; ++kb4) w4[kb4] = gfrag(a.packed, kP4 / kFrag + wave * 8 + kb4, lane);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2)
      w4t[j][k2] = gfrag(a.packed, kPackT4 / kFrag + (4 * wave + j) * 2 + k2, lane);
#pragma unroll
  for (int s = 0; s < NS; ++s) train_rows<NS>(z[2][s], lds, 0, ttile<NS>(lds, 0), s, wave, g, col, lane);
  __syncthreads();
  if_store<NS>(ttile<NS>(lds, 0), a.act[2], first, 16, kH, tid);

  // ---- layer 4 and the loss (waves 0..2: outputs 16 w .. 16 w + 15):
  // G_4 = scale (Y - T) into the small tile, the operand pieces, the output
  // bias partial and the block's loss partial
  if (wave < 3) {
    const int o0 = 16 * wave + 4 * g;
    f32x4_t out[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      bf16x8_t x[8];
#pragma unroll
      for (int k8 = 0; k8 < 8; ++k8) x[k8] = *act_slot<NS>(lds, 0, s, k8, lane);
      out[s] = *reinterpret_cast<const f32x4_t*>(bw + kTB4 + o0);
#pragma unroll
      for (int k8 = 0; k8 < 8; ++k8)
        out[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w4[k8], x[k8], out[s], 0, 0, 0);
    }
    load_rows(w, a.packed, kPackT3 / kFrag, wave, lane);  // W_3^T for G_2, in flight
    float bs4[4];
    double d2 = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      float gg[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float t = !live[s] ? 0.f
                        : a.staged ? yt[s][r]
                                   : (yt[s][r] - bw[kTOutMean + o0 + r]) * bw[kTOutIStd + o0 + r];
        const float d = live[s] ? out[s][r] - t : 0.f;
        gg[r] = a.scale * d;
        d2 += (double)d * d;
        small[(o0 + r) * IT + 16 * s + col] = (__bf16)gg[r];
        bs4[r] = s == 0 ? sum16(gg[r]) : bs4[r] + sum16(gg[r]);
      }
      typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
      *reinterpret_cast<bf16x4_t*>(lds + T::kG4 + ((s * 3 + wave) * 64 + lane) * 8) =
          bf16x4_t{(__bf16)gg[0], (__bf16)gg[1], (__bf16)gg[2], (__bf16)gg[3]};
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) d2 += __shfl_xor(d2, m);
    if (lane == 0) reinterpret_cast<double*>(lds + T::kLoss)[wave] = d2;
    float* bp = a.bpart[3] + (int64_t)blockIdx.x * kNO;
    if (col == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) bp[o0 + r] = bs4[r];
    }
  } else {
    load_rows(w, a.packed, kPackT3 / kFrag, wave, lane);
  }
  __syncthreads();
  if (tid == 0) {
    const double* lp = reinterpret_cast<const double*>(lds + T::kLoss);
    a.partial[blockIdx.x] = (lp[0] + lp[1]) + lp[2];
  }
  if_store<NS>(small, a.gb[3], first, 3, kNO, tid);

  // ---- backward: G_3 = (G_4 W_4) * silu'(Z_3), K = 48 (k-block 1 half
  // zero): lane (g, col) takes outputs 4g.., 16+4g.. and 32+4g.. from the
  // pieces of waves 0, 1, 2
  float bs[16];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
    const uint8_t* pc = lds + T::kG4 + (s * 3 * 64 + lane) * 8;
    const bf16x4_t p0 = *reinterpret_cast<const bf16x4_t*>(pc);
    const bf16x4_t p1 = *reinterpret_cast<const bf16x4_t*>(pc + 64 * 8);
    const bf16x4_t p2 = *reinterpret_cast<const bf16x4_t*>(pc + 2 * 64 * 8);
    bf16x8_t x4[2];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      x4[0][e] = p0[e];
      x4[0][4 + e] = p1[e];
      x4[1][e] = p2[e];
      x4[1][4 + e] = (__bf16)0.0f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[s][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k2 = 0; k2 < 2; ++k2)
        acc[s][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w4t[j][k2], x4[k2], acc[s][j], 0, 0, 0);
    }
    bwd_rows<NS>(acc[s], z[2][s], lds, 1, ttile<NS>(lds, 1), s, wave, g, col, lane, r0, bs);
  }
  write_bias_row(bs, col, r0, a.bpart[2] + (int64_t)blockIdx.x * kH);
  __syncthreads();
  if_store<NS>(ttile<NS>(lds, 1), a.gb[2], first, 16, kH, tid);

  // ---- G_2 = (G_3 W_3) * silu'(Z_2)
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[s][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  rows_mfma<NS>(acc, w, lds, 1, lane);
  load_rows(w, a.packed, kPackT2 / kFrag, wave, lane);  // W_2^T, in flight meanwhile
#pragma unroll
  for (int s = 0; s < NS; ++s)
    bwd_rows<NS>(acc[s], z[1][s], lds, 0, ttile<NS>(lds, 0), s, wave, g, col, lane, r0, bs);
  write_bias_row(bs, col, r0, a.bpart[1] + (int64_t)blockIdx.x * kH);
  __syncthreads();
  if_store<NS>(ttile<NS>(lds, 0), a.gb[1], first, 16, kH, tid);

  // ---- G_1 = (G_2 W_2) * silu'(Z_1)
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[s][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  rows_mfma<NS>(acc, w, lds, 0, lane);
#pragma unroll
  for (int s = 0; s < NS; ++s)
    bwd_rows<NS>(acc[s], z[0][s], lds, -1, ttile<NS>(lds, 1), s, wave, g, col, lane, r0, bs);
  write_bias_row(bs, col, r0, a.bpart[0] + (int64_t)blockIdx.x * kH);
  __syncthreads();
  if_store<NS>(ttile<NS>(lds, 1), a.gb[0], first, 16, kH, tid);
}

// ---- staged training set ---------------------------------------------------
// Item-major, normalised copy of a training set for the epochs of one
// training call: record i = (rho, x0, y0, z0) and the 48 targets of
// trajectory i, each as the forward kernel would normalise it, so that a
// minibatch gather reads 208 contiguous bytes per item instead of one
// scattered line from each of 52 rows.  A block takes 64 items: coalesced
// reads of the 52 rows into an LDS tile, then contiguous record writes.
// One 64-item tile of stage_items (the grid strides over tiles).
__device__ inline void stage_tile(const float* params, const float* u0, const float* y,
                                  int64_t n, const float* norm, float* D,
                                  float (&tile)[64][kStageW + 1], int64_t i0, int tid) {
  for (int e = tid; e < 64 * kStageW; e += 256) {
    const int c = e >> 6, i = e & 63;
    const int64_t it = i0 + i;
    float v = 0.f;
    if (it < n) {
      if (c < 4) {
        const float x = c == 0 ? params[n + it] : u0[(int64_t)(c - 1) * n + it];
        v = (x - norm[kInMean + c]) * norm[kInIStd + c];
      } else {
        const int o = c - 4;
        v = (y[(int64_t)o * n + it] - norm[kOutMean + o]) * norm[kOutIStd + o];
      }
    }
    tile[i][c] = v;
  }
  __syncthreads();
  const int64_t items = n - i0 < 64 ? n - i0 : 64;
  for (int e = tid; e < items * kStageW; e += 256) D[i0 * kStageW + e] = tile[e / kStageW][e % kStageW];
  __syncthreads();  // the tile is refilled by the next iteration
}

__global__ void __launch_bounds__(256) stage_items(const float* params, const float* u0,
                                                   const float* y, int64_t n, const float* norm,
                                                   float* D) {
  __shared__ float tile[64][kStageW + 1];
  const int tid = threadIdx.x;
  for (int64_t i0 = (int64_t)blockIdx.x * 64; i0 < n; i0 += (int64_t)gridDim.x * 64) {
    stage_tile(params, u0, y, n, norm, D, tile, i0, tid);
  }
}

// ---- weight gradients ------------------------------------------------------
// dW_l [o][i] = sum over items of G_l [item][o] A_{l-1} [item][i], both in the
// item-fragment layout: a fragment of G_l is exactly the A operand of
// v_mfma_f32_16x16x32_bf16 for 16 rows o and 32 items, a fragment of
// A_{l-1} the B operand for 16 columns i, so every wave reads its operands
// with 16-byte loads straight into registers and no LDS is involved.  A
// block takes a 64 x 64 tile of one layer's dW (wave (wm, wn) a 32 x 32
// quarter), or from 16,384 items a 128 x 128 one (64 x 64 per wave), over
// one of the step's item ranges and writes that range's partial; the Adam
// kernel sums the partials.
struct DwProblem {
  const uint16_t* G;  // item-fragment layout, nfo feature blocks
  const uint16_t* A;  // item-fragment layout, nfi feature blocks
  float* C;           // [splits][M][N]
  int M, N, nfo, nfi, tiles_m, tiles_n;
  int64_t block0;
};
struct DwGroup {
  DwProblem p[4];
  int count;
  int64_t nkb, kc;  // item blocks, item blocks per split
  // bias gradients: the blocks from bias_block0 on each sum the `rows`
  // per-block partial rows of 64 biases (layer l: bias_n[l] of them at
  // bias[l]) into row 0, so the Adam kernel reads one row
  float* bias[4];
  int bias_n[4];
  int64_t bias_block0;
  int rows;
};

// 16 biases per block, sixteen threads per bias each summing a sixteenth of
// the rows in order (16 loads in flight), the sixteen parts then added in
// order: a fixed summation order, and enough threads on the rows that a
// large batch's thousands of block rows do not make these blocks the
// launch's long pole.
constexpr int kBiasPerBlock = 16;
__device__ void bias_sums(const DwGroup& D, int64_t b) {
  __shared__ float part[16][kBiasPerBlock];
  int l = 0;  // layer l owns ceil(bias_n[l] / 16) consecutive blocks
  while (l < D.count - 1 && b >= (D.bias_n[l] + kBiasPerBlock - 1) / kBiasPerBlock) {
    b -= (D.bias_n[l] + kBiasPerBlock - 1) / kBiasPerBlock;
    ++l;
  }
  const int t = threadIdx.x, j = t & (kBiasPerBlock - 1), sixteenth = t >> 4;
  const int64_t f = b * kBiasPerBlock + j;
  const int n = D.bias_n[l];
  float sum = 0.f;
  if (f < n) {
    const int per = (D.rows + 15) / 16, r0 = sixteenth * per,
              r1 = r0 + per < D.rows ? r0 + per : D.rows;
    const float* col = D.bias[l] + f;
    int r = r0;
    for (; r + 16 <= r1; r += 16) {
      float u[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) u[k] = col[(int64_t)(r + k) * n];
#pragma unroll
      for (int k = 0; k < 16; ++k) sum += u[k];
    }
    for (; r < r1; ++r) sum += col[(int64_t)r * n];
  }
  part[sixteenth][j] = sum;
  __syncthreads();
  if (sixteenth == 0 && f < n) {
    float tot = part[0][j];
#pragma unroll
    for (int k = 1; k < 16; ++k) tot += part[k][j];
    D.bias[l][f] = tot;
  }
}

// WT 16-row blocks per wave in each dimension: WT = 2, a 64 x 64 tile per
// block (small batches: enough blocks); WT = 4, 128 x 128 (large batches:
// each operand fragment is read by half as many blocks).
template <int WT>
__global__ void __launch_bounds__(256) mlp_dw(const DwGroup D) {
  constexpr int RT = 16 / WT;  // item blocks per round: 4 WT operand fragments each
  if ((int64_t)blockIdx.x >= D.bias_block0) {
    bias_sums(D, (int64_t)blockIdx.x - D.bias_block0);
    return;
  }
  int pi = 0;
#pragma unroll
  for (int i = 1; i < 4; ++i)
    if (i < D.count && (int64_t)blockIdx.x >= D.p[i].block0) pi = i;
  const DwProblem& P = D.p[pi];
  // Blocks go to the eight XCDs round robin (block0 and the block count of
  // every problem are multiples of 8): every tile of item range z runs on
  // XCD z mod 8, so the range's operands are fetched into that XCD's L2
  // once and re-read from there by the range's other tiles
  const int64_t b = (int64_t)blockIdx.x - P.block0;
  const int per_split = P.tiles_m * P.tiles_n;
  const int64_t slot = b >> 3;
  const int split = (int)((b & 7) + 8 * (slot / per_split)), rem = (int)(slot % per_split);
  const int tm = rem / P.tiles_n, tn = rem % P.tiles_n;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int fo0 = 2 * WT * tm + WT * (wave >> 1), fi0 = 2 * WT * tn + WT * (wave & 1);
  const int64_t kb0 = split * D.kc, kb1 = kb0 + D.kc < D.nkb ? kb0 + D.kc : D.nkb;
  f32x4_t acc[WT][WT];
#pragma unroll
  for (int x = 0; x < WT; ++x)
#pragma unroll
    for (int y = 0; y < WT; ++y) acc[x][y] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const bf16x8_t zero = bf16x8_t{};
  for (int64_t k0 = kb0; k0 < kb1; k0 += RT) {  // RT item blocks' operands in flight
    bf16x8_t ga[RT][WT], ab[RT][WT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int x = 0; x < WT; ++x) {
        const bool kin = k0 + t < kb1;
        ga[t][x] = kin && fo0 + x < P.nfo
                       ? *reinterpret_cast<const bf16x8_t*>(
                             P.G + (((k0 + t) * P.nfo + fo0 + x) * kPackFrag + lane * 8))
                       : zero;
        ab[t][x] = kin && fi0 + x < P.nfi
                       ? *reinterpret_cast<const bf16x8_t*>(
                             P.A + (((k0 + t) * P.nfi + fi0 + x) * kPackFrag + lane * 8))
                       : zero;
      }
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int x = 0; x < WT; ++x)
#pragma unroll
        for (int y = 0; y < WT; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ga[t][x], ab[t][y], acc[x][y], 0, 0, 0);
  }
  // lane (g, c) holds rows 4 g + r, column c of each 16 x 16 block
  float* C = P.C + (int64_t)split * P.M * P.N;
  const int g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int x = 0; x < WT; ++x)
#pragma unroll
    for (int y = 0; y < WT; ++y) {
      const int i = 16 * (fi0 + y) + c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 16 * (fo0 + x) + 4 * g + r;
        if (o < P.M && i < P.N) C[(int64_t)o * P.N + i] = acc[x][y][r];
      }
    }
}

}  // namespace

int64_t mlp_packed_elems() { return kPackAll; }

hipError_t mlp_pack(const uint16_t* wb, const MlpLayout& L, uint16_t* packed, hipStream_t s) {
  hipLaunchKernelGGL(pack_weights, dim3((unsigned)((kPackAll + 255) / 256)), dim3(256), 0, s, wb,
                     L, packed);
  return hipGetLastError();
}

// out[o][q] for q in [0, n), o in [0, 48); `stride` is the row length of out.
hipError_t mlp_forward_fused(const MlpLayout& L, const uint16_t* packed, const float* w,
                             const float* norm, const float* params, const float* u0, int64_t n,
                             float* out, int64_t stride, int num_cu, int ns, hipStream_t s) {
  return mlp_forward_fused_list(L, packed, w, norm, params, u0, n, n, nullptr, 1, nullptr, 0, out,
                                stride, num_cu, ns, s);
}

// Queries from a list: item q < min(n, *n_dev) is row idx[q * idx_step] of
// the [.][in_stride] inputs; its answer goes to column q of out
// (out_compact) or to the row's own column.  idx = null: item q is row q.
hipError_t mlp_forward_fused_list(const MlpLayout& L, const uint16_t* packed, const float* w,
                                  const float* norm, const float* params, const float* u0,
                                  int64_t n, int64_t in_stride, const int64_t* idx,
                                  int64_t idx_step, const unsigned long long* n_dev,
                                  int out_compact, float* out, int64_t stride, int num_cu, int ns,
                                  hipStream_t s) {
  if (n <= 0) return hipSuccess;
  FusedArgs a{};
  a.packed = packed;
  a.w = w;
  a.norm = norm;
  a.params = params;
  a.u0 = u0;
  a.out = out;
  a.n = n;
  a.stride = stride;
  a.in_stride = in_stride;
  a.idx = idx;
  a.idx_step = idx_step;
  a.n_dev = n_dev;
  a.out_compact = out_compact;
  for (int l = 0; l < 4; ++l) a.b_off[l] = L.b_off[l];
  // ns = NS (one wave per SIMD, 4-wave blocks) or 10 + NS (two waves per
  // SIMD, 8-wave blocks)
  const int NS = ns % 10, NW = ns >= 10 ? 8 : 4;
  const int64_t tq = 16 * (int64_t)NS * NW;
  const int64_t ntiles = (n + tq - 1) / tq;
  const unsigned grid = (unsigned)(ntiles < num_cu ? ntiles : num_cu);
  const dim3 blk(64 * NW);
  switch (ns) {
    case 2: hipLaunchKernelGGL((mlp_fused_fwd<2, 4>), dim3(grid), blk, 0, s, a); break;
    case 3: hipLaunchKernelGGL((mlp_fused_fwd<3, 4>), dim3(grid), blk, 0, s, a); break;
    case 12: hipLaunchKernelGGL((mlp_fused_fwd<2, 8>), dim3(grid), blk, 0, s, a); break;
    case 13: hipLaunchKernelGGL((mlp_fused_fwd<3, 8>), dim3(grid), blk, 0, s, a); break;
    default: hipLaunchKernelGGL((mlp_fused_fwd<4, 4>), dim3(grid), blk, 0, s, a); break;
  }
  return hipGetLastError();
}

// The training step's fused launch: one block per 16 items, whole 32-item
// blocks of the item-fragment outputs.
hipError_t mlp_train_fused(const uint16_t* packed, const float* w, const MlpLayout& L,
                           const float* norm, const float* params, const float* u0,
                           const float* y, const float* staged, int64_t n, int64_t first,
                           int64_t B, uint64_t mult, uint64_t add, uint16_t* a0, MlpActs& acts,
                           GradParts& parts, double* partial, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if (L.layers != 4 || L.dims[0] != 4 || L.dims[1] != kH || L.dims[2] != kH ||
      L.dims[3] != kH || L.dims[4] != kNO || n <= 0)
    return hipErrorInvalidValue;
  // 16-item blocks for a small batch (so it still spreads over the CUs),
  // 32-item ones from 8192 items on; whole 32-item blocks of outputs either way
  const int NS = B >= 8192 ? 2 : 1;
  const int64_t blocks = (2 / NS) * ((B + 31) / 32);
  if (blocks > (1LL << 24)) return hipErrorInvalidValue;  // blocks x 256 work-items fit 32 bits
  StepArgs a{};
  a.packed = packed;
  a.w = w;
  a.norm = norm;
  a.params = params;
  a.u0 = u0;
  a.y = y;
  a.staged = staged;
  a.n = B;
  a.in_stride = n;
  a.first = first;
  a.mult = mult % (uint64_t)n;
  a.add = add % (uint64_t)n;
  for (int l = 0; l < 4; ++l) a.b_off[l] = L.b_off[l];
  a.a0 = a0;
  for (int l = 0; l < 3; ++l) a.act[l] = acts.act[l];
  for (int l = 0; l < 4; ++l) {
    a.gb[l] = acts.gb[l];
    a.bpart[l] = parts.b[l];
  }
  a.partial = partial;
  a.scale = (float)(2.0 / (double)(B * kNO));
  parts.tiles = (int)blocks;
  if (NS == 2)
    hipLaunchKernelGGL(mlp_train_step<2>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(mlp_train_step<1>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Weight-gradient partials from the item-fragment operands the fused
// forward and backward kernels leave (B items padded to whole 32-item
// blocks with zero gradients).
hipError_t mlp_weight_grads_if(const MlpLayout& L, int64_t B, MlpActs& acts, const uint16_t* a0,
                               GradParts& parts, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  DwGroup D{};
  D.count = L.layers;
  D.nkb = (B + 31) / 32;
  // about 16 item blocks per range, a multiple of the 8 XCDs
  int64_t splits = ((D.nkb + 15) / 16 + 7) / 8 * 8;
  const int WT = D.nkb >= 512 ? 4 : 2;  // 128 x 128 tiles from 16,384 items on
  const int tile = 32 * WT;
  splits = splits < kSplitsFusedMin ? kSplitsFusedMin : (splits > kSplitsMax ? kSplitsMax : splits);
  D.kc = (D.nkb + splits - 1) / splits;
  parts.splits = (int)splits;
  int64_t blocks = 0;
  for (int l = 0; l < L.layers; ++l) {
    DwProblem& P = D.p[l];
    P.G = acts.gb[l];
    P.A = l > 0 ? acts.act[l - 1] : a0;
    P.C = parts.w[l];
    P.M = L.dims[l + 1];
    P.N = L.dims[l];
    P.nfo = (P.M + 15) / 16;
    P.nfi = (P.N + 15) / 16;
    P.tiles_m = (P.M + tile - 1) / tile;
    P.tiles_n = (P.N + tile - 1) / tile;
    P.block0 = blocks;
    blocks += (int64_t)P.tiles_m * P.tiles_n * splits;
  }
  // bias blocks: each layer's biases in whole blocks of kBiasPerBlock
  D.bias_block0 = blocks;
  D.rows = parts.tiles;
  for (int l = 0; l < L.layers; ++l) {
    D.bias[l] = parts.b[l];
    D.bias_n[l] = L.dims[l + 1];
    blocks += (L.dims[l + 1] + kBiasPerBlock - 1) / kBiasPerBlock;
  }
  if (WT == 4)
    hipLaunchKernelGGL(mlp_dw<4>, dim3((unsigned)blocks), dim3(256), 0, s, D);
  else
    hipLaunchKernelGGL(mlp_dw<2>, dim3((unsigned)blocks), dim3(256), 0, s, D);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  parts.tiles = 1;  // the Adam kernel reads the summed row
  return hipSuccess;
}

hipError_t mlp_stage_items(const float* params, const float* u0, const float* y, int64_t n,
                           const float* norm, float* D, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t tiles = (n + 63) / 64;
  hipLaunchKernelGGL(stage_items, dim3((unsigned)(tiles < 65536 ? tiles : 65536)), dim3(256), 0, s,
                     params, u0, y, n, norm, D);
  return hipGetLastError();
}

}  // namespace ens
