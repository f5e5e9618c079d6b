// mlp.h -- host-visible structures of the surrogate's kernels (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ens {

constexpr int kMlpMaxLayers = 4;

// Flat parameter vector: for each layer l, W_l row-major [dims[l+1]][dims[l]]
// at w_off[l], then b_l [dims[l+1]] at b_off[l].
struct MlpLayout {
  int layers;
  int dims[kMlpMaxLayers + 1];
  int64_t w_off[kMlpMaxLayers];
  int64_t b_off[kMlpMaxLayers];
  int64_t total;
};

inline MlpLayout make_layout(const int* dims, int layers) {
  MlpLayout L{};
  L.layers = layers;
  int64_t off = 0;
  for (int l = 0; l <= layers; ++l) L.dims[l] = dims[l];
  for (int l = 0; l < layers; ++l) {
    L.w_off[l] = off;
    off += (int64_t)dims[l] * dims[l + 1];
    L.b_off[l] = off;
    off += dims[l + 1];
  }
  L.total = off;
  return L;
}

// Normalisation block (FP32, device): inputs (rho, x0, y0, z0) and the 48
// outputs, each with mean, 1/std, std; the inputs also with the min / max of
// the training set (the validated box).
constexpr int kInMean = 0, kInIStd = 4, kInLo = 8, kInHi = 12;
constexpr int kOutMean = 16, kOutIStd = 64, kOutStd = 112, kNormSize = 160;

// Operand storage of the tiled matrix-core product: element (r, k) at
// [r * ld + k] (kRowK) or [k * ld + r] (kKRow).
enum { kRowK = 0, kKRow = 1 };

struct MlpActs {
  bool keep_all;        // training: every hidden layer's Z and A are kept
  float* z[kMlpMaxLayers];
  uint16_t* act[kMlpMaxLayers];
  uint16_t* gb[kMlpMaxLayers];  // training: bf16 output gradient G_l of every layer
};

// Split-K factors of the weight-gradient products (K = batch): the tiled
// path's, and the fused path's range of them -- about 16 item blocks of 32
// per range, so a small batch takes few, longer ranges and a large one
// enough blocks to hide its loads; buffers are sized for the largest.
constexpr int kSplits = 16;
constexpr int kSplitsFusedMin = 8, kSplitsMax = 64;  // multiples of 8 (XCD-aware order)
static_assert(kSplits <= kSplitsMax, "partial buffers hold kSplitsMax ranges");

// Gradient partials of one training step, summed by the Adam kernel:
// w[l] [splits][dims[l+1] * dims[l]] split-K partials of dW_l (room for
// kSplitsMax), b[l] [tiles][dims[l+1]] partials of db_l over blocks of the
// batch.
struct GradParts {
  float* w[kMlpMaxLayers];
  float* b[kMlpMaxLayers];
  int tiles;
  int splits;
};

struct RowSet {
  const float* ptr[64];
};

hipError_t mlp_init(float* w, uint16_t* wb, const MlpLayout& L, uint64_t seed, hipStream_t s);
hipError_t mlp_to_bf16(const float* w, uint16_t* wb, int64_t n, hipStream_t s);
// packed (may be null; the 4-256-256-256-48 network only) receives each
// updated bf16 weight at its packed_pos, and those of layers 2..4 at their
// packed_pos_t as well.
hipError_t mlp_adam(float* w, float* m, float* v, float* g, uint16_t* wb, uint16_t* packed,
                    const MlpLayout& L, const GradParts& parts, float lr, float b1, float b2,
                    float eps, float c1, float c2, hipStream_t s);
hipError_t mlp_gather(const float* params, const float* u0, const float* y, int64_t n, int64_t q0,
                      int64_t count, uint64_t mult, uint64_t add, const float* norm, uint16_t* a0,
                      float* T, int nout, hipStream_t s);
hipError_t mlp_row_stats(const RowSet& rows, int nrows, int64_t n, float* mean, float* istd,
                         float* sd, float* lo, float* hi, hipStream_t s);
hipError_t mlp_forward(const MlpLayout& L, const uint16_t* wb, const float* w, const float* norm,
                       const uint16_t* a0, int64_t count, MlpActs& acts, float* Y,
                       float* soa_out, int64_t soa_stride, int64_t q0, hipStream_t s);
hipError_t mlp_backward(const MlpLayout& L, const uint16_t* wb, const uint16_t* a0, int64_t B,
                        MlpActs& acts, const float* Y, const float* T, GradParts& parts,
                        double* partial, float* loss, hipStream_t s);
// The split-K weight-gradient partials of every layer (the last launch of
// mlp_backward), from acts.gb and the kept activations.
hipError_t mlp_weight_grads(const MlpLayout& L, const uint16_t* a0, int64_t B, MlpActs& acts,
                            GradParts& parts, hipStream_t s);
// *loss = factor * sum(partial[0 .. count)), one block, fixed order.
hipError_t mlp_loss_sum(const double* partial, int64_t count, double factor, float* loss,
                        hipStream_t s);
// The split-K weight-gradient partials (parts.w) from the item-fragment
// G_l (acts.gb) and A_{l-1} (a0, acts.act) of the fused training path.
hipError_t mlp_weight_grads_if(const MlpLayout& L, int64_t B, MlpActs& acts, const uint16_t* a0,
                               GradParts& parts, hipStream_t s);

// Fragment-major weights of the fused kernels (mlp_fused.hip), for the
// 4 -> 256 -> 256 -> 256 -> 48 network only.  A fragment is 64 lanes x 8
// bf16: the A operand of one 16 x 32 block of W_l for
// v_mfma_f32_16x16x32_bf16; lane 16 g + r holds row r of the block and
// k-slots 8 g .. 8 g + 7, slot 8 g + e holding column perm32(8 g + e) of the
// 32-wide k-block.  Layer 1 (4 inputs) has one k-block, columns 0..3 in
// group 0 and zeros elsewhere; layers 2, 3 have 16 x 8 fragments, layer 4
// 3 x 8, each row block's k-blocks consecutive.
constexpr int kPackFrag = 512;
constexpr int64_t kPackL1 = 0;
constexpr int64_t kPackL2 = kPackL1 + 16 * kPackFrag;
constexpr int64_t kPackL3 = kPackL2 + 128 * kPackFrag;
constexpr int64_t kPackL4 = kPackL3 + 128 * kPackFrag;
constexpr int64_t kPackTotal = kPackL4 + 24 * kPackFrag;

// Logical k-slot (0..31) -> feature inside a 32-wide k-block: lane group g
// holds features 4g..4g+3 of the first 16-row accumulator tile and
// 16+4g..16+4g+3 of the second, so one layer's accumulators are the next
// layer's operands without a shuffle.
__host__ __device__ constexpr int perm32(int k) {
  return (k & 7) < 4 ? 4 * (k >> 3) + (k & 7) : 16 + 4 * (k >> 3) + (k & 7) - 4;
}

// Position of element (row, col) of layer l's W in the packed weights (the
// inverse of the packing: feature j of a k-block sits in group (j & 15) / 4,
// slot j & 3, plus 4 for the second half).
__host__ __device__ inline int64_t packed_pos(int l, int row, int col) {
  const int r16 = row & 15, rb = row >> 4;
  if (l == 0) return kPackL1 + (int64_t)rb * kPackFrag + r16 * 8 + col;
  const int j = col & 31, kb = col >> 5;
  const int g = (j & 15) >> 2, e = (j < 16 ? 0 : 4) + (j & 3);
  const int64_t base = l == 1 ? kPackL2 : (l == 2 ? kPackL3 : kPackL4);
  return base + (int64_t)(rb * 8 + kb) * kPackFrag + (16 * g + r16) * 8 + e;
}

// The fused backward pass reads W_l^T (l = 2, 3, 4) packed the same way
// after them: rows = the layer's 256 inputs, k = its outputs (perm32 order
// inside each 32-wide block; layer 4's 48 outputs zero-padded to two blocks).
constexpr int64_t kPackT2 = kPackTotal;                 // 16 row blocks x 8 k-blocks
constexpr int64_t kPackT3 = kPackT2 + 128 * kPackFrag;  // same
constexpr int64_t kPackT4 = kPackT3 + 128 * kPackFrag;  // 16 row blocks x 2 k-blocks
constexpr int64_t kPackAll = kPackT4 + 32 * kPackFrag;

// Position of element (row, col) of W_l (l = 1, 2, 3: the second to fourth
// layers) in the transposed copy, i.e. of element (col, row) of W_l^T.
__host__ __device__ inline int64_t packed_pos_t(int l, int row, int col) {
  const int r16 = col & 15, rb = col >> 4;
  const int j = row & 31, kb = row >> 5;
  const int g = (j & 15) >> 2, e = (j < 16 ? 0 : 4) + (j & 3);
  const int nkb = l == 3 ? 2 : 8;
  const int64_t base = l == 1 ? kPackT2 : (l == 2 ? kPackT3 : kPackT4);
  return base + (int64_t)(rb * nkb + kb) * kPackFrag + (16 * g + r16) * 8 + e;
}

// Fused inference kernel (mlp_fused.hip): weights re-laid out fragment-major
// by mlp_pack into a buffer of mlp_packed_elems() bf16 values (the forward
// layout, then the transposed one).
int64_t mlp_packed_elems();
hipError_t mlp_pack(const uint16_t* wb, const MlpLayout& L, uint16_t* packed, hipStream_t s);
hipError_t mlp_forward_fused(const MlpLayout& L, const uint16_t* packed, const float* w,
                             const float* norm, const float* params, const float* u0, int64_t n,
                             float* out, int64_t stride, int num_cu, int ns, hipStream_t s);
hipError_t mlp_forward_fused_list(const MlpLayout& L, const uint16_t* packed, const float* w,
                                  const float* norm, const float* params, const float* u0,
                                  int64_t n, int64_t in_stride, const int64_t* idx,
                                  int64_t idx_step, const unsigned long long* n_dev,
                                  int out_compact, float* out, int64_t stride, int num_cu, int ns,
                                  hipStream_t s);
// Item-fragment layout of a bf16 matrix X [item][feature] for the weight-
// gradient products of the fused training path (items padded to whole
// 32-item blocks, features to whole 16-feature blocks, padding zero): the
// fragment of item block kb and feature block fb sits at
// (kb * nfb + fb) * kPackFrag, lane 16 g + r holding feature 16 fb + r of
// items 32 kb + 8 g .. 32 kb + 8 g + 7 -- for G_l^T the A operand and for
// A_{l-1} the B operand of v_mfma_f32_16x16x32_bf16 with k = items.
__host__ __device__ inline int64_t item_frag_pos(int64_t item, int f, int nfb) {
  return ((item >> 5) * nfb + (f >> 4)) * kPackFrag + (16 * ((item & 31) >> 3) + (f & 15)) * 8 +
         (item & 7);
}

// Record width of a staged training set (mlp_stage_items): the normalised
// inputs (rho, x0, y0, z0) and 48 normalised targets of one trajectory.
constexpr int kStageW = 52;
hipError_t mlp_stage_items(const float* params, const float* u0, const float* y, int64_t n,
                           const float* norm, float* D, hipStream_t s);

// The fused training step's forward and backward passes in one launch
// (4-256-256-256-48 network, packed weights with the transposed part): item
// b < B is trajectory (mult * (first + b) + add) mod n of params / u0 [3][n]
// and y [48][n], or of the set staged by mlp_stage_items (`staged`, n
// records; params / u0 / y then unused).  Leaves, in the item-fragment
// layout, the normalised inputs (a0: 16 feature slots, 4 used), A_l of the
// hidden layers (acts.act) and every layer's bf16 output gradient G_l
// (acts.gb); the loss partials (partial [nb], nb = 2 ceil(B / 32) blocks of
// 16 items) and the bias-gradient partials of every layer (parts.b,
// [nb][width]; parts.tiles = nb).  The weight gradients follow with
// mlp_weight_grads_if.
hipError_t mlp_train_fused(const uint16_t* packed, const float* w, const MlpLayout& L,
                           const float* norm, const float* params, const float* u0,
                           const float* y, const float* staged, int64_t n, int64_t first,
                           int64_t B, uint64_t mult, uint64_t add, uint16_t* a0, MlpActs& acts,
                           GradParts& parts, double* partial, hipStream_t s);

}  // namespace ens
