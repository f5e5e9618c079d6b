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

// Split-K factor of the weight-gradient products (K = batch).
constexpr int kSplits = 16;

// Gradient partials of one training step, summed by the Adam kernel:
// w[l] [kSplits][dims[l+1] * dims[l]] split-K partials of dW_l, b[l]
// [tiles][dims[l+1]] partials of db_l over 64-row blocks of the batch.
struct GradParts {
  float* w[kMlpMaxLayers];
  float* b[kMlpMaxLayers];
  int tiles;
};

struct RowSet {
  const float* ptr[64];
};

hipError_t mlp_init(float* w, uint16_t* wb, const MlpLayout& L, uint64_t seed, hipStream_t s);
hipError_t mlp_to_bf16(const float* w, uint16_t* wb, int64_t n, hipStream_t s);
hipError_t mlp_adam(float* w, float* m, float* v, float* g, uint16_t* wb, const MlpLayout& L,
                    const GradParts& parts, float lr, float b1, float b2, float eps, float c1,
                    float c2, hipStream_t s);
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

// Fused inference kernel (mlp_fused.hip): weights re-laid out fragment-major
// by mlp_pack into a buffer of mlp_packed_elems() bf16 values.
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

}  // namespace ens
