// surrogate.hip -- C ABI of the learned surrogate (include/ens.h): model
// storage, normalisation, training, inference, and the audited solve in
// which the Tsit5 solver checks a random 1% of the answers and replaces the
// surrogate wherever it is not validated.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/ens.h"
#include "ens_internal.h"
#include "mlp.h"
#include "philox.h"

namespace {

using ens::DeviceGuard;
using ens::fail;

constexpr int kDims[5] = {4, 256, 256, 256, 48};
constexpr int kBins = 28;  // rho bins of the audit / fallback rule
static_assert(kBins <= 32, "audit_compare gathers a block's flagged bins in one word");
constexpr float kAdamB1 = 0.9f, kAdamB2 = 0.999f, kAdamEps = 1e-8f;

template <class T>
hipError_t alloc(T** p, int64_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)(count > 0 ? count : 1));
}

// ---- audit / fallback kernels ----------------------------------------------

// Append `value` to list[0, cap) where `take`, one atomic per block: the
// waves' ballot counts are combined in LDS and thread 0 reserves the block's
// slots, so a block's entries are contiguous and in thread order.  Every
// thread of the block must call it.
// With step -1 the entries are stored at list[0], list[-1], ... (a list
// that grows from the back of a buffer whose last element `list` points to).
template <int B>
__device__ inline void block_append(bool take, int64_t value, int64_t* list, int64_t cap,
                                    unsigned long long* count, int64_t step = 1) {
  __shared__ unsigned int woff[B / 64];
  __shared__ unsigned long long base;
  const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
  const unsigned long long m = __ballot(take);
  if (lane == 0) woff[wave] = (unsigned int)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int tot = 0;
    for (int w = 0; w < B / 64; ++w) {
      const unsigned int c = woff[w];
      woff[w] = tot;
      tot += c;
    }
    base = tot ? atomicAdd(count, (unsigned long long)tot) : 0ull;
  }
  __syncthreads();
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t slot = (int64_t)(base + woff[wave] + (unsigned long long)__popcll(m & below));
  if (take && slot < cap) list[slot * step] = value;
}

constexpr int kSelBlock = 1024;  // threads per block of the selection kernels

__device__ inline int rho_bin(float rho, const float* norm) {
  const float lo = norm[ens::kInLo], hi = norm[ens::kInHi];
  const float f = (rho - lo) / fmaxf(hi - lo, 1e-30f) * (float)kBins;
  const int b = (int)floorf(f);
  return b < 0 ? 0 : (b >= kBins ? kBins - 1 : b);
}

__device__ inline bool in_box(const float* params, const float* u0, int64_t n, int64_t i,
                              const float* norm) {
  const float x[4] = {params[n + i], u0[i], u0[n + i], u0[2 * n + i]};
  bool ok = true;
#pragma unroll
  for (int f = 0; f < 4; ++f) ok = ok && x[f] >= norm[ens::kInLo + f] && x[f] <= norm[ens::kInHi + f];
  return ok;
}

// Bernoulli(frac) audit draw per query from Philox4x32-10 (counter = query id).
__global__ void __launch_bounds__(kSelBlock) select_audit(int64_t n, uint32_t thr, uint64_t seed,
                                                          int64_t* list, int64_t cap,
                                                          unsigned long long* count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool take = false;
  if (i < n) {
    const ens::Philox4 r = ens::philox4x32_10((uint32_t)i, (uint32_t)((uint64_t)i >> 32), 7u, 0u,
                                              (uint32_t)seed, (uint32_t)(seed >> 32));
    take = r.x0 < thr;
  }
  block_append<kSelBlock>(take, i, list, cap, count);
}

// For each audited query k (list entry i): normwise error of the network's
// answer net[.][k] against the solver's sol[.][k] (max over save times of
// ||net - sol||_inf / ||sol||_inf); a bin with any error above tol (or
// non-finite) is flagged; the solver answer goes to out[.][i].
__global__ void audit_compare(const int64_t* list, const unsigned long long* count, int64_t cap,
                              const float* sol, const float* net, float* out, int64_t n,
                              int n_save, int ncomp,
                              const float* params, const float* norm, float tol,
                              unsigned int* bins, uint8_t* used, unsigned int* max_err_bits) {
  __shared__ unsigned int bmax, bflag;
  if (threadIdx.x == 0) bmax = bflag = 0u;
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cnt = (int64_t)(*count < (unsigned long long)cap ? *count : cap);
  if (k < cnt) {
    const int64_t i = list[k];
    float err = 0.0f;
    for (int j = 0; j < n_save; ++j) {
      float num = 0.0f, den = 0.0f;
      for (int c = 0; c < ncomp; ++c) {
        const int64_t row = (int64_t)j * ncomp + c;
        const float s = sol[row * cap + k];
        const float g = net[row * cap + k];
        num = fmaxf(num, fabsf(g - s));
        den = fmaxf(den, fabsf(s));
        out[row * n + i] = s;
      }
      const float e = num / den;
      err = (e == e) ? fmaxf(err, e) : 3.0e38f;
    }
    if (!(err <= tol)) atomicOr(&bflag, 1u << rho_bin(params[n + i], norm));
    if (used) used[i] = 1;
    atomicMax(&bmax, __float_as_uint(err));  // err >= 0: the bits order as the floats
  }
  __syncthreads();  // one global update per block
  if (threadIdx.x == 0) {
    if (bmax) atomicMax(max_err_bits, bmax);
    for (int b = 0; b < kBins; ++b)
      if (bflag & (1u << b)) atomicOr(&bins[b], 1u);
  }
}

// The queries left after the audit: to the solver (outside the training box
// or in a flagged rho bin; flag 2, list front, count[0]) or to the network
// (list back, count[1]).
__global__ void __launch_bounds__(kSelBlock) select_split(int64_t n, const float* params,
                                                          const float* u0, const float* norm,
                                                          const unsigned int* bins,
                                                          uint8_t* used, int64_t* list,
                                                          unsigned long long* count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool fb = false, nw = false;
  if (i < n && used[i] == 0) {
    fb = !in_box(params, u0, n, i, norm) || bins[rho_bin(params[n + i], norm)] != 0u;
    nw = !fb;
    if (fb) used[i] = 2;
  }
  block_append<kSelBlock>(fb, i, list, n, count);
  block_append<kSelBlock>(nw, i, list + (n - 1), n, count + 1, -1);
}

// net[row][k] = out[row][list[k]] for the first count[0] entries (rows of
// 48 outputs, row strides cap and n).
__global__ void gather_answers(const int64_t* list, const unsigned long long* count, int64_t cap,
                               const float* out, int64_t n, float* net) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cnt = (int64_t)(*count < (unsigned long long)cap ? *count : cap);
  if (k >= cnt) return;
  const int64_t i = list[k];
  for (int row = 0; row < kDims[4]; ++row) net[row * cap + k] = out[row * n + i];
}

__global__ void zero_u8(uint8_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void zero_words(unsigned int* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// report = {audited, fallback, flagged bins, max audit error}
__global__ void write_report(const unsigned long long* counts, const unsigned int* bins,
                             const unsigned int* max_err_bits, float* report) {
  if (threadIdx.x != 0) return;
  int flagged = 0;
  for (int b = 0; b < kBins; ++b) flagged += bins[b] != 0u;
  report[0] = (float)counts[0];
  report[1] = (float)counts[1];
  report[2] = (float)flagged;
  report[3] = __uint_as_float(*max_err_bits);
}

unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }
unsigned sel_grid(int64_t n) { return (unsigned)((n + kSelBlock - 1) / kSelBlock); }

}  // namespace

struct ens_surrogate {
  int device = 0;
  ens::MlpLayout L{};
  float* w = nullptr;
  uint16_t* wb = nullptr;
  // fragment-major copy of wb for the fused kernels, rewritten by every writer
  // of wb (create, copy, load, Adam) so it never goes stale
  uint16_t* packed = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  float* norm = nullptr;
  int64_t step = 0;
  // training workspace (batch capacity)
  int64_t cap_batch = 0;
  uint16_t* a0 = nullptr;
  float* z[3] = {};
  uint16_t* act[3] = {};
  float* Y = nullptr;
  float* T = nullptr;
  uint16_t* gb[4] = {};  // bf16 output gradient of every layer
  int64_t cap_staged = 0;
  float* staged = nullptr;  // a training call's set, item-major and normalised
  double* partial = nullptr;  // per 64-row block loss sums
  float* wparts = nullptr;    // split-K partials of the weight gradients, every layer
  float* bparts = nullptr;    // 64-row block partials of the bias gradients, every layer
  // inference workspace (chunk capacity)
  int64_t cap_chunk = 0;
  uint16_t* ia0 = nullptr;
  uint16_t* iact[2] = {};
  // audited solve workspace
  int64_t cap_n = 0, cap_audit = 0;
  int64_t* alist = nullptr;
  int64_t* flist = nullptr;
  float* scratch = nullptr;  // the solver's answers for the audited queries
  float* netans = nullptr;   // the network's answers for them
  uint8_t* used = nullptr;
  unsigned long long* counts = nullptr;  // [0] audited, [1] fallback, [2] network
  unsigned int* words = nullptr;         // [0, kBins) bins, [kBins] max error bits
};

namespace {

void free_all(ens_surrogate* s) {
  void* ps[] = {s->w, s->wb, s->packed, s->m, s->v, s->grad, s->norm, s->a0, s->z[0], s->z[1], s->z[2],
                s->act[0], s->act[1], s->act[2], s->Y, s->T, s->gb[0], s->gb[1], s->gb[2],
                s->gb[3], s->partial, s->wparts, s->bparts, s->staged, s->ia0, s->iact[0], s->iact[1], s->alist, s->flist,
                s->scratch, s->netans, s->used, s->counts, s->words};
  for (void* p : ps)
    if (p) (void)hipFree(p);
}

int64_t weight_count(const ens::MlpLayout& L) {
  int64_t w = 0;
  for (int l = 0; l < L.layers; ++l) w += (int64_t)L.dims[l] * L.dims[l + 1];
  return w;
}

// Where the step's gradient partials go inside the model's two buffers; the
// bias partials have one row per `tiles` block of the batch (64 items in the
// tiled backward, 16 in the fused one).
ens::GradParts grad_parts(const ens_surrogate* s, int64_t tiles) {
  ens::GradParts P{};
  int64_t wo = 0, bo = 0;
  for (int l = 0; l < s->L.layers; ++l) {
    P.w[l] = s->wparts + wo;
    P.b[l] = s->bparts + bo;
    wo += (int64_t)ens::kSplitsMax * s->L.dims[l] * s->L.dims[l + 1];
    bo += tiles * s->L.dims[l + 1];
  }
  return P;
}

int ensure_batch(ens_ctx* c, ens_surrogate* s, int64_t B) {
  if (B <= s->cap_batch) return ENS_OK;
  void* old[] = {s->a0, s->z[0], s->z[1], s->z[2], s->act[0], s->act[1], s->act[2], s->Y, s->T,
                 s->gb[0], s->gb[1], s->gb[2], s->gb[3], s->partial, s->wparts, s->bparts};
  for (void* p : old)
    if (p) (void)hipFree(p);
  const int H = kDims[1], O = kDims[4];
  // the fused path's blocks of 16 items and its item-fragment layouts
  // (items padded to whole 32-item blocks, a0 to 16 feature slots) are the
  // larger of the two paths' needs
  const int64_t Bp = (B + 31) / 32 * 32, blocks = Bp / 16;
  bool ok = alloc(&s->a0, Bp * 16) == hipSuccess && alloc(&s->Y, B * O) == hipSuccess &&
            alloc(&s->T, B * O) == hipSuccess && alloc(&s->partial, blocks) == hipSuccess &&
            alloc(&s->wparts, (int64_t)ens::kSplitsMax * weight_count(s->L)) == hipSuccess &&
            alloc(&s->bparts, blocks * (s->L.total - weight_count(s->L))) == hipSuccess;
  for (int l = 0; l < 3 && ok; ++l)
    ok = alloc(&s->z[l], B * H) == hipSuccess && alloc(&s->act[l], Bp * H) == hipSuccess;
  for (int l = 0; l < 4 && ok; ++l) ok = alloc(&s->gb[l], Bp * kDims[l + 1]) == hipSuccess;
  if (!ok) {
    s->cap_batch = 0;
    return fail(c, ENS_ENOMEM, "cannot allocate the training workspace for batch %lld",
                (long long)B);
  }
  s->cap_batch = B;
  return ENS_OK;
}

int ensure_chunk(ens_ctx* c, ens_surrogate* s, int64_t C) {
  if (C <= s->cap_chunk) return ENS_OK;
  void* old[] = {s->ia0, s->iact[0], s->iact[1]};
  for (void* p : old)
    if (p) (void)hipFree(p);
  if (alloc(&s->ia0, C * kDims[0]) != hipSuccess || alloc(&s->iact[0], C * kDims[1]) != hipSuccess ||
      alloc(&s->iact[1], C * kDims[1]) != hipSuccess) {
    s->cap_chunk = 0;
    return fail(c, ENS_ENOMEM, "cannot allocate the inference workspace");
  }
  s->cap_chunk = C;
  return ENS_OK;
}

int check_model(ens_ctx* c, ens_surrogate* s) {
  if (!c) return ENS_EINVAL;
  c->err.clear();
  if (!s) return fail(c, ENS_EINVAL, "null surrogate");
  if (s->device != c->device)
    return fail(c, ENS_EINVAL, "surrogate lives on device %d, context on %d", s->device,
                c->device);
  return ENS_OK;
}

int predict(ens_ctx* c, ens_surrogate* s, const float* params, const float* u0, int64_t n,
            float* out, hipStream_t st) {
  if (c->mlp_tile != 0) {  // fused kernel on the packed copy of the bf16 weights
    hipError_t e = ens::mlp_forward_fused(s->L, s->packed, s->w, s->norm, params, u0, n, out, n,
                                          c->num_cu, c->mlp_tile, st);
    if (e != hipSuccess) return fail(c, ENS_EDEVICE, "surrogate forward: %s", hipGetErrorString(e));
    return ENS_OK;
  }
  const int64_t C = n < ((int64_t)1 << 18) ? n : ((int64_t)1 << 18);
  int rc = ensure_chunk(c, s, C);
  if (rc != ENS_OK) return rc;
  ens::MlpActs acts{};
  acts.keep_all = false;
  acts.act[0] = s->iact[0];
  acts.act[1] = s->iact[1];
  for (int64_t q0 = 0; q0 < n; q0 += C) {
    const int64_t cnt = (n - q0) < C ? (n - q0) : C;
    hipError_t e = ens::mlp_gather(params, u0, nullptr, n, q0, cnt, 1, 0, s->norm, s->ia0,
                                   nullptr, kDims[4], st);
    if (e == hipSuccess)
      e = ens::mlp_forward(s->L, s->wb, s->w, s->norm, s->ia0, cnt, acts, nullptr, out, n, q0, st);
    if (e != hipSuccess) return fail(c, ENS_EDEVICE, "surrogate forward: %s", hipGetErrorString(e));
  }
  return ENS_OK;
}

// staged: the training set staged item-major by mlp_stage_items (fused path
// only), or null to gather from params / u0 / y.
int train_step(ens_ctx* c, ens_surrogate* s, const float* params, const float* u0,
               const float* y, int64_t n, int64_t first, int64_t B, uint64_t mult, uint64_t add,
               double lr, float* loss, hipStream_t st, const float* staged = nullptr) {
  int rc = ensure_batch(c, s, B);
  if (rc != ENS_OK) return rc;
  ens::MlpActs acts{};
  acts.keep_all = true;
  for (int l = 0; l < 3; ++l) {
    acts.z[l] = s->z[l];
    acts.act[l] = s->act[l];
  }
  for (int l = 0; l < 4; ++l) acts.gb[l] = s->gb[l];
  hipError_t e;
  ens::GradParts parts;
  if (c->mlp_tile != 0) {
    // gather, forward, loss and input gradients in one feature-split
    // launch; the weight gradients (and bias sums) in one more; Adam
    parts = grad_parts(s, 2 * ((B + 31) / 32));
    e = ens::mlp_train_fused(s->packed, s->w, s->L, s->norm, params, u0, y, staged, n, first,
                             B, mult, add, s->a0, acts, parts, s->partial, st);
    if (e == hipSuccess && loss)
      e = ens::mlp_loss_sum(s->partial, parts.tiles, 1.0 / (double)(B * kDims[4]), loss, st);
    if (e == hipSuccess) e = ens::mlp_weight_grads_if(s->L, B, acts, s->a0, parts, st);
  } else {
    parts = grad_parts(s, (B + 63) / 64);
    e = ens::mlp_gather(params, u0, y, n, first, B, mult, add, s->norm, s->a0, s->T, kDims[4], st);
    if (e == hipSuccess)
      e = ens::mlp_forward(s->L, s->wb, s->w, s->norm, s->a0, B, acts, s->Y, nullptr, 0, 0, st);
    if (e == hipSuccess)
      e = ens::mlp_backward(s->L, s->wb, s->a0, B, acts, s->Y, s->T, parts, s->partial, loss, st);
  }
  if (e == hipSuccess) {
    s->step += 1;
    const double c1 = 1.0 / (1.0 - std::pow((double)kAdamB1, (double)s->step));
    const double c2 = 1.0 / (1.0 - std::pow((double)kAdamB2, (double)s->step));
    e = ens::mlp_adam(s->w, s->m, s->v, s->grad, s->wb, s->packed, s->L, parts, (float)lr,
                      kAdamB1, kAdamB2, kAdamEps, (float)c1, (float)c2, st);
  }
  if (e != hipSuccess) return fail(c, ENS_EDEVICE, "surrogate train step: %s", hipGetErrorString(e));
  return ENS_OK;
}

uint64_t splitmix(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t gcd(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace

namespace {

// Workspace of one audited solve: audit list, the split list (fallback
// queries from the front, network queries from the back), the solver's and
// the network's answers for the audited queries, per-query flags, the three
// list counters and the bin flags (+ max error bits).  The model's own lazily
// grown buffers, or views into the static workspace below.
struct AuditWs {
  int64_t* alist;
  int64_t* flist;
  float* answers;
  float* net;                  // network answers of the audited queries [48][cap_audit]
  uint8_t* used;
  unsigned long long* counts;  // [0] audited, [1] fallback, [2] network
  unsigned int* words;         // [0, kBins) bins, [kBins] max error bits
  int64_t cap_audit;
};

// Audit-list capacity for n queries at audit_frac: 1.5x the expected count
// plus 4096, far beyond any Bernoulli fluctuation.
int64_t audit_capacity(double audit_frac, int64_t n) {
  return (int64_t)std::ceil(audit_frac * (double)n * 1.5) + 4096;
}

int check_solve_args(ens_ctx* c, ens_surrogate* s, const float* params, const float* u0,
                     const double* tspan, double abstol, double reltol, const double* save_times,
                     int n_save, int64_t n, double audit_frac, double fallback_tol,
                     const float* out) {
  int rc = check_model(c, s);
  if (rc != ENS_OK) return rc;
  if (n < 0 || n > ENS_MAX_TRAJ) return fail(c, ENS_EINVAL, "n out of range [0, ENS_MAX_TRAJ]");
  if (n_save * 3 != kDims[4]) return fail(c, ENS_EINVAL, "the surrogate predicts 16 save times");
  if (!(audit_frac >= 0.0 && audit_frac <= 1.0) || !(fallback_tol > 0.0))
    return fail(c, ENS_EINVAL, "audit_frac in [0, 1] and fallback_tol > 0 required");
  if (!save_times || !(abstol > 0.0) || !(reltol > 0.0))
    return fail(c, ENS_EINVAL, "save_times and positive tolerances required");
  for (int j = 0; j < n_save; ++j)
    if (!(save_times[j] > (j ? save_times[j - 1] : 0.0)) || !(save_times[j] <= 1.0))
      return fail(c, ENS_EINVAL, "save_times must be strictly increasing in (0, 1]");
  if (n > 0 && (!params || !u0 || !tspan || !out))
    return fail(c, ENS_EINVAL, "null device array");
  return ENS_OK;
}

// ---- the static workspace of ens_surrogate_solve_static ---------------------
// One copy per GPU, held until the process ends; every static call on a GPU
// shares it.  Layout (bytes): split list int64 [Q], audit list int64 [A],
// audited answers of the solver and of the network float [48][A] each, flags
// uint8 [Q], counters uint64 [3], bin words uint32 [kBins + 1], with
// Q = ENS_STATIC_MAX_QUERIES, A = kStaticAudit.
constexpr int64_t kStaticAudit = 40960;  // audit_frac up to 2% at the largest n
constexpr int64_t kOffFlist = 0;
constexpr int64_t kOffAlist = kOffFlist + 8 * ENS_STATIC_MAX_QUERIES;
constexpr int64_t kOffAnswers = kOffAlist + 8 * kStaticAudit;
constexpr int64_t kOffNet = kOffAnswers + 4 * 48 * kStaticAudit;
constexpr int64_t kOffUsed = kOffNet + 4 * 48 * kStaticAudit;
constexpr int64_t kOffCounts = (kOffUsed + ENS_STATIC_MAX_QUERIES + 255) / 256 * 256;
constexpr int64_t kOffWords = kOffCounts + 24;
constexpr int64_t kScratchBytes = kOffWords + 4 * (kBins + 1);
static_assert(kOffCounts % 8 == 0 && kOffAnswers % 4 == 0 && kOffNet % 4 == 0,
              "aligned counters and answers");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
unsigned char* g_scratch_addr[kMaxDevices] = {};
std::mutex g_scratch_mu;

}  // namespace

namespace ens {
// Device address of this GPU's copy of the static workspace, looked up once
// per device (ens_create calls it with the device current; the host-side name
// of the array is not a device address).
int init_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return ENS_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr[device]) return ENS_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return ENS_EDEVICE;
  g_scratch_addr[device] = static_cast<unsigned char*>(ptr);
  return ENS_OK;
}
}  // namespace ens

namespace {

unsigned char* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_addr[device];
}

// The audited solve on a given workspace (section 5.2's ensemble solve as the
// auditor and fallback of the learned answers).
int audited_solve(ens_ctx* c, ens_surrogate* s, const float* params, const float* u0,
                  const double* tspan, double abstol, double reltol, const double* save_times,
                  int n_save, int64_t n, double audit_frac, double fallback_tol,
                  uint64_t audit_seed, float* out, float* report, const AuditWs& ws,
                  hipStream_t st) {
  hipError_t e = hipSuccess;
#define ENS_TRY(x)                                                                   \
  do {                                                                               \
    if ((e = (x)) != hipSuccess)                                                     \
      return fail(c, ENS_EDEVICE, "surrogate solve: %s", hipGetErrorString(e));     \
  } while (0)
  hipLaunchKernelGGL(zero_u8, dim3(grid_of(n)), dim3(256), 0, st, ws.used, n);
  ENS_TRY(hipGetLastError());
  hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, st, ws.words, kBins + 1);
  ENS_TRY(hipGetLastError());
  hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, st,
                     reinterpret_cast<unsigned int*>(ws.counts), 6);
  ENS_TRY(hipGetLastError());

  // 1. audit sample: Bernoulli(audit_frac) per query
  const double thr_d = std::floor(audit_frac * 4294967296.0);
  const uint32_t thr = thr_d >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)thr_d;
  hipLaunchKernelGGL(select_audit, dim3(sel_grid(n)), dim3(kSelBlock), 0, st, n, thr, audit_seed,
                     ws.alist, ws.cap_audit, ws.counts);
  ENS_TRY(hipGetLastError());

  // 2. the network's answers for the audited queries (fused kernel: only
  // those; tiled path: every query into out, the audited ones gathered)
  const bool fused = c->mlp_tile != 0;
  int rc = ENS_OK;
  if (fused) {
    ENS_TRY(ens::mlp_forward_fused_list(s->L, s->packed, s->w, s->norm, params, u0,
                                        ws.cap_audit, n, ws.alist, 1, ws.counts, 1, ws.net,
                                        ws.cap_audit, c->num_cu, c->mlp_tile, st));
  } else {
    rc = predict(c, s, params, u0, n, out, st);
    if (rc != ENS_OK) return rc;
    hipLaunchKernelGGL(gather_answers, dim3(grid_of(ws.cap_audit)), dim3(256), 0, st, ws.alist,
                       ws.counts, ws.cap_audit, out, n, ws.net);
    ENS_TRY(hipGetLastError());
  }

  // 3. the solver's answers for the audited queries (sorted-form Tsit5, FP32,
  // count read on the device)
  ens::LaunchArgs a{};
  a.n = ws.cap_audit;
  a.in_stride = n;
  a.out_stride = ws.cap_audit;
  a.params = params;
  a.u0 = u0;
  a.tspan = tspan;
  a.out = ws.answers;
  a.idx = ws.alist;
  a.n_dev = ws.counts;
  a.scatter = 0;
  a.queue = c->queue;
  a.atol = abstol;
  a.rtol = reltol;
  a.h0 = 0.0;
  a.maxiters = (int64_t)c->maxiters;
  a.n_save = n_save;
  a.tspan_bcast = c->tspan_bcast;
  a.refill = c->refill;
  a.tpl = 1;
  a.dense = c->save_mode == 1;  // the context's save mode, as in ens_solve
  for (int j = 0; j < n_save; ++j) a.theta[j] = save_times[j];
  const int saved_prec = c->precision;
  c->precision = 32;
  // cost-sorted form (block 256): it reads the device-side count, the index
  // list and the scattered output columns as the other forms do, and is the
  // fastest on Lorenz (about 5.5 ms against 7.6 for the persistent form on a
  // full 2^24 ensemble with landing saves)
  ens::LaunchCfg cfg{2, 256, 0};
  rc = ens::launch_solve(c, ENS_SYS_LORENZ, ENS_ALG_TSIT5, a, cfg, st);
  c->precision = saved_prec;
  if (rc != ENS_OK) return rc;

  // 4. compare, flag bins, return the solver's answer for audited queries
  hipLaunchKernelGGL(audit_compare, dim3(grid_of(ws.cap_audit)), dim3(256), 0, st, ws.alist,
                     ws.counts, ws.cap_audit, ws.answers, ws.net, out, n, n_save, 3, params,
                     s->norm, (float)fallback_tol, ws.words, ws.used, ws.words + kBins);
  ENS_TRY(hipGetLastError());

  // 5. the rest: fallback set (outside the box or in a flagged bin) from the
  // front of the split list, the network's queries from its back
  hipLaunchKernelGGL(select_split, dim3(sel_grid(n)), dim3(kSelBlock), 0, st, n, params, u0,
                     s->norm, ws.words, ws.used, ws.flist, ws.counts + 1);
  ENS_TRY(hipGetLastError());

  // 6. the network answers its queries straight into out (already there on
  // the tiled path)
  if (fused)
    ENS_TRY(ens::mlp_forward_fused_list(s->L, s->packed, s->w, s->norm, params, u0, n, n,
                                        ws.flist + (n - 1), -1, ws.counts + 2, 0, out, n,
                                        c->num_cu, c->mlp_tile, st));

  // 7. the solver answers the fallback set straight into out
  a.n = n;
  a.out = out;
  a.out_stride = n;
  a.idx = ws.flist;
  a.n_dev = ws.counts + 1;
  a.scatter = 1;
  c->precision = 32;
  rc = ens::launch_solve(c, ENS_SYS_LORENZ, ENS_ALG_TSIT5, a, cfg, st);
  c->precision = saved_prec;
  if (rc != ENS_OK) return rc;

  if (report) {
    hipLaunchKernelGGL(write_report, dim3(1), dim3(64), 0, st, ws.counts, ws.words,
                       ws.words + kBins, report);
    ENS_TRY(hipGetLastError());
  }
#undef ENS_TRY
  return ENS_OK;
}

}  // namespace

extern "C" {

int ens_surrogate_create(ens_ctx* c, uint64_t seed, ens_surrogate** out) {
  if (!c || !out) return ENS_EINVAL;
  c->err.clear();
  *out = nullptr;
  DeviceGuard g(c->device);
  if (!g.ok) return fail(c, ENS_EDEVICE, "cannot make device %d current", c->device);
  ens_surrogate* s = new (std::nothrow) ens_surrogate();
  if (!s) return ENS_ENOMEM;
  s->device = c->device;
  s->L = ens::make_layout(kDims, 4);
  const int64_t P = s->L.total;
  bool ok = alloc(&s->w, P) == hipSuccess && alloc(&s->wb, P) == hipSuccess &&
            alloc(&s->packed, ens::mlp_packed_elems()) == hipSuccess &&
            alloc(&s->m, P) == hipSuccess && alloc(&s->v, P) == hipSuccess &&
            alloc(&s->grad, P) == hipSuccess && alloc(&s->norm, ens::kNormSize) == hipSuccess &&
            alloc(&s->counts, 3) == hipSuccess && alloc(&s->words, kBins + 1) == hipSuccess;
  if (ok) ok = hipMemset(s->m, 0, sizeof(float) * P) == hipSuccess &&
               hipMemset(s->v, 0, sizeof(float) * P) == hipSuccess &&
               hipMemset(s->grad, 0, sizeof(float) * P) == hipSuccess;
  if (ok) {
    // identity normalisation until ens_surrogate_fit_norm is called
    float nh[ens::kNormSize];
    for (int k = 0; k < ens::kNormSize; ++k) nh[k] = 0.0f;
    for (int f = 0; f < 4; ++f) {
      nh[ens::kInIStd + f] = 1.0f;
      nh[ens::kInLo + f] = -3.0e38f;
      nh[ens::kInHi + f] = 3.0e38f;
    }
    for (int o = 0; o < 48; ++o) nh[ens::kOutIStd + o] = nh[ens::kOutStd + o] = 1.0f;
    ok = hipMemcpy(s->norm, nh, sizeof nh, hipMemcpyHostToDevice) == hipSuccess;
  }
  if (ok) ok = ens::mlp_init(s->w, s->wb, s->L, seed, nullptr) == hipSuccess &&
               ens::mlp_pack(s->wb, s->L, s->packed, nullptr) == hipSuccess &&
               hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    free_all(s);
    delete s;
    return fail(c, ENS_ENOMEM, "cannot allocate or initialise the surrogate");
  }
  *out = s;
  return ENS_OK;
}

int ens_surrogate_destroy(ens_surrogate* s) {
  if (!s) return ENS_OK;
  {
    DeviceGuard g(s->device);
    free_all(s);
  }
  delete s;
  return ENS_OK;
}

int ens_surrogate_copy(ens_ctx* c, ens_surrogate* s, int which, void* p, int to_model,
                       void* stream) {
  int rc = check_model(c, s);
  if (rc != ENS_OK) return rc;
  if (!p || (to_model != 0 && to_model != 1)) return fail(c, ENS_EINVAL, "bad copy arguments");
  void* buf = nullptr;
  size_t bytes = sizeof(float) * (size_t)s->L.total;
  switch (which) {
    case ENS_SURR_MASTER: buf = s->w; break;
    case ENS_SURR_WEIGHTS_BF16: buf = s->wb; bytes = sizeof(uint16_t) * (size_t)s->L.total; break;
    case ENS_SURR_GRAD: buf = s->grad; break;
    case ENS_SURR_ADAM_M: buf = s->m; break;
    case ENS_SURR_ADAM_V: buf = s->v; break;
    case ENS_SURR_NORM: buf = s->norm; bytes = sizeof(float) * ens::kNormSize; break;
    default: return fail(c, ENS_EINVAL, "unknown surrogate buffer %d", which);
  }
  DeviceGuard g(c->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = to_model ? hipMemcpyAsync(buf, p, bytes, hipMemcpyDeviceToDevice, st)
                          : hipMemcpyAsync(p, buf, bytes, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && to_model && which == ENS_SURR_MASTER)
    e = ens::mlp_to_bf16(s->w, s->wb, s->L.total, st);
  if (e == hipSuccess && to_model && (which == ENS_SURR_MASTER || which == ENS_SURR_WEIGHTS_BF16))
    e = ens::mlp_pack(s->wb, s->L, s->packed, st);
  return e == hipSuccess ? ENS_OK : fail(c, ENS_EDEVICE, "%s", hipGetErrorString(e));
}

// File image: "ENSSURR1", uint32 version 1, uint32 parameter count, int64
// Adam step, uint32 normalisation size, then FP32 master weights, Adam
// first and second moments and the normalisation, little-endian.
int ens_surrogate_save(ens_ctx* c, ens_surrogate* s, const char* path) {
  int rc = check_model(c, s);
  if (rc != ENS_OK) return rc;
  if (!path) return fail(c, ENS_EINVAL, "null path");
  DeviceGuard g(c->device);
  const size_t P = (size_t)s->L.total;
  float* h = static_cast<float*>(std::malloc(sizeof(float) * (3 * P + ens::kNormSize)));
  if (!h) return fail(c, ENS_ENOMEM, "cannot allocate host staging for the model");
  bool ok = hipDeviceSynchronize() == hipSuccess &&
            hipMemcpy(h, s->w, sizeof(float) * P, hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(h + P, s->m, sizeof(float) * P, hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(h + 2 * P, s->v, sizeof(float) * P, hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(h + 3 * P, s->norm, sizeof(float) * ens::kNormSize,
                      hipMemcpyDeviceToHost) == hipSuccess;
  if (!ok) {
    std::free(h);
    return fail(c, ENS_EDEVICE, "cannot read the model from the device");
  }
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) {
    std::free(h);
    return fail(c, ENS_EINVAL, "cannot open %s for writing", tmp.c_str());
  }
  const uint32_t ver = 1, np = (uint32_t)P, nn = (uint32_t)ens::kNormSize;
  const int64_t step = s->step;
  ok = std::fwrite("ENSSURR1", 1, 8, f) == 8 && std::fwrite(&ver, 4, 1, f) == 1 &&
       std::fwrite(&np, 4, 1, f) == 1 && std::fwrite(&step, 8, 1, f) == 1 &&
       std::fwrite(&nn, 4, 1, f) == 1 &&
       std::fwrite(h, sizeof(float), 3 * P + nn, f) == 3 * P + nn;
  ok = (std::fclose(f) == 0) && ok;
  std::free(h);
  if (!ok || std::rename(tmp.c_str(), path) != 0)
    return fail(c, ENS_EINVAL, "cannot write %s", path);
  return ENS_OK;
}

int ens_surrogate_load(ens_ctx* c, ens_surrogate* s, const char* path) {
  int rc = check_model(c, s);
  if (rc != ENS_OK) return rc;
  if (!path) return fail(c, ENS_EINVAL, "null path");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(c, ENS_EINVAL, "cannot open %s", path);
  const size_t P = (size_t)s->L.total;
  char magic[8];
  uint32_t ver = 0, np = 0, nn = 0;
  int64_t step = 0;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "ENSSURR1", 8) == 0 &&
            std::fread(&ver, 4, 1, f) == 1 && std::fread(&np, 4, 1, f) == 1 &&
            std::fread(&step, 8, 1, f) == 1 && std::fread(&nn, 4, 1, f) == 1 && ver == 1 &&
            np == (uint32_t)P && nn == (uint32_t)ens::kNormSize && step >= 0;
  float* h = ok ? static_cast<float*>(std::malloc(sizeof(float) * (3 * P + nn))) : nullptr;
  ok = ok && h && std::fread(h, sizeof(float), 3 * P + nn, f) == 3 * P + nn &&
       std::fgetc(f) == EOF;
  std::fclose(f);
  if (!ok) {
    std::free(h);
    return fail(c, ENS_EINVAL, "%s is not a surrogate file of this architecture", path);
  }
  DeviceGuard g(c->device);
  ok = hipDeviceSynchronize() == hipSuccess &&
       hipMemcpy(s->w, h, sizeof(float) * P, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(s->m, h + P, sizeof(float) * P, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(s->v, h + 2 * P, sizeof(float) * P, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(s->norm, h + 3 * P, sizeof(float) * nn, hipMemcpyHostToDevice) == hipSuccess &&
       ens::mlp_to_bf16(s->w, s->wb, s->L.total, nullptr) == hipSuccess &&
       ens::mlp_pack(s->wb, s->L, s->packed, nullptr) == hipSuccess &&
       hipDeviceSynchronize() == hipSuccess;
  std::free(h);
  if (!ok) return fail(c, ENS_EDEVICE, "cannot write the model to the device");
  s->step = step;
  return ENS_OK;
}

int ens_surrogate_set_step(ens_surrogate* s, int64_t step) {
  if (!s || step < 0) return ENS_EINVAL;
  s->step = step;
  return ENS_OK;
}

int ens_surrogate_get_step(const ens_surrogate* s, int64_t* step) {
  if (!s || !step) return ENS_EINVAL;
  *step = s->step;
  return ENS_OK;
}

int ens_surrogate_fit_norm(ens_ctx* c, ens_surrogate* s, const float* params, const float* u0,
                           const float* y, int64_t n, void* stream) {
  int rc = check_model(c, s);
  if (rc != ENS_OK) return rc;
  if (n < 2 || n > ENS_MAX_TRAJ || !params || !u0 || !y)
    return fail(c, ENS_EINVAL, "need 2 <= n <= ENS_MAX_TRAJ and device arrays");
  DeviceGuard g(c->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  ens::RowSet in{}, outr{};
  in.ptr[0] = params + n;  // rho
  for (int f = 0; f < 3; ++f) in.ptr[1 + f] = u0 + (int64_t)f * n;
  for (int o = 0; o < kDims[4]; ++o) outr.ptr[o] = y + (int64_t)o * n;
  hipError_t e = ens::mlp_row_stats(in, 4, n, s->norm + ens::kInMean, s->norm + ens::kInIStd,
                                    nullptr, s->norm + ens::kInLo, s->norm + ens::kInHi, st);
  if (e == hipSuccess)
    e = ens::mlp_row_stats(outr, kDims[4], n, s->norm + ens::kOutMean, s->norm + ens::kOutIStd,
                           s->norm + ens::kOutStd, nullptr, nullptr, st);
  return e == hipSuccess ? ENS_OK : fail(c, ENS_EDEVICE, "%s", hipGetErrorString(e));
}

int ens_surrogate_train_step(ens_ctx* c, ens_surrogate* s, const float* params, const float* u0,
                             const float* y, int64_t n, int64_t first, int64_t batch,
                             uint64_t mult, uint64_t add, double lr, float* loss, void* stream) {
  int rc = check_model(c, s);
  if (rc != ENS_OK) return rc;
  if (n < 1 || n > ENS_MAX_TRAJ || batch < 1 || batch > ENS_SURR_MAX_BATCH || !params || !u0 ||
      !y || !(lr >= 0.0))
    return fail(c, ENS_EINVAL, "bad training arguments");
  if (gcd(mult % (uint64_t)n, (uint64_t)n) != 1 && n > 1)
    return fail(c, ENS_EINVAL, "mult must be coprime with n (a permutation of the set)");
  DeviceGuard g(c->device);
  return train_step(c, s, params, u0, y, n, first, batch, mult, add, lr, loss,
                    static_cast<hipStream_t>(stream));
}

int ens_surrogate_train(ens_ctx* c, ens_surrogate* s, const float* params, const float* u0,
                        const float* y, int64_t n, int epochs, int64_t batch, double lr_max,
                        double lr_min, uint64_t seed, float* epoch_loss, void* stream) {
  int rc = check_model(c, s);
  if (rc != ENS_OK) return rc;
  if (n < 1 || n > ENS_MAX_TRAJ || batch < 1 || batch > n || batch > ENS_SURR_MAX_BATCH ||
      epochs < 1 || !params || !u0 || !y ||
      !(lr_max >= lr_min) || !(lr_min >= 0.0))
    return fail(c, ENS_EINVAL, "bad training arguments");
  DeviceGuard g(c->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t steps = n / batch;
  const int64_t total = steps * epochs;
  // the fused path reads the set staged once, item-major and normalised
  // (kept by the model and grown on demand)
  const float* staged = nullptr;
  if (c->mlp_tile != 0) {
    if (n > s->cap_staged) {
      if (s->staged) (void)hipFree(s->staged);
      s->staged = nullptr;
      s->cap_staged = 0;
      if (alloc(&s->staged, n * ens::kStageW) != hipSuccess)
        return fail(c, ENS_ENOMEM, "cannot allocate the staged training set (%lld items)",
                    (long long)n);
      s->cap_staged = n;
    }
    hipError_t e = ens::mlp_stage_items(params, u0, y, n, s->norm, s->staged, st);
    if (e != hipSuccess) return fail(c, ENS_EDEVICE, "staging the training set: %s", hipGetErrorString(e));
    staged = s->staged;
  }
  uint64_t sm = seed;
  int64_t k = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    uint64_t mult = splitmix(sm) % (uint64_t)n;
    while (n > 1 && (mult == 0 || gcd(mult, (uint64_t)n) != 1)) mult = (mult + 1) % (uint64_t)n;
    if (n == 1) mult = 1;
    const uint64_t add = splitmix(sm) % (uint64_t)n;
    for (int64_t b = 0; b < steps; ++b, ++k) {
      const double lr =
          lr_min + 0.5 * (lr_max - lr_min) * (1.0 + std::cos(M_PI * (double)k / (double)total));
      float* lp = (epoch_loss && b == steps - 1) ? epoch_loss + ep : nullptr;
      rc = train_step(c, s, params, u0, y, n, b * batch, batch, mult, add, lr, lp, st, staged);
      if (rc != ENS_OK) return rc;
    }
  }
  return ENS_OK;
}

int ens_surrogate_predict(ens_ctx* c, ens_surrogate* s, const float* params, const float* u0,
                          int64_t n, float* out, void* stream) {
  int rc = check_model(c, s);
  if (rc != ENS_OK) return rc;
  if (n < 0 || n > ENS_MAX_TRAJ) return fail(c, ENS_EINVAL, "n out of range [0, ENS_MAX_TRAJ]");
  if (n == 0) return ENS_OK;
  if (!params || !u0 || !out) return fail(c, ENS_EINVAL, "null device array");
  DeviceGuard g(c->device);
  return predict(c, s, params, u0, n, out, static_cast<hipStream_t>(stream));
}

int ens_surrogate_solve(ens_ctx* c, ens_surrogate* s, const float* params, const float* u0,
                        const double* tspan, double abstol, double reltol,
                        const double* save_times, int n_save, int64_t n, double audit_frac,
                        double fallback_tol, uint64_t audit_seed, float* out,
                        uint8_t* used_solver, float* report, void* stream) {
  int rc = check_solve_args(c, s, params, u0, tspan, abstol, reltol, save_times, n_save, n,
                            audit_frac, fallback_tol, out);
  if (rc != ENS_OK || n == 0) return rc;
  DeviceGuard g(c->device);
  // workspace for n queries, grown on demand and kept by the model
  const int64_t cap_a = audit_capacity(audit_frac, n);
  if (n > s->cap_n || cap_a > s->cap_audit) {
    void* old[] = {s->alist, s->flist, s->scratch, s->netans, s->used};
    for (void* p : old)
      if (p) (void)hipFree(p);
    s->alist = s->flist = nullptr;
    s->scratch = s->netans = nullptr;
    s->used = nullptr;
    s->cap_n = s->cap_audit = 0;
    if (alloc(&s->alist, cap_a) != hipSuccess || alloc(&s->flist, n) != hipSuccess ||
        alloc(&s->scratch, cap_a * kDims[4]) != hipSuccess ||
        alloc(&s->netans, cap_a * kDims[4]) != hipSuccess || alloc(&s->used, n) != hipSuccess)
      return fail(c, ENS_ENOMEM, "cannot allocate the audit workspace");
    s->cap_n = n;
    s->cap_audit = cap_a;
  }
  AuditWs ws{s->alist, s->flist, s->scratch, s->netans, used_solver ? used_solver : s->used,
             s->counts, s->words, s->cap_audit};
  return audited_solve(c, s, params, u0, tspan, abstol, reltol, save_times, n_save, n,
                       audit_frac, fallback_tol, audit_seed, out, report, ws,
                       static_cast<hipStream_t>(stream));
}

int ens_surrogate_solve_static(ens_ctx* c, ens_surrogate* s, const float* params,
                               const float* u0, const double* tspan, double abstol,
                               double reltol, const double* save_times, int n_save, int64_t n,
                               double audit_frac, double fallback_tol, uint64_t audit_seed,
                               float* out, uint8_t* used_solver, float* report, void* stream) {
  int rc = check_solve_args(c, s, params, u0, tspan, abstol, reltol, save_times, n_save, n,
                            audit_frac, fallback_tol, out);
  if (rc != ENS_OK || n == 0) return rc;
  if (n > ENS_STATIC_MAX_QUERIES)
    return fail(c, ENS_EINVAL, "ens_surrogate_solve_static takes at most %lld queries, not %lld",
                (long long)ENS_STATIC_MAX_QUERIES, (long long)n);
  const int64_t cap_a = audit_capacity(audit_frac, n);
  if (cap_a > kStaticAudit)
    return fail(c, ENS_EINVAL,
                "audit_frac %g over %lld queries needs an audit list of %lld entries; the static "
                "workspace holds %lld",
                audit_frac, (long long)n, (long long)cap_a, (long long)kStaticAudit);
  if (c->mlp_tile == 0)
    return fail(c, ENS_EUNSUPPORTED,
                "the static audited solve runs the fused inference kernel only (ENS_OPT_MLP_TILE "
                "0 needs a workspace)");
  DeviceGuard g(c->device);
  unsigned char* base = static_scratch(c->device);
  if (!base)
    return fail(c, ENS_EDEVICE, "no address of the static workspace on device %d", c->device);
  AuditWs ws{reinterpret_cast<int64_t*>(base + kOffAlist),
             reinterpret_cast<int64_t*>(base + kOffFlist),
             reinterpret_cast<float*>(base + kOffAnswers),
             reinterpret_cast<float*>(base + kOffNet),
             used_solver ? used_solver : base + kOffUsed,
             reinterpret_cast<unsigned long long*>(base + kOffCounts),
             reinterpret_cast<unsigned int*>(base + kOffWords), kStaticAudit};
  return audited_solve(c, s, params, u0, tspan, abstol, reltol, save_times, n_save, n,
                       audit_frac, fallback_tol, audit_seed, out, report, ws,
                       static_cast<hipStream_t>(stream));
}

}  // extern "C"
