// capi.hip -- the C ABI declared in include/ens.h: context, options,
// argument validation, launch-shape selection and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/ens.h"
#include "ens_internal.h"

namespace ens {
int tsit5_blocks_per_cu(int sys, int prec, int block, int form, int tpl);
int rodas4_blocks_per_cu(int sys, int prec, int block, int form, int tpl);
int ros23_blocks_per_cu(int sys, int prec, int block, int form, int tpl);
int rodas5p_blocks_per_cu(int sys, int prec, int block, int form, int tpl);
hipError_t launch_tsit5_mixed(int prec, int grid, const MixedArgs& m, hipStream_t s);
hipError_t launch_rodas4_mixed(int prec, int grid, const MixedArgs& m, hipStream_t s);
hipError_t launch_rodas5p_mixed(int prec, int grid, const MixedArgs& m, hipStream_t s);
hipError_t launch_ros23_mixed(int prec, int grid, const MixedArgs& m, hipStream_t s);
int tsit5_mixed_blocks(int prec);
int rodas4_mixed_blocks(int prec);
int rodas5p_mixed_blocks(int prec);
int ros23_mixed_blocks(int prec);

hipError_t launch_mixed(int alg, int prec, int grid, const MixedArgs& m, hipStream_t s) {
  switch (alg) {
    case ENS_ALG_TSIT5: return launch_tsit5_mixed(prec, grid, m, s);
    case ENS_ALG_RODAS4: return launch_rodas4_mixed(prec, grid, m, s);
    case ENS_ALG_RODAS5P: return launch_rodas5p_mixed(prec, grid, m, s);
    case ENS_ALG_ROS23: return launch_ros23_mixed(prec, grid, m, s);
  }
  return hipErrorInvalidValue;
}

int mixed_blocks_per_cu(int alg, int prec) {
  switch (alg) {
    case ENS_ALG_TSIT5: return tsit5_mixed_blocks(prec);
    case ENS_ALG_RODAS4: return rodas4_mixed_blocks(prec);
    case ENS_ALG_RODAS5P: return rodas5p_mixed_blocks(prec);
    case ENS_ALG_ROS23: return ros23_mixed_blocks(prec);
  }
  return 1;
}

__global__ void zero_counter(unsigned long long* q) {
  if (threadIdx.x == 0) *q = 0ull;
}

hipError_t reset_queue(unsigned long long* q, hipStream_t s) {
  hipLaunchKernelGGL(zero_counter, dim3(1), dim3(64), 0, s, q);
  return hipGetLastError();
}

int persistent_grid(int alg, int sys, int prec, int block, int num_cu, int form, int tpl) {
  const int per_cu = alg == ENS_ALG_RODAS4    ? rodas4_blocks_per_cu(sys, prec, block, form, tpl)
                     : alg == ENS_ALG_ROS23   ? ros23_blocks_per_cu(sys, prec, block, form, tpl)
                     : alg == ENS_ALG_RODAS5P ? rodas5p_blocks_per_cu(sys, prec, block, form, tpl)
                                              : tsit5_blocks_per_cu(sys, prec, block, form, tpl);
  return per_cu * num_cu;
}
}  // namespace ens

namespace ens {
int fail(ens_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}
}  // namespace ens

namespace {
using ens::DeviceGuard;
using ens::fail;

bool supported(int sys, int alg) {
  switch (alg) {
    case ENS_ALG_TSIT5: return sys == ENS_SYS_LORENZ || sys == ENS_SYS_LINEAR;
    case ENS_ALG_RODAS4:
    case ENS_ALG_ROS23:
    case ENS_ALG_RODAS5P:
      return sys == ENS_SYS_ROBERTSON || sys == ENS_SYS_LORENZ || sys == ENS_SYS_LINEAR ||
             sys == ENS_SYS_OREGO || sys == ENS_SYS_HIRES || sys == ENS_SYS_POLLU;
    case ENS_ALG_EM: return sys == ENS_SYS_GBM4 || sys == ENS_SYS_CRN;
    case ENS_ALG_SIEA: return sys == ENS_SYS_GBM4;
  }
  return false;
}

// fixed-step SDE algorithms (ENS_OPT_DT, Philox key, FP32 only)
bool is_sde(int alg) { return alg == ENS_ALG_EM || alg == ENS_ALG_SIEA; }

int check_problem(ens_ctx* c, int sys, int64_t n, const void* params, const void* u0,
                  const double* tspan, int alg, double atol, double rtol,
                  const double* theta, int n_save, void* out) {
  int nn, mm;
  if (ens_system_dims(sys, &nn, &mm) != ENS_OK)
    return fail(c, ENS_EINVAL, "unknown system_id %d", sys);
  if (alg != ENS_ALG_TSIT5 && alg != ENS_ALG_RODAS4 && alg != ENS_ALG_EM &&
      alg != ENS_ALG_ROS23 && alg != ENS_ALG_SIEA && alg != ENS_ALG_RODAS5P)
    return fail(c, ENS_EINVAL, "unknown alg %d", alg);
  if (!supported(sys, alg))
    return fail(c, ENS_EUNSUPPORTED, "system %d has no kernel for alg %d", sys, alg);
  if (c->save_mode == 1 && alg != ENS_ALG_TSIT5)
    return fail(c, ENS_EUNSUPPORTED, "dense output (save mode 1) is implemented for Tsit5 only");
  if (is_sde(alg) && c->precision != 32)
    return fail(c, ENS_EUNSUPPORTED, "the SDE kernels are built for precision 32 only");
  // a dispatch counts its work-items in 32 bits: one lane per trajectory,
  // or a 32-lane group per trajectory for the grouped system
  const int64_t lanes = sys == ENS_SYS_POLLU ? 32 : 1;
  if (n < 0 || n > ENS_MAX_TRAJ / lanes)
    return fail(c, ENS_EINVAL, "n_traj %lld out of range [0, %lld] for system %d", (long long)n,
                (long long)(ENS_MAX_TRAJ / lanes), sys);
  if (n_save < 1 || n_save > ens::kMaxSave)
    return fail(c, ENS_EINVAL, "n_save %d out of range [1, %d]", n_save, ens::kMaxSave);
  if (!theta) return fail(c, ENS_EINVAL, "null save_times pointer");
  // an empty ensemble may come with null (zero-size) device arrays
  if (n > 0 && (!params || !u0 || !tspan || !out))
    return fail(c, ENS_EINVAL, "null params/u0/tspan/out pointer");
  double prev = 0.0;
  for (int j = 0; j < n_save; ++j) {
    if (!(theta[j] > prev) || !(theta[j] <= 1.0))
      return fail(c, ENS_EINVAL,
                  "save_times must be strictly increasing fractions in (0, 1]; "
                  "entry %d is %g",
                  j, theta[j]);
    prev = theta[j];
  }
  if (!is_sde(alg)) {
    if (!(atol > 0.0) || !std::isfinite(atol) || !(rtol > 0.0) || !std::isfinite(rtol))
      return fail(c, ENS_EINVAL, "abstol and reltol must be finite and > 0");
  } else if (!(c->dt > 0.0) || !std::isfinite(c->dt)) {
    return fail(c, ENS_EINVAL, "the fixed-step SDE algorithms need ENS_OPT_DT > 0");
  }
  return ENS_OK;
}

ens::LaunchArgs make_args(ens_ctx* c, int64_t n, const void* params, const void* u0,
                          const double* tspan, double atol, double rtol,
                          const double* theta, int n_save, void* out) {
  ens::LaunchArgs a;
  std::memset(&a, 0, sizeof a);
  a.n = n;
  a.in_stride = n;
  a.out_stride = n;
  a.params = params;
  a.u0 = u0;
  a.tspan = tspan;
  a.out = out;
  a.status = c->status;
  a.stats = c->stats;
  a.queue = c->queue;
  a.atol = atol;
  a.rtol = rtol;
  a.h0 = c->h0;
  a.dt = c->dt;
  a.seed = (uint64_t)c->seed;
  a.maxiters = (int64_t)c->maxiters;
  a.n_save = n_save;
  a.tspan_bcast = c->tspan_bcast;
  a.refill = c->refill;
  a.tpl = c->tpl;
  a.dense = c->save_mode == 1;
  a.stage = c->stage_saves;
  for (int j = 0; j < n_save; ++j) a.theta[j] = theta[j];
  return a;
}

int launch(ens_ctx* c, int sys, int alg, ens::LaunchArgs a, const ens::LaunchCfg& cfg0,
           hipStream_t s) {
  return ens::launch_solve(c, sys, alg, a, cfg0, s);
}

}  // namespace

int ens::launch_solve(ens_ctx* c, int sys, int alg, ens::LaunchArgs a,
                      const ens::LaunchCfg& cfg0, hipStream_t s) {
  ens::LaunchCfg cfg = cfg0;
  hipError_t e;
  if (sys == ENS_SYS_POLLU) {  // grouped system: plain form only, at most 8 groups a block
    cfg.form = 0;
    if (cfg.block > ens::kMaxBlock) cfg.block = ens::kMaxBlock;
  }
  if (!is_sde(alg)) {
    // blocks of 512 or 1024 threads exist only for the sorted form, which
    // needs a power of two of at least 256
    if (cfg.form == 2 && cfg.block != 256 && cfg.block != 512 && cfg.block != 1024)
      return fail(c, ENS_EINVAL, "the sorted form (2) needs block 256, 512 or 1024, not %d",
                  cfg.block);
    if (cfg.form != 2 && cfg.block > ens::kMaxBlock)
      return fail(c, ENS_EINVAL, "block %d needs the sorted form (2)", cfg.block);
  } else if (cfg.block > ens::kMaxBlock) {
    cfg.block = ens::kMaxBlock;
  }
  if (is_sde(alg)) {
    cfg.form = 0;
    e = alg == ENS_ALG_EM ? ens::launch_em(sys, c->precision, cfg, a, s)
                          : ens::launch_siea(sys, c->precision, cfg, a, s);
  } else {
    if (cfg.form == 1 || cfg.form == 3) {
      if (cfg.grid <= 0)
        cfg.grid = ens::persistent_grid(alg, sys, c->precision, cfg.block, c->num_cu, cfg.form,
                                        a.tpl);
      a.first_queued = (int64_t)cfg.grid * cfg.block;
      if (cfg.form == 1) a.tpl = 1;
      e = ens::reset_queue(c->queue, s);
      if (e != hipSuccess)
        return fail(c, ENS_EDEVICE, "queue reset launch failed: %s", hipGetErrorString(e));
    } else {
      a.refill = 64;
    }
    e = alg == ENS_ALG_TSIT5     ? ens::launch_tsit5(sys, c->precision, cfg, a, s)
        : alg == ENS_ALG_RODAS4  ? ens::launch_rodas4(sys, c->precision, cfg, a, s)
        : alg == ENS_ALG_RODAS5P ? ens::launch_rodas5p(sys, c->precision, cfg, a, s)
                                 : ens::launch_ros23(sys, c->precision, cfg, a, s);
  }
  if (e != hipSuccess) return fail(c, ENS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return ENS_OK;
}

namespace {

// ---- autotune cache: entries keyed by (system, algorithm, precision, save
// mode, floor(log2 n)) for one device signature, persisted as a small JSON
// file {"version": 1, "entries": [{"device": "...", "sys": ..., ...}, ...]}.

int log2_bucket(int64_t n) {
  int b = 0;
  while (b < 62 && (int64_t(1) << (b + 1)) <= n) ++b;
  return b;
}

// Number after "\"key\":" inside obj, or false.
bool json_num(const std::string& obj, const char* key, double* v) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = obj.find(k);
  if (p == std::string::npos) return false;
  p = obj.find(':', p + k.size());
  if (p == std::string::npos) return false;
  const char* s = obj.c_str() + p + 1;
  char* end = nullptr;
  *v = std::strtod(s, &end);
  return end != s;
}

bool json_str(const std::string& obj, const char* key, std::string* v) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = obj.find(k);
  if (p == std::string::npos) return false;
  p = obj.find(':', p + k.size());
  if (p == std::string::npos) return false;
  const size_t q0 = obj.find('"', p + 1);
  if (q0 == std::string::npos) return false;
  const size_t q1 = obj.find('"', q0 + 1);
  if (q1 == std::string::npos) return false;
  *v = obj.substr(q0 + 1, q1 - q0 - 1);
  return true;
}

// Entries of this device from a cache file; a missing file is an empty cache.
int tune_load(ens_ctx* c, const std::string& path) {
  c->tune.clear();
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return ENS_OK;
  std::string text;
  char buf[4096];
  size_t r;
  while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, r);
  std::fclose(f);
  const size_t e = text.find("\"entries\"");
  if (e == std::string::npos)
    return fail(c, ENS_EINVAL, "autotune cache %s: no \"entries\" array", path.c_str());
  size_t p = text.find('[', e);
  while (p != std::string::npos) {
    const size_t a = text.find('{', p);
    if (a == std::string::npos) break;
    const size_t b = text.find('}', a);
    if (b == std::string::npos) break;
    const std::string obj = text.substr(a, b - a + 1);
    std::string dev;
    double v[10];
    const char* keys[10] = {"sys", "alg", "prec", "save_mode", "log2n",
                            "form", "block", "tpl", "refill", "ms"};
    bool ok = json_str(obj, "device", &dev);
    for (int k = 0; k < 10 && ok; ++k) ok = json_num(obj, keys[k], &v[k]);
    if (!ok) return fail(c, ENS_EINVAL, "autotune cache %s: malformed entry", path.c_str());
    if (dev == c->dev_sig)
      c->tune.push_back({(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5],
                         (int)v[6], (int)v[7], (int)v[8], v[9]});
    p = b + 1;
  }
  return ENS_OK;
}

// Rewrite the file: entries of other devices are kept as they were.
int tune_store(ens_ctx* c) {
  if (c->tune_path.empty()) return ENS_OK;
  std::string others;
  if (FILE* f = std::fopen(c->tune_path.c_str(), "rb")) {
    std::string text;
    char buf[4096];
    size_t r;
    while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, r);
    std::fclose(f);
    size_t p = text.find("\"entries\"");
    while (p != std::string::npos) {
      const size_t a = text.find('{', p);
      if (a == std::string::npos) break;
      const size_t b = text.find('}', a);
      if (b == std::string::npos) break;
      const std::string obj = text.substr(a, b - a + 1);
      std::string dev;
      if (json_str(obj, "device", &dev) && dev != c->dev_sig) others += "    " + obj + ",\n";
      p = b + 1;
    }
  }
  const std::string tmp = c->tune_path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return fail(c, ENS_EINVAL, "cannot write autotune cache %s", tmp.c_str());
  std::fprintf(f, "{\"version\": 1, \"entries\": [\n%s", others.c_str());
  for (size_t k = 0; k < c->tune.size(); ++k) {
    const ens_tune_entry& t = c->tune[k];
    std::fprintf(f,
                 "    {\"device\": \"%s\", \"sys\": %d, \"alg\": %d, \"prec\": %d, "
                 "\"save_mode\": %d, \"log2n\": %d, \"form\": %d, \"block\": %d, "
                 "\"tpl\": %d, \"refill\": %d, \"ms\": %.6g}%s\n",
                 c->dev_sig.c_str(), t.sys, t.alg, t.prec, t.save_mode, t.log2n, t.form, t.block,
                 t.tpl, t.refill, t.ms, k + 1 < c->tune.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), c->tune_path.c_str()) != 0)
    return fail(c, ENS_EINVAL, "cannot write autotune cache %s", c->tune_path.c_str());
  return ENS_OK;
}

ens::LaunchCfg current_cfg(const ens_ctx* c) {
  ens::LaunchCfg cfg;
  cfg.form = c->form;
  cfg.block = c->block > 0 ? c->block : (c->form == 2 ? 1024 : 256);
  cfg.grid = c->grid;
  return cfg;
}

}  // namespace

extern "C" {

int ens_system_dims(int system_id, int* n, int* m) {
  int nn, mm;
  switch (system_id) {
    case ENS_SYS_LINEAR: nn = 3; mm = 9; break;
    case ENS_SYS_LORENZ: nn = 3; mm = 3; break;
    case ENS_SYS_ROBERTSON: nn = 3; mm = 3; break;
    case ENS_SYS_GBM4: nn = 4; mm = 2; break;
    case ENS_SYS_OREGO: nn = 3; mm = 3; break;
    case ENS_SYS_HIRES: nn = 8; mm = 12; break;
    case ENS_SYS_POLLU: nn = 20; mm = 25; break;
    case ENS_SYS_CRN: nn = 4; mm = 6; break;
    default: return ENS_EINVAL;
  }
  if (n) *n = nn;
  if (m) *m = mm;
  return ENS_OK;
}

int ens_create(ens_ctx** out, int device) {
  if (!out) return ENS_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return ENS_EINVAL;
  ens_ctx* c = new (std::nothrow) ens_ctx();
  if (!c) return ENS_ENOMEM;
  c->device = device;
  DeviceGuard g(device);
  if (!g.ok) {
    delete c;
    return ENS_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return ENS_EDEVICE;
  }
  c->num_cu = prop.multiProcessorCount;
  c->dev_sig = std::string(prop.gcnArchName) + "/" + std::to_string(c->num_cu);
  if (ens::init_static_scratch(device) != ENS_OK) {
    delete c;
    return ENS_EDEVICE;
  }
  if (hipMalloc(&c->queue, 256) != hipSuccess) {
    delete c;
    return ENS_ENOMEM;
  }
  *out = c;
  return ENS_OK;
}

int ens_destroy(ens_ctx* c) {
  if (!c) return ENS_OK;
  {
    DeviceGuard g(c->device);
    if (c->queue) (void)hipFree(c->queue);
  }
  delete c;
  return ENS_OK;
}

const char* ens_last_error(const ens_ctx* c) { return c ? c->err.c_str() : "null context"; }

int ens_set_option(ens_ctx* c, int key, double v) {
  if (!c) return ENS_EINVAL;
  if (!std::isfinite(v)) return fail(c, ENS_EINVAL, "option %d: value must be finite", key);
  const bool integral = v == std::floor(v);
  switch (key) {
    case ENS_OPT_PRECISION:
      if (v != 32 && v != 64) return fail(c, ENS_EINVAL, "precision must be 32 or 64");
      c->precision = (int)v;
      return ENS_OK;
    case ENS_OPT_FORM:
      if (v != 0 && v != 1 && v != 2 && v != 3)
        return fail(c, ENS_EINVAL, "form must be 0, 1, 2 or 3");
      c->form = (int)v;
      return ENS_OK;
    case ENS_OPT_BLOCK:
      if (v != 0 && v != 64 && v != 128 && v != 256 && v != 512 && v != 1024)
        return fail(c, ENS_EINVAL, "block must be 0, 64, 128, 256, 512 or 1024");
      c->block = (int)v;
      return ENS_OK;
    case ENS_OPT_DT:
      if (!(v > 0)) return fail(c, ENS_EINVAL, "dt must be > 0");
      c->dt = v;
      return ENS_OK;
    case ENS_OPT_SEED:
      if (!(v >= 0) || !integral || v >= 18446744073709551616.0)
        return fail(c, ENS_EINVAL, "seed must be an integer in [0, 2^64)");
      c->seed = v;
      return ENS_OK;
    case ENS_OPT_H0:
      if (!(v >= 0)) return fail(c, ENS_EINVAL, "h0 must be >= 0");
      c->h0 = v;
      return ENS_OK;
    case ENS_OPT_MAXITERS:
      if (!(v >= 1) || !integral || v > 2e9) return fail(c, ENS_EINVAL, "maxiters must be in [1, 2e9]");
      c->maxiters = v;
      return ENS_OK;
    case ENS_OPT_TSPAN_BROADCAST:
      if (v != 0 && v != 1) return fail(c, ENS_EINVAL, "tspan broadcast must be 0 or 1");
      c->tspan_bcast = (int)v;
      return ENS_OK;
    case ENS_OPT_REFILL:
      if (!integral || v < 1 || v > 64) return fail(c, ENS_EINVAL, "refill must be in [1, 64]");
      c->refill = (int)v;
      return ENS_OK;
    case ENS_OPT_GRID:
      if (!integral || v < 0 || v > 1e6) return fail(c, ENS_EINVAL, "grid must be in [0, 1e6]");
      c->grid = (int)v;
      return ENS_OK;
    case ENS_OPT_TPL:
      if (!integral || v < 1 || v > 8) return fail(c, ENS_EINVAL, "tpl must be in [1, 8]");
      c->tpl = (int)v;
      return ENS_OK;
    case ENS_OPT_SAVE_MODE:
      if (v != 0 && v != 1) return fail(c, ENS_EINVAL, "save mode must be 0 or 1");
      c->save_mode = (int)v;
      return ENS_OK;
    case ENS_OPT_STAGE_SAVES:
      if (v != 0 && v != 1) return fail(c, ENS_EINVAL, "stage_saves must be 0 or 1");
      c->stage_saves = (int)v;
      return ENS_OK;
    case ENS_OPT_AUTOTUNE_CACHED:
      return fail(c, ENS_EINVAL, "option %d is read-only", key);
    case ENS_OPT_MLP_TILE:
      if (v != 0 && v != 2 && v != 3 && v != 4 && v != 12 && v != 13)
        return fail(c, ENS_EINVAL, "mlp tile must be 0, 2, 3, 4, 12 or 13");
      c->mlp_tile = (int)v;
      return ENS_OK;
  }
  return fail(c, ENS_EINVAL, "unknown option key %d", key);
}

int ens_get_option(const ens_ctx* c, int key, double* v) {
  if (!c || !v) return ENS_EINVAL;
  switch (key) {
    case ENS_OPT_PRECISION: *v = c->precision; return ENS_OK;
    case ENS_OPT_FORM: *v = c->form; return ENS_OK;
    case ENS_OPT_BLOCK: *v = c->block; return ENS_OK;
    case ENS_OPT_DT: *v = c->dt; return ENS_OK;
    case ENS_OPT_SEED: *v = c->seed; return ENS_OK;
    case ENS_OPT_H0: *v = c->h0; return ENS_OK;
    case ENS_OPT_MAXITERS: *v = c->maxiters; return ENS_OK;
    case ENS_OPT_TSPAN_BROADCAST: *v = c->tspan_bcast; return ENS_OK;
    case ENS_OPT_REFILL: *v = c->refill; return ENS_OK;
    case ENS_OPT_GRID: *v = c->grid; return ENS_OK;
    case ENS_OPT_TPL: *v = c->tpl; return ENS_OK;
    case ENS_OPT_MLP_TILE: *v = c->mlp_tile; return ENS_OK;
    case ENS_OPT_SAVE_MODE: *v = c->save_mode; return ENS_OK;
    case ENS_OPT_STAGE_SAVES: *v = c->stage_saves; return ENS_OK;
    case ENS_OPT_AUTOTUNE_CACHED: *v = c->tune_cached; return ENS_OK;
  }
  return ENS_EINVAL;
}

int ens_set_ptr(ens_ctx* c, int key, void* p) {
  if (!c) return ENS_EINVAL;
  switch (key) {
    case ENS_PTR_STATUS: c->status = static_cast<uint8_t*>(p); return ENS_OK;
    case ENS_PTR_STATS: c->stats = static_cast<int32_t*>(p); return ENS_OK;
  }
  return fail(c, ENS_EINVAL, "unknown pointer key %d", key);
}

int ens_solve(ens_ctx* c, int sys, int64_t n, const void* params, const void* u0,
              const double* tspan, int alg, double atol, double rtol, const double* theta,
              int n_save, void* out, void* stream) {
  if (!c) return ENS_EINVAL;
  c->err.clear();
  int rc = check_problem(c, sys, n, params, u0, tspan, alg, atol, rtol, theta, n_save, out);
  if (rc != ENS_OK) return rc;
  if (n == 0) return ENS_OK;
  DeviceGuard g(c->device);
  if (!g.ok) return fail(c, ENS_EDEVICE, "cannot make device %d current", c->device);
  ens::LaunchArgs a = make_args(c, n, params, u0, tspan, atol, rtol, theta, n_save, out);
  return launch(c, sys, alg, a, current_cfg(c), static_cast<hipStream_t>(stream));
}

int ens_solve_mixed(ens_ctx* c, int n_groups, const ens_group* groups, int alg, double atol,
                    double rtol, const double* theta, int n_save, void* stream) {
  if (!c) return ENS_EINVAL;
  c->err.clear();
  if (n_groups < 1 || n_groups > ens::kMaxGroups || !groups)
    return fail(c, ENS_EINVAL, "n_groups %d out of range [1, %d] (or null groups)", n_groups,
                ens::kMaxGroups);
  if (alg != ENS_ALG_TSIT5 && alg != ENS_ALG_RODAS4 && alg != ENS_ALG_RODAS5P &&
      alg != ENS_ALG_ROS23)
    return fail(c, ENS_EUNSUPPORTED, "mixed solves take an adaptive algorithm, not %d", alg);
  ens::MixedArgs m;
  std::memset(&m, 0, sizeof m);
  int64_t chunks = 0;
  for (int g = 0; g < n_groups; ++g) {
    const ens_group& G = groups[g];
    const int sys = G.system_id;
    const bool ok_sys = alg == ENS_ALG_TSIT5
                            ? (sys == ENS_SYS_LORENZ || sys == ENS_SYS_LINEAR)
                            : (sys == ENS_SYS_ROBERTSON || sys == ENS_SYS_OREGO ||
                               sys == ENS_SYS_LORENZ || sys == ENS_SYS_LINEAR);
    if (!ok_sys)
      return fail(c, ENS_EUNSUPPORTED, "group %d: system %d is not in the mixed set of alg %d",
                  g, sys, alg);
    int rc = check_problem(c, sys, G.n_traj, G.params, G.u0, G.tspan, alg, atol, rtol, theta,
                           n_save, G.out);
    if (rc != ENS_OK) {
      const std::string msg = c->err;
      return fail(c, rc, "group %d: %s", g, msg.c_str());
    }
    if (G.tspan_broadcast != 0 && G.tspan_broadcast != 1)
      return fail(c, ENS_EINVAL, "group %d: tspan_broadcast must be 0 or 1", g);
    ens::GroupArgs& A = m.g[g];
    A.sys = sys;
    A.tspan_bcast = G.tspan_broadcast;
    A.n = G.n_traj;
    A.params = G.params;
    A.u0 = G.u0;
    A.tspan = G.tspan;
    A.out = G.out;
    A.status = G.status;
    A.stats = G.stats;
    A.chunks = (G.n_traj + ens::kMixedChunk - 1) / ens::kMixedChunk;
    chunks += A.chunks;
  }
  m.n_groups = n_groups;
  m.n_chunks = chunks;
  // queue order: the groups with fewer chunks first (a stable sort), so a
  // small group of long trajectories starts beside the large group instead
  // of forming the launch's tail (measured: interleaving the groups through
  // the queue instead is slower)
  std::stable_sort(m.g, m.g + n_groups, [](const ens::GroupArgs& x, const ens::GroupArgs& y) {
    return x.chunks < y.chunks;
  });
  for (int g = 0; g < n_groups; ++g) {
    m.g[g].chunk0 = g == 0 ? 0 : m.g[g - 1].chunk0 + m.g[g - 1].chunks;
  }
  if (chunks == 0) return ENS_OK;
  DeviceGuard dg(c->device);
  if (!dg.ok) return fail(c, ENS_EDEVICE, "cannot make device %d current", c->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  m.c = make_args(c, 0, nullptr, nullptr, nullptr, atol, rtol, theta, n_save, nullptr);
  // ENS_OPT_FORM 3: the persistent queue on a resident grid; otherwise one
  // block per chunk (grid 0 below), which measured faster
  const int grid = c->form != 3 ? 0
                   : c->grid > 0 ? c->grid
                                 : ens::mixed_blocks_per_cu(alg, c->precision) * c->num_cu;
  if (grid == 0 && chunks > (int64_t)0xFFFFFFFF / ens::kMixedChunk)
    return fail(c, ENS_EINVAL, "too many chunks for one block each: %lld", (long long)chunks);
  hipError_t e = ens::reset_queue(c->queue, s);
  if (e == hipSuccess) e = ens::launch_mixed(alg, c->precision, grid, m, s);
  if (e != hipSuccess) return fail(c, ENS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return ENS_OK;
}

int ens_philox_fill(ens_ctx* c, uint64_t seed, int64_t n, uint32_t step, uint32_t* out,
                    void* stream) {
  if (!c) return ENS_EINVAL;
  c->err.clear();
  if (n < 0 || n > ENS_MAX_TRAJ)
    return fail(c, ENS_EINVAL, "n_traj %lld out of range [0, %lld]", (long long)n,
                (long long)ENS_MAX_TRAJ);
  if (n == 0) return ENS_OK;
  if (!out) return fail(c, ENS_EINVAL, "null out pointer");
  DeviceGuard g(c->device);
  if (!g.ok) return fail(c, ENS_EDEVICE, "cannot make device %d current", c->device);
  const hipError_t e = ens::launch_philox_fill(seed, n, step, out, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(c, ENS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return ENS_OK;
}

int ens_autotune(ens_ctx* c, int sys, int64_t n, const void* params, const void* u0,
                 const double* tspan, int alg, double atol, double rtol, const double* theta,
                 int n_save, void* out, void* stream, double* best_ms) {
  if (!c) return ENS_EINVAL;
  c->err.clear();
  int rc = check_problem(c, sys, n, params, u0, tspan, alg, atol, rtol, theta, n_save, out);
  if (rc != ENS_OK) return rc;
  if (n == 0) return fail(c, ENS_EINVAL, "autotune needs a non-empty probe ensemble");
  c->tune_cached = 0;
  const int log2n = log2_bucket(n);
  for (const ens_tune_entry& t : c->tune) {
    if (t.sys == sys && t.alg == alg && t.prec == c->precision && t.save_mode == c->save_mode &&
        t.log2n == log2n) {
      c->form = t.form;
      c->block = t.block;
      c->tpl = t.tpl;
      if (t.form == 1) c->refill = t.refill;
      if (best_ms) *best_ms = t.ms;
      c->tune_cached = 1;
      return ENS_OK;
    }
  }
  DeviceGuard g(c->device);
  if (!g.ok) return fail(c, ENS_EDEVICE, "cannot make device %d current", c->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  ens::LaunchArgs a = make_args(c, n, params, u0, tspan, atol, rtol, theta, n_save, out);
  struct Cand {
    int form, block, tpl, refill;
  };
  Cand cands[64];
  int nc = 0;
  const int blocks[3] = {64, 128, 256};
  // the grouped system (POLLU) runs one trajectory per 32-lane group in the
  // plain form only: its launches differ by block size alone
  const bool grouped = sys == ENS_SYS_POLLU;
  for (int b : blocks) {
    if (grouped) {
      cands[nc++] = {0, b, 1, 64};
      continue;
    }
    for (int tpl : {1, 2, 4}) cands[nc++] = {0, b, tpl, 64};
    if (!is_sde(alg))
      for (int rf : {4, 16, 32}) cands[nc++] = {1, b, 1, rf};
  }
  if (!is_sde(alg) && !grouped) {
    for (int b : {256, 512, 1024}) cands[nc++] = {2, b, 1, 64};
    for (int b : {256, 512}) cands[nc++] = {2, b, 2, 64};  // sort over 2 * block items
    for (int b : {128, 256}) cands[nc++] = {3, b, 1, 64};  // persistent sorted chunks
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(c, ENS_EDEVICE, "hipEventCreate failed");
  double best = 1e300;
  Cand win = cands[0];
  for (int k = 0; k < nc; ++k) {
    ens::LaunchCfg cfg{cands[k].form, cands[k].block, c->grid};
    a.tpl = cands[k].tpl;
    a.refill = cands[k].refill;
    float ms_min = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {  // first run warms up
      if (hipEventRecord(e0, s) != hipSuccess) { rc = ENS_EDEVICE; break; }
      rc = launch(c, sys, alg, a, cfg, s);
      if (rc != ENS_OK) break;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = ENS_EDEVICE;
        break;
      }
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0 && ms < ms_min) ms_min = ms;
    }
    if (rc != ENS_OK) break;
    if (ms_min < best) {
      best = ms_min;
      win = cands[k];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != ENS_OK) return rc == ENS_EDEVICE ? fail(c, rc, "autotune: HIP event/launch failure") : rc;
  c->form = win.form;
  c->block = win.block;
  c->tpl = win.tpl;
  if (win.form == 1) c->refill = win.refill;
  if (best_ms) *best_ms = best;
  c->tune.push_back({sys, alg, c->precision, c->save_mode, log2n, win.form, win.block, win.tpl,
                     win.refill, best});
  return tune_store(c);
}

int ens_set_autotune_file(ens_ctx* c, const char* path) {
  if (!c) return ENS_EINVAL;
  c->err.clear();
  c->tune.clear();
  c->tune_path = path ? path : "";
  if (!path) return ENS_OK;
  return tune_load(c, c->tune_path);
}

}  // extern "C"
