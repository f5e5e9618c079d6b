// ens_internal.h -- launch arguments and kernel launchers shared by the C ABI
// (capi.hip) and the kernel translation units.  Not installed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace ens {

constexpr int kMaxSave = 64;
constexpr int kMaxBlock = 256;   // __launch_bounds__ of every solver kernel
constexpr int kWave = 64;

// Everything a solver kernel needs, passed by value (lands in the kernel
// argument segment, read through scalar loads).
struct LaunchArgs {
  int64_t n;                 // work items (an upper bound when n_dev is set)
  int64_t in_stride;         // row stride of params / u0 / tspan
  int64_t out_stride;        // row stride of out
  const void* params;        // [M][in_stride]
  const void* u0;            // [N][in_stride]
  const double* tspan;       // [2][in_stride] or [2]
  void* out;                 // [n_save][N][out_stride]
  const int64_t* idx;        // work item k reads column idx[k] (null: k)
  const unsigned long long* n_dev;  // device-side work count (null: n)
  int scatter;               // 1: work item k writes column idx[k]; 0: column k
  uint8_t* status;           // [n] (by work item) or null
  int32_t* stats;            // [2][n] (by work item) or null
  unsigned long long* queue; // persistent form: work counter (zeroed per launch)
  double atol, rtol;
  double h0;                 // <= 0: starting-step heuristic
  double dt;                 // fixed-step methods
  uint64_t seed;             // Philox key
  int64_t maxiters;
  int64_t first_queued;      // persistent form: trajectories handed out statically
  int n_save;
  int tspan_bcast;
  int refill;                // persistent form: idle lanes that trigger a refill
  int tpl;                   // plain form: trajectories per lane
  int dense;                 // Tsit5: 1 = save times from the dense output
  int stage;                 // sorted Tsit5: 1 = saves staged in LDS when they fit
  double theta[kMaxSave];
};

// One group of a mixed-system launch (ens_solve_mixed): its own system and
// arrays, and the index of its first chunk in the launch's work queue.
struct GroupArgs {
  int sys;
  int tspan_bcast;
  int64_t n;
  const void* params;
  const void* u0;
  const double* tspan;
  void* out;
  uint8_t* status;
  int32_t* stats;
  int64_t chunks;  // ceil(n / kMixedChunk)
  int64_t chunk0;  // queue position of its first chunk
};
constexpr int kMaxGroups = 8;
constexpr int64_t kMixedChunk = 256;  // trajectories per chunk (the block size)

// A mixed-system launch: the shared settings in `c` (queue, tolerances,
// save times, ...), the groups, and the total number of chunks.
struct MixedArgs {
  LaunchArgs c;
  GroupArgs g[kMaxGroups];
  int n_groups;
  int64_t n_chunks;  // sum of the groups' chunks
};

struct LaunchCfg {
  int form;   // 0 plain, 1 persistent, 2 cost-sorted, 3 persistent cost-sorted chunks
  int block;  // threads per block
  int grid;   // forms 1 and 3: blocks (0: occupancy-derived)
};

// Each returns hipSuccess or the launch error.  `sys` is ENS_SYS_*, `prec` 32|64.
hipError_t launch_tsit5(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a,
                        hipStream_t s);
hipError_t launch_rodas4(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a,
                         hipStream_t s);
hipError_t launch_ros23(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a,
                        hipStream_t s);
hipError_t launch_rodas5p(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a,
                          hipStream_t s);
hipError_t launch_em(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a,
                     hipStream_t s);

hipError_t launch_siea(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a,
                       hipStream_t s);

// Mixed-system persistent launch of `alg` in blocks of 256 (grid 0: fill
// every CU); blocks_per_cu gives the resident blocks of that kernel.
hipError_t launch_mixed(int alg, int prec, int grid, const MixedArgs& m, hipStream_t s);
int mixed_blocks_per_cu(int alg, int prec);

hipError_t launch_philox_fill(uint64_t seed, int64_t n, uint32_t step, uint32_t* out,
                              hipStream_t s);

// Blocks per CU the persistent kernel of (alg, sys, prec) can keep resident
// at `block` threads, and the grid that fills the device.
int persistent_grid(int alg, int sys, int prec, int block, int num_cu, int form, int tpl);

// Zero the persistent work counter (a one-thread kernel, so the solve can be
// captured into a graph without memset nodes).
hipError_t reset_queue(unsigned long long* q, hipStream_t s);

}  // namespace ens

// One autotuner result: the launch that was fastest for a problem class.
struct ens_tune_entry {
  int sys, alg, prec, save_mode, log2n;  // the key
  int form, block, tpl, refill;          // the winning launch
  double ms;                             // its time on the probe ensemble
};

// The context behind the opaque ens_ctx handle of include/ens.h.
struct ens_ctx {
  int device = 0;
  int num_cu = 0;
  int precision = 32;
  int form = 0;
  int block = 0;
  int tpl = 1;
  int refill = 16;
  int grid = 0;
  int mlp_tile = 13;
  int save_mode = 0;
  int stage_saves = 0;
  int tspan_bcast = 0;
  double dt = 0.0;
  double h0 = 0.0;
  double seed = 0.0;
  double maxiters = 1e6;
  uint8_t* status = nullptr;
  int32_t* stats = nullptr;
  unsigned long long* queue = nullptr;  // device workspace: persistent work counter
  std::vector<ens_tune_entry> tune;     // autotuner results of this device
  std::string tune_path;                // file the results persist to ("" = none)
  std::string dev_sig;                  // device architecture and CU count
  int tune_cached = 0;                  // the last ens_autotune was a cache hit
  std::string err;
};

namespace ens {

// Records a formatted message on the context and returns `code`.
int fail(ens_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));

// Makes `dev` current for the lifetime of the guard, restoring the caller's.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) return;
    ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceGuard() {
    if (ok && prev >= 0) (void)hipSetDevice(prev);
  }
};

// Looks up this device's address of the static workspace of
// ens_surrogate_solve_static (once per device; `device` must be current).
int init_static_scratch(int device);

// Launch one adaptive or fixed-step solve described by `a` with `cfg`
// (resets the persistent queue first when cfg.form == 1).
int launch_solve(ens_ctx* c, int sys, int alg, LaunchArgs a, const LaunchCfg& cfg, hipStream_t s);

}  // namespace ens
