// rodas4.hip -- adaptive Rosenbrock ensemble kernels (GPURodas4 of the paper,
// section 5.2.1), one whole trajectory per lane.
//
// Rosenbrock step (section 3.2.1, eqs. 5-8) in the transformed variables
// U_i = sum_j gamma_ij k_j of Hairer & Wanner (Solving ODEs II, IV.7):
//   W = I/(gamma h) - J   (one analytic Jacobian and one LU per step),
//   W U_i = f(u + sum_{j<i} a_ij U_j) + (1/h) sum_{j<i} C_ij U_j,  i = 1..6,
// stiffly accurate: the 6th stage point is the embedded 3rd-order solution,
// u_new = that point + U_6, and U_6 is the error estimate.
//
// Precision split: FP32 (or FP64) state and stage vectors; the Jacobian, W,
// its LU factorisation with partial pivoting (select-based, no branches) and
// the six triangular solves run in FP64 -- the per-system block-diagonal LU
// of section 5.1.3 (eq. 16), held in registers.
#include "pollu.h"
#include "rodas.h"
#include "rosenbrock.h"
#include "systems.h"

namespace ens {
namespace {

constexpr double kGamma4 = 0.25;
constexpr double RA[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.544, 0, 0, 0, 0, 0},
    {0.9466785280815826, 0.2557011698983284, 0, 0, 0, 0},
    {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0, 0}};
constexpr double RC[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {-5.6688, 0, 0, 0, 0, 0},
    {-2.430093356833875, -0.2063599157091915, 0, 0, 0, 0},
    {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0, 0},
    {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160, 0, 0},
    {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
     -6.058818238834054, 0}};

// RODAS4 as a stiffly accurate Rosenbrock tableau (the step is in rodas.h).
struct Rodas4Tab {
  static constexpr int kStages = 6;
  static constexpr double kGamma = kGamma4;
  static constexpr double kK = 4.0;  // PI exponent: embedded order 3 + 1
  static constexpr double kP = 4.0;
  __device__ static constexpr double a(int i, int j) { return RA[i][j]; }
  __device__ static constexpr double c(int i, int j) { return RC[i][j]; }
};
using Rodas4 = StifflyAccurateRosenbrock<Rodas4Tab>;

}  // namespace

hipError_t launch_rodas4(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a, hipStream_t s) {
  switch (sys) {
    case ENS_SYS_ROBERTSON: return ros_launch_prec<Robertson, Rodas4>(prec, cfg, a, s);
    case ENS_SYS_LORENZ: return ros_launch_prec<Lorenz, Rodas4>(prec, cfg, a, s);
    case ENS_SYS_LINEAR: return ros_launch_prec<Linear, Rodas4>(prec, cfg, a, s);
    case ENS_SYS_OREGO: return ros_launch_prec<Orego, Rodas4>(prec, cfg, a, s);
    case ENS_SYS_HIRES: return ros_launch_prec<Hires, Rodas4>(prec, cfg, a, s);
    case ENS_SYS_POLLU: return ros_launch_grouped<Pollu, Rodas4>(prec, cfg, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_rodas4_mixed(int prec, int grid, const MixedArgs& m, hipStream_t s) {
  return ros_launch_mixed<Rodas4, Robertson, Orego, Lorenz, Linear>(prec, grid, m, s);
}

int rodas4_mixed_blocks(int prec) {
  return ros_mixed_blocks<Rodas4, Robertson, Orego, Lorenz, Linear>(prec);
}

int rodas4_blocks_per_cu(int sys, int prec, int block, int form, int tpl) {
  switch (sys) {
    case ENS_SYS_ROBERTSON: return ros_occ_prec<Robertson, Rodas4>(prec, block, form, tpl);
    case ENS_SYS_LORENZ: return ros_occ_prec<Lorenz, Rodas4>(prec, block, form, tpl);
    case ENS_SYS_OREGO: return ros_occ_prec<Orego, Rodas4>(prec, block, form, tpl);
    case ENS_SYS_HIRES: return ros_occ_prec<Hires, Rodas4>(prec, block, form, tpl);
    default: return ros_occ_prec<Linear, Rodas4>(prec, block, form, tpl);
  }
}

}  // namespace ens
