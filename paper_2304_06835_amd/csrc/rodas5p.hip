// rodas5p.hip -- adaptive Rodas5P ensemble kernels (GPURodas5P of the paper,
// section 5.2.1, and the reference method of its stiff comparison, section
// 6.4), one whole trajectory per lane (one per 32-lane group for POLLU).
//
// Rodas5P (Steinebach 2023): an 8-stage stiffly accurate Rosenbrock method
// of order 5 with an embedded method of order 4, in the transformed
// variables of rodas.h.  Stage points 7 and 8 are the previous stage point
// plus the previous U (a_7j, a_8j below), the solution is the 8th stage point
// plus U_8, and U_8 is the error estimate.  Coefficients from the publication.
#include "pollu.h"
#include "rodas.h"
#include "rosenbrock.h"
#include "systems.h"

namespace ens {
namespace {

constexpr double kGamma5 = 0.21193756319429014;
constexpr double A5[8][8] = {
    {0, 0, 0, 0, 0, 0, 0, 0},
    {3.0, 0, 0, 0, 0, 0, 0, 0},
    {2.849394379747939, 0.45842242204463923, 0, 0, 0, 0, 0, 0},
    {-6.954028509809101, 2.489845061869568, -10.358996098473584, 0, 0, 0, 0, 0},
    {2.8029986275628964, 0.5072464736228206, -0.3988312541770524, -0.04721187230404641, 0, 0,
     0, 0},
    {-7.502846399306121, 2.561846144803919, -11.627539656261098, -0.18268767659942256,
     0.030198172008377946, 0, 0, 0},
    {-7.502846399306121, 2.561846144803919, -11.627539656261098, -0.18268767659942256,
     0.030198172008377946, 1.0, 0, 0},
    {-7.502846399306121, 2.561846144803919, -11.627539656261098, -0.18268767659942256,
     0.030198172008377946, 1.0, 1.0, 0}};
constexpr double C5[8][8] = {
    {0, 0, 0, 0, 0, 0, 0, 0},
    {-14.155112264123755, 0, 0, 0, 0, 0, 0, 0},
    {-17.97296035885952, -2.859693295451294, 0, 0, 0, 0, 0, 0},
    {147.12150275711716, -1.41221402718213, 71.68940251302358, 0, 0, 0, 0, 0},
    {165.43517024871676, -0.4592823456491126, 42.90938336958603, -5.961986721573306, 0, 0, 0,
     0},
    {24.854864614690072, -3.0009227002832186, 47.4931110020768, 5.5814197821558125,
     -0.6610691825249471, 0, 0, 0},
    {30.91273214028599, -3.1208243349937974, 77.79954646070892, 34.28646028294783,
     -19.097331116725623, -28.087943162872662, 0, 0},
    {37.80277123390563, -3.2571969029072276, 112.26918849496327, 66.9347231244047,
     -40.06618937091002, -54.66780262877968, -9.48861652309627, 0}};

struct Rodas5PTab {
  static constexpr int kStages = 8;
  static constexpr double kGamma = kGamma5;
  static constexpr double kK = 5.0;  // PI exponent: embedded order 4 + 1
  static constexpr double kP = 5.0;
  __device__ static constexpr double a(int i, int j) { return A5[i][j]; }
  __device__ static constexpr double c(int i, int j) { return C5[i][j]; }
};
using Rodas5P = StifflyAccurateRosenbrock<Rodas5PTab>;

}  // namespace

hipError_t launch_rodas5p(int sys, int prec, const LaunchCfg& cfg, LaunchArgs a, hipStream_t s) {
  switch (sys) {
    case ENS_SYS_ROBERTSON: return ros_launch_prec<Robertson, Rodas5P>(prec, cfg, a, s);
    case ENS_SYS_LORENZ: return ros_launch_prec<Lorenz, Rodas5P>(prec, cfg, a, s);
    case ENS_SYS_LINEAR: return ros_launch_prec<Linear, Rodas5P>(prec, cfg, a, s);
    case ENS_SYS_OREGO: return ros_launch_prec<Orego, Rodas5P>(prec, cfg, a, s);
    case ENS_SYS_HIRES: return ros_launch_prec<Hires, Rodas5P>(prec, cfg, a, s);
    case ENS_SYS_POLLU: return ros_launch_grouped<Pollu, Rodas5P>(prec, cfg, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_rodas5p_mixed(int prec, int grid, const MixedArgs& m, hipStream_t s) {
  return ros_launch_mixed<Rodas5P, Robertson, Orego, Lorenz, Linear>(prec, grid, m, s);
}

int rodas5p_mixed_blocks(int prec) {
  return ros_mixed_blocks<Rodas5P, Robertson, Orego, Lorenz, Linear>(prec);
}

int rodas5p_blocks_per_cu(int sys, int prec, int block, int form, int tpl) {
  switch (sys) {
    case ENS_SYS_ROBERTSON: return ros_occ_prec<Robertson, Rodas5P>(prec, block, form, tpl);
    case ENS_SYS_LORENZ: return ros_occ_prec<Lorenz, Rodas5P>(prec, block, form, tpl);
    case ENS_SYS_OREGO: return ros_occ_prec<Orego, Rodas5P>(prec, block, form, tpl);
    case ENS_SYS_HIRES: return ros_occ_prec<Hires, Rodas5P>(prec, block, form, tpl);
    default: return ros_occ_prec<Linear, Rodas5P>(prec, block, form, tpl);
  }
}

}  // namespace ens
