/*
 * oracle.c -- plain FP64 CPU reference for the ensemble ODE/SDE hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for readability against
 * the paper, not for speed: one trajectory at a time, textbook formulas, no
 * blocking or fusion.  Trajectories are independent, so an OpenMP loop over
 * them is the only concession to run time.
 *
 * Paper passages followed:
 *   - ODE problem statement: section 3.1, eq. 1.
 *   - Explicit Runge-Kutta step with tableau {A, b, c}: section 3.1, eqs. 2-3.
 *   - Embedded estimate, scaled error q and accept rule q < 1, PI step-size
 *     control h_new = eta q_{n-1}^{beta2} q_n^{beta1} h: section 3.1, eq. 4.
 *   - Tsitouras 5(4) pair (GPUTsit5): section 5.2.1.
 *   - Rosenbrock s-stage method: section 3.2.1, eqs. 5-8; 4th-order stiffly
 *     stable variant (GPURodas4) and the 2(3) pair (GPURosenbrock23):
 *     section 5.2.1; LU of W per system: section 5.1.3, eq. 16.
 *   - SDE definition dX = a dt + b dW, dW ~ N(0, dt): section 3.3, eq. 11;
 *     Euler-Maruyama (GPUEM) and a weak order-2 scheme (GPUSIEA): section
 *     5.2.2; the sigma-factor CRN SDE: appendix.
 *   - Models: appendix (Lorenz, Robertson, linear SDE); stiff test problems
 *     OREGO, HIRES and POLLU of appendix B.1.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NMAX 20 /* largest system: POLLU */
#define MMAX 32 /* most parameters: POLLU's 25 rate constants */

/* ------------------------------------------------------------------------ */
/* Systems                                                                   */
/* ------------------------------------------------------------------------ */

int orc_dims(int sys, int *n, int *m) {
  switch (sys) {
  case ORC_LINEAR: *n = 3; *m = 9; return 0;
  case ORC_LORENZ: *n = 3; *m = 3; return 0;
  case ORC_ROBERTSON: *n = 3; *m = 3; return 0;
  case ORC_GBM4: *n = 4; *m = 2; return 0;
  case ORC_OREGO: *n = 3; *m = 3; return 0;
  case ORC_HIRES: *n = 8; *m = 12; return 0;
  case ORC_POLLU: *n = 20; *m = 25; return 0;
  case ORC_CRN: *n = 4; *m = 6; return 0;
  }
  return -1;
}

/* POLLU (appendix B.1 of the paper, after Verwer 1994) as 25 reactions.
 * Reaction j runs at r_j = k_j * y[A_j] (* y[B_j] when B_j >= 0); its
 * effect on dy/dt is the column of the stoichiometric table: species
 * POLLU_S[j][0..] gain (positive) or lose (negative) r_j.  The table is the
 * paper's 20 equations read term by term (u_9 and u_16 in the equations for
 * dy5 and dy6 read as y9 and y16).  Indices are 0-based.                  */
static const int POLLU_A[25] = {0, 1, 4, 6, 6, 6, 8, 8, 10, 10, 12, 9, 13,
                                0, 2, 3, 3, 15, 15, 16, 18, 18, 0, 18, 19};
static const int POLLU_B[25] = {-1, 3, 1, -1, -1, 5, -1, 5, 1, 0, -1, 1, -1,
                                5, -1, -1, -1, -1, -1, 5, -1, -1, 3, 0, -1};
/* (species, coefficient) pairs per reaction, terminated by coefficient 0 */
static const int POLLU_S[25][6][2] = {
    {{0, -1}, {1, 1}, {2, 1}},                  /* r1:  y1 -> y2 + y3        */
    {{1, -1}, {3, -1}, {0, 1}},                 /* r2:  y2 + y4 -> y1        */
    {{4, -1}, {1, -1}, {0, 1}, {5, 1}},         /* r3:  y5 + y2 -> y1 + y6   */
    {{6, -1}, {4, 2}, {7, 1}},                  /* r4:  y7 -> 2 y5 + y8      */
    {{6, -1}, {7, 1}},                          /* r5:  y7 -> y8             */
    {{6, -1}, {5, -1}, {4, 1}, {7, 1}},         /* r6:  y7 + y6 -> y5 + y8   */
    {{8, -1}, {4, 1}, {7, 1}, {9, 1}},          /* r7:  y9 -> y5 + y8 + y10  */
    {{8, -1}, {5, -1}, {10, 1}},                /* r8:  y9 + y6 -> y11       */
    {{10, -1}, {1, -1}, {0, 1}, {9, 1}, {11, 1}},  /* r9: y11 + y2 -> y1 + y10 + y12 */
    {{10, -1}, {0, -1}, {12, 1}},               /* r10: y11 + y1 -> y13      */
    {{12, -1}, {0, 1}, {10, 1}},                /* r11: y13 -> y1 + y11      */
    {{9, -1}, {1, -1}, {0, 1}, {13, 1}},        /* r12: y10 + y2 -> y1 + y14 */
    {{13, -1}, {4, 1}, {6, 1}},                 /* r13: y14 -> y5 + y7       */
    {{0, -1}, {5, -1}, {14, 1}},                /* r14: y1 + y6 -> y15       */
    {{2, -1}, {3, 1}},                          /* r15: y3 -> y4             */
    {{3, -1}, {15, 1}},                         /* r16: y4 -> y16            */
    {{3, -1}, {2, 1}},                          /* r17: y4 -> y3             */
    {{15, -1}, {5, 2}},                         /* r18: y16 -> 2 y6          */
    {{15, -1}, {2, 1}},                         /* r19: y16 -> y3            */
    {{16, -1}, {5, -1}, {4, 1}, {17, 1}},       /* r20: y17 + y6 -> y5 + y18 */
    {{18, -1}, {1, 1}},                         /* r21: y19 -> y2            */
    {{18, -1}, {0, 1}, {2, 1}},                 /* r22: y19 -> y1 + y3       */
    {{0, -1}, {3, -1}, {18, 1}},                /* r23: y1 + y4 -> y19       */
    {{18, -1}, {0, -1}, {19, 1}},               /* r24: y19 + y1 -> y20      */
    {{19, -1}, {0, 1}, {18, 1}},                /* r25: y20 -> y1 + y19      */
};

static double pollu_rate(const double *k, const double *y, int j) {
  double r = k[j] * y[POLLU_A[j]];
  return POLLU_B[j] >= 0 ? r * y[POLLU_B[j]] : r;
}

/* Appendix, Lorenz problem: dy1 = sigma (y2 - y1), dy2 = rho y1 - y2 - y1 y3,
 * dy3 = y1 y2 - beta y3 (the paper writes beta as gamma).
 * Appendix, Robertson: dy1 = -k1 y1 + k3 y2 y3, dy2 = k1 y1 - k3 y2 y3 - k2 y2^2,
 * dy3 = k2 y2^2, with (k1, k2, k3) = (0.04, 3e7, 1e4) at the printed rates.
 * GBM drift (appendix, linear SDE): a(X) = mu X per component.              */
int orc_rhs(int sys, const double *p, const double *u, double *du) {
  switch (sys) {
  case ORC_LINEAR:
    for (int i = 0; i < 3; i++)
      du[i] = p[3 * i + 0] * u[0] + p[3 * i + 1] * u[1] + p[3 * i + 2] * u[2];
    return 0;
  case ORC_LORENZ: {
    double sigma = p[0], rho = p[1], beta = p[2];
    du[0] = sigma * (u[1] - u[0]);
    du[1] = rho * u[0] - u[1] - u[0] * u[2];
    du[2] = u[0] * u[1] - beta * u[2];
    return 0;
  }
  case ORC_ROBERTSON: {
    double k1 = p[0], k2 = p[1], k3 = p[2];
    du[0] = -k1 * u[0] + k3 * u[1] * u[2];
    du[1] = k1 * u[0] - k3 * u[1] * u[2] - k2 * u[1] * u[1];
    du[2] = k2 * u[1] * u[1];
    return 0;
  }
  case ORC_GBM4:
    for (int i = 0; i < 4; i++) du[i] = p[0] * u[i];
    return 0;
  case ORC_OREGO: {
    /* appendix B.1 (OREGO) with the textbook sign of dy1 (see oracle.h) */
    double k1 = p[0], k2 = p[1], k3 = p[2];
    du[0] = k1 * (u[1] + u[0] * (1.0 - k2 * u[0] - u[1]));
    du[1] = (u[2] - (1.0 + u[0]) * u[1]) / k1;
    du[2] = k3 * (u[0] - u[2]);
    return 0;
  }
  case ORC_HIRES: {
    /* appendix B.1 (HIRES); p = the 12 distinct rate constants in the order
     * (1.71, 0.43, 8.32, 0.0007, 8.75, 10.03, 0.035, 1.12, 1.745, 280,
     * 0.69, 1.81), each standing for every occurrence of its value */
    const double *k = p;
    const double *y = u;
    du[0] = -k[0] * y[0] + k[1] * y[1] + k[2] * y[2] + k[3];
    du[1] = k[0] * y[0] - k[4] * y[1];
    du[2] = -k[5] * y[2] + k[1] * y[3] + k[6] * y[4];
    du[3] = k[2] * y[1] + k[0] * y[2] - k[7] * y[3];
    du[4] = -k[8] * y[4] + k[1] * y[5] + k[1] * y[6];
    du[5] = -k[9] * y[5] * y[7] + k[10] * y[3] + k[0] * y[4] - k[1] * y[5] +
            k[10] * y[6];
    du[6] = k[9] * y[5] * y[7] - k[11] * y[6];
    du[7] = -k[9] * y[5] * y[7] + k[11] * y[6];
    return 0;
  }
  case ORC_POLLU:
    for (int i = 0; i < 20; i++) du[i] = 0.0;
    for (int j = 0; j < 25; j++) {
      double r = pollu_rate(p, u, j);
      for (int e = 0; e < 6 && POLLU_S[j][e][1] != 0; e++)
        du[POLLU_S[j][e][0]] += POLLU_S[j][e][1] * r;
    }
    return 0;
  }
  return -1;
}

/* J[i][j] = d f_i / d u_j, written out by hand from orc_rhs. */
int orc_jac(int sys, const double *p, const double *u, double *J) {
  switch (sys) {
  case ORC_LINEAR:
    for (int i = 0; i < 9; i++) J[i] = p[i];
    return 0;
  case ORC_LORENZ: {
    double sigma = p[0], rho = p[1], beta = p[2];
    J[0] = -sigma;        J[1] = sigma;  J[2] = 0.0;
    J[3] = rho - u[2];    J[4] = -1.0;   J[5] = -u[0];
    J[6] = u[1];          J[7] = u[0];   J[8] = -beta;
    return 0;
  }
  case ORC_ROBERTSON: {
    double k1 = p[0], k2 = p[1], k3 = p[2];
    J[0] = -k1; J[1] = k3 * u[2];                   J[2] = k3 * u[1];
    J[3] = k1;  J[4] = -k3 * u[2] - 2.0 * k2 * u[1]; J[5] = -k3 * u[1];
    J[6] = 0.0; J[7] = 2.0 * k2 * u[1];             J[8] = 0.0;
    return 0;
  }
  case ORC_GBM4:
    memset(J, 0, 16 * sizeof(double));
    for (int i = 0; i < 4; i++) J[5 * i] = p[0];
    return 0;
  case ORC_OREGO: {
    double k1 = p[0], k2 = p[1], k3 = p[2];
    J[0] = k1 * (1.0 - 2.0 * k2 * u[0] - u[1]);
    J[1] = k1 * (1.0 - u[0]);
    J[2] = 0.0;
    J[3] = -u[1] / k1;
    J[4] = -(1.0 + u[0]) / k1;
    J[5] = 1.0 / k1;
    J[6] = k3;
    J[7] = 0.0;
    J[8] = -k3;
    return 0;
  }
  case ORC_HIRES: {
    const double *k = p;
    const double *y = u;
    memset(J, 0, 64 * sizeof(double));
    J[0 * 8 + 0] = -k[0]; J[0 * 8 + 1] = k[1]; J[0 * 8 + 2] = k[2];
    J[1 * 8 + 0] = k[0];  J[1 * 8 + 1] = -k[4];
    J[2 * 8 + 2] = -k[5]; J[2 * 8 + 3] = k[1]; J[2 * 8 + 4] = k[6];
    J[3 * 8 + 1] = k[2];  J[3 * 8 + 2] = k[0]; J[3 * 8 + 3] = -k[7];
    J[4 * 8 + 4] = -k[8]; J[4 * 8 + 5] = k[1]; J[4 * 8 + 6] = k[1];
    J[5 * 8 + 3] = k[10]; J[5 * 8 + 4] = k[0];
    J[5 * 8 + 5] = -k[9] * y[7] - k[1];
    J[5 * 8 + 6] = k[10]; J[5 * 8 + 7] = -k[9] * y[5];
    J[6 * 8 + 5] = k[9] * y[7]; J[6 * 8 + 6] = -k[11]; J[6 * 8 + 7] = k[9] * y[5];
    J[7 * 8 + 5] = -k[9] * y[7]; J[7 * 8 + 6] = k[11]; J[7 * 8 + 7] = -k[9] * y[5];
    return 0;
  }
  case ORC_POLLU:
    /* J = S dr/dy: reaction j contributes S[:, j] times the gradient of
     * r_j, which has one or two non-zeros */
    memset(J, 0, 400 * sizeof(double));
    for (int j = 0; j < 25; j++) {
      int a = POLLU_A[j], b = POLLU_B[j];
      double da = b >= 0 ? p[j] * u[b] : p[j]; /* d r_j / d y_a */
      double db = b >= 0 ? p[j] * u[a] : 0.0;  /* d r_j / d y_b */
      for (int e = 0; e < 6 && POLLU_S[j][e][1] != 0; e++) {
        int i = POLLU_S[j][e][0];
        double c = POLLU_S[j][e][1];
        J[i * 20 + a] += c * da;
        if (b >= 0) J[i * 20 + b] += c * db;
      }
    }
    return 0;
  }
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Tableaus, written from the primary publications the paper cites.         */
/* ------------------------------------------------------------------------ */

/* Tsitouras (2011), "Runge-Kutta pairs of order 5(4) satisfying only the first
 * column simplifying assumption": 7 stages, FSAL (row 7 of A equals b).
 * TS_BT holds b - bhat, the weights of the embedded error estimate.         */
static const double TS_C[7] = {0.0, 0.161, 0.327, 0.9, 0.9800255409045097,
                               1.0, 1.0};
static const double TS_A[7][7] = {
    {0, 0, 0, 0, 0, 0, 0},
    {0.161, 0, 0, 0, 0, 0, 0},
    {-0.008480655492356989, 0.335480655492357, 0, 0, 0, 0, 0},
    {2.897153057105493, -6.359448489975075, 4.3622954328695815, 0, 0, 0, 0},
    {5.325864828439257, -11.748883564062828, 7.4955393428898365,
     -0.09249506636175525, 0, 0, 0},
    {5.86145544294642, -12.92096931784711, 8.159367898576159,
     -0.071584973281401, -0.028269050394068383, 0, 0},
    {0.09646076681806523, 0.01, 0.4798896504144996, 1.379008574103742,
     -3.290069515436081, 2.324710524099774, 0}};
static const double TS_BT[7] = {
    -0.00178001105222577714, -0.0008164344596567469, 0.007880878010261995,
    -0.1447110071732629,     0.5823571654525552,     -0.45808210592918697,
    0.015151515151515152};

/* Dense output (the "free" 4th-order interpolation of section 5.2.1, not
 * printed there): u(t + theta h) = u + h sum_i b_i(theta) k_i with
 * b_i(theta) = sum_m TS_DENSE[i][m-1] theta^m.  Derived from the order
 * conditions: every order-<=4 condition holds for every theta, b(1) = b,
 * b'(0) = e_1 and b'(1) = e_7 (C1 across steps), and the remaining free
 * parameter minimises the integral over theta of the squared order-5
 * defects.  The coefficients satisfy those conditions to ~1e-14, as closely
 * as the tableau's published digits allow.                                 */
static const double TS_DENSE[7][4] = {
    {1.0, -2.7697190860447156, 2.925281239361705, -1.059101386498926},
    {0.0, 0.12894207915150258, -0.2178841583029839, 0.09894207915151598},
    {0.0, 3.95691789344045, -5.994277185222965, 2.517248942196988},
    {0.0, -12.89991187880857, 31.315858054031978, -17.036937601119686},
    {0.0, 39.47651966255469, -92.1133173868537, 49.346728208862906},
    {0.0, -29.443930585810573, 68.18670326802032, -36.41806215810994},
    {0.0, 1.5511819155171473, -4.102363831034384, 2.55118191551721}};

/* RODAS4 of Hairer & Wanner, "Solving ODEs II", section IV.7, in the
 * transformed variables U_i = sum_j gamma_ij k_j, for which one stage reads
 *   (I/(gamma h) - J) U_i = f(u + sum_{j<i} a_ij U_j) + sum_{j<i} (C_ij / h) U_j.
 * Solution u + sum m_j U_j, embedded u + sum mhat_j U_j.  Stiffly accurate:
 * the 6th stage point is the embedded solution and U_6 is the error.       */
static const double RO_GAMMA = 0.25;
static const double RO_A[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.544, 0, 0, 0, 0, 0},
    {0.9466785280815826, 0.2557011698983284, 0, 0, 0, 0},
    {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087,
     -0.6878860361058950, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087,
     -0.6878860361058950, 1.0, 0}};
static const double RO_C[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {-5.6688, 0, 0, 0, 0, 0},
    {-2.430093356833875, -0.2063599157091915, 0, 0, 0, 0},
    {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0, 0},
    {7.496443313967647, -10.24680431464352, -33.99990352819905,
     11.70890893206160, 0, 0},
    {8.083246795921522, -7.981132988064893, -31.52159432874371,
     16.31930543123136, -6.058818238834054, 0}};
static const double RO_M[6] = {1.221224509226641, 6.019134481288629,
                               12.53708332932087, -0.6878860361058950, 1.0,
                               1.0};
static const double RO_MHAT[6] = {1.221224509226641, 6.019134481288629,
                                  12.53708332932087, -0.6878860361058950, 1.0,
                                  0.0};

/* Rodas5P of Steinebach (2023), the paper's GPURodas5P (section 5.2.1) and
 * the reference method of its stiff comparison (section 6.4): an 8-stage
 * stiffly accurate Rosenbrock method of order 5 with an embedded method of
 * order 4, in the same transformed variables as RODAS4.  The stage points of
 * stages 7 and 8 are the previous stage point plus the previous U, the
 * solution is the 8th stage point plus U_8 and the embedded solution is the
 * 8th stage point (so U_8 is the error estimate).  Coefficients from that
 * publication.                                                              */
static const double R5_GAMMA = 0.21193756319429014;
static const double R5_A[8][8] = {
    {0, 0, 0, 0, 0, 0, 0, 0},
    {3.0, 0, 0, 0, 0, 0, 0, 0},
    {2.849394379747939, 0.45842242204463923, 0, 0, 0, 0, 0, 0},
    {-6.954028509809101, 2.489845061869568, -10.358996098473584, 0, 0, 0, 0, 0},
    {2.8029986275628964, 0.5072464736228206, -0.3988312541770524,
     -0.04721187230404641, 0, 0, 0, 0},
    {-7.502846399306121, 2.561846144803919, -11.627539656261098,
     -0.18268767659942256, 0.030198172008377946, 0, 0, 0},
    {-7.502846399306121, 2.561846144803919, -11.627539656261098,
     -0.18268767659942256, 0.030198172008377946, 1.0, 0, 0},
    {-7.502846399306121, 2.561846144803919, -11.627539656261098,
     -0.18268767659942256, 0.030198172008377946, 1.0, 1.0, 0}};
static const double R5_C[8][8] = {
    {0, 0, 0, 0, 0, 0, 0, 0},
    {-14.155112264123755, 0, 0, 0, 0, 0, 0, 0},
    {-17.97296035885952, -2.859693295451294, 0, 0, 0, 0, 0, 0},
    {147.12150275711716, -1.41221402718213, 71.68940251302358, 0, 0, 0, 0, 0},
    {165.43517024871676, -0.4592823456491126, 42.90938336958603,
     -5.961986721573306, 0, 0, 0, 0},
    {24.854864614690072, -3.0009227002832186, 47.4931110020768,
     5.5814197821558125, -0.6610691825249471, 0, 0, 0},
    {30.91273214028599, -3.1208243349937974, 77.79954646070892,
     34.28646028294783, -19.097331116725623, -28.087943162872662, 0, 0},
    {37.80277123390563, -3.2571969029072276, 112.26918849496327,
     66.9347231244047, -40.06618937091002, -54.66780262877968,
     -9.48861652309627, 0}};
static const double R5_M[8] = {-7.502846399306121, 2.561846144803919,
                               -11.627539656261098, -0.18268767659942256,
                               0.030198172008377946, 1.0, 1.0, 1.0};
static const double R5_MHAT[8] = {-7.502846399306121, 2.561846144803919,
                                  -11.627539656261098, -0.18268767659942256,
                                  0.030198172008377946, 1.0, 1.0, 0.0};

void orc_rodas5p_tableau(double *gamma, double a[64], double C[64],
                         double m[8], double mhat[8]) {
  *gamma = R5_GAMMA;
  for (int i = 0; i < 8; i++) {
    m[i] = R5_M[i];
    mhat[i] = R5_MHAT[i];
    for (int j = 0; j < 8; j++) {
      a[8 * i + j] = R5_A[i][j];
      C[8 * i + j] = R5_C[i][j];
    }
  }
}

void orc_tsit5_tableau(double c[7], double a[49], double b[7],
                       double btilde[7]) {
  for (int i = 0; i < 7; i++) {
    c[i] = TS_C[i];
    b[i] = TS_A[6][i];
    btilde[i] = TS_BT[i];
    for (int j = 0; j < 7; j++) a[7 * i + j] = TS_A[i][j];
  }
}

void orc_tsit5_dense_table(double B[28]) {
  for (int i = 0; i < 7; i++)
    for (int m = 0; m < 4; m++) B[4 * i + m] = TS_DENSE[i][m];
}

/* u + h sum_i b_i(theta) k_i for the stages k of one Tsit5 step. */
static void tsit5_dense(int n, const double *u, double k[7][NMAX], double h,
                        double theta, double *out) {
  double bt[7];
  for (int i = 0; i < 7; i++) {
    double b = 0.0;
    for (int m = 3; m >= 0; m--) b = (b + TS_DENSE[i][m]) * theta;
    bt[i] = b;
  }
  for (int c = 0; c < n; c++) {
    double s = 0.0;
    for (int i = 0; i < 7; i++) s += bt[i] * k[i][c];
    out[c] = u[c] + h * s;
  }
}

void orc_rodas4_tableau(double *gamma, double a[36], double C[36],
                        double m[6], double mhat[6]) {
  *gamma = RO_GAMMA;
  for (int i = 0; i < 6; i++) {
    m[i] = RO_M[i];
    mhat[i] = RO_MHAT[i];
    for (int j = 0; j < 6; j++) {
      a[6 * i + j] = RO_A[i][j];
      C[6 * i + j] = RO_C[i][j];
    }
  }
}

/* ------------------------------------------------------------------------ */
/* One step of each method.  All systems are autonomous.                     */
/* ------------------------------------------------------------------------ */

/* Explicit RK step (eqs. 2-3) with the Tsit5 tableau.  k1 = f(u) on entry
 * (first-same-as-last).  Writes unew, the error vector err = h sum btilde_j k_j
 * (= unew - uhat) and k7 = f(unew).                                          */
static void tsit5_step(int sys, const double *p, int n, const double *u,
                       const double *k1, double h, double *unew, double *err,
                       double *k7, double kall[7][NMAX]) {
  double k[7][NMAX], y[NMAX];
  for (int c = 0; c < n; c++) k[0][c] = k1[c];
  for (int i = 1; i < 7; i++) {
    for (int c = 0; c < n; c++) {
      double s = 0.0;
      for (int j = 0; j < i; j++) s += TS_A[i][j] * k[j][c];
      y[c] = u[c] + h * s;
    }
    orc_rhs(sys, p, y, k[i]);
  }
  for (int c = 0; c < n; c++) {
    double s = 0.0;
    for (int j = 0; j < 7; j++) s += TS_BT[j] * k[j][c];
    unew[c] = y[c]; /* stage-7 point = u + h sum b_j k_j */
    err[c] = h * s;
    k7[c] = k[6][c];
  }
  if (kall)
    for (int i = 0; i < 7; i++)
      for (int c = 0; c < n; c++) kall[i][c] = k[i][c];
}

/* LU factorisation with partial pivoting of the n x n row-major matrix W. */
static void lu_factor(int n, double *W, int *piv) {
  for (int k = 0; k < n; k++) {
    int pr = k;
    for (int i = k + 1; i < n; i++)
      if (fabs(W[i * n + k]) > fabs(W[pr * n + k])) pr = i;
    piv[k] = pr;
    if (pr != k)
      for (int j = 0; j < n; j++) {
        double t = W[k * n + j];
        W[k * n + j] = W[pr * n + j];
        W[pr * n + j] = t;
      }
    for (int i = k + 1; i < n; i++) {
      W[i * n + k] /= W[k * n + k];
      for (int j = k + 1; j < n; j++) W[i * n + j] -= W[i * n + k] * W[k * n + j];
    }
  }
}

/* Solve (LU) x = b in place, applying the recorded row swaps first. */
static void lu_solve(int n, const double *LU, const int *piv, double *x) {
  for (int k = 0; k < n; k++)
    if (piv[k] != k) {
      double t = x[k];
      x[k] = x[piv[k]];
      x[piv[k]] = t;
    }
  for (int i = 0; i < n; i++)
    for (int j = 0; j < i; j++) x[i] -= LU[i * n + j] * x[j];
  for (int i = n - 1; i >= 0; i--) {
    for (int j = i + 1; j < n; j++) x[i] -= LU[i * n + j] * x[j];
    x[i] /= LU[i * n + i];
  }
}

/* Rosenbrock step (eqs. 5-8) in the transformed form stated above the
 * tableaus: one Jacobian, one LU of W = I/(gamma h) - J, one solve per
 * stage; ns stages with coefficient rows of stride ns.                      */
static void rodas_step(int ns, double gamma, const double *A, const double *C,
                       const double *M, const double *MHAT, int sys,
                       const double *p, int n, const double *u, double h,
                       double *unew, double *err) {
  double J[NMAX * NMAX], W[NMAX * NMAX], U[8][NMAX], y[NMAX], fy[NMAX];
  int piv[NMAX];
  orc_jac(sys, p, u, J);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++)
      W[i * n + j] = (i == j ? 1.0 / (gamma * h) : 0.0) - J[i * n + j];
  lu_factor(n, W, piv);
  for (int i = 0; i < ns; i++) {
    for (int c = 0; c < n; c++) {
      double s = 0.0;
      for (int j = 0; j < i; j++) s += A[ns * i + j] * U[j][c];
      y[c] = u[c] + s;
    }
    orc_rhs(sys, p, y, fy);
    for (int c = 0; c < n; c++) {
      double s = 0.0;
      for (int j = 0; j < i; j++) s += C[ns * i + j] / h * U[j][c];
      U[i][c] = fy[c] + s;
    }
    lu_solve(n, W, piv, U[i]);
  }
  for (int c = 0; c < n; c++) {
    double s = 0.0, e = 0.0;
    for (int j = 0; j < ns; j++) {
      s += M[j] * U[j][c];
      e += (M[j] - MHAT[j]) * U[j][c];
    }
    unew[c] = u[c] + s;
    err[c] = e;
  }
}

static void rodas4_step(int sys, const double *p, int n, const double *u,
                        double h, double *unew, double *err) {
  rodas_step(6, RO_GAMMA, &RO_A[0][0], &RO_C[0][0], RO_M, RO_MHAT, sys, p, n, u,
             h, unew, err);
}

static void rodas5p_step(int sys, const double *p, int n, const double *u,
                         double h, double *unew, double *err) {
  rodas_step(8, R5_GAMMA, &R5_A[0][0], &R5_C[0][0], R5_M, R5_MHAT, sys, p, n,
             u, h, unew, err);
}

/* ------------------------------------------------------------------------ */
/* Adaptive driver                                                           */
/* ------------------------------------------------------------------------ */

/* Rosenbrock23 (GPURosenbrock23 of section 5.2.1): the modified Rosenbrock
 * pair of Shampine & Reichelt (SIAM J. Sci. Comput. 18, 1997, the ode23s
 * formulas), written in its own variables.  With d = 1/(2 + sqrt 2),
 * e32 = 6 + sqrt 2, W = I - h d J and F0 = f(u):
 *   k1 = W^-1 F0
 *   F1 = f(u + h k1 / 2),      k2 = W^-1 (F1 - k1) + k1
 *   unew = u + h k2            (order 2, L-stable)
 *   F2 = f(unew),              k3 = W^-1 (F2 - e32 (k2 - F1) - 2 (k1 - F0))
 * and unew + h (k1 - 2 k2 + k3) / 6 is the order-3 companion.  err is unew
 * minus that companion, so the embedded solution is unew - err as for the
 * other methods.  Autonomous systems only (no df/dt terms).                */
static void ros23_step(int sys, const double *p, int n, const double *u,
                       double h, double *unew, double *err) {
  const double d = 1.0 / (2.0 + sqrt(2.0)), e32 = 6.0 + sqrt(2.0);
  double J[NMAX * NMAX], W[NMAX * NMAX], F0[NMAX], F1[NMAX], F2[NMAX];
  double k1[NMAX], k2[NMAX], k3[NMAX], y[NMAX];
  int piv[NMAX];
  orc_jac(sys, p, u, J);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++)
      W[i * n + j] = (i == j ? 1.0 : 0.0) - h * d * J[i * n + j];
  lu_factor(n, W, piv);
  orc_rhs(sys, p, u, F0);
  for (int c = 0; c < n; c++) k1[c] = F0[c];
  lu_solve(n, W, piv, k1);
  for (int c = 0; c < n; c++) y[c] = u[c] + 0.5 * h * k1[c];
  orc_rhs(sys, p, y, F1);
  for (int c = 0; c < n; c++) k2[c] = F1[c] - k1[c];
  lu_solve(n, W, piv, k2);
  for (int c = 0; c < n; c++) {
    k2[c] += k1[c];
    unew[c] = u[c] + h * k2[c];
  }
  orc_rhs(sys, p, unew, F2);
  for (int c = 0; c < n; c++)
    k3[c] = F2[c] - e32 * (k2[c] - F1[c]) - 2.0 * (k1[c] - F0[c]);
  lu_solve(n, W, piv, k3);
  for (int c = 0; c < n; c++) err[c] = -h / 6.0 * (k1[c] - 2.0 * k2[c] + k3[c]);
}

/* Scaled error proportion q of eq. 4, taking the norm as the root mean square
 * over the n components (Hairer, Norsett & Wanner I, section II.4).        */
static double error_q(int n, const double *err, const double *u,
                      const double *unew, double atol, double rtol) {
  double s = 0.0;
  for (int c = 0; c < n; c++) {
    double sc = atol + rtol * fmax(fabs(u[c]), fabs(unew[c]));
    double r = err[c] / sc;
    s += r * r;
  }
  return sqrt(s / n);
}

static double rms_scaled(int n, const double *v, const double *sc) {
  double s = 0.0;
  for (int c = 0; c < n; c++) s += (v[c] / sc[c]) * (v[c] / sc[c]);
  return sqrt(s / n);
}

/* Starting step of Hairer, Norsett & Wanner I, section II.4 (two f calls),
 * capped by the interval length.  p is the order of the method.            */
static double initial_step(int sys, const double *pp, int n, const double *u0,
                           const double *f0, double atol, double rtol, int p,
                           double hmax) {
  double sc[NMAX], u1[NMAX], f1[NMAX], df[NMAX];
  for (int c = 0; c < n; c++) sc[c] = atol + rtol * fabs(u0[c]);
  double d0 = rms_scaled(n, u0, sc), d1 = rms_scaled(n, f0, sc);
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
  h0 = fmin(h0, hmax);
  for (int c = 0; c < n; c++) u1[c] = u0[c] + h0 * f0[c];
  orc_rhs(sys, pp, u1, f1);
  for (int c = 0; c < n; c++) df[c] = f1[c] - f0[c];
  double d2 = rms_scaled(n, df, sc) / h0;
  double dm = fmax(d1, d2);
  double h1 = (dm <= 1e-15) ? fmax(1e-6, h0 * 1e-3)
                            : pow(0.01 / dm, 1.0 / (p + 1));
  return fmin(fmin(100.0 * h0, h1), hmax);
}

/* PI controller constants (section 3.1 names eta, beta1, beta2 without
 * values; taken from Hairer & Wanner's presentation of Gustafsson's PI
 * controller with k = embedded order + 1).                                 */
#define PI_ETA 0.9
#define PI_FMIN 0.2
#define PI_FMAX 10.0
#define PI_QFLOOR 1e-4
#define STRETCH 1.1 /* steps within 10% of the next save time land on it */

/* save_mode 0: every save time is a step end (steps land on it);
 * save_mode 1 (Tsit5 only): steps land only on the last save time and the
 * earlier ones are read off the dense output of the step that covers them. */
static void solve_one(int sys, int alg, int n, const double *p,
                      const double *u0, double t0, double tf, double atol,
                      double rtol, const double *theta, int n_save,
                      double *outcol /* [n_save][n] */, int *status,
                      int64_t *nacc, int64_t *nrej, double h0,
                      int64_t maxiters, int save_mode) {
  /* PI exponent k = embedded order + 1; p = order of the propagated
   * solution (starting-step heuristic) */
  const double kexp = (alg == ORC_TSIT5 || alg == ORC_RODAS5P)
                          ? 5.0
                          : (alg == ORC_RODAS4 ? 4.0 : 3.0);
  const int porder = (alg == ORC_TSIT5 || alg == ORC_RODAS5P)
                         ? 5
                         : (alg == ORC_RODAS4 ? 4 : 2);
  const int dense = save_mode == 1 && alg == ORC_TSIT5;
  double u[NMAX], k1[NMAX], unew[NMAX], err[NMAX], k7[NMAX], kall[7][NMAX];
  double hmax = tf - t0;
  int j = 0;
  int64_t acc = 0, rej = 0;
  *status = ORC_OK;
  for (int c = 0; c < n; c++) u[c] = u0[c];
  double t = t0;
  if (!(tf >= t0) || !isfinite(t0) || !isfinite(tf)) { /* invalid span */
    *status = ORC_NONFINITE;
    for (j = 0; j < n_save; j++)
      for (int c = 0; c < n; c++) outcol[j * n + c] = NAN;
    *nacc = 0;
    *nrej = 0;
    return;
  }
  /* save points that coincide with t0 (only when tf == t0) */
  while (j < n_save && t0 + theta[j] * (tf - t0) <= t) {
    for (int c = 0; c < n; c++) outcol[j * n + c] = u[c];
    j++;
  }
  orc_rhs(sys, p, u, k1);
  double h = h0;
  if (j < n_save && !(h0 > 0.0))
    h = initial_step(sys, p, n, u, k1, atol, rtol, porder, hmax);
  h = fmin(h, hmax);
  double qold = PI_QFLOOR;
  while (j < n_save) {
    if (acc + rej >= maxiters) { *status = ORC_MAXITERS; break; }
    /* the time the step may not pass: the next save time, or with dense
     * output the last one */
    double ts = t0 + theta[dense ? n_save - 1 : j] * (tf - t0);
    double rem = ts - t;
    /* a step that would end within 10% short of the save time is stretched
     * onto it (no spurious short step before the save); after a rejected
     * stretched step h <= 0.9 rem, so the stretch cannot repeat a rejection */
    int clamped = (h * STRETCH >= rem);
    double he = clamped ? rem : h;
    if (alg == ORC_TSIT5)
      tsit5_step(sys, p, n, u, k1, he, unew, err, k7, kall);
    else if (alg == ORC_RODAS4)
      rodas4_step(sys, p, n, u, he, unew, err);
    else if (alg == ORC_RODAS5P)
      rodas5p_step(sys, p, n, u, he, unew, err);
    else
      ros23_step(sys, p, n, u, he, unew, err);
    double q = error_q(n, err, u, unew, atol, rtol);
    if (!isfinite(q)) { *status = ORC_NONFINITE; break; }
    if (q <= 1.0) {
      acc++;
      double tn = clamped ? ts : t + he;
      if (dense) /* save times inside the step, read off its dense output */
        for (; j < n_save; j++) {
          double tj = t0 + theta[j] * (tf - t0);
          if (!(tj <= tn) || (clamped && j == n_save - 1)) break;
          tsit5_dense(n, u, kall, he, (tj - t) / he, outcol + j * n);
        }
      t = tn;
      for (int c = 0; c < n; c++) u[c] = unew[c];
      if (alg == ORC_TSIT5)
        for (int c = 0; c < n; c++) k1[c] = k7[c];
      double fac = PI_ETA * pow(fmax(q, 1e-10), -0.7 / kexp) *
                   pow(qold, 0.4 / kexp);
      fac = fmin(PI_FMAX, fmax(PI_FMIN, fac));
      qold = fmax(q, PI_QFLOOR);
      double hn = he * fac;
      if (clamped) hn = fmax(hn, h); /* keep the proposal made before the clamp */
      h = fmin(hn, hmax);
      while (j < n_save && t0 + theta[j] * (tf - t0) <= t) {
        for (int c = 0; c < n; c++) outcol[j * n + c] = u[c];
        j++;
      }
    } else {
      rej++;
      double fac = fmax(PI_FMIN, PI_ETA * pow(q, -1.0 / kexp));
      h = he * fac;
    }
    if (j < n_save && !(h > 16.0 * DBL_EPSILON * fabs(t))) {
      *status = ORC_DTMIN;
      break;
    }
  }
  /* trajectories that stopped early report NaN at the unreached save times */
  for (; j < n_save; j++)
    for (int c = 0; c < n; c++) outcol[j * n + c] = NAN;
  *nacc = acc;
  *nrej = rej;
}

int orc_solve_mode(int sys, int alg, int64_t N, const double *params,
                   const double *u0, const double *tspan, double atol,
                   double rtol, const double *theta, int n_save, double *out,
                   int *status, int64_t *naccept, int64_t *nreject, double h0,
                   int64_t maxiters, int nthreads, int save_mode) {
  int n, m;
  if (orc_dims(sys, &n, &m) != 0 || sys == ORC_GBM4) return -1;
  if (alg != ORC_TSIT5 && alg != ORC_RODAS4 && alg != ORC_ROS23 && alg != ORC_RODAS5P)
    return -1;
  if (N < 0 || n_save < 1 || !params || !u0 || !tspan || !theta || !out)
    return -1;
  if (save_mode != 0 && save_mode != 1) return -1;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 16)
  for (int64_t i = 0; i < N; i++) {
    double p[MMAX], uu[NMAX], col[64 * NMAX];
    for (int r = 0; r < m; r++) p[r] = params[r * N + i];
    for (int c = 0; c < n; c++) uu[c] = u0[c * N + i];
    int st;
    int64_t a, rj;
    double *colp = (n_save <= 64) ? col : (double *)malloc(sizeof(double) * n_save * n);
    solve_one(sys, alg, n, p, uu, tspan[i], tspan[N + i], atol, rtol, theta,
              n_save, colp, &st, &a, &rj, h0, maxiters, save_mode);
    for (int s = 0; s < n_save; s++)
      for (int c = 0; c < n; c++) out[((int64_t)s * n + c) * N + i] = colp[s * n + c];
    if (colp != col) free(colp);
    if (status) status[i] = st;
    if (naccept) naccept[i] = a;
    if (nreject) nreject[i] = rj;
  }
  return 0;
}

int orc_solve(int sys, int alg, int64_t N, const double *params,
              const double *u0, const double *tspan, double atol,
              double rtol, const double *theta, int n_save, double *out,
              int *status, int64_t *naccept, int64_t *nreject, double h0,
              int64_t maxiters, int nthreads) {
  return orc_solve_mode(sys, alg, N, params, u0, tspan, atol, rtol, theta,
                        n_save, out, status, naccept, nreject, h0, maxiters,
                        nthreads, 0);
}

/* n_steps fixed Tsit5 steps of size h from u0, the last one read at its
 * dense output: u(t0 + (n_steps - 1 + theta) h).                           */
int orc_fixed_dense(int sys, const double *p, const double *u0, double h,
                    int n_steps, double theta, double *u_out) {
  int n, m;
  if (orc_dims(sys, &n, &m) != 0 || sys == ORC_GBM4 || n_steps < 1) return -1;
  double u[NMAX], k1[NMAX], unew[NMAX], err[NMAX], k7[NMAX], kall[7][NMAX];
  for (int c = 0; c < n; c++) u[c] = u0[c];
  orc_rhs(sys, p, u, k1);
  for (int s = 0; s < n_steps; s++) {
    tsit5_step(sys, p, n, u, k1, h, unew, err, k7, kall);
    if (s == n_steps - 1) {
      tsit5_dense(n, u, kall, h, theta, u_out);
      return 0;
    }
    for (int c = 0; c < n; c++) {
      u[c] = unew[c];
      k1[c] = k7[c];
    }
  }
  return 0;
}

int orc_fixed(int sys, int alg, const double *p, const double *u0, double h,
              int n_steps, double *u_out, double *uhat_out) {
  int n, m;
  if (orc_dims(sys, &n, &m) != 0) return -1;
  if (alg != ORC_TSIT5 && alg != ORC_RODAS4 && alg != ORC_ROS23 && alg != ORC_RODAS5P)
    return -1;
  double u[NMAX], k1[NMAX], unew[NMAX], err[NMAX], k7[NMAX];
  for (int c = 0; c < n; c++) u[c] = u0[c];
  orc_rhs(sys, p, u, k1);
  for (int s = 0; s < n_steps; s++) {
    if (alg == ORC_TSIT5)
      tsit5_step(sys, p, n, u, k1, h, unew, err, k7, NULL);
    else if (alg == ORC_RODAS4)
      rodas4_step(sys, p, n, u, h, unew, err);
    else if (alg == ORC_RODAS5P)
      rodas5p_step(sys, p, n, u, h, unew, err);
    else
      ros23_step(sys, p, n, u, h, unew, err);
    if (s == n_steps - 1)
      for (int c = 0; c < n; c++) uhat_out[c] = unew[c] - err[c];
    for (int c = 0; c < n; c++) u[c] = unew[c];
    if (alg == ORC_TSIT5)
      for (int c = 0; c < n; c++) k1[c] = k7[c];
  }
  for (int c = 0; c < n; c++) u_out[c] = u[c];
  if (n_steps == 0)
    for (int c = 0; c < n; c++) uhat_out[c] = u[c];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, Box-Muller and Euler-Maruyama                              */
/* ------------------------------------------------------------------------ */

/* Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3"
 * (SC'11): Philox4x32 round = two 32x32->64 multiplies and a permutation
 * with key XOR; Weyl key schedule; 10 rounds.                               */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    uint64_t p0 = (uint64_t)M0 * x0, p1 = (uint64_t)M1 * x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Top 23 bits of x mapped to the midpoints (2k + 1) 2^-24, k < 2^23: exact in
 * single precision, strictly inside (0, 1).                                 */
double orc_uniform(uint32_t x) {
  return (double)(2u * (x >> 9) + 1u) * 0x1p-24;
}

/* Box-Muller: z0 = r cos(2 pi v), z1 = r sin(2 pi v), r = sqrt(-2 ln u). */
void orc_box_muller(uint32_t x0, uint32_t x1, double *z0, double *z1) {
  const double two_pi = 6.283185307179586476925287;
  double u = orc_uniform(x0), v = orc_uniform(x1);
  double r = sqrt(-2.0 * log(u));
  *z0 = r * cos(two_pi * v);
  *z1 = r * sin(two_pi * v);
}

/* ------------------------------------------------------------------------ */
/* SDEs (section 3.3, eq. 11): drift a(X) and noise matrix b(X) [n][m]       */
/* ------------------------------------------------------------------------ */

static int sde_dims(int sys, int *n, int *m) {
  switch (sys) {
  case ORC_GBM4: *n = 4; *m = 4; return 0;
  case ORC_CRN: *n = 4; *m = 8; return 0;
  }
  return -1;
}

/* Appendix, linear SDE: four GBMs dX_c = mu X_c dt + sigma X_c dW_c.
 * Appendix, sigma-factor CRN (chemical Langevin equation), X = (s, A1, A2,
 * A3), p = (S, D, tau, nu0, n, eta), with the Hill input
 * H = (S s)^n / ((S s)^n + (D A3)^n + 1):
 *   ds  = (nu0 + H - s) dt + eta sqrt(nu0 + H) dW1 - eta sqrt(s) dW2
 *   dA1 = (s - A1)/tau dt + eta sqrt(s/tau) dW3 - eta sqrt(A1/tau) dW4
 *   dA2 = (A1 - A2)/tau dt + eta sqrt(A1/tau) dW5 - eta sqrt(A2/tau) dW6
 *   dA3 = (A2 - A3)/tau dt + eta sqrt(A2/tau) dW7 - eta sqrt(A3/tau) dW8
 * Reading (the paper is silent): a concentration that an increment drives
 * below zero enters the Hill function and the square roots as 0.          */
static void sde_coeffs(int sys, const double *p, const double *x, double *a,
                       double *b /* [n][m] */) {
  if (sys == ORC_GBM4) {
    double mu = p[0], sigma = p[1];
    memset(b, 0, 16 * sizeof(double));
    for (int c = 0; c < 4; c++) {
      a[c] = mu * x[c];
      b[c * 4 + c] = sigma * x[c];
    }
    return;
  }
  /* ORC_CRN */
  double S = p[0], D = p[1], tau = p[2], nu0 = p[3], n = p[4], eta = p[5];
  double s = fmax(x[0], 0.0), a1 = fmax(x[1], 0.0), a2 = fmax(x[2], 0.0),
         a3 = fmax(x[3], 0.0);
  double hs = pow(S * s, n), hd = pow(D * a3, n);
  double H = hs / (hs + hd + 1.0);
  a[0] = nu0 + H - x[0];
  a[1] = (x[0] - x[1]) / tau;
  a[2] = (x[1] - x[2]) / tau;
  a[3] = (x[2] - x[3]) / tau;
  memset(b, 0, 32 * sizeof(double));
  b[0 * 8 + 0] = eta * sqrt(nu0 + H);
  b[0 * 8 + 1] = -eta * sqrt(s);
  b[1 * 8 + 2] = eta * sqrt(s / tau);
  b[1 * 8 + 3] = -eta * sqrt(a1 / tau);
  b[2 * 8 + 4] = eta * sqrt(a1 / tau);
  b[2 * 8 + 5] = -eta * sqrt(a2 / tau);
  b[3 * 8 + 6] = eta * sqrt(a2 / tau);
  b[3 * 8 + 7] = -eta * sqrt(a3 / tau);
}

/* The diagonal of b for a diagonal-noise system (m = n, b[c][c]). */
static void sde_bdiag(int sys, const double *p, const double *x, double *bd) {
  double a[8], b[64];
  sde_coeffs(sys, p, x, a, b);
  for (int c = 0; c < 4; c++) bd[c] = b[c * 4 + c];
}

/* Euler-Maruyama (GPUEM, section 5.2.2): X + a h + b dW. */
static void em_step(int sys, const double *p, int n, int m, const double *x,
                    double h, const double *dW, double *xo) {
  double a[8], b[64];
  sde_coeffs(sys, p, x, a, b);
  for (int c = 0; c < n; c++) {
    double s = x[c] + a[c] * h;
    for (int j = 0; j < m; j++) s += b[c * m + j] * dW[j];
    xo[c] = s;
  }
}

/* Weak order-2 explicit scheme for diagonal noise (GPUSIEA of section
 * 5.2.2; the paper cites Tocino & Vigo-Aguiar for it but prints no
 * coefficients).  Reading: the explicit order-2.0 weak scheme of Kloeden &
 * Platen (1992, eq. 15.1.1), a member of the stochastic Runge-Kutta family
 * of section 3.3 with stages Y, Ybar = Y + a h + b dW, Y+- = Y + a h +- b
 * sqrt(h) and fit term R = (b(Y+) - b(Y-)) (dW^2 - h) / (4 sqrt h):
 *   Y' = Y + (a(Ybar) + a) h / 2 + (b(Y+) + b(Y-) + 2 b) dW / 4 + R,
 * componentwise (each b_c depends on X_c alone for the diagonal systems). */
static void siea_step(int sys, const double *p, int n, const double *x,
                      double h, const double *dW, double *xo) {
  double a[8], b[64], bd[8], yb[8], yp[8], ym[8], ab[8], bb[64], bp[8], bm[8];
  sde_coeffs(sys, p, x, a, b);
  for (int c = 0; c < n; c++) bd[c] = b[c * n + c];
  double sq = sqrt(h);
  for (int c = 0; c < n; c++) {
    yb[c] = x[c] + a[c] * h + bd[c] * dW[c];
    yp[c] = x[c] + a[c] * h + bd[c] * sq;
    ym[c] = x[c] + a[c] * h - bd[c] * sq;
  }
  sde_coeffs(sys, p, yb, ab, bb);
  sde_bdiag(sys, p, yp, bp);
  sde_bdiag(sys, p, ym, bm);
  for (int c = 0; c < n; c++)
    xo[c] = x[c] + 0.5 * (ab[c] + a[c]) * h +
            0.25 * (bp[c] + bm[c] + 2.0 * bd[c]) * dW[c] +
            0.25 * (bp[c] - bm[c]) * (dW[c] * dW[c] - h) / sq;
}

int orc_sde_step(int sys, int alg, const double *p, const double *x, double h,
                 const double *dW, double *xout) {
  int n, m;
  if (sde_dims(sys, &n, &m) != 0) return -1;
  if (alg == ORC_EM)
    em_step(sys, p, n, m, x, h, dW, xout);
  else if (alg == ORC_SIEA && sys == ORC_GBM4)
    siea_step(sys, p, n, x, h, dW, xout);
  else
    return -1;
  return 0;
}

int orc_sde(int sys, int alg, int64_t N, const double *params,
            const double *u0, double dt, int n_steps, uint64_t seed,
            const int64_t *ids, double *out, int nthreads) {
  int n, m, np_;
  if (sde_dims(sys, &n, &m) != 0 || orc_dims(sys, &n, &np_) != 0) return -1;
  if (alg != ORC_EM && !(alg == ORC_SIEA && sys == ORC_GBM4)) return -1;
  if (N < 0 || n_steps < 0 || !(dt > 0.0)) return -1;
  if (nthreads < 1) nthreads = 1;
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const double sqdt = sqrt(dt);
#pragma omp parallel for num_threads(nthreads) schedule(static)
  for (int64_t i = 0; i < N; i++) {
    double p[8], X[8], Xn[8], dW[8];
    for (int r = 0; r < np_; r++) p[r] = params[r * N + i];
    for (int c = 0; c < n; c++) X[c] = u0[c * N + i];
    uint64_t id = ids ? (uint64_t)ids[i] : (uint64_t)i;
    for (int s = 0; s < n_steps; s++) {
      for (int call = 0; call * 4 < m; call++) {
        uint32_t ctr[4] = {(uint32_t)s, (uint32_t)id, (uint32_t)(id >> 32), (uint32_t)call};
        uint32_t r[4];
        double z[4];
        orc_philox4x32_10(ctr, key, r);
        orc_box_muller(r[0], r[1], &z[0], &z[1]);
        orc_box_muller(r[2], r[3], &z[2], &z[3]);
        for (int q = 0; q < 4; q++) dW[4 * call + q] = sqdt * z[q];
      }
      if (alg == ORC_EM)
        em_step(sys, p, n, m, X, dt, dW, Xn);
      else
        siea_step(sys, p, n, X, dt, dW, Xn);
      for (int c = 0; c < n; c++) X[c] = Xn[c];
    }
    for (int c = 0; c < n; c++) out[c * N + i] = X[c];
  }
  return 0;
}

int orc_em(int sys, int64_t N, const double *params, const double *u0,
           double dt, int n_steps, uint64_t seed, const int64_t *ids,
           double *out, int nthreads) {
  if (sys != ORC_GBM4) return -1;
  return orc_sde(sys, ORC_EM, N, params, u0, dt, n_steps, seed, ids, out,
                 nthreads);
}
