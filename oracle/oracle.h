/*
 * oracle.h -- plain, slow, FP64 CPU reference integrators for ensembles of one
 * small ODE/SDE system.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) may include, link or call this code; only the tests, the
 * smoke check and the benchmark's CPU-baseline leg do.  It shares no code,
 * header, table or constant with the GPU implementation.
 *
 * Layout convention (the array-ensemble formulation of the paper, section 5.1.1,
 * eqs. 12-15): a quantity with r rows per trajectory and N trajectories is a
 * row-major C array [r][N], i.e. column j of U (n x N) / P (m x N) holds
 * trajectory j.
 */
#ifndef ENS_ORACLE_H
#define ENS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Systems (all autonomous, so the df/dt term of the Rosenbrock formula is 0). */
enum {
  ORC_LINEAR = 0,    /* du/dt = A u, n = 3, p = A row-major (m = 9)              */
  ORC_LORENZ = 1,    /* appendix, Lorenz problem: p = (sigma, rho, beta), n = 3   */
  ORC_ROBERTSON = 2, /* appendix, Robertson equation: p = (k1, k2, k3), n = 3     */
  ORC_GBM4 = 3,      /* appendix, linear SDE with 4 components: p = (mu, sigma)   */
  ORC_OREGO = 4,     /* appendix B.1 (OREGO), Oregonator: p = (k1, k2, k3), n = 3;
                        dy1 = k1 (y2 + y1 (1 - k2 y1 - y2)) -- the textbook
                        (Field-Noyes) sign: the leading minus printed in the
                        paper makes the solution from y = (1, 2, 3) blow up   */
  ORC_HIRES = 5,     /* appendix B.1 (HIRES), n = 8, p = 12 distinct rate constants   */
  ORC_POLLU = 6,     /* appendix B.1 (POLLU), n = 20, p = (k1 .. k25)                 */
  ORC_CRN = 7        /* appendix, sigma-factor CRN SDE (chemical Langevin), n = 4,
                        p = (S, D, tau, nu0, n, eta), 8 Wiener processes         */
};
enum { ORC_TSIT5 = 1, ORC_RODAS4 = 2, ORC_ROS23 = 3, ORC_EM = 4, ORC_SIEA = 5,
       ORC_RODAS5P = 6 };
enum { ORC_OK = 0, ORC_MAXITERS = 1, ORC_DTMIN = 2, ORC_NONFINITE = 3 };

int orc_dims(int sys, int *n, int *m);

/* Right-hand side f(u, p) and analytic Jacobian J[n][n] (row-major). */
int orc_rhs(int sys, const double *p, const double *u, double *du);
int orc_jac(int sys, const double *p, const double *u, double *J);

/*
 * Adaptive solve of an ensemble.  params [m][N], u0 [n][N], tspan [2][N]
 * (row 0 = t0, row 1 = tf), theta [n_save] strictly increasing fractions in
 * (0, 1]: save time j of trajectory i is t0_i + theta_j (tf_i - t0_i).
 * out [n_save][n][N].  status [N], naccept [N], nreject [N] may be NULL.
 * h0 <= 0 selects the starting-step heuristic; h0 > 0 is used as given.
 * Returns 0, or -1 on a bad argument.
 */
int orc_solve(int sys, int alg, int64_t N, const double *params,
              const double *u0, const double *tspan, double atol,
              double rtol, const double *theta, int n_save, double *out,
              int *status, int64_t *naccept, int64_t *nreject, double h0,
              int64_t maxiters, int nthreads);

/* orc_solve with a save mode: 0 as orc_solve (steps land on every save
 * time); 1 (Tsit5) steps land only on the last save time and the others are
 * read off the dense output of the step covering them.                     */
int orc_solve_mode(int sys, int alg, int64_t N, const double *params,
                   const double *u0, const double *tspan, double atol,
                   double rtol, const double *theta, int n_save, double *out,
                   int *status, int64_t *naccept, int64_t *nreject, double h0,
                   int64_t maxiters, int nthreads, int save_mode);

/* Tsit5 dense-output coefficients B[i][m] (b_i(theta) = sum_m B[i][m] theta^(m+1)). */
void orc_tsit5_dense_table(double B[28]);

/* n_steps fixed Tsit5 steps of size h, the last one read at theta:
 * u(t0 + (n_steps - 1 + theta) h).                                          */
int orc_fixed_dense(int sys, const double *p, const double *u0, double h,
                    int n_steps, double theta, double *u_out);

/* n_steps fixed steps of size h from u0 for one trajectory.  u_out gets the
 * propagated solution, uhat_out the embedded (lower-order) one.            */
int orc_fixed(int sys, int alg, const double *p, const double *u0, double h,
              int n_steps, double *u_out, double *uhat_out);

/* Philox4x32 with 10 rounds (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);

/* Uniform in (0,1) from a 32-bit word and the Box-Muller pair of normals. */
double orc_uniform(uint32_t x);
void orc_box_muller(uint32_t x0, uint32_t x1, double *z0, double *z1);

/*
 * Euler-Maruyama, fixed step, diagonal noise, for ORC_GBM4 (section 3.3,
 * eq. 11; method GPUEM of section 5.2.2).  Step s of trajectory id draws its
 * four Wiener increments from Philox4x32-10 with key (seed_lo, seed_hi) and
 * counter (s, id_lo, id_hi, 0); column k has id ids[k] (ids NULL: id = k).
 * out [n][N] = state at t0 + n_steps*dt.
 */
int orc_em(int sys, int64_t N, const double *params, const double *u0,
           double dt, int n_steps, uint64_t seed, const int64_t *ids,
           double *out, int nthreads);

/*
 * Fixed-step SDE ensemble: alg ORC_EM (any system: ORC_GBM4, ORC_CRN) or
 * ORC_SIEA (diagonal noise: ORC_GBM4).  The m Wiener increments of step s of
 * trajectory id are sqrt(dt) z_j, z_0..z_3 from Philox counter
 * (s, id_lo, id_hi, 0) and z_4..z_7 from (s, id_lo, id_hi, 1), each word
 * pair through Box-Muller.  Arguments as orc_em.
 */
int orc_sde(int sys, int alg, int64_t N, const double *params,
            const double *u0, double dt, int n_steps, uint64_t seed,
            const int64_t *ids, double *out, int nthreads);

/* One step of size h from x with the given Wiener increments dW[m]. */
int orc_sde_step(int sys, int alg, const double *p, const double *x, double h,
                 const double *dW, double *xout);

/* Coefficient export for the order-condition tests. */
void orc_tsit5_tableau(double c[7], double a[49], double b[7],
                       double btilde[7]);
void orc_rodas4_tableau(double *gamma, double a[36], double C[36],
                        double m[6], double mhat[6]);
/* Rodas5P (8 stages, a and C row-major [8][8], weights m, mhat [8]). */
void orc_rodas5p_tableau(double *gamma, double a[64], double C[64],
                         double m[8], double mhat[8]);

#ifdef __cplusplus
}
#endif
#endif
