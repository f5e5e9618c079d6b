/*
 * ens.h -- C ABI of libens.so: ensembles of one small ODE/SDE system solved on
 * an AMD MI355X (gfx950), one whole trajectory per GPU lane inside one kernel.
 *
 * The calls follow the paper's problem statement:
 *   - du/dt = f(u, p, t), u(t0) = u0, t in (t0, tf)            section 3.1, eq. 1
 *   - N trajectories = N columns of U (n x N) and P (m x N)    section 5.1.1, eqs. 12-15
 *   - absolute/relative tolerances of the error control        section 3.1, eq. 4
 *   - solver choice: GPUTsit5, GPURodas4, GPUEM                section 5.2.1, 5.2.2
 *   - the whole integration of a trajectory in one kernel,
 *     saving at requested times                                section 5.2 (EnsembleGPUKernel)
 *   - a lower-level API on device arrays with no host
 *     conversions                                              section 6.1
 *
 * Conventions shared by every call:
 *   - Layout: structure of arrays.  A quantity with r rows per trajectory is a
 *     row-major [r][N] device array; column i (elements k*N + i) belongs to
 *     trajectory i.  Consecutive lanes touch consecutive addresses.
 *   - Ownership: every data pointer is owned by the caller.  The library never
 *     allocates, frees or retains caller memory beyond the call; the context
 *     owns only a small device workspace (queue counters) allocated at
 *     ens_create.
 *   - Streams: `stream` is a hipStream_t (NULL = the legacy default stream).
 *     ens_solve and ens_mlp_* only enqueue work and return; the caller
 *     synchronises.  ens_autotune synchronises the stream it is given.
 *   - Errors: argument errors are returned synchronously as negative codes,
 *     with a message in ens_last_error(ctx); nothing is enqueued then.
 *     Per-trajectory numerical failures never abort a batch: they go to the
 *     optional STATUS array and the unreached save slots are set to NaN.
 *   - Thread safety: one context per host thread; calls on one context must
 *     not overlap.  Calls that overlap on one GPU through different contexts
 *     are independent.
 */
#ifndef ENS_H
#define ENS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ens_ctx ens_ctx;

/* ---- return codes ------------------------------------------------------ */
#define ENS_OK 0
#define ENS_EINVAL (-1)       /* bad argument (null pointer, size, value)      */
#define ENS_ENOMEM (-2)       /* device allocation failed (ens_create only)    */
#define ENS_EDEVICE (-3)      /* a HIP call failed                             */
#define ENS_EUNSUPPORTED (-4) /* valid but unsupported (system, alg, precision) */

/* Largest ensemble of one call: 2^32 - 2^11 trajectories (2^27 - 64 for
 * ENS_SYS_POLLU, which takes a 32-lane group per trajectory), so that every
 * launch's work-items fit the 32-bit dispatch size.  Larger n: ENS_EINVAL. */
#define ENS_MAX_TRAJ 4294965248LL

/* ---- systems (compile-time right-hand sides and analytic Jacobians) ------
 *                         n  m   params rows
 * ENS_SYS_LINEAR          3  9   A row-major: du = A u
 * ENS_SYS_LORENZ          3  3   (sigma, rho, beta)      appendix, Lorenz problem
 * ENS_SYS_ROBERTSON       3  3   (k1, k2, k3): dy1 = -k1 y1 + k3 y2 y3,
 *                                dy2 = k1 y1 - k3 y2 y3 - k2 y2^2, dy3 = k2 y2^2
 *                                                         appendix, Robertson
 * ENS_SYS_GBM4            4  2   (mu, sigma): dX_c = mu X_c dt + sigma X_c dW_c
 *                                                         appendix, linear SDE
 * ENS_SYS_OREGO           3  3   (k1, k2, k3): dy1 = k1 (y2 + y1 (1 - k2 y1 - y2)),
 *                                dy2 = (y3 - (1 + y1) y2) / k1, dy3 = k3 (y1 - y3)
 *                                (textbook sign of dy1)    appendix B.1, OREGO
 * ENS_SYS_HIRES           8  12  the distinct rate constants (1.71, 0.43, 8.32,
 *                                0.0007, 8.75, 10.03, 0.035, 1.12, 1.745, 280,
 *                                0.69, 1.81), each for every occurrence of
 *                                its value                 appendix B.1, HIRES
 * ENS_SYS_POLLU           20 25  (k1 .. k25); one trajectory per 32-lane group
 *                                (plain form only: ENS_OPT_FORM, ENS_OPT_TPL
 *                                and ENS_OPT_GRID are ignored; block 64, 128
 *                                or 256 holds 2, 4 or 8)   appendix B.1, POLLU
 * ENS_SYS_CRN             4  6   (S, D, tau, nu0, n, eta): the sigma-factor
 *                                chemical Langevin SDE, state (s, A1, A2, A3),
 *                                8 Wiener processes; concentrations driven
 *                                below zero enter the Hill term and the
 *                                square roots as 0          appendix, CRN SDE
 */
#define ENS_SYS_LINEAR 0
#define ENS_SYS_LORENZ 1
#define ENS_SYS_ROBERTSON 2
#define ENS_SYS_GBM4 3
#define ENS_SYS_OREGO 4
#define ENS_SYS_HIRES 5
#define ENS_SYS_POLLU 6
#define ENS_SYS_CRN 7

/* ---- algorithms -------------------------------------------------------- */
#define ENS_ALG_TSIT5 1  /* adaptive Tsitouras 5(4), PI control   sec. 3.1, 5.2.1 */
#define ENS_ALG_RODAS4 2 /* adaptive Rosenbrock RODAS4, W = I - gamma h J,
                            FP64 LU and solves              sec. 3.2.1, 5.1.3, 5.2.1 */
#define ENS_ALG_EM 3     /* fixed-step Euler-Maruyama, Philox4x32-10 normals
                                                            sec. 3.3, 5.2.2     */
#define ENS_ALG_SIEA 5   /* fixed-step weak order-2 scheme for diagonal noise
                            (Kloeden-Platen explicit order-2.0 weak scheme, the
                            reading of GPUSIEA), Philox4x32-10 normals as for EM
                                                            sec. 3.3, 5.2.2     */
#define ENS_ALG_RODAS5P 6 /* adaptive Rodas5P (Steinebach 2023): 8-stage stiffly
                            accurate Rosenbrock method of order 5 with an
                            embedded order-4 estimate, W = I - gamma h J,
                            FP64 LU and solves      sec. 3.2.1, 5.2.1, 6.4 */
#define ENS_ALG_ROS23 4  /* adaptive Rosenbrock23: the L-stable 2(3) modified
                            Rosenbrock pair of Shampine & Reichelt, W = I - d h J
                            with d = 1/(2 + sqrt 2), FP64 LU, solves and stage
                            vectors, FSAL                    sec. 3.2.1, 5.2.1 */

/* ---- scalar options (ens_set_option) ------------------------------------ */
#define ENS_OPT_PRECISION 1 /* 32 (default): FP32 state, FP64 time with a
                               TwoSum compensation term (and FP64 W/LU/solves
                               for RODAS4, RODAS5P and ROS23);
                               64: FP64 throughout.  Also the dtype of params,
                               u0 and out.                                      */
#define ENS_OPT_FORM 2      /* 0 (default): one lane per trajectory;
                               1: persistent kernel fed by an atomic work queue,
                               idle lanes refilled one trajectory at a time;
                               2: one lane per trajectory, the trajectories of
                               each block sorted by expected work (span / first
                               step) so that a wave's lanes finish together;
                               3: persistent kernel whose blocks each claim a
                               chunk of `block` trajectories from the atomic
                               queue, sort it by expected work as form 2 does
                               and integrate it (one sorted group of 64 per
                               wave), then claim the next                    */
#define ENS_OPT_BLOCK 3     /* threads per block: 64, 128 or 256 (forms 0, 1, 3);
                               256, 512 or 1024 (form 2, the sorting group);
                               0 (default): 256, or 1024 for form 2            */
#define ENS_OPT_DT 4        /* fixed step of ENS_ALG_EM / SIEA (> 0)             */
#define ENS_OPT_SEED 5      /* 64-bit Philox key of ENS_ALG_EM / SIEA (integer value,
                               exact below 2^53)                                */
#define ENS_OPT_H0 6        /* first step of adaptive solves; 0 (default):
                               Hairer-Norsett-Wanner starting-step heuristic    */
#define ENS_OPT_MAXITERS 7  /* attempted steps per trajectory before status 1
                               (default 1e6)                                    */
#define ENS_OPT_TSPAN_BROADCAST 8 /* 1: tspan is [2] shared by all trajectories;
                                     0 (default): tspan is [2][N]              */
#define ENS_OPT_REFILL 9    /* persistent form: idle lanes per wave that trigger
                               a refill from the queue, 1..64 (default 16)      */
#define ENS_OPT_GRID 10     /* persistent forms (1, 3): blocks launched; 0
                               (default): enough to fill every CU               */
#define ENS_OPT_TPL 11      /* forms 0 and 2: trajectories each lane integrates
                               one after another, 1..8 (default 1).  Form 0:
                               lane g of G takes g, g + G, g + 2G, ...; form 2:
                               1, 2 or 4 rounds (larger values use 4), each
                               block sorting block x rounds trajectories      */
#define ENS_OPT_MLP_TILE 12 /* surrogate inference: fused kernel with 2, 3 or 4
                               16-query subtiles per wave and one wave per SIMD
                               (2, 3, 4), or 2 or 3 subtiles and two waves per
                               SIMD (12, 13; default 13); 0: the layer-by-layer
                               tiled-product path.  Training: any non-zero value
                               selects the fused training kernels, 0 the tiled
                               products                                       */
#define ENS_OPT_SAVE_MODE 13 /* 0 (default): steps land on every save time;
                                1 (ENS_ALG_TSIT5 only, else ENS_EUNSUPPORTED):
                                steps land on the last save time only and the
                                earlier ones are read off the step's 4th-order
                                dense output (section 5.2.1's interpolation) */
#define ENS_OPT_STAGE_SAVES 14 /* 1: the sorted form with block 256 and one
                                  round (ENS_ALG_TSIT5) keeps a block's saves in
                                  LDS (n_save x dim x 256 values, used when they
                                  fit in 64 KiB) and writes them out as whole
                                  rows when the block is done, so HBM writes
                                  equal the output size instead of several
                                  partial write-backs of each 128-byte line;
                                  the LDS it holds lowers the blocks resident
                                  per CU.  0 (default): saves are stored
                                  directly.  Results are bitwise identical.   */
#define ENS_OPT_AUTOTUNE_CACHED 15 /* read-only (ens_get_option): 1 when the
                                      last ens_autotune was answered from the
                                      autotune cache without timing, else 0 */

/* ---- pointer options (ens_set_ptr); NULL disables ------------------------ */
#define ENS_PTR_STATUS 1 /* uint8 [N]: 0 ok, 1 maxiters, 2 step below 16 eps|t|,
                            3 non-finite error estimate or an invalid span
                            (tf < t0 or a non-finite end point)              */
#define ENS_PTR_STATS 2  /* int32 [2][N]: accepted, rejected step counts        */

/* ---- status codes written to ENS_PTR_STATUS ------------------------------ */
#define ENS_ST_OK 0
#define ENS_ST_MAXITERS 1
#define ENS_ST_DTMIN 2
#define ENS_ST_NONFINITE 3

/* Create a context on HIP device `device` (allocates its small workspace).
 * On success *ctx is set and ENS_OK returned.                                */
int ens_create(ens_ctx **ctx, int device);

/* Destroy a context (waits for nothing; the caller must have synchronised
 * any stream that still runs work of this context).  NULL is accepted.      */
int ens_destroy(ens_ctx *ctx);

/* Message of the last error on this context ("" if none). Valid until the
 * next call on the context.                                                  */
const char *ens_last_error(const ens_ctx *ctx);

/* Set / read one scalar option (ENS_OPT_*).  ENS_EINVAL for an unknown key
 * or an out-of-range value.                                                  */
int ens_set_option(ens_ctx *ctx, int key, double value);
int ens_get_option(const ens_ctx *ctx, int key, double *value);

/* Set one optional device output array (ENS_PTR_*); NULL disables it. */
int ens_set_ptr(ens_ctx *ctx, int key, void *device_ptr);

/* n and m of a system; ENS_EINVAL for an unknown id. */
int ens_system_dims(int system_id, int *n, int *m);

/*
 * Solve an ensemble of n_traj trajectories of `system_id` with `alg`.
 *
 *   params     device, [m][n_traj], dtype of ENS_OPT_PRECISION
 *   u0         device, [n][n_traj], same dtype
 *   tspan      device, float64: [2][n_traj] (row 0 t0, row 1 tf, tf >= t0),
 *              or [2] with ENS_OPT_TSPAN_BROADCAST = 1
 *   alg        ENS_ALG_*; (system, alg) must be one of
 *              {LINEAR, LORENZ} x TSIT5,
 *              {LINEAR, LORENZ, ROBERTSON, OREGO, HIRES, POLLU} x {RODAS4,
 *              RODAS5P, ROS23}, {GBM4, CRN} x EM, GBM4 x SIEA
 *   abstol, reltol  > 0 for adaptive algorithms (ignored by EM and SIEA)
 *   save_times HOST, [n_save] fractions theta_j, 0 < theta_0 < ... <= 1; save
 *              j of trajectory i is at t0_i + theta_j (tf_i - t0_i).  Adaptive
 *              solvers step exactly onto every save time.  For EM and SIEA every
 *              theta_j * round((tf - t0)/dt) must be an integer step count.
 *              The array is copied into the launch; it may be freed on return.
 *   n_save     1..64
 *   out        device, [n_save][n][n_traj], same dtype as u0
 *   stream     hipStream_t or NULL
 *
 * n_traj == 0 is a no-op returning ENS_OK (the device pointers may then be
 * NULL).  Returns after enqueueing.
 */
int ens_solve(ens_ctx *ctx, int system_id, int64_t n_traj, const void *params,
              const void *u0, const double *tspan, int alg, double abstol,
              double reltol, const double *save_times, int n_save, void *out,
              void *stream);

/*
 * Mixed systems in one launch.  The paper's kernels give every thread a
 * whole trajectory (section 5.2) and note that adaptive steps make the work
 * per thread uneven (section 6.4); ens_solve_mixed extends the ensemble to
 * several groups, each an ensemble of its own system with its own arrays
 * (laid out as for ens_solve), solved by one kernel launch over a work queue
 * of chunks of 256 trajectories of any group: no chunk mixes systems, and
 * the groups' uneven work is balanced over the whole GPU in one launch
 * instead of one launch running after another.  The queue holds the groups
 * with fewer chunks first.  With ENS_OPT_FORM 3 a persistent grid drains it
 * through an atomic counter; with any other form every chunk is one block of
 * a grid the hardware dispatches (measured faster).  Each chunk is sorted by
 * expected work as in ENS_OPT_FORM 2, and every trajectory gets exactly the
 * bits ens_solve gives it.
 *
 *   groups[g]   system_id; n_traj; params [m][n_traj], u0 [n][n_traj], out
 *               [n_save][n][n_traj] (device, dtype of ENS_OPT_PRECISION);
 *               tspan device float64 [2][n_traj], or [2] when
 *               tspan_broadcast is 1; status uint8 [n_traj] and stats int32
 *               [2][n_traj] device arrays or NULL (as ENS_PTR_STATUS/STATS)
 *   n_groups    1..8; groups with n_traj 0 are allowed
 *   alg         ENS_ALG_TSIT5 (systems LORENZ, LINEAR) or ENS_ALG_RODAS4,
 *               ENS_ALG_RODAS5P, ENS_ALG_ROS23 (systems ROBERTSON, OREGO,
 *               LORENZ, LINEAR); other systems or algorithms ENS_EUNSUPPORTED
 *   abstol, reltol, save_times, n_save   shared by all groups, as ens_solve
 *
 * Context options used: ENS_OPT_PRECISION, H0, MAXITERS, SAVE_MODE, FORM
 * (3: persistent queue, else one block per chunk) and GRID (blocks of the
 * persistent grid; 0 fills every CU); BLOCK, TPL and the context's
 * STATUS/STATS pointers are not.  Returns after enqueueing.
 */
typedef struct ens_group {
  int system_id;
  int tspan_broadcast;
  int64_t n_traj;
  const void *params;
  const void *u0;
  const double *tspan;
  void *out;
  uint8_t *status;
  int32_t *stats;
} ens_group;

int ens_solve_mixed(ens_ctx *ctx, int n_groups, const ens_group *groups, int alg,
                    double abstol, double reltol, const double *save_times,
                    int n_save, void *stream);

/*
 * The raw Philox4x32-10 words the ENS_ALG_EM kernel draws at step `step`:
 * out[k][i] (k = 0..3, uint32, device, [4][n_traj]) = word k of
 * Philox4x32-10(counter = (step, i mod 2^32, i >> 32, 0), key = seed) (the
 * CRN's Wiener increments 5..8 come from a second call with last counter
 * word 1), the
 * generator of Salmon et al. (SC'11) that the paper's SDE kernels leave
 * unnamed (section 6.8.1).  Same device function as the solver kernel.
 */
int ens_philox_fill(ens_ctx *ctx, uint64_t seed, int64_t n_traj, uint32_t step,
                    uint32_t *out, void *stream);

/*
 * Autotuner: time every launch configuration -- block in {64, 128, 256} x
 * (plain form with trajectories per lane in {1, 2, 4}, or persistent form
 * with refill threshold in {4, 16, 32}), the sorted form with block in
 * {256, 512, 1024} sorting one block's worth of trajectories or block in
 * {256, 512} sorting two (ENS_OPT_TPL 2), and the persistent sorted-chunk
 * form with block 128 or 256; the plain form alone for the SDE
 * algorithms, and block alone for ENS_SYS_POLLU (one trajectory per 32-lane
 * group, plain form only) -- on the given probe ensemble (same
 * arguments as ens_solve; `out` is overwritten), and set ENS_OPT_FORM,
 * ENS_OPT_BLOCK, ENS_OPT_TPL and ENS_OPT_REFILL to the fastest.  Results are
 * bitwise identical across configurations, so tuning never changes answers.
 * best_ms (may be NULL) receives its time.  Synchronises `stream`.
 */
int ens_autotune(ens_ctx *ctx, int system_id, int64_t n_traj,
                 const void *params, const void *u0, const double *tspan,
                 int alg, double abstol, double reltol,
                 const double *save_times, int n_save, void *out, void *stream,
                 double *best_ms);
/*
 * The autotuner's results are cached in the context, keyed by (system_id,
 * alg, ENS_OPT_PRECISION, ENS_OPT_SAVE_MODE, floor(log2 n_traj)) -- the
 * occupancy-driven launch tuning of section 5.1.2 done once per problem
 * class instead of once per call.  A key already in the cache is answered
 * without timing anything: the stored configuration is set, *best_ms gets
 * its recorded time, ENS_OPT_AUTOTUNE_CACHED reads 1, and nothing is
 * enqueued.  ens_set_autotune_file attaches a JSON file to the cache: the
 * in-memory cache is replaced by the file's entries for this device
 * (architecture name and CU count; a missing file is an empty cache), and
 * every new result rewrites the file (entries of other devices are kept).
 * path NULL clears the cache and detaches the file.  ENS_EINVAL for an
 * unreadable or malformed file, or one that cannot be written.
 */
int ens_set_autotune_file(ens_ctx *ctx, const char *path);

/* ==========================================================================
 * Learned surrogate: a multilayer perceptron (rho, x0, y0, z0) -> 256 -> 256
 * -> 256 -> 48 (the Lorenz state at 16 save times), SiLU hidden activations,
 * bfloat16 weights and activations with FP32 accumulation on the matrix
 * cores, trained by the library's own forward / backward / Adam kernels on
 * trajectories that ens_solve produces, and audited by the Tsit5 solver,
 * which also answers every query the surrogate is not validated for.  The
 * paper has no such component; it extends the ensemble solve.
 *
 * Ownership: an ens_surrogate owns its device buffers (weights, Adam moments,
 * gradient, normalisation, workspaces) -- the one exception to "the library
 * allocates nothing of the caller's".  Everything else is caller-owned.
 * Inputs use the ens_solve layout of ENS_SYS_LORENZ at precision 32: params
 * [3][n] (sigma, rho, beta; only rho is a network input), u0 [3][n], outputs
 * [16][3][n] float32.
 * ======================================================================== */
typedef struct ens_surrogate ens_surrogate;

#define ENS_SURR_NIN 4
#define ENS_SURR_HIDDEN 256
#define ENS_SURR_NOUT 48
#define ENS_SURR_NPARAM 145200 /* flat: per layer W [out][in] row-major, b [out] */

/* buffers of a model, for ens_surrogate_copy */
#define ENS_SURR_MASTER 1       /* float  [NPARAM] FP32 master weights            */
#define ENS_SURR_WEIGHTS_BF16 2 /* uint16 [NPARAM] bfloat16 copy used by kernels  */
#define ENS_SURR_GRAD 3         /* float  [NPARAM] gradient of the last step      */
#define ENS_SURR_ADAM_M 4       /* float  [NPARAM] Adam first moment              */
#define ENS_SURR_ADAM_V 5       /* float  [NPARAM] Adam second moment             */
#define ENS_SURR_NORM 6         /* float  [160]: input mean[4], 1/std[4], min[4],
                                   max[4]; output mean[48], 1/std[48], std[48]   */

/* Allocate a model on the context's device; weights He-uniform from
 * Philox4x32-10(seed), biases 0, identity normalisation.  Synchronises the
 * device.                                                                    */
int ens_surrogate_create(ens_ctx *ctx, uint64_t seed, ens_surrogate **out);
int ens_surrogate_destroy(ens_surrogate *s);
/* Copy one model buffer (ENS_SURR_*) to (to_model = 0) or from (to_model = 1)
 * the caller's device array `dev_ptr` of the buffer's size, on `stream`.
 * Writing ENS_SURR_MASTER also refreshes the bfloat16 weights.               */
int ens_surrogate_copy(ens_ctx *ctx, ens_surrogate *s, int which, void *dev_ptr,
                       int to_model, void *stream);
/* Write the model -- FP32 master weights, Adam moments and step, and the
 * normalisation -- to a file, or read one back into a model (the bfloat16
 * weights are re-derived), so training can resume and a trained surrogate
 * can be served by another process.  Format: "ENSSURR1", uint32 version (1),
 * uint32 parameter count, int64 Adam step, uint32 normalisation size (160),
 * then the float32 arrays master, m, v, norm (little-endian).  Both
 * synchronise the device.  ENS_EINVAL for an unreadable, unwritable or
 * mismatched file (the model is then unchanged).                           */
int ens_surrogate_save(ens_ctx *ctx, ens_surrogate *s, const char *path);
int ens_surrogate_load(ens_ctx *ctx, ens_surrogate *s, const char *path);
/* Adam step counter (bias correction); restored with the moments on resume. */
int ens_surrogate_get_step(const ens_surrogate *s, int64_t *step);
int ens_surrogate_set_step(ens_surrogate *s, int64_t step);

/* Normalisation from a training set: per input feature and per output row,
 * mean and standard deviation over n trajectories (FP64 sums, fixed order),
 * and the input min / max that bound the validated region.  y [48][n].     */
int ens_surrogate_fit_norm(ens_ctx *ctx, ens_surrogate *s, const float *params,
                           const float *u0, const float *y, int64_t n,
                           void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * minibatch of items first .. first+batch-1, item b being trajectory
 * (mult * b + add) mod n (mult coprime with n: a permutation of the set).
 * Loss = mean squared error of the normalised outputs; written to *loss
 * (device float) when loss is not NULL.  batch <= ENS_SURR_MAX_BATCH, else
 * ENS_EINVAL (here and in ens_surrogate_train).                              */
#define ENS_SURR_MAX_BATCH 268435456LL /* 2^28 */
int ens_surrogate_train_step(ens_ctx *ctx, ens_surrogate *s,
                             const float *params, const float *u0,
                             const float *y, int64_t n, int64_t first,
                             int64_t batch, uint64_t mult, uint64_t add,
                             double lr, float *loss, void *stream);

/* `epochs` passes over floor(n / batch) minibatches, a fresh pseudo-random
 * permutation per epoch drawn from `seed`, learning rate decayed from lr_max
 * to lr_min on a cosine; epoch_loss (device float [epochs], may be NULL)
 * receives the loss of each epoch's last minibatch.  With the fused kernels
 * (ENS_OPT_MLP_TILE != 0) the call first stages the set item-major and
 * normalised in a workspace the model keeps (208 bytes per trajectory);
 * the steps are identical to ens_surrogate_train_step calls.                 */
int ens_surrogate_train(ens_ctx *ctx, ens_surrogate *s, const float *params,
                        const float *u0, const float *y, int64_t n, int epochs,
                        int64_t batch, double lr_max, double lr_min,
                        uint64_t seed, float *epoch_loss, void *stream);

/* Surrogate answers for n queries into out [48][n] = [16][3][n]. */
int ens_surrogate_predict(ens_ctx *ctx, ens_surrogate *s, const float *params,
                          const float *u0, int64_t n, float *out, void *stream);

/*
 * Audited surrogate solve of n Lorenz queries (same arguments as ens_solve
 * for ENS_SYS_LORENZ / ENS_ALG_TSIT5 at precision 32, n_save must be 16; the
 * solver runs in the context's ENS_OPT_SAVE_MODE):
 *   1. each query is audited with probability audit_frac (Philox4x32-10 on
 *      the query id and audit_seed): the surrogate and the FP32 Tsit5 kernel
 *      both answer it, and it returns the solver's answer;
 *   2. if an audited query's normwise error (max over save times of
 *      ||surrogate - solver||_inf / ||solver||_inf) exceeds fallback_tol, its
 *      rho bin (28 equal bins over the training range of rho) is flagged;
 *   3. every other query in a flagged bin, or outside the training box (any
 *      input outside its training min / max), is solved by the solver;
 *   4. the surrogate answers the rest.
 * With the fused inference kernel (ENS_OPT_MLP_TILE != 0) the network is
 * evaluated only on the audited queries and those of step 4; with the tiled
 * path it answers every query first (answers later replaced).
 * used_solver (device uint8 [n], may be NULL): 0 surrogate, 1 audited,
 * 2 fallback.  report (device float [4], may be NULL): audited count,
 * fallback count, flagged bins, max audited error.  Asynchronous.
 */
int ens_surrogate_solve(ens_ctx *ctx, ens_surrogate *s, const float *params,
                        const float *u0, const double *tspan, double abstol,
                        double reltol, const double *save_times, int n_save,
                        int64_t n, double audit_frac, double fallback_tol,
                        uint64_t audit_seed, float *out, uint8_t *used_solver,
                        float *report, void *stream);

/*
 * ens_surrogate_solve without any device allocation, for callers that cannot
 * allocate device memory during the call: code under stream capture, serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, results and
 * report as ens_surrogate_solve (the same kernels), but its workspace --
 * audit and fallback lists, the audited answers, per-query flags, counters
 * and bin flags -- is one static device array per GPU of about 25 MiB,
 * held from the first ens_create on that GPU until the process ends,
 * instead of buffers the model allocates on demand.  Limits: n at most
 * ENS_STATIC_MAX_QUERIES, an audit list of at most 40960 entries (audit_frac
 * up to 2% at that n; more is ENS_EINVAL), and the fused inference kernel
 * (ENS_OPT_MLP_TILE 0 gives ENS_EUNSUPPORTED).  Every static call on a GPU
 * shares that array and the previous call's contents remain (the call
 * clears its counters and flags itself), so calls that overlap on one GPU,
 * from any context or stream, race: serialise them.  Asynchronous.
 */
#define ENS_STATIC_MAX_QUERIES 1048576LL
int ens_surrogate_solve_static(ens_ctx *ctx, ens_surrogate *s,
                               const float *params, const float *u0,
                               const double *tspan, double abstol,
                               double reltol, const double *save_times,
                               int n_save, int64_t n, double audit_frac,
                               double fallback_tol, uint64_t audit_seed,
                               float *out, uint8_t *used_solver, float *report,
                               void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ENS_H */
