/*
 * rpr.h -- C ABI of librpr, RandNet-Parareal on AMD MI355X (gfx950).
 *
 * RandNet-Parareal (arXiv 2411.06225) solves the initial value problem
 *     du/dt = h(u),  u(t0) = u0,  t in [t0, tN]                (Sec. 1, eq. "ode")
 * parallel in time: [t0, tN] is cut into N equal slices, an accurate fine
 * propagator F runs on all unfinished slices at once, and a cheap coarse
 * propagator G is corrected by a random network whose readout is fitted by
 * ridge regression to the observed F - G discrepancies (Sec. 2-4).
 *
 * Conventions shared by every entry point
 *   - Every call returns rpr_status; no C++ exception crosses this boundary.
 *     On a non-OK status rpr_last_error() returns a message for the calling
 *     thread.
 *   - "device pointer" means memory allocated on the current HIP device
 *     (e.g. torch.Tensor.data_ptr() of a CUDA tensor); "host pointer" means
 *     ordinary CPU memory.  The library never frees memory it did not
 *     allocate.
 *   - `stream` is a hipStream_t passed as void* (0 = the null stream).  Work is
 *     enqueued asynchronously on it; results are valid once the stream has been
 *     synchronised.  Argument errors are reported synchronously, before
 *     anything is enqueued.
 *   - Arrays are row-major.  A state u in R^d is stored species-planar,
 *     [species][y][x] with x fastest (Burgers: [x]).
 *   - Slices are equal: t_i = t0 + i (tN - t0) / N.  A propagator with `steps`
 *     steps per slice uses dt = ((tN - t0) / N) / steps, computed in double
 *     precision in exactly this order.
 */
#ifndef RPR_H
#define RPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RPR_OK = 0,
    RPR_NOT_CONVERGED = 1,      /* iteration cap reached before every slot was final;
                                   outputs hold the last iterate */
    RPR_ERR_INVALID_ARG = -1,   /* bad argument; nothing was enqueued */
    RPR_ERR_NO_DEVICE = -2,     /* no usable gfx950 device */
    RPR_ERR_HIP = -3,           /* a HIP runtime call failed (message has the HIP error) */
    RPR_ERR_OOM = -4,           /* device allocation failed */
    RPR_ERR_NONFINITE = -5,     /* non-finite values where the method needs finite ones */
    RPR_ERR_NOT_SPD = -6,       /* ridge matrix not numerically positive definite */
    RPR_ERR_UNSTABLE = -7,      /* stability pre-check failed (opt.stability = 1 only) */
    RPR_ERR_UNSUPPORTED = -8    /* a valid combination the library does not implement */
} rpr_status;

/* Message of the last failed call on this thread ("" if none). */
const char *rpr_last_error(void);
/* Library version string, e.g. "rpr 0.1 gfx950". */
const char *rpr_version(void);

/* ---- problem: the spatial right-hand side h of eq. "ode" ----------------- */
typedef enum {
    RPR_BURGERS1D = 0,   /* Sec. 5.1, eq. "burg": nu u_xx - u u_x, periodic, central
                            differences; p[0] = nu; d = nx, ny = 1 */
    RPR_DIFFREACT2D = 1, /* Sec. 5.2: FitzHugh-Nagumo two-species diffusion-reaction,
                            cell-centred finite volumes, no-flux walls;
                            p = (Du, Dv, c); d = 2 nx ny, layout [u; v] */
    RPR_BRUSS2D = 2,     /* App. E: Brusselator, periodic; p = (A, B, Du, Dv);
                            d = 2 nx ny, layout [u; v] */
    RPR_SWE2D = 3,       /* Sec. 5.3: shallow water (h, hu, hv), flat bottom, first-order
                            finite volumes with the Rusanov flux, reflective walls;
                            p[0] = g; d = 3 nx ny, layout [h; hu; hv] */
    RPR_BRUSS3D = 4      /* App. E: Brusselator in three dimensions, periodic, seven-point
                            Laplacian on the box (x0, x1) x (y0, y1) x (x0, x1);
                            p = (A, B, Du, Dv); d = 2 nx ny nz, layout [u; v] with
                            cell (i, j, l) at i + nx (j + ny l) */
} rpr_rhs_kind;

typedef struct {
    int32_t kind;              /* rpr_rhs_kind */
    int32_t nx, ny;            /* points (1D) or cells (2D, 3D) per direction; ny = 1 in 1D */
    int32_t nz;                /* cells along z: >= 1 for RPR_BRUSS3D, 0 or 1 otherwise */
    double x0, x1, y0, y1;     /* domain; grid spacing (x1 - x0) / nx, (y1 - y0) / ny */
    double p[6];               /* physical parameters, see rpr_rhs_kind */
} rpr_rhs;

/* ---- propagators F and G (Sec. 2; App. G setup tables) ------------------ */
/* forward Euler, classical RK4, and the eighth-order 11-stage method of
 * Cooper and Verner (1972), the paper's fine solver for the 3D Brusselator */
typedef enum { RPR_RK1 = 1, RPR_RK4 = 4, RPR_RK8 = 8 } rpr_method;

typedef struct {
    int32_t method;            /* rpr_method */
    int32_t threads;           /* kernel of the propagator: 0 automatic (on chip,
                                  one work-group per slot state, with the
                                  autotuner's work-group size, else 1024, when the
                                  state fits one work-group; otherwise tiled);
                                  512 or 1024 fix the on-chip work-group size (512
                                  exists for the 64 x 64 grids only); 256 selects
                                  the tiled form (2D grids: slot states in memory,
                                  one pass over 64 x 16-cell tiles per RK stage, or
                                  for RK4 on the 5-point Laplacian systems one pass
                                  per step over 64 x 32-cell tiles with a 4-cell
                                  halo); 128 selects the generic form (any
                                  method, slot states in memory, one pass per
                                  stage over the cells of all states), the
                                  only form of RPR_RK8 and of RPR_BRUSS3D.
                                  Other sizes give RPR_ERR_INVALID_ARG, sizes
                                  without a kernel RPR_ERR_UNSUPPORTED.  Batch
                                  plans choose their own and ignore it. */
    int64_t steps;             /* fixed steps per slice, >= 1 */
} rpr_propagator;

/* ---- the random network of eq. "HA" and its ridge readout ----------------- */
typedef enum { RPR_TANH = 0, RPR_RELU = 1 } rpr_activation;

typedef struct {
    int32_t M;                 /* hidden neurons, 1 <= M <= 512 */
    int32_t activation;        /* rpr_activation (the paper uses ReLU, Sec. 4) */
    double lambda;             /* ridge penalty of eq. "ridgeless" (> 0) */
    double input_scale;        /* the network sees x / s; <= 0 selects the default:
                                  the smallest power of two s >= max(1, ||u0||_inf) */
    int32_t m_nn;              /* RPR_CORR_RANDNET_NN only: nearest stored pairs each
                                  prediction is fitted on, 1 <= m_nn <= 32 (the paper
                                  uses 3 or 4, App. G tables); ignored otherwise */
    int32_t reserved;          /* must be 0 */
} rpr_randnet;

typedef enum {
    RPR_FP64 = 0,              /* every step in double precision */
    RPR_MIXED = 1              /* slot states, F and G in single precision (state
                                  updates compensated); hidden layer in bfloat16
                                  with single-precision sums on the matrix cores;
                                  Gram and readout statistics, ridge Cholesky and
                                  convergence norm in double */
} rpr_precision;

typedef enum {
    RPR_CORR_RANDNET = 0,      /* eq. "HA" with the readout of eq. "ridgeless" fitted on
                                  every pair of eq. "Dk" collected so far */
    RPR_CORR_PARAREAL = 1,     /* eq. "fpara": (F - G)(U_{i-1}^{k-1}) */
    RPR_CORR_RANDNET_NN = 2    /* eq. "randnet": every prediction refits the readout
                                  of eq. "ridgeless" on the m_nn stored pairs whose
                                  inputs are nearest (Euclidean) to the slot input
                                  (Alg. "RandNets training procedure"; App. B), in
                                  the dual form W = Phi~^T (Phi~ Phi~^T + lambda I)^-1 Y~
                                  (identical to the primal form); ties between
                                  equal distances go to the earlier pair.  The plan
                                  stores every pair: 2 N k_max d states plus
                                  N k_max M doubles of features. */
} rpr_correction;

typedef enum {
    RPR_FEAT_AUTO = 0,         /* FP64 for RPR_FP64 plans, split bfloat16 for RPR_MIXED
                                  plans (training features; the predictor-corrector
                                  sweep evaluates the hidden layer in double) */
    RPR_FEAT_FP64 = 1,         /* training features in double precision */
    RPR_FEAT_BF16 = 2          /* split-bfloat16 products, single-precision sums on the
                                  matrix cores (see rpr_randnet_features_bf16) */
} rpr_feature_precision;

typedef struct {
    int32_t precision;         /* rpr_precision: slot states, F and G */
    int32_t correction;        /* rpr_correction */
    int32_t k_max;             /* iteration cap, 1 <= k_max <= N (0 selects N) */
    int32_t poll_every;        /* iterations enqueued between checks of the device
                                  "done" flag (0 selects 2) */
    int32_t features;          /* rpr_feature_precision */
    int32_t autotune;          /* 0: launch shapes from built-in rules; 1: time the
                                  candidate shapes at plan creation and keep the
                                  fastest (results cached per shape class in the
                                  process, and in the JSON file named by the
                                  environment variable RPR_TUNE_CACHE if set) */
    int32_t graph;             /* 1: capture a block of poll_every iterations as a
                                  hipGraph on the first execute (again when the input
                                  scale changes) and replay it; 0: plain launches */
    int32_t stability;         /* stability pre-check of F and G (rpr_stability at
                                  u0): 0 records the ratios in rpr_info; 1 (strict)
                                  also returns RPR_ERR_UNSTABLE from rpr_plan_create
                                  when a ratio exceeds 1 for every state (the
                                  state-independent part of the bound) and from
                                  rpr_plan_execute, before anything is enqueued,
                                  when it exceeds 1 at u0 */
    int32_t chain_wgs;         /* work-groups of the predictor-corrector sweep
                                  (0: automatic, or the autotuner's choice); more
                                  than the device holds at once are cut to that
                                  number.  The results do not depend on it except
                                  through the summation order of the hidden
                                  layer's partial sums, which follow the column
                                  blocks of the work-groups. */
    int32_t sweep_form;        /* how a plan without graph capture launches the
                                  predictor-corrector sweep (Sec. 2; the same
                                  values either way): 1 one cooperative kernel
                                  whose segments (per slot: coarse solve, then
                                  readout and update) are separated by grid
                                  barriers; 2 one kernel per segment, the kernel
                                  boundaries as the barriers (the form graph
                                  capture records); 0 automatic: 2 when the coarse
                                  solver runs over the whole grid (tiled and
                                  generic propagators), else 1.  Graph plans
                                  always use 2. */
} rpr_options;

/* ---- plans: one IVP solved by RandNet-Parareal -------------------------- */
typedef struct rpr_plan rpr_plan;

/*
 * Create a plan for the problem (h, u0 of dimension d, [t0, tN], N, F, G, tol)
 * of Sec. 2 and Algorithm "Parareal (generic)".
 *   h, F, G, net, opt : host pointers, read during the call only.
 *   d                 : state dimension; must equal species * nx * ny of h.
 *   tol               : epsilon of eq. "stop_crit" (>= 0; +inf stops after one
 *                       iteration, 0 forces N iterations).
 *   A, zeta           : optional host arrays (M x d and M, doubles) with the
 *                       hidden-layer weights and biases, copied during the call;
 *                       if both are NULL they are drawn on the device from the
 *                       counter-based generator rpr_uniform_pm1 with `seed`:
 *                       A[m][j] = counter m*d + j, zeta[m] = counter M*d + m.
 *                       Ignored (may be NULL) for RPR_CORR_PARAREAL.
 * Allocates every device buffer the solve needs (the plan owns them).
 * Errors: RPR_ERR_INVALID_ARG, RPR_ERR_NO_DEVICE, RPR_ERR_OOM, RPR_ERR_HIP,
 * RPR_ERR_UNSUPPORTED (e.g. a state too large for the library's kernels).
 */
rpr_status rpr_plan_create(rpr_plan **plan, const rpr_rhs *h, int32_t d, double t0, double tN,
                           int32_t N, const rpr_propagator *F, const rpr_propagator *G, double tol,
                           const rpr_randnet *net, const double *A, const double *zeta,
                           uint64_t seed, const rpr_options *opt);

/*
 * Run the solve.  u0: device pointer, d doubles.  U_out: device pointer,
 * (N + 1) x d doubles, caller-owned; receives U_0^K .. U_N^K.  Enqueued on
 * `stream`; the call returns once the run has finished on the device (it
 * polls a device flag every opt.poll_every iterations), so U_out is valid on
 * return.  Returns RPR_OK, or RPR_NOT_CONVERGED if k_max iterations ended
 * with unfinished slots (U_out then holds the last iterate), or an error.
 * A non-finite u0 returns RPR_ERR_NONFINITE.
 */
rpr_status rpr_plan_execute(rpr_plan *plan, const void *u0, void *U_out, void *stream);

typedef struct {
    int32_t K;                 /* iterations run */
    int32_t L_final;           /* slots U_0..U_L are final */
    int32_t converged;         /* 1 if L reached N */
    int32_t rows_used;         /* finite training pairs accumulated in the readout */
    int32_t nonfinite_rows;    /* pairs dropped because of a non-finite entry */
    int32_t chol_fail;         /* ridge matrices that failed Cholesky: iterations of
                                  RPR_CORR_RANDNET, predictions of RPR_CORR_RANDNET_NN
                                  (such a prediction adds no correction) */
    double input_scale;        /* s actually used */
    double t_total;            /* seconds of device time of the last execute */
    /* The same time by phase of Alg. "Parareal (generic)" (seconds of device
       time, from events recorded between the phases; -1 for plans that run
       as a captured graph, where no event separates them; for an instance of
       a batch plan, the batch's times, as t_total): the fine solves, the
       model (training pairs, features, ridge statistics and solve, or the
       pair store of the nearest-neighbour correction), and the sequential
       predictor-corrector sweeps, the first coarse sweep of the set-up
       included. */
    double t_fine;
    double t_model;
    double t_sweep;
    /* Stability pre-check at u0 (rpr_stability): dt / dt_max of F and G, and
       bit 0 (F) / bit 1 (G) set where that ratio exceeds 1.  Sec. 6: an
       unsuitable G keeps the iteration from converging; the run then degrades
       to K = N (non-finite pairs are dropped). */
    double stab_F;
    double stab_G;
    int32_t unstable;
    int32_t reserved;
} rpr_info;

/* Results of the last execute (host pointer `info`). */
rpr_status rpr_plan_info(const rpr_plan *plan, rpr_info *info);

/* Per-iteration history of the last execute into host arrays of length cap:
 * L_hist[k] = L after iteration k (k = 0..K), chg_hist[k] = largest
 * infinity-norm change of the predicted slots at iteration k (NaN counts as
 * +inf).  Either pointer may be NULL. */
rpr_status rpr_plan_history(const rpr_plan *plan, int32_t *L_hist, double *chg_hist, int32_t cap);

/*
 * Batches: n_inst independent IVPs (same right-hand-side kind, precision and
 * correction; sizes, parameters, slices and propagators may differ), solved
 * together.  Every argument is an array of n_inst entries with the meaning of
 * the rpr_plan_create argument of the same name (A, zeta: arrays of host
 * pointers, or NULL to draw instance b's weights with seed + b); opt is
 * shared.  Per iteration the fine solves of every unfinished slot of every
 * instance run in one persistent launch whose work-groups take (instance,
 * slot) items from a longest-first list, and all instances' predictor-
 * corrector sweeps run in one launch, one work-group per instance.
 * Errors as rpr_plan_create; RPR_ERR_UNSUPPORTED if the instances' grids
 * cannot share the strip shape of the largest one.
 */
rpr_status rpr_plan_create_batch(rpr_plan **plan, int32_t n_inst, const rpr_rhs *h, const int32_t *d,
                                 const double *t0, const double *tN, const int32_t *N,
                                 const rpr_propagator *F, const rpr_propagator *G, const double *tol,
                                 const rpr_randnet *net, const double *const *A, const double *const *zeta,
                                 uint64_t seed, const rpr_options *opt);

/* Run a batch: u0[b] and U_out[b] are device pointers of instance b (host
 * arrays of n_inst pointers), with the layout of rpr_plan_execute.  Returns
 * RPR_OK once every instance has converged, RPR_NOT_CONVERGED otherwise. */
rpr_status rpr_plan_execute_batch(rpr_plan *plan, const void *const *u0, void *const *U_out, void *stream);

/* The plan of instance b of a batch, for rpr_plan_info / rpr_plan_history.
 * The handle belongs to the batch: do not destroy it. */
rpr_status rpr_plan_instance(const rpr_plan *batch, int32_t b, const rpr_plan **inst);

/*
 * Stability pre-check of one propagator (host only: touches no device).
 * Sec. 6 notes that an unsuitable coarse solver keeps Parareal from
 * converging; an explicit Runge-Kutta step is stable only while dt times the
 * spectral radius of h's Jacobian lies in the method's stability region.
 * The spectral radius is bounded from the grid, h's parameters and the state
 * (a real part rho_r from diffusion, reaction and the Rusanov dissipation; an
 * imaginary part rho_i from central-difference advection):
 *   Burgers        rho_r = 4 nu/dx^2, rho_i = umax/dx
 *   diffusion-reaction  rho_r = max(Du,Dv)(4/dx^2 + 4/dy^2) + 2 + 3 umax^2
 *   Brusselator    rho_r = max(Du,Dv)(4/dx^2 + 4/dy^2) + B + 1 + 3 umax^2
 *   shallow water  rho_r = 2 speed (1/dx + 1/dy)
 * and *ratio = dt / dt_max with dt_max = min(2 / rho_r, rho_r / (2 rho_i^2))
 * for forward Euler and 2.78 / (rho_r + rho_i) for classical RK4; a ratio
 * above 1 flags the step as outside the stability region.
 *   umax  : max |u| of the state (>= 0);
 *   speed : largest wave speed |velocity| + sqrt(g h) (shallow water; ignored
 *           otherwise, >= 0).
 * Errors: RPR_ERR_INVALID_ARG.
 */
rpr_status rpr_stability(const rpr_rhs *h, int32_t d, const rpr_propagator *P, double dt, double umax,
                         double speed, double *ratio);

/*
 * The autotuner's table of launch shapes (rpr_options.autotune), shared by
 * every plan and call of the process; a shape changes the launch, not the
 * arithmetic of any value.  rpr_tune_set stores value under key (a negative
 * value removes the key, so that the autotuner measures that class again);
 * rpr_tune_get reads it (RPR_ERR_INVALID_ARG if absent).  Keys of the fine
 * propagator, for right-hand side kind on an nx x ny grid, values of
 * `bytes` (8 or 4) and method m:
 *   "prop:<kind>:<nx>x<ny>:<bytes>:<m>"    work-group size (1024, 512, or 256 =
 *                                          the tiled form)
 *   "prop:<kind>:<nx>x<ny>:<bytes>:<m>:v"  tile shape of the tiled form's
 *                                          one-pass RK4 kernel, 0 ..
 *                                          rpr_tile_shapes() - 1
 * and of the predictor-corrector sweep of a plan with M neurons, N slots,
 * correction c and bf16 training features f (0 or 1):
 *   "chain:<kind>:<nx>x<ny>:<bytes>:M<M>:N<N>:<c>:<f>"    work-groups
 *   "chain:...:<f>:B"  work-group size of a sweep in segment kernels over a
 *                      tiled grid with a forward-Euler G: 256, or 1024 for
 *                      four times the wavefronts per CU
 * (a plan with autotune = 1 takes the stored entries of its class and times
 * the missing ones).
 * rpr_propagate with threads 256 takes the tile shape stored for its class;
 * a shape that does not serve the grid returns RPR_ERR_UNSUPPORTED.
 * Errors: RPR_ERR_INVALID_ARG (null or empty key, null value).
 */
rpr_status rpr_tune_set(const char *key, int32_t value);
rpr_status rpr_tune_get(const char *key, int32_t *value);

/* Number of tile shapes of the one-pass RK4 kernel for right-hand side kind
 * at precision (1 where the kind has none), and the name of shape v
 * (NULL outside 0 .. count - 1): "R<rows per wavefront>NW<wavefronts>" for
 * 56-column tiles with a 4-cell halo, "rows:C<cells per lane>R..NW.." for
 * the full-row form (grids with nx <= 64 C and nx a multiple of C),
 * "FY<tile rows>NT<threads>" for the Laplacian systems. */
int32_t rpr_tile_shapes(int32_t kind, int32_t precision);
const char *rpr_tile_shape_name(int32_t kind, int32_t precision, int32_t v);

/* Release every buffer of the plan (a batch releases its instances).  NULL is accepted. */
rpr_status rpr_plan_destroy(rpr_plan *plan);

/* ---- building blocks (the same kernels the plan runs) -------------------- */

/*
 * Propagate n_states independent states over one slice: out[r] = P(in[r]).
 * Sec. 2: F and G map the state at the start of a slice to its end.
 *   in, out   : device pointers, n_states x d, doubles if precision = RPR_FP64,
 *               floats if RPR_MIXED; must not overlap.
 *   dt        : step length; P->steps steps are taken.
 * Work-group size: P->threads, or when 0 the one the autotuner chose for this
 * grid, precision and method in the same process (rpr_options.autotune), else
 * 1024.
 */
rpr_status rpr_propagate(const rpr_rhs *h, int32_t d, const rpr_propagator *P, int32_t precision,
                         double dt, int32_t n_states, const void *in, void *out, void *stream);

/*
 * Hidden-layer features of eq. "HA": Phi[r][m] = sigma(sum_j A[m][j] (X[r][j] / s) + zeta[m]).
 *   A (M x d), zeta (M), X (n x d), Phi (n x M): device pointers, doubles.
 */
rpr_status rpr_randnet_features(int32_t M, int32_t d, int32_t n, int32_t activation, double s,
                                const double *A, const double *zeta, const double *X, double *Phi,
                                void *stream);

/*
 * rpr_randnet_features for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the split-K partial sums in
 * a 16 MiB scratch array that the library keeps per device until the
 * process ends; nothing is allocated or freed.  The partial sums need
 * ceil(d / 512) (at most 64) x n x M doubles; larger calls return
 * RPR_ERR_INVALID_ARG before anything is enqueued.  Every call on one device
 * shares that device's scratch: calls that overlap on one GPU (two streams,
 * two threads) race and must be serialised by the caller.
 */
rpr_status rpr_randnet_features_noalloc(int32_t M, int32_t d, int32_t n, int32_t activation, double s,
                                        const double *A, const double *zeta, const double *X, double *Phi,
                                        void *stream);

/*
 * Split-bfloat16 features, the training features of RPR_MIXED plans: x/s and
 * A are each split into three bfloat16 pieces (each the bfloat16 rounding of
 * what the previous pieces leave), the six products of the pieces down to
 * 2^-16 relative are summed in single precision on the matrix cores, the
 * partial sums, zeta and sigma are taken in double.  The pre-activation is
 * within 2^-16 sum_j |A_mj x_j / s| of the exact one.
 *   A (M x d, doubles), zeta (M, doubles), X (n x d, floats), Phi (n x M,
 *   doubles): device pointers.  Allocates and frees its own workspace.
 */
rpr_status rpr_randnet_features_bf16(int32_t M, int32_t d, int32_t n, int32_t activation, double s,
                                     const double *A, const double *zeta, const float *X, double *Phi,
                                     void *stream);

/*
 * Ridge readout of eq. "ridgeless" at penalty lambda:
 *   W = (Phi^T Phi + lambda I_M)^{-1} Phi^T Y   (Cholesky, double precision).
 *   Phi (n x M), Y (n x d), W (M x d): device pointers, doubles.
 * Returns RPR_ERR_NOT_SPD (after synchronising the stream) if the matrix is
 * not numerically positive definite.  Allocates and frees its own workspace.
 */
rpr_status rpr_ridge_fit(int32_t M, int32_t d, int32_t n, const double *Phi, const double *Y,
                         double lambda, double *W, void *stream);

/*
 * Readout of eq. "HA": Yhat[r][j] = sum_m W[m][j] Phi[r][m].
 *   W (M x d), Phi (n x M), Yhat (n x d): device pointers, doubles.
 */
rpr_status rpr_randnet_readout(int32_t M, int32_t d, int32_t n, const double *W, const double *Phi,
                               double *Yhat, void *stream);

/*
 * Counter-based U(-1, 1) generator (SplitMix64 of Steele, Lea and Flood,
 * OOPSLA 2014, used as a hash of seed + (i + 1) * 0x9E3779B97F4A7C15):
 * out[k] = 2 ((r >> 11) 2^-53) - 1 with r the output for counter first + k.
 *   out: device pointer, n doubles.
 */
rpr_status rpr_uniform_pm1(uint64_t seed, uint64_t first, int64_t n, double *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* RPR_H */
