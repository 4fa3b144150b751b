/*
 * oracle.h -- plain serial FP64 CPU oracle for RandNet-Parareal.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the GPU library
 * against an independent, slow, obviously correct implementation written from
 * the paper (arXiv 2411.06225).  The product path never links, loads or calls
 * it, and it shares no code, header, table or helper with the GPU library.
 *
 * Everything is double precision, single threaded unless a thread count is
 * passed explicitly, compiled without FMA contraction or fast-math, so every
 * floating-point operation is the IEEE operation written in the source.
 *
 * What follows the paper (section / equation / algorithm labels of the paper):
 *   - the IVP du/dt = h(u), u(t0) = u0 on [t0, tN] split in N equal slices
 *     (Sec. 2, eq. "ode");
 *   - spatial right-hand sides h: viscous Burgers (Sec. 5.1, eq. "burg"),
 *     FitzHugh-Nagumo diffusion-reaction (Sec. 5.2), Brusselator (App. E),
 *     shallow water (Sec. 5.3; Rusanov finite volumes, flat bottom);
 *   - propagators: forward Euler (RK1) and classical RK4 with a fixed number
 *     of steps per slice (App. G setup tables);
 *   - the random network H(U) = W^T sigma(A U + zeta) (Sec. 4, eq. "HA"), its
 *     ridge readout (Sec. 4, eq. "ridgeless") fitted on the pairs of eq. "Dk";
 *   - the Parareal iteration with the generic predictor-corrector rule
 *     (Sec. 2, eqs. "update_rule_generic", "fpara", "stop_crit";
 *     Algorithms "Parareal (generic)" and "RandNets training procedure").
 */
#ifndef RPR_ORACLE_H
#define RPR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- problem definition ------------------------------------------------ */
enum { ORC_BURGERS1D = 0, ORC_DIFFREACT2D = 1, ORC_BRUSS2D = 2, ORC_SWE2D = 3, ORC_BRUSS3D = 4 };

typedef struct {
    int32_t kind;          /* ORC_* */
    int32_t nx, ny;        /* grid points / cells per direction (ny = 1 in 1D) */
    int32_t nz;            /* cells along z (3D Brusselator; ignored otherwise), z in (x0, x1) */
    double x0, x1, y0, y1; /* domain */
    double p[6];           /* Burgers: nu | DR: Du, Dv, c | Bruss (2D, 3D): A, B, Du, Dv | SWE: g */
} orc_problem;

int32_t orc_nspecies(const orc_problem *pb);
int32_t orc_dim(const orc_problem *pb);

/* h(u) written into out (both length orc_dim). Returns 0, or -1 on a bad problem. */
int32_t orc_rhs(const orc_problem *pb, const double *u, double *out);

/* Butcher tableau of an explicit Runge-Kutta method (method 1, 4 or 8):
 * *s stages, A (s x s, row-major, strictly lower), b (s), c (s); arrays of
 * at least 16 x 16, 16, 16.  Returns 0, or -1 for an unknown method. */
int32_t orc_rk_tableau(int32_t method, int32_t *s, double *A, double *b, double *c);

/* One slice of a fixed-step explicit Runge-Kutta method.
 * method: 1 = forward Euler (RK1), 4 = classical RK4, 8 = the eighth-order
 * method of Cooper and Verner (11 stages).
 * steps: number of steps; dt: step length.  in and out may alias. */
int32_t orc_propagate(const orc_problem *pb, int32_t method, int64_t steps, double dt,
                      const double *in, double *out);

/* Propagate n independent states (row-major n x d), optionally on nthreads
 * POSIX threads (the paper runs one fine solve per core). */
int32_t orc_propagate_many(const orc_problem *pb, int32_t method, int64_t steps, double dt,
                           int32_t n, const double *in, double *out, int32_t nthreads);

/* Serial fine solution: U[0] = u0, U[i] = F(U[i-1]), i = 1..N.  U is (N+1) x d. */
int32_t orc_serial_fine(const orc_problem *pb, int32_t method, int64_t steps, double dt,
                        int32_t N, const double *u0, double *U);

/* dt over the largest stable step of `method` (1 = forward Euler, 4 = RK4) for
 * h linearised at state u: > 1 flags the step as outside the stability
 * region (Sec. 6: an unsuitable G stalls the iteration). */
double orc_stability(const orc_problem *pb, int32_t method, double dt, const double *u);

/* ---- random network ----------------------------------------------------- */
enum { ORC_TANH = 0, ORC_RELU = 1 };

typedef struct {
    int32_t M;             /* hidden neurons */
    int32_t act;           /* ORC_TANH / ORC_RELU */
    double lambda;         /* ridge penalty; 0 = the ridgeless limit (pseudo-inverse) */
    double scale;          /* input scale s: the network sees x / s */
    const double *A;       /* M x d, row-major */
    const double *zeta;    /* M */
} orc_randnet;

/* Phi (n x M) = sigma(A (X_r / s) + zeta) for each row X_r of X (n x d). */
void orc_features(const orc_randnet *net, int32_t d, int32_t n, const double *X, double *Phi);

/* Ridge readout from explicit rows: W (M x d) = (Phi^T Phi + lambda I)^{-1} Phi^T Y,
 * by Cholesky.  Returns 0, or -6 if the matrix is not numerically positive definite;
 * lambda = 0 gives the ridgeless limit (orc_ridgeless_fit). */
int32_t orc_ridge_fit(int32_t M, int32_t d, int32_t n, const double *Phi, const double *Y,
                      double lambda, double *W);

/* Dual (kernel) form of the same estimator: W = Phi^T (Phi Phi^T + lambda I_n)^{-1} Y. */
int32_t orc_ridge_fit_dual(int32_t M, int32_t d, int32_t n, const double *Phi, const double *Y,
                           double lambda, double *W);

/* The limit lambda -> 0 of eq. "ridgeless": W = Phi^+ Y (Moore-Penrose), through
 * the pseudo-inverse of the smaller Gram; *rank (may be NULL) receives its rank.
 * orc_ridge_fit and orc_ridge_fit_dual take this branch for lambda = 0. */
int32_t orc_ridgeless_fit(int32_t M, int32_t d, int32_t n, const double *Phi, const double *Y, double *W,
                          int32_t *rank);

/* The same from accumulated statistics G = Phi^T Phi (M x M), B = Phi^T Y (M x d)
 * of n rows: W = G^+ B. */
int32_t orc_ridgeless_stats(int32_t M, int32_t d, int32_t n, const double *G, const double *B, double *W,
                            int32_t *rank);

/* Eigenvalues w (s) and eigenvectors (columns of V, s x s row-major) of a symmetric
 * s x s matrix S, cyclic Jacobi. */
void orc_sym_eig(int32_t s, const double *S, double *w, double *V);

/* Cholesky factor of an s x s symmetric matrix (lower triangle read), returned in
 * the lower triangle of Lout (upper part zeroed).  Returns 0 or -6. */
int32_t orc_cholesky(int32_t s, const double *S, double *Lout);

/* Indices of the m nearest rows of P (n x d) to q in Euclidean distance,
 * ascending distance, ties to the lower row index. */
void orc_nearest(int32_t d, int32_t n, const double *P, const double *q, int32_t m, int32_t *idx);

/* ---- counter-based generator ------------------------------------------- */
/* SplitMix64 output for counter i under seed: mix(seed + (i + 1) * golden gamma). */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i);
/* Fill out[0..n) with U(-1, 1) doubles from counters first..first+n-1. */
void orc_uniform_pm1(uint64_t seed, uint64_t first, int64_t n, double *out);

/* ---- Parareal driver ---------------------------------------------------- */
enum { ORC_CORR_RANDNET = 0, ORC_CORR_PARAREAL = 1, ORC_CORR_RANDNET_NN = 2 };

typedef struct {
    int32_t K;              /* iterations run */
    int32_t L_final;        /* last final slot */
    int32_t converged;      /* 1 if L reached N */
    int32_t rows_used;      /* finite training rows accumulated */
    int32_t nonfinite_rows; /* rows dropped for non-finite values */
    int32_t chol_fail;      /* ridge solves that failed */
} orc_info;

typedef struct {
    int32_t N;              /* slices */
    int32_t F_method, G_method;
    int32_t corr;           /* ORC_CORR_* */
    int64_t F_steps, G_steps;
    double t0, tN;
    double eps;             /* tolerance of eq. "stop_crit" */
    int32_t k_max;          /* iteration cap (<= N) */
    int32_t m_nn;           /* nearest neighbours for ORC_CORR_RANDNET_NN */
    int32_t nthreads;       /* threads for the fine solves (1 = serial) */
    int32_t pad;
} orc_parareal_cfg;

/* Default input scale: smallest power of two >= max(1, ||u0||_inf). */
double orc_input_scale(int32_t d, const double *u0);

/* Runs the iteration (a non-positive net->scale selects orc_input_scale).
 * U_out is (N+1) x d.  L_hist[k] (k = 0..K) gets L after iteration k and chg_hist[k] (k = 1..K) the largest slot change
 * max_{i>L_{k-1}+1} ||U_i^k - U_i^{k-1}||_inf (NaN-aware).  Either may be NULL.
 * U_iter, if not NULL, receives U^k for k = 0..k_max ((k_max+1) x (N+1) x d). */
int32_t orc_parareal(const orc_problem *pb, const orc_parareal_cfg *cfg, const orc_randnet *net,
                     const double *u0, double *U_out, int32_t *L_hist, double *chg_hist,
                     double *U_iter, orc_info *info);

#ifdef __cplusplus
}
#endif
#endif
