/*
 * randnet.c -- the random network, its ridge readout, nearest neighbours and
 * the counter-based generator.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/*
 * Hidden layer of eq. "HA" (Sec. 4): sigma(A U + zeta), applied to the
 * rescaled input U = x / s (Sec. 4 after Prop. 1 and the initialisation step of
 * Algorithm "Parareal (generic)": coordinates are brought into [-1, 1]).
 * sigma is ReLU in the paper, tanh is the alternative the workloads use.
 */
void orc_features(const orc_randnet *net, int32_t d, int32_t n, const double *X, double *Phi)
{
    for (int r = 0; r < n; ++r)
        for (int m = 0; m < net->M; ++m) {
            double z = 0.0;
            for (int j = 0; j < d; ++j)
                z += net->A[(size_t)m * d + j] * (X[(size_t)r * d + j] / net->scale);
            z += net->zeta[m];
            Phi[(size_t)r * net->M + m] = net->act == ORC_RELU ? (z > 0.0 ? z : 0.0) : tanh(z);
        }
}

/* Textbook Cholesky-Crout: S = L L^T, column by column. */
int32_t orc_cholesky(int32_t s, const double *S, double *L)
{
    memset(L, 0, sizeof(double) * (size_t)s * s);
    for (int j = 0; j < s; ++j) {
        double sum = S[(size_t)j * s + j];
        for (int p = 0; p < j; ++p) sum -= L[(size_t)j * s + p] * L[(size_t)j * s + p];
        if (!(sum > 0.0)) return -6;
        const double ljj = sqrt(sum);
        L[(size_t)j * s + j] = ljj;
        for (int i = j + 1; i < s; ++i) {
            double t = S[(size_t)i * s + j];
            for (int p = 0; p < j; ++p) t -= L[(size_t)i * s + p] * L[(size_t)j * s + p];
            L[(size_t)i * s + j] = t / ljj;
        }
    }
    return 0;
}

/* Solve L L^T X = Bm in place for the nrhs columns of Bm (s x nrhs, row-major). */
static void chol_solve(int s, const double *L, int nrhs, double *Bm)
{
    for (int c = 0; c < nrhs; ++c) {
        for (int i = 0; i < s; ++i) { /* forward: L z = b */
            double t = Bm[(size_t)i * nrhs + c];
            for (int p = 0; p < i; ++p) t -= L[(size_t)i * s + p] * Bm[(size_t)p * nrhs + c];
            Bm[(size_t)i * nrhs + c] = t / L[(size_t)i * s + i];
        }
        for (int i = s - 1; i >= 0; --i) { /* backward: L^T x = z */
            double t = Bm[(size_t)i * nrhs + c];
            for (int p = i + 1; p < s; ++p) t -= L[(size_t)p * s + i] * Bm[(size_t)p * nrhs + c];
            Bm[(size_t)i * nrhs + c] = t / L[(size_t)i * s + i];
        }
    }
}

/*
 * Eigendecomposition S = V diag(w) V^T of a symmetric s x s matrix by the
 * cyclic Jacobi method (Jacobi 1846; Golub and Van Loan, Matrix
 * Computations, Sec. 8.5): each off-diagonal entry in row order is zeroed by
 * a plane rotation, sweep after sweep, until the off-diagonal squares sum to
 * at most 2^-104 of all squares (at most 100 sweeps).  V row-major, its
 * columns the eigenvectors.
 */
void orc_sym_eig(int32_t s, const double *S, double *w, double *V)
{
    double *A = malloc(sizeof(double) * (size_t)s * s);
    memcpy(A, S, sizeof(double) * (size_t)s * s);
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) V[(size_t)i * s + j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, all = 0.0;
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < s; ++j) {
                const double a2 = A[(size_t)i * s + j] * A[(size_t)i * s + j];
                all += a2;
                if (i != j) off += a2;
            }
        if (off <= 0x1p-104 * all) break;
        for (int p = 0; p < s - 1; ++p)
            for (int q = p + 1; q < s; ++q) {
                const double apq = A[(size_t)p * s + q];
                if (apq == 0.0) continue;
                /* rotation [c sn; -sn c] in the (p, q) plane that zeroes apq */
                const double tau = (A[(size_t)q * s + q] - A[(size_t)p * s + p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
                const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
                for (int k = 0; k < s; ++k) { /* A <- A J */
                    const double akp = A[(size_t)k * s + p], akq = A[(size_t)k * s + q];
                    A[(size_t)k * s + p] = c * akp - sn * akq;
                    A[(size_t)k * s + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < s; ++k) { /* A <- J^T A */
                    const double apk = A[(size_t)p * s + k], aqk = A[(size_t)q * s + k];
                    A[(size_t)p * s + k] = c * apk - sn * aqk;
                    A[(size_t)q * s + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < s; ++k) { /* V <- V J */
                    const double vkp = V[(size_t)k * s + p], vkq = V[(size_t)k * s + q];
                    V[(size_t)k * s + p] = c * vkp - sn * vkq;
                    V[(size_t)k * s + q] = sn * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < s; ++i) w[i] = A[(size_t)i * s + i];
    free(A);
}

/*
 * Moore-Penrose pseudo-inverse of a symmetric positive semi-definite s x s
 * matrix S from its eigendecomposition: eigenvalues at or below
 * cut * max(eigenvalue) count as zero (their reciprocal is replaced by 0).
 * Returns the rank, the count of the others.
 */
static int32_t psd_pinv(int32_t s, const double *S, double cut, double *Sp)
{
    double *w = malloc(sizeof(double) * (size_t)s);
    double *V = malloc(sizeof(double) * (size_t)s * s);
    orc_sym_eig(s, S, w, V);
    double wmax = 0.0;
    for (int i = 0; i < s; ++i)
        if (w[i] > wmax) wmax = w[i];
    int32_t rank = 0;
    for (int i = 0; i < s; ++i) {
        if (w[i] > cut * wmax && wmax > 0.0) {
            w[i] = 1.0 / w[i];
            rank++;
        } else {
            w[i] = 0.0;
        }
    }
    for (int a = 0; a < s; ++a)
        for (int b = 0; b < s; ++b) {
            double t = 0.0;
            for (int i = 0; i < s; ++i) t += V[(size_t)a * s + i] * w[i] * V[(size_t)b * s + i];
            Sp[(size_t)a * s + b] = t;
        }
    free(w);
    free(V);
    return rank;
}

/*
 * Readout of eq. "ridgeless" at its limit lambda -> 0, the Moore-Penrose
 * solution W = X^+ Y (X = Phi, n x M; Y, n x d).  Alg. "RandNets training
 * procedure" writes it as (X^T X)^{-1} X^T Y when rank(X^T X) = M <= n and as
 * (X^T X)^+ X^T Y otherwise; both are X^+ Y, computed here as
 * (X^T X)^+ X^T Y when n >= M and as X^T (X X^T)^+ Y when n < M (the smaller
 * Gram), with eigenvalues of the Gram at or below max(n, M) 2^-52 times the
 * largest counted as zero.  *rank (if not NULL) receives the Gram's rank.
 */
int32_t orc_ridgeless_fit(int32_t M, int32_t d, int32_t n, const double *Phi, const double *Y, double *W,
                          int32_t *rank)
{
    const double cut = (double)(n > M ? n : M) * 0x1p-52;
    int32_t r;
    if (n >= M) {
        double *G = calloc((size_t)M * M, sizeof(double));
        double *Gp = malloc(sizeof(double) * (size_t)M * M);
        double *B = malloc(sizeof(double) * (size_t)M * d);
        if (!G || !Gp || !B) { free(G); free(Gp); free(B); return -4; }
        for (int a = 0; a < M; ++a)
            for (int b = 0; b < M; ++b) {
                double t = 0.0;
                for (int q = 0; q < n; ++q) t += Phi[(size_t)q * M + a] * Phi[(size_t)q * M + b];
                G[(size_t)a * M + b] = t;
            }
        for (int a = 0; a < M; ++a)
            for (int j = 0; j < d; ++j) {
                double t = 0.0;
                for (int q = 0; q < n; ++q) t += Phi[(size_t)q * M + a] * Y[(size_t)q * d + j];
                B[(size_t)a * d + j] = t;
            }
        r = psd_pinv(M, G, cut, Gp);
        for (int a = 0; a < M; ++a)
            for (int j = 0; j < d; ++j) {
                double t = 0.0;
                for (int b = 0; b < M; ++b) t += Gp[(size_t)a * M + b] * B[(size_t)b * d + j];
                W[(size_t)a * d + j] = t;
            }
        free(G);
        free(Gp);
        free(B);
    } else {
        double *K = calloc((size_t)n * n, sizeof(double));
        double *Kp = malloc(sizeof(double) * (size_t)n * n);
        double *Cm = malloc(sizeof(double) * (size_t)n * d);
        if (!K || !Kp || !Cm) { free(K); free(Kp); free(Cm); return -4; }
        for (int q = 0; q < n; ++q)
            for (int p = 0; p < n; ++p) {
                double t = 0.0;
                for (int a = 0; a < M; ++a) t += Phi[(size_t)q * M + a] * Phi[(size_t)p * M + a];
                K[(size_t)q * n + p] = t;
            }
        r = psd_pinv(n, K, cut, Kp);
        for (int q = 0; q < n; ++q)
            for (int j = 0; j < d; ++j) {
                double t = 0.0;
                for (int p = 0; p < n; ++p) t += Kp[(size_t)q * n + p] * Y[(size_t)p * d + j];
                Cm[(size_t)q * d + j] = t;
            }
        for (int a = 0; a < M; ++a)
            for (int j = 0; j < d; ++j) {
                double t = 0.0;
                for (int q = 0; q < n; ++q) t += Phi[(size_t)q * M + a] * Cm[(size_t)q * d + j];
                W[(size_t)a * d + j] = t;
            }
        free(K);
        free(Kp);
        free(Cm);
    }
    if (rank) *rank = r;
    return 0;
}

/*
 * The same limit from accumulated statistics G = X^T X (M x M) and
 * B = X^T Y (M x d) of n rows: W = G^+ B, the cut as in orc_ridgeless_fit.
 */
int32_t orc_ridgeless_stats(int32_t M, int32_t d, int32_t n, const double *G, const double *B, double *W,
                            int32_t *rank)
{
    double *Gp = malloc(sizeof(double) * (size_t)M * M);
    const int32_t r = psd_pinv(M, G, (double)(n > M ? n : M) * 0x1p-52, Gp);
    for (int a = 0; a < M; ++a)
        for (int j = 0; j < d; ++j) {
            double t = 0.0;
            for (int b = 0; b < M; ++b) t += Gp[(size_t)a * M + b] * B[(size_t)b * d + j];
            W[(size_t)a * d + j] = t;
        }
    free(Gp);
    if (rank) *rank = r;
    return 0;
}

/*
 * Ridge readout of eq. "ridgeless" at a fixed penalty:
 *   W = (X^T X + lambda I_M)^{-1} X^T Y, X = Phi (n x M), Y (n x d);
 * lambda = 0 is the limit itself (orc_ridgeless_fit).
 */
int32_t orc_ridge_fit(int32_t M, int32_t d, int32_t n, const double *Phi, const double *Y,
                      double lambda, double *W)
{
    if (lambda == 0.0) return orc_ridgeless_fit(M, d, n, Phi, Y, W, NULL);
    double *G = malloc(sizeof(double) * (size_t)M * M);
    double *L = malloc(sizeof(double) * (size_t)M * M);
    if (!G || !L) { free(G); free(L); return -4; }
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) {
            double t = 0.0;
            for (int r = 0; r < n; ++r) t += Phi[(size_t)r * M + a] * Phi[(size_t)r * M + b];
            G[(size_t)a * M + b] = t + (a == b ? lambda : 0.0);
        }
    for (int a = 0; a < M; ++a)
        for (int j = 0; j < d; ++j) {
            double t = 0.0;
            for (int r = 0; r < n; ++r) t += Phi[(size_t)r * M + a] * Y[(size_t)r * d + j];
            W[(size_t)a * d + j] = t;
        }
    int rc = orc_cholesky(M, G, L);
    if (rc == 0) chol_solve(M, L, d, W);
    free(G);
    free(L);
    return rc;
}

/* Same estimator in dual form: W = X^T (X X^T + lambda I_n)^{-1} Y
 * (lambda = 0: orc_ridgeless_fit). */
int32_t orc_ridge_fit_dual(int32_t M, int32_t d, int32_t n, const double *Phi, const double *Y,
                           double lambda, double *W)
{
    if (lambda == 0.0) return orc_ridgeless_fit(M, d, n, Phi, Y, W, NULL);
    double *K = malloc(sizeof(double) * (size_t)n * n);
    double *L = malloc(sizeof(double) * (size_t)n * n);
    double *C = malloc(sizeof(double) * (size_t)n * d);
    if (!K || !L || !C) { free(K); free(L); free(C); return -4; }
    for (int q = 0; q < n; ++q)
        for (int r = 0; r < n; ++r) {
            double t = 0.0;
            for (int a = 0; a < M; ++a) t += Phi[(size_t)q * M + a] * Phi[(size_t)r * M + a];
            K[(size_t)q * n + r] = t + (q == r ? lambda : 0.0);
        }
    memcpy(C, Y, sizeof(double) * (size_t)n * d);
    int rc = orc_cholesky(n, K, L);
    if (rc == 0) {
        chol_solve(n, L, d, C);
        for (int a = 0; a < M; ++a)
            for (int j = 0; j < d; ++j) {
                double t = 0.0;
                for (int r = 0; r < n; ++r) t += Phi[(size_t)r * M + a] * C[(size_t)r * d + j];
                W[(size_t)a * d + j] = t;
            }
    }
    free(K);
    free(L);
    free(C);
    return rc;
}

/* m nearest rows in Euclidean distance (App. B, eq. "fhat_mnn:U"); ties go to
 * the lower row index.  Plain repeated selection. */
void orc_nearest(int32_t d, int32_t n, const double *P, const double *q, int32_t m, int32_t *idx)
{
    double *dist = malloc(sizeof(double) * (size_t)n);
    char *taken = calloc((size_t)n, 1);
    for (int r = 0; r < n; ++r) {
        double t = 0.0;
        for (int j = 0; j < d; ++j) {
            const double e = P[(size_t)r * d + j] - q[j];
            t += e * e;
        }
        dist[r] = t;
    }
    for (int l = 0; l < m && l < n; ++l) {
        int best = -1;
        for (int r = 0; r < n; ++r) {
            if (taken[r]) continue;
            if (best < 0 || dist[r] < dist[best]) best = r;
        }
        taken[best] = 1;
        idx[l] = best;
    }
    free(dist);
    free(taken);
}

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), used as a counter hash. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* U(-1, 1): the top 53 bits as a fraction in [0, 1), mapped to [-1, 1). */
void orc_uniform_pm1(uint64_t seed, uint64_t first, int64_t n, double *out)
{
    for (int64_t k = 0; k < n; ++k) {
        const uint64_t r = orc_splitmix64(seed, first + (uint64_t)k);
        out[k] = 2.0 * ((double)(r >> 11) * 0x1.0p-53) - 1.0;
    }
}
