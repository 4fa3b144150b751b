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
 * Ridge readout of eq. "ridgeless" at a fixed penalty:
 *   W = (X^T X + lambda I_M)^{-1} X^T Y, X = Phi (n x M), Y (n x d).
 */
int32_t orc_ridge_fit(int32_t M, int32_t d, int32_t n, const double *Phi, const double *Y,
                      double lambda, double *W)
{
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

/* Same estimator in dual form: W = X^T (X X^T + lambda I_n)^{-1} Y. */
int32_t orc_ridge_fit_dual(int32_t M, int32_t d, int32_t n, const double *Phi, const double *Y,
                           double lambda, double *W)
{
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
