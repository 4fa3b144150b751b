/*
 * parareal.c -- the Parareal iteration with the RandNet (or classical)
 * correction.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Follows Algorithm "Parareal (generic)" with these readings of the paper:
 *   - slots U_0..U_N; U_0 = u0; L counts the slots that are final (U_0..U_L);
 *   - iteration k runs F only on the slots that are not final, i = L+1..N
 *     (converged slots are not iterated, Sec. 2 after eq. "stop_crit");
 *   - the leftmost unconverged slot takes the fine value F(U_L), which is
 *     exact because U_L is final (Sec. 2, the remark on the "leftmost" fine
 *     evaluation); this is what bounds the iteration count by N;
 *   - the other slots follow eq. "update_rule_generic",
 *     U_i^k = G(U_{i-1}^k) + fhat(U_{i-1}^k), sequentially;
 *   - fhat is eq. "fpara" (classical Parareal), or the random network of
 *     eq. "HA" whose readout solves eq. "ridgeless" at penalty lambda on every
 *     pair of eq. "Dk" collected so far (global mode), or on the m nearest
 *     pairs of the query (eq. "randnet", Algorithm "RandNets training
 *     procedure"; dual form); lambda = 0 takes the limit itself, the
 *     pseudo-inverse solution of that algorithm;
 *   - the pairs are (U_{i-1}^{k-1}, F(U_{i-1}^{k-1}) - G(U_{i-1}^{k-1})) for the
 *     slots run at iteration k; pairs with a non-finite entry are dropped;
 *   - convergence (eq. "stop_crit"): after the update L advances over the exact
 *     slot, then over every following slot whose infinity-norm change is
 *     below eps, stopping at the first that is not; NaN counts as not
 *     converged.  The run stops when L = N.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

static int all_finite(const double *v, int n)
{
    for (int j = 0; j < n; ++j)
        if (!isfinite(v[j])) return 0;
    return 1;
}

/* infinity norm of a - b with NaN mapped to +inf */
static double change_norm(const double *a, const double *b, int n)
{
    double m = 0.0;
    for (int j = 0; j < n; ++j) {
        double e = fabs(a[j] - b[j]);
        if (isnan(e)) e = INFINITY;
        if (e > m) m = e;
    }
    return m;
}

/* y = W^T phi, W is M x d */
static void readout(int M, int d, const double *W, const double *phi, double *y)
{
    for (int j = 0; j < d; ++j) {
        double t = 0.0;
        for (int m = 0; m < M; ++m) t += W[(size_t)m * d + j] * phi[m];
        y[j] = t;
    }
}

double orc_input_scale(int32_t d, const double *u0)
{
    double m = 1.0;
    for (int j = 0; j < d; ++j)
        if (fabs(u0[j]) > m) m = fabs(u0[j]);
    double s = 1.0;
    while (s < m) s *= 2.0;
    return s;
}

int32_t orc_parareal(const orc_problem *pb, const orc_parareal_cfg *cfg, const orc_randnet *net,
                     const double *u0, double *U_out, int32_t *L_hist, double *chg_hist,
                     double *U_iter, orc_info *info)
{
    const int d = orc_dim(pb);
    const int N = cfg->N;
    const int M = net ? net->M : 0;
    const int use_net = cfg->corr == ORC_CORR_RANDNET || cfg->corr == ORC_CORR_RANDNET_NN;
    if (d <= 0 || N < 1 || cfg->k_max < 0 || (use_net && (!net || M < 1))) return -1;
    const double T = (cfg->tN - cfg->t0) / N;
    const double dtF = T / (double)cfg->F_steps;
    const double dtG = T / (double)cfg->G_steps;
    const size_t sd = (size_t)d;

    double *U = calloc((size_t)(N + 1) * sd, sizeof(double));
    double *Uprev = calloc((size_t)(N + 1) * sd, sizeof(double));
    double *Fv = calloc((size_t)(N + 1) * sd, sizeof(double));
    double *Gc = calloc((size_t)(N + 1) * sd, sizeof(double));
    double *g = calloc(sd, sizeof(double));
    double *corr = calloc(sd, sizeof(double));
    double *y = calloc(sd, sizeof(double));
    double *phi = calloc((size_t)(M > 0 ? M : 1), sizeof(double));
    double *Gacc = calloc((size_t)(M > 0 ? M : 1) * (M > 0 ? M : 1), sizeof(double));
    double *Gl = calloc((size_t)(M > 0 ? M : 1) * (M > 0 ? M : 1), sizeof(double));
    double *Lf = calloc((size_t)(M > 0 ? M : 1) * (M > 0 ? M : 1), sizeof(double));
    double *Bacc = calloc((size_t)(M > 0 ? M : 1) * sd, sizeof(double));
    double *W = calloc((size_t)(M > 0 ? M : 1) * sd, sizeof(double));
    /* stored pairs (nn mode): at most N per iteration */
    const int max_rows = N * (cfg->k_max > 0 ? cfg->k_max : 1);
    const int nn_mode = cfg->corr == ORC_CORR_RANDNET_NN;
    double *Xs = nn_mode ? calloc((size_t)max_rows * sd, sizeof(double)) : NULL;
    double *Ys = nn_mode ? calloc((size_t)max_rows * sd, sizeof(double)) : NULL;
    int32_t *nn_idx = nn_mode ? calloc((size_t)(cfg->m_nn > 0 ? cfg->m_nn : 1), sizeof(int32_t)) : NULL;
    double *Xm = nn_mode ? calloc((size_t)(cfg->m_nn > 0 ? cfg->m_nn : 1) * sd, sizeof(double)) : NULL;
    double *Ym = nn_mode ? calloc((size_t)(cfg->m_nn > 0 ? cfg->m_nn : 1) * sd, sizeof(double)) : NULL;
    double *Pm = nn_mode ? calloc((size_t)(cfg->m_nn > 0 ? cfg->m_nn : 1) * (M > 0 ? M : 1), sizeof(double)) : NULL;
    if (!U || !Uprev || !Fv || !Gc || !g || !corr || !y || !phi || !Gacc || !Gl || !Lf || !Bacc ||
        !W || (nn_mode && (!Xs || !Ys || !nn_idx || !Xm || !Ym || !Pm)))
        return -4;

    /* input scale s (Algorithm "Parareal (generic)", initialisation): when not
     * given, the smallest power of two s >= max(1, ||u0||_inf), so x / s lies in
     * [-1, 1] at t0 and the division is exact */
    orc_randnet net_local;
    if (use_net) {
        net_local = *net;
        if (!(net_local.scale > 0.0)) net_local.scale = orc_input_scale(d, u0);
        net = &net_local;
    }
    orc_info inf = {0, 0, 0, 0, 0, 0};
    int rc = 0;
    int n_rows = 0;

    /* k = 0: coarse sweep U_i^0 = G(U_{i-1}^0); the G values are kept because
     * they are the G part of the next training pairs. */
    memcpy(U, u0, sizeof(double) * sd);
    for (int i = 1; i <= N; ++i) {
        orc_propagate(pb, cfg->G_method, cfg->G_steps, dtG, U + (i - 1) * sd, U + i * sd);
        memcpy(Gc + i * sd, U + i * sd, sizeof(double) * sd);
    }
    int L = 0;
    if (L_hist) L_hist[0] = 0;
    if (chg_hist) chg_hist[0] = 0.0;
    if (U_iter) memcpy(U_iter, U, sizeof(double) * (N + 1) * sd);

    int k;
    for (k = 1; k <= cfg->k_max; ++k) {
        /* fine solves of the slots that are not final */
        rc = orc_propagate_many(pb, cfg->F_method, cfg->F_steps, dtF, N - L, U + (size_t)L * sd,
                                Fv + (size_t)(L + 1) * sd, cfg->nthreads);
        if (rc) break;

        /* new pairs of eq. "Dk" and the global ridge statistics */
        if (use_net) {
            for (int i = L + 1; i <= N; ++i) {
                const double *x = U + (size_t)(i - 1) * sd;
                for (int j = 0; j < d; ++j) y[j] = Fv[i * sd + j] - Gc[i * sd + j];
                if (!all_finite(x, d) || !all_finite(y, d)) { inf.nonfinite_rows++; continue; }
                if (nn_mode) {
                    memcpy(Xs + (size_t)n_rows * sd, x, sizeof(double) * sd);
                    memcpy(Ys + (size_t)n_rows * sd, y, sizeof(double) * sd);
                } else {
                    orc_features(net, d, 1, x, phi);
                    for (int a = 0; a < M; ++a)
                        for (int b = 0; b < M; ++b) Gacc[a * M + b] += phi[a] * phi[b];
                    for (int a = 0; a < M; ++a)
                        for (int j = 0; j < d; ++j) Bacc[a * sd + j] += phi[a] * y[j];
                }
                n_rows++;
            }
            inf.rows_used = n_rows;
            if (!nn_mode && net->lambda == 0.0) {
                /* eq. "ridgeless" at its limit lambda -> 0 on every pair so far */
                orc_ridgeless_stats(M, d, n_rows, Gacc, Bacc, W, NULL);
            } else if (!nn_mode) {
                /* eq. "ridgeless" at penalty lambda on every pair so far */
                memcpy(Gl, Gacc, sizeof(double) * M * M);
                for (int a = 0; a < M; ++a) Gl[a * M + a] += net->lambda;
                memcpy(W, Bacc, sizeof(double) * M * sd);
                if (orc_cholesky(M, Gl, Lf) == 0) {
                    for (int c = 0; c < d; ++c) {
                        for (int i = 0; i < M; ++i) {
                            double t = W[i * sd + c];
                            for (int p = 0; p < i; ++p) t -= Lf[i * M + p] * W[p * sd + c];
                            W[i * sd + c] = t / Lf[i * M + i];
                        }
                        for (int i = M - 1; i >= 0; --i) {
                            double t = W[i * sd + c];
                            for (int p = i + 1; p < M; ++p) t -= Lf[p * M + i] * W[p * sd + c];
                            W[i * sd + c] = t / Lf[i * M + i];
                        }
                    }
                } else {
                    inf.chol_fail++;
                    memset(W, 0, sizeof(double) * M * sd);
                }
            }
        }

        /* predictor-corrector sweep */
        memcpy(Uprev, U, sizeof(double) * (N + 1) * sd);
        memcpy(U + (size_t)(L + 1) * sd, Fv + (size_t)(L + 1) * sd, sizeof(double) * sd);
        for (int i = L + 2; i <= N; ++i) {
            const double *x = U + (size_t)(i - 1) * sd;
            orc_propagate(pb, cfg->G_method, cfg->G_steps, dtG, x, g);
            if (cfg->corr == ORC_CORR_PARAREAL) {
                /* eq. "fpara": (F - G)(U_{i-1}^{k-1}) */
                for (int j = 0; j < d; ++j) corr[j] = Fv[i * sd + j] - Gc[i * sd + j];
            } else if (cfg->corr == ORC_CORR_RANDNET) {
                orc_features(net, d, 1, x, phi);
                readout(M, d, W, phi, corr);
            } else {
                /* eq. "randnet": refit on the m nearest stored pairs of x */
                int m = cfg->m_nn < n_rows ? cfg->m_nn : n_rows;
                if (m <= 0) {
                    memset(corr, 0, sizeof(double) * sd);
                } else {
                    orc_nearest(d, n_rows, Xs, x, m, nn_idx);
                    for (int l = 0; l < m; ++l) {
                        memcpy(Xm + (size_t)l * sd, Xs + (size_t)nn_idx[l] * sd, sizeof(double) * sd);
                        memcpy(Ym + (size_t)l * sd, Ys + (size_t)nn_idx[l] * sd, sizeof(double) * sd);
                    }
                    orc_features(net, d, m, Xm, Pm);
                    if (orc_ridge_fit_dual(M, d, m, Pm, Ym, net->lambda, W) == 0) {
                        orc_features(net, d, 1, x, phi);
                        readout(M, d, W, phi, corr);
                    } else {
                        inf.chol_fail++;
                        memset(corr, 0, sizeof(double) * sd);
                    }
                }
            }
            for (int j = 0; j < d; ++j) U[i * sd + j] = g[j] + corr[j];
            memcpy(Gc + i * sd, g, sizeof(double) * sd);
        }

        /* convergence: exact slot, then eq. "stop_crit" slot by slot */
        const int L_old = L;
        double chg = 0.0;
        for (int i = L_old + 2; i <= N; ++i) {
            const double e = change_norm(U + i * sd, Uprev + i * sd, d);
            if (e > chg) chg = e;
        }
        L = L_old + 1;
        for (int i = L_old + 2; i <= N; ++i) {
            const double e = change_norm(U + i * sd, Uprev + i * sd, d);
            if (e < cfg->eps) L = i;
            else break;
        }
        if (L_hist) L_hist[k] = L;
        if (chg_hist) chg_hist[k] = chg;
        if (U_iter) memcpy(U_iter + (size_t)k * (N + 1) * sd, U, sizeof(double) * (N + 1) * sd);
        inf.K = k;
        if (L >= N) { inf.converged = 1; break; }
    }
    inf.L_final = L;
    memcpy(U_out, U, sizeof(double) * (N + 1) * sd);
    if (info) *info = inf;

    free(U); free(Uprev); free(Fv); free(Gc); free(g); free(corr); free(y); free(phi);
    free(Gacc); free(Gl); free(Lf); free(Bacc); free(W);
    free(Xs); free(Ys); free(nn_idx); free(Xm); free(Ym); free(Pm);
    return rc;
}
