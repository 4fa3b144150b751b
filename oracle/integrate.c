/*
 * integrate.c -- fixed-step explicit Runge-Kutta propagators over one slice.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper's coarse and fine solvers G and F map the state at the start of a
 * slice to the state at its end (Sec. 2).  Both are explicit Runge-Kutta
 * methods with a fixed number of steps per slice (App. G setup tables):
 * forward Euler (RK1) and classical fourth-order Runge-Kutta (RK4).
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* u <- u + dt h(u) */
static int euler_steps(const orc_problem *pb, int64_t steps, double dt, double *u, double *k)
{
    const int d = orc_dim(pb);
    for (int64_t s = 0; s < steps; ++s) {
        if (orc_rhs(pb, u, k)) return -1;
        for (int j = 0; j < d; ++j) u[j] = u[j] + dt * k[j];
    }
    return 0;
}

/* Classical RK4: k1 = h(u), k2 = h(u + dt/2 k1), k3 = h(u + dt/2 k2),
 * k4 = h(u + dt k3), u <- u + dt/6 (k1 + 2 k2 + 2 k3 + k4). */
static int rk4_steps(const orc_problem *pb, int64_t steps, double dt, double *u, double *work)
{
    const int d = orc_dim(pb);
    double *k1 = work, *k2 = work + d, *k3 = work + 2 * d, *k4 = work + 3 * d, *y = work + 4 * d;
    for (int64_t s = 0; s < steps; ++s) {
        if (orc_rhs(pb, u, k1)) return -1;
        for (int j = 0; j < d; ++j) y[j] = u[j] + 0.5 * dt * k1[j];
        orc_rhs(pb, y, k2);
        for (int j = 0; j < d; ++j) y[j] = u[j] + 0.5 * dt * k2[j];
        orc_rhs(pb, y, k3);
        for (int j = 0; j < d; ++j) y[j] = u[j] + dt * k3[j];
        orc_rhs(pb, y, k4);
        for (int j = 0; j < d; ++j)
            u[j] = u[j] + (dt / 6.0) * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]);
    }
    return 0;
}

/*
 * Eighth-order explicit Runge-Kutta method of Cooper and Verner (SIAM J.
 * Numer. Anal. 9, 1972), 11 stages, with r = sqrt(21):
 *   c = (0, 1/2, 1/2, (7+r)/14, (7+r)/14, 1/2, (7-r)/14, (7-r)/14, 1/2,
 *        (7+r)/14, 1),
 *   b = (1/20, 0, 0, 0, 0, 0, 0, 49/180, 16/45, 49/180, 1/20),
 * and the coefficients a_ij below (the paper's fine solver of the Burgers
 * experiments is an RK8; it names no tableau).  Stage i: Y_i = u + dt
 * sum_j a_ij k_j, k_i = h(Y_i); step: u <- u + dt sum_i b_i k_i.
 */
static void cooper_verner(double *A, double *b, double *c)
{
    const double r = sqrt(21.0);
    for (int i = 0; i < 11 * 11; ++i) A[i] = 0.0;
#define a(i, j) A[(i) * 11 + (j)]
    a(1, 0) = 1.0 / 2.0;
    a(2, 0) = 1.0 / 4.0;
    a(2, 1) = 1.0 / 4.0;
    a(3, 0) = 1.0 / 7.0;
    a(3, 1) = (-7.0 - 3.0 * r) / 98.0;
    a(3, 2) = (21.0 + 5.0 * r) / 49.0;
    a(4, 0) = (11.0 + r) / 84.0;
    a(4, 2) = (18.0 + 4.0 * r) / 63.0;
    a(4, 3) = (21.0 - r) / 252.0;
    a(5, 0) = (5.0 + r) / 48.0;
    a(5, 2) = (9.0 + r) / 36.0;
    a(5, 3) = (-231.0 + 14.0 * r) / 360.0;
    a(5, 4) = (63.0 - 7.0 * r) / 80.0;
    a(6, 0) = (10.0 - r) / 42.0;
    a(6, 2) = (-432.0 + 92.0 * r) / 315.0;
    a(6, 3) = (633.0 - 145.0 * r) / 90.0;
    a(6, 4) = (-504.0 + 115.0 * r) / 70.0;
    a(6, 5) = (63.0 - 13.0 * r) / 35.0;
    a(7, 0) = 1.0 / 14.0;
    a(7, 4) = (14.0 - 3.0 * r) / 126.0;
    a(7, 5) = (13.0 - 3.0 * r) / 63.0;
    a(7, 6) = 1.0 / 9.0;
    a(8, 0) = 1.0 / 32.0;
    a(8, 4) = (91.0 - 21.0 * r) / 576.0;
    a(8, 5) = 11.0 / 72.0;
    a(8, 6) = (-385.0 - 75.0 * r) / 1152.0;
    a(8, 7) = (63.0 + 13.0 * r) / 128.0;
    a(9, 0) = 1.0 / 14.0;
    a(9, 4) = 1.0 / 9.0;
    a(9, 5) = (-733.0 - 147.0 * r) / 2205.0;
    a(9, 6) = (515.0 + 111.0 * r) / 504.0;
    a(9, 7) = (-51.0 - 11.0 * r) / 56.0;
    a(9, 8) = (132.0 + 28.0 * r) / 245.0;
    a(10, 4) = (-42.0 + 7.0 * r) / 18.0;
    a(10, 5) = (-18.0 + 28.0 * r) / 45.0;
    a(10, 6) = (-273.0 - 53.0 * r) / 72.0;
    a(10, 7) = (301.0 + 53.0 * r) / 72.0;
    a(10, 8) = (28.0 - 28.0 * r) / 45.0;
    a(10, 9) = (49.0 - 7.0 * r) / 18.0;
#undef a
    const double bb[11] = {1.0 / 20.0, 0, 0, 0, 0, 0, 0, 49.0 / 180.0, 16.0 / 45.0, 49.0 / 180.0, 1.0 / 20.0};
    for (int i = 0; i < 11; ++i) {
        b[i] = bb[i];
        double s = 0.0;
        for (int j = 0; j < i; ++j) s += A[i * 11 + j];
        c[i] = s;
    }
}

int32_t orc_rk_tableau(int32_t method, int32_t *s, double *A, double *b, double *c)
{
    for (int i = 0; i < 16 * 16; ++i) A[i] = 0.0;
    if (method == 1) {
        *s = 1;
        b[0] = 1.0;
        c[0] = 0.0;
        return 0;
    }
    if (method == 4) {
        /* classical RK4 (Kutta 1901), as rk4_steps applies it */
        *s = 4;
        A[1 * 4 + 0] = 0.5;
        A[2 * 4 + 1] = 0.5;
        A[3 * 4 + 2] = 1.0;
        const double bb[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0}, cc[4] = {0.0, 0.5, 0.5, 1.0};
        for (int i = 0; i < 4; ++i) { b[i] = bb[i]; c[i] = cc[i]; }
        return 0;
    }
    if (method == 8) {
        *s = 11;
        cooper_verner(A, b, c);
        return 0;
    }
    return -1;
}

/* Any explicit tableau: stage i evaluates h at Y_i = u + dt sum_{j<i} a_ij k_j,
 * the step adds dt sum_i b_i k_i. */
static int erk_steps(const orc_problem *pb, int s, const double *A, const double *b, int64_t steps, double dt,
                     double *u, double *work)
{
    const int d = orc_dim(pb);
    double *y = work, *k = work + d;  /* k: s x d */
    for (int64_t st = 0; st < steps; ++st) {
        for (int i = 0; i < s; ++i) {
            for (int j = 0; j < d; ++j) {
                double acc = 0.0;
                for (int l = 0; l < i; ++l) acc += A[i * s + l] * k[(size_t)l * d + j];
                y[j] = u[j] + dt * acc;
            }
            if (orc_rhs(pb, y, k + (size_t)i * d)) return -1;
        }
        for (int j = 0; j < d; ++j) {
            double acc = 0.0;
            for (int i = 0; i < s; ++i) acc += b[i] * k[(size_t)i * d + j];
            u[j] = u[j] + dt * acc;
        }
    }
    return 0;
}

int32_t orc_propagate(const orc_problem *pb, int32_t method, int64_t steps, double dt,
                      const double *in, double *out)
{
    const int d = orc_dim(pb);
    if (d <= 0 || steps < 0) return -1;
    double *u = malloc(sizeof(double) * d);
    double *work = malloc(sizeof(double) * 12 * d);
    if (!u || !work) { free(u); free(work); return -4; }
    memcpy(u, in, sizeof(double) * d);
    int rc;
    if (method == 1) rc = euler_steps(pb, steps, dt, u, work);
    else if (method == 4) rc = rk4_steps(pb, steps, dt, u, work);
    else if (method == 8) {
        double A[11 * 11], b[11], c[11];
        cooper_verner(A, b, c);
        rc = erk_steps(pb, 11, A, b, steps, dt, u, work);
    } else rc = -1;
    if (rc == 0) memcpy(out, u, sizeof(double) * d);
    free(u);
    free(work);
    return rc;
}

typedef struct {
    const orc_problem *pb;
    int32_t method;
    int64_t steps;
    double dt;
    int32_t first, last, d;
    const double *in;
    double *out;
    int32_t rc;
} prop_job;

static void *prop_worker(void *arg)
{
    prop_job *j = (prop_job *)arg;
    j->rc = 0;
    for (int r = j->first; r < j->last; ++r) {
        int rc = orc_propagate(j->pb, j->method, j->steps, j->dt, j->in + (size_t)r * j->d,
                               j->out + (size_t)r * j->d);
        if (rc) j->rc = rc;
    }
    return NULL;
}

int32_t orc_propagate_many(const orc_problem *pb, int32_t method, int64_t steps, double dt,
                           int32_t n, const double *in, double *out, int32_t nthreads)
{
    const int d = orc_dim(pb);
    if (n <= 0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > n) nthreads = n;
    prop_job *jobs = calloc((size_t)nthreads, sizeof(prop_job));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return -4; }
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (prop_job){pb, method, steps, dt, (int32_t)((int64_t)n * t / nthreads),
                             (int32_t)((int64_t)n * (t + 1) / nthreads), d, in, out, 0};
    }
    if (nthreads == 1) {
        prop_worker(&jobs[0]);
    } else {
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, prop_worker, &jobs[t]);
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
    int rc = 0;
    for (int t = 0; t < nthreads; ++t) if (jobs[t].rc) rc = jobs[t].rc;
    free(jobs);
    free(th);
    return rc;
}

int32_t orc_serial_fine(const orc_problem *pb, int32_t method, int64_t steps, double dt,
                        int32_t N, const double *u0, double *U)
{
    const int d = orc_dim(pb);
    memcpy(U, u0, sizeof(double) * d);
    for (int i = 1; i <= N; ++i) {
        int rc = orc_propagate(pb, method, steps, dt, U + (size_t)(i - 1) * d, U + (size_t)i * d);
        if (rc) return rc;
    }
    return 0;
}
