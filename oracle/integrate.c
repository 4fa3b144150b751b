/*
 * integrate.c -- fixed-step explicit Runge-Kutta propagators over one slice.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper's coarse and fine solvers G and F map the state at the start of a
 * slice to the state at its end (Sec. 2).  Both are explicit Runge-Kutta
 * methods with a fixed number of steps per slice (App. G setup tables):
 * forward Euler (RK1) and classical fourth-order Runge-Kutta (RK4).
 */
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

int32_t orc_propagate(const orc_problem *pb, int32_t method, int64_t steps, double dt,
                      const double *in, double *out)
{
    const int d = orc_dim(pb);
    if (d <= 0 || steps < 0) return -1;
    double *u = malloc(sizeof(double) * d);
    double *work = malloc(sizeof(double) * 5 * d);
    if (!u || !work) { free(u); free(work); return -4; }
    memcpy(u, in, sizeof(double) * d);
    int rc;
    if (method == 1) rc = euler_steps(pb, steps, dt, u, work);
    else if (method == 4) rc = rk4_steps(pb, steps, dt, u, work);
    else rc = -1;
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
