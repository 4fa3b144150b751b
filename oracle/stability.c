/*
 * stability.c -- bound on the step size of the explicit propagators.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Sec. 6 of the paper warns that a coarse solver unsuited to the problem keeps
 * Parareal from converging.  For an explicit Runge-Kutta method the first
 * thing that goes wrong is linear stability: every eigenvalue z of dt times
 * the Jacobian of h must lie in the method's stability region.  This file
 * bounds the eigenvalues of the Jacobian at a state u (no assembly: grid
 * spacings, parameters and the state's extremes) by a real extent rr and an
 * imaginary extent ri, then compares dt with the largest stable step:
 *   forward Euler: |1 + z| <= 1 for z = -a(1 - cos t) + i b sin t, a = rr / 2,
 *     b = ri, holds for all t iff dt <= 2 / rr and dt <= rr / (2 ri^2);
 *   classical RK4: the region reaches -2.785 on the real axis and 2.83 on the
 *     imaginary one; 2.78 / (rr + ri) is used;
 *   eighth-order RK (Cooper-Verner): -3.71 and 3.00; 2.9 / (rr + ri).
 */
#include <math.h>
#include "oracle.h"

static double dmax(double a, double b) { return a > b ? a : b; }

double orc_stability(const orc_problem *pb, int32_t method, double dt, const double *u)
{
    const int d = orc_dim(pb);
    const int nc = pb->nx * pb->ny * (pb->kind == ORC_BRUSS3D ? pb->nz : 1);
    const double dx = (pb->x1 - pb->x0) / pb->nx;
    const double dy = pb->kind == ORC_BURGERS1D ? 1.0 : (pb->y1 - pb->y0) / pb->ny;
    const double dz = pb->kind == ORC_BRUSS3D ? (pb->x1 - pb->x0) / pb->nz : 0.0;
    const double lapz = pb->kind == ORC_BRUSS3D ? 4.0 / (dz * dz) : 0.0;  /* seven-point Laplacian in 3D */
    double umax = 0.0;
    for (int j = 0; j < d; ++j) umax = dmax(umax, fabs(u[j]));
    double rr = 0.0, ri = 0.0;
    if (pb->kind == ORC_BURGERS1D) {
        /* nu D2 - u D1 (central): real part in [-4 nu / dx^2, 0], imaginary
         * part at most max|u| / dx */
        rr = 4.0 * pb->p[0] / (dx * dx);
        ri = umax / dx;
    } else if (pb->kind == ORC_DIFFREACT2D || pb->kind == ORC_BRUSS2D || pb->kind == ORC_BRUSS3D) {
        /* 5-point (7-point in 3D) Laplacian: eigenvalues in
         * [-(4/dx^2 + 4/dy^2 (+ 4/dz^2)), 0] times the
         * larger diffusion coefficient; the reaction Jacobian's eigenvalues are
         * bounded by its row-sum norm:
         *   FitzHugh-Nagumo  [[1 - 3u^2, -1], [1, -1]]       -> 2 + 3 max u^2
         *   Brusselator [[-(B+1) + 2uv, u^2], [B - 2uv, -u^2]] -> B + 1 + 3 max u^2 */
        const double D = pb->kind == ORC_DIFFREACT2D ? dmax(pb->p[0], pb->p[1]) : dmax(pb->p[2], pb->p[3]);
        rr = D * (4.0 / (dx * dx) + 4.0 / (dy * dy) + lapz);
        rr += pb->kind == ORC_DIFFREACT2D ? 2.0 + 3.0 * umax * umax : pb->p[1] + 1.0 + 3.0 * umax * umax;
    } else if (pb->kind == ORC_SWE2D) {
        /* first-order Rusanov: per direction the linearised scheme has the
         * symbol -(a/dx)(1 - e^{i t}) with a the largest wave speed, inside
         * the disc of radius a/dx about -a/dx */
        double a = 0.0;
        for (int c = 0; c < nc; ++c) {
            const double h = u[c];
            const double vel = dmax(fabs(u[nc + c]), fabs(u[2 * nc + c]));
            a = dmax(a, h > 0.0 ? vel / h + sqrt(pb->p[0] * h) : INFINITY);
        }
        rr = 2.0 * a * (1.0 / dx + 1.0 / dy);
    }
    if (dt < 0) dt = -dt;
    if (method == 4) return rr + ri > 0.0 ? dt * (rr + ri) / 2.78 : 0.0;
    /* the Cooper-Verner RK8 region reaches -3.71 on the real axis and 3.00 i
     * on the imaginary one (its stability function from the tableau) */
    if (method == 8) return rr + ri > 0.0 ? dt * (rr + ri) / 2.9 : 0.0;
    double r = rr > 0.0 ? dt * rr / 2.0 : 0.0;
    if (ri > 0.0) {
        if (!(rr > 0.0)) return INFINITY;
        r = dmax(r, dt * 2.0 * ri * ri / rr);
    }
    return r;
}
