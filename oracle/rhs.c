/*
 * rhs.c -- spatial right-hand sides h(u) of the semi-discretised PDEs.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain loops, one output point
 * at a time, no blocking or reuse.
 */
#include <math.h>
#include <stddef.h>
#include "oracle.h"

int32_t orc_nspecies(const orc_problem *pb)
{
    switch (pb->kind) {
    case ORC_BURGERS1D: return 1;
    case ORC_DIFFREACT2D: return 2;
    case ORC_BRUSS2D: return 2;
    case ORC_SWE2D: return 3;
    case ORC_BRUSS3D: return 2;
    default: return 0;
    }
}

/* cells along z: pb->nz for the 3D system, 1 otherwise */
static int zcells(const orc_problem *pb)
{
    return pb->kind == ORC_BRUSS3D ? pb->nz : 1;
}

int32_t orc_dim(const orc_problem *pb)
{
    return orc_nspecies(pb) * pb->nx * pb->ny * zcells(pb);
}

/*
 * Viscous Burgers v_t = nu v_xx - v v_x (Sec. 5.1, eq. "burg") on [x0, x1)
 * with periodic boundary conditions (the paper's conditions v(-L) = v(L),
 * v_x(-L) = v_x(L)), d equally spaced points x_j = x0 + j dx, dx = (x1-x0)/d,
 * second-order central differences for both derivatives.
 */
static void rhs_burgers(const orc_problem *pb, const double *u, double *h)
{
    const int n = pb->nx;
    const double dx = (pb->x1 - pb->x0) / n;
    const double nu = pb->p[0];
    for (int j = 0; j < n; ++j) {
        const double um = u[(j - 1 + n) % n];
        const double uc = u[j];
        const double up = u[(j + 1) % n];
        const double v_xx = (up - 2.0 * uc + um) / (dx * dx);
        const double v_x = (up - um) / (2.0 * dx);
        h[j] = nu * v_xx - uc * v_x;
    }
}

/* Index of the neighbour cell: periodic wrap, or the cell itself (mirror ghost,
 * zero normal gradient) at a Neumann boundary. */
static int nb(int i, int di, int n, int periodic)
{
    int k = i + di;
    if (k < 0) return periodic ? k + n : i;
    if (k >= n) return periodic ? k - n : i;
    return k;
}

/* Five-point cell-centred Laplacian of field f (ny x nx, row-major) at (x, y). */
static double laplacian(const double *f, int x, int y, int nx, int ny, double dx, double dy,
                        int periodic)
{
    const double c = f[y * nx + x];
    const double xm = f[y * nx + nb(x, -1, nx, periodic)];
    const double xp = f[y * nx + nb(x, +1, nx, periodic)];
    const double ym = f[nb(y, -1, ny, periodic) * nx + x];
    const double yp = f[nb(y, +1, ny, periodic) * nx + x];
    return (xm - 2.0 * c + xp) / (dx * dx) + (ym - 2.0 * c + yp) / (dy * dy);
}

/*
 * Two-species diffusion-reaction with FitzHugh-Nagumo kinetics (Sec. 5.2):
 *   u_t = Du (u_xx + u_yy) + u - u^3 - c - v,   v_t = Dv (v_xx + v_yy) + u - v,
 * finite volumes on nx x ny cells with no-flux (Neumann) walls.
 * State layout: [u(ny x nx), v(ny x nx)].
 */
static void rhs_diffreact(const orc_problem *pb, const double *s, double *h)
{
    const int nx = pb->nx, ny = pb->ny, nc = nx * ny;
    const double dx = (pb->x1 - pb->x0) / nx, dy = (pb->y1 - pb->y0) / ny;
    const double Du = pb->p[0], Dv = pb->p[1], c = pb->p[2];
    const double *u = s, *v = s + nc;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int i = y * nx + x;
            const double Ru = u[i] - u[i] * u[i] * u[i] - c - v[i];
            const double Rv = u[i] - v[i];
            h[i] = Du * laplacian(u, x, y, nx, ny, dx, dy, 0) + Ru;
            h[nc + i] = Dv * laplacian(v, x, y, nx, ny, dx, dy, 0) + Rv;
        }
}

/*
 * Brusselator (App. E):
 *   u_t = Du lap(u) + A - (B + 1) u + u^2 v,   v_t = Dv lap(v) + B u - u^2 v,
 * periodic square grid.  State layout: [u(ny x nx), v(ny x nx)].
 */
static void rhs_bruss(const orc_problem *pb, const double *s, double *h)
{
    const int nx = pb->nx, ny = pb->ny, nc = nx * ny;
    const double dx = (pb->x1 - pb->x0) / nx, dy = (pb->y1 - pb->y0) / ny;
    const double A = pb->p[0], B = pb->p[1], Du = pb->p[2], Dv = pb->p[3];
    const double *u = s, *v = s + nc;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int i = y * nx + x;
            const double u2v = u[i] * u[i] * v[i];
            h[i] = Du * laplacian(u, x, y, nx, ny, dx, dy, 1) + A - (B + 1.0) * u[i] + u2v;
            h[nc + i] = Dv * laplacian(v, x, y, nx, ny, dx, dy, 1) + B * u[i] - u2v;
        }
}

/*
 * Brusselator in three dimensions (App. E): the same reaction as in 2D,
 *   u_t = Du lap u + A - (B + 1) u + u^2 v,   v_t = Dv lap v + B u - u^2 v,
 * on the periodic box (x0, x1) x (y0, y1) x (x0, x1) (App. E takes (-1, 1)^3)
 * with nx x ny x nz cells, the seven-point Laplacian
 *   (f[x-1] - 2 f + f[x+1]) / dx^2 + (same in y) / dy^2 + (same in z) / dz^2,
 * and layout [u; v], each field [z][y][x] with x fastest.
 */
static void rhs_bruss3d(const orc_problem *pb, const double *s, double *h)
{
    const int nx = pb->nx, ny = pb->ny, nz = pb->nz, nc = nx * ny * nz;
    const double dx = (pb->x1 - pb->x0) / nx, dy = (pb->y1 - pb->y0) / ny, dz = (pb->x1 - pb->x0) / nz;
    const double A = pb->p[0], B = pb->p[1], Du = pb->p[2], Dv = pb->p[3];
    for (int f = 0; f < 2; ++f) {
        const double *q = s + (size_t)f * nc;
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int i = (z * ny + y) * nx + x;
                    const int xm = (z * ny + y) * nx + (x + nx - 1) % nx, xp = (z * ny + y) * nx + (x + 1) % nx;
                    const int ym = (z * ny + (y + ny - 1) % ny) * nx + x, yp = (z * ny + (y + 1) % ny) * nx + x;
                    const int zm = (((z + nz - 1) % nz) * ny + y) * nx + x, zp = (((z + 1) % nz) * ny + y) * nx + x;
                    const double lap = (q[xm] - 2.0 * q[i] + q[xp]) / (dx * dx) +
                                       (q[ym] - 2.0 * q[i] + q[yp]) / (dy * dy) +
                                       (q[zm] - 2.0 * q[i] + q[zp]) / (dz * dz);
                    const double u = s[i], v = s[nc + i];
                    const double u2v = u * u * v;
                    if (f == 0) h[i] = Du * lap + A - (B + 1.0) * u + u2v;
                    else h[nc + i] = Dv * lap + B * u - u2v;
                }
    }
}

/*
 * Shallow water (Sec. 5.3) with a flat bottom, conserved variables
 * q = (h, hu, hv), first-order finite volumes with the Rusanov (local
 * Lax-Friedrichs) numerical flux, reflective walls (ghost cell = mirror of
 * the wall cell with the normal momentum negated).
 */
typedef struct { double h, m, n; } swe_q; /* depth, normal momentum, tangential momentum */

/* Rusanov flux across a face with normal direction along "m". */
static swe_q rusanov(swe_q L, swe_q R, double g)
{
    const double uL = L.m / L.h, uR = R.m / R.h;
    const double cL = fabs(uL) + sqrt(g * L.h);
    const double cR = fabs(uR) + sqrt(g * R.h);
    const double a = cL > cR ? cL : cR;
    const double fL_h = L.m, fR_h = R.m;
    const double fL_m = L.m * uL + 0.5 * g * L.h * L.h;
    const double fR_m = R.m * uR + 0.5 * g * R.h * R.h;
    const double fL_n = L.n * uL, fR_n = R.n * uR;
    swe_q F;
    F.h = 0.5 * (fL_h + fR_h) - 0.5 * a * (R.h - L.h);
    F.m = 0.5 * (fL_m + fR_m) - 0.5 * a * (R.m - L.m);
    F.n = 0.5 * (fL_n + fR_n) - 0.5 * a * (R.n - L.n);
    return F;
}

/* state of cell (x, y) seen with normal along x (dir 0) or y (dir 1);
 * out-of-range cells are wall ghosts. */
static swe_q swe_cell(const double *s, int nx, int ny, int x, int y, int dir)
{
    const int nc = nx * ny;
    int gx = x, gy = y, ghost = 0;
    if (gx < 0) { gx = 0; ghost = 1; }
    if (gx >= nx) { gx = nx - 1; ghost = 1; }
    if (gy < 0) { gy = 0; ghost = 1; }
    if (gy >= ny) { gy = ny - 1; ghost = 1; }
    const int i = gy * nx + gx;
    swe_q q;
    q.h = s[i];
    if (dir == 0) { q.m = s[nc + i]; q.n = s[2 * nc + i]; }
    else          { q.m = s[2 * nc + i]; q.n = s[nc + i]; }
    if (ghost) q.m = -q.m;
    return q;
}

static void rhs_swe(const orc_problem *pb, const double *s, double *hdot)
{
    const int nx = pb->nx, ny = pb->ny, nc = nx * ny;
    const double dx = (pb->x1 - pb->x0) / nx, dy = (pb->y1 - pb->y0) / ny;
    const double g = pb->p[0];
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int i = y * nx + x;
            /* x direction: faces x-1/2 and x+1/2 */
            const swe_q Fw = rusanov(swe_cell(s, nx, ny, x - 1, y, 0), swe_cell(s, nx, ny, x, y, 0), g);
            const swe_q Fe = rusanov(swe_cell(s, nx, ny, x, y, 0), swe_cell(s, nx, ny, x + 1, y, 0), g);
            /* y direction: faces y-1/2 and y+1/2 */
            const swe_q Gs = rusanov(swe_cell(s, nx, ny, x, y - 1, 1), swe_cell(s, nx, ny, x, y, 1), g);
            const swe_q Gn = rusanov(swe_cell(s, nx, ny, x, y, 1), swe_cell(s, nx, ny, x, y + 1, 1), g);
            /* x-normal flux: m = hu, n = hv; y-normal flux: m = hv, n = hu */
            hdot[i] = -(Fe.h - Fw.h) / dx - (Gn.h - Gs.h) / dy;
            hdot[nc + i] = -(Fe.m - Fw.m) / dx - (Gn.n - Gs.n) / dy;
            hdot[2 * nc + i] = -(Fe.n - Fw.n) / dx - (Gn.m - Gs.m) / dy;
        }
}

int32_t orc_rhs(const orc_problem *pb, const double *u, double *out)
{
    if (pb->nx < 1 || pb->ny < 1 || zcells(pb) < 1) return -1;
    switch (pb->kind) {
    case ORC_BURGERS1D: rhs_burgers(pb, u, out); return 0;
    case ORC_DIFFREACT2D: rhs_diffreact(pb, u, out); return 0;
    case ORC_BRUSS2D: rhs_bruss(pb, u, out); return 0;
    case ORC_SWE2D: rhs_swe(pb, u, out); return 0;
    case ORC_BRUSS3D: rhs_bruss3d(pb, u, out); return 0;
    default: return -1;
    }
}
