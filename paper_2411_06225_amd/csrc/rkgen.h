// rkgen.h -- explicit Runge-Kutta steps of any Butcher tableau over slot
// states in memory: the eighth-order fine solver, and every propagator of
// the three-dimensional Brusselator.
//
// Sec. 2: F and G are fixed-step explicit Runge-Kutta methods; the paper's
// fine solver for the Burgers and diffusion-reaction runs is an RK8, which
// it does not specify.  This path takes the tableau as data: forward Euler,
// classical RK4, and the eighth-order method of Cooper and Verner (SIAM J.
// Numer. Anal. 9, 1972; 11 stages).  A stage is one pass over the cells:
// a thread evaluates h at its cell from the stage input Y_i in memory (the
// neighbours through L1/L2), stores the slope k_i, and forms the next stage
// input Y_{i+1} = u + dt sum_{j<=i} a_{i+1,j} k_j at its cell from the
// slopes stored there; the last stage forms u + dt sum_j b_j k_j instead
// (FP32 states: compensated).  Stage inputs alternate between two arrays,
// so a pass never overwrites what another thread may still read.
#pragma once

#include "common.h"

namespace rpr {

// Selects the generic path in rpr_propagator.threads and the shapes.
constexpr int GENERIC_THREADS = 128;
// Slopes per step of the largest tableau.
constexpr int RK_MAX_STAGES = 11;

struct Tableau {
    int s;                                  // stages
    double a[RK_MAX_STAGES][RK_MAX_STAGES]; // strictly lower
    double b[RK_MAX_STAGES];
};

// The library's tableaux (method 1, 4 or 8).
inline Tableau rk_tableau(int method)
{
    Tableau t{};
    if (method == RPR_RK4) {
        t.s = 4;
        t.a[1][0] = 0.5;
        t.a[2][1] = 0.5;
        t.a[3][2] = 1.0;
        t.b[0] = 1.0 / 6.0;
        t.b[1] = 1.0 / 3.0;
        t.b[2] = 1.0 / 3.0;
        t.b[3] = 1.0 / 6.0;
    } else if (method == RPR_RK8) {
        // Cooper and Verner's eighth-order method, with q = sqrt(21)
        const double q = 4.58257569495584000658804719372800848898445657676797190260724212390686842554777;
        t.s = 11;
        t.a[1][0] = 0.5;
        t.a[2][0] = 0.25;
        t.a[2][1] = 0.25;
        t.a[3][0] = 1.0 / 7.0;
        t.a[3][1] = -(7.0 + 3.0 * q) / 98.0;
        t.a[3][2] = (21.0 + 5.0 * q) / 49.0;
        t.a[4][0] = (11.0 + q) / 84.0;
        t.a[4][2] = (18.0 + 4.0 * q) / 63.0;
        t.a[4][3] = (21.0 - q) / 252.0;
        t.a[5][0] = (5.0 + q) / 48.0;
        t.a[5][2] = (9.0 + q) / 36.0;
        t.a[5][3] = (14.0 * q - 231.0) / 360.0;
        t.a[5][4] = (63.0 - 7.0 * q) / 80.0;
        t.a[6][0] = (10.0 - q) / 42.0;
        t.a[6][2] = (92.0 * q - 432.0) / 315.0;
        t.a[6][3] = (633.0 - 145.0 * q) / 90.0;
        t.a[6][4] = (115.0 * q - 504.0) / 70.0;
        t.a[6][5] = (63.0 - 13.0 * q) / 35.0;
        t.a[7][0] = 1.0 / 14.0;
        t.a[7][4] = (14.0 - 3.0 * q) / 126.0;
        t.a[7][5] = (13.0 - 3.0 * q) / 63.0;
        t.a[7][6] = 1.0 / 9.0;
        t.a[8][0] = 1.0 / 32.0;
        t.a[8][4] = (91.0 - 21.0 * q) / 576.0;
        t.a[8][5] = 11.0 / 72.0;
        t.a[8][6] = -(385.0 + 75.0 * q) / 1152.0;
        t.a[8][7] = (63.0 + 13.0 * q) / 128.0;
        t.a[9][0] = 1.0 / 14.0;
        t.a[9][4] = 1.0 / 9.0;
        t.a[9][5] = -(733.0 + 147.0 * q) / 2205.0;
        t.a[9][6] = (515.0 + 111.0 * q) / 504.0;
        t.a[9][7] = -(51.0 + 11.0 * q) / 56.0;
        t.a[9][8] = (132.0 + 28.0 * q) / 245.0;
        t.a[10][4] = (7.0 * q - 42.0) / 18.0;
        t.a[10][5] = (28.0 * q - 18.0) / 45.0;
        t.a[10][6] = -(273.0 + 53.0 * q) / 72.0;
        t.a[10][7] = (301.0 + 53.0 * q) / 72.0;
        t.a[10][8] = (28.0 - 28.0 * q) / 45.0;
        t.a[10][9] = (49.0 - 7.0 * q) / 18.0;
        t.b[0] = 1.0 / 20.0;
        t.b[7] = 49.0 / 180.0;
        t.b[8] = 16.0 / 45.0;
        t.b[9] = 49.0 / 180.0;
        t.b[10] = 1.0 / 20.0;
    } else {
        t.s = 1;
        t.b[0] = 1.0;
    }
    return t;
}

// Elements of the work arrays of the generic path for n states of d values:
// the state u, two stage inputs, the FP32 compensation, and s slopes.
inline size_t rkgen_work_elems(int method, size_t n, size_t d)
{
    return (4 + (size_t)rk_tableau(method).s) * n * d;
}

// The generic work arrays inside a TiledWork block of rkgen_work_elems:
// u, ya, yb, cmp (n x d each), then acc = the s slopes (slope j of state b at
// (j n + b) d).
template <typename T>
inline TiledWork<T> rkgen_work(void *base, size_t n, size_t d)
{
    T *p = static_cast<T *>(base);
    const size_t nd = n * d;
    return TiledWork<T>{p, p + 4 * nd, p + nd, p + 2 * nd, p + 3 * nd};
}

// h at cell c of state y (d values) with the neighbours read from memory and
// the boundary rule of the system: wrap (Burgers, the Brusselators), the cell
// itself beyond a wall (diffusion-reaction), the mirror with the normal
// momentum negated (shallow water, through rhs_swe's wall flags).
template <int KIND, typename T>
__device__ __forceinline__ void rhs_at(const Geom &g, const T *__restrict__ y, const int c, T *k)
{
    constexpr int NS = kind_ns<KIND>();
    const int nx = g.nx, ny = g.ny, nc = g.nc;
    if constexpr (KIND == RPR_BURGERS1D) {
        const int w = c == 0 ? nx - 1 : c - 1, e = c == nx - 1 ? 0 : c + 1;
        const T cc[1] = {y[c]}, ww[1] = {y[w]}, ee[1] = {y[e]};
        rhs_burgers<T>(cc, ww, ee, k, T(g.p[0]), T(g.idx2), T(g.i2dx));
    } else if constexpr (KIND == RPR_BRUSS3D) {
        const int nxy = nx * ny;
        const int z = c / nxy, r = c - z * nxy, yy = r / nx, x = r - yy * nx;
        const int xm = x == 0 ? c + nx - 1 : c - 1, xp = x == nx - 1 ? c - nx + 1 : c + 1;
        const int ym = yy == 0 ? c + nxy - nx : c - nx, yp = yy == ny - 1 ? c - nxy + nx : c + nx;
        const int zm = z == 0 ? c + nc - nxy : c - nxy, zp = z == g.nz - 1 ? c - nc + nxy : c + nxy;
        T cc[2], xs[2], ys[2], zs[2];
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            const T *f = y + sp * nc;
            cc[sp] = f[c];
            xs[sp] = f[xm] + f[xp];
            ys[sp] = f[ym] + f[yp];
            zs[sp] = f[zm] + f[zp];
        }
        rhs_bruss3d<T>(cc, xs, ys, zs, k, T(g.p[0]), T(g.p[1]), T(g.p[2] * g.idx2), T(g.p[2] * g.idy2),
                       T(g.p[2] * g.idz2), T(g.p[3] * g.idx2), T(g.p[3] * g.idy2), T(g.p[3] * g.idz2));
    } else {
        const bool per = g.periodic != 0;
        const int yy = c / nx, x = c - yy * nx;
        const bool ww = !per && x == 0, we = !per && x == nx - 1, ws = !per && yy == 0, wn = !per && yy == ny - 1;
        const int xm = x == 0 ? (per ? c + nx - 1 : c) : c - 1;
        const int xp = x == nx - 1 ? (per ? c - nx + 1 : c) : c + 1;
        const int ym = yy == 0 ? (per ? c + nc - nx : c) : c - nx;
        const int yp = yy == ny - 1 ? (per ? c - nc + nx : c) : c + nx;
        T cc[NS], w[NS], e[NS], s[NS], n[NS];
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const T *f = y + sp * nc;
            cc[sp] = f[c];
            w[sp] = f[xm];
            e[sp] = f[xp];
            s[sp] = f[ym];
            n[sp] = f[yp];
        }
        rhs_cell<KIND, T>(g, cc, w, e, s, n, ww, we, ws, wn, k);
    }
}

// One stage of one state at cell c.  y: this stage's input; k: the slope
// arrays (slope j at k + j kstride); u: the state at the start of the step;
// ynext: the next stage's input, or for the last stage the new state (uout,
// and uout2 if not null; cmp the FP32 compensation, cmp_zero: read as zero).
template <int KIND, typename T>
__device__ __forceinline__ void rkgen_cell(const Geom &g, const Tableau &tb, const int stage, const double dt,
                                           const int c, const T *__restrict__ y, T *__restrict__ k,
                                           const size_t kstride, const T *__restrict__ u, T *__restrict__ ynext,
                                           T *__restrict__ uout, T *__restrict__ uout2, T *__restrict__ cmp,
                                           const int cmp_zero)
{
    constexpr int NS = kind_ns<KIND>();
    constexpr bool KAHAN = sizeof(T) == 4;
    const int nc = g.nc;
    T ki[NS];
    rhs_at<KIND, T>(g, y, c, ki);
#pragma unroll
    for (int sp = 0; sp < NS; ++sp) k[(size_t)stage * kstride + sp * nc + c] = ki[sp];
    const bool last = stage == tb.s - 1;
#pragma unroll
    for (int sp = 0; sp < NS; ++sp) {
        const int idx = sp * nc + c;
        // sum over the slopes of this cell with the next row of the tableau
        // (or its weights b): slope `stage` from the register, the others
        // from memory
        T acc = T(0);
        for (int j = 0; j <= stage; ++j) {
            const double cf = last ? tb.b[j] : tb.a[stage + 1][j];
            if (cf == 0.0) continue;
            const T kj = j == stage ? ki[sp] : k[(size_t)j * kstride + idx];
            acc = acc + T(cf) * kj;
        }
        const T uu = u[idx];
        if (!last) {
            ynext[idx] = uu + T(dt) * acc;
        } else if constexpr (KAHAN) {
            const T cm = cmp_zero ? T(0) : cmp[idx];
            const T yk = T(dt) * acc - cm;
            const T un = uu + yk;
            cmp[idx] = (un - uu) - yk;
            uout[idx] = un;
            if (uout2) uout2[idx] = un;
        } else {
            const T un = uu + T(dt) * acc;
            uout[idx] = un;
            if (uout2) uout2[idx] = un;
        }
    }
}

// The arrays of stage `stage` of step `step` of a propagation src -> dst
// (dst2) over `steps` steps with work arrays w of one state (u, ya, yb, cmp,
// slopes at w.acc with stride kstride): the step starts from src (step 0) or
// w.u, stage 0 reads that state, stage i > 0 reads ya (i odd) or yb (i even),
// stage i < s - 1 writes the other; the last stage writes dst on the last
// step, else w.u.  With one stage (forward Euler) the last stage reads the
// state itself at the neighbours, so the state alternates between w.u and
// w.ya from step to step instead.
template <typename T>
struct RkIO {
    const T *y, *u;
    T *ynext, *uout, *uout2;
};

template <typename T>
__host__ __device__ inline RkIO<T> rkgen_io(const int s, const int stage, const long long step, const long long steps,
                                            const T *src, T *dst, T *dst2, const TiledWork<T> &w)
{
    RkIO<T> io{};
    const bool lastStep = step == steps - 1;
    io.uout2 = lastStep ? dst2 : nullptr;
    if (s == 1) {
        T *buf[2] = {w.u, w.ya};
        io.u = io.y = step == 0 ? src : buf[(step - 1) & 1];
        io.ynext = nullptr;
        io.uout = lastStep ? dst : buf[step & 1];
        return io;
    }
    const T *u = step == 0 ? src : w.u;
    io.u = u;
    io.y = stage == 0 ? u : ((stage & 1) ? w.ya : w.yb);
    io.ynext = (stage & 1) ? w.yb : w.ya;
    io.uout = lastStep ? dst : w.u;
    return io;
}

}  // namespace rpr
