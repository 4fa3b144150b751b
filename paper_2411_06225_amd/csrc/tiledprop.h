// tiledprop.h -- propagation of slot states too large for one work-group.
//
// Sec. 2: F and G are fixed-step explicit Runge-Kutta methods.  When a 2D
// slot state does not fit one compute unit, every RK stage becomes a pass
// over 64 x 16-cell tiles of the state in memory: a work-group of 256
// threads copies the tile of the stage input with a one-cell halo into LDS
// (the boundary rule applied while copying: wrap when periodic, the cell
// itself at a wall), evaluates the right-hand side of its cells (a column of
// 4 rows per thread, lane = column) and applies the stage update to the RK
// arrays in memory.  The
// update formulas, their order and the FP32 compensation are those of the
// on-chip propagator, so both agree to rounding.
#pragma once

#include "common.h"

namespace rpr {

constexpr int TT_X = 64, TT_Y = 16, TT_THREADS = 256;
constexpr int TT_RPT = TT_X * TT_Y / TT_THREADS;  // rows per thread

__host__ __device__ inline int tiles_x(const Geom &g) { return (g.nx + TT_X - 1) / TT_X; }
__host__ __device__ inline int tiles_of(const Geom &g) { return tiles_x(g) * ((g.ny + TT_Y - 1) / TT_Y); }

// Work-group id -> (tile, slot state) of a one-dimensional launch over
// tiles x n work-groups.  Work-groups go to the eight XCDs round robin
// (id % 8), each XCD with its own L2: each XCD gets whole slot states, their
// tiles in row-major order one after the other, so the halo rows and columns
// a tile shares with its neighbours come through the same L2.  States beyond
// the last multiple of 8 take the plain order.
__device__ __forceinline__ void tile_of_block(const int id, const int tiles, const int n, int &tile, int &slot)
{
    constexpr int XCD = 8;
    const int n8 = n / XCD * XCD, head = tiles * n8;
    if (id < head) {
        const int x = id % XCD, j = id / XCD;
        slot = (j / tiles) * XCD + x;
        tile = j % tiles;
    } else {
        const int r = id - head;
        slot = n8 + r / tiles;
        tile = r % tiles;
    }
}

// LDS of one haloed tile (shallow water: twice, for the per-cell flux
// quantities).
__host__ __device__ inline size_t tiled_lds(const Geom &g, size_t elem)
{
    return (size_t)g.ns * (TT_Y + 2) * (TT_X + 2) * elem * (g.kind == RPR_SWE2D ? 2 : 1);
}

// The arrays one stage touches in one slot state (d values each).
//   stage 0 (forward Euler): u_out = u + dt f(y), y = u
//   stage 1..3 (RK4):        acc (=, +=) k; y_out = u + c dt k
//   stage 4 (RK4):           u_out = u + dt/6 (acc + k)
// cmp: running compensation of FP32 states (null in FP64); cmp_zero: read
// it as zero (the first step of a propagation).
template <typename T>
struct StageIO {
    const T *y;
    const T *u;
    T *u_out;
    T *u_out2;  // optional second copy of the final state
    T *acc;
    T *y_out;
    T *cmp;
    int cmp_zero;
};

// Indices into one slot state are 32-bit (d < 2^31).
// Load from global memory.  The stage arrays reach the tile code through a
// struct, where the compiler no longer sees that they are global; a flat
// load also counts against the scalar-load counter, so every wait for a
// kernel argument would drain the tile's loads too.
template <typename T>
__device__ __forceinline__ T gload(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}

// Shallow-water fluxes of one tile (Rusanov, as in the on-chip form), with
// the per-cell quantities evaluated once per cell and each interface flux
// once per interface:
//   per cell  u = hu/h, v = hv/h, c = sqrt(g h), P = g h^2 / 2,
//             x: (hu u + P, hv u, |u| + c),  y: (hv v + P, hu v, |v| + c);
//   per face  a = max of the two speeds,
//             F = (f_L + f_R)/2 - a (q_R - q_L)/2 component by component.
// The stage input sits in lds[0 .. 3 PY PX) with wall ghosts already
// mirrored; lds[3 PY PX .. 6 PY PX) holds the x quantities, then the y
// quantities.  Threads: lane = column, TT_RPT rows per thread from cy0;
// waves 0 and 1 also evaluate the halo rows, wave 2 the halo columns.
template <typename T, typename Update>
__device__ __forceinline__ void swe_tile(const Geom &g, const int x0, const int y0, const int lane, const int wv,
                                         const int cy0, T *__restrict__ lds, const T (&uv)[TT_RPT][3],
                                         Update &update)
{
    constexpr int PX = TT_X + 2, PY = TT_Y + 2, SP = PY * PX, R = TT_RPT;
    const T gg = T(g.p[0]), idx = T(g.idx), idy = T(g.idy), half = T(0.5);
    const int nx = g.nx, ny = g.ny, nc = g.nc;
    const T *qb = lds;
    T *db = lds + 3 * SP;
    const int lx = lane + 1;

    // own cells: state, x quantities to LDS, y quantities kept
    T h[R], m[R], n[R], ym[R], yn[R], ys[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int o = (cy0 + q + 1) * PX + lx;
        h[q] = qb[o];
        m[q] = qb[SP + o];
        n[q] = qb[2 * SP + o];
        const T u = m[q] / h[q], v = n[q] / h[q], c = sqrt(gg * h[q]), P = half * gg * h[q] * h[q];
        db[o] = m[q] * u + P;
        db[SP + o] = n[q] * u;
        db[2 * SP + o] = fabs(u) + c;
        ym[q] = n[q] * v + P;
        yn[q] = m[q] * v;
        ys[q] = fabs(v) + c;
    }
    // halo rows (waves 0, 1: y quantities kept) and columns (wave 2: x quantities)
    T hym = T(0), hyn = T(0), hys = T(0);
    if (wv <= 1) {
        const int o = (wv == 0 ? 0 : PY - 1) * PX + lx;
        const T hh = qb[o], hm = qb[SP + o], hn = qb[2 * SP + o];
        const T v = hn / hh, c = sqrt(gg * hh), P = half * gg * hh * hh;
        hym = hn * v + P;
        hyn = hm * v;
        hys = fabs(v) + c;
    } else if (wv == 2 && lane < 2 * TT_Y) {
        const int o = (1 + (lane >> 1)) * PX + ((lane & 1) ? PX - 1 : 0);
        const T hh = qb[o], hm = qb[SP + o], hn = qb[2 * SP + o];
        const T u = hm / hh, c = sqrt(gg * hh), P = half * gg * hh * hh;
        db[o] = hm * u + P;
        db[SP + o] = hn * u;
        db[2 * SP + o] = fabs(u) + c;
    }
    __syncthreads();

    // x faces west and east of each own cell
    T dh[R], dm[R], dn[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int o = (cy0 + q + 1) * PX + lx;
        const T cm = db[o], cn = db[SP + o], cs = db[2 * SP + o];
        T Fh[2], Fm[2], Fn[2];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int on = side ? o + 1 : o - 1;
            const T oh = qb[on], om = qb[SP + on], onn = qb[2 * SP + on];
            const T fm = db[on], fn = db[SP + on], fs = db[2 * SP + on];
            // left and right states of the face
            const T hL = side ? h[q] : oh, hR = side ? oh : h[q];
            const T mL = side ? m[q] : om, mR = side ? om : m[q];
            const T nL = side ? n[q] : onn, nR = side ? onn : n[q];
            const T fmL = side ? cm : fm, fmR = side ? fm : cm;
            const T fnL = side ? cn : fn, fnR = side ? fn : cn;
            const T sL = side ? cs : fs, sR = side ? fs : cs;
            const T a = sL > sR ? sL : sR;
            Fh[side] = half * (mL + mR) - half * a * (hR - hL);
            Fm[side] = half * (fmL + fmR) - half * a * (mR - mL);
            Fn[side] = half * (fnL + fnR) - half * a * (nR - nL);
        }
        dh[q] = Fh[1] - Fh[0];
        dm[q] = Fm[1] - Fm[0];
        dn[q] = Fn[1] - Fn[0];
    }
    __syncthreads();

    // y quantities replace the x quantities
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int o = (cy0 + q + 1) * PX + lx;
        db[o] = ym[q];
        db[SP + o] = yn[q];
        db[2 * SP + o] = ys[q];
    }
    if (wv <= 1) {
        const int o = (wv == 0 ? 0 : PY - 1) * PX + lx;
        db[o] = hym;
        db[SP + o] = hyn;
        db[2 * SP + o] = hys;
    }
    __syncthreads();

    // y faces of the strip: face f lies below own row f (f = 0 .. R)
    T Gh[R + 1], Gm[R + 1], Gn[R + 1];
#pragma unroll
    for (int f = 0; f <= R; ++f) {
        T hL, nL, mL, gmL, gnL, sL, hR, nR, mR, gmR, gnR, sR;
        if (f == 0) {
            const int o = cy0 * PX + lx;
            hL = qb[o]; mL = qb[SP + o]; nL = qb[2 * SP + o];
            gmL = db[o]; gnL = db[SP + o]; sL = db[2 * SP + o];
        } else {
            hL = h[f - 1]; mL = m[f - 1]; nL = n[f - 1];
            gmL = ym[f - 1]; gnL = yn[f - 1]; sL = ys[f - 1];
        }
        if (f == R) {
            const int o = (cy0 + R + 1) * PX + lx;
            hR = qb[o]; mR = qb[SP + o]; nR = qb[2 * SP + o];
            gmR = db[o]; gnR = db[SP + o]; sR = db[2 * SP + o];
        } else {
            hR = h[f]; mR = m[f]; nR = n[f];
            gmR = ym[f]; gnR = yn[f]; sR = ys[f];
        }
        const T a = sL > sR ? sL : sR;
        Gh[f] = half * (nL + nR) - half * a * (hR - hL);
        Gm[f] = half * (gmL + gmR) - half * a * (nR - nL);  // normal (hv) component
        Gn[f] = half * (gnL + gnR) - half * a * (mR - mL);  // tangential (hu) component
    }

    const int gx = x0 + lane;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int gy = y0 + cy0 + q;
        if (gx < nx && gy < ny) {
            const int c0 = gy * nx + gx;
            const T k0 = -dh[q] * idx - (Gh[q + 1] - Gh[q]) * idy;
            const T k1 = -dm[q] * idx - (Gn[q + 1] - Gn[q]) * idy;
            const T k2 = -dn[q] * idx - (Gm[q + 1] - Gm[q]) * idy;
            update(q, 0, c0, uv[q][0], k0, h[q]);
            update(q, 1, nc + c0, uv[q][1], k1, m[q]);
            update(q, 2, 2 * nc + c0, uv[q][2], k2, n[q]);
        }
    }
}

// The boundary of each system, as the geometry records it: the Burgers
// equation and the Brusselator wrap, the other systems have walls.
template <int KIND>
constexpr bool kind_periodic()
{
    return KIND == RPR_BURGERS1D || KIND == RPR_BRUSS2D;
}

// The tile of the stage input with its one-cell halo goes to LDS; each wave
// copies whole rows (one cell per lane, the boundary rule applied to the
// row index), the two halo columns follow in one pass.  Every load of the
// tile is issued before the first LDS write, and the operands of the stage
// update are fetched before the right-hand side is evaluated, so a
// work-group waits for memory once per stage instead of once per access.
template <int KIND, typename T, int STAGE>
__device__ __forceinline__ void stage_tile(const Geom &g, const int tile, const double dt, const StageIO<T> &io,
                                           T *__restrict__ lds)
{
    constexpr int NS = kind_ns<KIND>();
    constexpr int PX = TT_X + 2, PY = TT_Y + 2;
    constexpr int NW = TT_THREADS / 64;                // waves
    constexpr int NR = (NS * PY + NW - 1) / NW;        // rows per wave
    constexpr int NH = NS * PY * 2;                    // halo-column cells
    constexpr bool KAHAN = sizeof(T) == 4;
    constexpr bool Y_IS_U = STAGE <= 1;                // Euler and the first RK4 stage read u itself
    static_assert(TT_X == 64 && NH <= TT_THREADS, "tile shape");
    const int nx = g.nx, ny = g.ny, nc = g.nc;
    constexpr bool per = kind_periodic<KIND>();
    const int x0 = (tile % tiles_x(g)) * TT_X, y0 = (tile / tiles_x(g)) * TT_Y;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;

    // Every load below is unconditional, with indices clamped into the
    // state (values of cells outside it are loaded but never used), so no
    // control flow separates a load from its use.
    // rows of the tile: lane = interior column
    int gxi = x0 + lane;
    gxi = gxi < nx ? gxi : (per ? gxi - nx : nx - 1);
    gxi = gxi < nx ? gxi : nx - 1;
    T rowv[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int r0 = wv + j * NW;  // species-major row index
        const int r = r0 < NS * PY ? r0 : NS * PY - 1;
        const int sp = r / PY, ly = r % PY;
        const int gy0 = y0 + ly - 1;
        const int gyw = gy0 < 0 ? gy0 + ny : (gy0 >= ny ? gy0 - ny : gy0);
        const int gyc = gy0 < 0 ? 0 : (gy0 >= ny ? ny - 1 : gy0);
        int gy = per ? gyw : gyc;
        gy = gy < ny ? gy : ny - 1;
        rowv[j] = gload(io.y + (sp * nc + gy * nx + gxi));
        if constexpr (KIND == RPR_SWE2D) {
            // a wall ghost is the mirror image: normal momentum negated
            const bool xg = !per && x0 + lane >= nx, yg = !per && (gy0 < 0 || gy0 >= ny);
            if ((sp == 1 && xg) || (sp == 2 && yg)) rowv[j] = -rowv[j];
        }
    }
    // halo columns x0 - 1 and x0 + TT_X
    T halov;
    {
        const int th = t < NH ? t : NH - 1;
        const int sp = th / (2 * PY), r = th % (2 * PY), ly = r >> 1, side = r & 1;
        const int gx0 = side ? x0 + TT_X : x0 - 1, gy0 = y0 + ly - 1;
        const int gxw = gx0 < 0 ? gx0 + nx : (gx0 >= nx ? gx0 - nx : gx0);
        const int gxc = gx0 < 0 ? 0 : (gx0 >= nx ? nx - 1 : gx0);
        const int gyw = gy0 < 0 ? gy0 + ny : (gy0 >= ny ? gy0 - ny : gy0);
        const int gyc = gy0 < 0 ? 0 : (gy0 >= ny ? ny - 1 : gy0);
        int gx = per ? gxw : gxc, gy = per ? gyw : gyc;
        gx = gx < nx ? gx : nx - 1;
        gy = gy < ny ? gy : ny - 1;
        halov = gload(io.y + (sp * nc + gy * nx + gx));
        if constexpr (KIND == RPR_SWE2D) {
            const bool xg = !per && (gx0 < 0 || gx0 >= nx), yg = !per && (gy0 < 0 || gy0 >= ny);
            if ((sp == 1 && xg) || (sp == 2 && yg)) halov = -halov;
        }
    }

    // operands of the stage update of this thread's cells
    const int cy0 = wv * TT_RPT;
    const int gx = x0 + lane;
    const int gxs = gx < nx ? gx : nx - 1;
    T uv[TT_RPT][NS], av[TT_RPT][NS], cv[TT_RPT][NS];
#pragma unroll
    for (int q = 0; q < TT_RPT; ++q) {
        const int gy = y0 + cy0 + q;
        const int gys = gy < ny ? gy : ny - 1;
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const int idx = sp * nc + gys * nx + gxs;
            uv[q][sp] = Y_IS_U ? T(0) : gload(io.u + idx);
            av[q][sp] = (STAGE == 2 || STAGE == 3 || STAGE == 4) ? gload(io.acc + idx) : T(0);
            if constexpr (KAHAN && (STAGE == 0 || STAGE == 4)) {
                const T cm = gload(io.cmp + idx);
                cv[q][sp] = io.cmp_zero ? T(0) : cm;
            } else {
                cv[q][sp] = T(0);
            }
        }
    }

    // keep every load above in flight before the first LDS write
    asm volatile("" ::: "memory");
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int r = wv + j * NW;
        if (r < NS * PY) lds[r * PX + 1 + lane] = rowv[j];
    }
    if (t < NH) {
        const int sp = t / (2 * PY), r = t % (2 * PY), ly = r >> 1, side = r & 1;
        lds[(sp * PY + ly) * PX + (side ? PX - 1 : 0)] = halov;
    }
    __syncthreads();

    const T dtT = T(dt), hdt = T(0.5 * dt), dt6 = T(dt / 6.0);
    // stage update of cell (q, sp) at idx with slope k: the RK base value is
    // uu, or the stage input yy where the stage reads u itself
    auto update = [&](const int q, const int sp, const int idx, const T uu, const T k, const T yy) {
        const T u = Y_IS_U ? yy : uu;
        if constexpr (STAGE == 1) {
            io.acc[idx] = k;
            io.y_out[idx] = u + hdt * k;
        } else if constexpr (STAGE == 2) {
            io.acc[idx] = av[q][sp] + T(2) * k;
            io.y_out[idx] = u + hdt * k;
        } else if constexpr (STAGE == 3) {
            io.acc[idx] = av[q][sp] + T(2) * k;
            io.y_out[idx] = u + dtT * k;
        } else {
            const T inc = STAGE == 4 ? dt6 * (av[q][sp] + k) : dtT * k;
            if constexpr (KAHAN) {
                const T yk = inc - cv[q][sp];
                const T un = u + yk;
                io.cmp[idx] = (un - u) - yk;
                io.u_out[idx] = un;
                if (io.u_out2) io.u_out2[idx] = un;
            } else {
                io.u_out[idx] = u + inc;
                if (io.u_out2) io.u_out2[idx] = u + inc;
            }
        }
    };

    if constexpr (KIND == RPR_SWE2D) {
        swe_tile<T>(g, x0, y0, lane, wv, cy0, lds, uv, update);
    } else {
#pragma unroll
        for (int q = 0; q < TT_RPT; ++q) {
            const int gy = y0 + cy0 + q;
            if (gx < nx && gy < ny) {
                const int lx = lane + 1, ly = cy0 + q + 1;
                T c[NS], w[NS], e[NS], s[NS], n[NS], k[NS];
#pragma unroll
                for (int sp = 0; sp < NS; ++sp) {
                    const T *b = lds + sp * PY * PX;
                    c[sp] = b[ly * PX + lx];
                    w[sp] = b[ly * PX + lx - 1];
                    e[sp] = b[ly * PX + lx + 1];
                    s[sp] = b[(ly - 1) * PX + lx];
                    n[sp] = b[(ly + 1) * PX + lx];
                }
                rhs_cell<KIND, T>(g, c, w, e, s, n, !per && gx == 0, !per && gx == nx - 1, !per && gy == 0,
                                  !per && gy == ny - 1, k);
#pragma unroll
                for (int sp = 0; sp < NS; ++sp)
                    update(q, sp, sp * nc + gy * nx + gx, uv[q][sp], k[sp], c[sp]);
            }
        }
    }
    __syncthreads();  // the tile buffer is reused by the next tile
}

// Several forward-Euler steps of one tile without leaving the work-group
// (the coarse solver of the sequential sweep, where a grid barrier per step
// would cost more than the step).  The tile is loaded with an EH-cell halo
// (the cells of the domain within EH of it: wrapped when periodic, cut at a
// wall), then step t = 1..steps (steps <= EH) updates the region shrunk by t
// cells on every side that is not a wall, in LDS; after the last step the
// tile's own cells are exact and go to dst (and dst2).  A cell at a wall
// takes itself as the missing neighbour, as the one-step form does.  Per
// cell and step the arithmetic is that of stage_tile<KIND, T, 0>, FP32 state
// compensation included: read from cmp_in (the halo included; cmp_zero: start
// from zero) and written for the tile's own cells to cmp_out.  The two must
// differ: the tiles of one pass run without a barrier between them, so a
// tile may read a neighbour's compensation while that neighbour writes its
// own; alternating the arrays between passes, as the state alternates, keeps
// every read on the previous pass's values.
// The tile: EX x EY cells with an EH-cell halo (so up to EH steps a pass).
template <int EX_, int EY_, int EH_>
struct EulerTile {
    static constexpr int EX = EX_, EY = EY_, EH = EH_;
    static constexpr int ERX = EX + 2 * EH, ERY = EY + 2 * EH;
    __host__ __device__ static int tiles_x(const Geom &g) { return (g.nx + EX - 1) / EX; }
    __host__ __device__ static int tiles(const Geom &g) { return tiles_x(g) * ((g.ny + EY - 1) / EY); }
    __host__ __device__ static size_t lds(const Geom &g, size_t elem)
    {
        return (size_t)(elem == 4 ? 3 : 2) * g.ns * ERY * ERX * elem;
    }
};
// The sweep's tiles: 16 x 16 cells when there are no more of them than
// work-groups (a 192 x 192 grid: 144 tiles, each a quarter of the halo
// region's cells per thread of the 64 x 16 form, 28 against 64 us for eight
// steps), else 64 x 16 (less halo per cell when the tiles take several
// rounds).  Both give the same values bit for bit: a cell's update depends
// only on its neighbours at the previous step.
using SweepEuler = EulerTile<64, 16, 8>;
using SweepEulerSmall = EulerTile<16, 16, 8>;
constexpr int EH = SweepEuler::EH;
static_assert(SweepEulerSmall::EH == EH, "one step count per pass for both tile shapes");

__host__ __device__ inline size_t euler_multi_lds(const Geom &g, size_t elem) { return SweepEuler::lds(g, elem); }

template <int KIND, typename T, typename ET = SweepEuler>
__device__ __forceinline__ void euler_tile_multi(const Geom &g, const int tile, const int steps, const double dt,
                                                 const T *__restrict__ src, T *__restrict__ dst,
                                                 T *__restrict__ dst2, const T *__restrict__ cmp_in,
                                                 T *__restrict__ cmp_out, const int cmp_zero, T *__restrict__ lds)
{
    constexpr int EX = ET::EX, EY = ET::EY, EH = ET::EH, ERX = ET::ERX, ERY = ET::ERY;
    constexpr int NS = kind_ns<KIND>();
    constexpr int RN = ERX * ERY;
    constexpr bool KAHAN = sizeof(T) == 4;
    const int nx = g.nx, ny = g.ny, nc = g.nc;
    constexpr bool per = kind_periodic<KIND>();
    const int x0 = (tile % ET::tiles_x(g)) * EX, y0 = (tile / ET::tiles_x(g)) * EY;
    const int gx0 = x0 - EH, gy0 = y0 - EH;  // domain cell of region cell (0, 0)
    T *buf[2] = {lds, lds + NS * RN};
    T *cm = lds + 2 * NS * RN;  // FP32 compensation
    // sides that cut the domain (the rest lie at a wall)
    const int cw = per || gx0 > 0, ce = per || gx0 + ERX < nx;
    const int cs = per || gy0 > 0, cn = per || gy0 + ERY < ny;
    auto gcoord = [&](int l, int o, int n) {  // region index -> domain index, or -1 outside a wall
        int v = o + l;
        if (per) return ((v % n) + n) % n;
        return (v < 0 || v >= n) ? -1 : v;
    };
    for (int e = threadIdx.x; e < RN; e += blockDim.x) {
        const int gx = gcoord(e % ERX, gx0, nx), gy = gcoord(e / ERX, gy0, ny);
        if (gx < 0 || gy < 0) continue;
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const int idx = sp * nc + gy * nx + gx;
            buf[0][sp * RN + e] = src[idx];
            if constexpr (KAHAN) cm[sp * RN + e] = cmp_zero ? T(0) : cmp_in[idx];
        }
    }
    __syncthreads();
    const T dtT = T(dt);
    int cur = 0;
    for (int t = 1; t <= steps; ++t) {
        const int lx0 = t * cw, lx1 = ERX - t * ce, ly0 = t * cs, ly1 = ERY - t * cn;
        const T *b = buf[cur];
        T *o = buf[cur ^ 1];
        for (int e = threadIdx.x; e < RN; e += blockDim.x) {
            const int lx = e % ERX, ly = e / ERX;
            if (lx < lx0 || lx >= lx1 || ly < ly0 || ly >= ly1) continue;
            const int gx = gcoord(lx, gx0, nx), gy = gcoord(ly, gy0, ny);
            if (gx < 0 || gy < 0) continue;
            const bool ww = !per && gx == 0, we = !per && gx == nx - 1;
            const bool ws = !per && gy == 0, wn = !per && gy == ny - 1;
            const int ew = ww ? e : e - 1, ee = we ? e : e + 1, es = ws ? e : e - ERX, en = wn ? e : e + ERX;
            T c[NS], w[NS], ea[NS], s[NS], n[NS], k[NS];
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) {
                const T *bb = b + sp * RN;
                c[sp] = bb[e];
                w[sp] = bb[ew];
                ea[sp] = bb[ee];
                s[sp] = bb[es];
                n[sp] = bb[en];
            }
            rhs_cell<KIND, T>(g, c, w, ea, s, n, ww, we, ws, wn, k);
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) {
                const T u = c[sp], inc = dtT * k[sp];
                if constexpr (KAHAN) {
                    const T yk = inc - cm[sp * RN + e];
                    const T un = u + yk;
                    cm[sp * RN + e] = (un - u) - yk;
                    o[sp * RN + e] = un;
                } else {
                    o[sp * RN + e] = u + inc;
                }
            }
        }
        __syncthreads();
        cur ^= 1;
    }
    // the tile's own cells
    for (int e = threadIdx.x; e < EX * EY; e += blockDim.x) {
        const int lx = EH + e % EX, ly = EH + e / EX;
        const int gx = x0 + e % EX, gy = y0 + e / EX;
        if (gx >= nx || gy >= ny) continue;
        const int r = ly * ERX + lx;
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const int idx = sp * nc + gy * nx + gx;
            const T v = buf[cur][sp * RN + r];
            dst[idx] = v;
            if (dst2) dst2[idx] = v;
            if constexpr (KAHAN) cmp_out[idx] = cm[sp * RN + r];
        }
    }
    __syncthreads();  // the region buffers are reused by the next tile
}

// One classical RK4 step of one tile in a single pass, for the 5-point
// Laplacian systems (a cheap right-hand side: recomputing a halo costs less
// than a pass through memory per stage): the tile (64 x FY cells, NT
// threads) is loaded with an RH-cell halo (cut at walls, wrapped when
// periodic), stage s = 1..3 updates the region shrunk by s cells on every
// side that is not a wall, stage 4 the tile's own cells.  Lane l of
// wavefront v holds the tile cells (l, ROWN v .. ROWN v + ROWN - 1) and the
// halo cells t + NT r of the region in registers (state, stage input, slope
// sum and FP32 compensation of the tile cells), so a tile cell reads only
// its west and east neighbours and, at the ends of its column, one north or
// south neighbour from LDS; the stage inputs live in one LDS buffer,
// rewritten between two barriers.  Per cell the arithmetic is that of
// stage_tile<KIND, T, 1..4>.
constexpr int RH = 4, RRX = TT_X + 2 * RH;
template <int FY>
struct FusedTile {
    static constexpr int RRY = FY + 2 * RH, RRN = RRX * RRY;
    static constexpr int RSB = RRN + 2 * RRX;  // species stride: one padding row above and below
    static constexpr int RHALO = RRN - TT_X * FY;  // halo cells of the region
};

template <int FY>
__host__ __device__ inline int fused_tiles_of(const Geom &g)
{
    return tiles_x(g) * ((g.ny + FY - 1) / FY);
}

template <int FY>
__host__ __device__ inline size_t rk4_fused_lds(const Geom &g, size_t elem)
{
    return (size_t)g.ns * FusedTile<FY>::RSB * elem;
}

template <int KIND, typename T, int FY, int NT>
__device__ __forceinline__ void rk4_tile_fused(const Geom &g, const int tile, const double dt,
                                               const T *__restrict__ src, T *__restrict__ dst, T *__restrict__ cmp,
                                               const int cmp_zero, T *__restrict__ lds)
{
    static_assert(KIND == RPR_DIFFREACT2D || KIND == RPR_BRUSS2D, "5-point Laplacian systems only");
    constexpr int RRY = FusedTile<FY>::RRY, RRN = FusedTile<FY>::RRN, RSB = FusedTile<FY>::RSB;
    constexpr int RHALO = FusedTile<FY>::RHALO;
    constexpr int ROWN = FY / (NT / 64);                // tile cells per thread (a column of them)
    constexpr int RHPT = (RHALO + NT - 1) / NT;         // halo cells per thread
    static_assert(TT_X == 64 && ROWN * NT == TT_X * FY && RH < 8, "tile shape");
    constexpr int NS = kind_ns<KIND>();
    constexpr bool KAHAN = sizeof(T) == 4;
    const int nx = g.nx, ny = g.ny, nc = g.nc;
    constexpr bool per = kind_periodic<KIND>();
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int x0 = (tile % tiles_x(g)) * TT_X, y0 = (tile / tiles_x(g)) * FY;
    const int gx0 = x0 - RH, gy0 = y0 - RH;
    const int cw = per || gx0 > 0, ce = per || gx0 + RRX < nx;
    const int cs = per || gy0 > 0, cn = per || gy0 + RRY < ny;
    T *const yb = lds + RRX;  // species sp at yb + sp RSB, region cell e = ly RRX + lx
    auto gcoord = [&](int l, int o, int n) {  // region index -> domain index, or -1 beyond a wall
        const int v = o + l;
        if (per) return ((v % n) + n) % n;
        return (v < 0 || v >= n) ? -1 : v;
    };

    // tile cells: region index eo + q RRX, domain coordinates (gxo, gyo[q]),
    // < 0 beyond a wall; a tile cell past the end of a periodic domain is a
    // copy of a cell at its start: it takes part in stages 1 to 3 but is
    // not written (ownm)
    const int eo = (RH + wv * ROWN) * RRX + RH + lane;
    const int gxo = gcoord(RH + lane, gx0, nx);
    int gyo[ROWN], ownm = 0;
#pragma unroll
    for (int q = 0; q < ROWN; ++q) {
        const int ly = RH + wv * ROWN + q;
        gyo[q] = gcoord(ly, gy0, ny);
        if (x0 + lane < nx && y0 + ly - RH < ny) ownm |= 1 << q;
    }
    auto valid_o = [&](int q) { return gxo >= 0 && gyo[q] >= 0; };
    // halo cells: region index, domain coordinates, stages they take part in (dh)
    int eh[RHPT], gxh[RHPT], gyh[RHPT], dh[RHPT];
#pragma unroll
    for (int r = 0; r < RHPT; ++r) {
        const int h = t + NT * r;
        int lx, ly;
        if (h < 2 * RH * RRX) {  // RH full rows below and above the tile
            const int br = h / RRX;
            lx = h - br * RRX;
            ly = br < RH ? br : br + FY;
        } else {  // RH columns left and right of the tile
            const int m = h - 2 * RH * RRX, c = m % (2 * RH);
            ly = RH + m / (2 * RH);
            lx = c < RH ? c : c + TT_X;
        }
        const bool in = h < RHALO;
        eh[r] = in ? ly * RRX + lx : 0;
        const int gx = gcoord(lx, gx0, nx), gy = gcoord(ly, gy0, ny);
        gxh[r] = gx;
        gyh[r] = gy;
        int dep = 3;
        if (cw) dep = min(dep, lx);
        if (ce) dep = min(dep, RRX - 1 - lx);
        if (cs) dep = min(dep, ly);
        if (cn) dep = min(dep, RRY - 1 - ly);
        dh[r] = (in && gx >= 0 && gy >= 0) ? dep : -1;
    }

    // state (and compensation) of the cells; every load is issued before the first use
    T uo[ROWN][NS], uh[RHPT][NS], cm[ROWN][NS];
#pragma unroll
    for (int q = 0; q < ROWN; ++q)
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const int idx = valid_o(q) ? sp * nc + gyo[q] * nx + gxo : 0;
            uo[q][sp] = src[idx];
            if constexpr (KAHAN) cm[q][sp] = cmp[idx];
        }
#pragma unroll
    for (int r = 0; r < RHPT; ++r)
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const int idx = dh[r] >= 0 ? sp * nc + gyh[r] * nx + gxh[r] : 0;
            uh[r][sp] = src[idx];
        }
#pragma unroll
    for (int q = 0; q < ROWN; ++q)
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            if (valid_o(q)) yb[sp * RSB + eo + q * RRX] = uo[q][sp];
            if constexpr (KAHAN) cm[q][sp] = cmp_zero ? T(0) : cm[q][sp];
        }
#pragma unroll
    for (int r = 0; r < RHPT; ++r)
#pragma unroll
        for (int sp = 0; sp < NS; ++sp)
            if (dh[r] >= 0) yb[sp * RSB + eh[r]] = uh[r][sp];
    __syncthreads();

    const T dtT = T(dt), hdt = T(0.5 * dt), dt6 = T(dt / 6.0);
    // right-hand side of a cell from its stage input c and neighbours; a
    // cell at a wall takes itself as the missing neighbour
    auto slope = [&](const int gx, const int gy, const T *c, const T *wr, const T *er, const T *sr, const T *nr,
                     T *k) {
        const bool ww = !per && gx == 0, we = !per && gx == nx - 1;
        const bool ws = !per && gy == 0, wn = !per && gy == ny - 1;
        T w[NS], ea[NS], sv[NS], nv[NS];
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            w[sp] = ww ? c[sp] : wr[sp];
            ea[sp] = we ? c[sp] : er[sp];
            sv[sp] = ws ? c[sp] : sr[sp];
            nv[sp] = wn ? c[sp] : nr[sp];
        }
        rhs_cell<KIND, T>(g, c, w, ea, sv, nv, ww, we, ws, wn, k);
    };
    // tile cell q from the stage inputs yc of this thread's column
    auto slope_o = [&](const int q, const T (*yc)[NS], T *k) {
        T wr[NS], er[NS], sr[NS], nr[NS];
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const T *bb = yb + sp * RSB + eo + q * RRX;
            wr[sp] = bb[-1];
            er[sp] = bb[1];
            sr[sp] = q > 0 ? yc[q > 0 ? q - 1 : 0][sp] : bb[-RRX];
            nr[sp] = q < ROWN - 1 ? yc[q < ROWN - 1 ? q + 1 : 0][sp] : bb[RRX];
        }
        slope(gxo, gyo[q], yc[q], wr, er, sr, nr, k);
    };
    // halo cell r from LDS
    auto slope_h = [&](const int r, T *k) {
        T c[NS], wr[NS], er[NS], sr[NS], nr[NS];
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const T *bb = yb + sp * RSB + eh[r];
            c[sp] = bb[0];
            wr[sp] = bb[-1];
            er[sp] = bb[1];
            sr[sp] = bb[-RRX];
            nr[sp] = bb[RRX];
        }
        slope(gxh[r], gyh[r], c, wr, er, sr, nr, k);
    };

    T acc[ROWN][NS], yc[ROWN][NS];  // yc: stage input of the tile cells
#pragma unroll
    for (int q = 0; q < ROWN; ++q)
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            yc[q][sp] = uo[q][sp];
            acc[q][sp] = T(0);
        }
#pragma unroll
    for (int st = 1; st <= 3; ++st) {
        const T cst = st == 3 ? dtT : hdt;
        T yn[ROWN][NS], yh[RHPT][NS];
#pragma unroll
        for (int q = 0; q < ROWN; ++q) {
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) yn[q][sp] = yc[q][sp];
            if (!valid_o(q)) continue;
            T k[NS];
            slope_o(q, yc, k);
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) {
                acc[q][sp] = st == 1 ? k[sp] : acc[q][sp] + T(2) * k[sp];
                yn[q][sp] = uo[q][sp] + cst * k[sp];
            }
        }
#pragma unroll
        for (int r = 0; r < RHPT; ++r) {
            if (dh[r] < st) continue;
            T k[NS];
            slope_h(r, k);
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) yh[r][sp] = uh[r][sp] + cst * k[sp];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < ROWN; ++q) {
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) {
                if (valid_o(q)) yb[sp * RSB + eo + q * RRX] = yn[q][sp];
                yc[q][sp] = yn[q][sp];
            }
        }
#pragma unroll
        for (int r = 0; r < RHPT; ++r)
            if (dh[r] >= st)
#pragma unroll
                for (int sp = 0; sp < NS; ++sp) yb[sp * RSB + eh[r]] = yh[r][sp];
        __syncthreads();
    }
    // stage 4 on the tile's cells
#pragma unroll
    for (int q = 0; q < ROWN; ++q) {
        if (!((ownm >> q) & 1)) continue;
        T k[NS];
        slope_o(q, yc, k);
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const int idx = sp * nc + gyo[q] * nx + gxo;
            const T inc = dt6 * (acc[q][sp] + k[sp]);
            if constexpr (KAHAN) {
                const T yk = inc - cm[q][sp];
                const T un = uo[q][sp] + yk;
                cmp[idx] = (un - uo[q][sp]) - yk;
                dst[idx] = un;
            } else {
                dst[idx] = uo[q][sp] + inc;
            }
        }
    }
}

// stage_tile with the stage chosen at run time.
template <int KIND, typename T>
__device__ __forceinline__ void stage_tile_any(const Geom &g, const int tile, const int stage, const double dt,
                                               const StageIO<T> &io, T *__restrict__ lds)
{
    switch (stage) {
        case 0: stage_tile<KIND, T, 0>(g, tile, dt, io, lds); break;
        case 1: stage_tile<KIND, T, 1>(g, tile, dt, io, lds); break;
        case 2: stage_tile<KIND, T, 2>(g, tile, dt, io, lds); break;
        case 3: stage_tile<KIND, T, 3>(g, tile, dt, io, lds); break;
        default: stage_tile<KIND, T, 4>(g, tile, dt, io, lds); break;
    }
}

// The arrays of stage `stage` (0 Euler, 1..4 RK4) of step `step` of a
// propagation src -> dst (and dst2 if not null) that takes `steps` steps, on
// work arrays w.  RK4 keeps the state in w.u (src on the first step, dst
// after the last); Euler alternates between w.u and w.ya.
template <typename T>
__host__ __device__ inline StageIO<T> stage_io(int method, int stage, long long step, long long steps,
                                               const T *src, T *dst, T *dst2, const TiledWork<T> &w)
{
    StageIO<T> io{};
    const bool first = step == 0, last = step == steps - 1;
    io.u_out2 = last ? dst2 : nullptr;
    io.cmp = w.cmp;
    io.cmp_zero = first ? 1 : 0;
    if (method == RPR_RK4) {
        const T *u = first ? src : w.u;
        io.u = u;
        if (stage == 1) {
            io.y = u;
            io.acc = w.acc;
            io.y_out = w.yb;
        } else if (stage == 2) {
            io.y = w.yb;
            io.acc = w.acc;
            io.y_out = w.ya;
        } else if (stage == 3) {
            io.y = w.ya;
            io.acc = w.acc;
            io.y_out = w.yb;
        } else {
            io.y = w.yb;
            io.acc = w.acc;
            io.u_out = last ? dst : w.u;
        }
    } else {
        T *buf[2] = {w.u, w.ya};
        const T *u = first ? src : buf[step % 2];
        io.y = u;
        io.u = u;
        io.u_out = last ? dst : buf[(step + 1) % 2];
    }
    return io;
}

}  // namespace rpr
