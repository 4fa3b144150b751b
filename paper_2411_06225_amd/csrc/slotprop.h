// slotprop.h -- propagation of one slot state by one work-group, on chip.
//
// Sec. 2: F and G map the state at the start of a slice to its end; both are
// fixed-step explicit Runge-Kutta methods (RK1 or classical RK4).
//
// Work decomposition.  Thread t owns a strip of CPT consecutive cells: in 1D
// cells t*CPT .. t*CPT+CPT-1; in 2D column x = t % nx, rows
// (t / nx)*CPT .. +CPT-1.  The strip's state u, the RK4 accumulator and the
// current stage input y stay in registers for the whole slice.  Neighbours
// inside the strip are read from registers; the others from an LDS copy of
// the stage input.  The LDS copy is padded with one ghost layer on every side
// (the boundary rule is applied when a boundary cell publishes its value into
// the ghost that mirrors or wraps it), so every neighbour sits at a fixed
// offset from its cell and the stencil needs no boundary branches.  With two
// LDS buffers the next stage input is written into the idle buffer while the
// current one is read, so each stage costs one barrier: a buffer is rewritten
// two stages later, after every thread has passed the barrier that follows its
// last read of it.  HBM is touched once to load the slot and once to store it.
#pragma once

#include "common.h"

namespace rpr {

// Value of the same register in the lane one to the west (WEST) or east of
// this one, across the whole wavefront (DPP wavefront shift / rotate by one
// lane: wave_shr / wave_ror give lane i the value of lane i-1, wave_shl /
// wave_rol that of lane i+1).  With ROT the row wraps around; without it the
// lane at the row end reads 0 (bound control), and the caller accounts for
// the wall in the centre weight instead.
template <bool WEST, bool ROT, typename T>
__device__ __forceinline__ T lane_neighbour(T v)
{
    constexpr int CTRL = WEST ? (ROT ? 0x13C : 0x138) : (ROT ? 0x134 : 0x130);
    if constexpr (sizeof(T) == 8) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        const int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
        const int rlo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, true);
        const int rhi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, true);
        return __longlong_as_double((long long)(((unsigned long long)(unsigned)rhi << 32) | (unsigned)rlo));
    } else {
        const int b = __float_as_int(v);
        return __int_as_float(__builtin_amdgcn_update_dpp(0, b, CTRL, 0xf, 0xf, true));
    }
}

// Elements of one padded LDS stage buffer.
__host__ __device__ inline int padded_elems(const Geom &g)
{
    return g.kind == RPR_BURGERS1D ? g.nc + 2 : g.ns * (g.nx + 2) * (g.ny + 2);
}

// FULL: every thread of the work-group owns a complete strip (the host picks
// it when the strip length divides the grid), which makes all per-cell
// validity tests compile-time constants.  NX, NY: grid extents fixed at compile
// time (0 = taken from g); fixed extents turn every neighbour address into an
// immediate offset from one base register per buffer.
template <int KIND, typename T, int CPT, bool DBUF, bool FULL, int NX = 0, int NY = 0>
__device__ __forceinline__ void slot_propagate(const Geom &g, int method, long long steps, double dt_d,
                                               const T *__restrict__ src, T *__restrict__ dst,
                                               T *__restrict__ lds, T *__restrict__ dst2 = nullptr)
{
    constexpr int NS = kind_ns<KIND>();
    constexpr bool ONE_D = KIND == RPR_BURGERS1D;
    // a grid row of 64 cells is exactly one wavefront: east / west neighbours
    // come from the adjacent lanes, and only the first and last row of each
    // strip go through LDS (for the strips above and below)
    constexpr bool XLANE = !ONE_D && NX == 64 && FULL && KIND != RPR_SWE2D;
    constexpr bool XROT = KIND == RPR_BRUSS2D;  // periodic in x
    const int t = threadIdx.x;
    const int nx = NX ? NX : g.nx, ny = NY ? NY : g.ny;
    const int nc = (NX && NY) ? NX * NY : g.nc;
    const bool per = g.periodic != 0;
    const T dt = T(dt_d), hdt = T(0.5 * dt_d), dt6 = T(dt_d / 6.0);

    // padded layout: 2D element (sp, y, x) at sp*PQ + (y+1)*P + (x+1); 1D at cell+1
    const int P = ONE_D ? 1 : nx + 2;
    const int PQ = ONE_D ? nc + 2 : P * (ny + 2);
    T *const buf0 = lds;
    T *const buf1 = DBUF ? lds + (ONE_D ? PQ : NS * PQ) : lds;

    // strip geometry: first cell in global and padded indexing, valid cells
    int x = 0, row0 = 0, cell0, gstride, pbase0, pstride, nvalid;
    if constexpr (ONE_D) {
        cell0 = t * CPT;
        gstride = 1;
        pbase0 = cell0 + 1;
        pstride = 1;
        nvalid = nc - cell0;
    } else {
        x = t % nx;
        row0 = (t / nx) * CPT;
        cell0 = row0 * nx + x;
        gstride = nx;
        pbase0 = (row0 + 1) * P + x + 1;
        pstride = P;
        nvalid = (t < nx * ((ny + CPT - 1) / CPT)) ? ny - row0 : 0;
    }
    nvalid = nvalid < 0 ? 0 : (nvalid > CPT ? CPT : nvalid);
    const int nv = FULL ? CPT : nvalid;

    // Ghost copies this thread writes besides its own cells, as offsets from
    // the padded index of the writing cell.  The west ghost of a row holds the
    // west neighbour of its first cell: the last cell when periodic, the cell
    // itself at a wall; likewise east, south and north.
    const int rowL = row0 + nv - 1;
    bool wall_w = false, wall_e = false, wall_s = false, wall_n = false;
    bool gx0 = false, gx1 = false, gfirst = false, glast = false;
    int ox0 = 0, ox1 = 0, ofirst = 0, olast = 0;
    if constexpr (ONE_D) {
        // the strip's first cell is cell0, its last cellL = cell0 + nv - 1
        if (cell0 == 0) { gfirst = true; ofirst = per ? nc : -1; }
        if (cell0 + nv - 1 == nc - 1) { glast = true; olast = per ? -nc : 1; }
    } else {
        wall_w = !per && x == 0;
        wall_e = !per && x == nx - 1;
        wall_s = !per && row0 == 0;
        wall_n = !per && rowL == ny - 1;
        if (per) {
            if (x == nx - 1) { gx0 = true; ox0 = -nx; }   // into the west ghost
            if (x == 0) { gx1 = true; ox1 = nx; }         // into the east ghost
            if (row0 == 0) { gfirst = true; ofirst = ny * P; }      // into the north ghost row
            if (rowL == ny - 1) { glast = true; olast = -ny * P; }  // into the south ghost row
        } else {
            if (x == 0) { gx0 = true; ox0 = -1; }
            if (x == nx - 1) { gx1 = true; ox1 = 1; }
            if (row0 == 0) { gfirst = true; ofirst = -P; }
            if (rowL == ny - 1) { glast = true; olast = P; }
        }
    }

    // In single precision the state update u += dt * (...) is compensated
    // (Kahan summation): the increments are ~1e-4 of the state, so plain
    // FP32 adds would lose their low bits every step.  cmp holds the running
    // compensation.  Double precision uses the plain update.
    constexpr bool KAHAN = sizeof(T) == 4;
    T u[CPT][NS], acc[CPT][NS], y[CPT][NS], cmp[KAHAN ? CPT : 1][NS];
    auto publish = [&](T *buf, const int c) {
        const int pi = pbase0 + c * pstride;
        // in 1D, and with lane neighbours in x, only the strip ends are read
        // by other threads
        if ((ONE_D || XLANE) && !(c == 0 || c == nv - 1)) return;
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            T *o = buf + sp * PQ + pi;
            o[0] = y[c][sp];
            if (!XLANE && gx0) o[ox0] = y[c][sp];
            if (!XLANE && gx1) o[ox1] = y[c][sp];
            if (c == 0 && gfirst) o[ofirst] = y[c][sp];
            if (c == nv - 1 && glast) o[olast] = y[c][sp];
        }
    };

#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        if (c < nv) {
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) {
                u[c][sp] = src[sp * nc + cell0 + c * gstride];
                acc[c][sp] = T(0);
                y[c][sp] = u[c][sp];
                if constexpr (KAHAN) cmp[c][sp] = T(0);
            }
            publish(buf0, c);
        }
    }

    // weight of the centre cell in the x part of the Laplacian when the x
    // neighbours come from lanes: -2, or -1 beside a zero-flux wall, whose
    // mirror ghost (the cell itself) the lane exchange leaves out
    const T mx = XROT ? T(-2) : T(-2) + T(x == 0 ? 1 : 0) + T(x == nx - 1 ? 1 : 0);
    int cur = 0;
    // which: 1..3 RK4 stages producing k1..k3, 4 the last RK4 stage, 0 Euler
    auto stage = [&](const int which) {
        __syncthreads();
        const T *rb = (DBUF && cur) ? buf1 : buf0;
        T *wb = DBUF ? (cur ? buf0 : buf1) : buf0;
        T prev[NS];  // stage input of the previous strip cell (its south / west neighbour)
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            if (c < nv) {
                const int pi = pbase0 + c * pstride;
                T w[NS], e[NS], s[NS], n[NS];
#pragma unroll
                for (int sp = 0; sp < NS; ++sp) {
                    const T *r = rb + sp * PQ + pi;
                    if constexpr (ONE_D) {
                        w[sp] = c == 0 ? r[-1] : prev[sp];
                        e[sp] = c + 1 < nv ? y[c + 1][sp] : r[1];
                    } else {
                        if constexpr (XLANE) {
                            // w holds the sum of both x neighbours (a wall's mirror ghost left out)
                            w[sp] = lane_neighbour<true, XROT>(y[c][sp]) + lane_neighbour<false, XROT>(y[c][sp]);
                        } else {
                            w[sp] = r[-1];
                            e[sp] = r[1];
                        }
                        s[sp] = c == 0 ? r[-P] : prev[sp];
                        n[sp] = c + 1 < nv ? y[c + 1][sp] : r[P];
                    }
                }
                T k[NS];
                if constexpr (XLANE)
                    rhs_cell_xsum<KIND, T>(g, y[c], w, mx, s, n, k);
                else
                    rhs_cell<KIND, T>(g, y[c], w, e, s, n, wall_w, wall_e, c == 0 && wall_s,
                                      c == nv - 1 && wall_n, k);
#pragma unroll
                for (int sp = 0; sp < NS; ++sp) {
                    prev[sp] = y[c][sp];
                    T nxt;
                    if (which == 1) {
                        acc[c][sp] = k[sp];
                        nxt = u[c][sp] + hdt * k[sp];
                    } else if (which == 2) {
                        acc[c][sp] = acc[c][sp] + T(2) * k[sp];
                        nxt = u[c][sp] + hdt * k[sp];
                    } else if (which == 3) {
                        acc[c][sp] = acc[c][sp] + T(2) * k[sp];
                        nxt = u[c][sp] + dt * k[sp];
                    } else {
                        const T inc = which == 4 ? dt6 * (acc[c][sp] + k[sp]) : dt * k[sp];
                        if constexpr (KAHAN) {
                            const T yk = inc - cmp[c][sp];
                            const T un = u[c][sp] + yk;
                            cmp[c][sp] = (un - u[c][sp]) - yk;
                            u[c][sp] = un;
                        } else {
                            u[c][sp] = u[c][sp] + inc;
                        }
                        nxt = u[c][sp];
                    }
                    y[c][sp] = nxt;
                }
                if constexpr (DBUF) publish(wb, c);
            }
        }
        if constexpr (!DBUF) {
            __syncthreads();
#pragma unroll
            for (int c = 0; c < CPT; ++c)
                if (c < nv) publish(wb, c);
        }
        cur ^= 1;
    };

    if (method == RPR_RK4) {
        for (long long st = 0; st < steps; ++st) {
            stage(1);
            stage(2);
            stage(3);
            stage(4);
        }
    } else {
        for (long long st = 0; st < steps; ++st) stage(0);
    }

#pragma unroll
    for (int c = 0; c < CPT; ++c)
        if (c < nv) {
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) {
                dst[sp * nc + cell0 + c * gstride] = u[c][sp];
                if (dst2) dst2[sp * nc + cell0 + c * gstride] = u[c][sp];
            }
        }
}

}  // namespace rpr

namespace rpr {

// Calls f.template run<CPT, DBUF, FULL, NX, NY, MAXT>() for the kernel
// instance of right-hand side KIND that serves geometry g with shape sh: the
// workloads' grids have compile-time extents and complete strips, every other
// grid takes the generic instance with per-thread strip lengths.
template <int KIND, typename T, typename Fn>
rpr_status visit_shape_kind(const Geom &g, const OnchipShape &sh, Fn &f)
{
    constexpr bool F64 = sizeof(T) == 8;
    auto is = [&](int nx, int ny, int cpt, int dbuf, int maxt) {
        return g.nx == nx && g.ny == ny && sh.cpt == cpt && sh.dbuf == dbuf && sh.full && sh.maxt == maxt;
    };
    if constexpr (KIND == RPR_DIFFREACT2D || KIND == RPR_BRUSS2D) {
        if (is(64, 64, 4, 1, 1024)) return f.template run<4, true, true, 64, 64, 1024>();
        if (is(64, 64, 8, 1, 512)) return f.template run<8, true, true, 64, 64, 512>();
    }
    if constexpr (KIND == RPR_BRUSS2D && !F64) {
        if (is(128, 128, 16, 0, 1024)) return f.template run<16, false, true, 128, 128, 1024>();
    }
    if (sh.maxt != 1024) return fail(RPR_ERR_UNSUPPORTED, "512-thread shape only for fixed grids");
#define RPR_GENERIC_CPT(DB)                                                                        \
    switch (sh.cpt) {                                                                              \
    case 1: return f.template run<1, DB, false, 0, 0, 1024>();                                     \
    case 2: return f.template run<2, DB, false, 0, 0, 1024>();                                     \
    case 4: return f.template run<4, DB, false, 0, 0, 1024>();                                     \
    case 8: return f.template run<8, DB, false, 0, 0, 1024>();                                     \
    case 16: return f.template run<16, DB, false, 0, 0, 1024>();                                   \
    default: return fail(RPR_ERR_UNSUPPORTED, "no kernel instance for this strip length");        \
    }
    if (sh.dbuf) {
        RPR_GENERIC_CPT(true)
    } else {
        RPR_GENERIC_CPT(false)
    }
#undef RPR_GENERIC_CPT
}

}  // namespace rpr
