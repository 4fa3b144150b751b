// tiledprop.h -- propagation of slot states too large for one work-group.
//
// Sec. 2: F and G are fixed-step explicit Runge-Kutta methods.  When a 2D
// slot state does not fit one compute unit, every RK stage becomes a pass
// over 64 x 16-cell tiles of the state in memory: a work-group of 256
// threads copies the tile of the stage input with a one-cell halo into LDS
// (the boundary rule applied while copying: wrap when periodic, the cell
// itself at a wall), evaluates the right-hand side of its cells (4 rows per
// thread) and applies the stage update to the RK arrays in memory.  The
// update formulas, their order and the FP32 compensation are those of the
// on-chip propagator, so both agree to rounding.
#pragma once

#include "common.h"

namespace rpr {

constexpr int TT_X = 64, TT_Y = 16, TT_THREADS = 256;
constexpr int TT_RPT = TT_X * TT_Y / TT_THREADS;  // rows per thread

__host__ __device__ inline int tiles_x(const Geom &g) { return (g.nx + TT_X - 1) / TT_X; }
__host__ __device__ inline int tiles_of(const Geom &g) { return tiles_x(g) * ((g.ny + TT_Y - 1) / TT_Y); }

// LDS of one haloed tile.
__host__ __device__ inline size_t tiled_lds(const Geom &g, size_t elem)
{
    return (size_t)g.ns * (TT_Y + 2) * (TT_X + 2) * elem;
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

template <int KIND, typename T>
__device__ __forceinline__ void stage_tile(const Geom &g, const int tile, const int stage, const double dt,
                                           const StageIO<T> &io, T *__restrict__ lds)
{
    constexpr int NS = kind_ns<KIND>();
    constexpr int PX = TT_X + 2, PY = TT_Y + 2;
    constexpr bool KAHAN = sizeof(T) == 4;
    const int nx = g.nx, ny = g.ny, nc = g.nc;
    const bool per = g.periodic != 0;
    const int x0 = (tile % tiles_x(g)) * TT_X, y0 = (tile / tiles_x(g)) * TT_Y;
    const int t = threadIdx.x;

    for (int e = t; e < NS * PY * PX; e += blockDim.x) {
        const int sp = e / (PY * PX), r = e % (PY * PX), ly = r / PX, lx = r % PX;
        int gx = x0 + lx - 1, gy = y0 + ly - 1;
        if (per) {
            gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
            gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
        } else {
            gx = gx < 0 ? 0 : (gx >= nx ? nx - 1 : gx);
            gy = gy < 0 ? 0 : (gy >= ny ? ny - 1 : gy);
        }
        lds[e] = io.y[sp * nc + gy * nx + gx];
    }
    __syncthreads();

    const T dtT = T(dt), hdt = T(0.5 * dt), dt6 = T(dt / 6.0);
    const int cx = t % TT_X, cy0 = (t / TT_X) * TT_RPT;
    const int gx = x0 + cx;
#pragma unroll
    for (int q = 0; q < TT_RPT; ++q) {
        const int gy = y0 + cy0 + q;
        if (t < TT_THREADS && gx < nx && gy < ny) {
            const int lx = cx + 1, ly = cy0 + q + 1;
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
            for (int sp = 0; sp < NS; ++sp) {
                const size_t idx = (size_t)sp * nc + (size_t)gy * nx + gx;
                if (stage == 1) {
                    io.acc[idx] = k[sp];
                    io.y_out[idx] = io.u[idx] + hdt * k[sp];
                } else if (stage == 2) {
                    io.acc[idx] = io.acc[idx] + T(2) * k[sp];
                    io.y_out[idx] = io.u[idx] + hdt * k[sp];
                } else if (stage == 3) {
                    io.acc[idx] = io.acc[idx] + T(2) * k[sp];
                    io.y_out[idx] = io.u[idx] + dtT * k[sp];
                } else {
                    const T inc = stage == 4 ? dt6 * (io.acc[idx] + k[sp]) : dtT * k[sp];
                    const T u = io.u[idx];
                    if constexpr (KAHAN) {
                        const T cm = io.cmp_zero ? T(0) : io.cmp[idx];
                        const T yk = inc - cm;
                        const T un = u + yk;
                        io.cmp[idx] = (un - u) - yk;
                        io.u_out[idx] = un;
                        if (io.u_out2) io.u_out2[idx] = un;
                    } else {
                        io.u_out[idx] = u + inc;
                        if (io.u_out2) io.u_out2[idx] = u + inc;
                    }
                }
            }
        }
    }
    __syncthreads();  // the tile buffer is reused by the next tile
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
