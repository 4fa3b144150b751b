// swefused.h -- one classical RK4 step of shallow-water slot states in a
// single pass over each tile (Sec. 5.3 system: first-order finite volumes,
// Rusanov flux, reflective walls).
//
// Layout.  A wavefront holds a region row of 64 cells in its 64 lanes (lane l
// = column x0 - 4 + l) and R consecutive rows in registers; NW wavefronts
// stack to a region of 64 x RY cells, RY = NW R.  The region is the tile (56
// columns, RY - 8 rows) with a 4-cell halo, one cell per RK stage: stage s
// produces valid values on the region shrunk by s cells, so after stage 4
// the tile's own cells are exact.
//
// Walls.  Beyond a wall the halo holds the mirror image of the cells inside
// it (h and the tangential momentum even, the normal momentum odd).  The
// Rusanov flux and the finite-volume update map mirrored inputs to mirrored
// results operation by operation (every operation used is odd or even under
// the reflection, rounding included), so a ghost cell evolves as the mirror
// of its partner and the face at the wall sees exactly the mirrored ghost
// that the per-cell form builds from the wall cell itself.  No wall branch
// is needed inside the stages.
//
// Neighbours.  x: the lane to the east by a DPP rotation of the wavefront
// (one instruction per value); each x face flux is computed once, by the
// lane west of it, and rotated to the lane east of it.  y: registers within
// a wavefront's R rows; the rows next to another wavefront's come through
// LDS (6 values per cell of the first and last row, double-buffered by stage
// so that one barrier per stage suffices).
//
// Traffic per RK4 step and degree of freedom: read u, write u (and read and
// write the FP32 compensation), plus the halo re-reads that L2 serves.
#pragma once

#include "common.h"
#include "slotprop.h"

namespace rpr {

constexpr int SWF_HALO = 4;                    // one cell per RK stage
constexpr int SWF_X = 64 - 2 * SWF_HALO;       // tile columns (56)

template <int R, int NW>
struct SweFused {
    static constexpr int RY = R * NW;          // region rows
    static constexpr int TY = RY - 2 * SWF_HALO;  // tile rows
    static constexpr int NT = 64 * NW;         // threads
};

__host__ __device__ inline int swf_tiles_x(const Geom &g) { return (g.nx + SWF_X - 1) / SWF_X; }
template <int R, int NW>
__host__ __device__ inline int swf_tiles_of(const Geom &g)
{
    return swf_tiles_x(g) * ((g.ny + SweFused<R, NW>::TY - 1) / SweFused<R, NW>::TY);
}
// LDS: two stage buffers x NW wavefronts x 2 edge rows x 6 values x 64 lanes
template <int R, int NW>
__host__ __device__ inline size_t swf_lds(size_t elem)
{
    return (size_t)2 * NW * 2 * 6 * 64 * elem;
}

// Domain index of region coordinate v (cells -4 .. n+3 around a wall-bounded
// axis of n cells): the cell itself, or its mirror partner beyond a wall
// (flip set); positions further out are clamped (never used for a tile cell).
__device__ __forceinline__ int swf_mirror(int v, int n, bool &flip)
{
    flip = false;
    if (v < 0) {
        v = -1 - v;
        flip = true;
    } else if (v >= n) {
        v = 2 * n - 1 - v;
        flip = true;
    }
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

// 1/h and sqrt(v) of the per-cell quantities.  Single precision takes the
// hardware reciprocal and square root (about 1 ulp; the IEEE sequences
// cost several instructions each and would be a fifth of the step), double
// precision the IEEE operations.
template <typename T>
__device__ __forceinline__ T swf_rcp(T v)
{
    if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(v);
    else return T(1) / v;
}
template <typename T>
__device__ __forceinline__ T swf_sqrt(T v)
{
    if constexpr (sizeof(T) == 4) return __builtin_amdgcn_sqrtf(v);
    else return sqrt(v);
}

// The larger of two wave speeds.  Speeds are |velocity| + sqrt(g h) >= +0
// (or NaN), and for such values the IEEE order is the integer order of the
// bit patterns: single precision takes one integer max (fmax would first
// quiet operands that come from lane moves or LDS, one more instruction
// each); a NaN speed wins either way.
template <typename T>
__device__ __forceinline__ T swf_smax(T a, T b)
{
    if constexpr (sizeof(T) == 4) return __int_as_float(max(__float_as_int(a), __float_as_int(b)));
    else return fmax(a, b);
}

// Twice the Rusanov flux across one face between left state (h, m = normal
// momentum, q = tangential momentum, f = m^2/h + g h^2/2, e = q m/h,
// s = |m/h| + sqrt(g h)) and right state: (mass, normal, tangential)
// components of (f_L + f_R) - a (q_R - q_L).  The factor 1/2 of the flux is
// folded into the grid factors of the update: halving is exact, so the
// update equals the one with the halved flux bit for bit.
template <typename T>
__device__ __forceinline__ void swf_face(T hL, T mL, T qL, T fL, T eL, T sL, T hR, T mR, T qR, T fR, T eR, T sR,
                                         T &Fh, T &Fm, T &Fq)
{
    const T a = swf_smax(sL, sR);
    Fh = (mL + mR) - a * (hR - hL);
    Fm = (fL + fR) - a * (mR - mL);
    Fq = (eL + eR) - a * (qR - qL);
}

// One RK4 step of one tile: src -> dst, both full slot states (d values);
// cmp: the FP32 compensation of the own cells (read and written in place;
// cmp_zero: start from zero), null in FP64.
template <typename T, int R, int NW>
__device__ __forceinline__ void swe_rk4_tile(const Geom &g, const int tile, const double dt, const T *__restrict__ src,
                                             T *__restrict__ dst, T *__restrict__ cmp, const int cmp_zero,
                                             T *__restrict__ lds)
{
    using S = SweFused<R, NW>;
    constexpr int RY = S::RY, H = SWF_HALO;
    constexpr bool KAHAN = sizeof(T) == 4;
    const int nx = g.nx, ny = g.ny, nc = g.nc;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int tx = tile % swf_tiles_x(g), ty = tile / swf_tiles_x(g);
    const int x0 = tx * SWF_X, y0 = ty * S::TY;
    // the slope of a cell is -idx (dF + rho dG) with dF, dG its x and y
    // flux differences (twice the fluxes, swf_face: the 1/2 sits in idx),
    // rho = dy^-1 / dx^-1 (1 on square cells); the stages accumulate
    // s = dF + rho dG and take the factor -idx in their weights
    const T gg = T(g.p[0]), half = T(0.5), rho = T(g.idy / g.idx);
    const double nidx = -0.5 * g.idx;
    const T c_half = T(0.5 * dt * nidx), c_full = T(dt * nidx), c_sixth = T(dt / 6.0 * nidx);

    // ---- load: the region with mirror ghosts beyond the walls
    bool fx;
    const int gx = swf_mirror(x0 - H + lane, nx, fx);
    const bool own_x = lane >= H && lane < H + SWF_X && x0 - H + lane < nx;
    T u[R][3], y[R][3], acc[R][3], cm[R][3];
    int gyq[R];
    bool own[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = wv * R + q;
        bool fy;
        const int gy = swf_mirror(y0 - H + r, ny, fy);
        gyq[q] = gy;
        own[q] = own_x && r >= H && r < RY - H && y0 - H + r < ny;
        const int c = gy * nx + gx;
        const T h = src[c], m = src[nc + c], n = src[2 * nc + c];
        u[q][0] = h;
        u[q][1] = fx ? -m : m;
        u[q][2] = fy ? -n : n;
        if constexpr (KAHAN) {
            // only the tile's own cells take the compensated last stage
            const bool rd = own[q] && !cmp_zero;
            cm[q][0] = rd ? cmp[c] : T(0);
            cm[q][1] = rd ? cmp[nc + c] : T(0);
            cm[q][2] = rd ? cmp[2 * nc + c] : T(0);
        } else {
            cm[q][0] = cm[q][1] = cm[q][2] = T(0);
        }
#pragma unroll
        for (int sp = 0; sp < 3; ++sp) {
            y[q][sp] = u[q][sp];
            acc[q][sp] = T(0);
        }
    }

#pragma unroll
    for (int s = 1; s <= 4; ++s) {
        T *eb = lds + (size_t)(s & 1) * NW * 2 * 6 * 64;  // this stage's edge-row buffer
        // per-cell quantities (rows outside this stage's region hold
        // finite stale values: h stays positive, nothing divides by zero)
        T xf[R], xe[R], xs[R], yf[R], ye[R], ys[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const T h = y[q][0], m = y[q][1], n = y[q][2];
            const T rh = swf_rcp(h);
            const T vx = m * rh, vy = n * rh, c = swf_sqrt(gg * h), P = half * gg * h * h;
            const T e = n * vx;  // hu hv / h: the tangential flux term of both directions
            xf[q] = m * vx + P;
            xe[q] = e;
            xs[q] = fabs(vx) + c;
            yf[q] = n * vy + P;
            ye[q] = e;
            ys[q] = fabs(vy) + c;
        }
        // edge rows to LDS: [wave][row 0 | row R-1][h, m, n, yf, ye, ys][lane]
        {
            T *e0 = eb + (size_t)(wv * 2 + 0) * 6 * 64 + lane;
            T *e1 = eb + (size_t)(wv * 2 + 1) * 6 * 64 + lane;
            e0[0] = y[0][0];
            e0[64] = y[0][1];
            e0[128] = y[0][2];
            e0[192] = yf[0];
            e0[256] = ye[0];
            e0[320] = ys[0];
            e1[0] = y[R - 1][0];
            e1[64] = y[R - 1][1];
            e1[128] = y[R - 1][2];
            e1[192] = yf[R - 1];
            e1[256] = ye[R - 1];
            e1[320] = ys[R - 1];
        }
        __syncthreads();
        // y faces: face f lies below row f (f = 0 .. R); y face components
        // (mass, normal = hv, tangential = hu)
        T Gh[R + 1], Gv[R + 1], Gu[R + 1];
        {
            const int ws = wv > 0 ? wv - 1 : 0, wn = wv < NW - 1 ? wv + 1 : NW - 1;
            const T *es = eb + (size_t)(ws * 2 + 1) * 6 * 64 + lane;  // south neighbour wave's last row
            const T *en = eb + (size_t)(wn * 2 + 0) * 6 * 64 + lane;  // north neighbour wave's first row
            swf_face<T>(es[0], es[128], es[64], es[192], es[256], es[320], y[0][0], y[0][2], y[0][1], yf[0], ye[0],
                        ys[0], Gh[0], Gv[0], Gu[0]);
            swf_face<T>(y[R - 1][0], y[R - 1][2], y[R - 1][1], yf[R - 1], ye[R - 1], ys[R - 1], en[0], en[128],
                        en[64], en[192], en[256], en[320], Gh[R], Gv[R], Gu[R]);
        }
#pragma unroll
        for (int f = 1; f < R; ++f)
            swf_face<T>(y[f - 1][0], y[f - 1][2], y[f - 1][1], yf[f - 1], ye[f - 1], ys[f - 1], y[f][0], y[f][2],
                        y[f][1], yf[f], ye[f], ys[f], Gh[f], Gv[f], Gu[f]);

        // x faces: the east face of each cell with the east lane's values,
        // then the west face from the west lane; update
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = wv * R + q;
            if (!(r >= s && r < RY - s)) continue;  // wave-uniform: rows beyond this stage's region
            const T hE = lane_neighbour<false, true>(y[q][0]);
            const T mE = lane_neighbour<false, true>(y[q][1]);
            const T nE = lane_neighbour<false, true>(y[q][2]);
            const T fE = lane_neighbour<false, true>(xf[q]);
            const T eE = lane_neighbour<false, true>(xe[q]);
            const T sE = lane_neighbour<false, true>(xs[q]);
            T Fh, Fm, Fn;
            swf_face<T>(y[q][0], y[q][1], y[q][2], xf[q], xe[q], xs[q], hE, mE, nE, fE, eE, sE, Fh, Fm, Fn);
            const T dh = Fh - lane_neighbour<true, true>(Fh);
            const T dm = Fm - lane_neighbour<true, true>(Fm);
            const T dn = Fn - lane_neighbour<true, true>(Fn);
            T k[3];  // the slopes divided by -idx
            k[0] = fma(rho, Gh[q + 1] - Gh[q], dh);
            k[1] = fma(rho, Gu[q + 1] - Gu[q], dm);
            k[2] = fma(rho, Gv[q + 1] - Gv[q], dn);
#pragma unroll
            for (int sp = 0; sp < 3; ++sp) {
                if (s == 1) {
                    acc[q][sp] = k[sp];
                    y[q][sp] = fma(c_half, k[sp], u[q][sp]);
                } else if (s == 2) {
                    acc[q][sp] = fma(T(2), k[sp], acc[q][sp]);
                    y[q][sp] = fma(c_half, k[sp], u[q][sp]);
                } else if (s == 3) {
                    acc[q][sp] = fma(T(2), k[sp], acc[q][sp]);
                    y[q][sp] = fma(c_full, k[sp], u[q][sp]);
                } else {
                    const T inc = c_sixth * (acc[q][sp] + k[sp]);
                    if constexpr (KAHAN) {
                        const T yk = inc - cm[q][sp];
                        const T un = u[q][sp] + yk;
                        cm[q][sp] = (un - u[q][sp]) - yk;
                        u[q][sp] = un;
                    } else {
                        u[q][sp] = u[q][sp] + inc;
                    }
                }
            }
        }
    }

    // ---- the tile's own cells (never mirrored: a tile cell lies inside the domain)
#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (!own[q]) continue;
        const int c = gyq[q] * nx + gx;
#pragma unroll
        for (int sp = 0; sp < 3; ++sp) {
            dst[sp * nc + c] = u[q][sp];
            if constexpr (KAHAN) cmp[sp * nc + c] = cm[q][sp];
        }
    }
}


// ---------------------------------------------------------------------------
// Full-row form, for grids whose rows fit one wavefront: lane l holds the C
// consecutive cells C l .. C l + C - 1 of a row (nx <= 64 C, nx a multiple of
// C), so the region has no x halo and no x tiling; tiles run along y only,
// with the same 4-row halo and mirror ghost rows as above.  The faces on the
// x walls take the mirror state of the wall cell explicitly (normal momentum
// negated, so the mass and tangential fluxes vanish and the normal one is
// 2 f -+ 2 a m from the wall cell's f = m u + g h^2 / 2 and speed a).  Lanes past the
// last column read the row's last C cells (finite values) and feed no grid
// cell.  Against the 56-column tiles: no halo columns or padding lanes to
// recompute, and 9 lane moves per C cells instead of per cell; but C R
// cells per lane hold about 25 VGPRs each, so the tall tiles that keep the
// 8 halo rows cheap leave one work-group per CU (at 192 x 192 in FP32, C = 3
// and R = 2 on 12 wavefronts take 155 VGPRs and run 0.164 ms per step
// against 0.138 ms for 4 x 8 rows of 56-column tiles; in FP64 the two
// forms tie).  Both are candidates of the autotuner.
template <int C, int R, int NW>
struct SweRows {
    static constexpr int RY = R * NW;             // region rows
    static constexpr int TY = RY - 2 * SWF_HALO;  // tile rows
    static constexpr int NT = 64 * NW;            // threads
};

__host__ __device__ inline bool swr_fits(const Geom &g, int C)
{
    return g.nx <= 64 * C && g.nx % C == 0 && g.ny >= SWF_HALO;
}
template <int C, int R, int NW>
__host__ __device__ inline int swr_tiles_of(const Geom &g)
{
    return (g.ny + SweRows<C, R, NW>::TY - 1) / SweRows<C, R, NW>::TY;
}
// LDS: per wavefront its first row (6 values x 64 C cells) and the fluxes of
// the face above its last row (3 values x 64 C cells)
template <int C, int R, int NW>
__host__ __device__ inline size_t swr_lds(size_t elem)
{
    return (size_t)NW * 9 * 64 * C * elem;
}

template <typename T, int C, int R, int NW>
__device__ __forceinline__ void swe_rk4_rows(const Geom &g, const int tile, const double dt, const T *__restrict__ src,
                                             T *__restrict__ dst, T *__restrict__ cmp, const int cmp_zero,
                                             T *__restrict__ lds)
{
    using S = SweRows<C, R, NW>;
    constexpr int RY = S::RY, H = SWF_HALO, W = 64 * C;  // W: cells per region row
    constexpr bool KAHAN = sizeof(T) == 4;
    const int nx = g.nx, ny = g.ny, nc = g.nc;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int y0 = tile * S::TY;
    const T gg = T(g.p[0]), half = T(0.5), rho = T(g.idy / g.idx);
    const double nidx = -0.5 * g.idx;
    const T c_half = T(0.5 * dt * nidx), c_full = T(dt * nidx), c_sixth = T(dt / 6.0 * nidx);

    // lane's first column (lanes past the grid re-read the last C columns)
    const bool lane_in = lane * C < nx;
    const int xb = lane_in ? lane * C : nx - C;
    const bool wall_w = lane == 0, wall_e = lane == nx / C - 1;

    T u[R][C][3], y[R][C][3], acc[R][C][3], cm[R][C][3];
    int rowc[R];
    bool own[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = wv * R + q;
        bool fy;
        const int gy = swf_mirror(y0 - H + r, ny, fy);
        rowc[q] = gy * nx + xb;
        own[q] = lane_in && r >= H && r < RY - H && y0 - H + r < ny;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int c = rowc[q] + j;
            const T h = src[c], m = src[nc + c], n = src[2 * nc + c];
            u[q][j][0] = h;
            u[q][j][1] = m;
            u[q][j][2] = fy ? -n : n;
#pragma unroll
            for (int sp = 0; sp < 3; ++sp) {
                y[q][j][sp] = u[q][j][sp];
                acc[q][j][sp] = T(0);
            }
        }
    }

#pragma unroll
    for (int s = 1; s <= 4; ++s) {
        if (s == 4) {
            // the compensation of the own cells, needed by the last stage
            // only (loaded here to keep it out of the registers of the
            // first three; the addresses are valid for every lane: load,
            // then keep the tile's own cells)
#pragma unroll
            for (int q = 0; q < R; ++q) {
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    if constexpr (KAHAN) {
                        const int c = rowc[q] + j;
                        const bool rd = own[q] && !cmp_zero;
                        const T c0 = cmp[c], c1 = cmp[nc + c], c2 = cmp[2 * nc + c];
                        cm[q][j][0] = rd ? c0 : T(0);
                        cm[q][j][1] = rd ? c1 : T(0);
                        cm[q][j][2] = rd ? c2 : T(0);
                    } else {
                        cm[q][j][0] = cm[q][j][1] = cm[q][j][2] = T(0);
                    }
                }
            }
        }
        T xf[R][C], xe[R][C], xs[R][C], yf[R][C], ye[R][C], ys[R][C];
#pragma unroll
        for (int q = 0; q < R; ++q) {
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const T h = y[q][j][0], m = y[q][j][1], n = y[q][j][2];
                const T rh = swf_rcp(h);
                const T vx = m * rh, vy = n * rh, c = swf_sqrt(gg * h), P = half * gg * h * h;
                const T e = n * vx;
                xf[q][j] = m * vx + P;
                xe[q][j] = e;
                xs[q][j] = fabs(vx) + c;
                yf[q][j] = n * vy + P;
                ye[q][j] = e;
                ys[q][j] = fabs(vy) + c;
            }
        }
        // The faces between two wavefronts' rows are computed once, by the
        // wavefront below: it reads the first row of the one above (LDS block
        // A: [wave][h, m, n, yf, ye, ys][cell j][lane]) and hands the face's
        // fluxes back (block B: [wave][mass, normal, tangential][cell j][lane]).
        // Two barriers per stage; a stage's writes to A come after the
        // previous stage's second barrier, its writes to B after its own
        // first, so every read of either block precedes the next write.
        T *la = lds, *lb = lds + (size_t)NW * 6 * W;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            T *e0 = la + (size_t)wv * 6 * W + j * 64 + lane;
            e0[0 * W] = y[0][j][0];
            e0[1 * W] = y[0][j][1];
            e0[2 * W] = y[0][j][2];
            e0[3 * W] = yf[0][j];
            e0[4 * W] = ye[0][j];
            e0[5 * W] = ys[0][j];
        }
        __syncthreads();
        // y faces: face f lies below row f; components (mass, normal = hv,
        // tangential = hu); the top wavefront's top face and the bottom
        // one's bottom face feed only rows that no stage updates
        T Gh[R + 1][C], Gv[R + 1][C], Gu[R + 1][C];
        {
            const int wn = wv < NW - 1 ? wv + 1 : NW - 1;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const T *en = la + (size_t)wn * 6 * W + j * 64 + lane;
                swf_face<T>(y[R - 1][j][0], y[R - 1][j][2], y[R - 1][j][1], yf[R - 1][j], ye[R - 1][j],
                            ys[R - 1][j], en[0], en[2 * W], en[W], en[3 * W], en[4 * W], en[5 * W], Gh[R][j],
                            Gv[R][j], Gu[R][j]);
                T *eo = lb + (size_t)wv * 3 * W + j * 64 + lane;
                eo[0] = Gh[R][j];
                eo[W] = Gv[R][j];
                eo[2 * W] = Gu[R][j];
#pragma unroll
                for (int f = 1; f < R; ++f)
                    swf_face<T>(y[f - 1][j][0], y[f - 1][j][2], y[f - 1][j][1], yf[f - 1][j], ye[f - 1][j],
                                ys[f - 1][j], y[f][j][0], y[f][j][2], y[f][j][1], yf[f][j], ye[f][j], ys[f][j],
                                Gh[f][j], Gv[f][j], Gu[f][j]);
            }
        }
        // the stage's update of cell (q, j) from its slope k (divided by -idx)
        auto update = [&](const int q, const int j, const T (&k)[3]) {
#pragma unroll
            for (int sp = 0; sp < 3; ++sp) {
                if (s == 1) {
                    acc[q][j][sp] = k[sp];
                    y[q][j][sp] = fma(c_half, k[sp], u[q][j][sp]);
                } else if (s == 2) {
                    acc[q][j][sp] = fma(T(2), k[sp], acc[q][j][sp]);
                    y[q][j][sp] = fma(c_half, k[sp], u[q][j][sp]);
                } else if (s == 3) {
                    acc[q][j][sp] = fma(T(2), k[sp], acc[q][j][sp]);
                    y[q][j][sp] = fma(c_full, k[sp], u[q][j][sp]);
                } else {
                    const T inc = c_sixth * (acc[q][j][sp] + k[sp]);
                    if constexpr (KAHAN) {
                        const T yk = inc - cm[q][j][sp];
                        const T un = u[q][j][sp] + yk;
                        cm[q][j][sp] = (un - u[q][j][sp]) - yk;
                        u[q][j][sp] = un;
                    } else {
                        u[q][j][sp] = u[q][j][sp] + inc;
                    }
                }
            }
        };

        // x faces: the east face of each cell (the next cell of the lane, or
        // the first cell of the east lane), the west face from the cell (or
        // lane) before it; the walls' faces from the mirror state.  Rows
        // 1 .. R-1 have both y faces and update at once; row 0 keeps its x
        // flux differences until the face below it arrives.
        T ph[C], pm[C], pn[C];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = wv * R + q;
            if (!(r >= s && r < RY - s)) continue;  // wave-uniform: rows beyond this stage's region
            T Fh[C], Fm[C], Fn[C];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                T hE, mE, nE, fE, eE, sE;
                if (j < C - 1) {
                    hE = y[q][j + 1][0];
                    mE = y[q][j + 1][1];
                    nE = y[q][j + 1][2];
                    fE = xf[q][j + 1];
                    eE = xe[q][j + 1];
                    sE = xs[q][j + 1];
                } else {
                    hE = lane_neighbour<false, true>(y[q][0][0]);
                    mE = lane_neighbour<false, true>(y[q][0][1]);
                    nE = lane_neighbour<false, true>(y[q][0][2]);
                    fE = lane_neighbour<false, true>(xf[q][0]);
                    eE = lane_neighbour<false, true>(xe[q][0]);
                    sE = lane_neighbour<false, true>(xs[q][0]);
                }
                swf_face<T>(y[q][j][0], y[q][j][1], y[q][j][2], xf[q][j], xe[q][j], xs[q][j], hE, mE, nE, fE, eE,
                            sE, Fh[j], Fm[j], Fn[j]);
            }
            // east wall: the last cell's east face against its mirror image
            {
                const T m = y[q][C - 1][1], f = xf[q][C - 1], a = xs[q][C - 1];
                const T Fw = (f + f) + a * (m + m);
                Fh[C - 1] = wall_e ? T(0) : Fh[C - 1];
                Fm[C - 1] = wall_e ? Fw : Fm[C - 1];
                Fn[C - 1] = wall_e ? T(0) : Fn[C - 1];
            }
            T Wh = lane_neighbour<true, true>(Fh[C - 1]);
            T Wm = lane_neighbour<true, true>(Fm[C - 1]);
            T Wn = lane_neighbour<true, true>(Fn[C - 1]);
            // west wall: the first cell's west face against its mirror image
            {
                const T m = y[q][0][1], f = xf[q][0], a = xs[q][0];
                const T Fw = (f + f) - a * (m + m);
                Wh = wall_w ? T(0) : Wh;
                Wm = wall_w ? Fw : Wm;
                Wn = wall_w ? T(0) : Wn;
            }
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const T dh = Fh[j] - (j == 0 ? Wh : Fh[j - 1]);
                const T dm = Fm[j] - (j == 0 ? Wm : Fm[j - 1]);
                const T dn = Fn[j] - (j == 0 ? Wn : Fn[j - 1]);
                if (q == 0) {
                    ph[j] = dh;
                    pm[j] = dm;
                    pn[j] = dn;
                } else {
                    const T k[3] = {fma(rho, Gh[q + 1][j] - Gh[q][j], dh), fma(rho, Gu[q + 1][j] - Gu[q][j], dm),
                                    fma(rho, Gv[q + 1][j] - Gv[q][j], dn)};
                    update(q, j, k);
                }
            }
        }
        __syncthreads();
        if (wv * R >= s && wv * R < RY - s) {  // wave-uniform: row 0 inside this stage's region
            const int ws = wv > 0 ? wv - 1 : 0;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const T *es = lb + (size_t)ws * 3 * W + j * 64 + lane;
                const T k[3] = {fma(rho, Gh[1][j] - es[0], ph[j]), fma(rho, Gu[1][j] - es[2 * W], pm[j]),
                                fma(rho, Gv[1][j] - es[W], pn[j])};
                update(0, j, k);
            }
        }
    }

    // ---- the tile's own cells
#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (!own[q]) continue;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int c = rowc[q] + j;
#pragma unroll
            for (int sp = 0; sp < 3; ++sp) {
                dst[sp * nc + c] = u[q][j][sp];
                if constexpr (KAHAN) cmp[sp * nc + c] = cm[q][j][sp];
            }
        }
    }
}

}  // namespace rpr
