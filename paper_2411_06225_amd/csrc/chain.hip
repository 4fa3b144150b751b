// chain.hip -- the sequential part of Parareal on the device.
//
// Coarse sweep (Sec. 2, k = 0): U_i^0 = G(U_{i-1}^0), i = 1..N.
//
// Predictor-corrector sweep of iteration k (eq. "update_rule_generic") with
// the stopping rule of eq. "stop_crit":
//   U_{L+1} = F(U_L)                     exact: U_L is final
//   U_i = G(U_{i-1}) + fhat(U_{i-1}),    i = L+2..N, in order
//   L <- L+1, then over i = L+2..N while ||U_i^k - U_i^{k-1}||_inf < eps.
// fhat is W^T sigma(A x / s + zeta) (eq. "HA") or (F - G)(U_{i-1}^{k-1})
// (eq. "fpara").
//
// One cooperative launch runs a whole sweep.  Per slot, work-group 0 runs the
// coarse propagator on chip while the other work-groups finish the hidden
// layer sigma(A x / s + zeta) of U_{i-1}; after a grid barrier every
// work-group applies the readout, the update and the change norm to its own
// block of columns of U_i and sums the hidden layer of U_i over those columns;
// a second grid barrier publishes U_i and the partial sums.  The converged-slot counter L and the done flag live
// in the device control block, so the host never waits on the sweep.
#include <hip/hip_cooperative_groups.h>

#include <type_traits>

#include "chain.h"
#include "slotprop.h"
#include "tiledprop.h"

namespace cg = cooperative_groups;

namespace rpr {

// Block-wide sum in a fixed order: wave shuffles, then the wave partials in
// wave order.  `red` holds at least 16 doubles of LDS.  Returns the sum in
// every thread.
__device__ __forceinline__ double block_sum(double v, double *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = (blockDim.x + 63) / 64;
    for (int w = 0; w < nw; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Same for floats (reduced-precision hidden layer).
__device__ __forceinline__ float block_sum_f(float v, float *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float s = 0.0f;
    const int nw = (blockDim.x + 63) / 64;
    for (int w = 0; w < nw; ++w) s += red[w];
    __syncthreads();
    return s;
}

__device__ __forceinline__ double nan_max(double a, double b)
{
    if (a != a) a = INFINITY;
    if (b != b) b = INFINITY;
    return a > b ? a : b;
}

// Hidden layer phi = sigma(A x / s + zeta), split over the work-groups by
// columns: the work-group that owns columns j0 .. j1 of a slot state (it has
// just written them) sums A[m][j] x_j / s over them for every neuron m
// (hidden_partial), and after the grid barrier the owner of neuron m adds the
// grid's partial sums in work-group order and applies sigma (hidden_finish).
// No work-group reads another's columns of x.  Sums and sigma in double in
// both precisions (the training features of reduced-precision plans come
// from the split-bfloat16 GEMM, accurate to the same order as FP32 states).
// V consecutive values of a weight row as doubles, in vector loads where the
// alignment allows (V * sizeof(T) bytes from an address that is a multiple
// of it, or of 16 for four doubles).
template <typename T, int V>
__device__ __forceinline__ void load_run(const T *__restrict__ p, double *v)
{
    if constexpr (V == 1) {
        v[0] = double(p[0]);
    } else if constexpr (sizeof(T) == 4) {
        using VT = typename std::conditional<V == 4, float4, float2>::type;
        const VT r = *reinterpret_cast<const VT *>(p);
        const float *f = reinterpret_cast<const float *>(&r);
#pragma unroll
        for (int u = 0; u < V; ++u) v[u] = f[u];
    } else {
#pragma unroll
        for (int u = 0; u < V; u += 2) {
            const double2 r = *reinterpret_cast<const double2 *>(p + u);
            v[u] = r.x;
            v[u + 1] = r.y;
        }
    }
}

// Partial sums of the hidden layer over columns j0 .. j1 with V neurons per
// thread: G = M / V neuron groups, R column classes (R x G <= B threads; at
// most 16 so that the per-class sums fit the LDS the kernels reserve).
// Thread (q, r) = (t mod G, t / G) sums A[m][j] x_j / s for its neurons
// m = V q .. V q + V - 1 over the columns j = j0 + r, j0 + r + R, ...: a
// wavefront reads a contiguous run of each row of A^T, and the loads of a
// batch of CB columns are in flight together (the column bounds are checked
// per batch, outside it).  With G > B (odd M above the block size) a thread
// takes the groups t, t + B, ... of one class.  The class sums meet in LDS
// (red, R x M doubles) and are added in class order.
template <typename T, int V>
__device__ __forceinline__ int hidden_partial_v(const ChainArgs<T> &a, const T *__restrict__ x, const int j0,
                                                const int j1, double *red)
{
    constexpr int CB = 8;
    const int t = threadIdx.x, B = blockDim.x, M = a.M;
    const int G = M / V;
    const int R = G <= B ? min(16, B / G) : 1;
    const int r = G <= B ? t / G : 0;
    if (r < R) {
        for (int q = G <= B ? t % G : t; q < G; q += G <= B ? G : B) {
            double p[V];
#pragma unroll
            for (int u = 0; u < V; ++u) p[u] = 0.0;
            const T *base = a.At + (size_t)V * q;
            int j = j0 + r;
            for (; j + (CB - 1) * R < j1; j += CB * R) {
                double w[CB][V], xv[CB];
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    load_run<T, V>(base + (size_t)(j + k * R) * M, w[k]);
                    xv[k] = double(x[j + k * R]) * a.inv_s;
                }
#pragma unroll
                for (int k = 0; k < CB; ++k)
#pragma unroll
                    for (int u = 0; u < V; ++u) p[u] = fma(w[k][u], xv[k], p[u]);
            }
            for (; j < j1; j += R) {
                double w[V];
                load_run<T, V>(base + (size_t)j * M, w);
                const double xv = double(x[j]) * a.inv_s;
#pragma unroll
                for (int u = 0; u < V; ++u) p[u] = fma(w[u], xv, p[u]);
            }
#pragma unroll
            for (int u = 0; u < V; ++u) red[r * M + V * q + u] = p[u];
        }
    }
    return R;
}

template <typename T>
__device__ __forceinline__ void hidden_partial(const ChainArgs<T> &a, const T *__restrict__ x, const int j0,
                                               const int j1, const int wg, double *red)
{
    // neurons per thread: the run length that keeps the most bytes in
    // flight (busy threads x V; ties to the longer run)
    const int M = a.M, B = blockDim.x;
    auto inflight = [&](int v) {
        const int G = M / v;
        return (G <= B ? min(16, B / G) * G : B) * v;
    };
    int R;
    if (M % 4 == 0 && inflight(4) >= inflight(2) && inflight(4) >= inflight(1))
        R = hidden_partial_v<T, 4>(a, x, j0, j1, red);
    else if (M % 2 == 0 && inflight(2) >= inflight(1))
        R = hidden_partial_v<T, 2>(a, x, j0, j1, red);
    else
        R = hidden_partial_v<T, 1>(a, x, j0, j1, red);
    __syncthreads();
    for (int m = threadIdx.x; m < M; m += B) {
        double z = 0.0;
        for (int w = 0; w < R; ++w) z += red[w * M + m];
        a.hpart[(size_t)wg * M + m] = z;
    }
}

// Neurons m = hw, hw + nh, ... of this work-group: one wavefront per neuron.
template <typename T>
__device__ __forceinline__ void hidden_finish(const ChainArgs<T> &a, const int hw, const int nh, const int nwg)
{
    const int t = threadIdx.x, B = blockDim.x;
    const int WL = B >= 64 ? 64 : B, nw = B >= 64 ? B / 64 : 1;
    const int lane = t & 63, wv = t >> 6;
    for (int m = hw + nh * wv; wv < nw && m < a.M; m += nh * nw) {
        double z = 0.0;
        for (int w = lane; w < nwg; w += WL) z += a.hpart[(size_t)w * a.M + m];
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_down(z, off, 64);
            if (lane + off < WL) z += o;
        }
        if (lane == 0) {
            z += a.zeta[m];
            a.phi[m] = a.act == RPR_RELU ? (z > 0.0 ? z : 0.0) : tanh(z);
        }
    }
}

// Nearest-neighbour mode (eq. "randnet"; App. B): squared Euclidean
// distances of a slot state x to the n stored inputs, split over the
// work-groups by columns like the hidden layer.  dist_partial: the owner of
// columns j0 .. j1 sums (Xs[l][j] - x[j])^2 over them for every stored row l;
// after the grid barrier dist_finish: the owner of row l adds the partial
// sums in work-group order.  Doubles in both precisions.
template <typename T>
__device__ __forceinline__ void dist_partial_wave(const ChainArgs<T> &a, const T *__restrict__ x, const int j0,
                                             const int j1, const int wg, const int n)
{
    const int t = threadIdx.x, B = blockDim.x, d = a.g.d;
    const int WL = B >= 64 ? 64 : B, nw = B >= 64 ? B / 64 : 1;
    const int lane = t & 63, wv = t >> 6;
    if (wv >= nw) return;
    constexpr int RB = 8, JB = 2;  // rows per wavefront and pass, columns per lane and load batch
    for (int l0 = wv * RB; l0 < n; l0 += nw * RB) {
        double acc[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[r] = 0.0;
        for (int jb = j0; jb < j1; jb += WL * JB) {
            // every load goes to a clamped in-range address and the masks
            // apply after it, so the RB x JB loads of a batch are in flight
            // together (a load under its own bound check waits for itself)
            double xv[JB], v[RB][JB];
            int jc[JB];
            bool jin[JB];
#pragma unroll
            for (int q = 0; q < JB; ++q) {
                const int j = jb + q * WL + lane;
                jin[q] = j < j1;
                jc[q] = jin[q] ? j : j1 - 1;
                const double xl = double(x[jc[q]]);
                xv[q] = jin[q] ? xl : 0.0;
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int l = l0 + r;
                const T *row = a.Xs + (size_t)(l < n ? l : n - 1) * d;
#pragma unroll
                for (int q = 0; q < JB; ++q) {
                    const double xl = double(row[jc[q]]);
                    v[r][q] = (l < n && jin[q]) ? xl : xv[q];
                }
            }
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int q = 0; q < JB; ++q) {
                    const double e = v[r][q] - xv[q];
                    acc[r] = fma(e, e, acc[r]);
                }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            double z = acc[r];
            for (int off = 32; off > 0; off >>= 1) {
                const double o = __shfl_down(z, off, 64);
                if (lane + off < WL) z += o;
            }
            if (lane == 0 && l0 + r < n) a.dpart[(size_t)wg * a.n_cap + l0 + r] = z;
        }
    }
}

// The same for a chunk of at most 2 G columns (G = 8, 16 or 32): groups of
// G lanes take a row each (64 / G rows per wavefront at a time, 8 G / 64 rows
// per group and pass), so that no lane idles and each row's sum needs a
// reduction over G lanes only.
template <typename T, int G>
__device__ __forceinline__ void dist_partial_groups(const ChainArgs<T> &a, const T *__restrict__ x, const int j0,
                                                    const int j1, const int wg, const int n)
{
    const int t = threadIdx.x, B = blockDim.x, d = a.g.d;
    const int nw = B >= 64 ? B / 64 : 1;
    const int lane = t & 63, wv = t >> 6;
    if (wv >= nw) return;
    constexpr int NG = 64 / G, RG = 8 / NG, JB = 2;  // groups per wavefront, rows per group and pass
    const int gi = lane / G, sub = lane % G;
    double xv[JB];
    int jc[JB];
    bool jin[JB];
#pragma unroll
    for (int q = 0; q < JB; ++q) {
        const int j = j0 + q * G + sub;
        jin[q] = j < j1;
        jc[q] = jin[q] ? j : j1 - 1;
        const double xl = double(x[jc[q]]);
        xv[q] = jin[q] ? xl : 0.0;
    }
    for (int l0 = wv * 8; l0 < n; l0 += nw * 8) {
        double acc[RG];
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            const int l = l0 + gi * RG + r;
            const T *row = a.Xs + (size_t)(l < n ? l : n - 1) * d;
            double v[JB];
#pragma unroll
            for (int q = 0; q < JB; ++q) {
                const double xl = double(row[jc[q]]);
                v[q] = (l < n && jin[q]) ? xl : xv[q];
            }
            acc[r] = 0.0;
#pragma unroll
            for (int q = 0; q < JB; ++q) {
                const double e = v[q] - xv[q];
                acc[r] = fma(e, e, acc[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            double z = acc[r];
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) z += __shfl_xor(z, off, 64);
            const int l = l0 + gi * RG + r;
            if (sub == 0 && l < n) a.dpart[(size_t)wg * a.n_cap + l] = z;
        }
    }
}

// Squared distances of x to the n stored rows over columns j0 .. j1 of this
// work-group: lane groups for narrow chunks, whole wavefronts otherwise.
template <typename T>
__device__ __forceinline__ void dist_partial(const ChainArgs<T> &a, const T *__restrict__ x, const int j0,
                                             const int j1, const int wg, const int n)
{
    const int chunk = j1 - j0;
    const bool groups = blockDim.x % 64 == 0 && chunk > 0;  // every row of dpart gets written either way
    if (groups && chunk <= 16) dist_partial_groups<T, 8>(a, x, j0, j1, wg, n);
    else if (groups && chunk <= 32) dist_partial_groups<T, 16>(a, x, j0, j1, wg, n);
    else if (groups && chunk <= 64) dist_partial_groups<T, 32>(a, x, j0, j1, wg, n);
    else dist_partial_wave<T>(a, x, j0, j1, wg, n);
}

// Rows l = hw, hw + nh, ... of the distance vector: one wavefront per row.
template <typename T>
__device__ __forceinline__ void dist_finish(const ChainArgs<T> &a, const int hw, const int nh, const int nwg,
                                            const int n)
{
    const int t = threadIdx.x, B = blockDim.x;
    const int WL = B >= 64 ? 64 : B, nw = B >= 64 ? B / 64 : 1;
    const int lane = t & 63, wv = t >> 6;
    for (int l = hw + nh * wv; wv < nw && l < n; l += nh * nw) {
        double z = 0.0;
        for (int w = lane; w < nwg; w += WL) z += a.dpart[(size_t)w * a.n_cap + l];
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_down(z, off, 64);
            if (lane + off < WL) z += o;
        }
        if (lane == 0) a.dist[l] = z;
    }
}

// (distance, row) of the lesser of two candidates; equal distances go to the
// lower row.
__device__ __forceinline__ void nn_min(double &bd, int &bi, const double od, const int oi)
{
    if (od < bd || (od == bd && oi < bi)) {
        bd = od;
        bi = oi;
    }
}

// The refit of one prediction (eq. "randnet", Alg. "RandNets training
// procedure"), by wavefront 0 of every work-group (the same result in each,
// so no barrier is needed): the m nearest finite stored pairs of the current
// slot input (distances from dist_finish, NaN read as +inf, ties to the lower
// row), then the dual ridge readout on them,
//   K = Phi~ Phi~^T + lambda I (m x m),  alpha = K^-1 Phi~ phi(x),
// so that the correction W^T phi(x) = Y~^T alpha.  sel / alpha (LDS, m
// entries, and sel[NN_MAX] the count) receive the rows and weights; K is LDS
// scratch of NN_MAX^2 doubles.  Returns m, or 0 when there is no pair or K
// is not positive definite (no correction; work-group 0 counts the failure).
template <typename T>
__device__ __forceinline__ int nn_refit(const ChainArgs<T> &a, const int n, const int wg, int *sel, double *alpha,
                                        double *K)
{
    int &m_sh = sel[NN_MAX];
    const int t = threadIdx.x, B = blockDim.x;
    const int WL = B >= 64 ? 64 : B;
    const int lane = t & 63;
    if (t < 64) {
        int m = a.m_nn < a.ctrl->rows_used ? a.m_nn : a.ctrl->rows_used;
        // selection in (distance, row) order, one pair per round
        double pd = -INFINITY;
        int pi = -1;
        for (int r = 0; r < m; ++r) {
            double bd = INFINITY;
            int bi = 0x7fffffff;
            for (int l = lane; l < n; l += WL) {
                if (!a.oks[l]) continue;
                double dl = a.dist[l];
                if (dl != dl) dl = INFINITY;
                if (dl > pd || (dl == pd && l > pi)) nn_min(bd, bi, dl, l);
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double od = __shfl_xor(bd, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if ((lane ^ off) < WL) nn_min(bd, bi, od, oi);
            }
            if (bi == 0x7fffffff) {  // fewer finite pairs than counted: cannot happen
                m = r;
                break;
            }
            if (lane == 0) sel[r] = bi;
            pd = bd;
            pi = bi;
        }
        __builtin_amdgcn_wave_barrier();
        // K (upper triangle) and the right-hand side Phi~ phi
        for (int p = 0; p < m; ++p) {
            const double *Pp = a.Ps + (size_t)sel[p] * a.M;
            for (int q = p; q <= m; ++q) {
                const double *Pq = q < m ? a.Ps + (size_t)sel[q] * a.M : a.phi;
                double z = 0.0;
                for (int c = lane; c < a.M; c += WL) z = fma(Pp[c], Pq[c], z);
                for (int off = 32; off > 0; off >>= 1) {
                    const double o = __shfl_xor(z, off, 64);
                    if ((lane ^ off) < WL) z += o;
                }
                if (lane == 0) {
                    if (q < m) K[p * NN_MAX + q] = z + (p == q ? a.lambda : 0.0);
                    else alpha[p] = z;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        // Cholesky K = L L^T (lower triangle, in place) and alpha = K^-1 b
        if (lane == 0) {
            bool spd = true;
            for (int j = 0; j < m && spd; ++j) {
                double s = K[j * NN_MAX + j];
                for (int k = 0; k < j; ++k) s -= K[j * NN_MAX + k] * K[j * NN_MAX + k];
                if (!(s > 0.0)) {
                    spd = false;
                    break;
                }
                const double ljj = sqrt(s);
                K[j * NN_MAX + j] = ljj;
                for (int i = j + 1; i < m; ++i) {
                    double v = K[j * NN_MAX + i];  // upper triangle holds K[j][i] = K[i][j]
                    for (int k = 0; k < j; ++k) v -= K[i * NN_MAX + k] * K[j * NN_MAX + k];
                    K[i * NN_MAX + j] = v / ljj;
                }
            }
            if (spd) {
                for (int i = 0; i < m; ++i) {
                    double v = alpha[i];
                    for (int k = 0; k < i; ++k) v -= K[i * NN_MAX + k] * alpha[k];
                    alpha[i] = v / K[i * NN_MAX + i];
                }
                for (int i = m - 1; i >= 0; --i) {
                    double v = alpha[i];
                    for (int k = i + 1; k < m; ++k) v -= K[k * NN_MAX + i] * alpha[k];
                    alpha[i] = v / K[i * NN_MAX + i];
                }
            } else {
                if (wg == 0) atomicAdd(&a.ctrl->chol_fail, 1);
                m = 0;
            }
            m_sh = m;
        }
    }
    __syncthreads();
    return m_sh;
}

// ---- the predictor-corrector sweep, segment by segment ----
// A sweep is a prologue, then for every predicted slot i = L+2..N a phase 1
// (coarse solve, hidden layer of U_{i-1}) and a phase 2 (readout, update,
// change norm, hidden-layer partial sums of U_i), then the stopping rule.
// The segments are separated by a barrier over the work-groups sharing the
// instance: a grid barrier inside one cooperative launch (chain_body), or
// the boundary between kernels of a captured graph (k_chain_seg).  Every
// segment reads L and the done flag from the control block, which only the
// stopping rule changes, so both forms take the same decisions and compute
// the same values bit for bit.  wg / nwg: this work-group and the number of
// work-groups sharing the instance.  TILED: the slot state does not fit one
// work-group; the coarse solver then runs on the whole grid in passes
// (tiled_coarse_pass) instead of on work-group 0.  NN_OK: the nearest-
// neighbour refit is compiled in (otherwise a kernel for the other modes
// carries none of its code or registers).

// Columns [j0, j1) of a slot state owned by work-group wg of nwg (an even
// count, so that FP32 rows of even length start 8-byte aligned).
__device__ __forceinline__ void chain_columns(const int d, const int wg, const int nwg, int &j0, int &j1)
{
    const int chunk = (((d + nwg - 1) / nwg) + 1) & ~1;
    j0 = min(d, wg * chunk);
    j1 = min(d, j0 + chunk);
}

// Coarse solver of the sweep: on one work-group (CM_ONCHIP), in tiles over
// the grid (CM_TILED), or cell by cell over the grid by its tableau
// (CM_GENERIC: the 3D system, the eighth-order method).  CM_TILED_EULER is
// CM_TILED for forward Euler only: its multi-step tiles take any work-group
// size (the per-stage tiles of the other methods assume TT_THREADS).
enum { CM_ONCHIP = 0, CM_TILED = 1, CM_GENERIC = 2, CM_TILED_EULER = 3 };

// Passes of the grid-wide coarse solvers per slot: tiled forward Euler takes
// up to EH steps per pass (euler_tile_multi), tiled RK4 one pass per stage,
// the generic form one pass per stage of its tableau (s stages).
__host__ __device__ inline long long coarse_passes(int cm, int method, long long steps, int s)
{
    if (cm == CM_GENERIC) return steps * s;
    return method == RPR_RK1 ? (steps + EH - 1) / EH : 4 * steps;
}

// Pass `pass` of the generic coarse propagation src -> dst (and dst2): stage
// pass % s of step pass / s over every cell, the cells spread over all the
// threads of the grid (work arrays in a.gw as rkgen_work lays them out for
// one state).
template <int KIND, typename T>
__device__ __forceinline__ void generic_coarse_pass(const ChainArgs<T> &a, const T *src, T *dst, T *dst2,
                                                    const long long pass, const int wg, const int nwg)
{
    const int s = a.tbG.s;
    const long long step = pass / s;
    const int stage = (int)(pass % s);
    const RkIO<T> io = rkgen_io<T>(s, stage, step, a.G_steps, src, dst, dst2, a.gw);
    const int B = blockDim.x;
    for (int c = wg * B + (int)threadIdx.x; c < a.g.nc; c += nwg * B)
        rkgen_cell<KIND, T>(a.g, a.tbG, stage, a.dtG, c, io.y, a.gw.acc, (size_t)a.g.d, io.u, io.ynext, io.uout,
                            io.uout2, a.gw.cmp, step == 0 ? 1 : 0);
}

// Pass `pass` of the tiled coarse propagation src -> dst (and dst2) by the
// work-groups of the grid (tiles spread over them).  Forward Euler: passes of
// up to EH steps without a barrier; the state alternates between the work
// arrays u and ya from pass to pass, the FP32 compensation between cmp and
// acc (forward Euler has no slope sum), so that no tile reads a value another
// tile of the same pass has already replaced.  RK4: one pass per stage.
template <int KIND, typename T, bool EULER_ONLY>
__device__ __forceinline__ void tiled_coarse_pass(const ChainArgs<T> &a, const T *src, T *dst, T *dst2,
                                                  const long long pass, const int wg, const int nwg, T *lds)
{
    if (EULER_ONLY || a.G_method == RPR_RK1) {
        T *buf[2] = {a.gw.u, a.gw.ya};
        T *cbuf[2] = {a.gw.cmp, a.gw.acc};
        const long long s = pass * EH;
        const int n = (int)(a.G_steps - s < EH ? a.G_steps - s : EH);
        const bool last = s + n >= a.G_steps;
        const T *in = s == 0 ? src : buf[(pass - 1) & 1];
        T *out = last ? dst : buf[pass & 1];
        auto run = [&](auto tile_tag) {
            using ET = decltype(tile_tag);
            const int nt = ET::tiles(a.g);
            for (int tile = wg; tile < nt; tile += nwg)
                euler_tile_multi<KIND, T, ET>(a.g, tile, n, a.dtG, in, out, last ? dst2 : (T *)nullptr,
                                              cbuf[(pass + 1) & 1], cbuf[pass & 1], s == 0 ? 1 : 0, lds);
        };
        if (SweepEulerSmall::tiles(a.g) <= nwg) run(SweepEulerSmall{});
        else run(SweepEuler{});
        return;
    }
    if constexpr (!EULER_ONLY) {
        const int nt = tiles_of(a.g);
        const long long step = pass / 4;
        const int stage = (int)(pass % 4) + 1;
        const StageIO<T> io = stage_io<T>(a.G_method, stage, step, a.G_steps, src, dst, dst2, a.gw);
        for (int tile = wg; tile < nt; tile += nwg) stage_tile_any<KIND, T>(a.g, tile, stage, a.dtG, io, lds);
    }
}

// One pass of a grid-wide coarse solver.
template <int KIND, typename T, int CM>
__device__ __forceinline__ void coarse_pass(const ChainArgs<T> &a, const T *src, T *dst, T *dst2,
                                            const long long pass, const int wg, const int nwg, T *lds)
{
    if constexpr (CM == CM_GENERIC) {
        (void)lds;
        generic_coarse_pass<KIND, T>(a, src, dst, dst2, pass, wg, nwg);
    } else if constexpr (KIND != RPR_BURGERS1D && KIND != RPR_BRUSS3D) {
        tiled_coarse_pass<KIND, T, CM == CM_TILED_EULER>(a, src, dst, dst2, pass, wg, nwg, lds);
    }
}

// The whole grid-wide coarse propagation, passes separated by sync().
template <int KIND, typename T, int CM, typename Sync>
__device__ __forceinline__ void grid_coarse(const ChainArgs<T> &a, const T *src, T *dst, T *dst2, const int wg,
                                            const int nwg, Sync sync, T *lds)
{
    const long long np = coarse_passes(CM, a.G_method, a.G_steps, a.tbG.s);
    for (long long pass = 0; pass < np; ++pass) {
        coarse_pass<KIND, T, CM>(a, src, dst, dst2, pass, wg, nwg, lds);
        sync();
    }
}

// Prologue: the exact slot U_{L+1} = F(U_L), and the hidden-layer (and
// distance) partial sums of its columns.
template <typename T, bool NN_OK>
__device__ __forceinline__ void chain_seg_pro(const ChainArgs<T> &a, const int wg, const int nwg, double *scratch)
{
    const int t = threadIdx.x, B = blockDim.x, d = a.g.d;
    const Ctrl *ctrl = a.ctrl;
    const int L = ctrl->L, N = a.N;
    int j0, j1;
    chain_columns(d, wg, nwg, j0, j1);
    const bool nn = NN_OK && a.mode == CHAIN_RANDNET_NN;
    const bool net = a.mode == CHAIN_RANDNET || nn;
    const int n_store = nn ? ctrl->nn_rows + *a.nrows : 0;
    for (int j = j0 + t; j < j1; j += B) a.U[(size_t)(L + 1) * d + j] = a.Fv[(size_t)(L + 1) * d + j];
    if (net && L + 2 <= N) {
        __syncthreads();
        hidden_partial(a, a.U + (size_t)(L + 1) * d, j0, j1, wg, scratch);
        if (nn) dist_partial(a, a.U + (size_t)(L + 1) * d, j0, j1, wg, n_store);
    }
}

// Phase 1 of slot i, on-chip coarse solver: work-group 0 propagates U_{i-1}
// into gtmp, the others (all, if there is one work-group) finish the hidden
// layer (and distances) of U_{i-1}.
template <int KIND, typename T, int CPT, bool DBUF, bool FULL, int NX, int NY, bool NN_OK>
__device__ __forceinline__ void chain_seg_p1_onchip(const ChainArgs<T> &a, const int i, const int wg, const int nwg,
                                                    T *lds)
{
    const int d = a.g.d;
    const bool nn = NN_OK && a.mode == CHAIN_RANDNET_NN;
    const bool net = a.mode == CHAIN_RANDNET || nn;
    const int n_store = nn ? a.ctrl->nn_rows + *a.nrows : 0;
    if (wg == 0) {
        slot_propagate<KIND, T, CPT, DBUF, FULL, NX, NY>(a.g, a.G_method, a.G_steps, a.dtG, a.U + (size_t)(i - 1) * d,
                                                         a.gtmp, lds);
        __syncthreads();
    }
    if (net && (wg > 0 || nwg == 1)) hidden_finish(a, nwg == 1 ? 0 : wg - 1, nwg == 1 ? 1 : nwg - 1, nwg);
    if (nn && (wg > 0 || nwg == 1)) dist_finish(a, nwg == 1 ? 0 : wg - 1, nwg == 1 ? 1 : nwg - 1, nwg, n_store);
}

// The hidden layer (and distances) of U_{i-1} on every work-group (the part
// of phase 1 beside the tiled coarse solver).
template <typename T, bool NN_OK>
__device__ __forceinline__ void chain_seg_hidden_all(const ChainArgs<T> &a, const int wg, const int nwg)
{
    const bool nn = NN_OK && a.mode == CHAIN_RANDNET_NN;
    const bool net = a.mode == CHAIN_RANDNET || nn;
    if (net) hidden_finish(a, wg, nwg, nwg);
    if (nn) dist_finish(a, wg, nwg, nwg, a.ctrl->nn_rows + *a.nrows);
}

// Phase 2 of slot i: readout, update, change norm on this work-group's
// columns of U_i, and the hidden-layer partial sums of U_i for slot i + 1.
template <typename T, bool NN_OK>
__device__ __forceinline__ void chain_seg_p2(const ChainArgs<T> &a, const int i, const int wg, const int nwg,
                                             double *scratch)
{
    const int t = threadIdx.x, B = blockDim.x, d = a.g.d, N = a.N;
    int j0, j1;
    chain_columns(d, wg, nwg, j0, j1);
    const bool nn = NN_OK && a.mode == CHAIN_RANDNET_NN;
    const bool net = a.mode == CHAIN_RANDNET || nn;
    const int n_store = nn ? a.ctrl->nn_rows + *a.nrows : 0;
    double emax = 0.0;
    const T *Fvi = a.Fv + (size_t)i * d;
    T *Ui = a.U + (size_t)i * d;
    T *Gci = a.Gc + (size_t)i * d;
    if (nn) {
        // refit on the nearest stored pairs, then U_i = G + Y~^T alpha on
        // columns j0 .. j1
        double *K = scratch;                          // NN_MAX x NN_MAX
        double *alpha = scratch + NN_MAX * NN_MAX;    // NN_MAX
        int *sel = reinterpret_cast<int *>(alpha + NN_MAX);
        const int m = nn_refit(a, n_store, wg, sel, alpha, K);
        for (int j = j0 + t; j < j1; j += B) {
            double c = 0.0;
            for (int r = 0; r < m; ++r) c = fma(alpha[r], double(a.Ys[(size_t)sel[r] * d + j]), c);
            const T gv = a.gtmp[j];
            const T unew = T(double(gv) + c);
            emax = nan_max(emax, fabs(double(unew) - double(Ui[j])));
            Ui[j] = unew;
            Gci[j] = gv;
        }
        if (i < N) {
            __syncthreads();
            hidden_partial(a, Ui, j0, j1, wg, scratch);
            dist_partial(a, Ui, j0, j1, wg, n_store);
        }
    } else if (net) {
        // readout W^T phi on columns j0 .. j1: wavefront v takes the tiles
        // of 2 WL columns jb = j0 + 2 WL (v + nw k), lane l the columns
        // jb + 2l and jb + 2l + 1, each summed over the M neurons in order.
        // The column checks sit outside the loop over neurons, so the loads
        // of a batch of neurons are in flight together (one load per neuron
        // and pair of columns where d is even)
        const int WL = B >= 64 ? 64 : B, nw = B >= 64 ? B / 64 : 1;
        const int lane = t & 63, wv = t >> 6;
        double *sphi = scratch;  // M
        for (int m = t; m < a.M; m += B) sphi[m] = a.phi[m];
        __syncthreads();
        const int M = a.M;
        const bool vec = d % 2 == 0;
        auto update = [&](const int j, const double c) {
            const T gv = a.gtmp[j];
            const T unew = T(double(gv) + c);
            emax = nan_max(emax, fabs(double(unew) - double(Ui[j])));
            Ui[j] = unew;
            Gci[j] = gv;
        };
        for (int jb = j0 + 2 * WL * wv; wv < nw && jb < j1; jb += 2 * WL * nw) {
            const int j = jb + 2 * lane;
            const T *wp = a.W + j;
            if (j + 1 < j1) {
                double c0 = 0.0, c1 = 0.0;
                auto sum = [&](auto vec_tag) {
                    constexpr bool VEC = decltype(vec_tag)::value;
                    constexpr int UR = 8;
                    int m0 = 0;
                    for (; m0 + UR <= M; m0 += UR) {
                        double w0[UR], w1[UR];
#pragma unroll
                        for (int u = 0; u < UR; ++u) {
                            const T *q = wp + (size_t)(m0 + u) * d;
                            if constexpr (VEC) {
                                double v2[2];
                                load_run<T, 2>(q, v2);
                                w0[u] = v2[0];
                                w1[u] = v2[1];
                            } else {
                                w0[u] = double(q[0]);
                                w1[u] = double(q[1]);
                            }
                        }
#pragma unroll
                        for (int u = 0; u < UR; ++u) {
                            const double ph = sphi[m0 + u];
                            c0 = fma(w0[u], ph, c0);
                            c1 = fma(w1[u], ph, c1);
                        }
                    }
                    for (; m0 < M; ++m0) {
                        const double ph = sphi[m0];
                        c0 = fma(double(wp[(size_t)m0 * d]), ph, c0);
                        c1 = fma(double(wp[(size_t)m0 * d + 1]), ph, c1);
                    }
                };
                if (vec) sum(std::true_type{});
                else sum(std::false_type{});
                update(j, c0);
                update(j + 1, c1);
            } else if (j < j1) {
                double c0 = 0.0;
                for (int m0 = 0; m0 < M; ++m0) c0 = fma(double(wp[(size_t)m0 * d]), sphi[m0], c0);
                update(j, c0);
            }
        }
        // the state's columns written by the other wavefronts; sphi free
        __syncthreads();
        // hidden-layer partial sums of the new state's columns, for slot i + 1
        if (i < N) hidden_partial(a, Ui, j0, j1, wg, scratch);
    } else {
        for (int j = j0 + t; j < j1; j += B) {
            const T gv = a.gtmp[j];
            const T unew = gv + (Fvi[j] - Gci[j]);
            emax = nan_max(emax, fabs(double(unew) - double(Ui[j])));
            Ui[j] = unew;
            Gci[j] = gv;
        }
    }
    // work-group maximum (order-free, NaN already mapped to +inf); only
    // lanes that exist in a partial wavefront take part
    {
        const int wl = min(64, B - (t & ~63));
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_down(emax, off, 64);
            if ((t & 63) + off < wl) emax = nan_max(emax, o);
        }
    }
    __syncthreads();
    if ((t & 63) == 0) scratch[t >> 6] = emax;
    __syncthreads();
    if (t == 0) {
        double m = 0.0;
        for (int w = 0; w < (B + 63) / 64; ++w) m = nan_max(m, scratch[w]);
        a.part[(size_t)i * nwg + wg] = m;
    }
}

// Stopping rule (eq. "stop_crit") on work-group 0: the change of slot i is
// the largest of the work-groups' maxima for it (one wavefront per slot;
// nan_max is order-free), staged in LDS in chunks of EPI_CHUNK slots; thread
// 0 then walks the slots in order.
constexpr int EPI_CHUNK = 1024;

template <typename T, bool NN_OK>
__device__ __forceinline__ void chain_seg_epi(const ChainArgs<T> &a, const int wg, const int nwg, double *scratch)
{
    if (wg != 0) return;
    const int t = threadIdx.x, B = blockDim.x;
    const int WL = B >= 64 ? 64 : B, nw = B >= 64 ? B / 64 : 1;
    const int lane = t & 63, wv = t >> 6;
    Ctrl *ctrl = a.ctrl;
    const int L = ctrl->L, N = a.N;
    double chg = 0.0;  // thread 0's
    int Lnew = L + 1;
    bool run = true;
    for (int c0 = L + 2; c0 <= N; c0 += EPI_CHUNK) {
        const int c1 = min(N + 1, c0 + EPI_CHUNK);
        for (int i = c0 + wv; wv < nw && i < c1; i += nw) {
            double e = 0.0;
            for (int w = lane; w < nwg; w += WL) e = nan_max(e, a.part[(size_t)i * nwg + w]);
            for (int off = 32; off > 0; off >>= 1) {
                const double o = __shfl_down(e, off, 64);
                if (lane + off < WL) e = nan_max(e, o);
            }
            if (lane == 0) scratch[i - c0] = e;
        }
        __syncthreads();
        if (t == 0) {
            for (int i = c0; i < c1; ++i) {
                const double e = scratch[i - c0];
                chg = nan_max(chg, e);
                if (run && e < a.eps) Lnew = i;
                else run = false;
            }
        }
        __syncthreads();
    }
    __syncthreads();  // every thread has read L before thread 0 moves it
    if (t != 0) return;
    const bool nn = NN_OK && a.mode == CHAIN_RANDNET_NN;
    const int n_store = nn ? ctrl->nn_rows + *a.nrows : 0;
    const int k = ctrl->k + 1;
    ctrl->k = k;
    ctrl->L = Lnew;
    if (nn) ctrl->nn_rows = n_store;
    if (Lnew >= N || k >= a.k_max) ctrl->done = 1;  // converged, or iteration cap reached
    if (a.L_hist) a.L_hist[k] = Lnew;
    if (a.chg_hist) a.chg_hist[k] = chg;
}

// One sweep of one instance in one launch: the segments separated by sync()
// (a grid barrier, or a work-group barrier when nwg == 1).
template <int KIND, typename T, int CPT, bool DBUF, bool FULL, int NX, int NY, int CM, bool NN_OK, typename Sync>
__device__ __forceinline__ void chain_body(const ChainArgs<T> &a, const int wg, const int nwg, Sync sync,
                                           unsigned char *lds_raw)
{
    T *lds = reinterpret_cast<T *>(lds_raw);
    double *scratch = reinterpret_cast<double *>(lds_raw);
    const int d = a.g.d;

    if (a.mode == CHAIN_SWEEP) {
        if constexpr (CM != CM_ONCHIP) {
            // k = 0 by the whole grid
            for (int i = 1; i <= a.N; ++i)
                grid_coarse<KIND, T, CM>(a, a.U + (size_t)(i - 1) * d, a.U + (size_t)i * d, a.Gc + (size_t)i * d, wg,
                                         nwg, sync, lds);
        } else {
            // k = 0 (single work-group): the state stays on chip from slot to slot
            if (wg != 0) return;
            for (int i = 1; i <= a.N; ++i) {
                slot_propagate<KIND, T, CPT, DBUF, FULL, NX, NY>(a.g, a.G_method, a.G_steps, a.dtG,
                                                                 a.U + (size_t)(i - 1) * d, a.U + (size_t)i * d,
                                                                 lds, a.Gc + (size_t)i * d);
                __syncthreads();
            }
        }
        return;
    }

    if (a.ctrl->done) return;  // same value in every work-group: nobody reaches a barrier
    const int L = a.ctrl->L;
    chain_seg_pro<T, NN_OK>(a, wg, nwg, scratch);
    sync();
    for (int i = L + 2; i <= a.N; ++i) {
        if constexpr (CM != CM_ONCHIP) {
            grid_coarse<KIND, T, CM>(a, a.U + (size_t)(i - 1) * d, a.gtmp, (T *)nullptr, wg, nwg, sync, lds);
            chain_seg_hidden_all<T, NN_OK>(a, wg, nwg);
        } else {
            chain_seg_p1_onchip<KIND, T, CPT, DBUF, FULL, NX, NY, NN_OK>(a, i, wg, nwg, lds);
        }
        sync();
        chain_seg_p2<T, NN_OK>(a, i, wg, nwg, scratch);
        sync();
    }
    chain_seg_epi<T, NN_OK>(a, wg, nwg, scratch);
}

// One segment of a sweep as a kernel of its own (captured graphs): seg 0 the
// prologue; 1 phase 1 of slot i (tiled coarse solver: pass `pass` of it, the
// hidden layer with pass 0); 2 phase 2 of slot i; 3 the stopping rule.
// Work-groups return at once when the run is done or slot i is final.
template <int KIND, typename T, int CPT, bool DBUF, bool FULL, int NX, int NY, int MAXT, int CM, bool NN_OK>
__global__ __launch_bounds__(MAXT) void k_chain_seg(const ChainArgs<T> *__restrict__ args, int seg, int i,
                                                    long long pass)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const ChainArgs<T> &a = *args;
    if (a.ctrl->done) return;
    const int L = a.ctrl->L;
    const int wg = blockIdx.x, nwg = gridDim.x;
    double *scratch = reinterpret_cast<double *>(lds_raw);
    if (seg == 0) {
        chain_seg_pro<T, NN_OK>(a, wg, nwg, scratch);
    } else if (seg == 3) {
        chain_seg_epi<T, NN_OK>(a, wg, nwg, scratch);
    } else {
        if (i < L + 2) return;
        if (seg == 2) {
            chain_seg_p2<T, NN_OK>(a, i, wg, nwg, scratch);
        } else if constexpr (CM != CM_ONCHIP) {
            coarse_pass<KIND, T, CM>(a, a.U + (size_t)(i - 1) * a.g.d, a.gtmp, (T *)nullptr, pass, wg, nwg,
                                     reinterpret_cast<T *>(lds_raw));
            if (pass == 0) chain_seg_hidden_all<T, NN_OK>(a, wg, nwg);
        } else {
            chain_seg_p1_onchip<KIND, T, CPT, DBUF, FULL, NX, NY, NN_OK>(a, i, wg, nwg, reinterpret_cast<T *>(lds_raw));
        }
    }
}

template <int KIND, typename T, int CPT, bool DBUF, bool FULL, int NX, int NY, int MAXT, bool NN_OK>
__global__ __launch_bounds__(MAXT) void k_chain(ChainArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cg::grid_group grid = cg::this_grid();
    chain_body<KIND, T, CPT, DBUF, FULL, NX, NY, CM_ONCHIP, NN_OK>(a, blockIdx.x, gridDim.x, [&]() { grid.sync(); },
                                                                  lds_raw);
}

// Independent instances: work-group b runs the whole sweep of instance b.
template <int KIND, typename T, int CPT, bool DBUF, bool FULL, int NX, int NY, int MAXT>
__global__ __launch_bounds__(MAXT) void k_chain_multi(const ChainArgs<T> *__restrict__ args)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const ChainArgs<T> a = args[blockIdx.x];
    chain_body<KIND, T, CPT, DBUF, FULL, NX, NY, CM_ONCHIP, true>(a, 0, 1, []() { __syncthreads(); }, lds_raw);
}

// ---------------------------------------------------------- tiled form --
template <int KIND, typename T>
__global__ __launch_bounds__(TT_THREADS) void k_chain_tiled(ChainArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cg::grid_group grid = cg::this_grid();
    chain_body<KIND, T, 1, false, false, 0, 0, CM_TILED, true>(a, blockIdx.x, gridDim.x, [&]() { grid.sync(); },
                                                               lds_raw);
}

template <int KIND, typename T>
__global__ __launch_bounds__(TT_THREADS) void k_chain_multi_tiled(const ChainArgs<T> *__restrict__ args)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const ChainArgs<T> a = args[blockIdx.x];
    chain_body<KIND, T, 1, false, false, 0, 0, CM_TILED, true>(a, 0, 1, []() { __syncthreads(); }, lds_raw);
}

// ---------------------------------------------------------- generic form --
constexpr int GENERIC_BLOCK = 256;  // work-group of the generic chain

template <int KIND, typename T>
__global__ __launch_bounds__(GENERIC_BLOCK) void k_chain_generic(ChainArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cg::grid_group grid = cg::this_grid();
    chain_body<KIND, T, 1, false, false, 0, 0, CM_GENERIC, true>(a, blockIdx.x, gridDim.x, [&]() { grid.sync(); },
                                                                 lds_raw);
}

template <int KIND, typename T>
struct ChainMultiLauncher {
    const ChainArgs<T> *args;
    int n_inst;
    const OnchipShape &sh;
    int M;
    hipStream_t st;

    template <int CPT, bool DBUF, bool FULL, int NX, int NY, int MAXT>
    rpr_status run()
    {
        auto kern = k_chain_multi<KIND, T, CPT, DBUF, FULL, NX, NY, MAXT>;
        static bool attr_set = false;
        if (!attr_set) {
            RPR_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)kMaxLds));
            attr_set = true;
        }
        hipLaunchKernelGGL(kern, dim3(n_inst), dim3(sh.block), chain_lds(sh, M), st, args);
        RPR_HIP(hipGetLastError());
        return RPR_OK;
    }
};

template <int KIND, typename T>
rpr_status launch_chain_multi_kind(const ChainArgs<T> *args_dev, int n_inst, const Geom &gmax,
                                   const OnchipShape &sh, int M, hipStream_t st)
{
    if (sh.maxt == GENERIC_THREADS) return fail(RPR_ERR_UNSUPPORTED, "batch instances must fit one work-group each");
    if constexpr (KIND == RPR_BRUSS3D) {
        return fail(RPR_ERR_UNSUPPORTED, "batch instances must fit one work-group each");
    } else {
    if (sh.maxt == TILED_THREADS) {
        if constexpr (KIND == RPR_BURGERS1D) {
            return fail(RPR_ERR_UNSUPPORTED, "the tiled chain serves 2D grids only");
        } else {
            auto kern = k_chain_multi_tiled<KIND, T>;
            static bool attr_set = false;
            if (!attr_set) {
                RPR_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)kMaxLds));
                attr_set = true;
            }
            hipLaunchKernelGGL(kern, dim3(n_inst), dim3(TT_THREADS), chain_lds(sh, M), st, args_dev);
            RPR_HIP(hipGetLastError());
            return RPR_OK;
        }
    }
    ChainMultiLauncher<KIND, T> L{args_dev, n_inst, sh, M, st};
    return visit_shape_kind<KIND, T>(gmax, sh, L);
    }
}

template rpr_status launch_chain_multi_kind<RPR_KIND, RPR_REAL>(const ChainArgs<RPR_REAL> *, int, const Geom &,
                                                                 const OnchipShape &, int, hipStream_t);

template <int KIND, typename T>
struct ChainLauncher {
    const ChainArgs<T> &a;
    const OnchipShape &sh;
    int nwg;
    hipStream_t st;
    int *max_wg;  // out: co-resident work-groups (query mode when non-null)

    template <int CPT, bool DBUF, bool FULL, int NX, int NY, int MAXT>
    rpr_status run()
    {
        if (a.mode == CHAIN_RANDNET_NN) return run_kern<CPT, DBUF, FULL, NX, NY, MAXT, true>();
        return run_kern<CPT, DBUF, FULL, NX, NY, MAXT, false>();
    }

    template <int CPT, bool DBUF, bool FULL, int NX, int NY, int MAXT, bool NN_OK>
    rpr_status run_kern()
    {
        auto kern = k_chain<KIND, T, CPT, DBUF, FULL, NX, NY, MAXT, NN_OK>;
        static bool attr_set = false;
        if (!attr_set) {
            RPR_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)kMaxLds));
            attr_set = true;
        }
        const size_t lds = chain_lds(sh, a.M);
        if (max_wg) {
            int per_cu = 0, dev = 0, cus = 0;
            RPR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, sh.block, lds));
            RPR_HIP(hipGetDevice(&dev));
            RPR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            *max_wg = per_cu * cus;
            return RPR_OK;
        }
        void *args[] = {(void *)&a};
        RPR_HIP(hipLaunchCooperativeKernel((const void *)kern, dim3(nwg), dim3(sh.block), args, lds, st));
        return RPR_OK;
    }
};

template <int KIND, typename T>
rpr_status launch_chain_kind(const ChainArgs<T> &a, const OnchipShape &sh, int nwg, hipStream_t st,
                             int *max_wg)
{
    if (sh.maxt == GENERIC_THREADS) {
        auto kern = k_chain_generic<KIND, T>;
        static bool attr_set = false;
        if (!attr_set) {
            RPR_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)kMaxLds));
            attr_set = true;
        }
        const size_t lds = chain_lds(sh, a.M);
        if (max_wg) {
            int per_cu = 0, dev = 0, cus = 0;
            RPR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, GENERIC_BLOCK, lds));
            RPR_HIP(hipGetDevice(&dev));
            RPR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            *max_wg = per_cu * cus;
            return RPR_OK;
        }
        void *args[] = {(void *)&a};
        RPR_HIP(hipLaunchCooperativeKernel((const void *)kern, dim3(nwg), dim3(GENERIC_BLOCK), args, lds, st));
        return RPR_OK;
    }
    if constexpr (KIND == RPR_BRUSS3D) {
        return fail(RPR_ERR_UNSUPPORTED, "the 3D system takes the generic chain only");
    } else {
    if (sh.maxt == TILED_THREADS) {
        if constexpr (KIND == RPR_BURGERS1D) {
            return fail(RPR_ERR_UNSUPPORTED, "the tiled chain serves 2D grids only");
        } else {
            auto kern = k_chain_tiled<KIND, T>;
            static bool attr_set = false;
            if (!attr_set) {
                RPR_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)kMaxLds));
                attr_set = true;
            }
            const size_t lds = chain_lds(sh, a.M);
            if (max_wg) {
                int per_cu = 0, dev = 0, cus = 0;
                RPR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, TT_THREADS, lds));
                RPR_HIP(hipGetDevice(&dev));
                RPR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
                *max_wg = per_cu * cus;
                return RPR_OK;
            }
            void *args[] = {(void *)&a};
            RPR_HIP(hipLaunchCooperativeKernel((const void *)kern, dim3(nwg), dim3(TT_THREADS), args, lds, st));
            return RPR_OK;
        }
    }
    ChainLauncher<KIND, T> L{a, sh, nwg, st, max_wg};
    return visit_shape_kind<KIND, T>(a.g, sh, L);
    }
}

// The k = 0 sweep of a grid-wide coarse solver as one kernel per pass:
// U_i = G(U_{i-1}) and Gc_i, i = 1..N, pass `pass` of slot i on the plan's
// grid (the arithmetic of the cooperative sweep's CHAIN_SWEEP mode, the
// kernel boundaries as its barriers).
template <int KIND, typename T, int MAXT, int CM>
__global__ __launch_bounds__(MAXT) void k_sweep_pass(ChainArgs<T> a, int i, long long pass)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const size_t d = a.g.d;
    coarse_pass<KIND, T, CM>(a, a.U + (size_t)(i - 1) * d, a.U + (size_t)i * d, a.Gc + (size_t)i * d, pass,
                             blockIdx.x, gridDim.x, reinterpret_cast<T *>(lds_raw));
}

template <int KIND, typename T>
rpr_status launch_sweep_segments_kind(const ChainArgs<T> &a, const OnchipShape &sh, int nwg, hipStream_t st)
{
    auto run = [&](auto kern, int block, long long passes) -> rpr_status {
        static bool attr_set = false;
        if (!attr_set) {
            RPR_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)kMaxLds));
            attr_set = true;
        }
        const size_t lds = chain_lds(sh, a.M);
        for (int i = 1; i <= a.N; ++i)
            for (long long pass = 0; pass < passes; ++pass)
                hipLaunchKernelGGL(kern, dim3(nwg), dim3(block), lds, st, a, i, pass);
        RPR_HIP(hipGetLastError());
        return RPR_OK;
    };
    if (sh.maxt == GENERIC_THREADS)
        return run(k_sweep_pass<KIND, T, GENERIC_BLOCK, CM_GENERIC>, GENERIC_BLOCK,
                   coarse_passes(CM_GENERIC, a.G_method, a.G_steps, a.tbG.s));
    if constexpr (KIND == RPR_BURGERS1D || KIND == RPR_BRUSS3D) {
        return fail(RPR_ERR_UNSUPPORTED, "sweep segments: no grid-wide coarse solver of this form");
    } else {
        if (sh.maxt != TILED_THREADS)
            return fail(RPR_ERR_UNSUPPORTED, "sweep segments: the on-chip coarse solver runs in one work-group");
        if (sh.block == SWEEP_WIDE && a.G_method == RPR_RK1)
            return run(k_sweep_pass<KIND, T, SWEEP_WIDE, CM_TILED_EULER>, SWEEP_WIDE,
                       coarse_passes(CM_TILED, a.G_method, a.G_steps, a.tbG.s));
        return run(k_sweep_pass<KIND, T, TT_THREADS, CM_TILED>, TT_THREADS,
                   coarse_passes(CM_TILED, a.G_method, a.G_steps, a.tbG.s));
    }
}

template rpr_status launch_sweep_segments_kind<RPR_KIND, RPR_REAL>(const ChainArgs<RPR_REAL> &, const OnchipShape &,
                                                                   int, hipStream_t);

// A sweep as a sequence of segment kernels (for capture in a graph): the
// prologue, per slot i = 2..N phase 1 (the tiled coarse solver's passes) and
// phase 2, then the stopping rule, each on nwg work-groups.
template <int KIND, typename T>
struct ChainSegLauncher {
    const ChainArgs<T> *args;
    const ChainArgs<T> &a;  // host copy: sizes, propagator, mode
    const OnchipShape &sh;
    int nwg;
    hipStream_t st;

    template <typename K>
    rpr_status sequence(K kern, int block, size_t lds, long long passes)
    {
        static bool attr_set = false;
        if (!attr_set) {
            RPR_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)kMaxLds));
            attr_set = true;
        }
        hipLaunchKernelGGL(kern, dim3(nwg), dim3(block), lds, st, args, 0, 0, 0LL);
        for (int i = 2; i <= a.N; ++i) {
            for (long long pass = 0; pass < passes; ++pass)
                hipLaunchKernelGGL(kern, dim3(nwg), dim3(block), lds, st, args, 1, i, pass);
            hipLaunchKernelGGL(kern, dim3(nwg), dim3(block), lds, st, args, 2, i, 0LL);
        }
        hipLaunchKernelGGL(kern, dim3(nwg), dim3(block), lds, st, args, 3, 0, 0LL);
        RPR_HIP(hipGetLastError());
        return RPR_OK;
    }

    template <int CPT, bool DBUF, bool FULL, int NX, int NY, int MAXT>
    rpr_status run()
    {
        const size_t lds = chain_lds(sh, a.M);
        if (a.mode == CHAIN_RANDNET_NN)
            return sequence(k_chain_seg<KIND, T, CPT, DBUF, FULL, NX, NY, MAXT, CM_ONCHIP, true>, sh.block, lds, 1);
        return sequence(k_chain_seg<KIND, T, CPT, DBUF, FULL, NX, NY, MAXT, CM_ONCHIP, false>, sh.block, lds, 1);
    }
};

template <int KIND, typename T>
rpr_status launch_chain_graph_kind(const ChainArgs<T> *args_dev, const ChainArgs<T> &a, const OnchipShape &sh,
                                   int nwg, hipStream_t st)
{
    ChainSegLauncher<KIND, T> L{args_dev, a, sh, nwg, st};
    if (sh.maxt == GENERIC_THREADS)
        return L.sequence(k_chain_seg<KIND, T, 1, false, false, 0, 0, GENERIC_BLOCK, CM_GENERIC, true>,
                          GENERIC_BLOCK, chain_lds(sh, a.M), coarse_passes(CM_GENERIC, a.G_method, a.G_steps, a.tbG.s));
    if constexpr (KIND == RPR_BRUSS3D) {
        return fail(RPR_ERR_UNSUPPORTED, "the 3D system takes the generic chain only");
    } else {
        if (sh.maxt == TILED_THREADS) {
            if constexpr (KIND == RPR_BURGERS1D) {
                return fail(RPR_ERR_UNSUPPORTED, "the tiled chain serves 2D grids only");
            } else {
                // work-groups of TT_THREADS, or for a forward-Euler G of
                // SWEEP_WIDE threads (four times the wavefronts per CU for
                // the latency-bound coarse passes and the readout's loads)
                const long long passes = coarse_passes(CM_TILED, a.G_method, a.G_steps, a.tbG.s);
                if (sh.block == SWEEP_WIDE && a.G_method == RPR_RK1)
                    return L.sequence(k_chain_seg<KIND, T, 1, false, false, 0, 0, SWEEP_WIDE, CM_TILED_EULER, true>,
                                      SWEEP_WIDE, chain_lds(sh, a.M), passes);
                return L.sequence(k_chain_seg<KIND, T, 1, false, false, 0, 0, TT_THREADS, CM_TILED, true>,
                                  TT_THREADS, chain_lds(sh, a.M), passes);
            }
        }
        return visit_shape_kind<KIND, T>(a.g, sh, L);
    }
}

template rpr_status launch_chain_graph_kind<RPR_KIND, RPR_REAL>(const ChainArgs<RPR_REAL> *, const ChainArgs<RPR_REAL> &,
                                                                 const OnchipShape &, int, hipStream_t);

// This file is compiled once per (right-hand side, precision) pair.
template rpr_status launch_chain_kind<RPR_KIND, RPR_REAL>(const ChainArgs<RPR_REAL> &, const OnchipShape &,
                                                           int, hipStream_t, int *);

}  // namespace rpr
