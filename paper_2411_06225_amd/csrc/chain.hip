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
// coarse propagator on chip while the other work-groups compute the hidden
// layer sigma(A x / s + zeta), one neuron per work-group at a time (both need
// only U_{i-1}); after a grid barrier every work-group applies the readout,
// the update and the change norm to its own block of columns; a second grid
// barrier publishes U_i.  The converged-slot counter L and the done flag live
// in the device control block, so the host never waits on the sweep.
#include <hip/hip_cooperative_groups.h>

#include "chain.h"
#include "slotprop.h"

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

// One sweep of one instance.  wg / nwg: this work-group and the number of
// work-groups sharing the instance; sync(): a barrier over those work-groups
// (a grid barrier, or a work-group barrier when nwg == 1).
template <int KIND, typename T, int CPT, bool DBUF, bool FULL, int NX, int NY, typename Sync>
__device__ __forceinline__ void chain_body(const ChainArgs<T> &a, const int wg, const int nwg, Sync sync,
                                           unsigned char *lds_raw)
{
    T *lds = reinterpret_cast<T *>(lds_raw);
    double *scratch = reinterpret_cast<double *>(lds_raw);
    const int t = threadIdx.x, B = blockDim.x;
    const Geom &g = a.g;
    const int d = g.d;
    Ctrl *ctrl = a.ctrl;

    if (a.mode == CHAIN_SWEEP) {
        // k = 0 (single work-group): the state stays on chip from slot to slot
        if (wg != 0) return;
        for (int i = 1; i <= a.N; ++i) {
            slot_propagate<KIND, T, CPT, DBUF, FULL, NX, NY>(g, a.G_method, a.G_steps, a.dtG,
                                                             a.U + (size_t)(i - 1) * d, a.U + (size_t)i * d,
                                                             lds, a.Gc + (size_t)i * d);
            __syncthreads();
        }
        return;
    }

    if (ctrl->done) return;  // same value in every work-group: nobody reaches a barrier
    const int L = ctrl->L;
    const int N = a.N;

    // columns of this work-group
    const int chunk = (d + nwg - 1) / nwg;
    const int j0 = wg * chunk, j1 = min(d, j0 + chunk);

    // exact slot
    for (int j = j0 + t; j < j1; j += B) a.U[(size_t)(L + 1) * d + j] = a.Fv[(size_t)(L + 1) * d + j];
    sync();

    const bool net = a.mode == CHAIN_RANDNET;
    for (int i = L + 2; i <= N; ++i) {
        const T *x = a.U + (size_t)(i - 1) * d;
        // ---- phase 1: coarse solve (work-group 0) and hidden layer (the others)
        if (wg == 0) {
            slot_propagate<KIND, T, CPT, DBUF, FULL, NX, NY>(g, a.G_method, a.G_steps, a.dtG, x, a.gtmp, lds);
            __syncthreads();
        }
        if (net && (wg > 0 || nwg == 1)) {
            const int first = nwg == 1 ? 0 : wg - 1, step = nwg == 1 ? 1 : nwg - 1;
            for (int m = first; m < a.M; m += step) {
                if (a.Ab != nullptr) {
                    // reduced precision: bf16 weights and inputs, FP32 sums and sigma, bf16 output
                    const uint16_t *Am = a.Ab + (size_t)m * d;
                    const float xs = (float)a.inv_s;
                    float part = 0.0f;
                    for (int j = t; j < d; j += B)
                        part = fmaf(from_bf16(Am[j]), from_bf16(to_bf16(float(x[j]) * xs)), part);
                    const float z = block_sum_f(part, reinterpret_cast<float *>(scratch)) + (float)a.zeta[m];
                    const float sg = a.act == RPR_RELU ? (z > 0.0f ? z : 0.0f) : tanhf(z);
                    if (t == 0) a.phi[m] = (double)from_bf16(to_bf16(sg));
                } else {
                    const double *Am = a.A + (size_t)m * d;
                    double part = 0.0;
                    for (int j = t; j < d; j += B) part = fma(Am[j], double(x[j]) * a.inv_s, part);
                    const double z = block_sum(part, scratch) + a.zeta[m];
                    if (t == 0) a.phi[m] = a.act == RPR_RELU ? (z > 0.0 ? z : 0.0) : tanh(z);
                }
            }
        }
        sync();

        // ---- phase 2: readout, update and change norm on this block of columns
        double emax = 0.0;
        const T *Fvi = a.Fv + (size_t)i * d;
        T *Ui = a.U + (size_t)i * d;
        T *Gci = a.Gc + (size_t)i * d;
        if (net) {
            double *sphi = scratch;            // M
            double *red = scratch + a.M;       // B
            for (int m = t; m < a.M; m += B) sphi[m] = a.phi[m];
            __syncthreads();
            // width-cw column tiles; each column's sum split over B / cw neuron groups
            const int cw = (j1 - j0) < 64 ? ((j1 - j0) > 0 ? (j1 - j0) : 1) : 64;
            const int groups = B / cw;
            const int jj = t % cw, mg = t / cw;
            for (int jb = j0; jb < j1; jb += cw) {
                const int j = jb + jj;
                double acc = 0.0;
                if (mg < groups && j < j1)
                    for (int m = mg; m < a.M; m += groups) acc = fma(a.W[(size_t)m * d + j], sphi[m], acc);
                if (mg < groups) red[mg * cw + jj] = acc;
                __syncthreads();
                if (mg == 0 && j < j1) {
                    double c = 0.0;
                    for (int q = 0; q < groups; ++q) c += red[q * cw + jj];
                    const T gv = a.gtmp[j];
                    const T unew = T(double(gv) + c);
                    emax = nan_max(emax, fabs(double(unew) - double(Ui[j])));
                    Ui[j] = unew;
                    Gci[j] = gv;
                }
                __syncthreads();
            }
        } else {
            for (int j = j0 + t; j < j1; j += B) {
                const T gv = a.gtmp[j];
                const T unew = gv + (Fvi[j] - Gci[j]);
                emax = nan_max(emax, fabs(double(unew) - double(Ui[j])));
                Ui[j] = unew;
                Gci[j] = gv;
            }
        }
        // work-group maximum (order-free, NaN already mapped to +inf)
        for (int off = 32; off > 0; off >>= 1) emax = nan_max(emax, __shfl_down(emax, off, 64));
        __syncthreads();
        if ((t & 63) == 0) scratch[t >> 6] = emax;
        __syncthreads();
        if (t == 0) {
            double m = 0.0;
            for (int w = 0; w < (B + 63) / 64; ++w) m = nan_max(m, scratch[w]);
            a.part[(size_t)i * nwg + wg] = m;
        }
        sync();
    }

    // ---- stopping rule (eq. "stop_crit"), work-group 0
    if (wg == 0 && t == 0) {
        double chg = 0.0;
        int Lnew = L + 1;
        bool run = true;
        for (int i = L + 2; i <= N; ++i) {
            double e = 0.0;
            for (int w = 0; w < nwg; ++w) e = nan_max(e, a.part[(size_t)i * nwg + w]);
            chg = nan_max(chg, e);
            if (run && e < a.eps) Lnew = i;
            else run = false;
        }
        const int k = ctrl->k + 1;
        ctrl->k = k;
        ctrl->L = Lnew;
        if (Lnew >= N || k >= a.k_max) ctrl->done = 1;  // converged, or iteration cap reached
        if (a.L_hist) a.L_hist[k] = Lnew;
        if (a.chg_hist) a.chg_hist[k] = chg;
    }
}

template <int KIND, typename T, int CPT, bool DBUF, bool FULL, int NX, int NY, int MAXT>
__global__ __launch_bounds__(MAXT) void k_chain(ChainArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cg::grid_group grid = cg::this_grid();
    chain_body<KIND, T, CPT, DBUF, FULL, NX, NY>(a, blockIdx.x, gridDim.x, [&]() { grid.sync(); }, lds_raw);
}

// Independent instances: work-group b runs the whole sweep of instance b.
template <int KIND, typename T, int CPT, bool DBUF, bool FULL, int NX, int NY, int MAXT>
__global__ __launch_bounds__(MAXT) void k_chain_multi(const ChainArgs<T> *__restrict__ args)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const ChainArgs<T> a = args[blockIdx.x];
    chain_body<KIND, T, CPT, DBUF, FULL, NX, NY>(a, 0, 1, []() { __syncthreads(); }, lds_raw);
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
rpr_status launch_chain_multi_kind(const ChainArgs<T> *args_dev, int n_inst, const Geom &gmax, const OnchipShape &sh,
                                   int M, hipStream_t st)
{
    ChainMultiLauncher<KIND, T> L{args_dev, n_inst, sh, M, st};
    return visit_shape_kind<KIND, T>(gmax, sh, L);
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
        auto kern = k_chain<KIND, T, CPT, DBUF, FULL, NX, NY, MAXT>;
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
    ChainLauncher<KIND, T> L{a, sh, nwg, st, max_wg};
    return visit_shape_kind<KIND, T>(a.g, sh, L);
}

// This file is compiled once per (right-hand side, precision) pair.
template rpr_status launch_chain_kind<RPR_KIND, RPR_REAL>(const ChainArgs<RPR_REAL> &, const OnchipShape &,
                                                           int, hipStream_t, int *);

}  // namespace rpr
