// plan.h -- internal: the plan object behind the C ABI (include/rpr.h) and the
// phases of a solve shared by single and batched plans.  Not part of the ABI.
#pragma once

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "chain.h"
#include "common.h"
#include "randnet.h"
#include "slotprop.h"
#include "tiledprop.h"

namespace rpr {

inline bool is_finite(double v) { return std::isfinite(v); }
// The calling thread's last error message (api.hip).
std::string &err_text();
rpr_status check_device();
rpr_status check_prop(const rpr_propagator *P, const char *name);

template <typename TI, typename TO>
__global__ void k_convert(const TI *__restrict__ in, TO *__restrict__ out, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = TO(in[i]);
}

template <typename TI, typename TO>
inline rpr_status convert(const TI *in, TO *out, size_t n, hipStream_t st)
{
    if (n == 0) return RPR_OK;
    hipLaunchKernelGGL((k_convert<TI, TO>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}

template <typename T>
__global__ void k_zero(T *p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = T(0);
}

template <typename T>
inline rpr_status zero(T *p, size_t n, hipStream_t st)
{
    if (n == 0) return RPR_OK;
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}

// control block reset and the u0 check (api.hip)
rpr_status launch_init_ctrl(Ctrl *c, int *L_hist, double *chg_hist, hipStream_t st);
rpr_status launch_absmax(const Geom &g, const double *u, double *out_max, int *out_bad, hipStream_t st);

// Stability pre-check (stability.hip): bounds on the real and imaginary parts
// of the spectral radius of h's Jacobian at a state with max |u| = umax (and
// largest shallow-water wave speed `speed`), and dt over the largest stable
// step of the method.
void stability_bounds(const Geom &g, double umax, double speed, double *rho_r, double *rho_i);
double stability_ratio(const Geom &g, int method, double dt, double umax, double speed);

}  // namespace rpr

using namespace rpr;

// ------------------------------------------------------------------- plan --
struct rpr_plan {
    Geom g{};
    int N = 0, M = 0, prec = 0, corr = 0, k_max = 0, poll = 2, act = 0;
    double t0 = 0, tN = 0, tol = 0, lambda = 0, scale_opt = 0, dtF = 0, dtG = 0;
    rpr_propagator F{}, G{};
    size_t esz = 8;  // bytes per state element
    // device buffers
    void *U = nullptr, *Fv = nullptr, *Gc = nullptr, *X = nullptr, *Y = nullptr, *gtmp = nullptr;
    double *A = nullptr, *zeta = nullptr, *Phi = nullptr, *fpart = nullptr, *Gm = nullptr, *Lf = nullptr,
           *Lt = nullptr, *Bm = nullptr, *W = nullptr, *phi = nullptr, *part = nullptr, *chg_hist = nullptr,
           *u0max = nullptr;
    int *ok = nullptr, *nrows = nullptr, *L_hist = nullptr, *cfail = nullptr, *u0bad = nullptr;
    uint16_t *Ab = nullptr;   // bf16 copy of A (reduced precision)
    uint16_t *Xb = nullptr;   // bf16 pieces of the training inputs (large-tile feature GEMM)
    double *At = nullptr;     // A^T, d x M (the chain's hidden layer)
    float *Atf = nullptr;     // reduced plans: FP32 copies of A^T and of W for the chain
    float *Wf = nullptr;
    float *fpart32 = nullptr; // split-K partials of the bf16 feature GEMM
    Ctrl *ctrl = nullptr;
    Ctrl *ctrl_host = nullptr;  // pinned
    OnchipShape shF{}, shG{};
    int nwg = 1;
    bool feat_bf16 = false;
    int autotune = 0;
    int use_graph = 0;
    bool seg_sweep = false;             // the sweep as segment kernels (rpr_options.sweep_form)
    int strict = 0;                     // opt.stability: 1 rejects solves the pre-check finds unstable
    int fvar = 0;                       // tile shape of the fine propagator's one-pass form
    bool fixed_nwg = false;             // opt.chain_wgs set: the autotuner keeps the chain grid
    double stab_F = 0, stab_G = 0;      // pre-check ratios dt / dt_max of the last execute
    hipGraph_t graph = nullptr;         // captured block of `poll` iterations
    hipGraphExec_t graph_exec = nullptr;
    double graph_s = 0.0;               // input scale the captured block was built for
    hipStream_t cap_stream = nullptr;   // private stream the block is captured on
    void *gchain = nullptr;             // device ChainArgs<T> of the captured chain
    double *hpart = nullptr;            // chain: per-work-group hidden-layer partial sums (grid x M)
    // nearest-neighbour correction: the store of every pair (n_cap rows)
    bool nn = false;
    int m_nn = 0, n_cap = 0;
    void *Xs = nullptr, *Ys = nullptr;  // n_cap x d states
    double *Ps = nullptr;               // n_cap x M features
    int *oks = nullptr;                 // n_cap finite flags
    double *dist = nullptr;             // n_cap squared distances of the current slot input
    double *dpart = nullptr;            // chain grid x n_cap partial distances
    void *fwork = nullptr;              // tiled F: u, acc, ya, yb, cmp (N x d each)
    void *gwork = nullptr;              // tiled coarse solver: u, acc, ya, yb, cmp (d each)
    std::vector<double> bscale;         // batch: input scales the captured block was built for
    // batch plans: one sub-plan per instance plus the shared persistent fine solve
    std::vector<rpr_plan *> sub;
    void *binsts = nullptr;   // device BatchInst<T>[n_inst]
    int2 *bitems = nullptr;   // device (instance, slot) items, longest first
    int bn_items = 0;
    int *bcounter = nullptr;
    void *bchain = nullptr;   // device ChainArgs<T>[n_inst]
    std::vector<char> hchain; // host staging of the chain arguments
    Geom bgmax{};
    OnchipShape bshF{}, bshG{};
    int bgrid = 0, bM = 0, bkmax = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> pev;  // phase boundaries of a burst of iterations (1 + 3 per iteration)
    rpr_info info{};
    std::vector<int> Lh;
    std::vector<double> ch;
};

// Work arrays of the tiled propagator carved from one block of n x 5 values.

#define RPR_TRY(expr)                          \
    do {                                       \
        rpr_status s_ = (expr);                \
        if (s_ != RPR_OK) return s_;           \
    } while (0)

template <typename T>
inline TiledWork<T> tiled_work(void *base, size_t n)
{
    if (!base) return TiledWork<T>{};
    T *b = static_cast<T *>(base);
    return TiledWork<T>{b, b + n, b + 2 * n, b + 3 * n, sizeof(T) == 4 ? b + 4 * n : nullptr};
}

// Elements of the work arrays of a propagator of shape sh and method over n
// states of d values (tiled: u, acc, ya, yb, cmp; generic: rkgen_work), or 0.
inline size_t work_elems(const OnchipShape &sh, int method, size_t n, size_t d)
{
    if (sh.maxt == GENERIC_THREADS) return rkgen_work_elems(method, n, d);
    if (sh.maxt == TILED_THREADS) return 5 * n * d;
    return 0;
}

// Releases every buffer of the plan (and of a batch's instances).
void plan_free(rpr_plan *p);

template <typename B>
inline rpr_status dalloc(B **ptr, size_t count)
{
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, count * sizeof(B) > 0 ? count * sizeof(B) : 8);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    *ptr = static_cast<B *>(q);
    return RPR_OK;
}

// Work arrays of the plan's fine (N states) and coarse (one state)
// propagators in their forms (empty for the on-chip form).
template <typename T>
inline TiledWork<T> fine_work(const rpr_plan *p)
{
    const size_t N = p->N, d = p->g.d;
    if (!p->fwork) return TiledWork<T>{};
    return p->shF.maxt == GENERIC_THREADS ? rkgen_work<T>(p->fwork, N, d) : tiled_work<T>(p->fwork, N * d);
}
template <typename T>
inline TiledWork<T> coarse_work(const rpr_plan *p)
{
    const size_t d = p->g.d;
    if (!p->gwork) return TiledWork<T>{};
    return p->shG.maxt == GENERIC_THREADS ? rkgen_work<T>(p->gwork, 1, d) : tiled_work<T>(p->gwork, d);
}

// The chain's weights in state precision: FP64 plans read W and A^T
// themselves, reduced plans their FP32 copies.
template <typename T>
inline const T *chain_W(const rpr_plan *p)
{
    if constexpr (sizeof(T) == 8) return p->W;
    else return p->Wf;
}
template <typename T>
inline const T *chain_At(const rpr_plan *p)
{
    if constexpr (sizeof(T) == 8) return p->At;
    else return p->Atf;
}

// Chain mode of a plan's iterations.
inline int chain_mode(const rpr_plan *p)
{
    if (p->nn) return CHAIN_RANDNET_NN;
    return p->corr == RPR_CORR_RANDNET ? CHAIN_RANDNET : CHAIN_PARAREAL;
}

// The nearest-neighbour store in the chain's arguments.
template <typename T>
inline void nn_args(const rpr_plan *p, ChainArgs<T> &a)
{
    a.m_nn = p->m_nn;
    a.lambda = p->lambda;
    a.Xs = static_cast<const T *>(p->Xs);
    a.Ys = static_cast<const T *>(p->Ys);
    a.Ps = p->Ps;
    a.oks = p->oks;
    a.nrows = p->nrows;
    a.n_cap = p->n_cap;
    a.dpart = p->dpart;
    a.dist = p->dist;
}

// ---- autotuner (autotune.hip) ----
// Work-group size the autotuner chose for this propagator class (1024 when
// it has not run for it).
int tuned_prop_threads(const Geom &g, int esz, int method);
// Tile shape of the one-pass RK4 form it chose (0 when it has not run).
int tuned_variant(const Geom &g, int esz, int method);
// Times the candidate launch shapes of plan p and keeps the fastest.
template <typename T>
rpr_status autotune_plan(rpr_plan *p, int max_wg, int cus);

// Times the persistent fine-solve launch of batch p over 1 to 4 work-groups
// per CU and keeps the fastest in p->bgrid.
template <typename T>
rpr_status autotune_batch(rpr_plan *p, int cus);

// ---- phases of a solve (shared by single and batched plans) ----
template <typename T>
inline ChainArgs<T> chain_args(rpr_plan *p, double s)
{
    ChainArgs<T> a{};
    a.g = p->g;
    a.N = p->N;
    a.M = p->M;
    a.act = p->act;
    a.k_max = p->k_max;
    a.G_method = p->G.method;
    a.G_steps = p->G.steps;
    a.dtG = p->dtG;
    a.inv_s = 1.0 / s;
    a.eps = p->tol;
    a.U = static_cast<T *>(p->U);
    a.Fv = static_cast<T *>(p->Fv);
    a.Gc = static_cast<T *>(p->Gc);
    a.gtmp = static_cast<T *>(p->gtmp);
    a.phi = p->phi;
    a.hpart = p->hpart;
    a.gw = coarse_work<T>(p);
    a.tbG = rk_tableau(p->G.method);
    a.A = p->A;
    a.zeta = p->zeta;
    a.W = chain_W<T>(p);
    a.At = chain_At<T>(p);
    a.part = p->part;
    a.ctrl = p->ctrl;
    a.L_hist = p->L_hist;
    a.chg_hist = p->chg_hist;
    a.mode = chain_mode(p);
    nn_args<T>(p, a);
    return a;
}

// max |u0| and the non-finite flag (enqueued; read after a stream sync)
// Stability pre-check from the u0 check's results (umax2 = {max |u0|,
// largest shallow-water wave speed}): ratios of F and G kept for rpr_info;
// RPR_ERR_UNSTABLE in strict mode when either exceeds 1.
inline rpr_status stability_gate(rpr_plan *p, const double *umax2)
{
    p->stab_F = stability_ratio(p->g, p->F.method, p->dtF, umax2[0], umax2[1]);
    p->stab_G = stability_ratio(p->g, p->G.method, p->dtG, umax2[0], umax2[1]);
    if (p->strict && (p->stab_F > 1.0 || p->stab_G > 1.0))
        return fail(RPR_ERR_UNSTABLE, "stability pre-check: dt / dt_max = " + std::to_string(p->stab_F) + " (F), " +
                                          std::to_string(p->stab_G) + " (G) at u0");
    return RPR_OK;
}

inline rpr_status phase_check_u0(rpr_plan *p, const double *u0, hipStream_t st)
{
    return launch_absmax(p->g, u0, p->u0max, p->u0bad, st);
}

// input scale (Algorithm "Parareal (generic)", initialisation), control block,
// U_0 = u0, zeroed ridge statistics, coarse sweep (left to the caller with
// sweep = false: a batch sweeps all its instances in one launch)
template <typename T>
inline rpr_status phase_setup(rpr_plan *p, const double *u0, double umax, hipStream_t st, ChainArgs<T> *out,
                              bool sweep = true)
{
    double s = p->scale_opt;
    if (!(s > 0)) {
        s = 1.0;
        while (s < umax) s *= 2.0;
    }
    p->info = rpr_info{};
    p->info.input_scale = s;
    p->info.stab_F = p->stab_F;
    p->info.stab_G = p->stab_G;
    p->info.unstable = (p->stab_F > 1.0 ? 1 : 0) | (p->stab_G > 1.0 ? 2 : 0);
    RPR_TRY(launch_init_ctrl(p->ctrl, p->L_hist, p->chg_hist, st));
    RPR_TRY((convert<double, T>(u0, static_cast<T *>(p->U), (size_t)p->g.d, st)));
    if (p->corr == RPR_CORR_RANDNET) {
        RPR_TRY(zero(p->Gm, (size_t)p->M * p->M, st));
        RPR_TRY(zero(p->Bm, (size_t)p->M * p->g.d, st));
    }
    ChainArgs<T> a = chain_args<T>(p, s);
    a.mode = CHAIN_SWEEP;
    // on chip the sweep's state stays in one work-group; the tiled and
    // generic coarse solvers spread each slot's tiles or cells over the plan's
    // grid, in one cooperative kernel or one kernel per pass
    const bool grid = p->shG.maxt == TILED_THREADS || p->shG.maxt == GENERIC_THREADS;
    if (sweep && grid && p->seg_sweep) RPR_TRY(launch_sweep_segments<T>(a, p->shG, p->nwg, st));
    else if (sweep) RPR_TRY(launch_chain<T>(a, p->shG, grid ? p->nwg : 1, st));
    a.mode = chain_mode(p);
    *out = a;
    return RPR_OK;
}

// training pairs, hidden layer, ridge statistics and solve of one iteration
template <typename T>
inline rpr_status phase_model(rpr_plan *p, double inv_s, hipStream_t st)
{
    if (p->corr != RPR_CORR_RANDNET && !p->nn) return RPR_OK;
    const int N = p->N, d = p->g.d, M = p->M;
    T *U = static_cast<T *>(p->U), *Fv = static_cast<T *>(p->Fv), *Gc = static_cast<T *>(p->Gc);
    T *X = static_cast<T *>(p->X), *Y = static_cast<T *>(p->Y);
    RPR_TRY(launch_pairs<T>(N, d, U, Fv, Gc, X, Y, p->ok, p->nrows, p->ctrl, st));
    if (p->Ab)
        RPR_TRY(launch_features_bf16<T>(N, M, d, p->act, inv_s, p->Ab, p->zeta, X, p->Phi, p->fpart32, p->nrows, st,
                                        p->Xb));
    else
        RPR_TRY(launch_features<T>(N, M, d, p->act, inv_s, p->A, p->zeta, X, p->Phi, p->fpart, p->nrows, st));
    if (p->nn)
        return launch_nn_append<T>(N, d, M, X, Y, p->Phi, p->ok, p->nrows, p->ctrl, static_cast<T *>(p->Xs),
                                   static_cast<T *>(p->Ys), p->Ps, p->oks, p->n_cap, st);
    RPR_TRY(launch_stats<T>(N, M, d, p->Phi, Y, p->ok, p->Gm, p->Bm, p->nrows, st));
    RPR_TRY(launch_ridge_solve(M, d, p->Gm, p->lambda, p->Lf, p->Lt, p->W, p->Bm, p->cfail, &p->ctrl->chol_fail,
                               &p->ctrl->done, st));
    if constexpr (sizeof(T) == 4) RPR_TRY((convert<double, float>(p->W, p->Wf, (size_t)M * d, st)));
    return RPR_OK;
}

// results after the final stream synchronisation
template <typename T>
inline rpr_status phase_finish(rpr_plan *p, double *U_out, float ms, hipStream_t st)
{
    const Ctrl &c = *p->ctrl_host;
    const int N = p->N;
    RPR_TRY((convert<T, double>(static_cast<T *>(p->U), U_out, (size_t)(N + 1) * p->g.d, st)));
    p->info.K = c.k;
    p->info.L_final = c.L;
    p->info.converged = c.L >= N;
    p->info.rows_used = c.rows_used;
    p->info.nonfinite_rows = c.nonfinite;
    p->info.chol_fail = c.chol_fail;
    p->info.t_total = ms * 1e-3;
    p->info.t_fine = p->info.t_model = p->info.t_sweep = -1.0;
    p->Lh.assign(N + 1, 0);
    p->ch.assign(N + 1, 0.0);
    RPR_HIP(hipMemcpyAsync(p->Lh.data(), p->L_hist, sizeof(int) * (c.k + 1), hipMemcpyDeviceToHost, st));
    RPR_HIP(hipMemcpyAsync(p->ch.data(), p->chg_hist, sizeof(double) * (c.k + 1), hipMemcpyDeviceToHost, st));
    return RPR_OK;
}

// Records what `enqueue` puts on the plan's capture stream as the plan's
// graph, replacing the previous one.  Nothing runs during the capture.
template <typename F>
inline rpr_status capture_block(rpr_plan *p, F enqueue)
{
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    RPR_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed));
    const rpr_status cap = enqueue();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
    if (cap != RPR_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return cap != RPR_OK ? cap : hip_fail(e, "hipStreamEndCapture");
    }
    p->graph = graph;
    RPR_HIP(hipGraphInstantiate(&p->graph_exec, graph, nullptr, nullptr, 0));
    return RPR_OK;
}

