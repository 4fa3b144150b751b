// api.hip -- the C ABI of librpr (include/rpr.h): argument checking, plans,
// the Parareal iteration loop and the building-block entry points.
//
// Iteration loop.  Every kernel of an iteration reads the converged-slot
// counter L and the done flag from the plan's device control block, so the
// host enqueues iterations back to back without waiting; it reads the done
// flag every `poll_every` iterations (one device-to-host copy) and stops
// enqueuing once it is set.  Kernels enqueued after convergence exit at once.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "chain.h"
#include "common.h"
#include "randnet.h"
#include "slotprop.h"

namespace rpr {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

rpr_status fail(rpr_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

rpr_status hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? RPR_ERR_OOM : RPR_ERR_HIP;
}

static bool is_finite(double v) { return std::isfinite(v); }

rpr_status make_geom(const rpr_rhs *h, int32_t d, Geom *g)
{
    if (!h) return fail(RPR_ERR_INVALID_ARG, "rhs is NULL");
    const int ns = nspecies(h->kind);
    if (ns == 0) return fail(RPR_ERR_INVALID_ARG, "rhs.kind is not a known right-hand side");
    if (h->reserved != 0) return fail(RPR_ERR_INVALID_ARG, "rhs.reserved must be 0");
    if (h->nx < 1 || h->ny < 1) return fail(RPR_ERR_INVALID_ARG, "rhs.nx and rhs.ny must be >= 1");
    if (h->kind == RPR_BURGERS1D && h->ny != 1) return fail(RPR_ERR_INVALID_ARG, "1D problem needs ny == 1");
    if ((int64_t)ns * h->nx * h->ny != d)
        return fail(RPR_ERR_INVALID_ARG, "d must equal species * nx * ny (" + std::to_string((int64_t)ns * h->nx * h->ny) + ")");
    const double lx = h->x1 - h->x0, ly = h->y1 - h->y0;
    if (!(lx > 0) || !is_finite(lx)) return fail(RPR_ERR_INVALID_ARG, "rhs domain needs x1 > x0");
    if (h->kind != RPR_BURGERS1D && (!(ly > 0) || !is_finite(ly)))
        return fail(RPR_ERR_INVALID_ARG, "rhs domain needs y1 > y0");
    for (int i = 0; i < 6; ++i)
        if (!is_finite(h->p[i])) return fail(RPR_ERR_INVALID_ARG, "rhs.p must be finite");
    Geom G{};
    G.kind = h->kind;
    G.nx = h->nx;
    G.ny = h->ny;
    G.nc = h->nx * h->ny;
    G.ns = ns;
    G.d = d;
    G.periodic = (h->kind == RPR_BURGERS1D || h->kind == RPR_BRUSS2D) ? 1 : 0;
    const double dx = lx / h->nx, dy = h->kind == RPR_BURGERS1D ? 1.0 : ly / h->ny;
    G.idx2 = 1.0 / (dx * dx);
    G.idy2 = 1.0 / (dy * dy);
    G.i2dx = 1.0 / (2.0 * dx);
    G.idx = 1.0 / dx;
    G.idy = 1.0 / dy;
    for (int i = 0; i < 6; ++i) G.p[i] = h->p[i];
    *g = G;
    return RPR_OK;
}

static rpr_status check_device()
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return fail(RPR_ERR_NO_DEVICE, "no HIP device");
    int dev = 0;
    RPR_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    RPR_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(RPR_ERR_NO_DEVICE, std::string("librpr is built for gfx950, device is ") + prop.gcnArchName);
    return RPR_OK;
}

static rpr_status check_prop(const rpr_propagator *P, const char *name)
{
    if (!P) return fail(RPR_ERR_INVALID_ARG, std::string(name) + " is NULL");
    if (P->method != RPR_RK1 && P->method != RPR_RK4)
        return fail(RPR_ERR_INVALID_ARG, std::string(name) + ".method must be RPR_RK1 or RPR_RK4");
    if (P->reserved != 0) return fail(RPR_ERR_INVALID_ARG, std::string(name) + ".reserved must be 0");
    if (P->steps < 1) return fail(RPR_ERR_INVALID_ARG, std::string(name) + ".steps must be >= 1");
    return RPR_OK;
}

// ------------------------------------------------------------ small kernels --
// max |u| and a non-finite flag over d doubles (one work-group).
__global__ __launch_bounds__(1024) void k_absmax(const double *__restrict__ u, int d, double *out_max,
                                                 int *out_bad)
{
    __shared__ double sm[16];
    __shared__ int sb[16];
    double m = 0.0;
    int bad = 0;
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        const double v = u[j];
        if (!isfinite(v)) bad = 1;
        else m = fmax(m, fabs(v));
    }
    for (int off = 32; off > 0; off >>= 1) {
        m = fmax(m, __shfl_down(m, off, 64));
        bad |= __shfl_down(bad, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sm[threadIdx.x >> 6] = m;
        sb[threadIdx.x >> 6] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mm = 0.0;
        int bb = 0;
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) {
            mm = fmax(mm, sm[w]);
            bb |= sb[w];
        }
        *out_max = mm;
        *out_bad = bb;
    }
}

template <typename TI, typename TO>
__global__ void k_convert(const TI *__restrict__ in, TO *__restrict__ out, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = TO(in[i]);
}

template <typename TI, typename TO>
static rpr_status convert(const TI *in, TO *out, size_t n, hipStream_t st)
{
    if (n == 0) return RPR_OK;
    hipLaunchKernelGGL((k_convert<TI, TO>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}

__global__ void k_init_ctrl(Ctrl *c, int *L_hist, double *chg_hist)
{
    c->L = 0;
    c->k = 0;
    c->done = 0;
    c->rows_used = 0;
    c->nonfinite = 0;
    c->chol_fail = 0;
    L_hist[0] = 0;
    chg_hist[0] = 0.0;
}

template <typename T>
__global__ void k_zero(T *p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = T(0);
}

template <typename T>
static rpr_status zero(T *p, size_t n, hipStream_t st)
{
    if (n == 0) return RPR_OK;
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}

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
    float *fpart32 = nullptr; // split-K partials of the bf16 feature GEMM
    Ctrl *ctrl = nullptr;
    Ctrl *ctrl_host = nullptr;  // pinned
    OnchipShape shF{}, shG{};
    int nwg = 1;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    rpr_info info{};
    std::vector<int> Lh;
    std::vector<double> ch;
};

static void plan_free(rpr_plan *p)
{
    void *bufs[] = {p->U, p->Fv, p->Gc, p->X, p->Y, p->gtmp, p->A, p->zeta, p->Phi, p->fpart, p->Gm, p->Lf,
                    p->Lt, p->Bm, p->W, p->phi, p->part, p->chg_hist, p->u0max, p->ok, p->nrows, p->L_hist,
                    p->cfail, p->u0bad, p->ctrl, p->Ab, p->fpart32};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (p->ctrl_host) (void)hipHostFree(p->ctrl_host);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    delete p;
}

template <typename B>
static rpr_status dalloc(B **ptr, size_t count)
{
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, count * sizeof(B) > 0 ? count * sizeof(B) : 8);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    *ptr = static_cast<B *>(q);
    return RPR_OK;
}

#define RPR_TRY(expr)                          \
    do {                                       \
        rpr_status s_ = (expr);                \
        if (s_ != RPR_OK) return s_;           \
    } while (0)

static rpr_status plan_alloc(rpr_plan *p, const double *A, const double *zeta, uint64_t seed)
{
    const int N = p->N, d = p->g.d, M = p->M;
    const size_t sd = (size_t)(N + 1) * d;
    char *c;
    RPR_TRY(dalloc(&c, sd * p->esz)); p->U = c;
    RPR_TRY(dalloc(&c, sd * p->esz)); p->Fv = c;
    RPR_TRY(dalloc(&c, sd * p->esz)); p->Gc = c;
    RPR_TRY(dalloc(&c, (size_t)d * p->esz)); p->gtmp = c;
    RPR_TRY(dalloc(&p->part, (size_t)(N + 1) * 4096));
    RPR_TRY(dalloc(&p->ctrl, 1));
    RPR_TRY(dalloc(&p->L_hist, N + 1));
    RPR_TRY(dalloc(&p->chg_hist, N + 1));
    RPR_TRY(dalloc(&p->u0max, 1));
    RPR_TRY(dalloc(&p->u0bad, 1));
    if (p->corr == RPR_CORR_RANDNET) {
        RPR_TRY(dalloc(&c, (size_t)N * d * p->esz)); p->X = c;
        RPR_TRY(dalloc(&c, (size_t)N * d * p->esz)); p->Y = c;
        RPR_TRY(dalloc(&p->A, (size_t)M * d));
        RPR_TRY(dalloc(&p->zeta, M));
        RPR_TRY(dalloc(&p->Phi, (size_t)N * M));
        RPR_TRY(dalloc(&p->fpart, (size_t)feat_splits(d) * N * M));
        RPR_TRY(dalloc(&p->Gm, (size_t)M * M));
        RPR_TRY(dalloc(&p->Lf, (size_t)M * M));
        RPR_TRY(dalloc(&p->Lt, (size_t)M * M));
        RPR_TRY(dalloc(&p->Bm, (size_t)M * d));
        RPR_TRY(dalloc(&p->W, (size_t)M * d));
        RPR_TRY(dalloc(&p->phi, M));
        RPR_TRY(dalloc(&p->ok, N));
        RPR_TRY(dalloc(&p->nrows, 1));
        RPR_TRY(dalloc(&p->cfail, 1));
        if (A && zeta) {
            RPR_HIP(hipMemcpy(p->A, A, sizeof(double) * M * d, hipMemcpyHostToDevice));
            RPR_HIP(hipMemcpy(p->zeta, zeta, sizeof(double) * M, hipMemcpyHostToDevice));
        } else {
            RPR_TRY(launch_uniform(seed, 0, (int64_t)M * d, p->A, nullptr));
            RPR_TRY(launch_uniform(seed, (uint64_t)M * d, M, p->zeta, nullptr));
        }
        if (p->prec == RPR_MIXED) {
            RPR_TRY(dalloc(&p->Ab, (size_t)M * d));
            RPR_TRY(dalloc(&p->fpart32, (size_t)feat_bf16_splits(d) * N * M));
            RPR_TRY(launch_to_bf16(p->A, p->Ab, (size_t)M * d, nullptr));
        }
        RPR_HIP(hipDeviceSynchronize());
    }
    void *h = nullptr;
    RPR_HIP(hipHostMalloc(&h, sizeof(Ctrl), hipHostMallocDefault));
    p->ctrl_host = static_cast<Ctrl *>(h);
    RPR_HIP(hipEventCreate(&p->ev0));
    RPR_HIP(hipEventCreate(&p->ev1));
    return RPR_OK;
}

extern "C" const char *rpr_last_error(void) { return g_err.c_str(); }

extern "C" const char *rpr_version(void) { return "rpr 0.1 gfx950"; }

extern "C" rpr_status rpr_plan_create(rpr_plan **plan, const rpr_rhs *h, int32_t d, double t0, double tN,
                                      int32_t N, const rpr_propagator *F, const rpr_propagator *G, double tol,
                                      const rpr_randnet *net, const double *A, const double *zeta,
                                      uint64_t seed, const rpr_options *opt)
{
    if (!plan) return fail(RPR_ERR_INVALID_ARG, "plan is NULL");
    *plan = nullptr;
    Geom g;
    RPR_TRY(make_geom(h, d, &g));
    if (N < 1) return fail(RPR_ERR_INVALID_ARG, "N must be >= 1");
    if (!(is_finite(t0) && is_finite(tN) && tN > t0)) return fail(RPR_ERR_INVALID_ARG, "need finite t0 < tN");
    RPR_TRY(check_prop(F, "F"));
    RPR_TRY(check_prop(G, "G"));
    if (!(tol >= 0)) return fail(RPR_ERR_INVALID_ARG, "tol must be >= 0");
    if (!opt) return fail(RPR_ERR_INVALID_ARG, "opt is NULL");
    if (opt->precision != RPR_FP64 && opt->precision != RPR_MIXED)
        return fail(RPR_ERR_INVALID_ARG, "opt.precision must be RPR_FP64 or RPR_MIXED");
    if (opt->correction != RPR_CORR_RANDNET && opt->correction != RPR_CORR_PARAREAL)
        return fail(RPR_ERR_INVALID_ARG, "opt.correction must be RPR_CORR_RANDNET or RPR_CORR_PARAREAL");
    if (opt->k_max < 0 || opt->k_max > N) return fail(RPR_ERR_INVALID_ARG, "opt.k_max must be in [0, N]");
    if (opt->poll_every < 0) return fail(RPR_ERR_INVALID_ARG, "opt.poll_every must be >= 0");
    const bool use_net = opt->correction == RPR_CORR_RANDNET;
    if (use_net) {
        if (!net) return fail(RPR_ERR_INVALID_ARG, "net is NULL");
        if (net->M < 1 || net->M > 512) return fail(RPR_ERR_INVALID_ARG, "net.M must be in [1, 512]");
        if (net->activation != RPR_TANH && net->activation != RPR_RELU)
            return fail(RPR_ERR_INVALID_ARG, "net.activation must be RPR_TANH or RPR_RELU");
        if (!(net->lambda > 0) || !is_finite(net->lambda)) return fail(RPR_ERR_INVALID_ARG, "net.lambda must be > 0");
        if (!is_finite(net->input_scale)) return fail(RPR_ERR_INVALID_ARG, "net.input_scale must be finite");
        if ((A == nullptr) != (zeta == nullptr)) return fail(RPR_ERR_INVALID_ARG, "pass both A and zeta, or neither");
    }
    RPR_TRY(check_device());

    rpr_plan *p = new rpr_plan();
    p->g = g;
    p->N = N;
    p->t0 = t0;
    p->tN = tN;
    p->F = *F;
    p->G = *G;
    p->tol = tol;
    p->prec = opt->precision;
    p->corr = opt->correction;
    p->k_max = opt->k_max == 0 ? N : opt->k_max;
    p->poll = opt->poll_every == 0 ? 2 : opt->poll_every;
    p->esz = p->prec == RPR_FP64 ? 8 : 4;
    if (use_net) {
        p->M = net->M;
        p->act = net->activation;
        p->lambda = net->lambda;
        p->scale_opt = net->input_scale;
    }
    const double T = (tN - t0) / N;
    p->dtF = T / (double)F->steps;
    p->dtG = T / (double)G->steps;
    if (!onchip_shape(g, p->esz, &p->shF, 1024) || !onchip_shape(g, p->esz, &p->shG, 1024)) {
        delete p;
        return fail(RPR_ERR_UNSUPPORTED, "the slot state does not fit one work-group's LDS in this build");
    }
    if (use_net && (size_t)p->M * 32 * sizeof(double) > kMaxLds) {
        delete p;
        return fail(RPR_ERR_UNSUPPORTED, "net.M too large for the ridge solve");
    }
    rpr_status st = plan_alloc(p, A, zeta, seed);
    if (st != RPR_OK) {
        const std::string keep = g_err;
        plan_free(p);
        g_err = keep;
        return st;
    }
    // chain grid: one work-group when the per-slot readout is small, else as
    // many co-resident work-groups as the device holds (at most one per CU)
    int max_wg = 1;
    if (p->esz == 8) {
        ChainArgs<double> a{};
        a.g = g;
        a.M = p->M;
        st = launch_chain<double>(a, p->shG, 0, nullptr, &max_wg);
    } else {
        ChainArgs<float> a{};
        a.g = g;
        a.M = p->M;
        st = launch_chain<float>(a, p->shG, 0, nullptr, &max_wg);
    }
    if (st != RPR_OK) {
        const std::string keep = g_err;
        plan_free(p);
        g_err = keep;
        return st;
    }
    int dev = 0, cus = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const double work = (double)g.d * (use_net ? p->M : 1);
    int nwg = work < 65536.0 ? 1 : cus;
    if (nwg > max_wg) nwg = max_wg;
    if (nwg > 4096) nwg = 4096;
    p->nwg = nwg < 1 ? 1 : nwg;
    *plan = p;
    return RPR_OK;
}

template <typename T>
static rpr_status execute_impl(rpr_plan *p, const double *u0, double *U_out, hipStream_t st)
{
    const Geom &g = p->g;
    const int N = p->N, d = g.d, M = p->M;
    T *U = static_cast<T *>(p->U), *Fv = static_cast<T *>(p->Fv), *Gc = static_cast<T *>(p->Gc);

    // setup: input checks and scale s (Algorithm "Parareal (generic)", initialisation)
    hipLaunchKernelGGL(k_absmax, dim3(1), dim3(1024), 0, st, u0, d, p->u0max, p->u0bad);
    RPR_HIP(hipGetLastError());
    double umax = 0.0;
    int bad = 0;
    RPR_HIP(hipMemcpyAsync(&umax, p->u0max, sizeof(double), hipMemcpyDeviceToHost, st));
    RPR_HIP(hipMemcpyAsync(&bad, p->u0bad, sizeof(int), hipMemcpyDeviceToHost, st));
    RPR_HIP(hipStreamSynchronize(st));
    if (bad) return fail(RPR_ERR_NONFINITE, "u0 has non-finite entries");
    double s = p->scale_opt;
    if (!(s > 0)) {
        s = 1.0;
        while (s < umax) s *= 2.0;
    }
    p->info = rpr_info{};
    p->info.input_scale = s;

    RPR_HIP(hipEventRecord(p->ev0, st));
    hipLaunchKernelGGL(k_init_ctrl, dim3(1), dim3(1), 0, st, p->ctrl, p->L_hist, p->chg_hist);
    RPR_HIP(hipGetLastError());
    RPR_TRY((convert<double, T>(u0, U, (size_t)d, st)));
    const bool net = p->corr == RPR_CORR_RANDNET;
    if (net) {
        RPR_TRY(zero(p->Gm, (size_t)M * M, st));
        RPR_TRY(zero(p->Bm, (size_t)M * d, st));
    }

    ChainArgs<T> a{};
    a.g = g;
    a.N = N;
    a.M = M;
    a.act = p->act;
    a.G_method = p->G.method;
    a.G_steps = p->G.steps;
    a.dtG = p->dtG;
    a.inv_s = 1.0 / s;
    a.eps = p->tol;
    a.U = U;
    a.Fv = Fv;
    a.Gc = Gc;
    a.gtmp = static_cast<T *>(p->gtmp);
    a.phi = p->phi;
    a.A = p->A;
    a.zeta = p->zeta;
    a.W = p->W;
    a.Ab = p->Ab;
    a.part = p->part;
    a.ctrl = p->ctrl;
    a.L_hist = p->L_hist;
    a.chg_hist = p->chg_hist;

    // k = 0: coarse sweep
    a.mode = CHAIN_SWEEP;
    RPR_TRY(launch_chain<T>(a, p->shG, 1, st));
    a.mode = net ? CHAIN_RANDNET : CHAIN_PARAREAL;

    const int *ctrl_i = reinterpret_cast<const int *>(p->ctrl);
    int k = 0;
    bool done = false;
    while (k < p->k_max && !done) {
        const int burst = (p->k_max - k) < p->poll ? (p->k_max - k) : p->poll;
        for (int b = 0; b < burst; ++b) {
            // fine solves of the slots that are not final: Fv[i] = F(U[i-1])
            RPR_TRY(launch_propagate<T>(g, p->F.method, p->F.steps, p->dtF, N, U, Fv + d, ctrl_i, st,
                                        p->shF.maxt));
            if (net) {
                T *X = static_cast<T *>(p->X), *Y = static_cast<T *>(p->Y);
                RPR_TRY(launch_pairs<T>(N, d, U, Fv, Gc, X, Y, p->ok, p->nrows, p->ctrl, st));
                if (p->Ab)
                    RPR_TRY(launch_features_bf16<T>(N, M, d, p->act, 1.0 / s, p->Ab, p->zeta, X, p->Phi, p->fpart32,
                                                    p->nrows, st));
                else
                    RPR_TRY(launch_features<T>(N, M, d, p->act, 1.0 / s, p->A, p->zeta, X, p->Phi, p->fpart,
                                               p->nrows, st));
                RPR_TRY(launch_stats<T>(N, M, d, p->Phi, Y, p->ok, p->Gm, p->Bm, p->nrows, st));
                RPR_TRY(launch_ridge_solve(M, d, p->Gm, p->lambda, p->Lf, p->Lt, p->W, p->Bm, p->cfail,
                                           &p->ctrl->chol_fail, &p->ctrl->done, st));
            }
            RPR_TRY(launch_chain<T>(a, p->shG, p->nwg, st));
            ++k;
        }
        RPR_HIP(hipMemcpyAsync(p->ctrl_host, p->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        RPR_HIP(hipStreamSynchronize(st));
        done = p->ctrl_host->done != 0;
    }
    RPR_TRY((convert<T, double>(U, U_out, (size_t)(N + 1) * d, st)));
    RPR_HIP(hipEventRecord(p->ev1, st));
    RPR_HIP(hipStreamSynchronize(st));
    float ms = 0.f;
    RPR_HIP(hipEventElapsedTime(&ms, p->ev0, p->ev1));

    const Ctrl &c = *p->ctrl_host;
    p->info.K = c.k;
    p->info.L_final = c.L;
    p->info.converged = c.done;
    p->info.rows_used = c.rows_used;
    p->info.nonfinite_rows = c.nonfinite;
    p->info.chol_fail = c.chol_fail;
    p->info.t_total = ms * 1e-3;
    p->Lh.assign(N + 1, 0);
    p->ch.assign(N + 1, 0.0);
    RPR_HIP(hipMemcpy(p->Lh.data(), p->L_hist, sizeof(int) * (c.k + 1), hipMemcpyDeviceToHost));
    RPR_HIP(hipMemcpy(p->ch.data(), p->chg_hist, sizeof(double) * (c.k + 1), hipMemcpyDeviceToHost));
    return c.done ? RPR_OK : RPR_NOT_CONVERGED;
}

extern "C" rpr_status rpr_plan_execute(rpr_plan *plan, const void *u0, void *U_out, void *stream)
{
    if (!plan) return fail(RPR_ERR_INVALID_ARG, "plan is NULL");
    if (!u0 || !U_out) return fail(RPR_ERR_INVALID_ARG, "u0 and U_out must be device pointers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (plan->esz == 8)
        return execute_impl<double>(plan, static_cast<const double *>(u0), static_cast<double *>(U_out), st);
    return execute_impl<float>(plan, static_cast<const double *>(u0), static_cast<double *>(U_out), st);
}

extern "C" rpr_status rpr_plan_info(const rpr_plan *plan, rpr_info *info)
{
    if (!plan || !info) return fail(RPR_ERR_INVALID_ARG, "plan and info must not be NULL");
    *info = plan->info;
    return RPR_OK;
}

extern "C" rpr_status rpr_plan_history(const rpr_plan *plan, int32_t *L_hist, double *chg_hist, int32_t cap)
{
    if (!plan || cap < 0) return fail(RPR_ERR_INVALID_ARG, "plan must not be NULL and cap >= 0");
    const int n = (int)plan->Lh.size() < cap ? (int)plan->Lh.size() : cap;
    for (int i = 0; i < n; ++i) {
        if (L_hist) L_hist[i] = plan->Lh[i];
        if (chg_hist) chg_hist[i] = plan->ch[i];
    }
    return RPR_OK;
}

extern "C" rpr_status rpr_plan_destroy(rpr_plan *plan)
{
    if (plan) plan_free(plan);
    return RPR_OK;
}

// ------------------------------------------------------- building blocks --
extern "C" rpr_status rpr_propagate(const rpr_rhs *h, int32_t d, const rpr_propagator *P, int32_t precision,
                                    double dt, int32_t n_states, const void *in, void *out, void *stream)
{
    Geom g;
    RPR_TRY(make_geom(h, d, &g));
    RPR_TRY(check_prop(P, "P"));
    if (precision != RPR_FP64 && precision != RPR_MIXED)
        return fail(RPR_ERR_INVALID_ARG, "precision must be RPR_FP64 or RPR_MIXED");
    if (!is_finite(dt)) return fail(RPR_ERR_INVALID_ARG, "dt must be finite");
    if (n_states < 0) return fail(RPR_ERR_INVALID_ARG, "n_states must be >= 0");
    if (n_states == 0) return RPR_OK;
    if (!in || !out) return fail(RPR_ERR_INVALID_ARG, "in and out must be device pointers");
    const size_t bytes = (size_t)n_states * d * (precision == RPR_FP64 ? 8 : 4);
    const char *a = static_cast<const char *>(in), *b = static_cast<const char *>(out);
    if (a < b + bytes && b < a + bytes) return fail(RPR_ERR_INVALID_ARG, "in and out must not overlap");
    RPR_TRY(check_device());
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (precision == RPR_FP64)
        return launch_propagate<double>(g, P->method, P->steps, dt, n_states, static_cast<const double *>(in),
                                        static_cast<double *>(out), nullptr, st);
    return launch_propagate<float>(g, P->method, P->steps, dt, n_states, static_cast<const float *>(in),
                                   static_cast<float *>(out), nullptr, st);
}

extern "C" rpr_status rpr_randnet_features(int32_t M, int32_t d, int32_t n, int32_t activation, double s,
                                           const double *A, const double *zeta, const double *X, double *Phi,
                                           void *stream)
{
    if (M < 1 || d < 1 || n < 0) return fail(RPR_ERR_INVALID_ARG, "need M >= 1, d >= 1, n >= 0");
    if (activation != RPR_TANH && activation != RPR_RELU) return fail(RPR_ERR_INVALID_ARG, "bad activation");
    if (!(s > 0) || !is_finite(s)) return fail(RPR_ERR_INVALID_ARG, "s must be > 0");
    if (n == 0) return RPR_OK;
    if (!A || !zeta || !X || !Phi) return fail(RPR_ERR_INVALID_ARG, "NULL device pointer");
    RPR_TRY(check_device());
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *part = nullptr;
    RPR_HIP(hipMallocAsync((void **)&part, sizeof(double) * feat_splits(d) * n * M, st));
    const rpr_status rc = launch_features<double>(n, M, d, activation, 1.0 / s, A, zeta, X, Phi, part, nullptr, st);
    RPR_HIP(hipFreeAsync(part, st));
    return rc;
}

extern "C" rpr_status rpr_randnet_features_bf16(int32_t M, int32_t d, int32_t n, int32_t activation, double s,
                                                const double *A, const double *zeta, const float *X, double *Phi,
                                                void *stream)
{
    if (M < 1 || d < 1 || n < 0) return fail(RPR_ERR_INVALID_ARG, "need M >= 1, d >= 1, n >= 0");
    if (activation != RPR_TANH && activation != RPR_RELU) return fail(RPR_ERR_INVALID_ARG, "bad activation");
    if (!(s > 0) || !is_finite(s)) return fail(RPR_ERR_INVALID_ARG, "s must be > 0");
    if (n == 0) return RPR_OK;
    if (!A || !zeta || !X || !Phi) return fail(RPR_ERR_INVALID_ARG, "NULL device pointer");
    RPR_TRY(check_device());
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint16_t *Ab = nullptr;
    float *part = nullptr;
    RPR_HIP(hipMallocAsync((void **)&Ab, sizeof(uint16_t) * (size_t)M * d, st));
    RPR_HIP(hipMallocAsync((void **)&part, sizeof(float) * feat_bf16_splits(d) * n * M, st));
    rpr_status rc = launch_to_bf16(A, Ab, (size_t)M * d, st);
    if (rc == RPR_OK) rc = launch_features_bf16<float>(n, M, d, activation, 1.0 / s, Ab, zeta, X, Phi, part, nullptr, st);
    RPR_HIP(hipFreeAsync(Ab, st));
    RPR_HIP(hipFreeAsync(part, st));
    return rc;
}

extern "C" rpr_status rpr_ridge_fit(int32_t M, int32_t d, int32_t n, const double *Phi, const double *Y,
                                    double lambda, double *W, void *stream)
{
    if (M < 1 || M > 512 || d < 1 || n < 0) return fail(RPR_ERR_INVALID_ARG, "need 1 <= M <= 512, d >= 1, n >= 0");
    if (!(lambda > 0) || !is_finite(lambda)) return fail(RPR_ERR_INVALID_ARG, "lambda must be > 0");
    if (!W || (n > 0 && (!Phi || !Y))) return fail(RPR_ERR_INVALID_ARG, "NULL device pointer");
    RPR_TRY(check_device());
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *ws = nullptr;
    const size_t mm = (size_t)M * M, md = (size_t)M * d;
    RPR_HIP(hipMallocAsync((void **)&ws, sizeof(double) * (3 * mm + md) + 64, st));
    double *G = ws, *L = ws + mm, *Lt = ws + 2 * mm, *Bm = ws + 3 * mm;
    int *flag = reinterpret_cast<int *>(ws + 3 * mm + md);
    rpr_status rc = zero(G, mm, st);
    if (rc == RPR_OK) rc = zero(Bm, md, st);
    if (rc == RPR_OK) rc = launch_stats<double>(n, M, d, Phi, Y, nullptr, G, Bm, nullptr, st);
    if (rc == RPR_OK) rc = launch_ridge_solve(M, d, G, lambda, L, Lt, W, Bm, flag, nullptr, nullptr, st);
    int failed = 0;
    if (rc == RPR_OK) {
        RPR_HIP(hipMemcpyAsync(&failed, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    }
    RPR_HIP(hipFreeAsync(ws, st));
    RPR_HIP(hipStreamSynchronize(st));
    if (rc != RPR_OK) return rc;
    if (failed) return fail(RPR_ERR_NOT_SPD, "ridge matrix is not numerically positive definite");
    return RPR_OK;
}

extern "C" rpr_status rpr_randnet_readout(int32_t M, int32_t d, int32_t n, const double *W, const double *Phi,
                                          double *Yhat, void *stream)
{
    if (M < 1 || d < 1 || n < 0) return fail(RPR_ERR_INVALID_ARG, "need M >= 1, d >= 1, n >= 0");
    if (n == 0) return RPR_OK;
    if (!W || !Phi || !Yhat) return fail(RPR_ERR_INVALID_ARG, "NULL device pointer");
    RPR_TRY(check_device());
    return launch_readout(n, M, d, W, Phi, Yhat, static_cast<hipStream_t>(stream));
}

extern "C" rpr_status rpr_uniform_pm1(uint64_t seed, uint64_t first, int64_t n, double *out, void *stream)
{
    if (n < 0) return fail(RPR_ERR_INVALID_ARG, "n must be >= 0");
    if (n == 0) return RPR_OK;
    if (!out) return fail(RPR_ERR_INVALID_ARG, "out is NULL");
    RPR_TRY(check_device());
    return launch_uniform(seed, first, n, out, static_cast<hipStream_t>(stream));
}
