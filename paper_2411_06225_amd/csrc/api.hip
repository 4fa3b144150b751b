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
#include <cstdlib>
#include <cstring>
#include <string>
#include <algorithm>
#include <vector>

#include "chain.h"
#include "tiledprop.h"
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
    if (P->threads != 0 && P->threads != TILED_THREADS && P->threads != 512 && P->threads != 1024)
        return fail(RPR_ERR_INVALID_ARG, std::string(name) + ".threads must be 0, 256, 512 or 1024");
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
    c->nn_rows = 0;
    c->pad = 0;
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
template <typename T>
static TiledWork<T> tiled_work(void *base, size_t n)
{
    if (!base) return TiledWork<T>{};
    T *b = static_cast<T *>(base);
    return TiledWork<T>{b, b + n, b + 2 * n, b + 3 * n, sizeof(T) == 4 ? b + 4 * n : nullptr};
}

static void plan_free(rpr_plan *p)
{
    for (rpr_plan *q : p->sub) plan_free(q);
    p->sub.clear();
    void *bb[] = {p->binsts, p->bitems, p->bcounter, p->bchain, p->hpart, p->fwork, p->gwork,
                  p->Xs, p->Ys, p->Ps, p->oks, p->dist, p->dpart};
    for (void *b : bb)
        if (b) (void)hipFree(b);
    void *bufs[] = {p->U, p->Fv, p->Gc, p->X, p->Y, p->gtmp, p->A, p->zeta, p->Phi, p->fpart, p->Gm, p->Lf,
                    p->Lt, p->Bm, p->W, p->phi, p->part, p->chg_hist, p->u0max, p->ok, p->nrows, p->L_hist,
                    p->cfail, p->u0bad, p->ctrl, p->Ab, p->fpart32, p->At, p->Xb, p->Atf, p->Wf};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (p->ctrl_host) (void)hipHostFree(p->ctrl_host);
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->gchain) (void)hipFree(p->gchain);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    for (hipEvent_t e : p->pev) (void)hipEventDestroy(e);
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
    if (p->shF.maxt == TILED_THREADS) {
        RPR_TRY(dalloc(&c, 5 * (size_t)N * d * p->esz));
        p->fwork = c;
    }
    if (p->shG.maxt == TILED_THREADS) {
        RPR_TRY(dalloc(&c, 5 * (size_t)d * p->esz));
        p->gwork = c;
    }
    RPR_TRY(dalloc(&p->part, (size_t)(N + 1) * 4096));
    RPR_TRY(dalloc(&p->ctrl, 1));
    RPR_TRY(dalloc(&p->L_hist, N + 1));
    RPR_TRY(dalloc(&p->chg_hist, N + 1));
    RPR_TRY(dalloc(&p->u0max, 1));
    RPR_TRY(dalloc(&p->u0bad, 1));
    if (p->corr == RPR_CORR_RANDNET || p->nn) {
        RPR_TRY(dalloc(&c, (size_t)N * d * p->esz)); p->X = c;
        RPR_TRY(dalloc(&c, (size_t)N * d * p->esz)); p->Y = c;
        RPR_TRY(dalloc(&p->A, (size_t)M * d));
        RPR_TRY(dalloc(&p->zeta, M));
        RPR_TRY(dalloc(&p->Phi, (size_t)N * M));
        RPR_TRY(dalloc(&p->fpart, (size_t)feat_splits(d) * N * M));
        if (p->nn) {
            // every pair of the run: at most N per iteration
            p->n_cap = N * p->k_max;
            RPR_TRY(dalloc(&c, (size_t)p->n_cap * d * p->esz)); p->Xs = c;
            RPR_TRY(dalloc(&c, (size_t)p->n_cap * d * p->esz)); p->Ys = c;
            RPR_TRY(dalloc(&p->Ps, (size_t)p->n_cap * M));
            RPR_TRY(dalloc(&p->oks, p->n_cap));
            RPR_TRY(dalloc(&p->dist, p->n_cap));
        } else {
            RPR_TRY(dalloc(&p->Gm, (size_t)M * M));
            RPR_TRY(dalloc(&p->Lf, (size_t)M * M));
            RPR_TRY(dalloc(&p->Lt, (size_t)M * M));
            RPR_TRY(dalloc(&p->Bm, (size_t)M * d));
            RPR_TRY(dalloc(&p->W, (size_t)M * d));
        }
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
        // the chain's hidden layer reads the weights column by column (A^T)
        RPR_TRY(dalloc(&p->At, (size_t)M * d));
        RPR_TRY(launch_transpose<double>(p->A, p->At, M, d, nullptr));
        if (p->esz == 4) {
            // the chain of a reduced plan reads its weights in FP32 (sums in FP64)
            RPR_TRY(dalloc(&p->Atf, (size_t)M * d));
            RPR_TRY((convert<double, float>(p->At, p->Atf, (size_t)M * d, nullptr)));
            if (!p->nn) RPR_TRY(dalloc(&p->Wf, (size_t)M * d));
        }
        if (p->feat_bf16) {
            RPR_TRY(dalloc(&p->Ab, 3 * (size_t)M * d));
            RPR_TRY(dalloc(&p->fpart32, (size_t)feat_bf16_splits(d) * N * M));
            RPR_TRY(launch_to_bf16(p->A, p->Ab, (size_t)M * d, nullptr));
            if (feat_bf16_large(N, d)) RPR_TRY(dalloc(&p->Xb, 3 * (size_t)N * d));
        }
        RPR_HIP(hipDeviceSynchronize());
    }
    void *h = nullptr;
    RPR_HIP(hipHostMalloc(&h, sizeof(Ctrl), hipHostMallocDefault));
    p->ctrl_host = static_cast<Ctrl *>(h);
    RPR_HIP(hipEventCreate(&p->ev0));
    RPR_HIP(hipEventCreate(&p->ev1));
    if (p->use_graph) {
        RPR_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        RPR_HIP(hipMalloc(&p->gchain, sizeof(ChainArgs<double>)));
    }
    return RPR_OK;
}

// The chain's weights in state precision: FP64 plans read W and A^T
// themselves, reduced plans their FP32 copies.
template <typename T>
static const T *chain_W(const rpr_plan *p)
{
    if constexpr (sizeof(T) == 8) return p->W;
    else return p->Wf;
}
template <typename T>
static const T *chain_At(const rpr_plan *p)
{
    if constexpr (sizeof(T) == 8) return p->At;
    else return p->Atf;
}

// Chain mode of a plan's iterations.
static int chain_mode(const rpr_plan *p)
{
    if (p->nn) return CHAIN_RANDNET_NN;
    return p->corr == RPR_CORR_RANDNET ? CHAIN_RANDNET : CHAIN_PARAREAL;
}

// The nearest-neighbour store in the chain's arguments.
template <typename T>
static void nn_args(const rpr_plan *p, ChainArgs<T> &a)
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

// --------------------------------------------------------------- autotuner --
// Candidate launch shapes are timed on the plan's own buffers (zero-filled)
// with events on a private stream; the fastest is kept.  Results are cached
// per shape class in the process and, if RPR_TUNE_CACHE names a file, in that
// JSON file ({"key": value, ...}).
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune;
static bool g_tune_loaded = false;

static void tune_load()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("RPR_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string txt = ss.str();
    size_t pos = 0;
    while ((pos = txt.find('"', pos)) != std::string::npos) {
        const size_t end = txt.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = txt.substr(pos + 1, end - pos - 1);
        const size_t colon = txt.find(':', end);
        if (colon == std::string::npos) break;
        g_tune[key] = std::atoi(txt.c_str() + colon + 1);
        pos = txt.find_first_of(",}", colon);
        if (pos == std::string::npos) break;
    }
}

static void tune_store()
{
    const char *path = std::getenv("RPR_TUNE_CACHE");
    if (!path) return;
    std::ofstream f(path);
    f << "{";
    bool first = true;
    for (const auto &kv : g_tune) {
        f << (first ? "" : ",") << "\n  \"" << kv.first << "\": " << kv.second;
        first = false;
    }
    f << "\n}\n";
}

static std::string prop_key(const Geom &g, int esz, int method)
{
    std::ostringstream k;
    k << "prop:" << g.kind << ":" << g.nx << "x" << g.ny << ":" << esz << ":" << method;
    return k.str();
}

// Work-group size the autotuner chose for this propagator class (1024 when
// it has not run for it).
static int tuned_prop_threads(const Geom &g, int esz, int method)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_load();
    const auto it = g_tune.find(prop_key(g, esz, method));
    return it == g_tune.end() ? 1024 : it->second;
}

// Device memory released when it goes out of scope.
struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

// Trials of the autotuner on its own stream; the caller holds the tuning
// table's lock.
template <typename T>
static rpr_status autotune_run(rpr_plan *p, int max_wg, int cus, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    const Geom &g = p->g;
    const int N = p->N, d = g.d;
    std::ostringstream kc;
    const std::string kf = prop_key(g, p->esz, p->F.method);
    kc << "chain:" << g.kind << ":" << g.nx << "x" << g.ny << ":" << p->esz << ":M" << p->M << ":N" << N << ":"
       << p->corr << ":" << (p->feat_bf16 ? 1 : 0);
    const bool haveF = g_tune.count(kf) != 0, haveC = g_tune.count(kc.str()) != 0;
    T *U = static_cast<T *>(p->U), *Fv = static_cast<T *>(p->Fv), *Gc = static_cast<T *>(p->Gc);
    RPR_TRY(zero(U, (size_t)(N + 1) * d, st));
    RPR_TRY(zero(Fv, (size_t)(N + 1) * d, st));
    RPR_TRY(zero(Gc, (size_t)(N + 1) * d, st));
    if (p->W) RPR_TRY(zero(p->W, (size_t)p->M * d, st));
    if (p->Wf) RPR_TRY(zero(p->Wf, (size_t)p->M * d, st));

    // fine propagator: on chip with 1024-thread (short strips) or 512-thread
    // (long strips) work-groups, or tiled through memory (2D grids)
    const bool forced_tiled = p->shF.maxt == TILED_THREADS;
    if (!haveF && p->F.threads == 0 && !forced_tiled) {
        const int64_t steps = p->F.steps < 32 ? p->F.steps : 32;
        float best = 1e30f;
        int best_mt = p->shF.maxt;
        DevBuf trial;  // work arrays of the tiled candidate
        for (int mt : {1024, 512, TILED_THREADS}) {
            if (check_threads(g, p->esz, mt) != RPR_OK) continue;
            TiledWork<T> w{};
            if (mt == TILED_THREADS) {
                if (hipMalloc(&trial.p, 5 * (size_t)N * d * p->esz) != hipSuccess) {
                    (void)hipGetLastError();
                    trial.p = nullptr;
                    continue;
                }
                w = tiled_work<T>(trial.p, (size_t)N * d);
            }
            const TiledWork<T> *wp = mt == TILED_THREADS ? &w : nullptr;
            RPR_TRY(launch_propagate<T>(g, p->F.method, steps, p->dtF, N, U, Fv + d, nullptr, st, mt, wp));
            float ms = 0.f;
            RPR_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < 3; ++r)
                RPR_TRY(launch_propagate<T>(g, p->F.method, steps, p->dtF, N, U, Fv + d, nullptr, st, mt, wp));
            RPR_HIP(hipEventRecord(e1, st));
            RPR_HIP(hipEventSynchronize(e1));
            RPR_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) { best = ms; best_mt = mt; }
        }
        g_tune[kf] = best_mt;
    }
    if (!forced_tiled) {
        const int mt = p->F.threads ? p->F.threads : g_tune[kf];
        if (mt == TILED_THREADS) {
            p->shF = tiled_shape(g, p->esz);
            if (!p->fwork) {
                char *c = nullptr;
                RPR_TRY(dalloc(&c, 5 * (size_t)N * d * p->esz));
                p->fwork = c;
            }
        } else if (!onchip_shape(g, p->esz, &p->shF, mt)) {
            return fail(RPR_ERR_HIP, "autotune: lost the F shape");
        }
    }

    // chain grid: one work-group, or 1/16, 1/8, a quarter, half or all of the CUs
    if (!haveC) {
        ChainArgs<T> a{};
        a.g = g;
        a.mode = chain_mode(p);
        a.N = N;
        a.M = p->M;
        a.act = p->act;
        a.k_max = N;
        a.G_method = p->G.method;
        a.G_steps = p->G.steps;
        a.dtG = p->dtG;
        a.inv_s = 1.0;
        a.eps = 0.0;
        a.U = U;
        a.Fv = Fv;
        a.Gc = Gc;
        a.gtmp = static_cast<T *>(p->gtmp);
        a.phi = p->phi;
        a.hpart = p->hpart;
        a.gw = tiled_work<T>(p->gwork, (size_t)d);
        a.A = p->A;
        a.zeta = p->zeta;
        a.W = chain_W<T>(p);
        a.At = chain_At<T>(p);
        a.part = p->part;
        a.ctrl = p->ctrl;
        nn_args<T>(p, a);
        if (p->nn) RPR_TRY(zero(p->nrows, 1, st));  // the trials run with an empty store
        float best = 1e30f;
        int best_n = p->nwg, best_gt = p->shG.maxt;
        // coarse-solver shapes: the plan's, and for an on-chip G of free
        // thread count the 512-thread one too (longer strips, twice the
        // registers per thread)
        OnchipShape gshapes[2] = {p->shG, p->shG};
        int n_shapes = 1;
        if (p->G.threads == 0 && p->shG.maxt == 1024 && onchip_shape(g, p->esz, &gshapes[1], 512) &&
            check_threads(g, p->esz, 512) == RPR_OK)
            n_shapes = 2;
        const int cands[] = {1, cus / 16, cus / 8, cus / 4, cus / 2, cus};
        for (int s = 0; s < n_shapes; ++s) {
            const OnchipShape &sh = gshapes[s];
            int mwg = max_wg;  // grids beyond the plan's max_wg have no partial-sum rows
            if (s > 0) {
                int m2 = 0;
                RPR_TRY(launch_chain<T>(a, sh, 0, nullptr, &m2));
                mwg = std::min(mwg, m2);
            }
            for (int c : cands) {
                if (c < 1 || c > mwg) continue;
                if (p->M > 0 && c > 1 && c - 1 > p->M && c != cus) continue;
                // the tiled coarse solver spreads its tiles over the grid: one
                // work-group would take all of them in turn (seconds per sweep)
                if (sh.maxt == TILED_THREADS && c < tiles_of(g)) continue;
                float ms = 0.f;
                hipLaunchKernelGGL(k_init_ctrl, dim3(1), dim3(1), 0, st, p->ctrl, p->L_hist, p->chg_hist);
                RPR_TRY(launch_chain<T>(a, sh, c, st));
                RPR_HIP(hipEventRecord(e0, st));
                hipLaunchKernelGGL(k_init_ctrl, dim3(1), dim3(1), 0, st, p->ctrl, p->L_hist, p->chg_hist);
                RPR_TRY(launch_chain<T>(a, sh, c, st));
                RPR_HIP(hipEventRecord(e1, st));
                RPR_HIP(hipEventSynchronize(e1));
                RPR_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) { best = ms; best_n = c; best_gt = sh.maxt; }
            }
        }
        g_tune[kc.str()] = best_n;
        g_tune[kc.str() + ":G"] = best_gt;
    }
    // the coarse solver's work-group size (tuned only where G's is free)
    const auto gt = g_tune.find(kc.str() + ":G");
    if (p->G.threads == 0 && p->shG.maxt == 1024 && gt != g_tune.end() && gt->second == 512) {
        OnchipShape sh;
        if (onchip_shape(g, p->esz, &sh, 512) && check_threads(g, p->esz, 512) == RPR_OK) {
            int m2 = 0;
            ChainArgs<T> q{};
            q.g = g;
            q.M = p->M;
            q.mode = chain_mode(p);
            RPR_TRY(launch_chain<T>(q, sh, 0, nullptr, &m2));
            if (m2 >= 1) {
                p->shG = sh;
                max_wg = std::min(max_wg, m2);
            }
        }
    }
    p->nwg = g_tune[kc.str()] < max_wg ? g_tune[kc.str()] : max_wg;
    if (!haveF || !haveC) tune_store();
    return RPR_OK;
}

template <typename T>
static rpr_status autotune_plan(rpr_plan *p, int max_wg, int cus)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_load();
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rpr_status rc = RPR_OK;
    if (hipStreamCreate(&st) != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = fail(RPR_ERR_HIP, "autotune: cannot create a stream or events");
    if (rc == RPR_OK) rc = autotune_run<T>(p, max_wg, cus, st, e0, e1);
    if (st) (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    return rc;
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
    if (opt->correction != RPR_CORR_RANDNET && opt->correction != RPR_CORR_PARAREAL &&
        opt->correction != RPR_CORR_RANDNET_NN)
        return fail(RPR_ERR_INVALID_ARG,
                    "opt.correction must be RPR_CORR_RANDNET, RPR_CORR_PARAREAL or RPR_CORR_RANDNET_NN");
    if (opt->k_max < 0 || opt->k_max > N) return fail(RPR_ERR_INVALID_ARG, "opt.k_max must be in [0, N]");
    if (opt->poll_every < 0) return fail(RPR_ERR_INVALID_ARG, "opt.poll_every must be >= 0");
    if (opt->features < RPR_FEAT_AUTO || opt->features > RPR_FEAT_BF16)
        return fail(RPR_ERR_INVALID_ARG, "opt.features must be an rpr_feature_precision");
    if (opt->autotune != 0 && opt->autotune != 1) return fail(RPR_ERR_INVALID_ARG, "opt.autotune must be 0 or 1");
    if (opt->graph != 0 && opt->graph != 1) return fail(RPR_ERR_INVALID_ARG, "opt.graph must be 0 or 1");
    if (opt->reserved != 0) return fail(RPR_ERR_INVALID_ARG, "opt.reserved must be 0");
    const bool use_net = opt->correction == RPR_CORR_RANDNET || opt->correction == RPR_CORR_RANDNET_NN;
    if (use_net) {
        if (!net) return fail(RPR_ERR_INVALID_ARG, "net is NULL");
        if (net->M < 1 || net->M > 512) return fail(RPR_ERR_INVALID_ARG, "net.M must be in [1, 512]");
        if (net->activation != RPR_TANH && net->activation != RPR_RELU)
            return fail(RPR_ERR_INVALID_ARG, "net.activation must be RPR_TANH or RPR_RELU");
        if (!(net->lambda > 0) || !is_finite(net->lambda)) return fail(RPR_ERR_INVALID_ARG, "net.lambda must be > 0");
        if (!is_finite(net->input_scale)) return fail(RPR_ERR_INVALID_ARG, "net.input_scale must be finite");
        if ((A == nullptr) != (zeta == nullptr)) return fail(RPR_ERR_INVALID_ARG, "pass both A and zeta, or neither");
        if (net->reserved != 0) return fail(RPR_ERR_INVALID_ARG, "net.reserved must be 0");
        if (opt->correction == RPR_CORR_RANDNET_NN && (net->m_nn < 1 || net->m_nn > NN_MAX))
            return fail(RPR_ERR_INVALID_ARG, "net.m_nn must be in [1, 32]");
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
    p->feat_bf16 = opt->features == RPR_FEAT_BF16 || (opt->features == RPR_FEAT_AUTO && p->prec == RPR_MIXED);
    p->autotune = opt->autotune;
    p->use_graph = opt->graph;
    if (use_net) {
        p->M = net->M;
        p->act = net->activation;
        p->lambda = net->lambda;
        p->scale_opt = net->input_scale;
        p->nn = opt->correction == RPR_CORR_RANDNET_NN;
        p->m_nn = p->nn ? net->m_nn : 0;
    }
    const double T = (tN - t0) / N;
    p->dtF = T / (double)F->steps;
    p->dtG = T / (double)G->steps;
    // on chip when the slot state fits one work-group (or as F/G.threads say),
    // else the tiled form
    for (const rpr_propagator *P : {F, G}) {
        OnchipShape &sh = P == F ? p->shF : p->shG;
        bool tiled = P->threads == TILED_THREADS;
        if (!tiled && !onchip_shape(g, p->esz, &sh, P->threads ? P->threads : 1024)) {
            if (P->threads) {
                delete p;
                return fail(RPR_ERR_UNSUPPORTED, "the slot state does not fit one work-group of that size");
            }
            tiled = true;
        }
        const rpr_status st = check_threads(g, p->esz, tiled ? TILED_THREADS : (P->threads ? P->threads : 1024));
        if (st != RPR_OK) {
            delete p;
            return st;
        }
        if (tiled) sh = tiled_shape(g, p->esz);
    }
    if (p->corr == RPR_CORR_RANDNET && ((size_t)p->M * 32 + 32 * 33) * sizeof(double) > kMaxLds) {
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
        a.mode = chain_mode(p);  // the kernel variant this plan launches
        st = launch_chain<double>(a, p->shG, 0, nullptr, &max_wg);
    } else {
        ChainArgs<float> a{};
        a.g = g;
        a.M = p->M;
        a.mode = chain_mode(p);
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
    int nwg = (work < 65536.0 && p->shG.maxt != TILED_THREADS) ? 1 : cus;  // the tiled coarse solver needs the grid
    if (nwg > max_wg) nwg = max_wg;
    if (nwg > 4096) nwg = 4096;
    p->nwg = nwg < 1 ? 1 : nwg;
    if (use_net) {
        // the autotuner tries grids of up to one work-group per CU
        const int hmax = p->autotune ? std::max(p->nwg, std::min(cus, max_wg)) : p->nwg;
        st = dalloc(&p->hpart, (size_t)hmax * p->M);
        if (st == RPR_OK && p->nn) st = dalloc(&p->dpart, (size_t)hmax * p->n_cap);
        if (st != RPR_OK) {
            const std::string keep = g_err;
            plan_free(p);
            g_err = keep;
            return st;
        }
    }
    if (p->autotune) {
        st = p->esz == 8 ? autotune_plan<double>(p, max_wg, cus) : autotune_plan<float>(p, max_wg, cus);
        if (st != RPR_OK) {
            const std::string keep = g_err;
            plan_free(p);
            g_err = keep;
            return st;
        }
    }
    *plan = p;
    return RPR_OK;
}

// ---- phases of a solve (shared by single and batched plans) ----
template <typename T>
static ChainArgs<T> chain_args(rpr_plan *p, double s)
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
    a.gw = tiled_work<T>(p->gwork, (size_t)p->g.d);
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
static rpr_status phase_check_u0(rpr_plan *p, const double *u0, hipStream_t st)
{
    hipLaunchKernelGGL(k_absmax, dim3(1), dim3(1024), 0, st, u0, p->g.d, p->u0max, p->u0bad);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}

// input scale (Algorithm "Parareal (generic)", initialisation), control block,
// U_0 = u0, zeroed ridge statistics, coarse sweep
template <typename T>
static rpr_status phase_setup(rpr_plan *p, const double *u0, double umax, hipStream_t st, ChainArgs<T> *out)
{
    double s = p->scale_opt;
    if (!(s > 0)) {
        s = 1.0;
        while (s < umax) s *= 2.0;
    }
    p->info = rpr_info{};
    p->info.input_scale = s;
    hipLaunchKernelGGL(k_init_ctrl, dim3(1), dim3(1), 0, st, p->ctrl, p->L_hist, p->chg_hist);
    RPR_HIP(hipGetLastError());
    RPR_TRY((convert<double, T>(u0, static_cast<T *>(p->U), (size_t)p->g.d, st)));
    if (p->corr == RPR_CORR_RANDNET) {
        RPR_TRY(zero(p->Gm, (size_t)p->M * p->M, st));
        RPR_TRY(zero(p->Bm, (size_t)p->M * p->g.d, st));
    }
    ChainArgs<T> a = chain_args<T>(p, s);
    a.mode = CHAIN_SWEEP;
    // on chip the sweep's state stays in one work-group; the tiled coarse
    // solver spreads each slot's tiles over the plan's grid
    RPR_TRY(launch_chain<T>(a, p->shG, p->shG.maxt == TILED_THREADS ? p->nwg : 1, st));
    a.mode = chain_mode(p);
    *out = a;
    return RPR_OK;
}

// training pairs, hidden layer, ridge statistics and solve of one iteration
template <typename T>
static rpr_status phase_model(rpr_plan *p, double inv_s, hipStream_t st)
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
static rpr_status phase_finish(rpr_plan *p, double *U_out, float ms, hipStream_t st)
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
static rpr_status capture_block(rpr_plan *p, F enqueue)
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

template <typename T>
static rpr_status execute_impl(rpr_plan *p, const double *u0, double *U_out, hipStream_t st)
{
    const Geom &g = p->g;
    const int N = p->N, d = g.d;
    T *U = static_cast<T *>(p->U), *Fv = static_cast<T *>(p->Fv);

    RPR_TRY(phase_check_u0(p, u0, st));
    double umax = 0.0;
    int bad = 0;
    RPR_HIP(hipMemcpyAsync(&umax, p->u0max, sizeof(double), hipMemcpyDeviceToHost, st));
    RPR_HIP(hipMemcpyAsync(&bad, p->u0bad, sizeof(int), hipMemcpyDeviceToHost, st));
    RPR_HIP(hipStreamSynchronize(st));
    if (bad) return fail(RPR_ERR_NONFINITE, "u0 has non-finite entries");

    // phase events (eager iterations only): pev[0] after the set-up or at
    // the start of a burst, then after the fine solves, the model and the
    // sweep of each iteration of the burst
    const bool timed = !p->use_graph;
    const size_t n_ev = 1 + 3 * (size_t)(p->poll < p->k_max ? p->poll : p->k_max);  // bursts are at most this long
    if (timed && p->pev.size() < n_ev) {
        for (size_t e = p->pev.size(); e < n_ev; ++e) {
            hipEvent_t ev = nullptr;
            RPR_HIP(hipEventCreate(&ev));
            p->pev.push_back(ev);
        }
    }
    double t_fine = 0.0, t_model = 0.0, t_sweep = 0.0;
    auto span = [&](int e0, int e1) -> double {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, p->pev[e0], p->pev[e1]);
        return ms * 1e-3;
    };
    RPR_HIP(hipEventRecord(p->ev0, st));
    ChainArgs<T> a;
    RPR_TRY(phase_setup<T>(p, u0, umax, st, &a));
    if (timed) RPR_HIP(hipEventRecord(p->pev[0], st));
    const int *ctrl_i = reinterpret_cast<const int *>(p->ctrl);
    // one iteration: fine solves of the unfinished slots (Fv[i] = F(U[i-1])),
    // the model, the predictor-corrector sweep with the stopping rule
    // `s` is the stream the iteration is enqueued on (the caller's, or the
    // capture stream); inside a graph the chain runs as one work-group with
    // plain barriers, so the graph holds no grid-wide barrier
    // (ev: the first of the iteration's three phase events, or -1)
    auto iteration = [&](hipStream_t s, bool graph, int ev) -> rpr_status {
        const TiledWork<T> fw = tiled_work<T>(p->fwork, (size_t)N * d);
        RPR_TRY(launch_propagate<T>(g, p->F.method, p->F.steps, p->dtF, N, U, Fv + d, ctrl_i, s, p->shF.maxt,
                                    p->fwork ? &fw : nullptr));
        if (ev >= 0) RPR_HIP(hipEventRecord(p->pev[ev], s));
        RPR_TRY(phase_model<T>(p, a.inv_s, s));
        if (ev >= 0) RPR_HIP(hipEventRecord(p->pev[ev + 1], s));
        if (graph)
            RPR_TRY(launch_chain_multi<T>(static_cast<const ChainArgs<T> *>(p->gchain), 1, g, p->shG, p->M, s));
        else
            RPR_TRY(launch_chain<T>(a, p->shG, p->nwg, s));
        if (ev >= 0) RPR_HIP(hipEventRecord(p->pev[ev + 2], s));
        return RPR_OK;
    };
    if (p->use_graph) RPR_HIP(hipMemcpyAsync(p->gchain, &a, sizeof(a), hipMemcpyHostToDevice, st));
    // graph mode: a block of `poll` iterations is captured once (again when
    // the input scale changes) and replayed; iterations after the stop flag
    // is raised return at once
    if (p->use_graph && (!p->graph_exec || p->graph_s != a.inv_s)) {
        RPR_TRY(capture_block(p, [&]() -> rpr_status {
            for (int b = 0; b < p->poll; ++b) RPR_TRY(iteration(p->cap_stream, true, -1));
            return RPR_OK;
        }));
        p->graph_s = a.inv_s;
    }
    int k = 0;
    bool done = false;
    bool first = true;
    while (k < p->k_max && !done) {
        const int burst = (p->k_max - k) < p->poll ? (p->k_max - k) : p->poll;
        if (p->use_graph) {
            RPR_HIP(hipGraphLaunch(p->graph_exec, st));
            k += p->poll;
        } else {
            // the first burst starts at the set-up's event (its time goes to the
            // sweeps); later ones at a new one
            if (!first) RPR_HIP(hipEventRecord(p->pev[0], st));
            for (int b = 0; b < burst; ++b) {
                RPR_TRY(iteration(st, false, 1 + 3 * b));
                ++k;
            }
        }
        RPR_HIP(hipMemcpyAsync(p->ctrl_host, p->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        RPR_HIP(hipStreamSynchronize(st));
        done = p->ctrl_host->done != 0;
        if (timed) {
            if (first) {
                float ms = 0.f;
                RPR_HIP(hipEventElapsedTime(&ms, p->ev0, p->pev[0]));
                t_sweep += ms * 1e-3;
            }
            for (int b = 0; b < burst; ++b) {
                const int e = 1 + 3 * b;
                t_fine += span(e - 1, e);
                t_model += span(e, e + 1);
                t_sweep += span(e + 1, e + 2);
            }
        }
        first = false;
    }
    RPR_HIP(hipEventRecord(p->ev1, st));
    RPR_HIP(hipEventSynchronize(p->ev1));
    float ms = 0.f;
    RPR_HIP(hipEventElapsedTime(&ms, p->ev0, p->ev1));
    RPR_TRY(phase_finish<T>(p, U_out, ms, st));
    if (timed) {
        p->info.t_fine = t_fine;
        p->info.t_model = t_model;
        p->info.t_sweep = t_sweep;
    }
    RPR_HIP(hipStreamSynchronize(st));
    return p->ctrl_host->L >= N ? RPR_OK : RPR_NOT_CONVERGED;
}

extern "C" rpr_status rpr_plan_execute(rpr_plan *plan, const void *u0, void *U_out, void *stream)
{
    if (!plan) return fail(RPR_ERR_INVALID_ARG, "plan is NULL");
    if (!u0 || !U_out) return fail(RPR_ERR_INVALID_ARG, "u0 and U_out must be device pointers");
    if (!plan->sub.empty()) return fail(RPR_ERR_INVALID_ARG, "batch plan: use rpr_plan_execute_batch");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (plan->esz == 8)
        return execute_impl<double>(plan, static_cast<const double *>(u0), static_cast<double *>(U_out), st);
    return execute_impl<float>(plan, static_cast<const double *>(u0), static_cast<double *>(U_out), st);
}

// ------------------------------------------------------------------ batches --
extern "C" rpr_status rpr_plan_create_batch(rpr_plan **plan, int32_t n_inst, const rpr_rhs *h, const int32_t *d,
                                            const double *t0, const double *tN, const int32_t *N,
                                            const rpr_propagator *F, const rpr_propagator *G, const double *tol,
                                            const rpr_randnet *net, const double *const *A,
                                            const double *const *zeta, uint64_t seed, const rpr_options *opt)
{
    if (!plan) return fail(RPR_ERR_INVALID_ARG, "plan is NULL");
    *plan = nullptr;
    if (n_inst < 1) return fail(RPR_ERR_INVALID_ARG, "n_inst must be >= 1");
    if (!h || !d || !t0 || !tN || !N || !F || !G || !tol || !opt)
        return fail(RPR_ERR_INVALID_ARG, "batch arrays must not be NULL");
    for (int b = 1; b < n_inst; ++b)
        if (h[b].kind != h[0].kind) return fail(RPR_ERR_INVALID_ARG, "all instances of a batch need the same rhs kind");
    rpr_plan *p = new rpr_plan();
    auto bail = [&](rpr_status st) {
        const std::string keep = g_err;
        plan_free(p);
        g_err = keep;
        return st;
    };
    rpr_options o = *opt;
    o.autotune = 0;
    o.graph = 0;  // the batch captures its own iteration block
    for (int b = 0; b < n_inst; ++b) {
        rpr_plan *q = nullptr;
        const rpr_status st = rpr_plan_create(&q, &h[b], d[b], t0[b], tN[b], N[b], &F[b], &G[b], tol[b],
                                              net ? &net[b] : nullptr, A ? A[b] : nullptr, zeta ? zeta[b] : nullptr,
                                              seed + (uint64_t)b, &o);
        if (st != RPR_OK) {
            g_err = "instance " + std::to_string(b) + ": " + g_err;
            return bail(st);
        }
        q->nwg = 1;
        p->sub.push_back(q);
    }
    rpr_plan *q0 = p->sub[0];
    p->prec = q0->prec;
    p->esz = q0->esz;
    p->corr = q0->corr;
    for (rpr_plan *q : p->sub)
        if (q->prec != p->prec || q->corr != p->corr)
            return bail(fail(RPR_ERR_INVALID_ARG, "all instances of a batch need the same precision and correction"));
    for (rpr_plan *q : p->sub)
        if (q->shF.maxt == TILED_THREADS || q->shG.maxt == TILED_THREADS)
            return bail(fail(RPR_ERR_UNSUPPORTED, "batch instances must fit one work-group each"));
    // the kernel shape of the largest instance serves every instance
    int big = 0;
    for (int b = 1; b < n_inst; ++b)
        if (padded_elems(p->sub[b]->g) > padded_elems(p->sub[big]->g)) big = b;
    p->bgmax = p->sub[big]->g;
    if (!onchip_shape(p->bgmax, p->esz, &p->bshF, 1024))
        return bail(fail(RPR_ERR_UNSUPPORTED, "largest batch instance does not fit one work-group"));
    p->bshF.full = 0;
    p->bshG = p->bshF;
    for (rpr_plan *q : p->sub) {
        const Geom &g = q->g;
        const int need = g.kind == RPR_BURGERS1D ? (g.nc + p->bshF.cpt - 1) / p->bshF.cpt
                                                 : g.nx * ((g.ny + p->bshF.cpt - 1) / p->bshF.cpt);
        if (need > p->bshF.block)
            return bail(fail(RPR_ERR_UNSUPPORTED, "batch instance grids do not share one strip shape"));
        p->bM = q->M > p->bM ? q->M : p->bM;
        p->bkmax = q->k_max > p->bkmax ? q->k_max : p->bkmax;
    }
    p->poll = q0->poll;
    // longest-first (LPT) list of (instance, slot) fine solves
    struct Work { int b, i; double cost; };
    std::vector<Work> work;
    for (int b = 0; b < n_inst; ++b) {
        const rpr_plan *q = p->sub[b];
        const double c = (double)q->g.d * (double)q->F.steps * (q->F.method == RPR_RK4 ? 4.0 : 1.0);
        for (int i = 1; i <= q->N; ++i) work.push_back({b, i, c});
    }
    std::stable_sort(work.begin(), work.end(), [](const Work &x, const Work &y) { return x.cost > y.cost; });
    std::vector<int2> items(work.size());
    for (size_t k = 0; k < work.size(); ++k) items[k] = make_int2(work[k].b, work[k].i);
    p->bn_items = (int)items.size();
    rpr_status st = dalloc(&p->bitems, items.size());
    if (st == RPR_OK) st = dalloc(&p->bcounter, 1);
    if (st != RPR_OK) return bail(st);
    if (hipMemcpy(p->bitems, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(RPR_ERR_HIP, "batch: item upload failed"));
    const size_t isz = p->esz == 8 ? sizeof(BatchInst<double>) : sizeof(BatchInst<float>);
    const size_t csz = p->esz == 8 ? sizeof(ChainArgs<double>) : sizeof(ChainArgs<float>);
    char *tmp;
    if ((st = dalloc(&tmp, isz * n_inst)) != RPR_OK) return bail(st);
    p->binsts = tmp;
    if ((st = dalloc(&tmp, csz * n_inst)) != RPR_OK) return bail(st);
    p->bchain = tmp;
    p->hchain.assign(csz * n_inst, 0);
    std::vector<char> hinst(isz * n_inst);
    for (int b = 0; b < n_inst; ++b) {
        rpr_plan *q = p->sub[b];
        if (p->esz == 8) {
            BatchInst<double> I{q->g, q->F.method, (long long)q->F.steps, q->dtF, static_cast<const double *>(q->U),
                                static_cast<double *>(q->Fv), reinterpret_cast<const int *>(q->ctrl)};
            std::memcpy(hinst.data() + b * isz, &I, isz);
        } else {
            BatchInst<float> I{q->g, q->F.method, (long long)q->F.steps, q->dtF, static_cast<const float *>(q->U),
                               static_cast<float *>(q->Fv), reinterpret_cast<const int *>(q->ctrl)};
            std::memcpy(hinst.data() + b * isz, &I, isz);
        }
    }
    if (hipMemcpy(p->binsts, hinst.data(), hinst.size(), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(RPR_ERR_HIP, "batch: instance upload failed"));
    int dev = 0, cus = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    p->bgrid = p->bn_items < 2 * cus ? p->bn_items : 2 * cus;
    if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess)
        return bail(fail(RPR_ERR_HIP, "batch: event creation failed"));
    p->use_graph = opt->graph;
    if (p->use_graph && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(RPR_ERR_HIP, "batch: capture stream creation failed"));
    *plan = p;
    return RPR_OK;
}

template <typename T>
static rpr_status execute_batch_impl(rpr_plan *p, const double *const *u0, double *const *U_out, hipStream_t st)
{
    const int n = (int)p->sub.size();
    for (int b = 0; b < n; ++b) RPR_TRY(phase_check_u0(p->sub[b], u0[b], st));
    std::vector<double> umax(n);
    std::vector<int> bad(n);
    for (int b = 0; b < n; ++b) {
        RPR_HIP(hipMemcpyAsync(&umax[b], p->sub[b]->u0max, sizeof(double), hipMemcpyDeviceToHost, st));
        RPR_HIP(hipMemcpyAsync(&bad[b], p->sub[b]->u0bad, sizeof(int), hipMemcpyDeviceToHost, st));
    }
    RPR_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < n; ++b)
        if (bad[b]) return fail(RPR_ERR_NONFINITE, "u0 of instance " + std::to_string(b) + " has non-finite entries");

    // phase events of eager iterations, as in execute_impl (batch-wide)
    const bool timed = !p->use_graph;
    const size_t n_ev = 1 + 3 * (size_t)(p->poll < p->bkmax ? p->poll : p->bkmax);
    if (timed && p->pev.size() < n_ev) {
        for (size_t e = p->pev.size(); e < n_ev; ++e) {
            hipEvent_t ev = nullptr;
            RPR_HIP(hipEventCreate(&ev));
            p->pev.push_back(ev);
        }
    }
    double t_fine = 0.0, t_model = 0.0, t_sweep = 0.0;
    auto span = [&](int e0, int e1) -> double {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, p->pev[e0], p->pev[e1]);
        return ms * 1e-3;
    };
    RPR_HIP(hipEventRecord(p->ev0, st));
    std::vector<ChainArgs<T>> args(n);
    for (int b = 0; b < n; ++b) RPR_TRY(phase_setup<T>(p->sub[b], u0[b], umax[b], st, &args[b]));
    std::memcpy(p->hchain.data(), args.data(), sizeof(ChainArgs<T>) * n);
    RPR_HIP(hipMemcpyAsync(p->bchain, p->hchain.data(), sizeof(ChainArgs<T>) * n, hipMemcpyHostToDevice, st));
    if (timed) RPR_HIP(hipEventRecord(p->pev[0], st));
    const auto *insts = static_cast<const BatchInst<T> *>(p->binsts);
    // (ev: the first of the iteration's three phase events, or -1)
    auto iteration = [&](hipStream_t s, int ev) -> rpr_status {
        // every unfinished (instance, slot) fine solve in one persistent launch
        RPR_TRY(zero(p->bcounter, 1, s));
        RPR_TRY(launch_prop_persistent<T>(insts, p->bitems, p->bn_items, p->bcounter, p->bgmax, p->bshF, p->bgrid,
                                          s));
        if (ev >= 0) RPR_HIP(hipEventRecord(p->pev[ev], s));
        for (int b = 0; b < n; ++b) RPR_TRY(phase_model<T>(p->sub[b], args[b].inv_s, s));
        if (ev >= 0) RPR_HIP(hipEventRecord(p->pev[ev + 1], s));
        // every instance's predictor-corrector sweep, one work-group each
        RPR_TRY(launch_chain_multi<T>(static_cast<const ChainArgs<T> *>(p->bchain), n, p->bgmax, p->bshG, p->bM, s));
        if (ev >= 0) RPR_HIP(hipEventRecord(p->pev[ev + 2], s));
        return RPR_OK;
    };
    if (p->use_graph) {
        // captured once per set of input scales (the feature kernels take the
        // scale by value); the chain arguments are read from device memory
        bool same = p->graph_exec != nullptr && p->bscale.size() == (size_t)n;
        for (int b = 0; same && b < n; ++b) same = p->bscale[b] == args[b].inv_s;
        if (!same) RPR_TRY(capture_block(p, [&]() -> rpr_status {
            for (int it = 0; it < p->poll; ++it) RPR_TRY(iteration(p->cap_stream, -1));
            return RPR_OK;
        }));
        p->bscale.resize(n);
        for (int b = 0; b < n; ++b) p->bscale[b] = args[b].inv_s;
    }
    int k = 0;
    bool done = false;
    bool first = true;
    while (k < p->bkmax && !done) {
        const int burst = (p->bkmax - k) < p->poll ? (p->bkmax - k) : p->poll;
        if (p->use_graph) {
            RPR_HIP(hipGraphLaunch(p->graph_exec, st));
            k += p->poll;
        } else {
            if (!first) RPR_HIP(hipEventRecord(p->pev[0], st));
            for (int it = 0; it < burst; ++it) {
                RPR_TRY(iteration(st, 1 + 3 * it));
                ++k;
            }
        }
        for (int b = 0; b < n; ++b)
            RPR_HIP(hipMemcpyAsync(p->sub[b]->ctrl_host, p->sub[b]->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        RPR_HIP(hipStreamSynchronize(st));
        done = true;
        for (int b = 0; b < n; ++b) done = done && p->sub[b]->ctrl_host->done != 0;
        if (timed) {
            if (first) {
                float ms0 = 0.f;
                RPR_HIP(hipEventElapsedTime(&ms0, p->ev0, p->pev[0]));
                t_sweep += ms0 * 1e-3;
            }
            for (int it = 0; it < burst; ++it) {
                const int e = 1 + 3 * it;
                t_fine += span(e - 1, e);
                t_model += span(e, e + 1);
                t_sweep += span(e + 1, e + 2);
            }
        }
        first = false;
    }
    RPR_HIP(hipEventRecord(p->ev1, st));
    RPR_HIP(hipEventSynchronize(p->ev1));
    float ms = 0.f;
    RPR_HIP(hipEventElapsedTime(&ms, p->ev0, p->ev1));
    for (int b = 0; b < n; ++b) {
        RPR_TRY(phase_finish<T>(p->sub[b], U_out[b], ms, st));
        if (timed) {
            p->sub[b]->info.t_fine = t_fine;
            p->sub[b]->info.t_model = t_model;
            p->sub[b]->info.t_sweep = t_sweep;
        }
    }
    RPR_HIP(hipStreamSynchronize(st));
    bool conv = true;
    for (int b = 0; b < n; ++b) conv = conv && p->sub[b]->ctrl_host->L >= p->sub[b]->N;
    return conv ? RPR_OK : RPR_NOT_CONVERGED;
}

extern "C" rpr_status rpr_plan_execute_batch(rpr_plan *plan, const void *const *u0, void *const *U_out,
                                             void *stream)
{
    if (!plan || plan->sub.empty()) return fail(RPR_ERR_INVALID_ARG, "not a batch plan");
    if (!u0 || !U_out) return fail(RPR_ERR_INVALID_ARG, "u0 and U_out must be host arrays of device pointers");
    for (size_t b = 0; b < plan->sub.size(); ++b)
        if (!u0[b] || !U_out[b]) return fail(RPR_ERR_INVALID_ARG, "NULL device pointer in u0 / U_out");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (plan->esz == 8)
        return execute_batch_impl<double>(plan, reinterpret_cast<const double *const *>(u0),
                                          reinterpret_cast<double *const *>(U_out), st);
    return execute_batch_impl<float>(plan, reinterpret_cast<const double *const *>(u0),
                                     reinterpret_cast<double *const *>(U_out), st);
}

extern "C" rpr_status rpr_plan_instance(const rpr_plan *batch, int32_t b, const rpr_plan **inst)
{
    if (!batch || !inst || b < 0 || b >= (int)batch->sub.size())
        return fail(RPR_ERR_INVALID_ARG, "need a batch plan, an instance index in range and an output pointer");
    *inst = batch->sub[b];
    return RPR_OK;
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
    const int esz = precision == RPR_FP64 ? 8 : 4;
    if (P->threads) RPR_TRY(check_threads(g, esz, P->threads));
    // automatic: on chip when the state fits one work-group, else tiled
    OnchipShape probe;
    const bool fits = onchip_shape(g, esz, &probe, 1024);
    if (!P->threads && !fits) RPR_TRY(check_threads(g, esz, TILED_THREADS));
    RPR_TRY(check_device());
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int mt = P->threads ? P->threads : (fits ? tuned_prop_threads(g, esz, P->method) : TILED_THREADS);
    if (mt != TILED_THREADS) {
        if (precision == RPR_FP64)
            return launch_propagate<double>(g, P->method, P->steps, dt, n_states, static_cast<const double *>(in),
                                            static_cast<double *>(out), nullptr, st, mt);
        return launch_propagate<float>(g, P->method, P->steps, dt, n_states, static_cast<const float *>(in),
                                       static_cast<float *>(out), nullptr, st, mt);
    }
    // tiled: five work arrays of n_states x d values, released on the stream
    const size_t nd = (size_t)n_states * d;
    void *ws = nullptr;
    RPR_HIP(hipMallocAsync(&ws, 5 * nd * esz, st));
    rpr_status rc;
    if (precision == RPR_FP64) {
        double *b = static_cast<double *>(ws);
        const TiledWork<double> w{b, b + nd, b + 2 * nd, b + 3 * nd, nullptr};
        rc = launch_propagate<double>(g, P->method, P->steps, dt, n_states, static_cast<const double *>(in),
                                      static_cast<double *>(out), nullptr, st, mt, &w);
    } else {
        float *b = static_cast<float *>(ws);
        const TiledWork<float> w{b, b + nd, b + 2 * nd, b + 3 * nd, b + 4 * nd};
        rc = launch_propagate<float>(g, P->method, P->steps, dt, n_states, static_cast<const float *>(in),
                                     static_cast<float *>(out), nullptr, st, mt, &w);
    }
    RPR_HIP(hipFreeAsync(ws, st));
    return rc;
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
    RPR_HIP(hipMallocAsync((void **)&Ab, 3 * sizeof(uint16_t) * (size_t)M * d, st));
    RPR_HIP(hipMallocAsync((void **)&part, sizeof(float) * feat_bf16_splits(d) * n * M, st));
    uint16_t *xb = nullptr;
    if (feat_bf16_large(n, d)) RPR_HIP(hipMallocAsync((void **)&xb, 3 * sizeof(uint16_t) * (size_t)n * d, st));
    rpr_status rc = launch_to_bf16(A, Ab, (size_t)M * d, st);
    if (rc == RPR_OK)
        rc = launch_features_bf16<float>(n, M, d, activation, 1.0 / s, Ab, zeta, X, Phi, part, nullptr, st, xb);
    RPR_HIP(hipFreeAsync(Ab, st));
    RPR_HIP(hipFreeAsync(part, st));
    if (xb) RPR_HIP(hipFreeAsync(xb, st));
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
