// api.hip -- the C ABI of librpr (include/rpr.h): argument checking, plans
// and the Parareal iteration loop of a single plan.  Batches (batch.hip), the
// autotuner (autotune.hip), the building-block entry points (blocks.hip) and
// the stability pre-check (stability.hip) live in their own units.
//
// Iteration loop.  Every kernel of an iteration reads the converged-slot
// counter L and the done flag from the plan's device control block, so the
// host enqueues iterations back to back without waiting; it reads the done
// flag every `poll_every` iterations (one device-to-host copy) and stops
// enqueuing once it is set.  Kernels enqueued after convergence exit at once.
#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "plan.h"

namespace rpr {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

std::string &err_text() { return g_err; }

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


rpr_status make_geom(const rpr_rhs *h, int32_t d, Geom *g)
{
    if (!h) return fail(RPR_ERR_INVALID_ARG, "rhs is NULL");
    const int ns = nspecies(h->kind);
    if (ns == 0) return fail(RPR_ERR_INVALID_ARG, "rhs.kind is not a known right-hand side");
    if (h->kind == RPR_BRUSS3D) {
        if (h->nz < 1) return fail(RPR_ERR_INVALID_ARG, "rhs.nz must be >= 1 for the 3D system");
    } else if (h->nz != 0 && h->nz != 1) {
        return fail(RPR_ERR_INVALID_ARG, "rhs.nz must be 0 or 1 for the 1D and 2D systems");
    }
    if (h->nx < 1 || h->ny < 1) return fail(RPR_ERR_INVALID_ARG, "rhs.nx and rhs.ny must be >= 1");
    if (h->kind == RPR_BURGERS1D && h->ny != 1) return fail(RPR_ERR_INVALID_ARG, "1D problem needs ny == 1");
    const int nz = h->kind == RPR_BRUSS3D ? h->nz : 1;
    if ((int64_t)ns * h->nx * h->ny * nz != d)
        return fail(RPR_ERR_INVALID_ARG, "d must equal species * nx * ny * nz (" +
                                             std::to_string((int64_t)ns * h->nx * h->ny * nz) + ")");
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
    G.nc = h->nx * h->ny * nz;
    G.nz = nz;
    G.ns = ns;
    G.d = d;
    G.periodic = (h->kind == RPR_BURGERS1D || h->kind == RPR_BRUSS2D || h->kind == RPR_BRUSS3D) ? 1 : 0;
    const double dx = lx / h->nx, dy = h->kind == RPR_BURGERS1D ? 1.0 : ly / h->ny;
    G.idx2 = 1.0 / (dx * dx);
    G.idy2 = 1.0 / (dy * dy);
    const double dz = lx / nz;  // the 3D box is a cube in x and z: (x0, x1) along z too
    G.idz2 = h->kind == RPR_BRUSS3D ? 1.0 / (dz * dz) : 0.0;
    G.i2dx = 1.0 / (2.0 * dx);
    G.idx = 1.0 / dx;
    G.idy = 1.0 / dy;
    for (int i = 0; i < 6; ++i) G.p[i] = h->p[i];
    *g = G;
    return RPR_OK;
}

rpr_status check_device()
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

rpr_status check_prop(const rpr_propagator *P, const char *name)
{
    if (!P) return fail(RPR_ERR_INVALID_ARG, std::string(name) + " is NULL");
    if (P->method != RPR_RK1 && P->method != RPR_RK4 && P->method != RPR_RK8)
        return fail(RPR_ERR_INVALID_ARG, std::string(name) + ".method must be RPR_RK1, RPR_RK4 or RPR_RK8");
    if (P->threads != 0 && P->threads != GENERIC_THREADS && P->threads != TILED_THREADS && P->threads != 512 &&
        P->threads != 1024)
        return fail(RPR_ERR_INVALID_ARG, std::string(name) + ".threads must be 0, 128, 256, 512 or 1024");
    if (P->method == RPR_RK8 && P->threads != 0 && P->threads != GENERIC_THREADS)
        return fail(RPR_ERR_UNSUPPORTED, std::string(name) + ": RPR_RK8 runs on the generic propagator (threads 0 or 128)");
    if (P->steps < 1) return fail(RPR_ERR_INVALID_ARG, std::string(name) + ".steps must be >= 1");
    return RPR_OK;
}

// ------------------------------------------------------------ small kernels --
// max |u| and a non-finite flag over d doubles (one work-group).
// out_max[0] = max |u|, out_max[1] = the largest wave speed |velocity| +
// sqrt(g h) of a shallow-water state (swe_nc cells; 0 for other systems, or
// +inf where h <= 0); *out_bad = 1 if u has a non-finite entry.
__global__ __launch_bounds__(1024) void k_absmax(const double *__restrict__ u, int d, int swe_nc, double gacc,
                                                 double *out_max, int *out_bad)
{
    __shared__ double sm[16], ss[16];
    __shared__ int sb[16];
    double m = 0.0, sp = 0.0;
    int bad = 0;
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        const double v = u[j];
        if (!isfinite(v)) bad = 1;
        else m = fmax(m, fabs(v));
    }
    for (int j = threadIdx.x; j < swe_nc; j += blockDim.x) {
        const double hh = u[j], vel = fmax(fabs(u[swe_nc + j]), fabs(u[2 * swe_nc + j]));
        sp = fmax(sp, hh > 0.0 ? vel / hh + sqrt(gacc * hh) : INFINITY);
    }
    for (int off = 32; off > 0; off >>= 1) {
        m = fmax(m, __shfl_down(m, off, 64));
        sp = fmax(sp, __shfl_down(sp, off, 64));
        bad |= __shfl_down(bad, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sm[threadIdx.x >> 6] = m;
        ss[threadIdx.x >> 6] = sp;
        sb[threadIdx.x >> 6] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mm = 0.0, s2 = 0.0;
        int bb = 0;
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) {
            mm = fmax(mm, sm[w]);
            s2 = fmax(s2, ss[w]);
            bb |= sb[w];
        }
        out_max[0] = mm;
        out_max[1] = s2;
        *out_bad = bb;
    }
}

rpr_status launch_absmax(const Geom &g, const double *u, double *out_max, int *out_bad, hipStream_t st)
{
    const int swe_nc = g.kind == RPR_SWE2D ? g.nc : 0;
    hipLaunchKernelGGL(k_absmax, dim3(1), dim3(1024), 0, st, u, g.d, swe_nc, g.p[0], out_max, out_bad);
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

rpr_status launch_init_ctrl(Ctrl *c, int *L_hist, double *chg_hist, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_ctrl, dim3(1), dim3(1), 0, st, c, L_hist, chg_hist);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}

}  // namespace rpr

void plan_free(rpr_plan *p)
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

static rpr_status plan_alloc(rpr_plan *p, const double *A, const double *zeta, uint64_t seed)
{
    const int N = p->N, d = p->g.d, M = p->M;
    const size_t sd = (size_t)(N + 1) * d;
    char *c;
    RPR_TRY(dalloc(&c, sd * p->esz)); p->U = c;
    RPR_TRY(dalloc(&c, sd * p->esz)); p->Fv = c;
    RPR_TRY(dalloc(&c, sd * p->esz)); p->Gc = c;
    RPR_TRY(dalloc(&c, (size_t)d * p->esz)); p->gtmp = c;
    if (const size_t fe = work_elems(p->shF, p->F.method, N, d)) {
        RPR_TRY(dalloc(&c, fe * p->esz));
        p->fwork = c;
    }
    if (const size_t ge = work_elems(p->shG, p->G.method, 1, d)) {
        RPR_TRY(dalloc(&c, ge * p->esz));
        p->gwork = c;
    }
    RPR_TRY(dalloc(&p->part, (size_t)(N + 1) * 4096));
    RPR_TRY(dalloc(&p->ctrl, 1));
    RPR_TRY(dalloc(&p->L_hist, N + 1));
    RPR_TRY(dalloc(&p->chg_hist, N + 1));
    RPR_TRY(dalloc(&p->u0max, 2));
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
    if (p->use_graph) RPR_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    if (p->use_graph || p->seg_sweep) RPR_HIP(hipMalloc(&p->gchain, sizeof(ChainArgs<double>)));
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
    if (opt->stability != 0 && opt->stability != 1) return fail(RPR_ERR_INVALID_ARG, "opt.stability must be 0 or 1");
    if (opt->chain_wgs < 0) return fail(RPR_ERR_INVALID_ARG, "opt.chain_wgs must be >= 0");
    if (opt->sweep_form < 0 || opt->sweep_form > 2) return fail(RPR_ERR_INVALID_ARG, "opt.sweep_form must be 0, 1 or 2");
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
    if (opt->stability == 1) {
        // the part of the bound that holds for any state (diffusion, and the
        // constant parts of the reactions), before any device call; execute
        // checks again at u0
        const double T = (tN - t0) / N;
        const double rF = stability_ratio(g, F->method, T / (double)F->steps, 0.0, 0.0);
        const double rG = stability_ratio(g, G->method, T / (double)G->steps, 0.0, 0.0);
        if (rF > 1.0 || rG > 1.0)
            return fail(RPR_ERR_UNSTABLE, "stability pre-check: dt / dt_max = " + std::to_string(rF) + " (F), " +
                                              std::to_string(rG) + " (G) for every state");
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
    p->strict = opt->stability;
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
        if (P->threads == GENERIC_THREADS || P->method == RPR_RK8 || g.kind == RPR_BRUSS3D) {
            // any tableau, states in memory, cell by cell
            sh = generic_shape(g, p->esz);
            continue;
        }
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
    // the sweep's form: segment kernels where the coarse solver runs over the
    // whole grid (its passes need grid-wide barriers, which cost more than
    // kernel boundaries), or as asked
    const bool grid_coarse = p->shG.maxt == TILED_THREADS || p->shG.maxt == GENERIC_THREADS;
    p->seg_sweep = opt->sweep_form == 2 || (opt->sweep_form == 0 && grid_coarse);
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
    // the tiled and generic coarse solvers need the grid
    int nwg = (work < 65536.0 && p->shG.maxt != TILED_THREADS && p->shG.maxt != GENERIC_THREADS) ? 1 : cus;
    if (opt->chain_wgs > 0) nwg = opt->chain_wgs;
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
    p->fixed_nwg = opt->chain_wgs > 0;
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

template <typename T>
static rpr_status execute_impl(rpr_plan *p, const double *u0, double *U_out, hipStream_t st)
{
    const Geom &g = p->g;
    const int N = p->N, d = g.d;
    T *U = static_cast<T *>(p->U), *Fv = static_cast<T *>(p->Fv);

    RPR_TRY(phase_check_u0(p, u0, st));
    double umax2[2] = {0.0, 0.0};
    int bad = 0;
    RPR_HIP(hipMemcpyAsync(umax2, p->u0max, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    RPR_HIP(hipMemcpyAsync(&bad, p->u0bad, sizeof(int), hipMemcpyDeviceToHost, st));
    RPR_HIP(hipStreamSynchronize(st));
    if (bad) return fail(RPR_ERR_NONFINITE, "u0 has non-finite entries");
    RPR_TRY(stability_gate(p, umax2));
    const double umax = umax2[0];

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
    // capture stream); inside a graph the sweep is a sequence of segment
    // kernels on the plan's grid (the kernel boundaries are its barriers), so
    // the graph holds no grid-wide barrier
    // (ev: the first of the iteration's three phase events, or -1)
    auto iteration = [&](hipStream_t s, bool graph, int ev) -> rpr_status {
        const TiledWork<T> fw = fine_work<T>(p);
        RPR_TRY(launch_propagate<T>(g, p->F.method, p->F.steps, p->dtF, N, U, Fv + d, ctrl_i, s, p->shF.maxt,
                                    p->fwork ? &fw : nullptr, p->fvar));
        if (ev >= 0) RPR_HIP(hipEventRecord(p->pev[ev], s));
        RPR_TRY(phase_model<T>(p, a.inv_s, s));
        if (ev >= 0) RPR_HIP(hipEventRecord(p->pev[ev + 1], s));
        if (graph || p->seg_sweep)
            RPR_TRY(launch_chain_graph<T>(static_cast<const ChainArgs<T> *>(p->gchain), a, p->shG, p->nwg, s));
        else
            RPR_TRY(launch_chain<T>(a, p->shG, p->nwg, s));
        if (ev >= 0) RPR_HIP(hipEventRecord(p->pev[ev + 2], s));
        return RPR_OK;
    };
    if (p->gchain) RPR_HIP(hipMemcpyAsync(p->gchain, &a, sizeof(a), hipMemcpyHostToDevice, st));
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

