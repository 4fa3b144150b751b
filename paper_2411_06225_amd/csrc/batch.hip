// batch.hip -- batches of independent IVPs solved together: one persistent
// launch runs the fine solves of every (instance, slot), one launch the
// predictor-corrector sweeps of every instance.
#include <algorithm>

#include "plan.h"

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
        const std::string keep = err_text();
        plan_free(p);
        err_text() = keep;
        return st;
    };
    rpr_options o = *opt;
    o.autotune = 0;  // the instances take the batch's shapes; the batch is tuned as a whole below
    o.graph = 0;     // the batch captures its own iteration block
    for (int b = 0; b < n_inst; ++b) {
        rpr_plan *q = nullptr;
        const rpr_status st = rpr_plan_create(&q, &h[b], d[b], t0[b], tN[b], N[b], &F[b], &G[b], tol[b],
                                              net ? &net[b] : nullptr, A ? A[b] : nullptr, zeta ? zeta[b] : nullptr,
                                              seed + (uint64_t)b, &o);
        if (st != RPR_OK) {
            err_text() = "instance " + std::to_string(b) + ": " + err_text();
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
        if (q->shF.maxt == TILED_THREADS || q->shG.maxt == TILED_THREADS || q->shF.maxt == GENERIC_THREADS ||
            q->shG.maxt == GENERIC_THREADS)
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
    // chain arguments of the iterations, then those of the k = 0 sweep
    if ((st = dalloc(&tmp, 2 * csz * n_inst)) != RPR_OK) return bail(st);
    p->bchain = tmp;
    p->hchain.assign(2 * csz * n_inst, 0);
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
    if (opt->autotune) {
        st = p->esz == 8 ? autotune_batch<double>(p, cus) : autotune_batch<float>(p, cus);
        if (st != RPR_OK) return bail(st);
    }
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
    std::vector<double> umax2(2 * n), umax(n);
    std::vector<int> bad(n);
    for (int b = 0; b < n; ++b) {
        RPR_HIP(hipMemcpyAsync(&umax2[2 * b], p->sub[b]->u0max, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        RPR_HIP(hipMemcpyAsync(&bad[b], p->sub[b]->u0bad, sizeof(int), hipMemcpyDeviceToHost, st));
    }
    RPR_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < n; ++b) {
        if (bad[b]) return fail(RPR_ERR_NONFINITE, "u0 of instance " + std::to_string(b) + " has non-finite entries");
        const rpr_status us = stability_gate(p->sub[b], &umax2[2 * b]);
        if (us != RPR_OK) {
            err_text() = "instance " + std::to_string(b) + ": " + err_text();
            return us;
        }
        umax[b] = umax2[2 * b];
    }

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
    // the k = 0 coarse sweeps of all instances in one launch, one work-group
    // each (each touches only its own instance's buffers), as the
    // iterations' sweeps run; the values are those of one sweep per instance
    std::vector<ChainArgs<T>> args(2 * n);
    for (int b = 0; b < n; ++b) RPR_TRY(phase_setup<T>(p->sub[b], u0[b], umax[b], st, &args[b], false));
    for (int b = 0; b < n; ++b) {
        args[n + b] = args[b];
        args[n + b].mode = CHAIN_SWEEP;
    }
    std::memcpy(p->hchain.data(), args.data(), sizeof(ChainArgs<T>) * 2 * n);
    RPR_HIP(hipMemcpyAsync(p->bchain, p->hchain.data(), sizeof(ChainArgs<T>) * 2 * n, hipMemcpyHostToDevice, st));
    RPR_TRY(launch_chain_multi<T>(static_cast<const ChainArgs<T> *>(p->bchain) + n, n, p->bgmax, p->bshG, p->bM,
                                  st));
    if (timed) RPR_HIP(hipEventRecord(p->pev[0], st));
    const auto *insts = static_cast<const BatchInst<T> *>(p->binsts);
    // instances not known to be done: eager bursts enqueue the model phase
    // of these only (a done instance's model kernels find no rows and return
    // at once, so leaving them out changes nothing but the launches);
    // captured blocks hold every instance
    std::vector<char> live(n, 1);
    // (ev: the first of the iteration's three phase events, or -1)
    auto iteration = [&](hipStream_t s, int ev) -> rpr_status {
        // every unfinished (instance, slot) fine solve in one persistent launch
        RPR_TRY(zero(p->bcounter, 1, s));
        RPR_TRY(launch_prop_persistent<T>(insts, p->bitems, p->bn_items, p->bcounter, p->bgmax, p->bshF, p->bgrid,
                                          s));
        if (ev >= 0) RPR_HIP(hipEventRecord(p->pev[ev], s));
        for (int b = 0; b < n; ++b)
            if (live[b]) RPR_TRY(phase_model<T>(p->sub[b], args[b].inv_s, s));
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
        for (int b = 0; b < n; ++b) {
            done = done && p->sub[b]->ctrl_host->done != 0;
            live[b] = p->sub[b]->ctrl_host->done == 0;
        }
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

