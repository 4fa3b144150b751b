// autotune.hip -- the launch-shape autotuner of plans.
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "plan.h"

// --------------------------------------------------------------- autotuner --
// Candidate launch shapes are timed on the plan's own buffers (zero-filled)
// with events on a private stream; the fastest is kept.  Results are cached
// per shape class in the process and, if RPR_TUNE_CACHE names a file, in that
// JSON file ({"key": value, ...}).

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
int tuned_prop_threads(const Geom &g, int esz, int method)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_load();
    const auto it = g_tune.find(prop_key(g, esz, method));
    return it == g_tune.end() ? 1024 : it->second;
}

// Tile shape of the one-pass RK4 form the autotuner chose for this
// propagator class (0, the default, when it has not run for it).
int tuned_variant(const Geom &g, int esz, int method)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_load();
    const auto it = g_tune.find(prop_key(g, esz, method) + ":v");
    return it == g_tune.end() ? 0 : it->second;
}

extern "C" rpr_status rpr_tune_set(const char *key, int32_t value)
{
    if (key == nullptr || *key == 0) return fail(RPR_ERR_INVALID_ARG, "rpr_tune_set: empty key");
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_load();
    if (value < 0) g_tune.erase(key);
    else g_tune[key] = value;
    return RPR_OK;
}

extern "C" rpr_status rpr_tune_get(const char *key, int32_t *value)
{
    if (key == nullptr || *key == 0 || value == nullptr) return fail(RPR_ERR_INVALID_ARG, "rpr_tune_get: null argument");
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_load();
    const auto it = g_tune.find(key);
    if (it == g_tune.end()) return fail(RPR_ERR_INVALID_ARG, std::string("rpr_tune_get: no entry ") + key);
    *value = it->second;
    return RPR_OK;
}

extern "C" int32_t rpr_tile_shapes(int32_t kind, int32_t precision)
{
    return fused_variants(kind, precision == RPR_FP64 ? 8 : 4);
}

extern "C" const char *rpr_tile_shape_name(int32_t kind, int32_t precision, int32_t v)
{
    const size_t elem = precision == RPR_FP64 ? 8 : 4;
    if (v < 0 || v >= fused_variants(kind, elem)) return nullptr;
    return fused_variant_name(kind, elem, v);
}

// Fraction by which a fine-propagator candidate must beat the best one timed
// before it (the work-group sizes, then the tile shapes in index order).
constexpr float kSwitchMargin = 0.05f;

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
    // (long strips) work-groups, or tiled through memory (2D grids) in each
    // tile shape of its one-pass form; every candidate's time (microseconds
    // per launch of min(steps, 32) steps) is kept in the table under
    // "<class>:t:<threads>:<shape>"
    const bool forced_tiled = p->shF.maxt == TILED_THREADS;
    const bool generic_F = p->shF.maxt == GENERIC_THREADS;  // one form, nothing to choose
    const std::string kv = kf + ":v";
    const bool haveV = g_tune.count(kv) != 0 || generic_F;
    const int nvar = fused_variants(g.kind, p->esz);
    if (!generic_F && ((!haveF && p->F.threads == 0 && !forced_tiled) || (forced_tiled && !haveV))) {
        const int64_t steps = p->F.steps < 32 ? p->F.steps : 32;
        float best = 1e30f;
        int best_mt = p->shF.maxt, best_v = 0;
        DevBuf trial;  // work arrays of the tiled candidate
        for (int mt : {1024, 512, TILED_THREADS}) {
            if (forced_tiled && mt != TILED_THREADS) continue;
            if (check_threads(g, p->esz, mt) != RPR_OK) continue;
            TiledWork<T> w{};
            if (mt == TILED_THREADS) {
                if (p->fwork) {
                    w = tiled_work<T>(p->fwork, (size_t)N * d);
                } else {
                    if (hipMalloc(&trial.p, 5 * (size_t)N * d * p->esz) != hipSuccess) {
                        (void)hipGetLastError();
                        trial.p = nullptr;
                        continue;
                    }
                    w = tiled_work<T>(trial.p, (size_t)N * d);
                }
            }
            const TiledWork<T> *wp = mt == TILED_THREADS ? &w : nullptr;
            for (int v = 0; v < (mt == TILED_THREADS ? nvar : 1); ++v) {
                if (mt == TILED_THREADS && !fused_variant_fits(g, p->esz, v)) continue;
                RPR_TRY(launch_propagate<T>(g, p->F.method, steps, p->dtF, N, U, Fv + d, nullptr, st, mt, wp, v));
                float ms = 0.f;
                RPR_HIP(hipEventRecord(e0, st));
                for (int r = 0; r < 3; ++r)
                    RPR_TRY(launch_propagate<T>(g, p->F.method, steps, p->dtF, N, U, Fv + d, nullptr, st, mt, wp, v));
                RPR_HIP(hipEventRecord(e1, st));
                RPR_HIP(hipEventSynchronize(e1));
                RPR_HIP(hipEventElapsedTime(&ms, e0, e1));
                std::ostringstream kt;
                kt << kf << ":t:" << mt << ":" << (mt == TILED_THREADS ? fused_variant_name(g.kind, p->esz, v) : "onchip");
                g_tune[kt.str()] = (int)(ms * 1000.f / 3.f);
                // a later candidate must win by kSwitchMargin: shapes within
                // the timing noise of each other would otherwise flip from
                // one process to the next
                if (ms < best * (1.f - kSwitchMargin)) { best = ms; best_mt = mt; best_v = mt == TILED_THREADS ? v : 0; }
            }
        }
        if (!forced_tiled) g_tune[kf] = best_mt;
        g_tune[kv] = best_v;
    }
    p->fvar = (!generic_F && g_tune.count(kv)) ? g_tune[kv] : 0;
    if (!forced_tiled && !generic_F) {
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
        a.gw = coarse_work<T>(p);
        a.tbG = rk_tableau(p->G.method);
        a.A = p->A;
        a.zeta = p->zeta;
        a.W = chain_W<T>(p);
        a.At = chain_At<T>(p);
        a.part = p->part;
        a.ctrl = p->ctrl;
        nn_args<T>(p, a);
        // the nearest-neighbour trials run with a store of two iterations'
        // pairs: the refit's distance pass grows with the store and is spread
        // over the sweep's work-groups, so an empty store would favour small
        // grids.  The trial pairs are zeros flagged non-finite (no refit
        // takes them); the store is emptied again after the trials.
        if (p->nn) {
            const int trial_rows = std::min(p->n_cap, 2 * N);
            RPR_TRY(zero(static_cast<T *>(p->Xs), (size_t)trial_rows * d, st));
            RPR_TRY(zero(p->Ps, (size_t)trial_rows * p->M, st));
            RPR_TRY(zero(p->oks, (size_t)trial_rows, st));
            RPR_HIP(hipStreamSynchronize(st));
            RPR_HIP(hipMemcpy(p->nrows, &trial_rows, sizeof(int), hipMemcpyHostToDevice));
        }
        float best = 1e30f;
        int best_n = p->nwg, best_gt = p->shG.maxt, best_b = p->shG.block;
        // coarse-solver shapes: the plan's, and for an on-chip G of free
        // thread count the 512-thread one too (longer strips, twice the
        // registers per thread)
        OnchipShape gshapes[2] = {p->shG, p->shG};
        int n_shapes = 1;
        if (p->G.threads == 0 && p->shG.maxt == 1024 && onchip_shape(g, p->esz, &gshapes[1], 512) &&
            check_threads(g, p->esz, 512) == RPR_OK)
            n_shapes = 2;
        // a tiled forward-Euler G in segment kernels: also the wide work-groups
        const bool wide_ok = p->seg_sweep && p->shG.maxt == TILED_THREADS && p->G.method == RPR_RK1;
        if (wide_ok) {
            gshapes[1].block = SWEEP_WIDE;
            n_shapes = 2;
        }
        const int cands[] = {1, cus / 16, cus / 8, cus / 4, cus / 2, cus};
        // the trials run the sweep in the plan's form
        if (p->seg_sweep) RPR_HIP(hipMemcpy(p->gchain, &a, sizeof(a), hipMemcpyHostToDevice));
        auto sweep = [&](const OnchipShape &sh, int c) -> rpr_status {
            if (p->seg_sweep)
                return launch_chain_graph<T>(static_cast<const ChainArgs<T> *>(p->gchain), a, sh, c, st);
            return launch_chain<T>(a, sh, c, st);
        };
        for (int s = 0; s < n_shapes; ++s) {
            const OnchipShape &sh = gshapes[s];
            int mwg = max_wg;  // grids beyond the plan's max_wg have no partial-sum rows
            if (s > 0 && !wide_ok) {
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
                RPR_TRY(launch_init_ctrl(p->ctrl, p->L_hist, p->chg_hist, st));
                RPR_TRY(sweep(sh, c));
                RPR_HIP(hipEventRecord(e0, st));
                RPR_TRY(launch_init_ctrl(p->ctrl, p->L_hist, p->chg_hist, st));
                RPR_TRY(sweep(sh, c));
                RPR_HIP(hipEventRecord(e1, st));
                RPR_HIP(hipEventSynchronize(e1));
                RPR_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) { best = ms; best_n = c; best_gt = sh.maxt; best_b = sh.block; }
            }
        }
        if (p->nn) RPR_TRY(zero(p->nrows, 1, st));
        g_tune[kc.str()] = best_n;
        g_tune[kc.str() + ":G"] = best_gt;
        g_tune[kc.str() + ":B"] = best_b;
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
    // the tiled sweep's work-group size
    const auto gb = g_tune.find(kc.str() + ":B");
    if (p->seg_sweep && p->shG.maxt == TILED_THREADS && p->G.method == RPR_RK1 && gb != g_tune.end() &&
        gb->second == SWEEP_WIDE)
        p->shG.block = SWEEP_WIDE;
    if (!p->fixed_nwg) p->nwg = g_tune[kc.str()] < max_wg ? g_tune[kc.str()] : max_wg;
    if (!haveF || !haveC || !haveV) tune_store();
    return RPR_OK;
}

template <typename T>
rpr_status autotune_plan(rpr_plan *p, int max_wg, int cus)
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

template rpr_status autotune_plan<double>(rpr_plan *, int, int);
template rpr_status autotune_plan<float>(rpr_plan *, int, int);

// ------------------------------------------------------- batch autotuner --
// The persistent fine-solve launch of a batch takes the next (instance, slot)
// item from a counter until the list is done; how many work-groups to launch
// (1 to 4 per CU) is timed on the batch's own buffers, zero-filled, with at
// most 32 steps per item, and kept per shape class of the batch (rhs, largest
// grid, precision, strip length, item count).  The chains have one shape per
// batch (one work-group per instance), so nothing else is left to choose.
template <typename T>
static rpr_status autotune_batch_run(rpr_plan *p, int cus, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    const int n = (int)p->sub.size();
    std::ostringstream key;
    key << "batch:" << p->bgmax.kind << ":" << p->bgmax.nx << "x" << p->bgmax.ny << ":" << p->esz << ":cpt"
        << p->bshF.cpt << ":items" << p->bn_items;
    const std::string kg = key.str() + ":grid";
    if (g_tune.count(kg) == 0) {
        std::vector<BatchInst<T>> hi(n);
        for (int b = 0; b < n; ++b) {
            rpr_plan *q = p->sub[b];
            RPR_TRY(zero(static_cast<T *>(q->U), (size_t)(q->N + 1) * q->g.d, st));
            RPR_TRY(zero(static_cast<T *>(q->Fv), (size_t)(q->N + 1) * q->g.d, st));
            RPR_TRY(launch_init_ctrl(q->ctrl, q->L_hist, q->chg_hist, st));
            hi[b] = BatchInst<T>{q->g, q->F.method, (long long)std::min<int64_t>(q->F.steps, 32), q->dtF,
                                 static_cast<const T *>(q->U), static_cast<T *>(q->Fv),
                                 reinterpret_cast<const int *>(q->ctrl)};
        }
        DevBuf ti;
        RPR_HIP(hipMalloc(&ti.p, sizeof(BatchInst<T>) * n));
        RPR_HIP(hipMemcpyAsync(ti.p, hi.data(), sizeof(BatchInst<T>) * n, hipMemcpyHostToDevice, st));
        RPR_HIP(hipStreamSynchronize(st));
        const auto *insts = static_cast<const BatchInst<T> *>(ti.p);
        float best = 1e30f;
        int best_m = 2;
        for (int m = 1; m <= 4; ++m) {
            const int grid = std::min(p->bn_items, m * cus);
            auto launch = [&]() -> rpr_status {
                RPR_TRY(zero(p->bcounter, 1, st));
                return launch_prop_persistent<T>(insts, p->bitems, p->bn_items, p->bcounter, p->bgmax, p->bshF, grid,
                                                 st);
            };
            RPR_TRY(launch());
            RPR_HIP(hipEventRecord(e0, st));
            RPR_TRY(launch());
            RPR_HIP(hipEventRecord(e1, st));
            RPR_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            RPR_HIP(hipEventElapsedTime(&ms, e0, e1));
            g_tune[kg + ":t:" + std::to_string(m)] = (int)(ms * 1000.f);
            if (ms < best) {
                best = ms;
                best_m = m;
            }
            if (grid == p->bn_items) break;  // more work-groups than items add nothing
        }
        g_tune[kg] = best_m;
        tune_store();
    }
    p->bgrid = std::min(p->bn_items, g_tune[kg] * cus);
    return RPR_OK;
}

template <typename T>
rpr_status autotune_batch(rpr_plan *p, int cus)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_load();
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rpr_status rc = RPR_OK;
    if (hipStreamCreate(&st) != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = fail(RPR_ERR_HIP, "autotune: cannot create a stream or events");
    if (rc == RPR_OK) rc = autotune_batch_run<T>(p, cus, st, e0, e1);
    if (st) (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    return rc;
}

template rpr_status autotune_batch<double>(rpr_plan *, int);
template rpr_status autotune_batch<float>(rpr_plan *, int);
