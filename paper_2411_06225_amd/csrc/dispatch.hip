// dispatch.hip -- host-side shape selection and the dispatch from a runtime
// right-hand-side kind to the per-kind kernel objects.
#include "chain.h"
#include "swefused.h"
#include "rkgen.h"
#include "slotprop.h"
#include "tiledprop.h"

namespace rpr {

static int pow2_at_least(int v)
{
    int p = 1;
    while (p < v) p *= 2;
    return p;
}

bool onchip_shape(const Geom &g, size_t elem, OnchipShape *sh, int max_threads)
{
    int cpt, block;
    if (max_threads != 512) max_threads = 1024;
    if (g.kind == RPR_BRUSS3D) return false;  // the generic propagator serves the 3D system
    if (g.kind == RPR_BURGERS1D) {
        cpt = pow2_at_least((g.nc + max_threads - 1) / max_threads);
        if (cpt < 2 && g.nc >= 128) cpt = 2;
        block = (g.nc + cpt - 1) / cpt;
    } else {
        if (g.nx > max_threads) return false;
        cpt = 1;
        while (g.nx * ((g.ny + cpt - 1) / cpt) > max_threads) cpt *= 2;
        block = g.nx * ((g.ny + cpt - 1) / cpt);
    }
    if (cpt > 16) return false;
    const size_t one = (size_t)padded_elems(g) * elem;
    if (one > kMaxLds) return false;
    sh->block = block;
    sh->maxt = max_threads;
    sh->cpt = cpt;
    sh->full = (g.kind == RPR_BURGERS1D ? g.nc : g.ny) % cpt == 0;
    sh->dbuf = 2 * one <= kMaxLds;
    sh->lds = sh->dbuf ? 2 * one : one;
    return true;
}

namespace {
struct NoLaunch {
    template <int CPT, bool DBUF, bool FULL, int NX, int NY, int MAXT>
    rpr_status run() { return RPR_OK; }
};
template <typename T>
rpr_status has_instance_t(const Geom &g, const OnchipShape &sh)
{
    NoLaunch f;
    switch (g.kind) {
    case RPR_BURGERS1D: return visit_shape_kind<RPR_BURGERS1D, T>(g, sh, f);
    case RPR_DIFFREACT2D: return visit_shape_kind<RPR_DIFFREACT2D, T>(g, sh, f);
    case RPR_BRUSS2D: return visit_shape_kind<RPR_BRUSS2D, T>(g, sh, f);
    case RPR_SWE2D: return visit_shape_kind<RPR_SWE2D, T>(g, sh, f);
    default: return fail(RPR_ERR_INVALID_ARG, "unknown right-hand side");
    }
}
}  // namespace

OnchipShape generic_shape(const Geom &g, size_t elem)
{
    (void)g;
    (void)elem;
    OnchipShape sh{};
    sh.block = 256;
    sh.maxt = GENERIC_THREADS;
    sh.lds = 0;
    return sh;
}

OnchipShape tiled_shape(const Geom &g, size_t elem)
{
    OnchipShape sh{};
    sh.block = TT_THREADS;
    sh.maxt = TILED_THREADS;
    // the coarse solver of the sweep also runs several Euler steps per tile
    sh.lds = std::max(tiled_lds(g, elem), euler_multi_lds(g, elem));
    return sh;
}

rpr_status check_threads(const Geom &g, size_t elem, int threads)
{
    if (threads == GENERIC_THREADS) return RPR_OK;
    if (g.kind == RPR_BRUSS3D)
        return fail(RPR_ERR_UNSUPPORTED, "the 3D system runs on the generic propagator only (threads 0 or 128)");
    if (threads == TILED_THREADS)
        return g.kind == RPR_BURGERS1D ? fail(RPR_ERR_UNSUPPORTED, "the tiled propagator serves 2D grids only")
                                       : RPR_OK;
    OnchipShape sh;
    if (!onchip_shape(g, elem, &sh, threads))
        return fail(RPR_ERR_UNSUPPORTED, "the slot state does not fit one work-group's LDS");
    const rpr_status st = elem == 8 ? has_instance_t<double>(g, sh) : has_instance_t<float>(g, sh);
    if (st != RPR_OK)
        return fail(RPR_ERR_UNSUPPORTED, "no " + std::to_string(threads) + "-thread kernel for this grid");
    return RPR_OK;
}

template <typename T>
rpr_status launch_propagate(const Geom &g, int method, int64_t steps, double dt, int n, const T *in, T *out,
                            const int *ctrl, hipStream_t st, int max_threads, const TiledWork<T> *tw, int variant)
{
    if (n <= 0) return RPR_OK;
    if (max_threads == GENERIC_THREADS) {
        if (!tw) return fail(RPR_ERR_INVALID_ARG, "propagate: the generic form needs work arrays");
        switch (g.kind) {
        case RPR_BURGERS1D: return launch_rkgen_kind<RPR_BURGERS1D, T>(g, method, steps, dt, n, in, out, *tw, ctrl, st);
        case RPR_DIFFREACT2D: return launch_rkgen_kind<RPR_DIFFREACT2D, T>(g, method, steps, dt, n, in, out, *tw, ctrl, st);
        case RPR_BRUSS2D: return launch_rkgen_kind<RPR_BRUSS2D, T>(g, method, steps, dt, n, in, out, *tw, ctrl, st);
        case RPR_SWE2D: return launch_rkgen_kind<RPR_SWE2D, T>(g, method, steps, dt, n, in, out, *tw, ctrl, st);
        case RPR_BRUSS3D: return launch_rkgen_kind<RPR_BRUSS3D, T>(g, method, steps, dt, n, in, out, *tw, ctrl, st);
        default: return fail(RPR_ERR_INVALID_ARG, "propagate: unknown right-hand side");
        }
    }
    if (g.kind == RPR_BRUSS3D) return fail(RPR_ERR_UNSUPPORTED, "the 3D system runs on the generic propagator only");
    if (max_threads == TILED_THREADS) {
        if (!tw) return fail(RPR_ERR_INVALID_ARG, "propagate: the tiled form needs work arrays");
        switch (g.kind) {
        case RPR_DIFFREACT2D: return launch_prop_tiled_kind<RPR_DIFFREACT2D, T>(g, method, steps, dt, n, in, out, *tw, ctrl, st, variant);
        case RPR_BRUSS2D: return launch_prop_tiled_kind<RPR_BRUSS2D, T>(g, method, steps, dt, n, in, out, *tw, ctrl, st, variant);
        case RPR_SWE2D: return launch_prop_tiled_kind<RPR_SWE2D, T>(g, method, steps, dt, n, in, out, *tw, ctrl, st, variant);
        default: return fail(RPR_ERR_UNSUPPORTED, "propagate: the tiled form serves 2D grids only");
        }
    }
    OnchipShape sh;
    if (!onchip_shape(g, sizeof(T), &sh, max_threads))
        return fail(RPR_ERR_UNSUPPORTED, "propagate: the state does not fit one work-group's LDS");
    switch (g.kind) {
    case RPR_BURGERS1D: return launch_propagate_kind<RPR_BURGERS1D, T>(g, sh, method, steps, dt, n, in, out, ctrl, st);
    case RPR_DIFFREACT2D: return launch_propagate_kind<RPR_DIFFREACT2D, T>(g, sh, method, steps, dt, n, in, out, ctrl, st);
    case RPR_BRUSS2D: return launch_propagate_kind<RPR_BRUSS2D, T>(g, sh, method, steps, dt, n, in, out, ctrl, st);
    case RPR_SWE2D: return launch_propagate_kind<RPR_SWE2D, T>(g, sh, method, steps, dt, n, in, out, ctrl, st);
    default: return fail(RPR_ERR_INVALID_ARG, "propagate: unknown right-hand side");
    }
}
template rpr_status launch_propagate<double>(const Geom &, int, int64_t, double, int, const double *, double *,
                                             const int *, hipStream_t, int, const TiledWork<double> *, int);
template rpr_status launch_propagate<float>(const Geom &, int, int64_t, double, int, const float *, float *,
                                            const int *, hipStream_t, int, const TiledWork<float> *, int);

// Tile shapes of the one-pass RK4 kernels (the order of the switches in
// tiled.hip): shallow water (rows per wavefront R, wavefronts NW), the
// Laplacian systems (tile rows FY, threads NT).
namespace {
const char *const kSweF32[] = {"R5NW8", "R4NW8", "R4NW10", "R8NW5", "R2NW16", "rows:C3R2NW12", "rows:C2R3NW12"};
const char *const kSweF64[] = {"R4NW8", "R4NW6", "R3NW8", "R2NW12", "rows:C3R2NW8", "rows:C2R3NW8"};
const char *const kLap[] = {"FY32NT512", "FY16NT256", "FY32NT256", "FY64NT512"};
// cells per lane of the full-row shapes (0: the 56-column tiles, any grid)
const int kSweF32C[] = {0, 0, 0, 0, 0, 3, 2};
const int kSweF64C[] = {0, 0, 0, 0, 3, 2};
}  // namespace

int fused_variants(int kind, size_t elem)
{
    if (kind == RPR_SWE2D) return elem == 4 ? 7 : 6;
    if (kind == RPR_DIFFREACT2D || kind == RPR_BRUSS2D) return 4;
    return 1;
}

const char *fused_variant_name(int kind, size_t elem, int v)
{
    if (v < 0 || v >= fused_variants(kind, elem)) return "default";
    if (kind == RPR_SWE2D) return elem == 4 ? kSweF32[v] : kSweF64[v];
    if (kind == RPR_DIFFREACT2D || kind == RPR_BRUSS2D) return kLap[v];
    return "default";
}

bool fused_variant_fits(const Geom &g, size_t elem, int v)
{
    if (v < 0 || v >= fused_variants(g.kind, elem)) return false;
    if (g.kind != RPR_SWE2D) return true;
    const int C = elem == 4 ? kSweF32C[v] : kSweF64C[v];
    return C == 0 || swr_fits(g, C);
}

size_t chain_lds(const OnchipShape &sh, int M)
{
    // the coarse solver's stage buffers, or the readout's neuron vector and
    // partial sums (up to 16 wavefronts x 2 tiles x 64 columns), or the hidden
    // layer's per-wavefront sums (16 x M), whichever is larger
    size_t red = (size_t)(M + 2048 + 64) * sizeof(double);
    if ((size_t)16 * M * sizeof(double) > red) red = (size_t)16 * M * sizeof(double);
    return sh.lds > red ? sh.lds : red;
}

template <typename T>
rpr_status launch_chain(const ChainArgs<T> &a, const OnchipShape &sh, int nwg, hipStream_t st, int *max_wg)
{
    switch (a.g.kind) {
    case RPR_BURGERS1D: return launch_chain_kind<RPR_BURGERS1D, T>(a, sh, nwg, st, max_wg);
    case RPR_DIFFREACT2D: return launch_chain_kind<RPR_DIFFREACT2D, T>(a, sh, nwg, st, max_wg);
    case RPR_BRUSS2D: return launch_chain_kind<RPR_BRUSS2D, T>(a, sh, nwg, st, max_wg);
    case RPR_SWE2D: return launch_chain_kind<RPR_SWE2D, T>(a, sh, nwg, st, max_wg);
    case RPR_BRUSS3D: return launch_chain_kind<RPR_BRUSS3D, T>(a, sh, nwg, st, max_wg);
    default: return fail(RPR_ERR_INVALID_ARG, "chain: unknown right-hand side");
    }
}
template rpr_status launch_chain<double>(const ChainArgs<double> &, const OnchipShape &, int, hipStream_t, int *);
template rpr_status launch_chain<float>(const ChainArgs<float> &, const OnchipShape &, int, hipStream_t, int *);

template <typename T>
rpr_status launch_sweep_segments(const ChainArgs<T> &a, const OnchipShape &sh, int nwg, hipStream_t st)
{
    switch (a.g.kind) {
    case RPR_BURGERS1D: return launch_sweep_segments_kind<RPR_BURGERS1D, T>(a, sh, nwg, st);
    case RPR_DIFFREACT2D: return launch_sweep_segments_kind<RPR_DIFFREACT2D, T>(a, sh, nwg, st);
    case RPR_BRUSS2D: return launch_sweep_segments_kind<RPR_BRUSS2D, T>(a, sh, nwg, st);
    case RPR_SWE2D: return launch_sweep_segments_kind<RPR_SWE2D, T>(a, sh, nwg, st);
    case RPR_BRUSS3D: return launch_sweep_segments_kind<RPR_BRUSS3D, T>(a, sh, nwg, st);
    default: return fail(RPR_ERR_INVALID_ARG, "chain: unknown right-hand side");
    }
}
template rpr_status launch_sweep_segments<double>(const ChainArgs<double> &, const OnchipShape &, int, hipStream_t);
template rpr_status launch_sweep_segments<float>(const ChainArgs<float> &, const OnchipShape &, int, hipStream_t);

template <typename T>
rpr_status launch_chain_graph(const ChainArgs<T> *args_dev, const ChainArgs<T> &a, const OnchipShape &sh, int nwg,
                              hipStream_t st)
{
    switch (a.g.kind) {
    case RPR_BURGERS1D: return launch_chain_graph_kind<RPR_BURGERS1D, T>(args_dev, a, sh, nwg, st);
    case RPR_DIFFREACT2D: return launch_chain_graph_kind<RPR_DIFFREACT2D, T>(args_dev, a, sh, nwg, st);
    case RPR_BRUSS2D: return launch_chain_graph_kind<RPR_BRUSS2D, T>(args_dev, a, sh, nwg, st);
    case RPR_SWE2D: return launch_chain_graph_kind<RPR_SWE2D, T>(args_dev, a, sh, nwg, st);
    case RPR_BRUSS3D: return launch_chain_graph_kind<RPR_BRUSS3D, T>(args_dev, a, sh, nwg, st);
    default: return fail(RPR_ERR_INVALID_ARG, "chain: unknown right-hand side");
    }
}
template rpr_status launch_chain_graph<double>(const ChainArgs<double> *, const ChainArgs<double> &,
                                               const OnchipShape &, int, hipStream_t);
template rpr_status launch_chain_graph<float>(const ChainArgs<float> *, const ChainArgs<float> &, const OnchipShape &,
                                              int, hipStream_t);

template <typename T>
rpr_status launch_prop_persistent(const BatchInst<T> *insts, const int2 *items, int n_items, int *counter,
                                  const Geom &gmax, const OnchipShape &sh, int grid, hipStream_t st)
{
    switch (gmax.kind) {
    case RPR_BURGERS1D: return launch_prop_persistent_kind<RPR_BURGERS1D, T>(insts, items, n_items, counter, gmax, sh, grid, st);
    case RPR_DIFFREACT2D: return launch_prop_persistent_kind<RPR_DIFFREACT2D, T>(insts, items, n_items, counter, gmax, sh, grid, st);
    case RPR_BRUSS2D: return launch_prop_persistent_kind<RPR_BRUSS2D, T>(insts, items, n_items, counter, gmax, sh, grid, st);
    case RPR_SWE2D: return launch_prop_persistent_kind<RPR_SWE2D, T>(insts, items, n_items, counter, gmax, sh, grid, st);
    default: return fail(RPR_ERR_INVALID_ARG, "batch: unknown right-hand side");
    }
}
template rpr_status launch_prop_persistent<double>(const BatchInst<double> *, const int2 *, int, int *, const Geom &,
                                                   const OnchipShape &, int, hipStream_t);
template rpr_status launch_prop_persistent<float>(const BatchInst<float> *, const int2 *, int, int *, const Geom &,
                                                  const OnchipShape &, int, hipStream_t);

template <typename T>
rpr_status launch_chain_multi(const ChainArgs<T> *args_dev, int n_inst, const Geom &gmax, const OnchipShape &sh,
                              int M, hipStream_t st)
{
    switch (gmax.kind) {
    case RPR_BURGERS1D: return launch_chain_multi_kind<RPR_BURGERS1D, T>(args_dev, n_inst, gmax, sh, M, st);
    case RPR_DIFFREACT2D: return launch_chain_multi_kind<RPR_DIFFREACT2D, T>(args_dev, n_inst, gmax, sh, M, st);
    case RPR_BRUSS2D: return launch_chain_multi_kind<RPR_BRUSS2D, T>(args_dev, n_inst, gmax, sh, M, st);
    case RPR_SWE2D: return launch_chain_multi_kind<RPR_SWE2D, T>(args_dev, n_inst, gmax, sh, M, st);
    case RPR_BRUSS3D: return launch_chain_multi_kind<RPR_BRUSS3D, T>(args_dev, n_inst, gmax, sh, M, st);
    default: return fail(RPR_ERR_INVALID_ARG, "batch: unknown right-hand side");
    }
}
template rpr_status launch_chain_multi<double>(const ChainArgs<double> *, int, const Geom &, const OnchipShape &, int,
                                               hipStream_t);
template rpr_status launch_chain_multi<float>(const ChainArgs<float> *, int, const Geom &, const OnchipShape &, int,
                                              hipStream_t);

}  // namespace rpr
