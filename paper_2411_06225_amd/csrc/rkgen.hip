// rkgen.hip -- the propagators F and G over one slice (Sec. 2) by any
// explicit Runge-Kutta tableau over states in memory (rkgen.h): the
// eighth-order fine solver for every system, and every propagator of the 3D
// Brusselator.  One launch per stage over the cells of all states.
#include "rkgen.h"

namespace rpr {

// Stage `stage` of step `step` of n states; block (x: cells, y: state b).
// States of final slots (b < ctrl[0]) and finished runs (ctrl[2]) return.
template <int KIND, typename T>
__global__ __launch_bounds__(256) void k_rkgen_stage(Geom g, Tableau tb, int stage, long long step, long long steps,
                                                     double dt, const T *__restrict__ in, T *__restrict__ out,
                                                     TiledWork<T> w, size_t nd, const int *__restrict__ ctrl)
{
    const int b = blockIdx.y;
    if (ctrl != nullptr && (ctrl[2] != 0 || b < ctrl[0])) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nc) return;
    const size_t off = (size_t)b * g.d;
    const TiledWork<T> wb{w.u + off, w.acc + off, w.ya + off, w.yb + off, w.cmp + off};
    const RkIO<T> io = rkgen_io<T>(tb.s, stage, step, steps, in + off, out + off, nullptr, wb);
    rkgen_cell<KIND, T>(g, tb, stage, dt, c, io.y, wb.acc, nd, io.u, io.ynext, io.uout, io.uout2, wb.cmp,
                        step == 0 ? 1 : 0);
}

template <int KIND, typename T>
rpr_status launch_rkgen_kind(const Geom &g, int method, int64_t steps, double dt, int n, const T *in, T *out,
                             const TiledWork<T> &w, const int *ctrl, hipStream_t st)
{
    if (n <= 0) return RPR_OK;
    if (n > 65535) return fail(RPR_ERR_UNSUPPORTED, "generic propagator: more than 65535 states per launch");
    const Tableau tb = rk_tableau(method);
    const dim3 grid((unsigned)((g.nc + 255) / 256), (unsigned)n);
    const size_t nd = (size_t)n * g.d;
    for (long long s = 0; s < (long long)steps; ++s)
        for (int i = 0; i < tb.s; ++i) {
            hipLaunchKernelGGL((k_rkgen_stage<KIND, T>), grid, dim3(256), 0, st, g, tb, i, s, (long long)steps, dt,
                               in, out, w, nd, ctrl);
            RPR_HIP(hipGetLastError());
        }
    return RPR_OK;
}

// This file is compiled once per (right-hand side, precision) pair.
template rpr_status launch_rkgen_kind<RPR_KIND, RPR_REAL>(const Geom &, int, int64_t, double, int, const RPR_REAL *,
                                                           RPR_REAL *, const TiledWork<RPR_REAL> &, const int *,
                                                           hipStream_t);

}  // namespace rpr
