// propagate.hip -- the propagators F and G over one slice (Sec. 2), on chip.
//
// One work-group per slot; see slotprop.h for the decomposition.  The grid is
// indexed by slot; with a control block the work-groups of final slots exit
// at once, so the same launch serves every Parareal iteration.
#include "slotprop.h"

namespace rpr {

template <int KIND, typename T, int CPT, bool DBUF, bool FULL, int NX, int NY, int MAXT>
__global__ __launch_bounds__(MAXT) void k_prop_onchip(Geom g, int method, long long steps, double dt,
                                                      const T *__restrict__ in, T *__restrict__ out,
                                                      const int *__restrict__ ctrl)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int b = blockIdx.x;
    if (ctrl != nullptr && (ctrl[2] != 0 || b < ctrl[0])) return;
    slot_propagate<KIND, T, CPT, DBUF, FULL, NX, NY>(g, method, steps, dt, in + (size_t)b * g.d, out + (size_t)b * g.d,
                                       reinterpret_cast<T *>(lds_raw));
}


template <int KIND, typename T>
struct PropLauncher {
    const Geom &g;
    const OnchipShape &sh;
    int method;
    int64_t steps;
    double dt;
    int n;
    const T *in;
    T *out;
    const int *ctrl;
    hipStream_t st;

    template <int CPT, bool DBUF, bool FULL, int NX, int NY, int MAXT>
    rpr_status run()
    {
        auto kern = k_prop_onchip<KIND, T, CPT, DBUF, FULL, NX, NY, MAXT>;
        static bool attr_set = false;
        if (!attr_set) {
            RPR_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)kMaxLds));
            attr_set = true;
        }
        hipLaunchKernelGGL(kern, dim3(n), dim3(sh.block), sh.lds, st, g, method, (long long)steps, dt, in,
                           out, ctrl);
        RPR_HIP(hipGetLastError());
        return RPR_OK;
    }
};

template <int KIND, typename T>
rpr_status launch_propagate_kind(const Geom &g, const OnchipShape &sh, int method, int64_t steps, double dt,
                                 int n, const T *in, T *out, const int *ctrl, hipStream_t st)
{
    PropLauncher<KIND, T> L{g, sh, method, steps, dt, n, in, out, ctrl, st};
    return visit_shape_kind<KIND, T>(g, sh, L);
}

// This file is compiled once per (right-hand side, precision) pair.
template rpr_status launch_propagate_kind<RPR_KIND, RPR_REAL>(const Geom &, const OnchipShape &, int, int64_t,
                                                               double, int, const RPR_REAL *, RPR_REAL *,
                                                               const int *, hipStream_t);

}  // namespace rpr
