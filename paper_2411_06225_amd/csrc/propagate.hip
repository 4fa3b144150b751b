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

// ------------------------------------------------------- persistent batch --
template <int KIND, typename T, int CPT, bool DBUF>
__global__ __launch_bounds__(1024) void k_prop_persistent(const BatchInst<T> *__restrict__ insts,
                                                          const int2 *__restrict__ items, int n_items,
                                                          int *__restrict__ counter)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();  // also: every thread has finished the previous item's LDS reads
        const int q = next;
        __syncthreads();  // every thread has read `next` before thread 0 replaces it
        if (q >= n_items) return;
        const int2 it = items[q];
        const BatchInst<T> &I = insts[it.x];
        if (I.ctrl[2] != 0 || it.y <= I.ctrl[0]) continue;  // slot final, or instance done
        slot_propagate<KIND, T, CPT, DBUF, false, 0, 0>(I.g, I.method, I.steps, I.dt,
                                                        I.U + (size_t)(it.y - 1) * I.g.d,
                                                        I.Fv + (size_t)it.y * I.g.d, reinterpret_cast<T *>(lds_raw));
    }
}

template <int KIND, typename T, int CPT, bool DBUF>
static rpr_status launch_persistent_one(const BatchInst<T> *insts, const int2 *items, int n_items, int *counter,
                                        const OnchipShape &sh, int grid, hipStream_t st)
{
    auto kern = k_prop_persistent<KIND, T, CPT, DBUF>;
    static bool attr_set = false;
    if (!attr_set) {
        RPR_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
        attr_set = true;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(sh.block), sh.lds, st, insts, items, n_items, counter);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}

template <int KIND, typename T>
rpr_status launch_prop_persistent_kind(const BatchInst<T> *insts, const int2 *items, int n_items, int *counter,
                                       const Geom &gmax, const OnchipShape &sh, int grid, hipStream_t st)
{
    (void)gmax;
    if (sh.maxt != 1024) return fail(RPR_ERR_UNSUPPORTED, "persistent batch needs the 1024-thread shape");
#define RPR_P_CPT(DB)                                                                                     \
    switch (sh.cpt) {                                                                                     \
    case 1: return launch_persistent_one<KIND, T, 1, DB>(insts, items, n_items, counter, sh, grid, st);   \
    case 2: return launch_persistent_one<KIND, T, 2, DB>(insts, items, n_items, counter, sh, grid, st);   \
    case 4: return launch_persistent_one<KIND, T, 4, DB>(insts, items, n_items, counter, sh, grid, st);   \
    case 8: return launch_persistent_one<KIND, T, 8, DB>(insts, items, n_items, counter, sh, grid, st);   \
    case 16: return launch_persistent_one<KIND, T, 16, DB>(insts, items, n_items, counter, sh, grid, st); \
    default: return fail(RPR_ERR_UNSUPPORTED, "no persistent instance for this strip length");          \
    }
    if (sh.dbuf) {
        RPR_P_CPT(true)
    } else {
        RPR_P_CPT(false)
    }
#undef RPR_P_CPT
}

// This file is compiled once per (right-hand side, precision) pair.
template rpr_status launch_prop_persistent_kind<RPR_KIND, RPR_REAL>(const BatchInst<RPR_REAL> *, const int2 *, int,
                                                                     int *, const Geom &, const OnchipShape &, int,
                                                                     hipStream_t);
template rpr_status launch_propagate_kind<RPR_KIND, RPR_REAL>(const Geom &, const OnchipShape &, int, int64_t,
                                                               double, int, const RPR_REAL *, RPR_REAL *,
                                                               const int *, hipStream_t);

}  // namespace rpr
