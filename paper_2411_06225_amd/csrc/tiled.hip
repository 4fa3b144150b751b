// tiled.hip -- the propagators F and G over one slice (Sec. 2) for slot
// states too large for one work-group: passes over the tiles of every slot
// state (tiledprop.h), one per RK stage (64 x 16-cell tiles), or one per RK4
// step for the 5-point Laplacian systems (64 x 32-cell tiles) and for
// shallow water (swefused.h: 56-column tiles, or whole rows per wavefront).
#include "swefused.h"
#include "tiledprop.h"

namespace rpr {

// Tile of the one-pass RK4 kernel: 64 x 32 cells on 512 threads (against
// 64 x 16 on 256: 1.41 instead of 1.69 region cells per tile cell, 11 %
// less time per step in FP32 and 3 % in FP64 on 128 x 128 Brusselator states)
#ifndef FUSED_FY
#define FUSED_FY 32
#define FUSED_NT 512
#endif

// ------------------------------------------------------------ tiled form --
// One stage of the propagation of n slot states too large for one
// work-group: a block updates one tile of slot b (in + b d -> out + b d,
// work arrays at b d), the pair taken from the block id by tile_of_block.
// Blocks of final slots exit at once.
template <int KIND, typename T, int STAGE>
__global__ __launch_bounds__(TT_THREADS) void k_prop_tiled(Geom g, int method, long long step, long long steps,
                                                           double dt, int n, const T *__restrict__ in,
                                                           T *__restrict__ out, TiledWork<T> w,
                                                           const int *__restrict__ ctrl)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int tile, b;
    tile_of_block((int)blockIdx.x, tiles_of(g), n, tile, b);
    if (ctrl != nullptr && (ctrl[2] != 0 || b < ctrl[0])) return;
    const size_t off = (size_t)b * g.d;
    const TiledWork<T> wb{w.u + off, w.acc ? w.acc + off : nullptr, w.ya + off, w.yb ? w.yb + off : nullptr,
                          w.cmp ? w.cmp + off : nullptr};
    const StageIO<T> io = stage_io<T>(method, STAGE, step, steps, in + off, out + off, nullptr, wb);
    stage_tile<KIND, T, STAGE>(g, tile, dt, io, reinterpret_cast<T *>(lds_raw));
}

// One whole RK4 step (rk4_tile_fused) of a tile of slot b; the state
// alternates between the work arrays u and ya, in on the first step and out
// after the last.
template <int KIND, typename T, int FY, int NT>
__global__ __launch_bounds__(NT) void k_prop_rk4_fused(Geom g, long long step, long long steps, double dt, int n,
                                                       const T *__restrict__ in, T *__restrict__ out, TiledWork<T> w,
                                                       const int *__restrict__ ctrl)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int tile, b;
    tile_of_block((int)blockIdx.x, fused_tiles_of<FY>(g), n, tile, b);
    if (ctrl != nullptr && (ctrl[2] != 0 || b < ctrl[0])) return;
    const size_t off = (size_t)b * g.d;
    T *buf[2] = {w.u + off, w.ya + off};
    const T *src = step == 0 ? in + off : buf[(step - 1) & 1];
    T *dst = step == steps - 1 ? out + off : buf[step & 1];
    rk4_tile_fused<KIND, T, FY, NT>(g, tile, dt, src, dst, w.cmp ? w.cmp + off : nullptr, step == 0 ? 1 : 0,
                                    reinterpret_cast<T *>(lds_raw));
}

// One whole RK4 step of a shallow-water tile (swe_rk4_tile); the state
// alternates between the work arrays u and ya as in k_prop_rk4_fused.
template <typename T, int R, int NW>
__global__ __launch_bounds__(64 * NW) void k_prop_swe_fused(Geom g, long long step, long long steps, double dt, int n,
                                                            const T *__restrict__ in, T *__restrict__ out,
                                                            TiledWork<T> w, const int *__restrict__ ctrl)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int tile, b;
    tile_of_block((int)blockIdx.x, swf_tiles_of<R, NW>(g), n, tile, b);
    if (ctrl != nullptr && (ctrl[2] != 0 || b < ctrl[0])) return;
    const size_t off = (size_t)b * g.d;
    T *buf[2] = {w.u + off, w.ya + off};
    const T *src = step == 0 ? in + off : buf[(step - 1) & 1];
    T *dst = step == steps - 1 ? out + off : buf[step & 1];
    swe_rk4_tile<T, R, NW>(g, tile, dt, src, dst, w.cmp ? w.cmp + off : nullptr, step == 0 ? 1 : 0,
                           reinterpret_cast<T *>(lds_raw));
}

// One whole RK4 step of a shallow-water tile in the full-row form
// (swe_rk4_rows).
template <typename T, int C, int R, int NW>
__global__ __launch_bounds__(64 * NW) void k_prop_swe_rows(Geom g, long long step, long long steps, double dt, int n,
                                                           const T *__restrict__ in, T *__restrict__ out,
                                                           TiledWork<T> w, const int *__restrict__ ctrl)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int tile, b;
    tile_of_block((int)blockIdx.x, swr_tiles_of<C, R, NW>(g), n, tile, b);
    if (ctrl != nullptr && (ctrl[2] != 0 || b < ctrl[0])) return;
    const size_t off = (size_t)b * g.d;
    T *buf[2] = {w.u + off, w.ya + off};
    const T *src = step == 0 ? in + off : buf[(step - 1) & 1];
    T *dst = step == steps - 1 ? out + off : buf[step & 1];
    swe_rk4_rows<T, C, R, NW>(g, tile, dt, src, dst, w.cmp ? w.cmp + off : nullptr, step == 0 ? 1 : 0,
                              reinterpret_cast<T *>(lds_raw));
}

template <typename T, int C, int R, int NW>
static rpr_status launch_swe_rows(const Geom &g, int64_t steps, double dt, int n, const T *in, T *out,
                                  const TiledWork<T> &w, const int *ctrl, hipStream_t st)
{
    static_assert((size_t)NW * 9 * 64 * C * sizeof(T) <= kMaxLds, "full-row tile exceeds LDS");
    if (!swr_fits(g, C)) return fail(RPR_ERR_UNSUPPORTED, "shallow-water full-row tile: grid rows do not fit");
    auto kern = k_prop_swe_rows<T, C, R, NW>;
    static bool attr_set = false;
    if (!attr_set) {
        RPR_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
        attr_set = true;
    }
    if ((long long)swr_tiles_of<C, R, NW>(g) * n > 0x7fffffffLL)
        return fail(RPR_ERR_UNSUPPORTED, "tiled propagator: more than 2^31 tiles per launch");
    const dim3 grid((unsigned)(swr_tiles_of<C, R, NW>(g) * n));
    const size_t lds = swr_lds<C, R, NW>(sizeof(T));
    for (long long s = 0; s < (long long)steps; ++s) {
        hipLaunchKernelGGL(kern, grid, dim3(64 * NW), lds, st, g, s, (long long)steps, dt, n, in, out, w, ctrl);
        RPR_HIP(hipGetLastError());
    }
    return RPR_OK;
}

template <typename T, int R, int NW>
static rpr_status launch_swe_fused(const Geom &g, int64_t steps, double dt, int n, const T *in, T *out,
                                   const TiledWork<T> &w, const int *ctrl, hipStream_t st)
{
    auto kern = k_prop_swe_fused<T, R, NW>;
    static bool attr_set = false;
    if (!attr_set) {
        RPR_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
        attr_set = true;
    }
    if ((long long)swf_tiles_of<R, NW>(g) * n > 0x7fffffffLL)
        return fail(RPR_ERR_UNSUPPORTED, "tiled propagator: more than 2^31 tiles per launch");
    const dim3 grid((unsigned)(swf_tiles_of<R, NW>(g) * n));
    const size_t lds = swf_lds<R, NW>(sizeof(T));
    for (long long s = 0; s < (long long)steps; ++s) {
        hipLaunchKernelGGL(kern, grid, dim3(64 * NW), lds, st, g, s, (long long)steps, dt, n, in, out, w, ctrl);
        RPR_HIP(hipGetLastError());
    }
    return RPR_OK;
}

template <int KIND, typename T, int FY, int NT>
static rpr_status launch_lap_fused(const Geom &g, int64_t steps, double dt, int n, const T *in, T *out,
                                   const TiledWork<T> &w, const int *ctrl, hipStream_t st)
{
    auto kern = k_prop_rk4_fused<KIND, T, FY, NT>;
    const size_t flds = rk4_fused_lds<FY>(g, sizeof(T));
    if (flds > 64 * 1024) {
        static bool attr_set = false;
        if (!attr_set) {
            RPR_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)kMaxLds));
            attr_set = true;
        }
    }
    if ((long long)fused_tiles_of<FY>(g) * n > 0x7fffffffLL)
        return fail(RPR_ERR_UNSUPPORTED, "tiled propagator: more than 2^31 tiles per launch");
    const dim3 fgrid((unsigned)(fused_tiles_of<FY>(g) * n));
    for (long long s = 0; s < (long long)steps; ++s) {
        hipLaunchKernelGGL(kern, fgrid, dim3(NT), flds, st, g, s, (long long)steps, dt, n, in, out, w, ctrl);
        RPR_HIP(hipGetLastError());
    }
    return RPR_OK;
}

template <int KIND, typename T>
rpr_status launch_prop_tiled_kind(const Geom &g, int method, int64_t steps, double dt, int n, const T *in, T *out,
                                  const TiledWork<T> &w, const int *ctrl, hipStream_t st, int variant)
{
    if constexpr (KIND == RPR_BURGERS1D) {
        return fail(RPR_ERR_UNSUPPORTED, "the tiled propagator serves 2D grids only");
    } else {
        if (n <= 0) return RPR_OK;
        if ((long long)tiles_of(g) * n > 0x7fffffffLL)
            return fail(RPR_ERR_UNSUPPORTED, "tiled propagator: more than 2^31 tiles per launch");
        const dim3 grid((unsigned)(tiles_of(g) * n));
        const size_t lds = tiled_lds(g, sizeof(T));
        const long long ns = (long long)steps;
        if constexpr (KIND == RPR_SWE2D) {
            // a whole RK4 step per pass over 56-column tiles with a 4-cell
            // halo (mirror ghosts need 4 cells inside each wall)
            if (method == RPR_RK4 && g.nx >= SWF_HALO && g.ny >= SWF_HALO) {
                if constexpr (sizeof(T) == 4) {
                    switch (variant) {
                    case 1: return launch_swe_fused<T, 4, 8>(g, steps, dt, n, in, out, w, ctrl, st);
                    case 2: return launch_swe_fused<T, 4, 10>(g, steps, dt, n, in, out, w, ctrl, st);
                    case 3: return launch_swe_fused<T, 8, 5>(g, steps, dt, n, in, out, w, ctrl, st);
                    case 4: return launch_swe_fused<T, 2, 16>(g, steps, dt, n, in, out, w, ctrl, st);
                    case 5: return launch_swe_rows<T, 3, 2, 12>(g, steps, dt, n, in, out, w, ctrl, st);
                    case 6: return launch_swe_rows<T, 2, 3, 12>(g, steps, dt, n, in, out, w, ctrl, st);
                    default: return launch_swe_fused<T, 5, 8>(g, steps, dt, n, in, out, w, ctrl, st);
                    }
                } else {
                    switch (variant) {
                    case 1: return launch_swe_fused<T, 4, 6>(g, steps, dt, n, in, out, w, ctrl, st);
                    case 2: return launch_swe_fused<T, 3, 8>(g, steps, dt, n, in, out, w, ctrl, st);
                    case 3: return launch_swe_fused<T, 2, 12>(g, steps, dt, n, in, out, w, ctrl, st);
                    case 4: return launch_swe_rows<T, 3, 2, 8>(g, steps, dt, n, in, out, w, ctrl, st);
                    case 5: return launch_swe_rows<T, 2, 3, 8>(g, steps, dt, n, in, out, w, ctrl, st);
                    default: return launch_swe_fused<T, 4, 8>(g, steps, dt, n, in, out, w, ctrl, st);
                    }
                }
            }
        }
        if constexpr (KIND == RPR_DIFFREACT2D || KIND == RPR_BRUSS2D) {
            if (method == RPR_RK4) {
                // a whole step per pass: the Laplacian right-hand side is
                // cheap to recompute on a 4-cell halo
                switch (variant) {
                case 1: return launch_lap_fused<KIND, T, 16, 256>(g, steps, dt, n, in, out, w, ctrl, st);
                case 2: return launch_lap_fused<KIND, T, 32, 256>(g, steps, dt, n, in, out, w, ctrl, st);
                case 3: return launch_lap_fused<KIND, T, 64, 512>(g, steps, dt, n, in, out, w, ctrl, st);
                default: return launch_lap_fused<KIND, T, FUSED_FY, FUSED_NT>(g, steps, dt, n, in, out, w, ctrl, st);
                }
            }
        }
        for (long long s = 0; s < ns; ++s) {
            if (method == RPR_RK4) {
                hipLaunchKernelGGL((k_prop_tiled<KIND, T, 1>), grid, dim3(TT_THREADS), lds, st, g, method, s, ns, dt,
                                   n, in, out, w, ctrl);
                hipLaunchKernelGGL((k_prop_tiled<KIND, T, 2>), grid, dim3(TT_THREADS), lds, st, g, method, s, ns, dt,
                                   n, in, out, w, ctrl);
                hipLaunchKernelGGL((k_prop_tiled<KIND, T, 3>), grid, dim3(TT_THREADS), lds, st, g, method, s, ns, dt,
                                   n, in, out, w, ctrl);
                hipLaunchKernelGGL((k_prop_tiled<KIND, T, 4>), grid, dim3(TT_THREADS), lds, st, g, method, s, ns, dt,
                                   n, in, out, w, ctrl);
            } else {
                hipLaunchKernelGGL((k_prop_tiled<KIND, T, 0>), grid, dim3(TT_THREADS), lds, st, g, method, s, ns, dt,
                                   n, in, out, w, ctrl);
            }
            RPR_HIP(hipGetLastError());
        }
        return RPR_OK;
    }
}

template rpr_status launch_prop_tiled_kind<RPR_KIND, RPR_REAL>(const Geom &, int, int64_t, double, int,
                                                                const RPR_REAL *, RPR_REAL *,
                                                                const TiledWork<RPR_REAL> &, const int *,
                                                                hipStream_t, int);

}  // namespace rpr
