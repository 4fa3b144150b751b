// common.h -- internal declarations of librpr (not part of the C ABI).
//
// Geometry of a state, the per-cell right-hand sides h(u) of the four PDE
// families, error plumbing and launch helpers shared by the .hip sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "rpr.h"

namespace rpr {

// ---------------------------------------------------------------- errors --
void set_error(const std::string &msg);
rpr_status fail(rpr_status st, const std::string &msg);
rpr_status hip_fail(hipError_t e, const char *what);

#define RPR_HIP(call)                                                      \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess) return ::rpr::hip_fail(e_, #call);           \
    } while (0)

// --------------------------------------------------------------- geometry --
// Kernel-side description of h.  Spacings are folded into reciprocals once on
// the host; the stencils multiply by them.
struct Geom {
    int kind;      // rpr_rhs_kind
    int nx, ny;    // grid
    int nc;        // cells = nx * ny * nz
    int ns;        // species
    int d;         // ns * nc
    int periodic;  // 1: wrap, 0: wall (Neumann mirror / reflective)
    double idx2, idy2;   // 1 / dx^2, 1 / dy^2
    double i2dx;         // 1 / (2 dx)            (Burgers advection)
    double idx, idy;     // 1 / dx, 1 / dy         (finite-volume flux differences)
    double p[6];
    int nz;              // cells along z (3D Brusselator; 1 otherwise)
    double idz2;         // 1 / dz^2 (3D)
};

inline int nspecies(int kind)
{
    switch (kind) {
    case RPR_BURGERS1D: return 1;
    case RPR_DIFFREACT2D: return 2;
    case RPR_BRUSS2D: return 2;
    case RPR_SWE2D: return 3;
    case RPR_BRUSS3D: return 2;
    default: return 0;
    }
}

rpr_status make_geom(const rpr_rhs *h, int32_t d, Geom *g);

// ------------------------------------------------------- right-hand sides --
// Each function evaluates h at one cell from the cell's own species values
// `c` and the values of its four neighbours after the boundary rule has been
// applied (w/e: x - 1, x + 1; s/n: y - 1, y + 1).  Results go to k[species].

// Viscous Burgers, eq. "burg": nu u_xx - u u_x with central differences.
template <typename T>
__device__ __forceinline__ void rhs_burgers(const T *c, const T *w, const T *e, T *k, T nu, T idx2,
                                            T i2dx)
{
    const T uxx = (e[0] - T(2) * c[0] + w[0]) * idx2;
    const T ux = (e[0] - w[0]) * i2dx;
    k[0] = nu * uxx - c[0] * ux;
}

// D times the 5-point Laplacian plus r, from the sum xs of the two x
// neighbours and the centre weight mx in x (-2 when both neighbours are in
// xs), with the diffusion coefficient folded into the axis weights
// (Dx = D / dx^2, Dy = D / dy^2).
template <typename T>
__device__ __forceinline__ T diffuse5(T c, T xs, T mx, T s, T n, T Dx, T Dy, T r)
{
    return Dx * (xs + mx * c) + (Dy * (s - T(2) * c + n) + r);
}

// FitzHugh-Nagumo diffusion-reaction (Sec. 5.2).  D*: diffusion
// coefficients over dx^2 and dy^2; xs, mx as in diffuse5.
template <typename T>
__device__ __forceinline__ void rhs_diffreact(const T *c, const T *xs, T mx, const T *s, const T *n, T *k, T Dux,
                                              T Duy, T Dvx, T Dvy, T cc)
{
    const T u = c[0], v = c[1];
    k[0] = diffuse5(u, xs[0], mx, s[0], n[0], Dux, Duy, (u - u * u * u) - (cc + v));
    k[1] = diffuse5(v, xs[1], mx, s[1], n[1], Dvx, Dvy, u - v);
}

// Brusselator (App. E).
template <typename T>
__device__ __forceinline__ void rhs_bruss(const T *c, const T *xs, T mx, const T *s, const T *n, T *k, T A, T B,
                                          T Dux, T Duy, T Dvx, T Dvy)
{
    const T u = c[0], v = c[1];
    const T u2v = u * u * v;
    k[0] = diffuse5(u, xs[0], mx, s[0], n[0], Dux, Duy, (A - (B + T(1)) * u) + u2v);
    k[1] = diffuse5(v, xs[1], mx, s[1], n[1], Dvx, Dvy, B * u - u2v);
}

// Shallow water: Rusanov flux across one face; (h, m, n) = depth, momentum
// normal to the face, momentum along it.
template <typename T>
struct SweQ {
    T h, m, n;
};

template <typename T>
__device__ __forceinline__ SweQ<T> rusanov(const SweQ<T> &L, const SweQ<T> &R, T g)
{
    const T uL = L.m / L.h, uR = R.m / R.h;
    const T cL = fabs(uL) + sqrt(g * L.h);
    const T cR = fabs(uR) + sqrt(g * R.h);
    const T a = cL > cR ? cL : cR;
    SweQ<T> F;
    F.h = T(0.5) * (L.m + R.m) - T(0.5) * a * (R.h - L.h);
    F.m = T(0.5) * ((L.m * uL + T(0.5) * g * L.h * L.h) + (R.m * uR + T(0.5) * g * R.h * R.h)) -
          T(0.5) * a * (R.m - L.m);
    F.n = T(0.5) * (L.n * uL + R.n * uR) - T(0.5) * a * (R.n - L.n);
    return F;
}

// Shallow water at one cell.  Species order (h, hu, hv).  A wall neighbour
// arrives as the cell itself with the wall flag set; its ghost is the mirror
// image with the normal momentum negated.
template <typename T>
__device__ __forceinline__ void rhs_swe(const T *c, const T *w, const T *e, const T *s, const T *n,
                                        bool ww, bool we, bool ws, bool wn, T *k, T g, T idx, T idy)
{
    const SweQ<T> qx{c[0], c[1], c[2]};
    const SweQ<T> qy{c[0], c[2], c[1]};
    const SweQ<T> W{w[0], ww ? -w[1] : w[1], w[2]};
    const SweQ<T> E{e[0], we ? -e[1] : e[1], e[2]};
    const SweQ<T> S{s[0], ws ? -s[2] : s[2], s[1]};
    const SweQ<T> N{n[0], wn ? -n[2] : n[2], n[1]};
    const SweQ<T> Fw = rusanov(W, qx, g), Fe = rusanov(qx, E, g);
    const SweQ<T> Gs = rusanov(S, qy, g), Gn = rusanov(qy, N, g);
    k[0] = -(Fe.h - Fw.h) * idx - (Gn.h - Gs.h) * idy;
    k[1] = -(Fe.m - Fw.m) * idx - (Gn.n - Gs.n) * idy;
    k[2] = -(Fe.n - Fw.n) * idx - (Gn.m - Gs.m) * idy;
}

template <int KIND>
constexpr int kind_ns()
{
    return KIND == RPR_BURGERS1D ? 1 : (KIND == RPR_SWE2D ? 3 : 2);
}

// Brusselator in three dimensions (App. E): the reaction of rhs_bruss with
// the seven-point Laplacian; xs, ys, zs: sums of the two neighbours along
// each axis, D*x = D / dx^2 etc.
template <typename T>
__device__ __forceinline__ void rhs_bruss3d(const T *c, const T *xs, const T *ys, const T *zs, T *k, T A, T B, T Dux,
                                            T Duy, T Duz, T Dvx, T Dvy, T Dvz)
{
    const T u = c[0], v = c[1];
    const T u2v = u * u * v;
    const T lu = Dux * (xs[0] - T(2) * u) + Duy * (ys[0] - T(2) * u) + Duz * (zs[0] - T(2) * u);
    const T lv = Dvx * (xs[1] - T(2) * v) + Dvy * (ys[1] - T(2) * v) + Dvz * (zs[1] - T(2) * v);
    k[0] = lu + ((A - (B + T(1)) * u) + u2v);
    k[1] = lv + (B * u - u2v);
}

// Right-hand side of the Laplacian-coupled systems (diffusion-reaction,
// Brusselator) at one cell from the sum xs of its x neighbours, the centre
// weight mx in x and its y neighbours.
template <int KIND, typename T>
__device__ __forceinline__ void rhs_cell_xsum(const Geom &g, const T *c, const T *xs, T mx, const T *s, const T *n,
                                              T *k)
{
    static_assert(KIND == RPR_DIFFREACT2D || KIND == RPR_BRUSS2D, "5-point Laplacian systems only");
    if constexpr (KIND == RPR_DIFFREACT2D)
        rhs_diffreact<T>(c, xs, mx, s, n, k, T(g.p[0] * g.idx2), T(g.p[0] * g.idy2), T(g.p[1] * g.idx2),
                         T(g.p[1] * g.idy2), T(g.p[2]));
    else
        rhs_bruss<T>(c, xs, mx, s, n, k, T(g.p[0]), T(g.p[1]), T(g.p[2] * g.idx2), T(g.p[2] * g.idy2),
                     T(g.p[3] * g.idx2), T(g.p[3] * g.idy2));
}

// Dispatch for a compile-time kind.
template <int KIND, typename T>
__device__ __forceinline__ void rhs_cell(const Geom &g, const T *c, const T *w, const T *e, const T *s,
                                         const T *n, bool ww, bool we, bool ws, bool wn, T *k)
{
    if constexpr (KIND == RPR_BURGERS1D) {
        rhs_burgers<T>(c, w, e, k, T(g.p[0]), T(g.idx2), T(g.i2dx));
    } else if constexpr (KIND == RPR_DIFFREACT2D || KIND == RPR_BRUSS2D) {
        T xs[2] = {w[0] + e[0], w[1] + e[1]};
        rhs_cell_xsum<KIND, T>(g, c, xs, T(-2), s, n, k);
    } else {
        rhs_swe<T>(c, w, e, s, n, ww, we, ws, wn, k, T(g.p[0]), T(g.idx), T(g.idy));
    }
}

// --------------------------------------------------------------- bfloat16 --
// Round a float to bfloat16 with round-to-nearest-even (NaN kept quiet).
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)(u >> 16);  // NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------- on-chip propagation --
constexpr size_t kMaxLds = 160 * 1024 - 1024;  // dynamic LDS per work-group on gfx950 (160 KB),
                                               // less 1 KB kept for static LDS buffers

// A slot whose whole state fits in one work-group's LDS is propagated by that
// work-group; thread t owns a strip of `cpt` consecutive cells (slotprop.h).
struct OnchipShape {
    int block;     // threads per work-group
    int maxt;      // launch bound the kernel instance was built for (512 or 1024)
    int cpt;       // cells per thread (template instance)
    int dbuf;      // 1: two LDS stage buffers (one barrier per stage)
    int full;      // 1: every thread owns a complete strip
    size_t lds;    // bytes of dynamic LDS
};

// Fills *sh for a state of geometry g in elements of `elem` bytes; false if
// the state does not fit one work-group.
// max_threads (512 or 1024) bounds the work-group: with 512 threads each
// strip is twice as long and a thread may hold 256 VGPRs instead of 128.
bool onchip_shape(const Geom &g, size_t elem, OnchipShape *sh, int max_threads = 1024);
// Launch shape of the tiled propagator (block TT_THREADS, maxt TILED_THREADS,
// LDS of one haloed tile).
OnchipShape tiled_shape(const Geom &g, size_t elem);

// RPR_OK when a kernel instance with work-groups of `threads` (512 or 1024
// on chip, TILED_THREADS tiled) serves grid g at element size elem, else
// RPR_ERR_UNSUPPORTED.
rpr_status check_threads(const Geom &g, size_t elem, int threads);

// Per right-hand side instance (propagate.hip, one object per kind and precision).
template <int KIND, typename T>
rpr_status launch_propagate_kind(const Geom &g, const OnchipShape &sh, int method, int64_t steps, double dt,
                                 int n, const T *in, T *out, const int *ctrl, hipStream_t st);

// Work arrays of the tiled propagator for n slot states (n x d values each,
// slot b at b d): the work state u, the RK4 accumulator, two stage inputs and
// the FP32 compensation (acc and yb unused by forward Euler, cmp by FP64).
template <typename T>
struct TiledWork {
    T *u, *acc, *ya, *yb, *cmp;
};

// Work-group size that selects the tiled propagator (states in memory).
constexpr int TILED_THREADS = 256;

// Tiled propagation of n states (2D grids): one launch per RK stage, or per
// RK4 step for the systems with a one-pass form.  variant picks the tile
// shape of the one-pass form (0 = the built-in default; see
// fused_variants), ignored otherwise.
template <int KIND, typename T>
rpr_status launch_prop_tiled_kind(const Geom &g, int method, int64_t steps, double dt, int n, const T *in, T *out,
                                  const TiledWork<T> &w, const int *ctrl, hipStream_t st, int variant);

// Number of tile shapes of the one-pass RK4 form of right-hand side `kind` at
// element size elem (1 where the kind has none: the variant is then ignored),
// and a short name of shape v for the autotuner's records.
int fused_variants(int kind, size_t elem);
const char *fused_variant_name(int kind, size_t elem, int v);
// Whether tile shape v of the one-pass RK4 kernel serves this grid.
bool fused_variant_fits(const Geom &g, size_t elem, int v);

// The generic propagator (rkgen.hip): any explicit tableau (method 1, 4 or
// 8), one launch per stage over the cells of all n states; work arrays as
// rkgen_work lays them out (rkgen.h).
template <int KIND, typename T>
rpr_status launch_rkgen_kind(const Geom &g, int method, int64_t steps, double dt, int n, const T *in, T *out,
                             const TiledWork<T> &w, const int *ctrl, hipStream_t st);

// Launch shape of the generic propagator (block 256, maxt GENERIC_THREADS).
OnchipShape generic_shape(const Geom &g, size_t elem);

// Launch of the propagator: out[b] = P(in[b]) for b in [0, n), where the
// work of state b is skipped when ctrl != nullptr and b < ctrl[0] (slot b + 1
// is already final) or ctrl[2] != 0 (run finished).  max_threads 512 / 1024
// selects the on-chip kernel with that work-group size, TILED_THREADS the
// tiled one, which needs the work arrays tw, GENERIC_THREADS (rkgen.h) the
// generic one (work arrays tw laid out by rkgen_work).
template <typename T>
rpr_status launch_propagate(const Geom &g, int method, int64_t steps, double dt, int n, const T *in,
                            T *out, const int *ctrl, hipStream_t st, int max_threads = 1024,
                            const TiledWork<T> *tw = nullptr, int variant = 0);

// One instance of a batch, as the persistent fine-solve kernel sees it.
template <typename T>
struct BatchInst {
    Geom g;
    int method;
    long long steps;
    double dt;
    const T *U;        // (N+1) x d slot states of the instance
    T *Fv;             // (N+1) x d fine values (row i = F(U[i-1]))
    const int *ctrl;   // the instance's control block (L at [0], done at [2])
};

// Persistent fine solves over a batch: items[q] = (instance, slot), processed
// in list order (longest first) by work-groups that take the next index from
// *counter (zeroed before the launch) until the list is exhausted.  sh: the
// generic strip shape of the largest instance; grid: work-groups launched.
template <int KIND, typename T>
rpr_status launch_prop_persistent_kind(const BatchInst<T> *insts, const int2 *items, int n_items, int *counter,
                                       const Geom &gmax, const OnchipShape &sh, int grid, hipStream_t st);
template <typename T>
rpr_status launch_prop_persistent(const BatchInst<T> *insts, const int2 *items, int n_items, int *counter,
                                  const Geom &gmax, const OnchipShape &sh, int grid, hipStream_t st);

// Control block of a plan, in device memory.
struct Ctrl {
    int L;           // slots 0..L are final
    int k;           // iterations done
    int done;        // stop flag: 1 once L == N or k == k_max
    int rows_used;   // finite pairs in the readout
    int nonfinite;   // dropped pairs
    int chol_fail;   // failed ridge factorisations
    int nn_rows;     // pairs in the nearest-neighbour store (finite or not)
    int pad;
};

}  // namespace rpr
