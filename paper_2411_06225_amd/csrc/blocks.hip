// blocks.hip -- the building-block entry points of the C ABI: the same kernels
// a plan runs, one call each.
#include <map>
#include <mutex>

#include "plan.h"

namespace rpr {

// Scratch of the entry points that allocate nothing (16 MiB per device, held
// until the process ends).  Host code never uses the symbol itself: it is a
// host-side stand-in; the device address comes from hipGetSymbolAddress, once
// per device, with that device current.
constexpr size_t kScratchDoubles = (size_t)2 << 20;
static __device__ __align__(256) double scratch[kScratchDoubles];

static std::mutex g_scratch_mu;
static std::map<int, double *> g_scratch_ptr;

static rpr_status scratch_address(double **out)
{
    int dev = 0;
    RPR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    const auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return RPR_OK;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
    *out = static_cast<double *>(ptr);
    return RPR_OK;
}

}  // namespace rpr

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
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (P->threads == GENERIC_THREADS || P->method == RPR_RK8 || g.kind == RPR_BRUSS3D) {
        // generic form: the work arrays of rkgen_work, released on the stream
        RPR_TRY(check_device());
        void *ws = nullptr;
        RPR_HIP(hipMallocAsync(&ws, rkgen_work_elems(P->method, n_states, d) * esz, st));
        rpr_status rc;
        if (precision == RPR_FP64) {
            const TiledWork<double> w = rkgen_work<double>(ws, n_states, d);
            rc = launch_propagate<double>(g, P->method, P->steps, dt, n_states, static_cast<const double *>(in),
                                          static_cast<double *>(out), nullptr, st, GENERIC_THREADS, &w);
        } else {
            const TiledWork<float> w = rkgen_work<float>(ws, n_states, d);
            rc = launch_propagate<float>(g, P->method, P->steps, dt, n_states, static_cast<const float *>(in),
                                         static_cast<float *>(out), nullptr, st, GENERIC_THREADS, &w);
        }
        RPR_HIP(hipFreeAsync(ws, st));
        return rc;
    }
    // automatic: on chip when the state fits one work-group, else tiled
    OnchipShape probe;
    const bool fits = onchip_shape(g, esz, &probe, 1024);
    if (!P->threads && !fits) RPR_TRY(check_threads(g, esz, TILED_THREADS));
    RPR_TRY(check_device());
    const int mt = P->threads ? P->threads : (fits ? tuned_prop_threads(g, esz, P->method) : TILED_THREADS);
    if (mt != TILED_THREADS) {
        if (precision == RPR_FP64)
            return launch_propagate<double>(g, P->method, P->steps, dt, n_states, static_cast<const double *>(in),
                                            static_cast<double *>(out), nullptr, st, mt);
        return launch_propagate<float>(g, P->method, P->steps, dt, n_states, static_cast<const float *>(in),
                                       static_cast<float *>(out), nullptr, st, mt);
    }
    // tiled: five work arrays of n_states x d values, released on the
    // stream; the one-pass form in the tile shape the autotuner chose for
    // this class of propagators in this process (else the default)
    const int var = tuned_variant(g, esz, P->method);
    const size_t nd = (size_t)n_states * d;
    void *ws = nullptr;
    RPR_HIP(hipMallocAsync(&ws, 5 * nd * esz, st));
    rpr_status rc;
    if (precision == RPR_FP64) {
        double *b = static_cast<double *>(ws);
        const TiledWork<double> w{b, b + nd, b + 2 * nd, b + 3 * nd, nullptr};
        rc = launch_propagate<double>(g, P->method, P->steps, dt, n_states, static_cast<const double *>(in),
                                      static_cast<double *>(out), nullptr, st, mt, &w, var);
    } else {
        float *b = static_cast<float *>(ws);
        const TiledWork<float> w{b, b + nd, b + 2 * nd, b + 3 * nd, b + 4 * nd};
        rc = launch_propagate<float>(g, P->method, P->steps, dt, n_states, static_cast<const float *>(in),
                                     static_cast<float *>(out), nullptr, st, mt, &w, var);
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

extern "C" rpr_status rpr_randnet_features_noalloc(int32_t M, int32_t d, int32_t n, int32_t activation, double s,
                                                   const double *A, const double *zeta, const double *X,
                                                   double *Phi, void *stream)
{
    if (M < 1 || d < 1 || n < 0) return fail(RPR_ERR_INVALID_ARG, "need M >= 1, d >= 1, n >= 0");
    if (activation != RPR_TANH && activation != RPR_RELU) return fail(RPR_ERR_INVALID_ARG, "bad activation");
    if (!(s > 0) || !is_finite(s)) return fail(RPR_ERR_INVALID_ARG, "s must be > 0");
    if (n == 0) return RPR_OK;
    if (!A || !zeta || !X || !Phi) return fail(RPR_ERR_INVALID_ARG, "NULL device pointer");
    const size_t need = (size_t)feat_splits(d) * (size_t)n * (size_t)M;
    if (need > kScratchDoubles)
        return fail(RPR_ERR_INVALID_ARG, "rpr_randnet_features_noalloc: the split-K partial sums need " +
                                             std::to_string(need) + " doubles (K splits x n x M), more than the " +
                                             std::to_string(kScratchDoubles) + " of the scratch (16 MiB)");
    RPR_TRY(check_device());
    double *part = nullptr;
    RPR_TRY(scratch_address(&part));
    return launch_features<double>(n, M, d, activation, 1.0 / s, A, zeta, X, Phi, part, nullptr,
                                   static_cast<hipStream_t>(stream));
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

