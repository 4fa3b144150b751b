// randnet.hip -- the random network of eq. "HA" and its ridge readout
// (eq. "ridgeless"), in double precision.
//
//   features : Phi = sigma(X A^T / s + zeta)      split-K tiled GEMM + epilogue
//   gram     : G += Phi^T Phi, B += Phi^T Y        over the finite rows only
//   cholesky : G + lambda I = L L^T                one work-group, pivot-checked
//   solve    : W = L^-T L^-1 B                     column blocks of B in LDS
//   readout  : Yhat = Phi W
// Every reduction runs in a fixed order (no floating-point atomics), so
// results are bitwise reproducible run to run.
#include "common.h"
#include "randnet.h"

namespace rpr {

// ------------------------------------------------------------- features ---
// Z = X A^T with X (n x d) and A (M x d) both K-contiguous.  Work-group tile:
// 16 rows of X x 16 rows of A, K staged through LDS in chunks of 64; the K
// range is split over gridDim.z into partial sums reduced in order later.
// X rows may be FP64 or FP32 (the state precision); the product is FP64.
constexpr int FT = 16, FK = 64;

template <typename TX>
__global__ __launch_bounds__(256) void k_feat_partial(int n, int M, int d, int kchunk,
                                                      const TX *__restrict__ X, const double *__restrict__ A,
                                                      double xs, double *__restrict__ part,
                                                      const int *__restrict__ nrows_dev)
{
    const int nr = nrows_dev ? *nrows_dev : n;
    const int r0 = blockIdx.x * FT, m0 = blockIdx.y * FT;
    if (r0 >= nr) return;
    const int k0 = blockIdx.z * kchunk, k1 = min(d, k0 + kchunk);
    __shared__ double sx[FT][FK + 1], sa[FT][FK + 1];
    const int tx = threadIdx.x % FT, ty = threadIdx.x / FT;  // output (ty, tx) = (row, neuron)
    double acc = 0.0;
    for (int kb = k0; kb < k1; kb += FK) {
        for (int i = threadIdx.x; i < FT * FK; i += 256) {
            const int rr = i / FK, kk = i % FK, k = kb + kk;
            sx[rr][kk] = (r0 + rr < nr && k < k1) ? double(X[(size_t)(r0 + rr) * d + k]) * xs : 0.0;
            sa[rr][kk] = (m0 + rr < M && k < k1) ? A[(size_t)(m0 + rr) * d + k] : 0.0;
        }
        __syncthreads();
#pragma unroll 16
        for (int kk = 0; kk < FK; ++kk) acc = fma(sx[ty][kk], sa[tx][kk], acc);
        __syncthreads();
    }
    if (r0 + ty < nr && m0 + tx < M) part[((size_t)blockIdx.z * n + r0 + ty) * M + m0 + tx] = acc;
}

__global__ void k_feat_finish(int n, int M, int nsplit, const double *__restrict__ part,
                              const double *__restrict__ zeta, int act, double *__restrict__ Phi,
                              const int *__restrict__ nrows_dev)
{
    const int nr = nrows_dev ? *nrows_dev : n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr * M) return;
    double z = 0.0;
    for (int s = 0; s < nsplit; ++s) z += part[(size_t)s * n * M + i];
    z += zeta[i % M];
    Phi[i] = act == RPR_RELU ? (z > 0.0 ? z : 0.0) : tanh(z);
}

int feat_splits(int d)
{
    int s = (d + 511) / 512;  // about 512 of K per work-group
    return s < 1 ? 1 : (s > 64 ? 64 : s);
}

template <typename TX>
rpr_status launch_features(int n, int M, int d, int act, double inv_s, const double *A, const double *zeta,
                           const TX *X, double *Phi, double *part, const int *nrows_dev, hipStream_t st)
{
    if (n <= 0) return RPR_OK;
    const int ns = feat_splits(d);
    const int kchunk = ((d + ns - 1) / ns + FK - 1) / FK * FK;
    dim3 grid((n + FT - 1) / FT, (M + FT - 1) / FT, ns);
    hipLaunchKernelGGL(k_feat_partial<TX>, grid, dim3(256), 0, st, n, M, d, kchunk, X, A, inv_s, part,
                       nrows_dev);
    RPR_HIP(hipGetLastError());
    const int tot = n * M;
    hipLaunchKernelGGL(k_feat_finish, dim3((tot + 255) / 256), dim3(256), 0, st, n, M, ns, part, zeta, act,
                       Phi, nrows_dev);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}
template rpr_status launch_features<double>(int, int, int, int, double, const double *, const double *,
                                            const double *, double *, double *, const int *, hipStream_t);
template rpr_status launch_features<float>(int, int, int, int, double, const double *, const double *,
                                           const float *, double *, double *, const int *, hipStream_t);

// ------------------------------------------------- reduced-precision features ---
// Mixed-precision hidden layer: inputs x/s and weights rounded to bfloat16
// (round to nearest even), products accumulated in FP32 on the matrix cores
// (v_mfma_f32_16x16x32_bf16), zeta and sigma in FP32, result rounded to bf16
// and stored as a double (exactly representable) for the FP64 statistics.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__global__ void k_to_bf16(const double *__restrict__ in, uint16_t *__restrict__ out, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = to_bf16((float)in[i]);
}

rpr_status launch_to_bf16(const double *in, uint16_t *out, size_t n, hipStream_t st)
{
    if (n == 0) return RPR_OK;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}

// Work-group tile: 64 rows of X x 64 neurons, 4 waves; wave w owns rows
// 16w..16w+15 and all four 16-neuron tiles.  K advances 32 at a time through
// LDS.  Operand layout of the 16x16x32 instruction: lane l holds A[l%16][8(l/16)..+7],
// B[8(l/16)..+7][l%16], and D[4(l/16)+e][l%16], e = 0..3.
constexpr int BT = 64, BK = 32, BKP = 40;  // LDS row pitch 80 B keeps 16-byte alignment

template <typename TX>
__global__ __launch_bounds__(256) void k_feat_bf16_partial(int n, int M, int d, int kchunk,
                                                           const TX *__restrict__ X,
                                                           const uint16_t *__restrict__ Ab, float xs,
                                                           float *__restrict__ part,
                                                           const int *__restrict__ nrows_dev)
{
    const int nr = nrows_dev ? *nrows_dev : n;
    const int r0 = blockIdx.x * BT, m0 = blockIdx.y * BT;
    if (r0 >= nr) return;
    const int k0 = blockIdx.z * kchunk, k1 = min(d, k0 + kchunk);
    __shared__ __align__(16) uint16_t Xs[BT][BKP], As[BT][BKP];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int lr = t >> 2, lk = (t & 3) * 8;  // loader: row, first k of 8
    f32x4_t acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    for (int kb = k0; kb < k1; kb += BK) {
        {
            const int r = r0 + lr, m = m0 + lr;
            uint16_t xv[8], av[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = kb + lk + e;
                const bool kin = k < k1;
                xv[e] = (r < nr && kin) ? to_bf16(float(X[(size_t)r * d + k]) * xs) : (uint16_t)0;
                av[e] = (m < M && kin) ? Ab[(size_t)m * d + k] : (uint16_t)0;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                Xs[lr][lk + e] = xv[e];
                As[lr][lk + e] = av[e];
            }
        }
        __syncthreads();
        const uint4 a4 = *reinterpret_cast<const uint4 *>(&Xs[w * 16 + (lane & 15)][8 * (lane >> 4)]);
        const bf16x8_t a = __builtin_bit_cast(bf16x8_t, a4);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint4 b4 = *reinterpret_cast<const uint4 *>(&As[j * 16 + (lane & 15)][8 * (lane >> 4)]);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8_t, b4), acc[j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = r0 + w * 16 + 4 * (lane >> 4) + e, m = m0 + j * 16 + (lane & 15);
            if (r < nr && m < M) part[((size_t)blockIdx.z * n + r) * M + m] = acc[j][e];
        }
}

__global__ void k_feat_bf16_finish(int n, int M, int nsplit, const float *__restrict__ part,
                                   const double *__restrict__ zeta, int act, double *__restrict__ Phi,
                                   const int *__restrict__ nrows_dev)
{
    const int nr = nrows_dev ? *nrows_dev : n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr * M) return;
    float z = 0.0f;
    for (int s = 0; s < nsplit; ++s) z += part[(size_t)s * n * M + i];
    z += (float)zeta[i % M];
    const float sg = act == RPR_RELU ? (z > 0.0f ? z : 0.0f) : tanhf(z);
    Phi[i] = (double)from_bf16(to_bf16(sg));
}

int feat_bf16_splits(int d)
{
    int s = (d + 2047) / 2048;  // about 2048 of K per work-group
    return s < 1 ? 1 : (s > 64 ? 64 : s);
}

template <typename TX>
rpr_status launch_features_bf16(int n, int M, int d, int act, double inv_s, const uint16_t *Ab,
                                const double *zeta, const TX *X, double *Phi, float *part,
                                const int *nrows_dev, hipStream_t st)
{
    if (n <= 0) return RPR_OK;
    const int ns = feat_bf16_splits(d);
    const int kchunk = ((d + ns - 1) / ns + BK - 1) / BK * BK;
    dim3 grid((n + BT - 1) / BT, (M + BT - 1) / BT, ns);
    hipLaunchKernelGGL(k_feat_bf16_partial<TX>, grid, dim3(256), 0, st, n, M, d, kchunk, X, Ab, (float)inv_s,
                       part, nrows_dev);
    RPR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_feat_bf16_finish, dim3((n * M + 255) / 256), dim3(256), 0, st, n, M, ns, part, zeta,
                       act, Phi, nrows_dev);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}
template rpr_status launch_features_bf16<float>(int, int, int, int, double, const uint16_t *, const double *,
                                                const float *, double *, float *, const int *, hipStream_t);
template rpr_status launch_features_bf16<double>(int, int, int, int, double, const uint16_t *, const double *,
                                                 const double *, double *, float *, const int *, hipStream_t);

// ----------------------------------------------------------- statistics ---
// G[a][b] += sum_r ok_r Phi[r][a] Phi[r][b]; rows in order r = 0..n-1.
__global__ __launch_bounds__(256) void k_gram(int n, int M, const double *__restrict__ Phi,
                                              const int *__restrict__ ok, double *__restrict__ G,
                                              const int *__restrict__ nrows_dev)
{
    const int nr = nrows_dev ? *nrows_dev : n;
    const int a = blockIdx.y * 16 + threadIdx.x / 16, b = blockIdx.x * 16 + threadIdx.x % 16;
    if (a >= M || b >= M) return;
    double acc = 0.0;
    for (int r = 0; r < nr; ++r)
        if (ok == nullptr || ok[r]) acc = fma(Phi[(size_t)r * M + a], Phi[(size_t)r * M + b], acc);
    G[(size_t)a * M + b] += acc;
}

// B[a][j] += sum_r ok_r Phi[r][a] Y[r][j]: a block of 16 neurons x 256 columns;
// the 16 Phi columns of the block are staged in LDS.
template <typename TY>
__global__ __launch_bounds__(256) void k_bstat(int n, int M, int d, const double *__restrict__ Phi,
                                               const TY *__restrict__ Y, const int *__restrict__ ok,
                                               double *__restrict__ Bm, const int *__restrict__ nrows_dev)
{
    const int nr = nrows_dev ? *nrows_dev : n;
    const int a0 = blockIdx.y * 16, j = blockIdx.x * 256 + threadIdx.x;
    extern __shared__ double sphi[];  // n x 16
    for (int i = threadIdx.x; i < nr * 16; i += 256) {
        const int r = i / 16, aa = i % 16;
        const bool use = (ok == nullptr || ok[r]) && a0 + aa < M;
        sphi[i] = use ? Phi[(size_t)r * M + a0 + aa] : 0.0;
    }
    __syncthreads();
    if (j >= d) return;
    double acc[16];
#pragma unroll
    for (int aa = 0; aa < 16; ++aa) acc[aa] = 0.0;
    for (int r = 0; r < nr; ++r) {
        const double yv = (ok == nullptr || ok[r]) ? double(Y[(size_t)r * d + j]) : 0.0;
#pragma unroll
        for (int aa = 0; aa < 16; ++aa) acc[aa] = fma(sphi[r * 16 + aa], yv, acc[aa]);
    }
#pragma unroll
    for (int aa = 0; aa < 16; ++aa)
        if (a0 + aa < M) Bm[(size_t)(a0 + aa) * d + j] += acc[aa];
}

template <typename TY>
rpr_status launch_stats(int n, int M, int d, const double *Phi, const TY *Y, const int *ok, double *G,
                        double *Bm, const int *nrows_dev, hipStream_t st)
{
    if (n <= 0) return RPR_OK;
    hipLaunchKernelGGL(k_gram, dim3((M + 15) / 16, (M + 15) / 16), dim3(256), 0, st, n, M, Phi, ok, G,
                       nrows_dev);
    RPR_HIP(hipGetLastError());
    const size_t lds = (size_t)n * 16 * sizeof(double);
    hipLaunchKernelGGL(k_bstat<TY>, dim3((d + 255) / 256, (M + 15) / 16), dim3(256), lds, st, n, M, d, Phi,
                       Y, ok, Bm, nrows_dev);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}
template rpr_status launch_stats<double>(int, int, int, const double *, const double *, const int *,
                                         double *, double *, const int *, hipStream_t);
template rpr_status launch_stats<float>(int, int, int, const double *, const float *, const int *,
                                        double *, double *, const int *, hipStream_t);

// ------------------------------------------------------------- cholesky ---
// Left-looking (Cholesky-Crout) factorisation of S = G + lambda I, one column
// per step: the finished row j of L is broadcast through LDS, its diagonal is
// a block reduction, and thread i computes L[i][j] from its own row.
// Writes L (lower, row-major) and Lt = L^T; a non-positive or NaN pivot sets
// *fail = 1 and counts in *fail_count (both may be null).
__global__ __launch_bounds__(1024) void k_cholesky(int M, const double *__restrict__ G, double lambda,
                                                   double *__restrict__ L, double *__restrict__ Lt,
                                                   int *__restrict__ fail, int *__restrict__ fail_count,
                                                   const int *__restrict__ done)
{
    if (done && *done) return;
    if (threadIdx.x == 0 && fail) *fail = 0;
    extern __shared__ double srow[];  // M + 32
    double *red = srow + M;
    __shared__ int bad;
    const int t = threadIdx.x, B = blockDim.x;
    if (t == 0) bad = 0;
    for (int i = t; i < M * M; i += B) {
        L[i] = 0.0;
        Lt[i] = 0.0;
    }
    __syncthreads();
    for (int j = 0; j < M; ++j) {
        // row j of L (entries < j) into LDS
        for (int p = t; p < j; p += B) srow[p] = L[(size_t)j * M + p];
        __syncthreads();
        // diagonal: G[j][j] + lambda - sum_p L[j][p]^2, reduced in a fixed order
        double part = 0.0;
        for (int p = t; p < j; p += B) part = fma(srow[p], srow[p], part);
        for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
        if ((t & 63) == 0) red[t >> 6] = part;
        __syncthreads();
        if (t == 0) {
            double ssum = 0.0;
            for (int w = 0; w < (B + 63) / 64; ++w) ssum += red[w];
            const double piv = G[(size_t)j * M + j] + lambda - ssum;
            if (!(piv > 0.0)) bad = 1;
            const double ljj = sqrt(piv > 0.0 ? piv : 1.0);
            red[32] = ljj;
            L[(size_t)j * M + j] = ljj;
            Lt[(size_t)j * M + j] = ljj;
        }
        __syncthreads();
        const double ljj = red[32];
        for (int i = j + 1 + t; i < M; i += B) {
            double s = G[(size_t)i * M + j];
            const double *Li = L + (size_t)i * M;
            for (int p = 0; p < j; ++p) s = fma(-Li[p], srow[p], s);
            const double lij = s / ljj;
            L[(size_t)i * M + j] = lij;
            Lt[(size_t)j * M + i] = lij;
        }
        __syncthreads();
    }
    if (t == 0 && bad) {
        if (fail) *fail = 1;
        if (fail_count) *fail_count += 1;
    }
}

// ---------------------------------------------------------------- solve ---
// W = (L L^T)^{-1} B for a block of SC columns of B: forward substitution with
// L, then backward with L^T, the block kept in LDS (M x SC doubles).  Each
// column is served by 8 threads that split the inner product and combine it
// with shuffles.  If the factorisation failed (*fail), W is set to zero.
constexpr int SC = 32;

__global__ __launch_bounds__(256) void k_trsm(int M, int d, const double *__restrict__ L,
                                              const double *__restrict__ Lt, const double *__restrict__ Bm,
                                              double *__restrict__ W, const int *__restrict__ fail,
                                              const int *__restrict__ done)
{
    if (done && *done) return;
    extern __shared__ double sb[];  // M x SC
    const int j0 = blockIdx.x * SC;
    const int col = threadIdx.x / 8, q = threadIdx.x % 8;
    const int j = j0 + col;
    const bool failed = fail && *fail;
    for (int i = threadIdx.x; i < M * SC; i += 256) {
        const int r = i / SC, c = i % SC;
        sb[i] = (j0 + c < d && !failed) ? Bm[(size_t)r * d + j0 + c] : 0.0;
    }
    __syncthreads();
    if (!failed) {
        // forward: z_r = (b_r - sum_{p<r} L[r][p] z_p) / L[r][r]
        for (int r = 0; r < M; ++r) {
            double s = 0.0;
            const double *Lr = L + (size_t)r * M;
            for (int p = q; p < r; p += 8) s = fma(Lr[p], sb[p * SC + col], s);
            s += __shfl_xor(s, 1, 8);
            s += __shfl_xor(s, 2, 8);
            s += __shfl_xor(s, 4, 8);
            if (q == 0) sb[r * SC + col] = (sb[r * SC + col] - s) / Lr[r];
            __syncthreads();
        }
        // backward: w_r = (z_r - sum_{p>r} L[p][r] w_p) / L[r][r]
        for (int r = M - 1; r >= 0; --r) {
            double s = 0.0;
            const double *Ltr = Lt + (size_t)r * M;
            for (int p = r + 1 + q; p < M; p += 8) s = fma(Ltr[p], sb[p * SC + col], s);
            s += __shfl_xor(s, 1, 8);
            s += __shfl_xor(s, 2, 8);
            s += __shfl_xor(s, 4, 8);
            if (q == 0) sb[r * SC + col] = (sb[r * SC + col] - s) / Ltr[r];
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < M * SC; i += 256) {
        const int r = i / SC, c = i % SC;
        if (j0 + c < d) W[(size_t)r * d + j0 + c] = sb[i];
    }
}

rpr_status launch_ridge_solve(int M, int d, const double *G, double lambda, double *L, double *Lt,
                              double *W, const double *Bm, int *fail, int *fail_count, const int *done,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), (M + 40) * sizeof(double), st, M, G, lambda, L, Lt,
                       fail, fail_count, done);
    RPR_HIP(hipGetLastError());
    const size_t lds = (size_t)M * SC * sizeof(double);
    if (lds > kMaxLds) return rpr::fail(RPR_ERR_UNSUPPORTED, "ridge solve: M too large for LDS block");
    static bool attr_set = false;
    if (!attr_set) {
        RPR_HIP(hipFuncSetAttribute((const void *)k_trsm, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
        attr_set = true;
    }
    hipLaunchKernelGGL(k_trsm, dim3((d + SC - 1) / SC), dim3(256), lds, st, M, d, L, Lt, Bm, W, fail, done);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}

// -------------------------------------------------------------- readout ---
// Yhat[r][j] = sum_m W[m][j] Phi[r][m]
__global__ void k_readout(int n, int M, int d, const double *__restrict__ W, const double *__restrict__ Phi,
                          double *__restrict__ Y)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (j >= d || r >= n) return;
    double acc = 0.0;
    for (int m = 0; m < M; ++m) acc = fma(W[(size_t)m * d + j], Phi[(size_t)r * M + m], acc);
    Y[(size_t)r * d + j] = acc;
}

rpr_status launch_readout(int n, int M, int d, const double *W, const double *Phi, double *Y, hipStream_t st)
{
    if (n <= 0) return RPR_OK;
    hipLaunchKernelGGL(k_readout, dim3((d + 255) / 256, n), dim3(256), 0, st, n, M, d, W, Phi, Y);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}

// ------------------------------------------------------------ generator ---
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as a counter hash.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long seed, unsigned long long i)
{
    unsigned long long z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_uniform(unsigned long long seed, unsigned long long first, long long n, double *out)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const unsigned long long r = splitmix64(seed, first + (unsigned long long)k);
    out[k] = 2.0 * (double(r >> 11) * 0x1.0p-53) - 1.0;
}

rpr_status launch_uniform(uint64_t seed, uint64_t first, int64_t n, double *out, hipStream_t st)
{
    if (n <= 0) return RPR_OK;
    const long long blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_uniform, dim3((unsigned)blocks), dim3(256), 0, st, (unsigned long long)seed,
                       (unsigned long long)first, (long long)n, out);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}

// ------------------------------------------------------------- pairs ------
// Training pairs of iteration k (eq. "Dk"), for the slots i = L+1..N:
//   X[r] = U[L + r], Y[r] = Fv[L+1+r] - Gc[L+1+r], ok[r] = all entries finite,
// and *nrows = N - L (0 once the run is done).  One work-group per row.
template <typename T>
__global__ __launch_bounds__(256) void k_pairs(int N, int d, const T *__restrict__ U, const T *__restrict__ Fv,
                                               const T *__restrict__ Gc, T *__restrict__ X, T *__restrict__ Y,
                                               int *__restrict__ ok, int *__restrict__ nrows, Ctrl *ctrl)
{
    const int r = blockIdx.x;
    const int L = ctrl->L, done = ctrl->done;
    if (r == 0 && threadIdx.x == 0) *nrows = done ? 0 : N - L;
    if (done || r >= N - L) return;
    const int i = L + 1 + r;
    int bad = 0;
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        const T xv = U[(size_t)(i - 1) * d + j];
        const T yv = Fv[(size_t)i * d + j] - Gc[(size_t)i * d + j];
        X[(size_t)r * d + j] = xv;
        Y[(size_t)r * d + j] = yv;
        bad |= !(isfinite(double(xv)) && isfinite(double(yv)));
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) {
        ok[r] = !bad;
        atomicAdd(bad ? &ctrl->nonfinite : &ctrl->rows_used, 1);
    }
}

template <typename T>
rpr_status launch_pairs(int N, int d, const T *U, const T *Fv, const T *Gc, T *X, T *Y, int *ok, int *nrows,
                        Ctrl *ctrl, hipStream_t st)
{
    hipLaunchKernelGGL(k_pairs<T>, dim3(N), dim3(256), 0, st, N, d, U, Fv, Gc, X, Y, ok, nrows, ctrl);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}
template rpr_status launch_pairs<double>(int, int, const double *, const double *, const double *, double *,
                                         double *, int *, int *, Ctrl *, hipStream_t);
template rpr_status launch_pairs<float>(int, int, const float *, const float *, const float *, float *,
                                        float *, int *, int *, Ctrl *, hipStream_t);

}  // namespace rpr
