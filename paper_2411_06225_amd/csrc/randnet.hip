// randnet.hip -- the random network of eq. "HA" and its ridge readout
// (eq. "ridgeless"), in double precision.
//
//   features : Phi = sigma(X A^T / s + zeta)      split-K tiled GEMM + epilogue
//   gram     : G += Phi^T Phi, B += Phi^T Y        over the finite rows only (matrix cores)
//   cholesky : G + lambda I = L L^T                one work-group, pivot-checked
//   solve    : W = L^-T L^-1 B                     column blocks of B in LDS, updates on
//                                                   the matrix cores
//   readout  : Yhat = Phi W
// Every reduction runs in a fixed order (no floating-point atomics), so
// results are bitwise reproducible run to run.
#include <type_traits>

#include "common.h"
#include "mfma64.h"
#include "randnet.h"

namespace rpr {

// ------------------------------------------------------------- features ---
// Z = (X / s) A^T with X (n x d) and A (M x d) both K-contiguous, on the
// matrix cores: a work-group takes 64 rows of X x 64 neurons, wavefront w
// the 32 x 32 quarter (w / 2, w % 2) as 2 x 2 tiles of 16 x 16, k in order,
// 4 per product.  The K range is split over gridDim.z into partial sums
// reduced in order later.  X rows may be FP64 or FP32 (the state
// precision); the product is FP64.  Rows past the device row count and
// neurons past M read as zero (clamped loads, masked after them).
constexpr int FK = 64;  // K chunks are multiples of this

template <typename TX>
__global__ __launch_bounds__(256) void k_feat_partial(int n, int M, int d, int kchunk,
                                                      const TX *__restrict__ X, const double *__restrict__ A,
                                                      double xs, double *__restrict__ part,
                                                      const int *__restrict__ nrows_dev)
{
    const int nr = nrows_dev ? *nrows_dev : n;
    if ((int)blockIdx.x * 64 >= nr) return;  // the whole work-group
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = blockIdx.x * 64 + 32 * (w >> 1), m0 = blockIdx.y * 64 + 32 * (w & 1);
    const int k0 = blockIdx.z * kchunk, k1 = min(d, k0 + kchunk);
    const int kq = lane >> 4, li = lane & 15;
    const TX *xp[2];
    const double *ap[2];
    bool xok[2], aok[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = r0 + 16 * q + li, m = m0 + 16 * q + li;
        xok[q] = r < nr;
        aok[q] = m < M;
        xp[q] = X + (size_t)(xok[q] ? r : nr - 1) * d;
        ap[q] = A + (size_t)(aok[q] ? m : M - 1) * d;
    }
    dbl4 acc[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = dbl4{0.0, 0.0, 0.0, 0.0};
    auto product = [&](const double (&xv)[2], const double (&av)[2]) {
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = mfma64(xv[ti], av[tj], acc[ti][tj]);
    };
    int k = k0;
    for (; k + 16 <= k1; k += 16) {
        double xv[4][2], av[4][2];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                xv[u][q] = double(xp[q][k + 4 * u + kq]);
                av[u][q] = ap[q][k + 4 * u + kq];
            }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                xv[u][q] = xok[q] ? xv[u][q] * xs : 0.0;
                av[u][q] = aok[q] ? av[u][q] : 0.0;
            }
            product(xv[u], av[u]);
        }
    }
    for (; k < k1; k += 4) {
        const int kk = k + kq;
        const bool in = kk < k1;
        const int kc = in ? kk : k;
        double xv[2], av[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double x = double(xp[q][kc]), a = ap[q][kc];
            xv[q] = in && xok[q] ? x * xs : 0.0;
            av[q] = in && aok[q] ? a : 0.0;
        }
        product(xv, av);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = r0 + 16 * ti + mfma64_row(lane, e), m = m0 + 16 * tj + mfma64_col(lane);
                if (r < nr && m < M) part[((size_t)blockIdx.z * n + r) * M + m] = acc[ti][tj][e];
            }
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
    dim3 grid((n + 63) / 64, (M + 63) / 64, ns);
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
// Mixed-precision hidden layer: inputs x/s and weights split into three
// bfloat16 pieces each (round to nearest even), the six leading products of
// the pieces accumulated in FP32 on the matrix cores
// (v_mfma_f32_16x16x32_bf16) over K chunks; the chunks' partial sums, zeta
// and sigma are taken in double, and Phi is stored in double for the FP64
// statistics.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Three-piece bfloat16 split of v: v ~ p0 + p1 + p2, each piece the
// bfloat16 rounding of what the previous ones leave (24 significant bits in
// all; |v - p0 - p1 - p2| <= 2^-27 |v|).
__device__ __forceinline__ void split_bf16(double v, uint16_t &p0, uint16_t &p1, uint16_t &p2)
{
    p0 = to_bf16((float)v);
    const double r1 = v - (double)from_bf16(p0);
    p1 = to_bf16((float)r1);
    const double r2 = r1 - (double)from_bf16(p1);
    p2 = to_bf16((float)r2);
}

// out = the three pieces of in, piece p at out + p n.
__global__ void k_to_bf16(const double *__restrict__ in, uint16_t *__restrict__ out, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) split_bf16(in[i], out[i], out[n + i], out[2 * n + i]);
}

rpr_status launch_to_bf16(const double *in, uint16_t *out, size_t n, hipStream_t st)
{
    if (n == 0) return RPR_OK;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}

// out (cols x rows) = in^T (in: rows x cols, row-major), through 32 x 32 LDS
// tiles (padded against bank conflicts); 32 x 8 threads.
template <typename E>
__global__ __launch_bounds__(256) void k_transpose(const E *__restrict__ in, E *__restrict__ out, int rows, int cols)
{
    __shared__ E tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    for (int k = ty; k < 32; k += 8)
        if (r0 + k < rows && c0 + tx < cols) tile[k][tx] = in[(size_t)(r0 + k) * cols + c0 + tx];
    __syncthreads();
    for (int k = ty; k < 32; k += 8)
        if (c0 + k < cols && r0 + tx < rows) out[(size_t)(c0 + k) * rows + r0 + tx] = tile[tx][k];
}

template <typename E>
rpr_status launch_transpose(const E *in, E *out, int rows, int cols, hipStream_t st)
{
    if (rows <= 0 || cols <= 0) return RPR_OK;
    hipLaunchKernelGGL(k_transpose<E>, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, st, in, out, rows,
                       cols);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}
template rpr_status launch_transpose<double>(const double *, double *, int, int, hipStream_t);
template rpr_status launch_transpose<uint16_t>(const uint16_t *, uint16_t *, int, int, hipStream_t);

// Split-bfloat16 feature GEMM Z = (X / s) A^T on MFMA: both operands are
// split in three bfloat16 pieces (X on the fly, A beforehand) and the six
// products of the pieces down to 2^-16 relative, x0 a0, x0 a1, x1 a0, x0 a2,
// x2 a0, x1 a1, are accumulated in FP32 (bfloat16 products are exact in
// FP32).  The dropped products are below 2^-24 |x a|.
// Work-group tile: 64 rows of X x 64 neurons, 4 waves; wave w owns rows
// 16w..16w+15 and all four 16-neuron tiles.  K advances 32 at a time through
// LDS.  Operand layout of the 16x16x32 instruction: lane l holds A[l%16][8(l/16)..+7],
// B[8(l/16)..+7][l%16], and D[4(l/16)+e][l%16], e = 0..3.
constexpr int BT = 64, BK = 32, BKP = 40;  // LDS row pitch 80 B keeps 16-byte alignment

template <typename TX>
__global__ __launch_bounds__(256) void k_feat_bf16_partial(int n, int M, int d, int kchunk,
                                                           const TX *__restrict__ X,
                                                           const uint16_t *__restrict__ Ab, double xs,
                                                           float *__restrict__ part,
                                                           const int *__restrict__ nrows_dev)
{
    const int nr = nrows_dev ? *nrows_dev : n;
    const int r0 = blockIdx.x * BT, m0 = blockIdx.y * BT;
    if (r0 >= nr) return;
    const int k0 = blockIdx.z * kchunk, k1 = min(d, k0 + kchunk);
    const size_t md = (size_t)M * d;
    __shared__ __align__(16) uint16_t Xs[3][BT][BKP], As[3][BT][BKP];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int lr = t >> 2, lk = (t & 3) * 8;  // loader: row, first k of 8
    f32x4_t acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    for (int kb = k0; kb < k1; kb += BK) {
        {
            const int r = r0 + lr, m = m0 + lr;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = kb + lk + e;
                const bool kin = k < k1;
                uint16_t x0 = 0, x1 = 0, x2 = 0;
                if (r < nr && kin) split_bf16(double(X[(size_t)r * d + k]) * xs, x0, x1, x2);
                Xs[0][lr][lk + e] = x0;
                Xs[1][lr][lk + e] = x1;
                Xs[2][lr][lk + e] = x2;
#pragma unroll
                for (int p = 0; p < 3; ++p)
                    As[p][lr][lk + e] = (m < M && kin) ? Ab[p * md + (size_t)m * d + k] : (uint16_t)0;
            }
        }
        __syncthreads();
        bf16x8_t xa[3];
#pragma unroll
        for (int p = 0; p < 3; ++p)
            xa[p] = __builtin_bit_cast(bf16x8_t,
                                       *reinterpret_cast<const uint4 *>(&Xs[p][w * 16 + (lane & 15)][8 * (lane >> 4)]));
        bf16x8_t ab[4][3];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int p = 0; p < 3; ++p)
                ab[j][p] = __builtin_bit_cast(
                    bf16x8_t, *reinterpret_cast<const uint4 *>(&As[p][j * 16 + (lane & 15)][8 * (lane >> 4)]));
        // smallest products first: x1 a1, x2 a0, x0 a2, x1 a0, x0 a1, x0 a0,
        // the four accumulators interleaved so consecutive MFMAs are independent
        constexpr int PX[6] = {1, 2, 0, 1, 0, 0}, PA[6] = {1, 0, 2, 0, 1, 0};
#pragma unroll
        for (int q = 0; q < 6; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[PX[q]], ab[j][PA[q]], acc[j], 0, 0, 0);
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

// The same partial sums for large tiles: 128 rows of X x 128 neurons per
// work-group (4 waves in 2 x 2, each 64 x 64 = 4 x 4 MFMA tiles), for
// d % 8 == 0 so that every lane moves 16 bytes per load.  The inputs come
// split beforehand (k_split_rows: the pieces split_bf16 gives on the fly in
// k_feat_bf16_partial), so the K-loop is loads, LDS and MFMA only.  The
// K-split, the K-steps of 32 and the six products per step are in the same
// order as k_feat_bf16_partial, so both kernels give identical partial
// sums.  The next K-step's global loads are in flight while the current one
// is multiplied out of LDS.
constexpr int GT = 128;

// LDS rows of the large-tile kernel are 64 bytes (32 bfloat16, no padding);
// 16-byte chunk c of row r sits at chunk c ^ lds_swz(r).  Writes (4 lanes
// per row) and fragment reads (16 rows at one chunk) then hit distinct banks
// for 32 as for 64 banks of 4 bytes.
__device__ __forceinline__ int lds_swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

// The three bfloat16 pieces of X / s, rows r < nr: piece p of X[r][k] at
// out[p n d + r d + k].
template <typename TX>
__global__ __launch_bounds__(256) void k_split_rows(int n, int d, const TX *__restrict__ X, double xs,
                                                    uint16_t *__restrict__ out, const int *__restrict__ nrows_dev)
{
    const int nr = nrows_dev ? *nrows_dev : n;
    const size_t nd = (size_t)n * d, e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)nr * d) return;
    uint16_t x0, x1, x2;
    split_bf16(double(X[e]) * xs, x0, x1, x2);
    out[e] = x0;
    out[nd + e] = x1;
    out[2 * nd + e] = x2;
}

__global__ __launch_bounds__(256, 2) void k_feat_bf16_gemm(int n, int M, int d, int kchunk,
                                                        const uint16_t *__restrict__ Xb,
                                                        const uint16_t *__restrict__ Ab, float *__restrict__ part,
                                                        const int *__restrict__ nrows_dev)
{
    constexpr int LQ = GT * BK / 8 / 256;  // 16-byte loads per thread, K-step and piece, for X and for A
    const int nr = nrows_dev ? *nrows_dev : n;
    const int r0 = blockIdx.x * GT, m0 = blockIdx.y * GT;
    if (r0 >= nr) return;
    const int k0 = blockIdx.z * kchunk, k1 = min(d, k0 + kchunk);
    const size_t md = (size_t)M * d, nd = (size_t)n * d;
    __shared__ __align__(16) uint16_t Xs[3][GT][BK], As[3][GT][BK];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;  // this wave's 64 x 64 quadrant

    // load group q of this thread: tile row (t + 256 q) / 4, k offset
    // 8 ((t + 256 q) % 4), for every piece of X and of A
    uint4 xv[3][LQ], av[3][LQ];
    auto load = [&](int kb) {
#pragma unroll
        for (int q = 0; q < LQ; ++q) {
            const int g = t + 256 * q, lr = g >> 2, k = kb + 8 * (g & 3);
            const int r = r0 + lr, m = m0 + lr;
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                xv[p][q] = (r < nr && k < k1) ? *reinterpret_cast<const uint4 *>(Xb + p * nd + (size_t)r * d + k)
                                              : uint4{0u, 0u, 0u, 0u};
                av[p][q] = (m < M && k < k1) ? *reinterpret_cast<const uint4 *>(Ab + p * md + (size_t)m * d + k)
                                             : uint4{0u, 0u, 0u, 0u};
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < LQ; ++q) {
            const int g = t + 256 * q, lr = g >> 2, lk = 8 * ((g & 3) ^ lds_swz(lr));
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                *reinterpret_cast<uint4 *>(&Xs[p][lr][lk]) = xv[p][q];
                *reinterpret_cast<uint4 *>(&As[p][lr][lk]) = av[p][q];
            }
        }
    };

    f32x4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    load(k0);
    store();
    __syncthreads();
    for (int kb = k0; kb < k1; kb += BK) {
        const bool more = kb + BK < k1;
        if (more) load(kb + BK);
        bf16x8_t ab[4][3];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int R = wc * 64 + j * 16 + (lane & 15), c = 8 * ((lane >> 4) ^ lds_swz(R));
#pragma unroll
            for (int p = 0; p < 3; ++p)
                ab[j][p] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4 *>(&As[p][R][c]));
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bf16x8_t xa[3];
            const int R = wr * 64 + i * 16 + (lane & 15), c = 8 * ((lane >> 4) ^ lds_swz(R));
#pragma unroll
            for (int p = 0; p < 3; ++p)
                xa[p] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4 *>(&Xs[p][R][c]));
            // smallest products first (as k_feat_bf16_partial); the four
            // accumulators of the row block interleaved, so consecutive
            // MFMAs are independent
            constexpr int PX[6] = {1, 2, 0, 1, 0, 0}, PA[6] = {1, 0, 2, 0, 1, 0};
#pragma unroll
            for (int q = 0; q < 6; ++q)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[PX[q]], ab[j][PA[q]], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
        if (more) {
            store();
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = r0 + wr * 64 + i * 16 + 4 * (lane >> 4) + e;
                const int m = m0 + wc * 64 + j * 16 + (lane & 15);
                if (r < nr && m < M) part[((size_t)blockIdx.z * n + r) * M + m] = acc[i][j][e];
            }
}

// Phi = sigma(sum of the K-split partials + zeta), in double.
__global__ void k_feat_bf16_finish(int n, int M, int nsplit, const float *__restrict__ part,
                                   const double *__restrict__ zeta, int act, double *__restrict__ Phi,
                                   const int *__restrict__ nrows_dev)
{
    const int nr = nrows_dev ? *nrows_dev : n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr * M) return;
    double z = 0.0;
    for (int s = 0; s < nsplit; ++s) z += (double)part[(size_t)s * n * M + i];
    z += zeta[i % M];
    Phi[i] = act == RPR_RELU ? (z > 0.0 ? z : 0.0) : tanh(z);
}

int feat_bf16_splits(int d)
{
    int s = (d + 1023) / 1024;  // about 1024 of K per work-group
    return s < 1 ? 1 : (s > 64 ? 64 : s);
}

// The large-tile kernel's vector loads keep a K-step's loads in flight
// together; the small one issues element loads and serves only a few rows.
bool feat_bf16_large(int n, int d) { return n > 16 && d % 8 == 0; }

template <typename TX>
rpr_status launch_features_bf16(int n, int M, int d, int act, double inv_s, const uint16_t *Ab,
                                const double *zeta, const TX *X, double *Phi, float *part,
                                const int *nrows_dev, hipStream_t st, uint16_t *xb)
{
    if (n <= 0) return RPR_OK;
    const int ns = feat_bf16_splits(d);
    const int kchunk = ((d + ns - 1) / ns + BK - 1) / BK * BK;
    if (xb && feat_bf16_large(n, d)) {
        const size_t nd = (size_t)n * d;
        hipLaunchKernelGGL(k_split_rows<TX>, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, st, n, d, X, inv_s,
                           xb, nrows_dev);
        dim3 grid((n + GT - 1) / GT, (M + GT - 1) / GT, ns);
        hipLaunchKernelGGL(k_feat_bf16_gemm, grid, dim3(256), 0, st, n, M, d, kchunk, xb, Ab, part, nrows_dev);
    } else {
        dim3 grid((n + BT - 1) / BT, (M + BT - 1) / BT, ns);
        hipLaunchKernelGGL(k_feat_bf16_partial<TX>, grid, dim3(256), 0, st, n, M, d, kchunk, X, Ab, inv_s, part,
                           nrows_dev);
    }
    RPR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_feat_bf16_finish, dim3((n * M + 255) / 256), dim3(256), 0, st, n, M, ns, part, zeta,
                       act, Phi, nrows_dev);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}
template rpr_status launch_features_bf16<float>(int, int, int, int, double, const uint16_t *, const double *,
                                                const float *, double *, float *, const int *, hipStream_t,
                                                uint16_t *);
template rpr_status launch_features_bf16<double>(int, int, int, int, double, const uint16_t *, const double *,
                                                 const double *, double *, float *, const int *, hipStream_t,
                                                 uint16_t *);

// ----------------------------------------------------------- statistics ---
// S[a][j] += sum_r ok_r Phi[r][a] Y[r][j] (B = Phi^T Y with Y the targets,
// and the Gram matrix G = Phi^T Phi with Y = Phi) on the matrix cores: a
// work-group takes 64 neurons x 64 columns, wavefront w the 32 x 32 quarter
// (w / 2, w % 2) as 2 x 2 tiles of 16 x 16; the rows r in order, 4 per
// product.  Rows with ok_r = 0 (dropped pairs) contribute nothing whatever
// they hold: their values are replaced by zero, not multiplied by it.
// Loads go to clamped in-range addresses and the masks are applied after
// them, so that the loads of a batch are in flight together.
template <typename TY>
__global__ __launch_bounds__(256) void k_stat(int n, int M, int d, const double *__restrict__ Phi,
                                              const TY *__restrict__ Y, const int *__restrict__ ok,
                                              double *__restrict__ S, const int *__restrict__ nrows_dev)
{
    const int nr = nrows_dev ? *nrows_dev : n;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int a0 = blockIdx.y * 64 + 32 * (w >> 1), j0 = blockIdx.x * 64 + 32 * (w & 1);
    const int kq = lane >> 4, li = lane & 15;
    int ac[2], bc[2];
    bool aok[2], bok[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        ac[q] = a0 + 16 * q + li;
        bc[q] = j0 + 16 * q + li;
        aok[q] = ac[q] < M;
        bok[q] = bc[q] < d;
        ac[q] = aok[q] ? ac[q] : M - 1;
        bc[q] = bok[q] ? bc[q] : d - 1;
    }
    dbl4 acc[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = dbl4{0.0, 0.0, 0.0, 0.0};
    auto product = [&](const double (&av)[2], const double (&bv)[2]) {
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = mfma64(av[ti], bv[tj], acc[ti][tj]);
    };
    int r = 0;
    for (; r + 16 <= nr; r += 16) {
        double av[4][2], bv[4][2];
        bool use[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int rr = r + 4 * u + kq;
            use[u] = ok == nullptr || ok[rr] != 0;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                av[u][q] = Phi[(size_t)rr * M + ac[q]];
                bv[u][q] = double(Y[(size_t)rr * d + bc[q]]);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                av[u][q] = use[u] && aok[q] ? av[u][q] : 0.0;
                bv[u][q] = use[u] && bok[q] ? bv[u][q] : 0.0;
            }
            product(av[u], bv[u]);
        }
    }
    for (; r < nr; r += 4) {
        const int rr = r + kq;
        const bool in = rr < nr;
        const int rc = in ? rr : r;
        const bool use = in && (ok == nullptr || ok[rc] != 0);
        double av[2], bv[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double x = Phi[(size_t)rc * M + ac[q]];
            const double y = double(Y[(size_t)rc * d + bc[q]]);
            av[q] = use && aok[q] ? x : 0.0;
            bv[q] = use && bok[q] ? y : 0.0;
        }
        product(av, bv);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int a = a0 + 16 * ti + mfma64_row(lane, e), j = j0 + 16 * tj + mfma64_col(lane);
                if (a < M && j < d) S[(size_t)a * d + j] += acc[ti][tj][e];
            }
}

template <typename TY>
rpr_status launch_stats(int n, int M, int d, const double *Phi, const TY *Y, const int *ok, double *G,
                        double *Bm, const int *nrows_dev, hipStream_t st)
{
    if (n <= 0) return RPR_OK;
    hipLaunchKernelGGL(k_stat<double>, dim3((M + 63) / 64, (M + 63) / 64), dim3(256), 0, st, n, M, M, Phi, Phi, ok,
                       G, nrows_dev);
    RPR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_stat<TY>, dim3((d + 63) / 64, (M + 63) / 64), dim3(256), 0, st, n, M, d, Phi, Y, ok, Bm,
                       nrows_dev);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}
template rpr_status launch_stats<double>(int, int, int, const double *, const double *, const int *,
                                         double *, double *, const int *, hipStream_t);
template rpr_status launch_stats<float>(int, int, int, const double *, const float *, const int *,
                                        double *, double *, const int *, hipStream_t);

// ------------------------------------------------------------- cholesky ---
// Blocked left-looking Cholesky factorisation S = G + lambda I = L L^T with
// 32-column panels, one work-group of 32 x 32 threads (thread (j, rl): panel
// column j, row lane rl).  For the panel of columns c0 .. c0+nb:
//   1. P = S[c0:, c0:c0+nb] - L[c0:, :c0] L[c0:c0+nb, :c0]^T for rows
//      c0+rl+32q; the panel's top rows L[c0:c0+nb, :c0] are staged in LDS
//      once, the other factor is read from L directly;
//   2. the nb x nb top block of P is factored by one wavefront, lane = row,
//      each row in registers, the columns passed between lanes by shuffles;
//   3. every row x below it solves x L_kk^T = P[row] by substitution along
//      the 32 lanes of its half-wavefront.
// Writes L (lower, row-major, zero above) and Lt = L^T.  A non-positive or
// NaN pivot sets *fail = 1, counts in *fail_count (both may be null) and
// continues with pivot 1.
constexpr int CB = 32;
constexpr int CB_MAX_M = 512;

__global__ __launch_bounds__(1024) void k_cholesky(int M, const double *__restrict__ G, double lambda,
                                                   double *__restrict__ L, double *__restrict__ Lt,
                                                   int *__restrict__ fail, int *__restrict__ fail_count,
                                                   const int *__restrict__ done)
{
    if (done && *done) return;
    extern __shared__ double top[];  // top[p * 33 + j] = L[c0 + j][p], p < c0
    __shared__ double D[CB][CB + 1]; // diagonal block of the panel
    __shared__ int bad;
    const int t = threadIdx.x, j = t % CB, rl = t / CB;
    if (t == 0) {
        bad = 0;
        if (fail) *fail = 0;
    }
    for (int i = t; i < M * M; i += CB * CB) {
        L[i] = 0.0;
        Lt[i] = 0.0;
    }
    const int nblk = (M + CB - 1) / CB;
    __syncthreads();

    for (int k = 0; k < nblk; ++k) {
        const int c0 = k * CB, nb = min(CB, M - c0);
        const int nq = rl < M - c0 ? (M - c0 - rl + CB - 1) / CB : 0;  // rows c0 + rl + 32 q < M

        // 1. panel update against the finished columns 0 .. c0
        for (int e = t; e < c0 * CB; e += CB * CB) {
            const int jj = e / c0, p = e % c0;  // coalesced along each row of L
            top[p * (CB + 1) + jj] = jj < nb ? L[(size_t)(c0 + jj) * M + p] : 0.0;
        }
        __syncthreads();
        // P of the rows below the block goes to L (solved in place in step 3),
        // the block's own rows to D
        for (int q = 0; q < nq; ++q) {
            const int r = c0 + rl + CB * q;
            const double *X = L + (size_t)r * M;
            double sacc = 0.0;
            // c0 is a multiple of 32: batches of 16 independent loads
            for (int p0 = 0; p0 < c0; p0 += 16) {
                double xv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) xv[u] = X[p0 + u];
#pragma unroll
                for (int u = 0; u < 16; ++u) sacc = fma(xv[u], top[(p0 + u) * (CB + 1) + j], sacc);
            }
            if (q == 0) {
                if (j < nb && rl < nb) {
                    double sv = rl >= j ? G[(size_t)r * M + c0 + j] : 0.0;
                    if (rl == j) sv += lambda;
                    D[rl][j] = sv - sacc;
                }
            } else if (j < nb) {
                L[(size_t)r * M + c0 + j] = G[(size_t)r * M + c0 + j] - sacc;
            }
        }
        __syncthreads();

        // 2. factor the diagonal block: wavefront 0, lane r = row r
        if (t < 64) {
            const int r = t & (CB - 1);
            double row[CB];
#pragma unroll
            for (int x = 0; x < CB; ++x) row[x] = (r < nb && x < nb) ? D[r][x] : 0.0;
            bool badw = false;
#pragma unroll
            for (int jj = 0; jj < CB; ++jj) {
                if (jj < nb) {
                    const double piv = __shfl(row[jj], jj, CB);
                    badw = badw || !(piv > 0.0);
                    const double djj = sqrt(piv > 0.0 ? piv : 1.0);
                    const double lr = r > jj ? row[jj] / djj : (r == jj ? djj : 0.0);
                    row[jj] = lr;
#pragma unroll
                    for (int j2 = jj + 1; j2 < CB; ++j2) {
                        if (j2 < nb) {
                            const double lj = __shfl(lr, j2, CB);  // L[j2][jj]
                            if (r >= j2) row[j2] = fma(-lr, lj, row[j2]);
                        }
                    }
                }
            }
            if (r < nb)
#pragma unroll
                for (int x = 0; x < CB; ++x) D[r][x] = x <= r ? row[x] : 0.0;
            if (t == 0 && badw) bad = 1;
        }
        __syncthreads();

        // 3. rows below the block
        const double rinv = j < nb ? 1.0 / D[j][j] : 0.0;
        auto solve_row = [&](double pv) {
            for (int jj = 0; jj < nb; ++jj) {
                if (j == jj) pv *= rinv;
                const double xb = __shfl(pv, jj, CB);
                if (j > jj && j < nb) pv = fma(-xb, D[j][jj], pv);
            }
            return pv;
        };
        for (int q = 1; q < nq; ++q) {
            const int r = c0 + rl + CB * q;
            const double x = solve_row(j < nb ? L[(size_t)r * M + c0 + j] : 0.0);
            if (j < nb) {
                L[(size_t)r * M + c0 + j] = x;
                Lt[(size_t)(c0 + j) * M + r] = x;
            }
        }
        if (rl < nb && j <= rl) {
            L[(size_t)(c0 + rl) * M + c0 + j] = D[rl][j];
            Lt[(size_t)(c0 + j) * M + c0 + rl] = D[rl][j];
        }
        __syncthreads();
    }
    if (t == 0 && bad) {
        if (fail) *fail = 1;
        if (fail_count) *fail_count += 1;
    }
}

// ---------------------------------------------------------------- solve ---
// W = (L L^T)^{-1} B = L^-T L^-1 B for a block of 32 columns of B per
// work-group of 256 threads.  Block forward then backward substitution over
// 32-row blocks: each block first subtracts the product with the rows already
// solved (a 32 x 32 product over those rows on the matrix cores, one 16 x 16
// tile per wavefront), then is solved against its diagonal block by
// substitution along the 32 lanes of a half-wavefront (lane = row; each
// half-wavefront takes 4 columns).  The M x 32 block of B stays in LDS.  If
// the factorisation failed (*fail), W is set to zero.
__global__ __launch_bounds__(256) void k_trsm(int M, int d, const double *__restrict__ L,
                                              const double *__restrict__ Lt, const double *__restrict__ Bm,
                                              double *__restrict__ W, const int *__restrict__ fail,
                                              const int *__restrict__ done)
{
    if (done && *done) return;
    extern __shared__ double Y[];  // M x 32
    const int t = threadIdx.x, c = t % CB, g = t / CB;
    const int j0 = blockIdx.x * CB;
    const bool failed = fail && *fail;
    {
        // thread t fills column t % 32 of the block, rows t / 32 + 8 i, in
        // batches of 8 loads in flight (clamped addresses, masked after)
        const int cc = t % CB;
        const bool colok = !failed && j0 + cc < d;
        const double *bp = Bm + (colok ? j0 + cc : 0);
        for (int r = t / CB; r < M; r += 64) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = bp[(size_t)min(r + 8 * u, M - 1) * d];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (r + 8 * u < M) Y[(r + 8 * u) * CB + cc] = colok ? v[u] : 0.0;
        }
    }
    const int nblk = (M + CB - 1) / CB;
    if (!failed) {
        for (int pass = 0; pass < 2; ++pass) {
            const bool fwd = pass == 0;
            for (int bi = 0; bi < nblk; ++bi) {
                const int b = fwd ? bi : nblk - 1 - bi;
                const int r0 = b * CB, rb = min(CB, M - r0);
                // rows already solved: forward rows 0 .. r0 of L, backward rows
                // r0+32 .. M of L^T (the columns below the block)
                __syncthreads();  // the previous block's rows of Y are final
                // Y[block] -= src[block rows][p_lo, p_hi) Y[p_lo, p_hi) on the
                // matrix cores: wavefront w takes the 16 x 16 tile (rows
                // 16 (w / 2), columns 16 (w % 2)) of the 32 x 32 block, the
                // rows of L (or L^T) from memory, the solved rows of Y from
                // LDS, 4 k per product in order
                const int p_lo = fwd ? 0 : r0 + CB, p_hi = fwd ? r0 : M;
                const double *src = fwd ? L : Lt;
                const int lane = t & 63, w = t >> 6, ti = w >> 1, tj = w & 1;
                const int ar = r0 + 16 * ti + (lane & 15);  // this lane's row of the A tile
                const bool arow_ok = ar < M;                // rows past M read as zero
                const double *arow = src + (size_t)(arow_ok ? ar : M - 1) * M;
                const int kq = lane >> 4, bc = 16 * tj + (lane & 15);
                dbl4 acc = {0.0, 0.0, 0.0, 0.0};
                int p = p_lo;
                for (; p + 16 <= p_hi; p += 16) {
                    double av[4], bv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int pp = p + 4 * u + kq;
                        av[u] = arow[pp];
                        bv[u] = Y[pp * CB + bc];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc = mfma64(arow_ok ? av[u] : 0.0, bv[u], acc);
                }
                for (; p < p_hi; p += 4) {
                    const int pp = p + kq;
                    const bool in = pp < p_hi;
                    const double av = arow[in ? pp : p_lo];
                    const double bv = Y[(in ? pp : p_lo) * CB + bc];
                    acc = mfma64(arow_ok && in ? av : 0.0, in ? bv : 0.0, acc);
                }
                __syncthreads();
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = r0 + 16 * ti + mfma64_row(lane, e);
                    if (r < M) Y[r * CB + 16 * tj + mfma64_col(lane)] -= acc[e];
                }
                // the diagonal block of L in registers: lane rr holds row rr of
                // it (forward: L[r0 + rr][r0 + jj]) or column rr (backward:
                // L[r0 + jj][r0 + rr]), the 32 loads in flight together
                const int rr = c;  // lane within the half-wavefront = row of the block
                double lw[CB];
#pragma unroll
                for (int jj = 0; jj < CB; ++jj) {
                    const int ra = min(r0 + (fwd ? rr : jj), M - 1), cb = min(r0 + (fwd ? jj : rr), M - 1);
                    lw[jj] = L[(size_t)ra * M + cb];
                }
                const double dg = L[(size_t)min(r0 + rr, M - 1) * (M + 1)];
                const double rinv = rr < rb ? 1.0 / dg : 0.0;
                double z[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) z[i] = rr < rb ? Y[(r0 + rr) * CB + g + 8 * i] : 0.0;
                // forward: x_jj = z_jj / L[jj][jj], then z_rr -= L[rr][jj] x_jj
                // (rr > jj), jj = 0 .. rb - 1; backward: z_rr -= L[jj][rr] x_jj
                // (rr < jj), jj = rb - 1 .. 0.  Unrolled over the 32 positions
                // (those past rb skipped) so that lw is indexed by constants.
                auto substitute = [&](auto fwd_tag) {
                    constexpr bool FWD = decltype(fwd_tag)::value;
#pragma unroll
                    for (int s2 = 0; s2 < CB; ++s2) {
                        const int jj = FWD ? s2 : CB - 1 - s2;
                        if (jj >= rb) continue;  // uniform
                        const bool upd = FWD ? (rr > jj && rr < rb) : rr < jj;
                        const double l = upd ? lw[jj] : 0.0;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (rr == jj) z[i] *= rinv;
                            const double xb = __shfl(z[i], jj, CB);
                            if (upd) z[i] = fma(-l, xb, z[i]);
                        }
                    }
                };
                if (fwd) substitute(std::true_type{});
                else substitute(std::false_type{});
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (rr < rb) Y[(r0 + rr) * CB + g + 8 * i] = z[i];
            }
        }
    }
    __syncthreads();
    for (int i = t; i < M * CB; i += 256) {
        const int r = i / CB, cc = i % CB;
        if (j0 + cc < d) W[(size_t)r * d + j0 + cc] = Y[i];
    }
}

rpr_status launch_ridge_solve(int M, int d, const double *G, double lambda, double *L, double *Lt, double *W,
                              const double *Bm, int *fail, int *fail_count, const int *done, hipStream_t st)
{
    if (M > CB_MAX_M) return rpr::fail(RPR_ERR_UNSUPPORTED, "ridge solve: M > 512");
    static bool chol_attr = false;
    if (!chol_attr) {
        RPR_HIP(hipFuncSetAttribute((const void *)k_cholesky, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(kMaxLds - sizeof(double) * CB * (CB + 1) - 64)));
        chol_attr = true;
    }
    // the largest panel offset c0 = 32 (ceil(M / 32) - 1) sets the staged rows
    const size_t c0_max = (size_t)CB * ((M + CB - 1) / CB - 1);
    const size_t top_lds = sizeof(double) * (c0_max > 0 ? c0_max : 1) * (CB + 1);
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(CB * CB), top_lds, st, M, G, lambda, L, Lt, fail, fail_count,
                       done);
    RPR_HIP(hipGetLastError());
    const size_t lds = (size_t)M * CB * sizeof(double);
    if (lds > kMaxLds) return rpr::fail(RPR_ERR_UNSUPPORTED, "ridge solve: M too large for LDS block");
    static bool attr_set = false;
    if (!attr_set) {
        RPR_HIP(hipFuncSetAttribute((const void *)k_trsm, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
        attr_set = true;
    }
    hipLaunchKernelGGL(k_trsm, dim3((d + CB - 1) / CB), dim3(256), lds, st, M, d, L, Lt, Bm, W, fail, done);
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

// ------------------------------------------------- nearest-neighbour store --
template <typename T>
__global__ __launch_bounds__(256) void k_nn_append(int d, int M, const T *__restrict__ X, const T *__restrict__ Y,
                                                   const double *__restrict__ Phi, const int *__restrict__ ok,
                                                   const int *__restrict__ nrows, const Ctrl *__restrict__ ctrl,
                                                   T *__restrict__ Xs, T *__restrict__ Ys, double *__restrict__ Ps,
                                                   int *__restrict__ oks, int n_cap)
{
    const int r = blockIdx.x;
    if (r >= *nrows) return;
    const int row = ctrl->nn_rows + r;
    if (row >= n_cap) return;  // the store holds N k_max rows: cannot happen
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        Xs[(size_t)row * d + j] = X[(size_t)r * d + j];
        Ys[(size_t)row * d + j] = Y[(size_t)r * d + j];
    }
    for (int m = threadIdx.x; m < M; m += blockDim.x) Ps[(size_t)row * M + m] = Phi[(size_t)r * M + m];
    if (threadIdx.x == 0) oks[row] = ok[r];
}

template <typename T>
rpr_status launch_nn_append(int N, int d, int M, const T *X, const T *Y, const double *Phi, const int *ok,
                            const int *nrows, const Ctrl *ctrl, T *Xs, T *Ys, double *Ps, int *oks, int n_cap,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_nn_append<T>, dim3(N), dim3(256), 0, st, d, M, X, Y, Phi, ok, nrows, ctrl, Xs, Ys, Ps, oks,
                       n_cap);
    RPR_HIP(hipGetLastError());
    return RPR_OK;
}
template rpr_status launch_nn_append<double>(int, int, int, const double *, const double *, const double *,
                                             const int *, const int *, const Ctrl *, double *, double *, double *,
                                             int *, int, hipStream_t);
template rpr_status launch_nn_append<float>(int, int, int, const float *, const float *, const double *, const int *,
                                            const int *, const Ctrl *, float *, float *, double *, int *, int,
                                            hipStream_t);

}  // namespace rpr
