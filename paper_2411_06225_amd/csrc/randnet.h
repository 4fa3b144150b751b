// randnet.h -- launchers of the random-network kernels (randnet.hip).
// All matrices are row-major doubles in device memory unless noted.
// `nrows_dev`, when not null, points to the number of valid rows on the device
// (row count decided by earlier kernels); `n` is then the capacity.
#pragma once

#include "common.h"

namespace rpr {

// Number of K-splits of the feature GEMM (partial buffer: splits x n x M).
int feat_splits(int d);

// Phi = sigma(X A^T * inv_s + zeta); X is n x d of TX (double or float).
template <typename TX>
rpr_status launch_features(int n, int M, int d, int act, double inv_s, const double *A, const double *zeta,
                           const TX *X, double *Phi, double *part, const int *nrows_dev, hipStream_t st);

// Split-bfloat16 features: inputs and weights (Ab, three pieces of M x d,
// from launch_to_bf16) split in three bfloat16 pieces, the six leading
// products of the pieces accumulated in FP32 on the matrix cores, the K-split
// partials and sigma in double.  part holds feat_bf16_splits(d) x n x M floats.
// With xb (3 n d bfloat16 workspace) non-null and feat_bf16_large(n, d),
// the inputs are split in a pass of their own and a 128 x 128-tile kernel
// forms the same partial sums (bit for bit).
int feat_bf16_splits(int d);
bool feat_bf16_large(int n, int d);
template <typename TX>
rpr_status launch_features_bf16(int n, int M, int d, int act, double inv_s, const uint16_t *Ab,
                                const double *zeta, const TX *X, double *Phi, float *part,
                                const int *nrows_dev, hipStream_t st, uint16_t *xb = nullptr);

// The three bfloat16 pieces of in (round to nearest even each): out holds
// 3 n values, piece p at out + p n.
rpr_status launch_to_bf16(const double *in, uint16_t *out, size_t n, hipStream_t st);

// G += Phi^T Phi and B += Phi^T Y over the rows r with ok[r] != 0 (ok may be null).
template <typename TY>
rpr_status launch_stats(int n, int M, int d, const double *Phi, const TY *Y, const int *ok, double *G,
                        double *Bm, const int *nrows_dev, hipStream_t st);

// L L^T = G + lambda I (L, Lt = L^T: M x M workspaces), then W = (L L^T)^{-1} B.
// M <= 512.  A failed factorisation sets *fail, increments *fail_count and
// zeroes W.  With `done` non-null and *done != 0 both kernels return at once.
rpr_status launch_ridge_solve(int M, int d, const double *G, double lambda, double *L, double *Lt, double *W,
                              const double *Bm, int *fail, int *fail_count, const int *done, hipStream_t st);

// out (cols x rows) = in^T for a row-major rows x cols matrix.
template <typename E>
rpr_status launch_transpose(const E *in, E *out, int rows, int cols, hipStream_t st);

// Yhat = Phi W (n x d).
rpr_status launch_readout(int n, int M, int d, const double *W, const double *Phi, double *Y, hipStream_t st);

// Training pairs of the current iteration (eq. "Dk") for slots L+1..N:
// X[r] = U[L+r], Y[r] = Fv[L+1+r] - Gc[L+1+r], ok[r] = all finite; *nrows = N-L.
template <typename T>
rpr_status launch_pairs(int N, int d, const T *U, const T *Fv, const T *Gc, T *X, T *Y, int *ok, int *nrows,
                        Ctrl *ctrl, hipStream_t st);

// Nearest-neighbour store: this iteration's pairs (rows r < *nrows of X, Y,
// Phi and ok) are copied to rows ctrl->nn_rows + r of Xs, Ys, Ps and oks
// (n_cap rows).  The chain of the same iteration advances ctrl->nn_rows.
template <typename T>
rpr_status launch_nn_append(int N, int d, int M, const T *X, const T *Y, const double *Phi, const int *ok,
                            const int *nrows, const Ctrl *ctrl, T *Xs, T *Ys, double *Ps, int *oks, int n_cap,
                            hipStream_t st);

// out[k] = U(-1, 1) from counter first + k (SplitMix64).
rpr_status launch_uniform(uint64_t seed, uint64_t first, int64_t n, double *out, hipStream_t st);

}  // namespace rpr
