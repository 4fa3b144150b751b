// mfma64.h -- double-precision products on the matrix cores of gfx950.
//
// v_mfma_f64_16x16x4f64 multiplies a 16 x 4 by a 4 x 16 FP64 tile and adds
// a 16 x 16 accumulator, per wavefront.  Operand layout (measured on the
// device against a host product): lane i + 16 k holds A[i][k] and B[k][i]
// (i < 16, k < 4); element e of lane j + 16 q holds D[4 e + q][j].  Each
// wavefront accumulates its own tiles over K in a fixed order, so results
// are reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>

namespace rpr {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma64(double a, double b, dbl4 acc)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

// Row of the 16 x 16 tile held in element e of this lane's accumulator, and
// its column.
__device__ __forceinline__ int mfma64_row(int lane, int e) { return 4 * e + (lane >> 4); }
__device__ __forceinline__ int mfma64_col(int lane) { return lane & 15; }

}  // namespace rpr
