// Complex matrix products on the matrix cores (gfx950 MFMA) for the blocked LU
// of the dense solve (Sec. 3.4, eq. (3.29)).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ffbie {

// C -= A B for complex column-major blocks sharing the leading dimension ld
// (in complex elements): A is m x k, B is k x n, C is m x n, element (r, c) of
// X at X[2 (c ld + r)] (re) and X[2 (c ld + r) + 1] (im).  A and B must not
// overlap C.  Enqueued on `stream`; m, n or k <= 0 is a no-op.  complex128:
// FP64 MFMA; complex64: FP32 MFMA with FP32 accumulation.
hipError_t gemm_sub_c128(hipStream_t stream, double* C, const double* A, const double* B, int64_t ld,
                         int64_t m, int64_t n, int64_t k);
hipError_t gemm_sub_c64(hipStream_t stream, float* C, const float* A, const float* B, int64_t ld,
                        int64_t m, int64_t n, int64_t k);

}  // namespace ffbie
