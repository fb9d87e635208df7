// The original Kronecker-product formalism (Sec. II.A) for comparison with the
// batched solve: every mode product is a separate small GEMM, one per frontal
// slice for modes 1 and 2 and one over the whole grid for mode 3, so a solve
// takes 4 n3 + 2 GEMM launches plus the eigen-scaling.  FP64, real plans.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"

namespace kx {
namespace {

// C(m x n) = A(m x k) B(k x n), column-major FP64.  64 x 64 tile per block of
// 256 threads (4 x 4 outputs each), 16-deep K steps through LDS.
__global__ void __launch_bounds__(256) k_gemm_nn_f64(int m, int n, int k, const double* __restrict__ A,
                                                     int64_t lda, const double* __restrict__ B, int64_t ldb,
                                                     double* __restrict__ C, int64_t ldc) {
  __shared__ double As[16][65], Bs[16][65];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  double acc[4][4] = {};
  for (int p0 = 0; p0 < k; p0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int r = e % 64, p = e / 64;   // A[i0 + r][p0 + p]
      As[p][r] = (i0 + r < m && p0 + p < k) ? A[(i0 + r) + (int64_t)(p0 + p) * lda] : 0.0;
      const int pp = e % 16, c = e / 16;  // B[p0 + pp][j0 + c]
      Bs[pp][c] = (j0 + c < n && p0 + pp < k) ? B[(p0 + pp) + (int64_t)(j0 + c) * ldb] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int p = 0; p < 16; ++p) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[p][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[p][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = i0 + tx + 16 * a, j = j0 + ty + 16 * b;
      if (i < m && j < n) C[i + (int64_t)j * ldc] = acc[a][b];
    }
}

}  // namespace

hipError_t launch_gemm_nn_f64(int m, int n, int k, const double* A, int64_t lda, const double* B, int64_t ldb,
                              double* C, int64_t ldc, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_nn_f64, dim3((m + 63) / 64, (n + 63) / 64), dim3(256), 0, s, m, n, k, A, lda, B, ldb,
                     C, ldc);
  return hipGetLastError();
}

}  // namespace kx
