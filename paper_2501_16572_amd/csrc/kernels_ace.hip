// Adaptively compressed exchange (ACE) on one GPU, FP64 real and complex128.
//
// Construction (Sec. III.A): M = dV Psi^H W, -M = L L^H (lower Cholesky
// factor), xi = W L^{-H}.  Application (Sec. III.B): chi = dV xi^H Phi, then
// V Phi -= xi chi.  All orbital sets are column-major N x n (one orbital per
// column, leading dimension ld >= N); the small matrices are column-major with
// leading dimension equal to their row count.
//
// The two products with the long dimension N are bound by HBM traffic (each
// reads tall matrices once or twice); they are tiled FP64 VALU kernels:
//   gram:  C(m x n) = alpha * sum_k conj(A[k, i]) B[k, j], split over K in
//          chunks whose partial tiles are summed in a fixed order (bitwise
//          reproducible results);
//   tsmm:  C(K x n) = beta * C + alpha * A(K x m) B(m x n).
// The Cholesky factorization and the triangular inverse of the n_s x n_s
// matrix run in one workgroup each.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "launch.h"

namespace kx {
namespace {

struct Z {
  double re, im;
};

// element operations for double and complex128
__device__ __forceinline__ double conj_(double a) { return a; }
__device__ __forceinline__ Z conj_(Z a) { return Z{a.re, -a.im}; }
__device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ Z fma_(Z a, Z b, Z c) {
  return Z{fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
__device__ __forceinline__ double scale_(double s, double a) { return s * a; }
__device__ __forceinline__ Z scale_(double s, Z a) { return Z{s * a.re, s * a.im}; }
__device__ __forceinline__ double add_(double a, double b) { return a + b; }
__device__ __forceinline__ Z add_(Z a, Z b) { return Z{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ double sub_(double a, double b) { return a - b; }
__device__ __forceinline__ Z sub_(Z a, Z b) { return Z{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ double mul_(double a, double b) { return a * b; }
__device__ __forceinline__ Z mul_(Z a, Z b) { return Z{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
template <typename T>
__device__ __forceinline__ T zero_();
template <>
__device__ __forceinline__ double zero_<double>() { return 0.0; }
template <>
__device__ __forceinline__ Z zero_<Z>() { return Z{0.0, 0.0}; }
template <typename T>
__device__ __forceinline__ T one_();
template <>
__device__ __forceinline__ double one_<double>() { return 1.0; }
template <>
__device__ __forceinline__ Z one_<Z>() { return Z{1.0, 0.0}; }
__device__ __forceinline__ double from_real_(double v, double) { return v; }
__device__ __forceinline__ Z from_real_(double v, Z) { return Z{v, 0.0}; }
__device__ __forceinline__ double real_(double a) { return a; }
__device__ __forceinline__ double real_(Z a) { return a.re; }
__device__ __forceinline__ double abs2_(double a) { return a * a; }
__device__ __forceinline__ double abs2_(Z a) { return a.re * a.re + a.im * a.im; }

constexpr int TB = 64;   // output tile edge
constexpr int KB = 32;   // K rows staged per step
constexpr int THR = 256; // 16 x 16 threads, 4 x 4 outputs each

// Partial Gram tiles: part[c][i + j*m] = sum over rows k of chunk c of
// conj(A[k + i*lda]) B[k + j*ldb].  grid = (chunks, tiles over m, tiles over n).
template <typename T>
__global__ void __launch_bounds__(THR) k_gram_partial(int64_t K, int m, int n, const T* __restrict__ A,
                                                      int64_t lda, const T* __restrict__ B, int64_t ldb,
                                                      T* __restrict__ part, int64_t kc) {
  __shared__ T As[KB][TB + 1], Bs[KB][TB + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t k0 = (int64_t)blockIdx.x * kc, k1 = min(K, k0 + kc);
  const int i0 = blockIdx.y * TB, j0 = blockIdx.z * TB;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = zero_<T>();
  // rows ks .. ks+KB-1 of the block's 64 columns of A and B, loaded into
  // registers one step ahead of the LDS tile being consumed
  constexpr int EPT = TB * KB / THR;
  T ra[EPT], rb[EPT];
  auto fetch = [&](int64_t ks) {
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
      const int e = tid + r * THR, kk = e % KB, c = e / KB;
      const int64_t k = ks + kk;
      ra[r] = (k < k1 && i0 + c < m) ? A[k + (int64_t)(i0 + c) * lda] : zero_<T>();
      rb[r] = (k < k1 && j0 + c < n) ? B[k + (int64_t)(j0 + c) * ldb] : zero_<T>();
    }
  };
  fetch(k0);
  for (int64_t ks = k0; ks < k1; ks += KB) {
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
      const int e = tid + r * THR, kk = e % KB, c = e / KB;
      As[kk][c] = ra[r];
      Bs[kk][c] = rb[r];
    }
    __syncthreads();
    if (ks + KB < k1) fetch(ks + KB);
#pragma unroll 4
    for (int kk = 0; kk < KB; ++kk) {
      T av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = conj_(As[kk][tx + 16 * a]);
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma_(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  T* out = part + (int64_t)blockIdx.x * m * n;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = i0 + tx + 16 * a, j = j0 + ty + 16 * b;
      if (i < m && j < n) out[i + (int64_t)j * m] = acc[a][b];
    }
}

// C[i + j*m] = alpha * sum_c part[c][i + j*m], chunks summed in order.
template <typename T>
__global__ void k_gram_reduce(int chunks, int m, int n, const T* __restrict__ part, double alpha,
                              T* __restrict__ C) {
  const int64_t mn = (int64_t)m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < mn; e += (int64_t)gridDim.x * blockDim.x) {
    T s = zero_<T>();
    for (int c = 0; c < chunks; ++c) s = add_(s, part[c * mn + e]);
    C[e] = scale_(alpha, s);
  }
}

// In-place lower Cholesky factor of the Hermitian positive definite n x n
// matrix S (column-major, ld n): S = L L^H, L overwrites the lower triangle.
// One workgroup; *info = 0, or j+1 if the j-th pivot is not positive (then
// the factor is incomplete).  Left-looking: column j needs columns < j.
template <typename T>
__global__ void __launch_bounds__(1024) k_potrf_lower(int n, T* S, int* info) {
  __shared__ double red[32];
  __shared__ int bad;
  const int tid = threadIdx.x, nthr = blockDim.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    // pivot: d = S[j][j] - sum_k |L[j][k]|^2, fixed-order reduction
    double part = 0.0;
    for (int k = tid; k < j; k += nthr) part += abs2_(S[j + (int64_t)k * n]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = part;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < (nthr + 63) / 64; ++w) s += red[w];
      const double d = real_(S[j + (int64_t)j * n]) - s;
      if (!(d > 0.0)) {
        bad = j + 1;
      } else {
        S[j + (int64_t)j * n] = from_real_(sqrt(d), zero_<T>());
      }
    }
    __syncthreads();
    if (bad) break;
    const double inv = 1.0 / real_(S[j + (int64_t)j * n]);
    for (int i = j + 1 + tid; i < n; i += nthr) {
      T s = S[i + (int64_t)j * n];
      for (int k = 0; k < j; ++k) s = sub_(s, mul_(S[i + (int64_t)k * n], conj_(S[j + (int64_t)k * n])));
      S[i + (int64_t)j * n] = scale_(inv, s);
    }
    __syncthreads();
  }
  if (tid == 0) *info = bad;
}

// The same two factorizations with the working matrix in LDS (n <= NMAX):
// the serial chains of the column steps then run on LDS latency instead of
// global-memory latency.
template <typename T, int NMAX>
__global__ void __launch_bounds__(1024) k_potrf_lower_lds(int n, T* S, int* info) {
  __shared__ T A[NMAX * NMAX];
  __shared__ double red[32];
  __shared__ int bad;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int e = tid; e < n * n; e += nthr) A[e] = S[e];
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double part = 0.0;
    for (int k = tid; k < j; k += nthr) part += abs2_(A[j + k * n]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = part;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int w = 0; w < (nthr + 63) / 64; ++w) sum += red[w];
      const double d = real_(A[j + j * n]) - sum;
      if (!(d > 0.0)) bad = j + 1;
      else A[j + j * n] = from_real_(sqrt(d), zero_<T>());
    }
    __syncthreads();
    if (bad) break;
    const double inv = 1.0 / real_(A[j + j * n]);
    for (int i = j + 1 + tid; i < n; i += nthr) {
      T sum = A[i + j * n];
      for (int k = 0; k < j; ++k) sum = sub_(sum, mul_(A[i + k * n], conj_(A[j + k * n])));
      A[i + j * n] = scale_(inv, sum);
    }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += nthr) S[e] = A[e];
  if (tid == 0) *info = bad;
}

// U = L^{-H} with X = L^{-1} in LDS (row-major, so the threads of a row read
// consecutive words): rows of X in order, the columns of a row in parallel (thread j: X[i][j] = (delta_ij - sum_{j<=k<i} L[i][k] X[k][j]) / L[i][i]).
template <typename T, int NMAX>
__global__ void __launch_bounds__(1024) k_trtri_lower_ch_lds(int n, const T* L, T* U, const int* info) {
  if (*info) return;
  __shared__ T X[NMAX * NMAX];
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int i = 0; i < n; ++i) {
    const double inv = 1.0 / real_(L[i + (int64_t)i * n]);
    for (int j = tid; j <= i; j += nthr) {
      T sum = (i == j) ? one_<T>() : zero_<T>();
      for (int k = j; k < i; ++k) sum = sub_(sum, mul_(L[i + (int64_t)k * n], X[k * n + j]));
      X[i * n + j] = scale_(inv, sum);
    }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += nthr) {
    const int i = e % n, j = e / n;  // U[i][j] = conj(X[j][i]) for j >= i
    U[e] = (j >= i) ? conj_(X[j * n + i]) : zero_<T>();
  }
}

// U = L^{-H} (upper triangular, column-major, ld n) from the lower factor L
// (ld n).  Thread j solves L x = e_j for column j of X = L^{-1} and writes
// row j of U = X^H.  Skipped when *info != 0.
template <typename T>
__global__ void __launch_bounds__(1024) k_trtri_lower_ch(int n, const T* L, T* U, T* X, const int* info) {
  if (*info) return;
  const int j = threadIdx.x;
  if (j >= n) return;
  for (int i = 0; i < j; ++i) {
    X[i + (int64_t)j * n] = zero_<T>();
    U[j + (int64_t)i * n] = zero_<T>();
  }
  for (int i = j; i < n; ++i) {
    T s = (i == j) ? one_<T>() : zero_<T>();
    for (int k = j; k < i; ++k) s = sub_(s, mul_(L[i + (int64_t)k * n], X[k + (int64_t)j * n]));
    const T x = scale_(1.0 / real_(L[i + (int64_t)i * n]), s);
    X[i + (int64_t)j * n] = x;
    U[j + (int64_t)i * n] = conj_(x);
  }
}

// C(K x n) = beta * C + alpha * A(K x m) B(m x n); B small (ld m).
// grid = (row tiles of 64, column tiles of 64); skipped when info && *info.
template <typename T>
__global__ void __launch_bounds__(THR) k_tsmm(int64_t K, int m, int n, const T* __restrict__ A, int64_t lda,
                                              const T* __restrict__ B, double alpha, double beta, T* C,
                                              int64_t ldc, const int* info) {
  if (info && *info) return;
  __shared__ T As[KB][TB + 1], Bs[KB][TB + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t k0 = (int64_t)blockIdx.x * TB;
  const int j0 = blockIdx.y * TB;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = zero_<T>();
  for (int i0 = 0; i0 < m; i0 += KB) {
    // As[ii][r] = A[k0 + r, i0 + ii] (rows contiguous); Bs[ii][c] = B[i0 + ii, j0 + c]
#pragma unroll
    for (int r = 0; r < TB * KB / THR; ++r) {
      const int e = tid + r * THR;
      {
        const int rr = e % TB, ii = e / TB;
        const int64_t k = k0 + rr;
        As[ii][rr] = (k < K && i0 + ii < m) ? A[k + (int64_t)(i0 + ii) * lda] : zero_<T>();
      }
      {
        const int ii = e % KB, c = e / KB;
        Bs[ii][c] = (i0 + ii < m && j0 + c < n) ? B[(i0 + ii) + (int64_t)(j0 + c) * m] : zero_<T>();
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int ii = 0; ii < KB; ++ii) {
      T av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[ii][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[ii][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma_(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t k = k0 + tx + 16 * a;
      const int j = j0 + ty + 16 * b;
      if (k < K && j < n) {
        T* c = C + k + (int64_t)j * ldc;
        *c = (beta == 0.0) ? scale_(alpha, acc[a][b]) : add_(scale_(beta, *c), scale_(alpha, acc[a][b]));
      }
    }
}

template <typename T>
hipError_t gram(int64_t K, int m, int n, const void* A, int64_t lda, const void* B, int64_t ldb, double alpha,
                void* part, int64_t kc, void* C, hipStream_t s) {
  if (K <= 0 || m <= 0 || n <= 0) return hipSuccess;
  const int chunks = (int)((K + kc - 1) / kc);
  dim3 grid(chunks, (m + TB - 1) / TB, (n + TB - 1) / TB);
  hipLaunchKernelGGL(k_gram_partial<T>, grid, dim3(THR), 0, s, K, m, n, (const T*)A, lda, (const T*)B, ldb,
                     (T*)part, kc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t mn = (int64_t)m * n;
  const int blocks = (int)std::min<int64_t>((mn + 255) / 256, 4096);
  hipLaunchKernelGGL(k_gram_reduce<T>, dim3(blocks), dim3(256), 0, s, chunks, m, n, (const T*)part, alpha, (T*)C);
  return hipGetLastError();
}

}  // namespace

// Launchers (declared in launch.h).  cplx selects complex128.
hipError_t launch_ace_gram(bool cplx, int64_t K, int m, int n, const void* A, int64_t lda, const void* B,
                           int64_t ldb, double alpha, void* part, int64_t kc, void* C, hipStream_t s) {
  return cplx ? gram<Z>(K, m, n, A, lda, B, ldb, alpha, part, kc, C, s)
              : gram<double>(K, m, n, A, lda, B, ldb, alpha, part, kc, C, s);
}

// LDS-resident factorization up to these orders (128 KiB of LDS)
constexpr int kLdsNReal = 128, kLdsNCplx = 90;

hipError_t launch_ace_potrf(bool cplx, int n, void* S, int* info, hipStream_t s) {
  const int th = std::min(1024, std::max(64, (n + 63) / 64 * 64));
  if (cplx) {
    if (n <= kLdsNCplx) hipLaunchKernelGGL((k_potrf_lower_lds<Z, kLdsNCplx>), dim3(1), dim3(th), 0, s, n, (Z*)S, info);
    else hipLaunchKernelGGL(k_potrf_lower<Z>, dim3(1), dim3(th), 0, s, n, (Z*)S, info);
  } else {
    if (n <= kLdsNReal)
      hipLaunchKernelGGL((k_potrf_lower_lds<double, kLdsNReal>), dim3(1), dim3(th), 0, s, n, (double*)S, info);
    else hipLaunchKernelGGL(k_potrf_lower<double>, dim3(1), dim3(th), 0, s, n, (double*)S, info);
  }
  return hipGetLastError();
}

hipError_t launch_ace_trtri(bool cplx, int n, const void* L, void* U, void* X, const int* info, hipStream_t s) {
  const int th = std::min(1024, std::max(64, (n + 63) / 64 * 64));
  if (cplx) {
    if (n <= kLdsNCplx)
      hipLaunchKernelGGL((k_trtri_lower_ch_lds<Z, kLdsNCplx>), dim3(1), dim3(th), 0, s, n, (const Z*)L, (Z*)U, info);
    else hipLaunchKernelGGL(k_trtri_lower_ch<Z>, dim3(1), dim3(th), 0, s, n, (const Z*)L, (Z*)U, (Z*)X, info);
  } else {
    if (n <= kLdsNReal)
      hipLaunchKernelGGL((k_trtri_lower_ch_lds<double, kLdsNReal>), dim3(1), dim3(th), 0, s, n, (const double*)L,
                         (double*)U, info);
    else
      hipLaunchKernelGGL(k_trtri_lower_ch<double>, dim3(1), dim3(th), 0, s, n, (const double*)L, (double*)U,
                         (double*)X, info);
  }
  return hipGetLastError();
}

hipError_t launch_ace_tsmm(bool cplx, int64_t K, int m, int n, const void* A, int64_t lda, const void* B,
                           double alpha, double beta, void* C, int64_t ldc, const int* info, hipStream_t s) {
  if (K <= 0 || n <= 0) return hipSuccess;
  dim3 grid((unsigned)((K + TB - 1) / TB), (n + TB - 1) / TB);
  if (cplx)
    hipLaunchKernelGGL(k_tsmm<Z>, grid, dim3(THR), 0, s, K, m, n, (const Z*)A, lda, (const Z*)B, alpha, beta,
                       (Z*)C, ldc, info);
  else
    hipLaunchKernelGGL(k_tsmm<double>, grid, dim3(THR), 0, s, K, m, n, (const double*)A, lda,
                       (const double*)B, alpha, beta, (double*)C, ldc, info);
  return hipGetLastError();
}

}  // namespace kx
