// Adaptively compressed exchange (ACE) on one GPU, FP64 real and complex128.
//
// Construction (Sec. III.A): M = dV Psi^H W, -M = L L^H (lower Cholesky
// factor), xi = W L^{-H}.  Application (Sec. III.B): chi = dV xi^H Phi, then
// V Phi -= xi chi.  All orbital sets are column-major N x n (one orbital per
// column, leading dimension ld >= N); the small matrices are column-major with
// leading dimension equal to their row count.
//
// The two products with the long dimension N are FP64 contractions of 2 n^2
// flops per grid point against 16 n bytes, so for n_s of order 100 they are
// bound by the FP64 matrix units rather than HBM; both run on MFMA:
//   gram:  C(m x n) = alpha * sum_k conj(A[k, i]) B[k, j], split over K in
//          chunks whose partial tiles are summed in a fixed order (bitwise
//          reproducible results);
//   tsmm:  C(K x n) = beta * C + alpha * A(K x m) B(m x n).
// The Cholesky factorization and the triangular inverse of the n_s x n_s
// matrix run in one workgroup with the matrix in registers (n_s <= 128), or
// tile by tile (128-tiles, small GEMM updates) for larger n_s.
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

// ---------------------------------------------------------------------------
// MFMA forms (v_mfma_f64_16x16x4).  Operand layout, lane l = 16*lg + lr:
// A fragment A[row = lr][k = lg], B fragment B[k = lg][col = lr], accumulator
// element r at D[row = lg + 4*r][col = lr].
//
// Complex operands are read as doubles (re, im interleaved), so that a complex
// product becomes two real contractions over twice the length:
//   Re(conj(a) b) = ar br + ai bi     = sum_q a_q b_q
//   Im(conj(a) b) = ar bi - ai br     = sum_q a_q bt_q,  bt_{2c} = b_{2c+1}, bt_{2c+1} = -b_{2c}
// and for the tall-skinny product C = A B (no conjugate):
//   Re(a b) = ar br - ai bi = sum_q a_q x_q,   x_{2c} = br, x_{2c+1} = -bi
//   Im(a b) = ar bi + ai br = sum_q a_q xt_q,  xt_{2c} = bi, xt_{2c+1} = br
// ---------------------------------------------------------------------------
typedef double d4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ d4_t mfma64(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int GKB = 32;           // rows (doubles) of A and B staged per step
constexpr int GP = GKB + 2;       // LDS pitch (2 mod 32): conflict-free fragment reads
constexpr int GBLOCKS = 512;      // Gram blocks to aim for: two per CU
constexpr int GTILE = 128 * 128;  // doubles of one output tile's partial

// Partial Gram tiles, split over K (in doubles: K2 = K or 2K).  A block of
// four waves owns one output tile (128 x 128 real, 128 x 64 complex with
// separate Re / Im accumulators) and one chunk of rows; wave w computes a
// 64-row x (64 | 32)-column quadrant.  Partials are stored in accumulator
// order (every store is a contiguous 512-byte wave line); k_gram_mfma_reduce
// maps them back to (i, j).
template <bool CPLX>
__global__ void __launch_bounds__(256, 2) k_gram_mfma(int64_t K2, int m, int n, const double* __restrict__ A,
                                                   int64_t lda2, const double* __restrict__ B, int64_t ldb2,
                                                   double* __restrict__ part, int64_t kc2) {
  constexpr int BN = CPLX ? 64 : 128, WN = BN / 2, NTJ = WN / 16, SETS = CPLX ? 2 : 1;
  constexpr int LA = 128 * GKB / 256, LB = BN * GKB / 256;
  __shared__ double As[128 * GP], Bs[BN * GP];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, lr = lane & 15, lg = lane >> 4;
  const int wm = w & 1, wn = w >> 1;
  const int64_t k0 = (int64_t)blockIdx.x * kc2, k1 = min(K2, k0 + kc2);
  const int i0 = blockIdx.y * 128, j0 = blockIdx.z * BN;
  d4_t acc[SETS][4][NTJ];
#pragma unroll
  for (int st = 0; st < SETS; ++st)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < NTJ; ++b) acc[st][a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
  // Each slab is loaded when it is needed (the other block on the CU keeps
  // the matrix units busy meanwhile; a register prefetch would not fit two
  // blocks' worth of registers), 16 elements per operand at a time.  Loads
  // are unconditional, with row and column indices clamped into the
  // matrices; rows past the chunk and columns past m / n are zeroed on the
  // way to LDS.
  auto stage = [&](const double* __restrict__ M, int64_t ldm, int c0, int cmax, double* S, int cnt,
                   int64_t ks) {
#pragma unroll 1
    for (int r0 = 0; r0 < cnt; r0 += 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * (r0 + u), c = min(c0 + e / GKB, cmax - 1);
        const int64_t k = min(ks + e % GKB, K2 - 1);
        if (r0 + u < cnt) v[u] = M[k + (int64_t)c * ldm];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * (r0 + u);
        const bool ok = ks + e % GKB < k1 && c0 + e / GKB < cmax;
        if (r0 + u < cnt) S[(e / GKB) * GP + e % GKB] = ok ? v[u] : 0.0;
      }
    }
  };
  for (int64_t ks = k0; ks < k1; ks += GKB) {
    stage(A, lda2, i0, m, As, LA, ks);
    stage(B, ldb2, j0, n, Bs, LB, ks);
    __syncthreads();
#pragma unroll
    for (int s4 = 0; s4 < GKB / 4; ++s4) {
      const int kk = 4 * s4 + lg;
      double av[4], bv[NTJ], bt[NTJ];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[(wm * 64 + 16 * a + lr) * GP + kk];
#pragma unroll
      for (int b = 0; b < NTJ; ++b) {
        const double* col = Bs + (wn * WN + 16 * b + lr) * GP;
        bv[b] = col[kk];
        if (CPLX) bt[b] = (lg & 1) ? -col[kk - 1] : col[kk + 1];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NTJ; ++b) {
          acc[0][a][b] = mfma64(av[a], bv[b], acc[0][a][b]);
          if (CPLX) acc[SETS - 1][a][b] = mfma64(av[a], bt[b], acc[SETS - 1][a][b]);
        }
    }
    __syncthreads();
  }
  // partial of this chunk and tile, in accumulator order
  const int64_t tile = (int64_t)blockIdx.y * gridDim.z + blockIdx.z;
  double* out = part + ((int64_t)blockIdx.x * gridDim.y * gridDim.z + tile) * GTILE;
#pragma unroll
  for (int st = 0; st < SETS; ++st)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < NTJ; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          out[((((w * SETS + st) * 4 + a) * NTJ + b) * 4 + r) * 64 + lane] = acc[st][a][b][r];
}

// C[i + j*m] = alpha * sum_c partial_c(i, j), the chunks summed in a fixed
// order: block = 64 consecutive partial entries x 4 waves; wave g sums chunks
// g, g+4, ... and the four sums are added in wave order.
template <bool CPLX>
__global__ void __launch_bounds__(256) k_gram_mfma_reduce(int chunks, int tiles_n, int64_t per_chunk, int m,
                                                          int n, const double* __restrict__ part, double alpha,
                                                          double* __restrict__ C) {
  constexpr int BN = CPLX ? 64 : 128, WN = BN / 2, NTJ = WN / 16, SETS = CPLX ? 2 : 1;
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  double s = 0.0;
#pragma unroll 8
  for (int c = g; c < chunks; c += 4) s += part[(int64_t)c * per_chunk + e];
  red[g][lane] = s;
  __syncthreads();
  if (g != 0) return;
  s = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
  // decode (tile, w, set, a, b, r, lane) of the accumulator-order index
  const int64_t tile = e / GTILE;
  int q = (int)(e % GTILE);
  const int l = q & 63;
  q >>= 6;
  const int r = q & 3;
  q >>= 2;
  const int b = q % NTJ;
  q /= NTJ;
  const int a = q & 3;
  q >>= 2;
  const int st = q % SETS, w = q / SETS;
  const int i = (int)(tile / tiles_n) * 128 + (w & 1) * 64 + 16 * a + (l >> 4) + 4 * r;
  const int j = (int)(tile % tiles_n) * BN + (w >> 1) * WN + 16 * b + (l & 15);
  if (i < m && j < n) C[(i + (int64_t)j * m) * SETS + st] = alpha * s;
}

// C(K x n) = beta C + alpha A(K x m) B(m x n) for m <= 128, computed as
// C^T = B^T A^T so that each accumulator row is a run of 16 consecutive rows
// of C (whole cache lines per store).  B (its n-tile of 128 real / 64 complex
// columns) stays in LDS for the whole launch; A is read straight from global
// memory into fragment registers, one group of 8 steps ahead.  Each wave owns
// 32-row tiles of C, taken in a grid stride.  Skipped when info && *info.
constexpr int TQ = 258;     // LDS pitch (doubles) of the B tile: 2 mod 32
constexpr int TS_TT = 1;     // 16-row accumulator tiles per wave tile
constexpr int TS_WPB = 8;    // waves per block: two per SIMD beside the LDS-resident B
template <bool CPLX>
__global__ void __launch_bounds__(64 * TS_WPB) k_tsmm_mfma(int64_t K, int m, int n, const double* __restrict__ A,
                                                   int64_t lda, const double* __restrict__ B, int ldb,
                                                   double alpha, double beta, double* C, int64_t ldc,
                                                   const int* info) {
  if (info && *info) return;
  constexpr int NJ = CPLX ? 64 : 128, NTJ = 4, SETS = CPLX ? 2 : 1, G = 4;
  constexpr int PITCH = CPLX ? TQ : 130;
  __shared__ double Xs[NJ * PITCH];
  const int tid = threadIdx.x, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int Q = CPLX ? 2 * m : m;  // contraction length in doubles
  const int QS = (Q + 3) / 4;      // 4-deep steps (the last group may run past QS)
  const int j0 = blockIdx.y * NJ;
  // X[j][q] = B as doubles: column j of B is contiguous in q
  for (int e = tid; e < NJ * PITCH; e += 64 * TS_WPB) {
    const int j = e / PITCH, q = e % PITCH;
    Xs[e] = (q < Q && j0 + j < n) ? B[q + (int64_t)(j0 + j) * (CPLX ? 2 * ldb : ldb)] : 0.0;
  }
  __syncthreads();
  constexpr int ROWS = 16 * TS_TT;  // rows of C per wave tile
  const int tiles = (int)((K + ROWS - 1) / ROWS);
  const int wstride = gridDim.x * TS_WPB;
  // real: the wave covers all 128 columns in 8 tiles, one set; complex: 64
  // columns in 4 tiles, two sets (Re, Im)
  constexpr int TJ = CPLX ? 4 : 8;
  d4_t acc[SETS][TJ][TS_TT];
  double y[TS_TT][G], yn[TS_TT][G];
  const int ngroups = (QS + G - 1) / G;
  // Unconditional loads with clamped indices, so that no branch separates
  // them from the MFMA loop: rows past K produce results that are not stored,
  // contraction indices past Q meet zero rows of X.
  auto load = [&](double (&dst)[TS_TT][G], int tile, int grp) {
#pragma unroll
    for (int t = 0; t < TS_TT; ++t) {
      const int64_t k = min((int64_t)tile * ROWS + 16 * t + lr, K - 1);
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int q = 4 * (grp * G + u) + lg;
        if (CPLX) {
          // q = 2c + p: A[k, c] part p
          const int c = min(q >> 1, m - 1);
          dst[t][u] = A[2 * (k + (int64_t)c * lda) + (q & 1)];
        } else {
          const int c = min(q, m - 1);
          dst[t][u] = A[k + (int64_t)c * lda];
        }
      }
    }
  };
  int tile = blockIdx.x * TS_WPB + w;
  if (tile >= tiles) return;
  load(y, tile, 0);
  for (;;) {
#pragma unroll
    for (int st = 0; st < SETS; ++st)
#pragma unroll
      for (int a = 0; a < TJ; ++a)
#pragma unroll
        for (int t = 0; t < TS_TT; ++t) acc[st][a][t] = d4_t{0.0, 0.0, 0.0, 0.0};
    for (int grp = 0; grp < ngroups; ++grp) {
      // prefetch the next group of this wave's sequence (past the last tile:
      // a clamped, harmless reload of the last one)
      const bool last = grp + 1 == ngroups;
      load(yn, last ? min(tile + wstride, tiles - 1) : tile, last ? 0 : grp + 1);
      // steps past QS read zero rows of X (staged up to the padded pitch)
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int q = 4 * (grp * G + u) + lg;
        double x0[TJ], x1[TJ];
#pragma unroll
        for (int a = 0; a < TJ; ++a) {
          const double* row = Xs + (16 * a + lr) * PITCH;
          if (CPLX) {
            const double ev = row[q & ~1], od = row[q | 1];
            x0[a] = (lg & 1) ? -od : ev;  // Re: (br, -bi)
            x1[a] = (lg & 1) ? ev : od;   // Im: (bi, br)
          } else {
            x0[a] = row[q];
          }
        }
#pragma unroll
        for (int a = 0; a < TJ; ++a)
#pragma unroll
          for (int t = 0; t < TS_TT; ++t) {
            acc[0][a][t] = mfma64(x0[a], y[t][u], acc[0][a][t]);
            if (CPLX) acc[SETS - 1][a][t] = mfma64(x1[a], y[t][u], acc[SETS - 1][a][t]);
          }
      }
#pragma unroll
      for (int t = 0; t < TS_TT; ++t)
#pragma unroll
        for (int u = 0; u < G; ++u) y[t][u] = yn[t][u];
    }
    // tile done: D[j][k], j = j0 + 16a + lg + 4r, k = ROWS tile + 16t + lr.
    // With beta != 0 the old values of C are loaded for two j-tiles at a
    // time before any of them is stored (a load after a store to C cannot
    // be hoisted by the compiler, which would serialize every update).
#pragma unroll
    for (int a0 = 0; a0 < TJ; a0 += 2) {
      double old[2][TS_TT][4][SETS];
      if (beta != 0.0) {
#pragma unroll
        for (int da = 0; da < 2; ++da)
#pragma unroll
          for (int t = 0; t < TS_TT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int j = min(j0 + 16 * (a0 + da) + lg + 4 * r, n - 1);
              const int64_t k = min((int64_t)tile * ROWS + 16 * t + lr, K - 1);
#pragma unroll
              for (int st = 0; st < SETS; ++st) old[da][t][r][st] = C[(k + (int64_t)j * ldc) * SETS + st];
            }
      }
#pragma unroll
      for (int da = 0; da < 2; ++da)
#pragma unroll
        for (int t = 0; t < TS_TT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j = j0 + 16 * (a0 + da) + lg + 4 * r;
            const int64_t k = (int64_t)tile * ROWS + 16 * t + lr;
            if (k < K && j < n) {
#pragma unroll
              for (int st = 0; st < SETS; ++st) {
                double v = alpha * acc[st][a0 + da][t][r];
                if (beta != 0.0) v += beta * old[da][t][r][st];
                C[(k + (int64_t)j * ldc) * SETS + st] = v;
              }
            }
          }
    }
    tile += wstride;
    if (tile >= tiles) break;
  }
}

// Cholesky factor and triangular inverse of the n x n Hermitian matrix S
// (n <= 128) in one workgroup of 1024 threads, the matrix held in registers:
// thread (row = tid % 128, grp = tid / 128) keeps the 16 elements of row
// `row` in columns grp, grp + 8, ..., grp + 120.  Each column step publishes
// one column through a small LDS vector (double-buffered, so one barrier per
// factorization step); the matrix itself never goes through LDS.
//
// Factorization, right-looking without square roots inside the loop: step j
// subtracts A_ij conj(A_kj) / A_jj from the trailing triangle (j < k <= i),
// taken in panels of 8 columns (within a panel by one wave, then one rank-8
// update of the later columns); afterwards l_ij = A_ij / sqrt(A_jj),
// l_jj = sqrt(A_jj).
// Inverse, in place, columns right to left (X_22 = inverse of the trailing
// block, already in place):
//   x_jj = 1/l_jj,  x_(j+1:, j) = -X_22 l_(j+1:, j) / l_jj,
// the products split over the 8 groups and summed in group order.
// Writes U = L^{-H} = X^H (upper, zeros below, ld ldu) and *info: j+1+base at
// the first non-positive pivot (U then left untouched); on success *info is
// set to 0 when base == 0 and left alone otherwise.  With base > 0 (a
// diagonal tile of a larger matrix) the kernel does nothing if *info != 0.
template <typename T>
__global__ void __launch_bounds__(1024) k_chol_inv_reg(int n, const T* __restrict__ S, int lds, T* __restrict__ U,
                                                       int ldu, int* info, int base) {
  if (base > 0 && *info) return;
  constexpr int KT = 16;
  constexpr int RHD = sizeof(T) > 8 ? 4 : 8;
  __shared__ T pan[2][128][9];      // panel of 8 columns (pitch 9)
  __shared__ T red2[8][128][RHD];   // per-group partial sums of the inverse
  __shared__ T tl[128][8];          // T = Y22 L21 (and the pivots)
  __shared__ T y11[8][8];           // inverse of the diagonal 8 x 8 block
  __shared__ double pan_inv[2][8];  // 1 / pivot of the panel's columns
  __shared__ int pan_bad;
  const int tid = threadIdx.x, i = tid & 127, grp = tid >> 7;
  if (tid == 0) pan_bad = 0;
  const bool live = i < n;
  T a[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int k = grp + 8 * t;
    a[t] = zero_<T>();
    if (live && k < n) a[t] = S[i + (int64_t)k * lds];
  }
  // Slot t holds column block (t + R) mod 16 (column j = 8 * block + grp).
  // The block being eliminated is kept in slot 0 by rotating the slots once
  // per block, so that every slot index is a compile-time constant (a runtime
  // index would move `a` to scratch memory).
  auto rot_left = [&]() {  // R += 1
    const T f = a[0];
#pragma unroll
    for (int t = 0; t < KT - 1; ++t) a[t] = a[t + 1];
    a[KT - 1] = f;
  };
  auto rot_right = [&]() {  // R -= 1
    const T l = a[KT - 1];
#pragma unroll
    for (int t = KT - 1; t > 0; --t) a[t] = a[t - 1];
    a[0] = l;
  };
  const int nblk = (n + 7) / 8;
  int buf = 0;
  // Factorization in panels of 8 columns (block jb in slot 0):
  //  (1) the rows >= 8 jb publish the panel to LDS;
  //  (2) wave 0 eliminates within the panel (8 column steps, two rows per
  //      lane, no barrier: one wave's LDS accesses stay in program order);
  //  (3) every thread takes its factored panel value back and applies the
  //      panel's 8 rank-1 updates to its later columns at once.
  for (int jb = 0; jb < nblk; ++jb) {  // R = jb here
    if (live && i >= 8 * jb) pan[buf][i][grp] = a[0];
    __syncthreads();
    if (tid < 64) {
      for (int jr = 0; jr < 8; ++jr) {
        const int j = 8 * jb + jr;
        if (j >= n) break;
        const double d = real_(pan[buf][j][jr]);
        if (!(d > 0.0)) {  // the same value in every lane: uniform
          if (tid == 0) pan_bad = j + 1;
          break;
        }
        const double inv = 1.0 / d;
        if (tid == 0) pan_inv[buf][jr] = inv;
        // rows 8 jb + lane and 8 jb + lane + 64
        if constexpr (sizeof(T) == 8) {
          // real: all operands loaded before the updates (one LDS round trip
          // per step)
          T lr[2], prow[2][8], pcol[8];
#pragma unroll
          for (int c = 0; c < 8; ++c)
            if (c > jr) pcol[c] = pan[buf][j - jr + c][jr];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int r = min(j - jr + tid + 64 * h, 127);
            lr[h] = scale_(inv, pan[buf][r][jr]);
#pragma unroll
            for (int c = 0; c < 8; ++c)
              if (c > jr) prow[h][c] = pan[buf][r][c];
          }
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int r = j - jr + tid + 64 * h;
            if (r > j && r < n) {
#pragma unroll
              for (int c = 0; c < 8; ++c)
                if (c > jr) pan[buf][r][c] = sub_(prow[h][c], mul_(lr[h], conj_(pcol[c])));
            }
          }
        } else {  // complex: row by row (register budget)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int r = j - jr + tid + 64 * h;
            if (r > j && r < n) {
              const T lr = scale_(inv, pan[buf][r][jr]);
              for (int c = jr + 1; c < 8; ++c)
                pan[buf][r][c] = sub_(pan[buf][r][c], mul_(lr, conj_(pan[buf][j - jr + c][jr])));
            }
          }
        }
      }
    }
    __syncthreads();
    if (pan_bad) {
      if (tid == 0) *info = pan_bad + base;
      return;
    }
    if (live && i >= 8 * jb) a[0] = pan[buf][i][grp];
    if (live && i >= 8 * (jb + 1)) {
      // the panel's columns in two halves of four (register budget)
#pragma unroll
      for (int h = 0; h < 8; h += 4) {
        T li[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) li[r] = scale_(pan_inv[buf][h + r], pan[buf][i][h + r]);
#pragma unroll
        for (int t = 1; t < KT; ++t) {
          const int k = grp + 8 * (jb + t);
          if (t < nblk - jb && k <= i) {
            T v = a[t];
#pragma unroll
            for (int r = 0; r < 4; ++r) v = sub_(v, mul_(li[r], conj_(pan[buf][k][h + r])));
            a[t] = v;
          }
        }
      }
    }
    rot_left();
    buf ^= 1;
  }
  int R = nblk & (KT - 1);
  // l_ij = A_ij / sqrt(A_jj): publish the pivots, then scale
#pragma unroll
  for (int t = 0; t < KT; ++t)
    if (live && grp + 8 * ((t + R) & (KT - 1)) == i) tl[i][0] = a[t];
  __syncthreads();
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int k = grp + 8 * ((t + R) & (KT - 1));
    if (live && k <= i) {
      const double sd = sqrt(real_(tl[k][0]));
      if (k == i) a[t] = from_real_(sd, zero_<T>());
      else a[t] = scale_(1.0 / sd, a[t]);
    }
  }
  __syncthreads();
  // In-place inverse by panels of 8 columns, right to left (the current
  // panel in slot 0, Y22 = the inverse of the trailing block in slots >= 1):
  //   Y11 = L11^{-1} (one lane per column, from the published panel),
  //   T = Y22 L21 (partial sums per group, added in group order),
  //   Y21 = -T Y11.
  constexpr int RH = sizeof(T) > 8 ? 4 : 8;  // panel columns per partial-sum round
  for (int jb = nblk - 1; jb >= 0; --jb) {
    rot_right();  // R = jb
    const int j0 = 8 * jb;
    if (live && i >= j0) pan[buf][i][grp] = a[0];
    __syncthreads();
    if (tid < 8) {  // column c = tid of Y11, forward substitution
      const int c = tid;
      if constexpr (sizeof(T) == 8) {  // real: the column in registers
        T y[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          T v = zero_<T>();
          if (j0 + r < n && r >= c) {
            if (r == c) v = one_<T>();
#pragma unroll
            for (int q = 0; q < r; ++q)
              if (q >= c) v = sub_(v, mul_(pan[buf][j0 + r][q], y[q]));
            v = scale_(1.0 / real_(pan[buf][j0 + r][r]), v);
          }
          y[r] = v;
          y11[r][c] = v;
        }
      } else {  // complex: through LDS (register budget)
        for (int r = 0; r < 8; ++r) {
          T v = zero_<T>();
          if (j0 + r < n && r >= c) {
            if (r == c) v = one_<T>();
            for (int q = c; q < r; ++q) v = sub_(v, mul_(pan[buf][j0 + r][q], y11[q][c]));
            v = scale_(1.0 / real_(pan[buf][j0 + r][r]), v);
          }
          y11[r][c] = v;
        }
      }
    }
    for (int h = 0; h < 8; h += RH) {
      if (live && i >= j0 + 8) {
        T p[RH];
#pragma unroll
        for (int r = 0; r < RH; ++r) p[r] = zero_<T>();
#pragma unroll
        for (int t = 1; t < KT; ++t) {
          const int k = grp + 8 * (jb + t);
          if (t < nblk - jb && k <= i) {
#pragma unroll
            for (int r = 0; r < RH; ++r) p[r] = fma_(a[t], pan[buf][k][h + r], p[r]);
          }
        }
#pragma unroll
        for (int r = 0; r < RH; ++r) red2[grp][i][r] = p[r];
      }
      __syncthreads();
      if (live && i >= j0 + 8 && grp >= h && grp < h + RH) {
        T v = red2[0][i][grp - h];
#pragma unroll
        for (int g = 1; g < 8; ++g) v = add_(v, red2[g][i][grp - h]);
        tl[i][grp] = v;
      }
      __syncthreads();
    }
    if (live && i >= j0) {
      T v = zero_<T>();
      if (i < j0 + 8) {  // diagonal block: Y11
        if (grp <= i - j0) v = y11[i - j0][grp];
      } else {          // Y21 = -T Y11
#pragma unroll
        for (int r = 0; r < 8; ++r)
          if (r >= grp) v = sub_(v, mul_(tl[i][r], y11[r][grp]));
      }
      a[0] = v;
    }
    buf ^= 1;
  }
  R = 0;
  // U[k][i] = conj(X[i][k]) for k <= i, zero below the diagonal of U
  if (live) {
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const int k = grp + 8 * ((t + R) & (KT - 1));
      if (k < n) {
        if (k <= i) U[k + (int64_t)i * ldu] = conj_(a[t]);
        else U[k + (int64_t)i * ldu] = zero_<T>();
      }
    }
  }
  if (tid == 0 && base == 0) *info = 0;
}

// Small dense products for the tiled factorization (orders above 128):
// C(m x n) = beta C + alpha A(m x k) op(B), op(B) = B (k x n) or, with BH,
// B^H for B stored n x k; all column-major.  64 x 64 tile per block of 256
// threads (4 x 4 outputs each), 16-deep K steps through LDS.  Skipped when
// *info != 0.
template <typename T, bool BH>
__global__ void __launch_bounds__(256) k_small_gemm(int m, int n, int k, double alpha, const T* __restrict__ A,
                                                    int lda, const T* __restrict__ B, int ldb, double beta,
                                                    T* __restrict__ C, int ldc, const int* info) {
  if (*info) return;
  __shared__ T As[16][65], Bs[16][65];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = zero_<T>();
  for (int p0 = 0; p0 < k; p0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int r = e % 64, p = e / 64;  // A[i0 + r][p0 + p]
      As[p][r] = (i0 + r < m && p0 + p < k) ? A[(i0 + r) + (int64_t)(p0 + p) * lda] : zero_<T>();
      if (BH) {  // op(B)[p][c] = conj(B[c][p])
        const int c = e % 64, pp = e / 64;
        Bs[pp][c] = (j0 + c < n && p0 + pp < k) ? conj_(B[(j0 + c) + (int64_t)(p0 + pp) * ldb]) : zero_<T>();
      } else {
        const int pp = e % 16, c = e / 16;
        Bs[pp][c] = (j0 + c < n && p0 + pp < k) ? B[(p0 + pp) + (int64_t)(j0 + c) * ldb] : zero_<T>();
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int p = 0; p < 16; ++p) {
      T av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[p][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[p][ty + 16 * b];
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
      const int i = i0 + tx + 16 * a, j = j0 + ty + 16 * b;
      if (i < m && j < n) {
        T* c = C + i + (int64_t)j * ldc;
        const T v = scale_(alpha, acc[a][b]);
        *c = (beta == 0.0) ? v : add_(scale_(beta, *c), v);
      }
    }
}

// dst(m x n) = src^H for src n x m; with LOWER only the lower triangle of src
// is read (dst gets zeros below its diagonal).  Skipped when *info != 0.
template <typename T, bool LOWER>
__global__ void k_conj_transpose(int m, int n, const T* __restrict__ src, int lds, T* __restrict__ dst, int ldd,
                                 const int* info) {
  if (*info) return;
  const int64_t total = (int64_t)m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);  // dst[i][j] = conj(src[j][i])
    dst[i + (int64_t)j * ldd] = (!LOWER || j >= i) ? conj_(src[j + (int64_t)i * lds]) : zero_<T>();
  }
}

// Split-K chunk count of a Gram product: about two blocks per compute unit
// over all output tiles, chunks a multiple of GKB doubles long.
struct GramShape {
  int tiles_m, tiles_n, chunks;
  int64_t kc2;
};
GramShape gram_shape(bool cplx, int64_t K, int m, int n) {
  GramShape g;
  g.tiles_m = (m + 127) / 128;
  g.tiles_n = (n + (cplx ? 63 : 127)) / (cplx ? 64 : 128);
  const int64_t K2 = cplx ? 2 * K : K;
  const int64_t tiles = (int64_t)g.tiles_m * g.tiles_n;
  int64_t chunks = std::max<int64_t>(1, GBLOCKS / tiles);
  chunks = std::min<int64_t>(chunks, (K2 + GKB - 1) / GKB);
  g.kc2 = ((K2 + chunks - 1) / chunks + GKB - 1) / GKB * GKB;
  g.chunks = (int)((K2 + g.kc2 - 1) / g.kc2);
  return g;
}
}  // namespace

// Launchers (declared in launch.h).  cplx selects complex128.
int64_t ace_gram_part_bytes(bool cplx, int64_t K, int m, int n) {
  if (K <= 0 || m <= 0 || n <= 0) return 0;
  const GramShape g = gram_shape(cplx, K, m, n);
  return (int64_t)g.chunks * g.tiles_m * g.tiles_n * GTILE * (int64_t)sizeof(double);
}

hipError_t launch_ace_gram(bool cplx, int64_t K, int m, int n, const void* A, int64_t lda, const void* B,
                           int64_t ldb, double alpha, void* part, void* C, hipStream_t s) {
  if (K <= 0 || m <= 0 || n <= 0) return hipSuccess;
  const GramShape g = gram_shape(cplx, K, m, n);
  const int64_t K2 = cplx ? 2 * K : K, f = cplx ? 2 : 1;
  dim3 grid(g.chunks, g.tiles_m, g.tiles_n);
  if (cplx)
    hipLaunchKernelGGL(k_gram_mfma<true>, grid, dim3(256), 0, s, K2, m, n, (const double*)A, f * lda,
                       (const double*)B, f * ldb, (double*)part, g.kc2);
  else
    hipLaunchKernelGGL(k_gram_mfma<false>, grid, dim3(256), 0, s, K2, m, n, (const double*)A, f * lda,
                       (const double*)B, f * ldb, (double*)part, g.kc2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t per_chunk = (int64_t)g.tiles_m * g.tiles_n * GTILE;
  const int blocks = (int)(per_chunk / 64);
  if (cplx)
    hipLaunchKernelGGL(k_gram_mfma_reduce<true>, dim3(blocks), dim3(256), 0, s, g.chunks, g.tiles_n, per_chunk, m,
                       n, (const double*)part, alpha, (double*)C);
  else
    hipLaunchKernelGGL(k_gram_mfma_reduce<false>, dim3(blocks), dim3(256), 0, s, g.chunks, g.tiles_n, per_chunk,
                       m, n, (const double*)part, alpha, (double*)C);
  return hipGetLastError();
}

// Register-resident factorization and inverse of one tile of up to this order
constexpr int kRegN = 128;

namespace {
template <typename T>
hipError_t small_gemm(bool bh, int m, int n, int k, double alpha, const T* A, int lda, const T* B, int ldb,
                      double beta, T* C, int ldc, const int* info, hipStream_t s) {
  dim3 grid((m + 63) / 64, (n + 63) / 64);
  if (bh) hipLaunchKernelGGL((k_small_gemm<T, true>), grid, dim3(256), 0, s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, info);
  else hipLaunchKernelGGL((k_small_gemm<T, false>), grid, dim3(256), 0, s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, info);
  return hipGetLastError();
}

// Tiled Cholesky factor and inverse of the n x n Hermitian S (tiles of 128):
//   for each diagonal tile kb: U_kk = L_kk^{-H} (register kernel, into X);
//   panel L_ik = S_ik U_kk (into X); trailing S_ij -= L_ik L_jk^H.
//   Y = L^{-1} (into S): Y_jj = U_jj^H; Y_ij = -Y_ii (sum_{k=j}^{i-1} L_ik Y_kj)
//   with the sums in U as scratch; finally U = Y^H.
template <typename T>
hipError_t factor_tiled(int n, T* S, T* U, T* X, int* info, hipStream_t s) {
  const int nt = (n + kRegN - 1) / kRegN;
  auto off = [&](int ib, int jb) { return (int64_t)ib * kRegN + (int64_t)jb * kRegN * n; };
  auto sz = [&](int ib) { return std::min(kRegN, n - ib * kRegN); };
  hipError_t e = hipSuccess;
  for (int kb = 0; kb < nt && e == hipSuccess; ++kb) {
    hipLaunchKernelGGL(k_chol_inv_reg<T>, dim3(1), dim3(1024), 0, s, sz(kb), (const T*)(S + off(kb, kb)), n,
                       X + off(kb, kb), n, info, kb * kRegN);
    e = hipGetLastError();
    for (int ib = kb + 1; ib < nt && e == hipSuccess; ++ib)
      e = small_gemm<T>(false, sz(ib), sz(kb), sz(kb), 1.0, S + off(ib, kb), n, X + off(kb, kb), n, 0.0,
                        X + off(ib, kb), n, info, s);
    for (int jb = kb + 1; jb < nt && e == hipSuccess; ++jb)
      for (int ib = jb; ib < nt && e == hipSuccess; ++ib)
        e = small_gemm<T>(true, sz(ib), sz(jb), sz(kb), -1.0, X + off(ib, kb), n, X + off(jb, kb), n, 1.0,
                          S + off(ib, jb), n, info, s);
  }
  for (int jb = 0; jb < nt && e == hipSuccess; ++jb) {
    const int64_t tot = (int64_t)sz(jb) * sz(jb);
    hipLaunchKernelGGL((k_conj_transpose<T, false>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, sz(jb),
                       sz(jb), (const T*)(X + off(jb, jb)), n, S + off(jb, jb), n, (const int*)info);
    e = hipGetLastError();
  }
  for (int jb = 0; jb < nt && e == hipSuccess; ++jb)
    for (int ib = jb + 1; ib < nt && e == hipSuccess; ++ib) {
      for (int kb = jb; kb < ib && e == hipSuccess; ++kb)
        e = small_gemm<T>(false, sz(ib), sz(jb), sz(kb), 1.0, X + off(ib, kb), n, S + off(kb, jb), n,
                          kb == jb ? 0.0 : 1.0, U + off(ib, jb), n, info, s);
      if (e == hipSuccess)
        e = small_gemm<T>(false, sz(ib), sz(jb), sz(ib), -1.0, S + off(ib, ib), n, U + off(ib, jb), n, 0.0,
                          S + off(ib, jb), n, info, s);
    }
  if (e == hipSuccess) {
    const int64_t tot = (int64_t)n * n;
    hipLaunchKernelGGL((k_conj_transpose<T, true>), dim3((unsigned)std::min<int64_t>((tot + 255) / 256, 4096)),
                       dim3(256), 0, s, n, n, (const T*)S, n, U, n, (const int*)info);
    e = hipGetLastError();
  }
  return e;
}
}  // namespace

hipError_t launch_ace_factor(bool cplx, int n, void* S, void* U, void* X, int* info, hipStream_t s) {
  if (n <= kRegN) {
    if (cplx)
      hipLaunchKernelGGL(k_chol_inv_reg<Z>, dim3(1), dim3(1024), 0, s, n, (const Z*)S, n, (Z*)U, n, info, 0);
    else
      hipLaunchKernelGGL(k_chol_inv_reg<double>, dim3(1), dim3(1024), 0, s, n, (const double*)S, n, (double*)U, n,
                         info, 0);
    return hipGetLastError();
  }
  return cplx ? factor_tiled<Z>(n, (Z*)S, (Z*)U, (Z*)X, info, s)
              : factor_tiled<double>(n, (double*)S, (double*)U, (double*)X, info, s);
}

hipError_t launch_ace_tsmm(bool cplx, int64_t K, int m, int n, const void* A, int64_t lda, const void* B,
                           double alpha, double beta, void* C, int64_t ldc, const int* info, hipStream_t s) {
  if (K <= 0 || m <= 0 || n <= 0) return hipSuccess;
  // contraction slabs of at most 128 (B's column tile must fit in LDS);
  // slabs after the first accumulate
  const int64_t tiles = (K + 16 * TS_TT - 1) / (16 * TS_TT);
  const int bx = (int)std::min<int64_t>((tiles + TS_WPB - 1) / TS_WPB, device_cu_count());
  const int nj = cplx ? 64 : 128;
  const int64_t f = cplx ? 2 : 1;  // doubles per element
  dim3 grid(bx, (n + nj - 1) / nj);
  for (int q0 = 0; q0 < m; q0 += 128) {
    const int mq = std::min(128, m - q0);
    const double* As = (const double*)A + f * (int64_t)q0 * lda;
    const double* Bs = (const double*)B + f * q0;
    const double bq = q0 == 0 ? beta : 1.0;
    if (cplx)
      hipLaunchKernelGGL(k_tsmm_mfma<true>, grid, dim3(64 * TS_WPB), 0, s, K, mq, n, As, lda, Bs, m, alpha, bq, (double*)C,
                         ldc, info);
    else
      hipLaunchKernelGGL(k_tsmm_mfma<false>, grid, dim3(64 * TS_WPB), 0, s, K, mq, n, As, lda, Bs, m, alpha, bq,
                         (double*)C, ldc, info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace kx
