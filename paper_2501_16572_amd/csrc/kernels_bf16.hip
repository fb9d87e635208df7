// Split-BF16 mode products for gfx950 (v_mfma_f32_16x16x32_bf16, FP32
// accumulation).  Each FP32 operand x is written as a sum of bf16 parts
// (round-to-nearest-even at every step, the remainders are exact in FP32):
//   SPL = 2 (BF16X3): x ~ hi + lo,        products hi*hi + hi*lo + lo*hi
//   SPL = 3 (BF16X6): x ~ hi + mid + lo,  products down to relative weight
//                     2^-16: hh, hm, mh, hl, mm, lh
// Intermediates stay FP32 in HBM; the f(Lambda~) scaling and the Vx / E_x
// accumulation are FP64 as in the other precisions.
//
// The data operand is split once when it is written to LDS, into SPL bf16
// planes laid out with K contiguous ("line" = tile row/column, 16-byte
// aligned), so a fragment is one 16-byte LDS read per plane.  The eigenvector
// operand is pre-split on the host in [c][k] layout (K contiguous), so a
// fragment is one 16-byte global (L2) load per part, prefetched one K step
// ahead.
//
// MFMA 16x16x32 bf16 layout (lane l = 16*lg + lr), measured on gfx950:
//   A fragment: A[row = lr][k = 8*lg + i], i = 0..7
//   B fragment: B[k = 8*lg + i][col = lr]
//   accumulator element r: D[row = 4*lg + r][col = lr]
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "kernels.h"
#include "launch.h"

namespace kx {

// Block barrier for LDS hand-offs only: waits for this wave's LDS operations
// and meets the other waves, but leaves global loads in flight (a full
// __syncthreads() also waits for them, which would serialize the prefetch of
// the next work unit with the current one's MFMA work).  Nothing in these
// kernels communicates through global memory within a block.
__device__ __forceinline__ void lds_barrier_bf() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

namespace {

template <int SPL>
struct Prods;
template <>
struct Prods<2> {
  static constexpr int n = 3;
  static constexpr int v[3] = {0, 0, 1};  // part of the eigenvector operand
  static constexpr int d[3] = {0, 1, 0};  // part of the data operand
};
template <>
struct Prods<3> {
  static constexpr int n = 6;
  static constexpr int v[6] = {0, 0, 1, 0, 1, 2};
  static constexpr int d[6] = {0, 1, 0, 2, 1, 0};
};

template <int SPL>
__device__ __forceinline__ void split_parts(float x, __bf16* out) {
  const __bf16 h = (__bf16)x;
  out[0] = h;
  const float r1 = x - (float)h;
  const __bf16 m = (__bf16)r1;
  out[1] = m;
  if (SPL == 3) out[2] = (__bf16)(r1 - (float)m);
}

// Geometry of one operand buffer: NT 16-row tiles of lines, K padded to 32.
template <int NT>
struct BfGeo {
  static constexpr int P = 16 * NT;                 // lines (and output length)
  static constexpr int NK32 = (NT + 1) / 2;         // 32-deep K steps
  static constexpr int KP = 32 * NK32;              // padded K
  static constexpr int LINES = P > KP ? P : KP;     // lines addressable as K too
  static constexpr int LD = KP + 8;                 // bf16 elements per line
};

// Write one FP32 value, split, into the SPL planes at (line, k).
template <int SPL, int LD, int PLANE>
__device__ __forceinline__ void put(__bf16* S, int line, int k, float x) {
  __bf16 p[3];
  split_parts<SPL>(x, p);
#pragma unroll
  for (int q = 0; q < SPL; ++q) S[q * PLANE + line * LD + k] = p[q];
}

// Strip GEMM on split operands.  For each of the wave's SPW eigenvector
// strips (columns c0 + 16 j) and each data tile t < NTD:
//   V_IS_A: acc[j][t] += sum_k V(c, k) D(16t + lr, k)  (D[row c][col line])
//   else  : acc[j][t] += sum_k D(16t + lr, k) V(c, k)  (D[row line][col c])
// V parts: vp[part][c * KPV + k] (bf16, K contiguous); D planes in LDS with
// K contiguous per line.
template <int SPL, int SPW, int NTD, int LD, int PLANE, bool V_IS_A>
__device__ __forceinline__ void strip_gemm_bf(f4_t (*acc)[NTD], const __bf16* S,
                                              const __bf16* __restrict__ vp, int vpart_stride,
                                              int KPV, int c0, int nk32, int lr, int lg) {
  using PR = Prods<SPL>;
  const __bf16* vrow[SPW];
#pragma unroll
  for (int j = 0; j < SPW; ++j) vrow[j] = vp + (size_t)(c0 + 16 * j + lr) * KPV + 8 * lg;
  bf8_t vn[SPW][SPL];
#pragma unroll
  for (int j = 0; j < SPW; ++j)
#pragma unroll
    for (int q = 0; q < SPL; ++q) vn[j][q] = *(const bf8_t*)(vrow[j] + (size_t)q * vpart_stride);
  for (int s = 0; s < nk32; ++s) {
    bf8_t vc[SPW][SPL];
#pragma unroll
    for (int j = 0; j < SPW; ++j)
#pragma unroll
      for (int q = 0; q < SPL; ++q) vc[j][q] = vn[j][q];
    if (s + 1 < nk32) {
#pragma unroll
      for (int j = 0; j < SPW; ++j)
#pragma unroll
        for (int q = 0; q < SPL; ++q)
          vn[j][q] = *(const bf8_t*)(vrow[j] + (size_t)q * vpart_stride + 32 * (s + 1));
    }
#pragma unroll
    for (int t = 0; t < NTD; ++t) {
      bf8_t df[SPL];
#pragma unroll
      for (int q = 0; q < SPL; ++q)
        df[q] = *(const bf8_t*)(S + q * PLANE + (16 * t + lr) * LD + 32 * s + 8 * lg);
#pragma unroll
      for (int j = 0; j < SPW; ++j)
#pragma unroll
        for (int u = 0; u < PR::n; ++u) {
          if (V_IS_A)
            acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vc[j][PR::v[u]], df[PR::d[u]],
                                                               acc[j][t], 0, 0, 0);
          else
            acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(df[PR::d[u]], vc[j][PR::v[u]],
                                                               acc[j][t], 0, 0, 0);
        }
    }
  }
}

__device__ __forceinline__ double block_sum_bf(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[w] = v;
  lds_barrier_bf();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  lds_barrier_bf();
  return s;
}

__device__ __forceinline__ int div_small_bf(int e, unsigned m) { return (int)__umulhi((unsigned)e, m); }

template <int NT, int SPW>
struct BfWaves {
  static constexpr int W = (NT + SPW - 1) / SPW;
  static constexpr int THREADS = 64 * W;
};

// ---------------------------------------------------------------------------
// Pass A: pair density (IN = 0) or plain load (IN = 1), mode-1 forward
// (V1^T S), mode-2 forward (S V2) per frontal slice.
// V parts: a.V1 = split(V1^T) [a][k], a.V2 = split(V2^T) [b][k].
// ---------------------------------------------------------------------------
template <int SPL, int NT, int SPW, int IN, bool MT = false>
__global__ void __launch_bounds__((BfWaves<NT, SPW>::THREADS))
k_slice_fwd_bf(SliceArgs a0, int vpart_stride, int KPV, TaskTab tt) {
  using G = BfGeo<NT>;
  constexpr int LD = G::LD, PLANE = G::LINES * LD;
  constexpr int NW = BfWaves<NT, SPW>::W;
  __shared__ __attribute__((aligned(16))) __bf16 S[SPL * PLANE];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, lr = lane & 15, lg = lane >> 4;
  for (int i = tid; i < SPL * PLANE; i += nthr) S[i] = (__bf16)0.f;
  lds_barrier_bf();
  constexpr int EPT0 = (G::P * G::P + 64 * NW - 1) / (64 * NW);
  constexpr int CH = EPT0 < 16 ? EPT0 : 16;
  constexpr int EPT = (EPT0 + CH - 1) / CH * CH;
  const int64_t total = MT ? tt.pre[tt.ntasks] : (int64_t)a0.npairs * a0.n3;
  for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
    int64_t item = g;
    SliceArgs a = a0;
    if constexpr (MT) {
      int t;
      a = task_args<SliceArgs>(tt, g, item, t);
    }
    const int nk32 = (max(a.n1, a.n2) + 31) / 32;
    const unsigned m1 = 0xffffffffu / (unsigned)a.n1 + 1u;
    // pair-density items run target-fastest (as the FP64/FP32 kernel)
    int p, i3;
    if (IN == 0) {
      const int n_t = a.npairs / a.n_occ;
      const int64_t rest = item / n_t;
      const int t = (int)(item - rest * n_t);
      i3 = (int)(rest / a.n_occ);
      p = t * a.n_occ + (int)(rest - (int64_t)i3 * a.n_occ);
    } else {
      p = (int)(item / a.n3);
      i3 = (int)(item - (int64_t)p * a.n3);
    }
    const int64_t soff = (int64_t)i3 * a.n12;
    float* out = (float*)a.dst + (int64_t)p * a.ld_dst + soff;
    const float* pa;
    const float* pb = nullptr;
    if (IN == 0) {
      const int t = p / a.n_occ, m = p - t * a.n_occ;
      pa = (const float*)a.psi + (int64_t)m * a.ld_psi + soff;
      pb = (const float*)a.phi + (int64_t)t * a.ld_phi + soff;
    } else {
      pa = (const float*)a.src + (int64_t)p * a.ld_src + soff;
    }
    // stage in chunks of CH elements per thread, all loads of a chunk in flight
    for (int k0 = 0; k0 < EPT; k0 += CH) {
      float v[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int e = tid + (k0 + k) * nthr;
        v[k] = e < a.n12 ? pa[e] : 0.f;
      }
      if (IN == 0) {
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int e = tid + (k0 + k) * nthr;
          if (e < a.n12) v[k] *= pb[e];
        }
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int e = tid + (k0 + k) * nthr;
        if (e < a.n12) {
          const int i2 = div_small_bf(e, m1), i1 = e - i2 * a.n1;
          put<SPL, LD, PLANE>(S, i2, i1, v[k]);  // line j = i2, k = i1
        }
      }
    }
    lds_barrier_bf();
    // mode 1: T1[a][j] = sum_k V1^T[a][k] rho[k][j]; wave strips a = 16(w*SPW + jj)
    f4_t acc[SPW][NT];
#pragma unroll
    for (int j = 0; j < SPW; ++j)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[j][t] = f4_t{0.f, 0.f, 0.f, 0.f};
    const int c0 = 16 * SPW * w;
    if (c0 < G::P)
      strip_gemm_bf<SPL, SPW, NT, LD, PLANE, true>(acc, S, (const __bf16*)a.V1, vpart_stride, KPV,
                                                   c0, nk32, lr, lg);
    lds_barrier_bf();
    // T1 back into the planes as [line a][k = j]
    if (c0 < G::P) {
#pragma unroll
      for (int j = 0; j < SPW; ++j)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int arow = c0 + 16 * j + 4 * lg + r;
            if (arow < G::P) put<SPL, LD, PLANE>(S, arow, 16 * t + lr, acc[j][t][r]);
          }
    }
    lds_barrier_bf();
    // mode 2: T2[a][b] = sum_k T1[a][k] V2[k][b]; wave strips b
#pragma unroll
    for (int j = 0; j < SPW; ++j)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[j][t] = f4_t{0.f, 0.f, 0.f, 0.f};
    if (c0 < G::P)
      strip_gemm_bf<SPL, SPW, NT, LD, PLANE, false>(acc, S, (const __bf16*)a.V2, vpart_stride,
                                                    KPV, c0, nk32, lr, lg);
#pragma unroll
    for (int j = 0; j < SPW; ++j) {
      const int b = c0 + 16 * j + lr;
      if (b < a.n2) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ai = 16 * t + 4 * lg + r;
            if (ai < a.n1) out[b * a.n1 + ai] = acc[j][t][r];
          }
      }
    }
    lds_barrier_bf();
  }
}

// ---------------------------------------------------------------------------
// Pass B: mode-3 forward (X V3), f(Lambda~) scaling in FP64, mode-3 inverse
// (Z V3^T) on chunks of 64 pencils, in place.
// V parts: a.V3 = split(V3^T) [c][k], a.V3T = split(V3) [i][c].
// ---------------------------------------------------------------------------
template <int SPL, int NT, int SPW, bool MT = false>
__global__ void __launch_bounds__((BfWaves<NT, SPW>::THREADS))
k_pencil_bf(PencilArgs a0, int vpart_stride, int KPV, TaskTab tt) {
  using G = BfGeo<NT>;
  constexpr int QT = 4, Q = 64;
  constexpr int LD = G::LD, PLANE = Q * LD;
  constexpr int NW = BfWaves<NT, SPW>::W;
  __shared__ __attribute__((aligned(16))) __bf16 S[SPL * PLANE];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, lr = lane & 15, lg = lane >> 4;
  const int c0 = 16 * SPW * w;
  for (int i = tid; i < SPL * PLANE; i += nthr) S[i] = (__bf16)0.f;
  double fr[SPW][QT][4];
  auto load_f = [&](const PencilArgs& a, int q0) {
#pragma unroll
    for (int j = 0; j < SPW; ++j) {
      const int c = c0 + 16 * j + lr;
#pragma unroll
      for (int qt = 0; qt < QT; ++qt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = q0 + 16 * qt + 4 * lg + r;
          fr[j][qt][r] = (q < a.n12 && c < a.n3) ? a.ftab[q + (int64_t)a.n12 * c] : 0.0;
        }
    }
  };
  constexpr int EPT0 = (Q * G::P + 64 * NW - 1) / (64 * NW);
  constexpr int CH = EPT0 < 16 ? EPT0 : 16;
  constexpr int EPT = (EPT0 + CH - 1) / CH * CH;
  auto run = [&](const PencilArgs& a, int q0, int p) {
    const int nk32 = (a.n3 + 31) / 32;
    float* base = (float*)a.T + (int64_t)p * a.ld;
    for (int j0 = 0; j0 < EPT; j0 += CH) {
      float v[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int e = tid + (j0 + j) * nthr;
        const int k = e / Q, qq = e - k * Q, q = q0 + qq;
        v[j] = (k < a.n3 && q < a.n12) ? base[q + (int64_t)a.n12 * k] : 0.f;
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int e = tid + (j0 + j) * nthr;
        const int k = e / Q, qq = e - k * Q;
        if (k < a.n3) put<SPL, LD, PLANE>(S, qq, k, v[j]);  // line q, k = i3
      }
    }
    lds_barrier_bf();
    f4_t acc[SPW][QT];
#pragma unroll
    for (int j = 0; j < SPW; ++j)
#pragma unroll
      for (int t = 0; t < QT; ++t) acc[j][t] = f4_t{0.f, 0.f, 0.f, 0.f};
    if (c0 < G::P)
      strip_gemm_bf<SPL, SPW, QT, LD, PLANE, false>(acc, S, (const __bf16*)a.V3, vpart_stride,
                                                    KPV, c0, nk32, lr, lg);
    lds_barrier_bf();
    if (c0 < G::P) {
#pragma unroll
      for (int j = 0; j < SPW; ++j) {
        const int c = c0 + 16 * j + lr;
#pragma unroll
        for (int t = 0; t < QT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float z = (float)((double)acc[j][t][r] * fr[j][t][r]);
            put<SPL, LD, PLANE>(S, 16 * t + 4 * lg + r, c, z);  // line q, k = c
          }
      }
    }
    lds_barrier_bf();
#pragma unroll
    for (int j = 0; j < SPW; ++j)
#pragma unroll
      for (int t = 0; t < QT; ++t) acc[j][t] = f4_t{0.f, 0.f, 0.f, 0.f};
    if (c0 < G::P)
      strip_gemm_bf<SPL, SPW, QT, LD, PLANE, false>(acc, S, (const __bf16*)a.V3T, vpart_stride,
                                                    KPV, c0, nk32, lr, lg);
#pragma unroll
    for (int j = 0; j < SPW; ++j) {
      const int i = c0 + 16 * j + lr;
      if (i < a.n3) {
#pragma unroll
        for (int t = 0; t < QT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int q = q0 + 16 * t + 4 * lg + r;
            if (q < a.n12) base[q + (int64_t)a.n12 * i] = acc[j][t][r];
          }
      }
    }
    lds_barrier_bf();

  };
  if constexpr (!MT) {
    const int chunk = blockIdx.x % a0.nchunks;
    const int pstep = gridDim.x / a0.nchunks;
    const int q0 = chunk * Q;
    load_f(a0, q0);
    lds_barrier_bf();
    for (int p = blockIdx.x / a0.nchunks; p < a0.npairs; p += pstep) run(a0, q0, p);
  } else {
    // contiguous runs of (chunk, pair) items, the pair fastest (as the FP32/FP64 kernel)
    lds_barrier_bf();
    const int64_t total = tt.pre[tt.ntasks];
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    const int64_t g0 = (int64_t)blockIdx.x * per, g1 = min(total, g0 + per);
    int cur_t = -1, cur_c = -1;
    for (int64_t g = g0; g < g1; ++g) {
      int64_t item;
      int t;
      const PencilArgs a = task_args<PencilArgs>(tt, g, item, t);
      const int chunk = (int)(item / a.npairs), p = (int)(item - (int64_t)chunk * a.npairs);
      if (t != cur_t || chunk != cur_c) {
        load_f(a, chunk * Q);
        cur_t = t;
        cur_c = chunk;
      }
      run(a, chunk * Q, p);
    }
  }
}

// ---------------------------------------------------------------------------
// Pass C: mode-1 inverse (V1 X), mode-2 inverse (X V2^T); ACC: psi_m product
// and FP64 accumulation into Vx with E_x partials, else store.
// V parts: a.V1 = split(V1) [i][a], a.V2 = split(V2) [b][k].
// ---------------------------------------------------------------------------
template <int SPL, int NT, int SPW, bool ACC, bool MT = false>
__global__ void __launch_bounds__((BfWaves<NT, SPW>::THREADS))
k_slice_inv_bf(AccArgs a0, int vpart_stride, int KPV, TaskTab tt) {
  using G = BfGeo<NT>;
  constexpr int LD = G::LD, PLANE = G::LINES * LD;
  constexpr int NW = BfWaves<NT, SPW>::W;
  __shared__ __attribute__((aligned(16))) __bf16 S[SPL * PLANE];
  __shared__ double red[16];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, lr = lane & 15, lg = lane >> 4;
  for (int i = tid; i < SPL * PLANE; i += nthr) S[i] = (__bf16)0.f;
  lds_barrier_bf();
  const int c0 = 16 * SPW * w;
  constexpr int EPT0 = (G::P * G::P + 64 * NW - 1) / (64 * NW);
  constexpr int CH = EPT0 < 16 ? EPT0 : 16;
  constexpr int EPT = (EPT0 + CH - 1) / CH * CH;
  const int64_t total =
      MT ? tt.pre[tt.ntasks] : (int64_t)(ACC ? a0.n_t : a0.n_t * a0.n_occ) * a0.n3;
  for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
    int64_t item = g;
    AccArgs a = a0;
    if constexpr (MT) {
      int t;
      a = task_args<AccArgs>(tt, g, item, t);
    }
    const int nk32 = (max(a.n1, a.n2) + 31) / 32;
    const unsigned m1 = 0xffffffffu / (unsigned)a.n1 + 1u;
    const int n_inner = ACC ? a.n_occ : 1;
    // items run target-fastest ((i3, u), u fastest)
    const int nu = ACC ? a.n_t : a.n_t * a.n_occ;
    const int i3 = (int)(item / nu), u = (int)(item - (int64_t)i3 * nu);
    const int64_t soff = (int64_t)i3 * a.n12;
    double wacc[ACC ? SPW : 1][ACC ? NT : 1][4];
    if (ACC) {
#pragma unroll
      for (int j = 0; j < SPW; ++j)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) wacc[j][t][r] = 0.0;
    }
    for (int mi = 0; mi < n_inner; ++mi) {
      const int p = ACC ? u * a.n_occ + mi : u;
      const float* src = (const float*)a.T + (int64_t)p * a.ld_T + soff;
      for (int k0 = 0; k0 < EPT; k0 += CH) {
        float v[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int e = tid + (k0 + k) * nthr;
          v[k] = e < a.n12 ? src[e] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int e = tid + (k0 + k) * nthr;
          if (e < a.n12) {
            const int i2 = div_small_bf(e, m1), i1 = e - i2 * a.n1;
            put<SPL, LD, PLANE>(S, i2, i1, v[k]);  // line j = i2, k = a = i1
          }
        }
      }
      lds_barrier_bf();
      f4_t acc[SPW][NT];
#pragma unroll
      for (int j = 0; j < SPW; ++j)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[j][t] = f4_t{0.f, 0.f, 0.f, 0.f};
      if (c0 < G::P)
        strip_gemm_bf<SPL, SPW, NT, LD, PLANE, true>(acc, S, (const __bf16*)a.V1, vpart_stride,
                                                     KPV, c0, nk32, lr, lg);
      lds_barrier_bf();
      if (c0 < G::P) {
#pragma unroll
        for (int j = 0; j < SPW; ++j)
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int irow = c0 + 16 * j + 4 * lg + r;
              if (irow < G::P) put<SPL, LD, PLANE>(S, irow, 16 * t + lr, acc[j][t][r]);
            }
      }
      lds_barrier_bf();
#pragma unroll
      for (int j = 0; j < SPW; ++j)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[j][t] = f4_t{0.f, 0.f, 0.f, 0.f};
      if (c0 < G::P)
        strip_gemm_bf<SPL, SPW, NT, LD, PLANE, false>(acc, S, (const __bf16*)a.V2, vpart_stride,
                                                      KPV, c0, nk32, lr, lg);
      if (ACC) {
        const double coef = -a.occ[mi];
        const float* pm = (const float*)a.psi + (int64_t)mi * a.ld_psi + soff;
#pragma unroll
        for (int j = 0; j < SPW; ++j) {
          const int b = c0 + 16 * j + lr;
          if (b < a.n2) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int ai = 16 * t + 4 * lg + r;
                if (ai < a.n1)
                  wacc[j][t][r] += coef * (double)pm[b * a.n1 + ai] * (double)acc[j][t][r];
              }
          }
        }
      } else {
        float* out = (float*)a.dst + (int64_t)p * a.ld_dst + soff;
#pragma unroll
        for (int j = 0; j < SPW; ++j) {
          const int b = c0 + 16 * j + lr;
          if (b < a.n2) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int ai = 16 * t + 4 * lg + r;
                if (ai < a.n1) out[b * a.n1 + ai] = acc[j][t][r];
              }
          }
        }
      }
      lds_barrier_bf();
    }
    if (ACC) {
      double* vx = a.vx + (int64_t)u * a.ld_vx + soff;
      const float* pt = (const float*)a.phi + (int64_t)u * a.ld_phi + soff;
      double ex = 0.0;
#pragma unroll
      for (int j = 0; j < SPW; ++j) {
        const int b = c0 + 16 * j + lr;
        if (b < a.n2) {
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int ai = 16 * t + 4 * lg + r;
              if (ai < a.n1) {
                const int e = b * a.n1 + ai;
                vx[e] += wacc[j][t][r];
                ex += (double)pt[e] * wacc[j][t][r];
              }
            }
        }
      }
      if (a.partials) {
        const double s = block_sum_bf(ex, red);
        if (tid == 0) a.partials[(int64_t)u * a.n3 + i3] = s;
      }
    }
  }
}

template <typename K>
int bf_resident(K kernel, int threads) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find((const void*)kernel);
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1)
    nb = 1;
  cache[(const void*)kernel] = nb;
  return nb;
}

template <typename K>
int bf_grid(K kernel, int threads, int64_t items, int max_blocks) {
  int64_t cap = (int64_t)bf_resident(kernel, threads) * device_cu_count();
  if (max_blocks > 0) cap = std::min<int64_t>(cap, max_blocks);
  return (int)std::max<int64_t>(1, std::min<int64_t>(items, cap));
}

// Two strips per wave when the tile count is even and at least 4 (a data
// fragment then feeds both strips), else one.
template <int NT>
constexpr int spw_for() { return (NT >= 4 && NT % 2 == 0) ? 2 : 1; }

template <int SPL, int NT>
hipError_t fwd_nt(int variant, const SliceArgs& a, int64_t items, int max_blocks, int vps, int kpv,
                  hipStream_t s, const TaskTab& tt) {
  constexpr int SPW = spw_for<NT>();
  constexpr int TH = BfWaves<NT, SPW>::THREADS;
  void (*k)(SliceArgs, int, int, TaskTab) = tt.ntasks ? k_slice_fwd_bf<SPL, NT, SPW, 0, true>
                                             : variant == SF_PAIR12 ? k_slice_fwd_bf<SPL, NT, SPW, 0>
                                                                    : k_slice_fwd_bf<SPL, NT, SPW, 1>;
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k, dim3(bf_grid(k, TH, items, max_blocks)), dim3(TH), 0, s, a, vps, kpv, tt);
  return hipGetLastError();
}

template <int SPL, int NT>
hipError_t pencil_nt(const PencilArgs& a, int max_blocks, int vps, int kpv, hipStream_t s,
                     const TaskTab& tt, int64_t items) {
  constexpr int SPW = 1;  // the per-block f-table slice is kept per strip
  constexpr int TH = BfWaves<NT, SPW>::THREADS;
  void (*k)(PencilArgs, int, int, TaskTab) = tt.ntasks ? k_pencil_bf<SPL, NT, SPW, true> : k_pencil_bf<SPL, NT, SPW>;
  if (tt.ntasks) {
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k, dim3(bf_grid(k, TH, items, max_blocks)), dim3(TH), 0, s, a, vps, kpv, tt);
    return hipGetLastError();
  }
  if (a.npairs <= 0 || a.nchunks <= 0) return hipSuccess;
  int64_t cap = (int64_t)bf_resident(k, TH) * device_cu_count();
  if (max_blocks > 0) cap = std::min<int64_t>(cap, max_blocks);
  int64_t groups = std::max<int64_t>(1, cap / a.nchunks);
  groups = std::min<int64_t>(groups, a.npairs);
  hipLaunchKernelGGL(k, dim3((unsigned)(groups * a.nchunks)), dim3(TH), 0, s, a, vps, kpv, tt);
  return hipGetLastError();
}

template <int SPL, int NT>
hipError_t inv_nt(int variant, const AccArgs& a, int64_t items, int max_blocks, int vps, int kpv,
                  hipStream_t s, const TaskTab& tt) {
  constexpr int SPW = 1;  // the FP64 Vx accumulator is kept per strip
  constexpr int TH = BfWaves<NT, SPW>::THREADS;
  void (*k)(AccArgs, int, int, TaskTab) = tt.ntasks ? k_slice_inv_bf<SPL, NT, SPW, true, true>
                                           : variant == SI_ACC12 ? k_slice_inv_bf<SPL, NT, SPW, true>
                                                                 : k_slice_inv_bf<SPL, NT, SPW, false>;
  if (items <= 0) return hipSuccess;
  if (g_grid_probe) {
    *g_grid_probe = bf_grid(k, TH, items, max_blocks);
    return hipSuccess;
  }
  hipLaunchKernelGGL(k, dim3(bf_grid(k, TH, items, max_blocks)), dim3(TH), 0, s, a, vps, kpv, tt);
  return hipGetLastError();
}

#define KX_NT_CASES(F) F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9) F(10)

}  // namespace

hipError_t launch_slice_fwd_bf(int spl, int nt, int variant, const SliceArgs& a, int64_t items,
                               int max_blocks, int vps, int kpv, hipStream_t s, const TaskTab& tt) {
  if (variant != SF_PAIR12 && variant != SF_LOAD12) return hipErrorInvalidValue;
  switch (nt) {
#define C(n)                                                                        \
  case n:                                                                           \
    return spl == 2 ? fwd_nt<2, n>(variant, a, items, max_blocks, vps, kpv, s, tt)  \
                    : fwd_nt<3, n>(variant, a, items, max_blocks, vps, kpv, s, tt);
    KX_NT_CASES(C)
#undef C
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pencil_bf(int spl, int nt, const PencilArgs& a, int max_blocks, int vps, int kpv,
                            hipStream_t s, const TaskTab& tt, int64_t items) {
  switch (nt) {
#define C(n) \
  case n:    \
    return spl == 2 ? pencil_nt<2, n>(a, max_blocks, vps, kpv, s, tt, items) \
                    : pencil_nt<3, n>(a, max_blocks, vps, kpv, s, tt, items);
    KX_NT_CASES(C)
#undef C
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_slice_inv_bf(int spl, int nt, int variant, const AccArgs& a, int64_t items,
                               int max_blocks, int vps, int kpv, hipStream_t s, const TaskTab& tt) {
  if (variant != SI_ACC12 && variant != SI_ST12) return hipErrorInvalidValue;
  switch (nt) {
#define C(n)                                                                        \
  case n:                                                                           \
    return spl == 2 ? inv_nt<2, n>(variant, a, items, max_blocks, vps, kpv, s, tt)  \
                    : inv_nt<3, n>(variant, a, items, max_blocks, vps, kpv, s, tt);
    KX_NT_CASES(C)
#undef C
    default: return hipErrorInvalidValue;
  }
}

}  // namespace kx
