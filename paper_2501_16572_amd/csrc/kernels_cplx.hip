// Complex (Bloch-periodic, k != q) kernels of the batched Kronecker solver.
//
// With a Bloch wavevector k - q the 1D operators are Hermitian with complex
// eigenvectors (Sec. II; Eq. (FinalRepfL) with V^{*T}), the pair density is
// conj(psi_mq) (.) phi_nk (Eq. (Poisson)), the forward transform uses
// V1^{*T}, V2^*, V3^* and the inverse V1, V2^T, V3^T (Sec. II.A).  Each
// complex mode product is four real MFMA products on (re, im) planes:
//   (Ar + i Ai)(Br + i Bi) = (Ar Br - Ai Bi) + i (Ar Bi + Ai Br).
// Element type T: double (complex128 data, v_mfma_f64_16x16x4) or float
// (complex64 data, v_mfma_f32_16x16x4 with FP32 accumulation).  Global data
// is interleaved (re, im); LDS holds separate re / im planes.  The f table,
// the Vx accumulation and the E_x partials are FP64.
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
__device__ __forceinline__ void lds_barrier_c() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}
namespace {

template <typename T>
struct Cm;
template <>
struct Cm<double> {
  typedef d4_t acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ constexpr int row(int lg, int r) { return lg + 4 * r; }
};
template <>
struct Cm<float> {
  typedef f4_t acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ constexpr int row(int lg, int r) { return 4 * lg + r; }
};

template <int NK>
struct CTiles {
  static constexpr int NT = (NK + 3) / 4;
  static constexpr int P = 16 * NT;
  static constexpr int THREADS = 64 * NT;
};

template <typename T>
struct C2 {
  T re, im;
};

__device__ __forceinline__ int cdiv_small(int e, unsigned m) { return (int)__umulhi((unsigned)e, m); }

// Complex strip GEMM: V operand from the (re, im) planes vr, vi (row-major
// P x P, fragment element (k, c) at v[k*P + c]), conjugated when CONJ; data
// operand from the LDS planes Sr, Si (element (row, col) at S[col*LD + row]).
template <typename T, int NT, int LD, bool V_IS_A, bool CONJ>
__device__ __forceinline__ void cstrip(typename Cm<T>::acc_t* ar, typename Cm<T>::acc_t* ai,
                                       const T* Sr, const T* Si, const T* __restrict__ vr,
                                       const T* __restrict__ vi, int P, int c0, int nk, int lr,
                                       int lg) {
  using M = Cm<T>;
  const int off = lg * P + c0 + lr, vstep = 4 * P;
  T nr = vr[off], ni = vi[off];
  for (int s = 0; s < nk; ++s) {
    const T xr0 = nr;
    const T xi0 = CONJ ? -ni : ni;
    if (s + 1 < nk) {
      nr = vr[off + (s + 1) * vstep];
      ni = vi[off + (s + 1) * vstep];
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int idx = V_IS_A ? (16 * t + lr) * LD + 4 * s + lg : (4 * s + lg) * LD + 16 * t + lr;
      const T dr = Sr[idx], di = Si[idx];
      if (V_IS_A) {  // V (A) times data (B)
        ar[t] = M::mma(xr0, dr, ar[t]);
        ar[t] = M::mma(-xi0, di, ar[t]);
        ai[t] = M::mma(xr0, di, ai[t]);
        ai[t] = M::mma(xi0, dr, ai[t]);
      } else {  // data (A) times V (B)
        ar[t] = M::mma(dr, xr0, ar[t]);
        ar[t] = M::mma(-di, xi0, ar[t]);
        ai[t] = M::mma(dr, xi0, ai[t]);
        ai[t] = M::mma(di, xr0, ai[t]);
      }
    }
  }
}

// Stage one complex slice (n12 interleaved values at pa, times conj(...)
// when pb: rho = conj(pa) * pb) into the LDS planes, column-major, LD.
template <typename T, int EPT, int LD>
__device__ __forceinline__ void cstage(T* Sr, T* Si, const C2<T>* __restrict__ pa,
                                       const C2<T>* __restrict__ pb, int n1, int n12, unsigned m1,
                                       int tid, int nthr) {
  C2<T> v[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = tid + k * nthr;
    v[k] = e < n12 ? pa[e] : C2<T>{T(0), T(0)};
  }
  if (pb) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = tid + k * nthr;
      if (e < n12) {
        const C2<T> b = pb[e];
        const T r = v[k].re * b.re + v[k].im * b.im;  // conj(a) * b
        const T i = v[k].re * b.im - v[k].im * b.re;
        v[k].re = r;
        v[k].im = i;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = tid + k * nthr;
    if (e < n12) {
      const int i2 = cdiv_small(e, m1), i1 = e - i2 * n1;
      Sr[i2 * LD + i1] = v[k].re;
      Si[i2 * LD + i1] = v[k].im;
    }
  }
}

__device__ __forceinline__ double cblock_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[w] = v;
  lds_barrier_c();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  lds_barrier_c();
  return s;
}

// Pass A: pair density (IN = 0) or load (IN = 1), V1^{*T} S, S V2^*.
// a.V1, a.V2: (re, im) planes of V1, V2 (re plane at V, im plane at V + P*P).
template <typename T, int NK, int IN, bool MT = false>
__global__ void __launch_bounds__(CTiles<NK>::THREADS)
k_slice_fwd_c(SliceArgs a0, TaskTab tt) {
  constexpr int NT = CTiles<NK>::NT, P = CTiles<NK>::P, LD = P + 1;
  constexpr int EPT = (16 * NK * NK + CTiles<NK>::THREADS - 1) / CTiles<NK>::THREADS;
  using M = Cm<T>;
  using acc_t = typename M::acc_t;
  __shared__ T Sr[P * LD], Si[P * LD];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, lr = lane & 15, lg = lane >> 4;
  for (int i = tid; i < P * LD; i += nthr) Sr[i] = Si[i] = T(0);
  lds_barrier_c();
  const int64_t total = MT ? tt.pre[tt.ntasks] : (int64_t)a0.npairs * a0.n3;
  for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
    int64_t item = g;
    SliceArgs a = a0;
    if constexpr (MT) {
      int t;
      a = task_args<SliceArgs>(tt, g, item, t);
    }
    const T* V1 = (const T*)a.V1;
    const T* V2 = (const T*)a.V2;
    const int PP = a.P * a.P;
    const int nk = (max(a.n1, a.n2) + 3) / 4;
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
    const C2<T>* pa;
    const C2<T>* pb = nullptr;
    if (IN == 0) {
      const int t = p / a.n_occ, m = p - t * a.n_occ;
      pa = (const C2<T>*)a.psi + (int64_t)m * a.ld_psi + soff;
      pb = (const C2<T>*)a.phi + (int64_t)t * a.ld_phi + soff;
    } else {
      pa = (const C2<T>*)a.src + (int64_t)p * a.ld_src + soff;
    }
    cstage<T, EPT, LD>(Sr, Si, pa, pb, a.n1, a.n12, m1, tid, nthr);
    lds_barrier_c();
    acc_t ar[NT], ai[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) ar[t] = ai[t] = M::zero();
    cstrip<T, NT, LD, true, true>(ar, ai, Sr, Si, V1, V1 + PP, a.P, 16 * w, nk, lr, lg);
    lds_barrier_c();
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int idx = (16 * t + lr) * LD + 16 * w + M::row(lg, r);
        Sr[idx] = ar[t][r];
        Si[idx] = ai[t][r];
      }
    lds_barrier_c();
#pragma unroll
    for (int t = 0; t < NT; ++t) ar[t] = ai[t] = M::zero();
    cstrip<T, NT, LD, false, true>(ar, ai, Sr, Si, V2, V2 + PP, a.P, 16 * w, nk, lr, lg);
    C2<T>* out = (C2<T>*)a.dst + (int64_t)p * a.ld_dst + soff;
    const int b = 16 * w + lr;
    if (b < a.n2) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ai_ = 16 * t + M::row(lg, r);
          if (ai_ < a.n1) out[b * a.n1 + ai_] = C2<T>{ar[t][r], ai[t][r]};
        }
    }
    lds_barrier_c();
  }
}

// Pass B: Z = X V3^*, Z *= f, Y = Z V3^T on chunks of 64 pencils, in place.
// a.V3 = planes of V3, a.V3T = planes of V3^T.
template <typename T, int NK, bool MT = false>
__global__ void __launch_bounds__(CTiles<NK>::THREADS)
k_pencil_c(PencilArgs a0, TaskTab tt) {
  constexpr int NT = CTiles<NK>::NT, P = CTiles<NK>::P;
  constexpr int QT = 4, Q = 64, LDQ = Q + 1;
  using M = Cm<T>;
  using acc_t = typename M::acc_t;
  __shared__ T Sr[P * LDQ], Si[P * LDQ];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, lr = lane & 15, lg = lane >> 4;
  for (int i = tid; i < P * LDQ; i += nthr) Sr[i] = Si[i] = T(0);
  double fr[QT][4];
  auto load_f = [&](const PencilArgs& a, int q0) {
    const int c = 16 * w + lr;
#pragma unroll
    for (int qt = 0; qt < QT; ++qt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = q0 + 16 * qt + M::row(lg, r);
        fr[qt][r] = (q < a.n12 && c < a.n3) ? a.ftab[q + (int64_t)a.n12 * c] : 0.0;
      }
  };
  constexpr int EPT = Q * P / CTiles<NK>::THREADS;
  auto run = [&](const PencilArgs& a, int q0, int p) {
    const int nk = (a.n3 + 3) / 4;
    const int PP = a.P3 * a.P3;
    const T* V3 = (const T*)a.V3;
    const T* V3T = (const T*)a.V3T;
    C2<T>* base = (C2<T>*)a.T + (int64_t)p * a.ld;
    {
      C2<T> v[EPT];
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int e = tid + j * nthr;
        const int k = e / Q, qq = e - k * Q, q = q0 + qq;
        v[j] = (k < a.n3 && q < a.n12) ? base[q + (int64_t)a.n12 * k] : C2<T>{T(0), T(0)};
      }
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int e = tid + j * nthr;
        const int k = e / Q, qq = e - k * Q;
        if (k < a.n3) {
          Sr[k * LDQ + qq] = v[j].re;
          Si[k * LDQ + qq] = v[j].im;
        }
      }
    }
    lds_barrier_c();
    acc_t ar[QT], ai[QT];
#pragma unroll
    for (int t = 0; t < QT; ++t) ar[t] = ai[t] = M::zero();
    cstrip<T, QT, LDQ, false, true>(ar, ai, Sr, Si, V3, V3 + PP, a.P3, 16 * w, nk, lr, lg);
#pragma unroll
    for (int t = 0; t < QT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        ar[t][r] = (T)((double)ar[t][r] * fr[t][r]);
        ai[t][r] = (T)((double)ai[t][r] * fr[t][r]);
      }
    lds_barrier_c();
#pragma unroll
    for (int t = 0; t < QT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int idx = (16 * w + lr) * LDQ + 16 * t + M::row(lg, r);
        Sr[idx] = ar[t][r];
        Si[idx] = ai[t][r];
      }
    lds_barrier_c();
#pragma unroll
    for (int t = 0; t < QT; ++t) ar[t] = ai[t] = M::zero();
    cstrip<T, QT, LDQ, false, false>(ar, ai, Sr, Si, V3T, V3T + PP, a.P3, 16 * w, nk, lr, lg);
    const int i = 16 * w + lr;
    if (i < a.n3) {
#pragma unroll
      for (int t = 0; t < QT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = q0 + 16 * t + M::row(lg, r);
          if (q < a.n12) base[q + (int64_t)a.n12 * i] = C2<T>{ar[t][r], ai[t][r]};
        }
    }
    lds_barrier_c();
  };
  if constexpr (!MT) {
    const int chunk = blockIdx.x % a0.nchunks;
    const int pstep = gridDim.x / a0.nchunks;
    const int q0 = chunk * Q;
    load_f(a0, q0);
    lds_barrier_c();
    for (int p = blockIdx.x / a0.nchunks; p < a0.npairs; p += pstep) run(a0, q0, p);
  } else {
    // contiguous runs of (chunk, pair) items, the pair fastest (as the real kernel)
    lds_barrier_c();
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

// Pass C: V1 S (planes of V1^T in a.V1), S V2^T (planes of V2^T in a.V2);
// ACC: vx_t -= sum_m occ[m] psi_m (.) phi_mt (complex, FP64) and the E_x
// partial sum_r Re(conj(phi_t) dVx_t); else store.
template <typename T, int NK, bool ACC, bool MT = false>
__global__ void __launch_bounds__(CTiles<NK>::THREADS)
k_slice_inv_c(AccArgs a0, TaskTab tt) {
  constexpr int NT = CTiles<NK>::NT, P = CTiles<NK>::P, LD = P + 1;
  constexpr int EPT = (16 * NK * NK + CTiles<NK>::THREADS - 1) / CTiles<NK>::THREADS;
  using M = Cm<T>;
  using acc_t = typename M::acc_t;
  __shared__ T Sr[P * LD], Si[P * LD];
  __shared__ double red[16];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, lr = lane & 15, lg = lane >> 4;
  for (int i = tid; i < P * LD; i += nthr) Sr[i] = Si[i] = T(0);
  lds_barrier_c();
  const int64_t total =
      MT ? tt.pre[tt.ntasks] : (int64_t)(ACC ? a0.n_t : a0.n_t * a0.n_occ) * a0.n3;
  for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
    int64_t item = g;
    AccArgs a = a0;
    if constexpr (MT) {
      int t;
      a = task_args<AccArgs>(tt, g, item, t);
    }
    const T* V1T = (const T*)a.V1;
    const T* V2T = (const T*)a.V2;
    const int PP = a.P * a.P;
    const int nk = (max(a.n1, a.n2) + 3) / 4;
    const unsigned m1 = 0xffffffffu / (unsigned)a.n1 + 1u;
    const int n_inner = ACC ? a.n_occ : 1;
    // items run target-fastest ((i3, u), u fastest)
    const int nu = ACC ? a.n_t : a.n_t * a.n_occ;
    const int i3 = (int)(item / nu), u = (int)(item - (int64_t)i3 * nu);
    const int64_t soff = (int64_t)i3 * a.n12;
    double wr[ACC ? NT : 1][4], wi[ACC ? NT : 1][4];
    if (ACC) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) wr[t][r] = wi[t][r] = 0.0;
    }
    for (int mi = 0; mi < n_inner; ++mi) {
      const int p = ACC ? u * a.n_occ + mi : u;
      cstage<T, EPT, LD>(Sr, Si, (const C2<T>*)a.T + (int64_t)p * a.ld_T + soff, nullptr, a.n1,
                         a.n12, m1, tid, nthr);
      lds_barrier_c();
      acc_t ar[NT], ai[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) ar[t] = ai[t] = M::zero();
      cstrip<T, NT, LD, true, false>(ar, ai, Sr, Si, V1T, V1T + PP, a.P, 16 * w, nk, lr, lg);
      lds_barrier_c();
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int idx = (16 * t + lr) * LD + 16 * w + M::row(lg, r);
          Sr[idx] = ar[t][r];
          Si[idx] = ai[t][r];
        }
      lds_barrier_c();
#pragma unroll
      for (int t = 0; t < NT; ++t) ar[t] = ai[t] = M::zero();
      cstrip<T, NT, LD, false, false>(ar, ai, Sr, Si, V2T, V2T + PP, a.P, 16 * w, nk, lr, lg);
      const int b = 16 * w + lr;
      if (ACC) {
        const double coef = -a.occ[mi];
        const C2<T>* pm = (const C2<T>*)a.psi + (int64_t)mi * a.ld_psi + soff;
        if (b < a.n2) {
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int ai_ = 16 * t + M::row(lg, r);
              if (ai_ < a.n1) {
                const C2<T> ps = pm[b * a.n1 + ai_];
                const double yr = (double)ar[t][r], yi = (double)ai[t][r];
                wr[t][r] += coef * ((double)ps.re * yr - (double)ps.im * yi);
                wi[t][r] += coef * ((double)ps.re * yi + (double)ps.im * yr);
              }
            }
        }
      } else if (b < a.n2) {
        C2<T>* out = (C2<T>*)a.dst + (int64_t)p * a.ld_dst + soff;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ai_ = 16 * t + M::row(lg, r);
            if (ai_ < a.n1) out[b * a.n1 + ai_] = C2<T>{ar[t][r], ai[t][r]};
          }
      }
      lds_barrier_c();
    }
    if (ACC) {
      const int b = 16 * w + lr;
      C2<double>* vx = (C2<double>*)a.vx + (int64_t)u * a.ld_vx + soff;
      const C2<T>* pt = (const C2<T>*)a.phi + (int64_t)u * a.ld_phi + soff;
      double ex = 0.0;
      if (b < a.n2) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ai_ = 16 * t + M::row(lg, r);
            if (ai_ < a.n1) {
              const int e = b * a.n1 + ai_;
              C2<double> o = vx[e];
              o.re += wr[t][r];
              o.im += wi[t][r];
              vx[e] = o;
              const C2<T> f = pt[e];
              ex += (double)f.re * wr[t][r] + (double)f.im * wi[t][r];  // Re(conj(phi) w)
            }
          }
      }
      if (a.partials) {
        const double s = cblock_sum(ex, red);
        if (tid == 0) a.partials[(int64_t)u * a.n3 + i3] = s;
      }
    }
  }
}

template <typename K>
int c_resident(K kernel, int threads) {
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

template <typename T, int NK>
constexpr bool cslice_fits() {
  return (size_t)2 * CTiles<NK>::P * (CTiles<NK>::P + 1) * sizeof(T) + 256 <= 160 * 1024;
}

template <typename T, int NK>
hipError_t cfwd(int variant, const SliceArgs& a, int64_t items, int max_blocks, hipStream_t s,
                const TaskTab& tt) {
  if constexpr (!cslice_fits<T, NK>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int TH = CTiles<NK>::THREADS;
    void (*k)(SliceArgs, TaskTab) = tt.ntasks ? k_slice_fwd_c<T, NK, 0, true>
                                    : variant == SF_PAIR12 ? k_slice_fwd_c<T, NK, 0> : k_slice_fwd_c<T, NK, 1>;
    if (items <= 0) return hipSuccess;
    int64_t cap = (int64_t)c_resident(k, TH) * device_cu_count();
    if (max_blocks > 0) cap = std::min<int64_t>(cap, max_blocks);
    hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(1, std::min(items, cap))), dim3(TH), 0, s, a, tt);
    return hipGetLastError();
  }
}

template <typename T, int NK>
hipError_t cpencil(const PencilArgs& a, int max_blocks, hipStream_t s, const TaskTab& tt, int64_t items) {
  if constexpr ((size_t)2 * CTiles<NK>::P * 65 * sizeof(T) + 256 > 160 * 1024) {
    return hipErrorInvalidValue;
  } else {
  constexpr int TH = CTiles<NK>::THREADS;
  void (*k)(PencilArgs, TaskTab) = tt.ntasks ? k_pencil_c<T, NK, true> : k_pencil_c<T, NK>;
  int64_t cap = (int64_t)c_resident(k, TH) * device_cu_count();
  if (max_blocks > 0) cap = std::min<int64_t>(cap, max_blocks);
  if (tt.ntasks) {
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(1, std::min(items, cap))), dim3(TH), 0, s, a, tt);
    return hipGetLastError();
  }
  if (a.npairs <= 0 || a.nchunks <= 0) return hipSuccess;
  int64_t groups = std::max<int64_t>(1, cap / a.nchunks);
  groups = std::min<int64_t>(groups, a.npairs);
  hipLaunchKernelGGL(k, dim3((unsigned)(groups * a.nchunks)), dim3(TH), 0, s, a, tt);
  return hipGetLastError();
  }
}

template <typename T, int NK>
hipError_t cinv(int variant, const AccArgs& a, int64_t items, int max_blocks, hipStream_t s,
                const TaskTab& tt) {
  if constexpr (!cslice_fits<T, NK>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int TH = CTiles<NK>::THREADS;
    void (*k)(AccArgs, TaskTab) = tt.ntasks ? k_slice_inv_c<T, NK, true, true>
                                  : variant == SI_ACC12 ? k_slice_inv_c<T, NK, true> : k_slice_inv_c<T, NK, false>;
    if (items <= 0) return hipSuccess;
    int64_t cap = (int64_t)c_resident(k, TH) * device_cu_count();
    if (max_blocks > 0) cap = std::min<int64_t>(cap, max_blocks);
    if (g_grid_probe) {
      *g_grid_probe = std::max<int64_t>(1, std::min(items, cap));
      return hipSuccess;
    }
    hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(1, std::min(items, cap))), dim3(TH), 0, s, a, tt);
    return hipGetLastError();
  }
}

#define KX_CNK_CASES(F) F(6) F(8) F(12) F(14) F(16) F(18) F(20) F(24) F(28) F(30) F(32) F(36) F(40)

}  // namespace

hipError_t launch_slice_fwd_c(bool f64, int nk, int variant, const SliceArgs& a, int64_t items,
                              int max_blocks, hipStream_t s, const TaskTab& tt) {
  if (variant != SF_PAIR12 && variant != SF_LOAD12) return hipErrorInvalidValue;
  switch (nk) {
#define C(n) \
  case n:    \
    return f64 ? cfwd<double, n>(variant, a, items, max_blocks, s, tt) : cfwd<float, n>(variant, a, items, max_blocks, s, tt);
    KX_CNK_CASES(C)
#undef C
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pencil_c(bool f64, int nk, const PencilArgs& a, int max_blocks, hipStream_t s,
                           const TaskTab& tt, int64_t items) {
  switch (nk) {
#define C(n) \
  case n:    \
    return f64 ? cpencil<double, n>(a, max_blocks, s, tt, items) : cpencil<float, n>(a, max_blocks, s, tt, items);
    KX_CNK_CASES(C)
#undef C
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_slice_inv_c(bool f64, int nk, int variant, const AccArgs& a, int64_t items,
                              int max_blocks, hipStream_t s, const TaskTab& tt) {
  if (variant != SI_ACC12 && variant != SI_ST12) return hipErrorInvalidValue;
  switch (nk) {
#define C(n) \
  case n:    \
    return f64 ? cinv<double, n>(variant, a, items, max_blocks, s, tt) : cinv<float, n>(variant, a, items, max_blocks, s, tt);
    KX_CNK_CASES(C)
#undef C
    default: return hipErrorInvalidValue;
  }
}

}  // namespace kx
