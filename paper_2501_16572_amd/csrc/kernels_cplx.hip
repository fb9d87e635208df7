// Complex (Bloch-periodic, k != q) kernels of the batched Kronecker solver.
//
// With a Bloch wavevector k - q the 1D operators are Hermitian with complex
// eigenvectors (Sec. II; Eq. (FinalRepfL) with V^{*T}), the pair density is
// conj(psi_mq) (.) phi_nk (Eq. (Poisson)), the forward transform uses
// V1^{*T}, V2^*, V3^* and the inverse V1, V2^T, V3^T (Sec. II.A).  Each
// complex mode product is three real MFMA products on (re, im) planes:
//   (Ar + i Ai)(Br + i Bi) = (P1 - P2) + i (P3 - P1 - P2),
//   P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi).
// Element type T: double (complex128 data, v_mfma_f64_16x16x4) or float
// (complex64 data, v_mfma_f32_16x16x4 with FP32 accumulation).  Global data
// is interleaved (re, im); LDS holds separate re / im planes.  The f table,
// the Vx accumulation and the E_x partials are FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "kernels.h"
#include "kernels_cplx.inc"
#include "launch.h"

namespace kx {
namespace {

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
    const bool alt = variant & TUNE_ALT;
    void (*k)(SliceArgs, TaskTab) =
        tt.ntasks ? (alt ? k_slice_fwd_c<T, NK, 0, true, true> : k_slice_fwd_c<T, NK, 0, true>)
        : (variant & ~TUNE_ALT) == SF_PAIR12 ? (alt ? k_slice_fwd_c<T, NK, 0, false, true> : k_slice_fwd_c<T, NK, 0>)
                                             : k_slice_fwd_c<T, NK, 1>;
    if (items <= 0) return hipSuccess;
    int64_t cap = (int64_t)c_resident(k, TH) * device_cu_count();
    if (max_blocks > 0) cap = std::min<int64_t>(cap, max_blocks);
    hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(1, std::min(items, cap))), dim3(TH), 0, s, a, tt);
    return hipGetLastError();
  }
}

template <typename T, int NK>
hipError_t cpencil(int variant, const PencilArgs& a, int max_blocks, hipStream_t s, const TaskTab& tt,
                   int64_t items) {
  if constexpr ((size_t)2 * CTiles<NK>::P * 65 * sizeof(T) + 256 > 160 * 1024) {
    return hipErrorInvalidValue;
  } else {
  constexpr int TH = CTiles<NK>::THREADS;
  const bool alt = variant & TUNE_ALT;
  void (*k)(PencilArgs, TaskTab) = tt.ntasks ? (alt ? k_pencil_c<T, NK, true, true> : k_pencil_c<T, NK, true>)
                                             : (alt ? k_pencil_c<T, NK, false, true> : k_pencil_c<T, NK>);
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
    const bool alt = variant & TUNE_ALT;
    void (*k)(AccArgs, TaskTab) =
        tt.ntasks ? (alt ? k_slice_inv_c<T, NK, true, true, true> : k_slice_inv_c<T, NK, true, true>)
        : (variant & ~TUNE_ALT) == SI_ACC12 ? (alt ? k_slice_inv_c<T, NK, true, false, true> : k_slice_inv_c<T, NK, true>)
                                            : k_slice_inv_c<T, NK, false>;
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
  const int base = variant & ~TUNE_ALT;
  if (base != SF_PAIR12 && base != SF_LOAD12) return hipErrorInvalidValue;
  switch (nk) {
#define C(n) \
  case n:    \
    return f64 ? cfwd<double, n>(variant, a, items, max_blocks, s, tt) : cfwd<float, n>(variant, a, items, max_blocks, s, tt);
    KX_CNK_CASES(C)
#undef C
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pencil_c(bool f64, int nk, int variant, const PencilArgs& a, int max_blocks, hipStream_t s,
                           const TaskTab& tt, int64_t items) {
  switch (nk) {
#define C(n) \
  case n:    \
    return f64 ? cpencil<double, n>(variant, a, max_blocks, s, tt, items) \
               : cpencil<float, n>(variant, a, max_blocks, s, tt, items);
    KX_CNK_CASES(C)
#undef C
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_slice_inv_c(bool f64, int nk, int variant, const AccArgs& a, int64_t items,
                              int max_blocks, hipStream_t s, const TaskTab& tt) {
  const int base = variant & ~TUNE_ALT;
  if (base != SI_ACC12 && base != SI_ST12) return hipErrorInvalidValue;
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
