// FP64 instantiation: v_mfma_f64_16x16x4, fused and plain paths.
#define KX_T double
#define KX_SUFFIX f64
#define KX_PLAIN 1
#include "instantiate.inc"

namespace kx {

thread_local int64_t* g_grid_probe = nullptr;

hipError_t launch_scale_f64(double* T, int64_t ld, int npairs, int64_t N, const double* ftab,
                            hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  const int grid = 8 * device_cu_count();
  hipLaunchKernelGGL(k_scale<double>, dim3(grid), dim3(256), 0, s, T, ld, npairs, N, ftab);
  return hipGetLastError();
}

hipError_t launch_accumulate_f64(const AccArgs& a, int blocks_per_target, hipStream_t s) {
  if (a.n_t <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_accumulate<double>, dim3(blocks_per_target, a.n_t), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace kx
