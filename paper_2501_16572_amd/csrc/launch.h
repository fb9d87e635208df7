// Launchers for the templated kernels (one translation unit per element type).
#pragma once

#include "kernels.h"

namespace kx {

// K-step counts with compiled kernels; an axis of length n uses the smallest
// NK with 4*NK >= n (the eigenvector matrices are zero-padded).
static const int kNKList[] = {6, 8, 12, 14, 16, 18, 20, 24, 28, 30, 32, 36, 40};
static const int kNKCount = sizeof(kNKList) / sizeof(kNKList[0]);
static const int kMaxAxis = 160;

inline int pick_nk(int n) {
  for (int i = 0; i < kNKCount; ++i)
    if (4 * kNKList[i] >= n) return kNKList[i];
  return -1;
}
inline int padded_len(int nk) { return 16 * ((nk + 3) / 4); }

enum SliceFwdVariant { SF_PAIR12 = 0, SF_LOAD12, SF_PAIR, SF_LOAD1, SF_LOAD2 };
// OR-ed into a fused variant by the autotuner: TUNE_ALT selects the
// alternative occupancy target of the same kernel, TUNE_TR the transposed
// mode-2 product of the slice passes (x1 along the MFMA columns).
// TUNE_VL selects the pass-B / pass-C kernels with the eigenvector matrices
// resident in LDS (where they fit; elsewhere the streamed kernel runs).
// TUNE_RH selects the register hand-off kernels (the second product of a
// pass takes the first one's accumulators as its operand; kernels_rh.inc).
enum { TUNE_ALT = 64, TUNE_TR = 128, TUNE_VL = 256, TUNE_RH = 512 };
enum PencilVariant { PC_FSI = 0, PC_F, PC_I };
enum SliceInvVariant { SI_ACC12 = 0, SI_ST12, SI_ST2, SI_ST1 };

// Each launcher picks a persistent grid of at most `max_blocks` blocks
// (0 = as many as are co-resident on the device) for `items` work items and
// returns the HIP status of the launch.  With a task table (tt.ntasks > 0)
// the launch runs every batch of the table, `a` is ignored, and `items` is
// the table's total item count (for the pencil launchers: the sum over
// entries of nchunks * npairs).
constexpr TaskTab kNoTasks{nullptr, nullptr, 0};
hipError_t launch_slice_fwd_f64(int nk, int variant, const SliceArgs& a, int64_t items,
                                int max_blocks, hipStream_t s, const TaskTab& tt = kNoTasks);
hipError_t launch_pencil_f64(int nk, int variant, const PencilArgs& a, int max_blocks,
                             hipStream_t s, const TaskTab& tt = kNoTasks, int64_t items = 0);
hipError_t launch_slice_inv_f64(int nk, int variant, const AccArgs& a, int64_t items,
                                int max_blocks, hipStream_t s, const TaskTab& tt = kNoTasks);
hipError_t launch_slice_fwd_f32(int nk, int variant, const SliceArgs& a, int64_t items,
                                int max_blocks, hipStream_t s, const TaskTab& tt = kNoTasks);
hipError_t launch_pencil_f32(int nk, int variant, const PencilArgs& a, int max_blocks,
                             hipStream_t s, const TaskTab& tt = kNoTasks, int64_t items = 0);
hipError_t launch_slice_inv_f32(int nk, int variant, const AccArgs& a, int64_t items,
                                int max_blocks, hipStream_t s, const TaskTab& tt = kNoTasks);
hipError_t launch_scale_f64(double* T, int64_t ld, int npairs, int64_t N, const double* ftab,
                            hipStream_t s);
hipError_t launch_accumulate_f64(const AccArgs& a, int blocks_per_target, hipStream_t s);
hipError_t launch_ex_finalize(const double* partials, int n_t, int per_target,
                              const double* gphi, double dV, double* ex, hipStream_t s);

// Split-BF16 launchers (spl = 2 for BF16X3, 3 for BF16X6; nt = 16-wide tiles
// per padded axis).  vps: element stride between the split parts of one
// eigenvector operand; kpv: its K padding (32 * ceil(nt / 2)).
hipError_t launch_slice_fwd_bf(int spl, int nt, int variant, const SliceArgs& a, int64_t items,
                               int max_blocks, int vps, int kpv, hipStream_t s,
                               const TaskTab& tt = kNoTasks);
hipError_t launch_pencil_bf(int spl, int nt, const PencilArgs& a, int max_blocks, int vps, int kpv,
                            hipStream_t s, const TaskTab& tt = kNoTasks, int64_t items = 0);
hipError_t launch_slice_inv_bf(int spl, int nt, int variant, const AccArgs& a, int64_t items,
                               int max_blocks, int vps, int kpv, hipStream_t s,
                               const TaskTab& tt = kNoTasks);
inline int bf_nt(int n) { return (n + 15) / 16; }
inline int bf_kp(int nt) { return 32 * ((nt + 1) / 2); }
inline int bf_lines(int nt) { return 16 * nt > bf_kp(nt) ? 16 * nt : bf_kp(nt); }

// Complex (Bloch) launchers: f64 selects complex128 data (else complex64).
// V arguments point at (re, im) planes, each P x P.
hipError_t launch_slice_fwd_c(bool f64, int nk, int variant, const SliceArgs& a, int64_t items,
                              int max_blocks, hipStream_t s, const TaskTab& tt = kNoTasks);
hipError_t launch_pencil_c(bool f64, int nk, int variant, const PencilArgs& a, int max_blocks, hipStream_t s,
                           const TaskTab& tt = kNoTasks, int64_t items = 0);
hipError_t launch_slice_inv_c(bool f64, int nk, int variant, const AccArgs& a, int64_t items,
                              int max_blocks, hipStream_t s, const TaskTab& tt = kNoTasks);

// ACE kernels (kernels_ace.hip); cplx selects complex128, else FP64.
//   gram:  C(m x n, ld m) = alpha * sum_k conj(A[k, i]) B[k, j] over K rows,
//          split in chunks of kc rows; part holds ceil(K/kc) * m * n elements
//   potrf: lower Cholesky factor of S (n x n) in place; *info = 0 or j+1
//   trtri: U = L^{-H} (upper), X = L^{-1} scratch, both n x n; skipped if *info
//   tsmm:  C(K x n) = beta C + alpha A(K x m) B(m x n, ld m); skipped if info && *info
// Bytes of split-K partials launch_ace_gram needs for a K x m by K x n product.
int64_t ace_gram_part_bytes(bool cplx, int64_t K, int m, int n);
hipError_t launch_ace_gram(bool cplx, int64_t K, int m, int n, const void* A, int64_t lda, const void* B,
                           int64_t ldb, double alpha, void* part, void* C, hipStream_t s);
// Cholesky factor and inverse of the Hermitian n x n S: S = L L^H, U = L^{-H}; X is n x n scratch for orders above the
// LDS-resident kernel's limit; *info = 0 or the failing pivot (1-based).
hipError_t launch_ace_factor(bool cplx, int n, void* S, void* U, void* X, int* info, hipStream_t s);
hipError_t launch_ace_tsmm(bool cplx, int64_t K, int m, int n, const void* A, int64_t lda, const void* B,
                           double alpha, double beta, void* C, int64_t ldc, const int* info, hipStream_t s);

// C(m x n) = A(m x k) B(k x n), FP64 column-major: one small GEMM of the
// slice-wise (Sec. II.A) solve.
hipError_t launch_gemm_nn_f64(int m, int n, int k, const double* A, int64_t lda, const double* B, int64_t ldb,
                              double* C, int64_t ldc, hipStream_t s);

// Number of compute units of the current device (cached).
int device_cu_count();

// Work-queue kernel of the batched entry point (kernels_queue.hip).
// queue_shape: the instantiated tile counts covering real plans of up to
// nk_real K steps and complex plans of up to nk_cplx (false: none);
// queue_grid: its co-resident blocks on the device; launch_queue: a counter
// reset kernel, then the queue over `grid` blocks.
bool queue_shape(int nk_real, int nk_cplx, int* nkr, int* nkc);
int queue_grid(bool f64, int nkr, int nkc);
hipError_t launch_queue(bool f64, int nkr, int nkc, const QueueArgs& q, int grid, hipStream_t s);

// When non-null, the inverse-slice (pass C) launchers store in *g_grid_probe
// the grid they would launch for the given item count and launch nothing
// (the batch-size choice asks how many pass-C blocks are resident at once).
extern thread_local int64_t* g_grid_probe;

}  // namespace kx
