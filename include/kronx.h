/*
 * kronx -- exact-exchange application Vx.psi on one AMD MI355X (gfx950)
 * through a batched Kronecker-product Poisson solver.
 *
 * Operation (arXiv 2501.16572):
 *   Eq. (Vx:Poisson)  Vx phi_n = - sum_m w g_m psi_m (.) phi_mn, where
 *   Eq. (Poisson)     -(1/4 pi) L phi_mn = conj(psi_m) (.) phi_n   (unscreened), or
 *   Eq. (Poisson:SR)  the screened counterpart (erfc(omega r)/r interaction),
 *   solved as Eq. (LS:Discrete:Solution) X = f(L) B with f of Eq. (fL) and the
 *   Kronecker eigendecomposition of Eq. (FinalRepfL), L = (V1 (x) V2 (x) V3)
 *   Lambda (...)^H, applied to a batch of right-hand sides at once (Sec. II.B).
 *   The screened kernel is f(lambda) = -(4 pi/lambda)(1 - exp(lambda/(4 omega^2)))
 *   (the erfc(omega r)/r interaction; the exponent printed in Eq. (fL) is
 *   read this way), with the zero mode f(0) = pi/omega^2; unscreened
 *   f(lambda) = -4 pi/lambda with f(0) = 0 (zero-mean solution).
 *
 * Conventions shared by every call:
 *   - Grid: n1 x n2 x n3 uniform points, flat index i1 + n1*(i2 + n2*i3) (x1
 *     fastest; B(:,:,k) is the k-th frontal slice, Sec. II.A).  Units: bohr,
 *     Hartree.
 *   - A set of grid functions is column-major: column j starts at
 *     base + j*ld elements, ld >= N = n1*n2*n3.
 *   - Element types follow the plan's precision: KX_PREC_FP64 -> double;
 *     KX_PREC_FP32 / KX_PREC_BF16X3 / KX_PREC_BF16X6 -> float.  Plans with a
 *     nonzero Bloch wavevector are complex: interleaved (re, im) pairs of that
 *     type.  Outputs of exx_apply are always double (complex: (re, im)
 *     doubles): they accumulate in FP64.
 *   - Pointers named d_* are device pointers (hipMalloc'd or torch CUDA
 *     tensors) owned by the caller; the library never frees them.  Host
 *     pointers are read during the call only.
 *   - Every call that takes a stream enqueues work on that hipStream_t (passed
 *     as void*; NULL = the default stream) and returns without waiting.
 *   - Errors: every call returns a kx_status.  Argument errors are detected
 *     before any work is enqueued (nothing is modified).  A device error
 *     surfaces as KX_EDEVICE from the call that observes it.  kx_last_error()
 *     returns this thread's text for the last non-OK status.  No call aborts
 *     or throws across this boundary.
 */
#ifndef KRONX_H
#define KRONX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kx_plan_s* kx_plan;

typedef enum {
  KX_OK = 0,
  KX_EINVAL = 1,        /* invalid argument (null pointer, bad size, ld < N, ...) */
  KX_EUNSUPPORTED = 2,  /* valid but not implemented (e.g. an axis longer than 160) */
  KX_ENOMEM = 3,        /* device or host allocation failed */
  KX_EDEVICE = 4,       /* HIP runtime error */
  KX_ESTATE = 5         /* call not valid in the current state */
} kx_status;

/* Boundary condition per axis (Sec. II): periodic (Bloch-periodic when the
 * axis' component of the wavevector k - q is nonzero) along extended
 * directions, zero Dirichlet along vacuum directions (n interior nodes, the
 * wall one spacing beyond each end node). */
enum { KX_BC_PERIODIC = 0, KX_BC_DIRICHLET = 1 };

/* Arithmetic of the mode products (the dense matrix products of Sec. II.B).
 * The 1D eigendecompositions, the f(Lambda~) table, the eigen-scaling
 * multiply, the Vx accumulation and the E_x reduction are FP64 in all modes.
 *   FP64   : FP64 MFMA, FP64 intermediates.
 *   FP32   : FP32 MFMA with FP32 accumulation, FP32 intermediates.
 *   BF16X3 : each FP32 operand split into bf16 hi + lo; hi*hi + hi*lo + lo*hi
 *            on bf16 MFMA with FP32 accumulation.
 *   BF16X6 : three-way split hi + mid + lo, the six products down to
 *            relative weight 2^-16. */
enum { KX_PREC_FP64 = 0, KX_PREC_FP32 = 1, KX_PREC_BF16X3 = 2, KX_PREC_BF16X6 = 3 };

/* OR-ed into kron_setup's prec: complex data even when k - q = 0 (the k = q
 * blocks of a k-point calculation, whose orbitals are complex Bloch functions
 * although the pair problem is plain periodic).  Complex plans run in FP64
 * (complex128) or FP32 (complex64). */
enum { KX_FLAG_COMPLEX = 16 };

/* Kernel organisation for exx_apply / kron_solve.
 *   FUSED : three passes per batch -- (A) pair density + mode-1 + mode-2
 *           forward on frontal slices, (B) mode-3 forward, eigen-scaling,
 *           mode-3 inverse on x3 pencils, (C) mode-2 + mode-1 inverse, the
 *           psi_m product and the accumulation into Vx, with E_x partials.
 *   PLAIN : one kernel per step (pair density, three forward mode products,
 *           scaling, three inverse mode products, accumulation), each a full
 *           pass over the batch in device memory.  FP64 only.
 *   SLICEWISE (kron_solve only): the original formalism of Sec. II.A, one
 *           right-hand side at a time and one small GEMM per frontal slice
 *           for modes 1 and 2 (4 n3 + 2 GEMM launches per solve); the
 *           comparison point for the batched solve.  FP64, real plans only. */
enum { KX_PATH_FUSED = 0, KX_PATH_PLAIN = 1, KX_PATH_SLICEWISE = 2 };

/* kron_setup -- build a plan for X = f(L) B on one grid (Sec. II.A,
 * Eqs. (fL), (FinalRepfL)).
 *   n[3]      grid points per axis, 1 <= n_d <= 160.
 *   h[3]      grid spacing per axis (bohr), > 0.
 *   bc[3]     KX_BC_PERIODIC or KX_BC_DIRICHLET per axis.
 *   fd_order  even order of the central second-derivative stencil, 2..16.
 *   omega     screening parameter (bohr^-1); <= 0 selects the unscreened
 *             Coulomb kernel.
 *   kq[3]     Bloch wavevector k - q (bohr^-1) per axis, or NULL for zero.
 *             A nonzero component requires a periodic axis and makes the
 *             plan complex.
 *   prec      KX_PREC_*, optionally | KX_FLAG_COMPLEX.
 *   out       receives the plan.  On error *out is set to NULL.
 * Host-side FP64 work (weights, eigenpairs, f table), then device uploads on
 * the current device (synchronous).  The plan is immutable afterwards and may
 * be used from several streams, but its internal workspace is shared: calls
 * on different streams must not overlap in time. */
kx_status kron_setup(const int n[3], const double h[3], const int bc[3], int fd_order,
                     double omega, const double kq[3], int prec, kx_plan* out);

/* kron_destroy -- release a plan (waits for the device).  NULL is a no-op. */
kx_status kron_destroy(kx_plan p);

/* kron_solve -- X = f(L) B for nrhs right-hand sides (Sec. II.B, Eq.
 * (LS:Discrete:Solution:Block)).
 *   d_B  nrhs columns, leading dimension ldb >= N, plan element type.
 *   d_X  nrhs columns, leading dimension ldx >= N, plan element type;
 *        overwritten.  d_X may not overlap d_B.
 *   path KX_PATH_*; KX_PATH_SLICEWISE uses N doubles of plan-owned
 *        workspace (allocated on first use, KX_ENOMEM if that fails). */
kx_status kron_solve(kx_plan p, const void* d_B, int64_t ldb, void* d_X, int64_t ldx,
                     int nrhs, int path, void* stream);

/* exx_apply -- Vx phi_n for n = 0..n_b-1, Eqs. (Vx:Poisson), (W):
 *   d_vx[:, n] += - sum_{m < n_occ} d_occ[m] * psi_m (.) phi_mn,
 *   phi_mn = f(L) (conj(psi_m) (.) phi_n).
 *   d_psi    occupied orbitals psi_m (at q), n_occ columns, leading dim ld_psi.
 *   d_occ    n_occ doubles (device): the weights w_q * g_mq.
 *   d_phi    the functions the operator is applied to (at k), n_b columns,
 *            leading dim ld_phi.  May alias d_psi.
 *   d_vx     n_b columns of doubles (complex plans: (re, im) doubles),
 *            leading dim ld_vx; ACCUMULATED (+=), so callers may loop over q
 *            and over batches.
 *   d_ex     one device double, ACCUMULATED: += dV * sum_n d_gphi[n] *
 *            Re <phi_n, Delta vx_n>, where Delta vx_n is this call's
 *            contribution; with phi = psi at one k and d_gphi = g_n * w_k this
 *            is the exchange energy E_x = sum_n g_n Re <psi_n, Vx psi_n> dV.
 *            May be NULL (then d_gphi is ignored).
 *   d_gphi   n_b doubles (device) or NULL when d_ex is NULL.
 *   path     KX_PATH_*.
 * Work: n_b * n_occ Poisson solves.  The reduction order is fixed, so two
 * identical calls give bitwise identical results. */
kx_status exx_apply(kx_plan p, const void* d_psi, int64_t ld_psi, int n_occ, const double* d_occ,
                    const void* d_phi, int64_t ld_phi, int n_b, double* d_vx, int64_t ld_vx,
                    double* d_ex, const double* d_gphi, int path, void* stream);

/* exx_apply_static -- exx_apply that allocates nothing, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Arguments, results, layout and
 * errors as exx_apply; the plan's device must be the current device.
 * The pair workspace and the E_x partials live in a fixed device array of
 * kx_static_scratch_bytes() bytes (256 MiB) inside the library: one copy per
 * GPU, held until the process ends, shared by every call on that GPU and
 * keeping the last call's contents (nothing in it needs clearing: each call
 * writes what it reads).  Calls that overlap in time on one GPU (other
 * streams, other threads) race on it: serialize them.  A call whose single
 * target needs more than the array holds, i.e.
 *   max(64, n3) * 8 * n_b (rounded up to 256) + n_occ * N * element bytes
 * above 256 MiB, returns KX_EINVAL before any work.  No hipMalloc, hipFree,
 * memset or trace event. */
kx_status exx_apply_static(kx_plan p, const void* d_psi, int64_t ld_psi, int n_occ,
                           const double* d_occ, const void* d_phi, int64_t ld_phi, int n_b,
                           double* d_vx, int64_t ld_vx, double* d_ex, const double* d_gphi,
                           int path, void* stream);

/* kx_static_scratch_bytes -- size of exx_apply_static's device array. */
size_t kx_static_scratch_bytes(void);

/* One unit of a batched call: an exx_apply with its own plan.  Field
 * meanings are those of exx_apply's arguments. */
typedef struct {
  kx_plan plan;
  const void* d_psi;
  int64_t ld_psi;
  int n_occ;
  const double* d_occ;
  const void* d_phi;
  int64_t ld_phi;
  int n_b;
  double* d_vx;
  int64_t ld_vx;
  double* d_ex;
  const double* d_gphi;
} kx_task;

/* exx_apply_batched -- run ntasks exx_apply units (several k-point pairs and
 * several systems of uneven grid sizes) as one captured HIP graph on
 * `stream` (the batched n_c-style scheduling of Sec. II.B over a whole task
 * list).  Each task is cut into batches of targets as exx_apply does; the
 * batches are scheduled in rounds such that two batches of one plan, or two
 * batches with overlapping d_vx, never share a round (overlapping outputs
 * accumulate in task order).
 *   Work-queue form (FP64 / FP32 plans, real grids up to 120 points per axis
 *   and complex grids up to 80): the graph is a counter reset and ONE
 *   persistent launch in which every block takes tickets (a virtual block of
 *   one pass of one batch, or a batch's E_x finalize) in order and waits on
 *   device counters for what each ticket depends on.  A wait that gives up
 *   (after about half a minute of polling; with KX_QUEUE_SPIN = r set, after
 *   r + 1 polls) ends the launch early with incomplete results and is
 *   reported by kx_batched_check.
 *   Grouped form (otherwise, or with KX_BATCHED=rounds): in each round the
 *   batches of every pass whose plans share a kernel instantiation run as
 *   one persistent launch that walks a task table.
 * The list's plans hold their workspaces at once and share one budget (60 %
 * of the free device memory plus what they hold already, split in
 * proportion to each plan's need for all its targets in one batch; a plan
 * holding far more than its share gives the excess back), or
 * KX_WORKSPACE_MB per plan when set.
 * The first call with a given task list captures the graph (and allocates
 * its tables); later calls with the same plans, pointers and sizes replay
 * it.  All plans must share one precision.  Results are bitwise reproducible
 * across replays. */
kx_status exx_apply_batched(const kx_task* tasks, int ntasks, void* stream);

/* kx_batched_check -- wait for `stream`, then KX_EDEVICE if the last
 * work-queue replay of exx_apply_batched ended early (a dependency wait gave
 * up), else KX_OK. */
kx_status kx_batched_check(void* stream);

/* kx_workspace_bytes -- device bytes that exx_apply (or a batched task) on
 * plan p with n_b targets and n_occ occupied orbitals holds: one batch of
 * pair intermediates (targets per batch x n_occ x N elements of the plan's
 * type; within the workspace limit, 60 % of the free device memory or
 * KX_WORKSPACE_MB, the batch size with the fewest rounds of pass-C items
 * over the persistent grid) plus the E_x partials.  The plan allocates them
 * at its first such call, grows them when a later call needs more (a
 * batched call may also shrink them to its share), and frees them in
 * kron_destroy.  Host only, no allocation.
 * *bytes = 0 when n_b or n_occ is 0. */
kx_status kx_workspace_bytes(kx_plan p, int n_b, int n_occ, int64_t* bytes);

/* kx_graph_cache_info -- state of exx_apply_batched's cache of captured
 * graphs: out[0] = task lists held now, out[1] = the most it holds (8; a new
 * capture beyond that drops the least recently replayed list and frees its
 * graph and device task tables), out[2] = captures so far in this process.
 * A cached list is replayed only when every field of every task matches and
 * no plan of it has reallocated a buffer or been retuned (kx_autotune) since
 * the capture; otherwise it is captured again.  Host only. */
kx_status kx_graph_cache_info(int64_t out[3]);

/* kx_batched_schedule -- shape of the schedule that the last capture of
 * exx_apply_batched in this process built: out[0] = rounds, out[1] = batches
 * (one task contributes ceil(n_b / targets per batch)), out[2] = launches of
 * the three fused passes (1 in the work-queue form), out[3] = the most
 * batches that one launch ran.
 * Host only; all zero before the first capture. */
kx_status kx_batched_schedule(int out[4]);

/* kx_plan_info -- sizes the plan chose (for reports and tests).
 *   out[0..2]  n1, n2, n3           out[3]  complex flag
 *   out[4]     precision            out[5]  padded slice size (x1, x2)
 *   out[6]     padded pencil size (x3)
 *   out[7]     target bands per batch the last exx_apply used (0 before any) */
kx_status kx_plan_info(kx_plan p, int64_t out[8]);

/* kx_plan_tables -- copy the plan's host FP64 tables (no device work).
 *   axis 0..2: lam (n_d doubles, ascending) and the eigenvectors as V[k*n + a]
 *   = component k of eigenvector a (V_re, V_im; V_im may be NULL for real
 *   plans).  axis = 3: lam receives the N-entry f(Lambda~) table in the flat
 *   grid order (V_re, V_im ignored). Any output pointer may be NULL. */
kx_status kx_plan_tables(kx_plan p, int axis, double* lam, double* V_re, double* V_im);

/* kx_host_eig1d -- host only, no device use: the 1D second-derivative
 * operator's eigenpairs exactly as kron_setup computes them (for tests of the
 * host plan).  lam: n doubles; V_re, V_im: n*n doubles each, V[k*n + a]
 * (V_im may be NULL when kappa == 0 or bc is Dirichlet). */
kx_status kx_host_eig1d(int n, double h, int bc, int fd_order, double kappa, double* lam,
                        double* V_re, double* V_im);

/* kx_host_fd_weights -- host only: the weights c_0..c_p (p = fd_order/2) of
 * the central second-derivative stencil, f'' ~ sum_s c_|s| f(x + s h) / h^2. */
kx_status kx_host_fd_weights(int fd_order, double* c);

/* Kernel-level tracing.  While enabled, every kernel the library enqueues
 * outside graph capture is bracketed by two HIP events recorded on its launch
 * stream; kx_trace_read waits for those events and folds the elapsed times
 * into per-kind totals.  Kinds (kx_trace_name gives the text):
 *   0..3   fused exx_apply: pass A, pass B, pass C, E_x finalize
 *   4..12  plain exx_apply: pair density, mode-1/2/3 forward, scaling,
 *          mode-3/2/1 inverse, accumulation
 *   13..15 fused kron_solve: forward slices, pencils, inverse slices
 *   16..21 plain kron_solve: mode-1/2/3 forward, scaling, mode-3/2 inverse
 *   22     plain kron_solve: mode-1 inverse
 * kx_trace_enable(1) clears the totals; kx_trace_enable(0) stops recording.
 * kx_trace_read copies min(nkinds, KX_TRACE_KINDS) totals: ms[k] summed
 * milliseconds, count[k] launches (either pointer may be NULL). */
#define KX_TRACE_KINDS 23
kx_status kx_trace_enable(int on);
kx_status kx_trace_read(double* ms, int64_t* count, int nkinds);
const char* kx_trace_name(int kind);

/* kx_autotune -- choose the launch configuration of the three fused passes
 * for this plan and workload (the batch Kronecker solve's analogue of the
 * batch size n_c, Sec. II.B): for each candidate (variant bits x resident
 * blocks per CU, see kx_plan_tuning) it runs passes A, B, C on the first
 * batch that exx_apply would make of the given data (as many target columns
 * as the workspace holds), times every pass with HIP events, and keeps the
 * fastest candidate per pass in the plan (later exx_apply calls on any
 * stream use it).  Arguments as exx_apply; nothing the caller owns is written
 * (a private Vx buffer of one batch receives the results).  Synchronous;
 * costs two batches of device time per candidate (24 candidates for real
 * FP64 plans, 28 for real FP32 plans, 10 for complex plans, 5 for
 * split-BF16 plans, which tune the resident blocks per CU only), once per
 * key.  If the environment variable
 * KX_TUNE_CACHE names a file, choices are read from and appended to it (one
 * line per key: arch, grid, precision, complex flag, n_occ), and a cached key
 * skips the timing. */
kx_status kx_autotune(kx_plan p, const void* d_psi, int64_t ld_psi, int n_occ, const double* d_occ,
                      const void* d_phi, int64_t ld_phi, int n_b, void* stream);

/* kx_plan_tuning -- the plan's current launch configuration per fused pass:
 * out[2*i] = variant bits (bit 0: alternative occupancy target, real and
 * complex plans; bit 1, passes A and C: mode-2 product computed transposed,
 * x1 along the MFMA columns; bit 2, passes B and C: eigenvector matrices
 * resident in LDS, the next work item's data prefetched into registers; it
 * overrides bits 0 and 1; bit 3: register hand-off, the second product of
 * the pass taking the first one's accumulators as its operand; it
 * overrides bits 0-2; bit 4, real FP32 plans: the pass runs the six-product
 * split-BF16 kernel, which keeps the FP32 accuracy class; it overrides the
 * others), out[2*i+1] = resident blocks per CU (0 = as many as fit), for
 * passes i = A, B, C; out[6] = 1 if it came from kx_autotune (timed or
 * cached). */
kx_status kx_plan_tuning(kx_plan p, int out[7]);

/* ---- Adaptively compressed exchange (ACE) --------------------------------
 * FP64 (cplx = 0, real orbitals at Gamma) or complex128 (cplx = 1, interleaved
 * (re, im)).  Orbital sets are column-major N x n (one orbital per column,
 * leading dimension >= N); dV is the grid's volume element, so inner products
 * are <a, b> = dV sum conj(a) b.  Every call is asynchronous on `stream` and
 * needs a caller-owned device workspace (256-byte aligned) of at least
 * kx_ace_workspace_bytes bytes; nothing is allocated.  Argument errors:
 * KX_EINVAL before any device work. */

/* kx_ace_workspace_bytes -- workspace for ace_construct (n_phi = 0) or
 * ace_apply on n_phi trial orbitals, for N grid points and n_s orbitals
 * (1 <= n_s <= 1024).  A workspace sized with n_phi > 0 serves both calls.
 * It holds the split-K partials of the Gram products (about 512 x 128 KiB,
 * fixed by the sizes, not by the device) and the n_s x n_s matrices.  Host
 * only. */
kx_status kx_ace_workspace_bytes(int64_t N, int n_s, int n_phi, int cplx, int64_t* bytes);

/* ace_construct -- the ACE operator of Sec. III.A from n_s orbitals Psi and
 * W = Vx Psi (e.g. exx_apply with phi = Psi): M = dV Psi^H W (Hermitian,
 * negative definite), -M = L L^H (lower Cholesky factor),
 * xi = W L^{-H} (N x n_s, written to d_xi; the operator is -xi xi^H dV).
 * d_info: one device int, set to 0, or to j+1 if the j-th pivot of -M is not
 * positive (then d_xi is left unspecified); read it after synchronizing.
 * Results are bitwise reproducible: every sum runs in a fixed order. */
kx_status ace_construct(int64_t N, int n_s, int cplx, double dV, const void* d_psi, int64_t ld_psi,
                        const void* d_w, int64_t ld_w, void* d_xi, int64_t ld_xi, void* d_work,
                        int64_t work_bytes, int* d_info, void* stream);

/* ace_apply -- the compressed operator on n_phi trial orbitals (Sec. III.B):
 * chi = dV xi^H Phi (n_s x n_phi), then d_vphi += -xi chi (ACCUMULATES, like
 * exx_apply).  n_phi = 0 is a no-op. */
kx_status ace_apply(int64_t N, int n_s, int cplx, double dV, const void* d_xi, int64_t ld_xi,
                    const void* d_phi, int64_t ld_phi, int n_phi, void* d_vphi, int64_t ld_vphi, void* d_work,
                    int64_t work_bytes, void* stream);

/* kx_last_error -- text for this thread's last non-OK status ("" if none).
 * The pointer stays valid until the next call on this thread. */
const char* kx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KRONX_H */
