// C ABI of the library: plans, exx_apply, kron_solve, batched graph replay.
//
// Work per exx_apply (arXiv 2501.16572, Eq. (Vx:Poisson) with the batch
// Kronecker solve of Sec. II.B): the n_b x n_occ pair solves are cut into
// batches of n_t target columns x all n_occ occupied columns; one batch's
// pair intermediates live in a plan-owned device workspace and go through
//   pass A  pair density + forward modes 1, 2        (k_slice_fwd)
//   pass B  forward mode 3, f(Lambda~), inverse mode 3 (k_pencil)
//   pass C  inverse modes 2, 1, psi_m product, Vx accumulation, E_x partials
//   finalize  fixed-order FP64 reduction of the E_x partials into *ex.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/kronx.h"
#include "launch.h"
#include "plan_host.h"
#include "queue_plan.h"

namespace {

thread_local std::string g_err;

kx_status fail(kx_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

kx_status dev_fail(hipError_t e, const char* what) {
  return fail(KX_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int elem_bytes(int prec) { return prec == KX_PREC_FP64 ? 8 : 4; }

}  // namespace

namespace kx {

int device_cu_count() {
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (cache[dev] == 0) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1)
      cu = 1;
    cache[dev] = cu;
  }
  return cache[dev];
}

// *ex += dV * sum_t gphi[t] * sum_j partials[t*per_target + j], fixed order.
__global__ void __launch_bounds__(256)
k_ex_finalize(const double* partials, int n_t, int per_target, const double* gphi, double dV,
              double* ex) {
  __shared__ double red[256];
  double s = 0.0;
  const int total = n_t * per_target;
  for (int i = threadIdx.x; i < total; i += blockDim.x) s += gphi[i / per_target] * partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *ex += dV * red[0];
}

hipError_t launch_ex_finalize(const double* partials, int n_t, int per_target, const double* gphi,
                              double dV, double* ex, hipStream_t s) {
  hipLaunchKernelGGL(k_ex_finalize, dim3(1), dim3(256), 0, s, partials, n_t, per_target, gphi, dV,
                     ex);
  return hipGetLastError();
}

}  // namespace kx

// ---------------------------------------------------------------------------
// Kernel tracing (HIP events around each launch, outside graph capture).
// ---------------------------------------------------------------------------
namespace {

enum TraceKind {
  TK_A = 0, TK_B, TK_C, TK_FIN,
  TK_P_PAIR, TK_P_M1F, TK_P_M2F, TK_P_M3F, TK_P_SCALE, TK_P_M3I, TK_P_M2I, TK_P_M1I, TK_P_ACC,
  TK_S_A, TK_S_B, TK_S_C,
  TK_SP_M1F, TK_SP_M2F, TK_SP_M3F, TK_SP_SCALE, TK_SP_M3I, TK_SP_M2I, TK_SP_M1I,
  TK_COUNT
};
static_assert(TK_COUNT == KX_TRACE_KINDS, "trace kinds");
const char* const kTraceNames[TK_COUNT] = {
    "exx_fused_passA", "exx_fused_passB", "exx_fused_passC", "exx_ex_finalize",
    "exx_plain_pair_density", "exx_plain_mode1_fwd", "exx_plain_mode2_fwd", "exx_plain_mode3_fwd",
    "exx_plain_scale", "exx_plain_mode3_inv", "exx_plain_mode2_inv", "exx_plain_mode1_inv",
    "exx_plain_accumulate",
    "solve_fused_passA", "solve_fused_passB", "solve_fused_passC",
    "solve_plain_mode1_fwd", "solve_plain_mode2_fwd", "solve_plain_mode3_fwd", "solve_plain_scale",
    "solve_plain_mode3_inv", "solve_plain_mode2_inv", "solve_plain_mode1_inv"};

struct TraceRec {
  int kind;
  hipEvent_t a, b;
};
std::mutex g_tr_mu;
bool g_trace_on = false;
std::vector<TraceRec> g_tr_pending;
double g_tr_ms[TK_COUNT];
int64_t g_tr_n[TK_COUNT];

// Launch `fn` (returning hipError_t) on stream s, bracketed by events when
// tracing is on and s is not being captured.
template <typename F>
hipError_t traced(int kind, hipStream_t s, F fn) {
  bool on;
  {
    std::lock_guard<std::mutex> lock(g_tr_mu);
    on = g_trace_on;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (on && hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
    TraceRec r{kind, nullptr, nullptr};
    if (hipEventCreate(&r.a) == hipSuccess && hipEventCreate(&r.b) == hipSuccess) {
      hipEventRecord(r.a, s);
      hipError_t e = fn();
      hipEventRecord(r.b, s);
      std::lock_guard<std::mutex> lock(g_tr_mu);
      g_tr_pending.push_back(r);
      return e;
    }
  }
  return fn();
}

}  // namespace

struct kx_graph_entry {
  std::vector<kx_task> tasks;
  std::vector<unsigned> generations;  // generation of each task's plan at capture
  hipStream_t stream;
  hipGraph_t graph;
  hipGraphExec_t exec;
  void* d_tables;                     // task tables of the grouped launches (device)
  uint64_t last_use;                  // replay clock of the last capture or replay
  unsigned* d_err = nullptr;          // the work queue's error flag (queue form), in d_tables
};

// Error flag and stream of the last work-queue replay (kx_batched_check).
unsigned* g_last_err = nullptr;
hipStream_t g_last_err_stream = nullptr;

void destroy_graph_entry(kx_graph_entry& g) {
  if (g.d_err && g.d_err == g_last_err) g_last_err = nullptr;
  if (g.exec) hipGraphExecDestroy(g.exec);
  if (g.graph) hipGraphDestroy(g.graph);
  if (g.d_tables) hipFree(g.d_tables);
  g.exec = nullptr;
  g.graph = nullptr;
  g.d_tables = nullptr;
}

struct kx_plan_s {
  int n[3];
  double h[3];
  int bc[3];
  int order;
  double omega;
  double kq[3];
  int prec;
  bool cplx;
  int64_t N;
  int n12;
  double dV;
  std::vector<double> lam[3], Vre[3], Vim[3], f;
  int nk12, nk3, P12, P3;
  int device;
  void* dVmat[3] = {nullptr, nullptr, nullptr};   // padded V_d, V[k*P + a]
  void* dVmatT[3] = {nullptr, nullptr, nullptr};  // padded V_d^T
  // split-BF16 eigenvector parts, [c][k] with K contiguous:
  // [d][0] = split(V_d^T) (forward products), [d][1] = split(V_d) (inverse)
  void* dVbf[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  int bf_nt12 = 0, bf_nt3 = 0, bf_vps12 = 0, bf_vps3 = 0, bf_kp12 = 0, bf_kp3 = 0;
  double* d_f = nullptr;
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  double* d_part = nullptr;
  size_t part_bytes = 0;
  int last_nt = 0;
  int max_blocks = 0;    // 0: as many as are co-resident
  // Bumped whenever a device buffer is reallocated or the launch
  // configuration changes (kx_autotune): graphs captured at an older
  // generation hold stale pointers or configurations and are captured again.
  unsigned gen = 0;
  // launch configuration per fused pass (A, B, C): occupancy variant and
  // resident blocks per CU (0 = all that fit); set by kx_autotune
  int tune_tv[3] = {0, 0, 0};
  int tune_bpc[3] = {0, 0, 0};
  bool tuned = false;
};

namespace {

std::mutex g_graph_mu;
std::vector<kx_graph_entry> g_graphs;
// At most this many captured task lists are kept; the least recently
// replayed one is dropped to make room for a new capture.
constexpr size_t kGraphCacheCap = 8;
uint64_t g_graph_clock = 0;
uint64_t g_graph_captures = 0;

bool same_task(const kx_task& a, const kx_task& b) {
  return a.plan == b.plan && a.d_psi == b.d_psi && a.ld_psi == b.ld_psi && a.n_occ == b.n_occ &&
         a.d_occ == b.d_occ && a.d_phi == b.d_phi && a.ld_phi == b.ld_phi && a.n_b == b.n_b &&
         a.d_vx == b.d_vx && a.ld_vx == b.ld_vx && a.d_ex == b.d_ex && a.d_gphi == b.d_gphi;
}

size_t workspace_limit() {
  const char* env = std::getenv("KX_WORKSPACE_MB");
  if (env && *env) {
    long long mb = std::atoll(env);
    if (mb > 0) return (size_t)mb << 20;
  }
  // 60 % of the free device memory: on a 288 GB device a whole band block
  // of a 120^3 FP64 workload (32 targets x 320 occupied, 141 GB) fits one
  // batch, which the pass-C item count needs to fill the chip evenly
  size_t free_b = 0, total_b = 0;
  size_t lim = (size_t)4 << 30;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) lim = free_b / 5 * 3;
  return std::max(lim, (size_t)64 << 20);
}

// Device buffer of at least `need` bytes; with shrink, one holding more than
// 5/4 of it (and 64 MiB more) is given back and allocated again at `need`.
kx_status ensure_buffer(void** ptr, size_t* have, size_t need, const char* what, bool shrink = false) {
  const bool oversized = shrink && *have > need / 4 * 5 + ((size_t)64 << 20);
  if (*have >= need && *ptr && !oversized) return KX_OK;
  if (*ptr) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return dev_fail(e, "synchronize before regrow");
    hipFree(*ptr);
    *ptr = nullptr;
    *have = 0;
  }
  hipError_t e = hipMalloc(ptr, need);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return fail(KX_ENOMEM, "cannot allocate %zu bytes of %s", need, what);
  }
  *have = need;
  return KX_OK;
}

void free_plan_device(kx_plan p) {
  for (int d = 0; d < 3; ++d) {
    if (p->dVmat[d]) hipFree(p->dVmat[d]);
    if (p->dVmatT[d]) hipFree(p->dVmatT[d]);
    for (int k = 0; k < 2; ++k)
      if (p->dVbf[d][k]) hipFree(p->dVbf[d][k]);
  }
  if (p->d_f) hipFree(p->d_f);
  if (p->d_ws) hipFree(p->d_ws);
  if (p->d_part) hipFree(p->d_part);
}

// Checks shared by exx_apply and the batched form.  Returns KX_OK if valid.
kx_status check_exx_args(kx_plan p, const void* psi, int64_t ld_psi, int n_occ, const double* occ,
                         const void* phi, int64_t ld_phi, int n_b, double* vx, int64_t ld_vx,
                         double* ex, const double* gphi, int path) {
  if (!p) return fail(KX_EINVAL, "exx_apply: plan is NULL");
  if (n_occ < 0 || n_b < 0) return fail(KX_EINVAL, "exx_apply: negative n_occ (%d) or n_b (%d)", n_occ, n_b);
  if (path != KX_PATH_FUSED && path != KX_PATH_PLAIN)
    return fail(KX_EINVAL, "exx_apply: unknown path %d", path);
  if (path == KX_PATH_PLAIN && p->prec != KX_PREC_FP64)
    return fail(KX_EUNSUPPORTED, "exx_apply: the plain path is FP64 only");
  if (n_occ == 0 || n_b == 0) return KX_OK;
  if (!psi || !occ || !phi || !vx) return fail(KX_EINVAL, "exx_apply: NULL data pointer");
  if (ex && !gphi) return fail(KX_EINVAL, "exx_apply: d_ex given without d_gphi");
  if (ld_psi < p->N || ld_phi < p->N || ld_vx < p->N)
    return fail(KX_EINVAL, "exx_apply: leading dimension below N = %lld", (long long)p->N);
  const size_t eb = elem_bytes(p->prec) * (p->cplx ? 2 : 1);
  if (((uintptr_t)psi % eb) || ((uintptr_t)phi % eb) || ((uintptr_t)vx % 8) || ((uintptr_t)occ % 8))
    return fail(KX_EINVAL, "exx_apply: misaligned pointer");
  if (p->cplx && path == KX_PATH_PLAIN)
    return fail(KX_EUNSUPPORTED, "exx_apply: the plain path is real (Gamma) only");
  return KX_OK;
}

// Precision dispatch of the three fused passes.
bool is_bf(const kx_plan p) { return p->prec == KX_PREC_BF16X3 || p->prec == KX_PREC_BF16X6; }
int bf_spl(const kx_plan p) { return p->prec == KX_PREC_BF16X3 ? 2 : 3; }
// Pass `pass` of plan p runs the split-BF16 kernels: every pass of a
// split-BF16 plan, and a pass of a real FP32 plan whose tuned variant has
// bit 16 -- the six-product split, in the accuracy class of FP32 (both keep
// the pair intermediates in FP32 storage and accumulate in FP32), which is
// the faster kernel on some passes.
bool pass_bf(const kx_plan p, int pass) {
  return is_bf(p) || (!p->cplx && p->prec == KX_PREC_FP32 && (p->tune_tv[pass] & 16));
}

int tuned_blocks(const kx_plan p, int pass) {
  return p->tune_bpc[pass] > 0 ? p->tune_bpc[pass] * kx::device_cu_count() : p->max_blocks;
}
// Launch variant bits of pass `pass` (bit 0: alternative occupancy target;
// bit 1: transposed mode-2 product, passes A and C; bit 2: eigenvector
// matrices resident in LDS, passes B and C; bit 3: register hand-off, all
// passes) for the FP64/FP32 real kernels; the complex kernels take bit 0
// (a higher occupancy target), the split-BF16 kernels have one variant.
int tuned_variant(const kx_plan p, int pass, int variant) {
  const bool real_mfma = !p->cplx && (p->prec == KX_PREC_FP64 || p->prec == KX_PREC_FP32);
  if (p->cplx) return (p->tune_tv[pass] & 1) ? (variant | kx::TUNE_ALT) : variant;
  if (!real_mfma) return variant;
  const int bits = p->tune_tv[pass];
  if (bits & 8) return variant | kx::TUNE_RH;
  if ((bits & 4) && pass != 0) return variant | kx::TUNE_VL;
  if (bits & 1) variant |= kx::TUNE_ALT;
  if ((bits & 2) && pass != 1) variant |= kx::TUNE_TR;
  return variant;
}

// The argument structs as the kernels of plan p read them: the split-BF16
// kernels (bf) take the split eigenvector parts in place of the matrices.
kx::SliceArgs kernel_args_a(const kx_plan p, kx::SliceArgs A, bool bf) {
  if (bf && !p->cplx) {
    A.V1 = p->dVbf[0][0];
    A.V2 = p->dVbf[1][0];
  }
  return A;
}
kx::PencilArgs kernel_args_b(const kx_plan p, kx::PencilArgs B, bool bf) {
  if (bf && !p->cplx) {
    B.V3 = p->dVbf[2][0];
    B.V3T = p->dVbf[2][1];
  }
  return B;
}
kx::AccArgs kernel_args_c(const kx_plan p, kx::AccArgs C, bool bf) {
  if (bf && !p->cplx) {
    C.V1 = p->dVbf[0][1];
    C.V2 = p->dVbf[1][1];
  }
  return C;
}

// The three fused passes for plan p.  With a task table (tt.ntasks > 0) the
// launch runs every entry of the table (all of them batches of plans with
// p's kernel instantiation, see launch_key) and `items` is the table's total.
hipError_t launch_pass_a(kx_plan p, int variant, const kx::SliceArgs& A0, int64_t items, hipStream_t s,
                         const kx::TaskTab& tt = kx::kNoTasks) {
  using namespace kx;
  const int mb = tuned_blocks(p, 0);
  const bool bf = pass_bf(p, 0);
  const SliceArgs A = kernel_args_a(p, A0, bf);
  if (bf) variant &= ~(kx::TUNE_ALT | kx::TUNE_TR | kx::TUNE_VL | kx::TUNE_RH);
  else if (variant == SF_PAIR12) variant = tuned_variant(p, 0, variant);
  if (p->cplx) return launch_slice_fwd_c(p->prec == KX_PREC_FP64, p->nk12, variant, A, items, mb, s, tt);
  if (!bf && p->prec == KX_PREC_FP64) return launch_slice_fwd_f64(p->nk12, variant, A, items, mb, s, tt);
  if (!bf && p->prec == KX_PREC_FP32) return launch_slice_fwd_f32(p->nk12, variant, A, items, mb, s, tt);
  return launch_slice_fwd_bf(bf_spl(p), p->bf_nt12, variant & ~kx::TUNE_ALT, A, items, mb, p->bf_vps12,
                             p->bf_kp12, s, tt);
}

hipError_t launch_pass_b(kx_plan p, const kx::PencilArgs& B0, hipStream_t s,
                         const kx::TaskTab& tt = kx::kNoTasks, int64_t items = 0) {
  using namespace kx;
  const int mb = tuned_blocks(p, 1), v = tuned_variant(p, 1, PC_FSI);
  const bool bf = pass_bf(p, 1);
  const PencilArgs B = kernel_args_b(p, B0, bf);
  if (p->cplx) return launch_pencil_c(p->prec == KX_PREC_FP64, p->nk3, v, B, mb, s, tt, items);
  if (!bf && p->prec == KX_PREC_FP64) return launch_pencil_f64(p->nk3, v, B, mb, s, tt, items);
  if (!bf && p->prec == KX_PREC_FP32) return launch_pencil_f32(p->nk3, v, B, mb, s, tt, items);
  return launch_pencil_bf(bf_spl(p), p->bf_nt3, B, mb, p->bf_vps3, p->bf_kp3, s, tt, items);
}

hipError_t launch_pass_c(kx_plan p, int variant, const kx::AccArgs& C0, int64_t items, hipStream_t s,
                         const kx::TaskTab& tt = kx::kNoTasks) {
  using namespace kx;
  const int mb = tuned_blocks(p, 2);
  const bool bf = pass_bf(p, 2);
  const AccArgs C = kernel_args_c(p, C0, bf);
  if (bf) variant &= ~(kx::TUNE_ALT | kx::TUNE_TR | kx::TUNE_VL | kx::TUNE_RH);
  else if (variant == SI_ACC12) variant = tuned_variant(p, 2, variant);
  if (p->cplx) return launch_slice_inv_c(p->prec == KX_PREC_FP64, p->nk12, variant, C, items, mb, s, tt);
  if (!bf && p->prec == KX_PREC_FP64) return launch_slice_inv_f64(p->nk12, variant, C, items, mb, s, tt);
  if (!bf && p->prec == KX_PREC_FP32) return launch_slice_inv_f32(p->nk12, variant, C, items, mb, s, tt);
  return launch_slice_inv_bf(bf_spl(p), p->bf_nt12, variant & ~kx::TUNE_ALT, C, items, mb, p->bf_vps12,
                             p->bf_kp12, s, tt);
}

// Blocks of plan p's pass-C persistent grid (its tuned configuration), asked
// of the launcher without launching; the device's CU count if it has none.
int64_t pass_c_grid(kx_plan p) {
  int64_t g = 0;
  kx::g_grid_probe = &g;
  (void)launch_pass_c(p, kx::SI_ACC12, kx::AccArgs{}, (int64_t)1 << 40, nullptr);
  kx::g_grid_probe = nullptr;
  return g > 0 ? g : kx::device_cu_count();
}

// Plans whose batches can share one launch of pass `pass` (0 = A, 1 = B,
// 2 = C) have equal keys: same kernel family, element type, tile count and
// tuned variant.
std::array<int, 6> launch_key(const kx_plan p, int pass) {
  const int fam = p->cplx ? 2 : (pass_bf(p, pass) ? 1 : 0);
  const int tiles = fam == 1 ? (pass == 1 ? p->bf_nt3 : p->bf_nt12) : (pass == 1 ? p->nk3 : p->nk12);
  const int vps = fam == 1 ? (pass == 1 ? p->bf_vps3 : p->bf_vps12) : 0;
  return {fam, p->prec, tiles, tuned_variant(p, pass, 0), vps, tuned_blocks(p, pass)};
}

// Arguments of one batch (targets n0 .. n0+cur-1) of an exx_apply on plan p.
struct BatchArgs {
  kx::SliceArgs A;
  kx::PencilArgs B;
  kx::AccArgs C;
};
BatchArgs batch_args(kx_plan p, const void* psi, int64_t ld_psi, int n_occ, const double* occ,
                     const void* phi, int64_t ld_phi, double* vx, int64_t ld_vx, bool want_ex, int n0,
                     int cur, void* ws = nullptr, double* part = nullptr) {
  if (!ws) ws = p->d_ws;
  if (!part) part = p->d_part;
  const size_t eb = elem_bytes(p->prec) * (p->cplx ? 2 : 1);  // bytes per grid value
  const size_t vxw = p->cplx ? 2 : 1;                          // doubles per Vx value
  const int npairs = cur * n_occ;
  const char* phi0 = (const char*)phi + (size_t)n0 * ld_phi * eb;
  BatchArgs b{};
  kx::SliceArgs& A = b.A;
  A.n1 = p->n[0]; A.n2 = p->n[1]; A.n3 = p->n[2]; A.n12 = p->n12; A.N = p->N;
  A.npairs = npairs; A.n_occ = n_occ;
  A.psi = psi; A.ld_psi = ld_psi; A.phi = phi0; A.ld_phi = ld_phi;
  A.src = ws; A.ld_src = p->N;
  A.dst = ws; A.ld_dst = p->N;
  A.V1 = p->dVmat[0]; A.V2 = p->dVmat[1]; A.P = p->P12;
  kx::PencilArgs& B = b.B;
  B.n1 = p->n[0]; B.n2 = p->n[1]; B.n3 = p->n[2]; B.n12 = p->n12;
  B.npairs = npairs; B.nchunks = (p->n12 + 63) / 64;
  B.T = ws; B.ld = p->N; B.V3 = p->dVmat[2]; B.V3T = p->dVmatT[2]; B.P3 = p->P3; B.ftab = p->d_f;
  kx::AccArgs& C = b.C;
  C.n1 = p->n[0]; C.n2 = p->n[1]; C.n3 = p->n[2]; C.n12 = p->n12; C.N = p->N;
  C.n_t = cur; C.n_occ = n_occ;
  C.T = ws; C.ld_T = p->N;
  C.psi = psi; C.ld_psi = ld_psi; C.occ = occ;
  C.phi = phi0; C.ld_phi = ld_phi;
  C.vx = vx + (size_t)n0 * ld_vx * vxw; C.ld_vx = ld_vx;
  C.partials = want_ex ? part : nullptr;
  C.dst = ws; C.ld_dst = p->N;
  C.V1 = p->dVmatT[0]; C.V2 = p->dVmatT[1]; C.P = p->P12;
  return b;
}

// n_b targets in batches of at most `cap`: as few batches as that allows, of
// equal size up to one target (a small ragged last batch would leave most of
// the device idle in its launches).
int balanced_batch(int n_b, size_t cap) {
  cap = std::max<size_t>(1, std::min<size_t>(cap, (size_t)n_b));
  const size_t nbatch = ((size_t)n_b + cap - 1) / cap;
  return (int)(((size_t)n_b + nbatch - 1) / nbatch);
}

// Targets per batch within what the plan's buffers hold (prepare_exx sized
// them), balanced over the batches; 0 if the buffers hold no target.
int held_batch(const kx_plan p, int n_occ, int n_b) {
  const size_t per_t_ws = (size_t)n_occ * p->N * elem_bytes(p->prec) * (p->cplx ? 2 : 1);
  const size_t per_t_part = std::max<size_t>(64, (size_t)p->n[2]) * sizeof(double);
  const size_t cap = std::min(p->ws_bytes / per_t_ws, p->part_bytes / per_t_part);
  return cap == 0 ? 0 : balanced_batch(n_b, cap);
}

// Enqueue one exx_apply.  Arguments already validated; buffers allocated for
// the batch size returned by batch_targets().
//
// Pass C has one work item per (target, slice) and its persistent grid holds
// R blocks at once, so a batch of t targets takes ceil(t n3 / R) rounds of
// items, each round as long as one item (a loop over all occupied orbitals):
// at 120^3 in FP64 (R = 256) a batch of 7 targets runs 4 rounds for 3.3
// rounds of work.  Among the batch sizes the workspace limit allows, take
// the one with the fewest pass-C rounds over all batches (a small charge per
// batch for its launches breaks ties toward fewer batches).
//
// limit: workspace bytes the plan may hold (0: workspace_limit()).
int batch_targets(kx_plan p, int n_occ, int n_b, size_t limit = 0) {
  if (!limit) limit = workspace_limit();
  const size_t per_t = (size_t)n_occ * p->N * elem_bytes(p->prec) * (p->cplx ? 2 : 1);
  const int cap = (int)std::max<size_t>(1, std::min<size_t>(limit / std::max<size_t>(per_t, 1), (size_t)n_b));
  const int64_t R = std::max<int64_t>(1, pass_c_grid(p));
  const int64_t n3 = p->n[2];
  int best = balanced_batch(n_b, cap);
  double best_cost = 1e300;
  for (int nt = cap; nt >= 1 && nt * 4 >= cap; --nt) {
    const int k = (n_b + nt - 1) / nt, last = n_b - (k - 1) * nt;
    const double cost = (double)(k - 1) * ((nt * n3 + R - 1) / R) + (double)((last * n3 + R - 1) / R) + 0.05 * k;
    if (cost < best_cost - 1e-9) {
      best_cost = cost;
      best = nt;
    }
  }
  return best;
}

// Buffers of plan p for calls with n_b targets x n_occ occupied (limit as
// in batch_targets; shrink: give back a workspace far larger than that).
kx_status prepare_exx(kx_plan p, int n_occ, int n_b, int path, size_t limit = 0, bool shrink = false) {
  const int nt = batch_targets(p, n_occ, n_b, limit);
  const size_t eb = elem_bytes(p->prec) * (p->cplx ? 2 : 1);
  void* ws0 = p->d_ws;
  void* part0 = p->d_part;
  kx_status st = ensure_buffer(&p->d_ws, &p->ws_bytes, (size_t)nt * n_occ * p->N * eb, "workspace", shrink);
  if (st != KX_OK) return st;
  const size_t per_t = std::max<size_t>(64, (size_t)p->n[2]);
  st = ensure_buffer((void**)&p->d_part, &p->part_bytes, (size_t)nt * per_t * sizeof(double),
                     "E_x partials");
  if (p->d_ws != ws0 || p->d_part != part0) ++p->gen;
  return st;
}

// ws / part / nt: the pair workspace, the E_x partials and the targets per
// batch they hold; null / 0 selects the plan-owned buffers.  With
// untraced, no trace events are created (the allocation-free entry point).
kx_status enqueue_exx(kx_plan p, const void* psi, int64_t ld_psi, int n_occ, const double* occ,
                      const void* phi, int64_t ld_phi, int n_b, double* vx, int64_t ld_vx,
                      double* ex, const double* gphi, int path, hipStream_t s, void* ws = nullptr,
                      double* part = nullptr, int nt = 0, bool untraced = false) {
  using namespace kx;
  if (n_occ == 0 || n_b == 0) return KX_OK;
  if (nt == 0) {
    nt = held_batch(p, n_occ, n_b);
    if (nt < 1) return fail(KX_ESTATE, "exx_apply: workspace not prepared");
    p->last_nt = nt;
  }
  if (!ws) ws = p->d_ws;
  if (!part) part = p->d_part;
  auto traced = [untraced](int kind, hipStream_t st, auto fn) -> hipError_t {
    return untraced ? fn() : ::traced(kind, st, fn);
  };
  for (int n0 = 0; n0 < n_b; n0 += nt) {
    const int cur = std::min(nt, n_b - n0);
    const int npairs = cur * n_occ;
    const BatchArgs ba = batch_args(p, psi, ld_psi, n_occ, occ, phi, ld_phi, vx, ld_vx, ex != nullptr, n0, cur,
                                    ws, part);
    const kx::SliceArgs& A = ba.A;
    const kx::PencilArgs& B = ba.B;
    const kx::AccArgs& C = ba.C;
    const int64_t items_pairs = (int64_t)npairs * p->n[2];
    hipError_t e = hipSuccess;
    int per_target = p->n[2];
    if (path == KX_PATH_FUSED) {
      e = traced(TK_A, s, [&] { return launch_pass_a(p, SF_PAIR12, A, items_pairs, s); });
      if (e == hipSuccess) e = traced(TK_B, s, [&] { return launch_pass_b(p, B, s); });
      if (e == hipSuccess)
        e = traced(TK_C, s, [&] { return launch_pass_c(p, SI_ACC12, C, (int64_t)cur * p->n[2], s); });
    } else {
      // plain FP64: one kernel per step, each a full pass over the batch
      const int mb = p->max_blocks;
      e = traced(TK_P_PAIR, s, [&] { return launch_slice_fwd_f64(p->nk12, SF_PAIR, A, items_pairs, mb, s); });
      if (e == hipSuccess)
        e = traced(TK_P_M1F, s, [&] { return launch_slice_fwd_f64(p->nk12, SF_LOAD1, A, items_pairs, mb, s); });
      if (e == hipSuccess)
        e = traced(TK_P_M2F, s, [&] { return launch_slice_fwd_f64(p->nk12, SF_LOAD2, A, items_pairs, mb, s); });
      if (e == hipSuccess) e = traced(TK_P_M3F, s, [&] { return launch_pencil_f64(p->nk3, PC_F, B, mb, s); });
      if (e == hipSuccess)
        e = traced(TK_P_SCALE, s, [&] { return launch_scale_f64((double*)ws, p->N, npairs, p->N, p->d_f, s); });
      if (e == hipSuccess) e = traced(TK_P_M3I, s, [&] { return launch_pencil_f64(p->nk3, PC_I, B, mb, s); });
      AccArgs Cs = C;
      Cs.n_t = npairs; Cs.n_occ = 1;
      if (e == hipSuccess)
        e = traced(TK_P_M2I, s, [&] { return launch_slice_inv_f64(p->nk12, SI_ST2, Cs, items_pairs, mb, s); });
      if (e == hipSuccess)
        e = traced(TK_P_M1I, s, [&] { return launch_slice_inv_f64(p->nk12, SI_ST1, Cs, items_pairs, mb, s); });
      per_target = 64;
      if (e == hipSuccess) e = traced(TK_P_ACC, s, [&] { return launch_accumulate_f64(C, per_target, s); });
    }
    if (e == hipSuccess && ex)
      e = traced(TK_FIN, s, [&] { return launch_ex_finalize(part, cur, per_target, gphi + n0, p->dV, ex, s); });
    if (e != hipSuccess) return dev_fail(e, "exx_apply launch");
  }
  return KX_OK;
}

// Round to bf16 (nearest even) through FP32; returns the bf16 bit pattern and
// its value.
uint16_t to_bf16(double v, double* back) {
  float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  const uint16_t h = (uint16_t)(u >> 16);
  uint32_t w = (uint32_t)h << 16;
  float g;
  std::memcpy(&g, &w, 4);
  *back = g;
  return h;
}

// Upload the split parts of M (n x n, M[r*n + c]) as [c][k] = M^T or M:
// transpose == true stores part(M[k][c]) at [c][k]; false stores part(M[c][k]).
// Layout: nparts x rows x kp bf16 values, zero outside n x n.
hipError_t upload_bf_parts(const std::vector<double>& M, int n, bool transpose, int nparts,
                           int rows, int kp, void** out) {
  std::vector<uint16_t> h((size_t)nparts * rows * kp, 0);
  for (int c = 0; c < n; ++c)
    for (int k = 0; k < n; ++k) {
      double v = transpose ? M[(size_t)k * n + c] : M[(size_t)c * n + k];
      for (int q = 0; q < nparts; ++q) {
        double b;
        h[((size_t)q * rows + c) * kp + k] = to_bf16(v, &b);
        v -= b;
      }
    }
  hipError_t e = hipMalloc(out, h.size() * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMemcpy(*out, h.data(), h.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  return e;
}

}  // namespace

extern "C" {

const char* kx_last_error(void) { return g_err.c_str(); }

kx_status kx_trace_enable(int on) {
  std::vector<TraceRec> drop;
  {
    std::lock_guard<std::mutex> lock(g_tr_mu);
    g_trace_on = on != 0;
    if (on) {
      drop.swap(g_tr_pending);
      for (int k = 0; k < TK_COUNT; ++k) {
        g_tr_ms[k] = 0.0;
        g_tr_n[k] = 0;
      }
    }
  }
  for (TraceRec& r : drop) {
    hipEventSynchronize(r.b);
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  return KX_OK;
}

kx_status kx_trace_read(double* ms, int64_t* count, int nkinds) {
  if (nkinds < 0) return fail(KX_EINVAL, "kx_trace_read: nkinds < 0");
  std::vector<TraceRec> recs;
  {
    std::lock_guard<std::mutex> lock(g_tr_mu);
    recs.swap(g_tr_pending);
  }
  kx_status st = KX_OK;
  std::vector<double> add(TK_COUNT, 0.0);
  std::vector<int64_t> addn(TK_COUNT, 0);
  for (TraceRec& r : recs) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess && st == KX_OK) st = dev_fail(e, "kx_trace_read");
    add[r.kind] += t;
    addn[r.kind] += 1;
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  std::lock_guard<std::mutex> lock(g_tr_mu);
  for (int k = 0; k < TK_COUNT; ++k) {
    g_tr_ms[k] += add[k];
    g_tr_n[k] += addn[k];
  }
  const int m = std::min(nkinds, (int)TK_COUNT);
  for (int k = 0; k < m; ++k) {
    if (ms) ms[k] = g_tr_ms[k];
    if (count) count[k] = g_tr_n[k];
  }
  return st;
}

const char* kx_trace_name(int kind) {
  if (kind < 0 || kind >= TK_COUNT) return "";
  return kTraceNames[kind];
}

kx_status kx_host_fd_weights(int fd_order, double* c) {
  if (fd_order < 2 || fd_order > 16 || fd_order % 2) return fail(KX_EINVAL, "fd_order must be even in [2, 16]");
  if (!c) return fail(KX_EINVAL, "NULL output");
  std::vector<double> w = kx::fd_weights(fd_order);
  std::copy(w.begin(), w.end(), c);
  return KX_OK;
}

kx_status kx_host_eig1d(int n, double h, int bc, int fd_order, double kappa, double* lam,
                        double* V_re, double* V_im) {
  if (n < 1 || n > kx::kMaxAxis) return fail(KX_EINVAL, "n must be in [1, %d]", kx::kMaxAxis);
  if (!(h > 0) || !std::isfinite(h)) return fail(KX_EINVAL, "h must be positive");
  if (bc != KX_BC_PERIODIC && bc != KX_BC_DIRICHLET) return fail(KX_EINVAL, "unknown bc %d", bc);
  if (fd_order < 2 || fd_order > 16 || fd_order % 2) return fail(KX_EINVAL, "fd_order must be even in [2, 16]");
  if (!std::isfinite(kappa) || (kappa != 0.0 && bc != KX_BC_PERIODIC))
    return fail(KX_EINVAL, "a Bloch wavevector needs a periodic axis");
  std::vector<double> l, vr, vi;
  kx::eig1d(n, h, bc, fd_order, kappa, l, vr, vi);
  if (lam) std::copy(l.begin(), l.end(), lam);
  if (V_re) std::copy(vr.begin(), vr.end(), V_re);
  if (V_im) std::copy(vi.begin(), vi.end(), V_im);
  return KX_OK;
}

kx_status kron_setup(const int n[3], const double h[3], const int bc[3], int fd_order, double omega,
                     const double kq[3], int prec, kx_plan* out) {
  if (!out) return fail(KX_EINVAL, "kron_setup: out is NULL");
  *out = nullptr;
  if (!n || !h || !bc) return fail(KX_EINVAL, "kron_setup: NULL n, h or bc");
  for (int d = 0; d < 3; ++d) {
    if (n[d] < 1) return fail(KX_EINVAL, "kron_setup: n[%d] = %d < 1", d, n[d]);
    if (n[d] > kx::kMaxAxis) return fail(KX_EUNSUPPORTED, "kron_setup: n[%d] = %d > %d", d, n[d], kx::kMaxAxis);
    if (!(h[d] > 0) || !std::isfinite(h[d])) return fail(KX_EINVAL, "kron_setup: h[%d] must be positive", d);
    if (bc[d] != KX_BC_PERIODIC && bc[d] != KX_BC_DIRICHLET)
      return fail(KX_EINVAL, "kron_setup: unknown bc[%d] = %d", d, bc[d]);
    if (kq && (!std::isfinite(kq[d]) || (kq[d] != 0.0 && bc[d] != KX_BC_PERIODIC)))
      return fail(KX_EINVAL, "kron_setup: kq[%d] needs a periodic axis", d);
  }
  if (fd_order < 2 || fd_order > 16 || fd_order % 2)
    return fail(KX_EINVAL, "kron_setup: fd_order must be even in [2, 16]");
  if (!std::isfinite(omega)) return fail(KX_EINVAL, "kron_setup: omega is not finite");
  const bool force_cplx = (prec & KX_FLAG_COMPLEX) != 0;
  prec &= ~KX_FLAG_COMPLEX;
  if (prec < KX_PREC_FP64 || prec > KX_PREC_BF16X6) return fail(KX_EINVAL, "kron_setup: unknown precision %d", prec);
  if (prec == KX_PREC_FP64 && std::max(n[0], n[1]) > 128)
    return fail(KX_EUNSUPPORTED, "kron_setup: FP64 slices are limited to n1, n2 <= 128 (LDS)");
  {
    const bool cplx = force_cplx || (kq && (kq[0] != 0.0 || kq[1] != 0.0 || kq[2] != 0.0));
    if (cplx && prec != KX_PREC_FP64 && prec != KX_PREC_FP32)
      return fail(KX_EUNSUPPORTED, "kron_setup: complex (Bloch) plans run in FP64 or FP32");
    if (cplx && prec == KX_PREC_FP64 && n[2] > 144)
      return fail(KX_EUNSUPPORTED, "kron_setup: complex FP64 pencils are limited to n3 <= 144 (LDS)");
    if (cplx && std::max(n[0], n[1]) > (prec == KX_PREC_FP64 ? 96 : 128))
      return fail(KX_EUNSUPPORTED, "kron_setup: complex slices are limited to n1, n2 <= %d (LDS)",
                  prec == KX_PREC_FP64 ? 96 : 128);
  }

  kx_plan p = new (std::nothrow) kx_plan_s();
  if (!p) return fail(KX_ENOMEM, "kron_setup: host allocation");
  for (int d = 0; d < 3; ++d) {
    p->n[d] = n[d];
    p->h[d] = h[d];
    p->bc[d] = bc[d];
    p->kq[d] = kq ? kq[d] : 0.0;
  }
  p->order = fd_order;
  p->omega = omega;
  p->prec = prec;
  p->cplx = force_cplx || p->kq[0] != 0.0 || p->kq[1] != 0.0 || p->kq[2] != 0.0;
  p->N = (int64_t)n[0] * n[1] * n[2];
  p->n12 = n[0] * n[1];
  p->dV = h[0] * h[1] * h[2];
  for (int d = 0; d < 3; ++d) kx::eig1d(n[d], h[d], bc[d], fd_order, p->kq[d], p->lam[d], p->Vre[d], p->Vim[d]);
  kx::f_table(p->lam, omega, p->f);
  p->nk12 = kx::pick_nk(std::max(n[0], n[1]));
  p->nk3 = kx::pick_nk(n[2]);
  p->P12 = kx::padded_len(p->nk12);
  p->P3 = kx::padded_len(p->nk3);
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(KX_EDEVICE, "kron_setup: no HIP device");
  }
  // Zero-padded eigenvector matrices, V[k*P + a] (k grid index, a mode).
  const int eb = elem_bytes(prec);
  for (int d = 0; d < 3; ++d) {
    const int P = d < 2 ? p->P12 : p->P3;
    const int nd = n[d];
    // real plans: one plane; complex plans: re plane then im plane
    const int planes = p->cplx ? 2 : 1;
    std::vector<char> host((size_t)planes * P * P * eb, 0), hostT((size_t)planes * P * P * eb, 0);
    for (int pl = 0; pl < planes; ++pl)
      for (int k = 0; k < nd; ++k)
        for (int a = 0; a < nd; ++a) {
          const double v = (pl == 0 ? p->Vre[d] : p->Vim[d])[(size_t)k * nd + a];
          const size_t o = (size_t)pl * P * P;
          if (eb == 8) {
            ((double*)host.data())[o + (size_t)k * P + a] = v;
            ((double*)hostT.data())[o + (size_t)a * P + k] = v;
          } else {
            ((float*)host.data())[o + (size_t)k * P + a] = (float)v;
            ((float*)hostT.data())[o + (size_t)a * P + k] = (float)v;
          }
        }
    hipError_t e = hipMalloc(&p->dVmat[d], host.size());
    if (e == hipSuccess) e = hipMemcpy(p->dVmat[d], host.data(), host.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&p->dVmatT[d], hostT.size());
    if (e == hipSuccess) e = hipMemcpy(p->dVmatT[d], hostT.data(), hostT.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      free_plan_device(p);
      delete p;
      return e == hipErrorOutOfMemory ? fail(KX_ENOMEM, "kron_setup: device allocation")
                                      : dev_fail(e, "kron_setup upload");
    }
  }
  hipError_t e = hipMalloc((void**)&p->d_f, p->f.size() * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(p->d_f, p->f.data(), p->f.size() * sizeof(double), hipMemcpyHostToDevice);
  // split-BF16 parts: the split plans' matrices, and for real FP32 plans the
  // six-product parts their passes may run (tuned variant bit 16)
  if (e == hipSuccess && (prec == KX_PREC_BF16X3 || prec == KX_PREC_BF16X6 || (prec == KX_PREC_FP32 && !p->cplx))) {
    const int parts = prec == KX_PREC_BF16X3 ? 2 : 3;
    p->bf_nt12 = kx::bf_nt(std::max(n[0], n[1]));
    p->bf_nt3 = kx::bf_nt(n[2]);
    p->bf_kp12 = kx::bf_kp(p->bf_nt12);
    p->bf_kp3 = kx::bf_kp(p->bf_nt3);
    const int rows12 = kx::bf_lines(p->bf_nt12), rows3 = kx::bf_lines(p->bf_nt3);
    p->bf_vps12 = rows12 * p->bf_kp12;
    p->bf_vps3 = rows3 * p->bf_kp3;
    for (int d = 0; d < 3 && e == hipSuccess; ++d) {
      const int rows = d < 2 ? rows12 : rows3, kp = d < 2 ? p->bf_kp12 : p->bf_kp3;
      e = upload_bf_parts(p->Vre[d], n[d], true, parts, rows, kp, &p->dVbf[d][0]);
      if (e == hipSuccess) e = upload_bf_parts(p->Vre[d], n[d], false, parts, rows, kp, &p->dVbf[d][1]);
    }
  }
  if (e != hipSuccess) {
    free_plan_device(p);
    delete p;
    return dev_fail(e, "kron_setup tables");
  }
  *out = p;
  return KX_OK;
}

kx_status kron_destroy(kx_plan p) {
  if (!p) return KX_OK;
  (void)hipDeviceSynchronize();
  {
    std::lock_guard<std::mutex> lock(g_graph_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
      bool uses = false;
      for (const kx_task& t : it->tasks) uses |= t.plan == p;
      if (uses) {
        destroy_graph_entry(*it);
        it = g_graphs.erase(it);
      } else {
        ++it;
      }
    }
  }
  free_plan_device(p);
  delete p;
  return KX_OK;
}

kx_status kx_plan_info(kx_plan p, int64_t out[8]) {
  if (!p || !out) return fail(KX_EINVAL, "kx_plan_info: NULL argument");
  out[0] = p->n[0]; out[1] = p->n[1]; out[2] = p->n[2];
  out[3] = p->cplx ? 1 : 0;
  out[4] = p->prec;
  out[5] = p->P12;
  out[6] = p->P3;
  out[7] = p->last_nt;
  return KX_OK;
}

kx_status kx_plan_tables(kx_plan p, int axis, double* lam, double* V_re, double* V_im) {
  if (!p) return fail(KX_EINVAL, "kx_plan_tables: plan is NULL");
  if (axis < 0 || axis > 3) return fail(KX_EINVAL, "kx_plan_tables: axis must be 0..3");
  if (axis == 3) {
    if (lam) std::copy(p->f.begin(), p->f.end(), lam);
    return KX_OK;
  }
  if (lam) std::copy(p->lam[axis].begin(), p->lam[axis].end(), lam);
  if (V_re) std::copy(p->Vre[axis].begin(), p->Vre[axis].end(), V_re);
  if (V_im) std::copy(p->Vim[axis].begin(), p->Vim[axis].end(), V_im);
  return KX_OK;
}

namespace {
// Sec. II.A, one right-hand side at a time: per frontal slice k,
//   X_k = V1^T B_k V2 (two GEMMs), then X = X V3 over the whole grid, the
// eigen-scaling, X = X V3^T, and per slice X_k = V1 X_k V2^T (two GEMMs):
// 4 n3 + 2 GEMM launches per solve.  The plan's eigenvector copies are padded
// (leading dimension P12 for V1, V2 and P3 for V3); W is N doubles of plan
// workspace (a slice of it holds each slice's intermediate product).
kx_status kron_solve_slicewise(kx_plan p, const double* B, int64_t ldb, double* X, int64_t ldx, int nrhs,
                               hipStream_t s) {
  void* ws0 = p->d_ws;
  kx_status st = ensure_buffer(&p->d_ws, &p->ws_bytes, (size_t)p->N * sizeof(double), "slice-wise workspace");
  if (st != KX_OK) return st;
  if (p->d_ws != ws0) ++p->gen;  // cached exx graphs must re-capture
  const int n1 = p->n[0], n2 = p->n[1], n3 = p->n[2], n12 = p->n12;
  // dVmat[d] holds V_d[grid k][mode a] at k*P + a, i.e. V_d^T as a
  // column-major matrix; dVmatT[d] is V_d itself, column-major
  const double* V1 = (const double*)p->dVmatT[0];
  const double* V1T = (const double*)p->dVmat[0];
  const double* V2 = (const double*)p->dVmatT[1];
  const double* V2T = (const double*)p->dVmat[1];
  const double* V3 = (const double*)p->dVmatT[2];
  const double* V3T = (const double*)p->dVmat[2];
  double* W = (double*)p->d_ws;
  hipError_t e = hipSuccess;
  for (int r = 0; r < nrhs && e == hipSuccess; ++r) {
    const double* b = B + (int64_t)r * ldb;
    double* x = X + (int64_t)r * ldx;
    for (int k = 0; k < n3 && e == hipSuccess; ++k) {
      e = kx::launch_gemm_nn_f64(n1, n2, n1, V1T, p->P12, b + (int64_t)k * n12, n1, W + (int64_t)k * n12, n1, s);
      if (e == hipSuccess)
        e = kx::launch_gemm_nn_f64(n1, n2, n2, W + (int64_t)k * n12, n1, V2, p->P12, x + (int64_t)k * n12, n1, s);
    }
    if (e == hipSuccess) e = kx::launch_gemm_nn_f64(n12, n3, n3, x, n12, V3, p->P3, W, n12, s);
    if (e == hipSuccess) e = kx::launch_scale_f64(W, p->N, 1, p->N, p->d_f, s);
    if (e == hipSuccess) e = kx::launch_gemm_nn_f64(n12, n3, n3, W, n12, V3T, p->P3, x, n12, s);
    for (int k = 0; k < n3 && e == hipSuccess; ++k) {
      e = kx::launch_gemm_nn_f64(n1, n2, n1, V1, p->P12, x + (int64_t)k * n12, n1, W + (int64_t)k * n12, n1, s);
      if (e == hipSuccess)
        e = kx::launch_gemm_nn_f64(n1, n2, n2, W + (int64_t)k * n12, n1, V2T, p->P12, x + (int64_t)k * n12, n1, s);
    }
  }
  if (e != hipSuccess) return dev_fail(e, "kron_solve slice-wise launch");
  return KX_OK;
}
}  // namespace

kx_status kron_solve(kx_plan p, const void* B, int64_t ldb, void* X, int64_t ldx, int nrhs, int path,
                     void* stream) {
  using namespace kx;
  if (!p) return fail(KX_EINVAL, "kron_solve: plan is NULL");
  if (nrhs < 0) return fail(KX_EINVAL, "kron_solve: nrhs < 0");
  if (path != KX_PATH_FUSED && path != KX_PATH_PLAIN && path != KX_PATH_SLICEWISE)
    return fail(KX_EINVAL, "kron_solve: unknown path");
  if (path != KX_PATH_FUSED && p->prec != KX_PREC_FP64)
    return fail(KX_EUNSUPPORTED, "kron_solve: the plain and slice-wise paths are FP64 only");
  if (nrhs == 0) return KX_OK;
  if (!B || !X) return fail(KX_EINVAL, "kron_solve: NULL data pointer");
  if (ldb < p->N || ldx < p->N) return fail(KX_EINVAL, "kron_solve: leading dimension below N");
  if (p->cplx && path != KX_PATH_FUSED)
    return fail(KX_EUNSUPPORTED, "kron_solve: the plain and slice-wise paths are real (Gamma) only");
  const size_t eb = elem_bytes(p->prec) * (p->cplx ? 2 : 1);
  {
    const char* b0 = (const char*)B;
    const char* b1 = b0 + ((size_t)(nrhs - 1) * ldb + p->N) * eb;
    const char* x0 = (const char*)X;
    const char* x1 = x0 + ((size_t)(nrhs - 1) * ldx + p->N) * eb;
    if (b0 < x1 && x0 < b1) return fail(KX_EINVAL, "kron_solve: B and X overlap");
  }
  hipStream_t s = (hipStream_t)stream;
  if (path == KX_PATH_SLICEWISE) return kron_solve_slicewise(p, (const double*)B, ldb, (double*)X, ldx, nrhs, s);
  SliceArgs A{};
  A.n1 = p->n[0]; A.n2 = p->n[1]; A.n3 = p->n[2]; A.n12 = p->n12; A.N = p->N;
  A.npairs = nrhs; A.n_occ = 1;
  A.src = B; A.ld_src = ldb; A.dst = X; A.ld_dst = ldx;
  A.V1 = p->dVmat[0]; A.V2 = p->dVmat[1]; A.P = p->P12;
  PencilArgs Pn{};
  Pn.n1 = p->n[0]; Pn.n2 = p->n[1]; Pn.n3 = p->n[2]; Pn.n12 = p->n12;
  Pn.npairs = nrhs; Pn.nchunks = (p->n12 + 63) / 64;
  Pn.T = X; Pn.ld = ldx; Pn.V3 = p->dVmat[2]; Pn.V3T = p->dVmatT[2]; Pn.P3 = p->P3; Pn.ftab = p->d_f;
  AccArgs C{};
  C.n1 = p->n[0]; C.n2 = p->n[1]; C.n3 = p->n[2]; C.n12 = p->n12; C.N = p->N;
  C.n_t = nrhs; C.n_occ = 1;
  C.T = X; C.ld_T = ldx; C.dst = X; C.ld_dst = ldx;
  C.V1 = p->dVmatT[0]; C.V2 = p->dVmatT[1]; C.P = p->P12;
  const int64_t items = (int64_t)nrhs * p->n[2];
  hipError_t e;
  const int mb = p->max_blocks;
  if (path == KX_PATH_FUSED) {
    e = traced(TK_S_A, s, [&] { return launch_pass_a(p, SF_LOAD12, A, items, s); });
    if (e == hipSuccess) e = traced(TK_S_B, s, [&] { return launch_pass_b(p, Pn, s); });
    if (e == hipSuccess) e = traced(TK_S_C, s, [&] { return launch_pass_c(p, SI_ST12, C, items, s); });
  } else {
    e = traced(TK_SP_M1F, s, [&] { return launch_slice_fwd_f64(p->nk12, SF_LOAD1, A, items, mb, s); });
    A.src = X; A.ld_src = ldx;
    if (e == hipSuccess) e = traced(TK_SP_M2F, s, [&] { return launch_slice_fwd_f64(p->nk12, SF_LOAD2, A, items, mb, s); });
    if (e == hipSuccess) e = traced(TK_SP_M3F, s, [&] { return launch_pencil_f64(p->nk3, PC_F, Pn, mb, s); });
    if (e == hipSuccess)
      e = traced(TK_SP_SCALE, s, [&] { return launch_scale_f64((double*)X, ldx, nrhs, p->N, p->d_f, s); });
    if (e == hipSuccess) e = traced(TK_SP_M3I, s, [&] { return launch_pencil_f64(p->nk3, PC_I, Pn, mb, s); });
    if (e == hipSuccess) e = traced(TK_SP_M2I, s, [&] { return launch_slice_inv_f64(p->nk12, SI_ST2, C, items, mb, s); });
    if (e == hipSuccess) e = traced(TK_SP_M1I, s, [&] { return launch_slice_inv_f64(p->nk12, SI_ST1, C, items, mb, s); });
  }
  if (e != hipSuccess) return dev_fail(e, "kron_solve launch");
  return KX_OK;
}

kx_status exx_apply(kx_plan p, const void* d_psi, int64_t ld_psi, int n_occ, const double* d_occ,
                    const void* d_phi, int64_t ld_phi, int n_b, double* d_vx, int64_t ld_vx,
                    double* d_ex, const double* d_gphi, int path, void* stream) {
  kx_status st = check_exx_args(p, d_psi, ld_psi, n_occ, d_occ, d_phi, ld_phi, n_b, d_vx, ld_vx,
                                d_ex, d_gphi, path);
  if (st != KX_OK || n_occ == 0 || n_b == 0) return st;
  st = prepare_exx(p, n_occ, n_b, path);
  if (st != KX_OK) return st;
  return enqueue_exx(p, d_psi, ld_psi, n_occ, d_occ, d_phi, ld_phi, n_b, d_vx, ld_vx, d_ex, d_gphi,
                     path, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// exx_apply_static: exx_apply without any device allocation.  The pair
// workspace and the E_x partials live in `scratch`, a fixed device array of
// this translation unit (one copy per GPU, held until the process ends).  In
// host code `scratch` names a host-side stand-in; its device address on each
// GPU comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address reaches kernels.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr size_t kStaticScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // device address of `scratch`, per device

kx_status static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dev_fail(e, "exx_apply_static: hipGetDevice");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(KX_EDEVICE, "exx_apply_static: hipGetSymbolAddress(scratch) failed: %s",
                  hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return KX_OK;
}

}  // namespace

extern "C" {

size_t kx_static_scratch_bytes(void) { return kStaticScratchBytes; }

kx_status exx_apply_static(kx_plan p, const void* d_psi, int64_t ld_psi, int n_occ, const double* d_occ,
                           const void* d_phi, int64_t ld_phi, int n_b, double* d_vx, int64_t ld_vx,
                           double* d_ex, const double* d_gphi, int path, void* stream) {
  kx_status st = check_exx_args(p, d_psi, ld_psi, n_occ, d_occ, d_phi, ld_phi, n_b, d_vx, ld_vx,
                                d_ex, d_gphi, path);
  if (st != KX_OK || n_occ == 0 || n_b == 0) return st;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(KX_EINVAL, "exx_apply_static: the plan's device (%d) is not the current device (%d)",
                p->device, dev);
  // layout: E_x partials of every target (max(64, n3) doubles each, 256-byte
  // aligned), then the pair workspace of one batch
  const size_t per_t_part = std::max<size_t>(64, (size_t)p->n[2]) * sizeof(double);
  const size_t part_bytes = ((size_t)n_b * per_t_part + 255) / 256 * 256;
  const size_t per_t_ws = (size_t)n_occ * p->N * elem_bytes(p->prec) * (p->cplx ? 2 : 1);
  if (part_bytes + per_t_ws > kStaticScratchBytes)
    return fail(KX_EINVAL,
                "exx_apply_static: one target needs %zu bytes of scratch (%d occupied x N = %lld), "
                "more than its fixed %zu bytes; use exx_apply",
                part_bytes + per_t_ws, n_occ, (long long)p->N, kStaticScratchBytes);
  const int nt = balanced_batch(n_b, (kStaticScratchBytes - part_bytes) / per_t_ws);
  void* base = nullptr;
  st = static_scratch(&base);
  if (st != KX_OK) return st;
  double* part = (double*)base;
  void* ws = (char*)base + part_bytes;
  return enqueue_exx(p, d_psi, ld_psi, n_occ, d_occ, d_phi, ld_phi, n_b, d_vx, ld_vx, d_ex, d_gphi, path,
                     (hipStream_t)stream, ws, part, nt, true);
}

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------
namespace {

// One fused batch (targets n0 .. n0+cur-1) with events ev[0..3] around the
// three passes; buffers already sized.
hipError_t timed_batch(kx_plan p, const void* psi, int64_t ld_psi, int n_occ, const double* occ,
                       const void* phi, int64_t ld_phi, int cur, double* vx, int64_t ld_vx,
                       hipEvent_t* ev, hipStream_t s) {
  using namespace kx;
  const int npairs = cur * n_occ;
  const BatchArgs ba = batch_args(p, psi, ld_psi, n_occ, occ, phi, ld_phi, vx, ld_vx, false, 0, cur);
  const SliceArgs& A = ba.A;
  const PencilArgs& B = ba.B;
  const AccArgs& C = ba.C;
  hipEventRecord(ev[0], s);
  hipError_t e = launch_pass_a(p, SF_PAIR12, A, (int64_t)npairs * p->n[2], s);
  hipEventRecord(ev[1], s);
  if (e == hipSuccess) e = launch_pass_b(p, B, s);
  hipEventRecord(ev[2], s);
  if (e == hipSuccess) e = launch_pass_c(p, SI_ACC12, C, (int64_t)cur * p->n[2], s);
  hipEventRecord(ev[3], s);
  return e;
}

std::string tune_key(kx_plan p, int n_occ) {
  hipDeviceProp_t prop;
  char arch[64] = "unknown";
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
    std::snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
    for (char* c = arch; *c; ++c)
      if (*c == ' ' || *c == ':') *c = '_';
  }
  int rt = 0;
  (void)hipRuntimeGetVersion(&rt);
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s|hip%d|%dx%dx%d|prec%d|cplx%d|occ%d", arch, rt, p->n[0], p->n[1],
                p->n[2], p->prec, p->cplx ? 1 : 0, n_occ);
  return buf;
}

bool tune_cache_lookup(const std::string& key, int tv[3], int bpc[3]) {
  const char* path = std::getenv("KX_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char k[256];
  int a[6];
  bool found = false;
  while (std::fscanf(f, "%255s %d %d %d %d %d %d", k, &a[0], &a[1], &a[2], &a[3], &a[4], &a[5]) == 7) {
    if (key == k) {
      for (int i = 0; i < 3; ++i) {
        tv[i] = a[2 * i];
        bpc[i] = a[2 * i + 1];
      }
      found = true;  // the last matching line wins
    }
  }
  std::fclose(f);
  return found;
}

void tune_cache_store(const std::string& key, const int tv[3], const int bpc[3]) {
  const char* path = std::getenv("KX_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d %d %d\n", key.c_str(), tv[0], bpc[0], tv[1], bpc[1], tv[2], bpc[2]);
  std::fclose(f);
}

}  // namespace

kx_status kx_plan_tuning(kx_plan p, int out[7]) {
  if (!p || !out) return fail(KX_EINVAL, "kx_plan_tuning: NULL argument");
  for (int i = 0; i < 3; ++i) {
    out[2 * i] = p->tune_tv[i];
    out[2 * i + 1] = p->tune_bpc[i];
  }
  out[6] = p->tuned ? 1 : 0;
  return KX_OK;
}

kx_status kx_autotune(kx_plan p, const void* d_psi, int64_t ld_psi, int n_occ, const double* d_occ,
                      const void* d_phi, int64_t ld_phi, int n_b, void* stream) {
  double* dummy_vx = reinterpret_cast<double*>(alignof(double) * 64);  // validated, never used
  kx_status st = check_exx_args(p, d_psi, ld_psi, n_occ, d_occ, d_phi, ld_phi, n_b, dummy_vx, p ? p->N : 0,
                                nullptr, nullptr, KX_PATH_FUSED);
  if (st != KX_OK) return st;
  if (n_occ == 0 || n_b == 0) return KX_OK;
  const bool real_mfma = !p->cplx && (p->prec == KX_PREC_FP64 || p->prec == KX_PREC_FP32);
  const std::string key = tune_key(p, n_occ);
  int tv[3], bpc[3];
  if (tune_cache_lookup(key, tv, bpc)) {
    for (int i = 0; i < 3; ++i) {
      p->tune_tv[i] = tv[i];
      p->tune_bpc[i] = bpc[i];
    }
    p->tuned = true;
    ++p->gen;  // graphs captured with the previous configuration are stale
    return KX_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  // Time the batch size a real call makes: the persistent grids fill the
  // device differently on a smaller batch (pass C has one item per target
  // slice), so a reduced sample picks configurations that lose at full size.
  const int ns = n_b;
  st = prepare_exx(p, n_occ, ns, KX_PATH_FUSED);
  if (st != KX_OK) return st;
  const int cur = held_batch(p, n_occ, ns);
  if (cur < 1) return fail(KX_ESTATE, "kx_autotune: workspace not prepared");
  double* vx = nullptr;
  if (hipMalloc((void**)&vx, (size_t)cur * p->N * sizeof(double) * (p->cplx ? 2 : 1)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(KX_ENOMEM, "kx_autotune: sample Vx buffer");
  }
  // candidates: (variant bits, resident blocks per CU; 0 = all that fit).
  // The first 24 serve the FP64/FP32 real kernels, the last 4 (the
  // six-product split-BF16 kernels) real FP32 plans only; complex plans take
  // the first 10 (bit 0 only), split-BF16 plans the first 5.
  static const int cand[][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {0, 4}, {1, 0}, {1, 1}, {1, 2},
                                {1, 3}, {1, 4}, {2, 0}, {2, 1}, {2, 2}, {2, 3}, {2, 4}, {3, 0},
                                {3, 1}, {3, 2}, {3, 3}, {3, 4}, {4, 0}, {4, 1}, {4, 2}, {8, 0},
                                {16, 0}, {16, 1}, {16, 2}, {16, 3}};
  const int ncand = real_mfma ? (p->prec == KX_PREC_FP32 ? 28 : 24) : (p->cplx ? 10 : 5);
  hipEvent_t ev[4];
  for (int i = 0; i < 4; ++i) hipEventCreate(&ev[i]);
  float best[3] = {1e30f, 1e30f, 1e30f};
  int best_c[3] = {0, 0, 0};
  hipError_t e = hipSuccess;
  const int save_tv[3] = {p->tune_tv[0], p->tune_tv[1], p->tune_tv[2]};
  const int save_bpc[3] = {p->tune_bpc[0], p->tune_bpc[1], p->tune_bpc[2]};
  for (int c = 0; c < ncand && e == hipSuccess; ++c) {
    for (int i = 0; i < 3; ++i) {
      p->tune_tv[i] = cand[c][0];
      p->tune_bpc[i] = cand[c][1];
    }
    // the first run warms up; the best of the next two counts (one timing
    // per candidate let run-to-run noise of ~2 % pick a slower variant)
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      e = timed_batch(p, d_psi, ld_psi, n_occ, d_occ, d_phi, ld_phi, cur, vx, p->N, ev, s);
      if (e == hipSuccess) e = hipEventSynchronize(ev[3]);
      if (e == hipSuccess && rep >= 1) {
        for (int i = 0; i < 3; ++i) {
          float ms = 0.f;
          hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
          if (ms < best[i]) {
            best[i] = ms;
            best_c[i] = c;
          }
        }
      }
    }
  }
  for (int i = 0; i < 4; ++i) hipEventDestroy(ev[i]);
  hipFree(vx);
  if (e != hipSuccess) {
    for (int i = 0; i < 3; ++i) {
      p->tune_tv[i] = save_tv[i];
      p->tune_bpc[i] = save_bpc[i];
    }
    return dev_fail(e, "kx_autotune");
  }
  for (int i = 0; i < 3; ++i) {
    p->tune_tv[i] = cand[best_c[i]][0];
    p->tune_bpc[i] = cand[best_c[i]][1];
    tv[i] = p->tune_tv[i];
    bpc[i] = p->tune_bpc[i];
  }
  p->tuned = true;
  ++p->gen;
  tune_cache_store(key, tv, bpc);
  return KX_OK;
}

namespace {

// One batch of one task of exx_apply_batched: targets n0 .. n0+cur-1.
struct SubTask {
  int task, n0, cur;
};

// Schedule of a task list: rounds of batches such that within a round no two
// batches share a plan (they would share its workspace) or overlap in their
// Vx output (batches of one launch update Vx concurrently).  A batch whose Vx
// overlaps an earlier batch's goes to a later round, so overlapping outputs
// accumulate in task order.  Greedy, in task order: each batch goes to the
// first round that admits it.
std::vector<std::vector<SubTask>> schedule_rounds(const kx_task* tasks, int ntasks) {
  struct Placed {
    SubTask st;
    const kx_plan plan;
    const double *lo, *hi;
    size_t round;
  };
  std::vector<Placed> placed;
  std::vector<std::vector<SubTask>> rounds;
  for (int i = 0; i < ntasks; ++i) {
    const kx_task& t = tasks[i];
    if (t.n_occ == 0 || t.n_b == 0) continue;
    const int nt = held_batch(t.plan, t.n_occ, t.n_b);
    const size_t vxw = t.plan->cplx ? 2 : 1;
    for (int n0 = 0; n0 < t.n_b; n0 += nt) {
      const SubTask st{i, n0, std::min(nt, t.n_b - n0)};
      const double* lo = t.d_vx + (size_t)n0 * t.ld_vx * vxw;
      const double* hi = lo + (size_t)(st.cur - 1) * t.ld_vx * vxw + (size_t)t.plan->N * vxw;
      size_t r = 0;
      for (const Placed& q : placed)
        if (lo < q.hi && q.lo < hi) r = std::max(r, q.round + 1);
      for (;; ++r) {
        bool ok = true;
        for (const Placed& q : placed)
          if (q.round == r && q.plan == t.plan) ok = false;
        if (ok) break;
      }
      if (r >= rounds.size()) rounds.resize(r + 1);
      rounds[r].push_back(st);
      placed.push_back(Placed{st, t.plan, lo, hi, r});
    }
  }
  return rounds;
}

// Workspaces of a batched call's plans.  Every plan of the list holds its
// buffers at once, so they share one budget: KX_WORKSPACE_MB per plan when
// set, else 60 % of the free device memory plus what these plans hold
// already, split in proportion to what each plan would need for all its
// targets in one batch (each gets that need when the budget covers them
// all).  A plan's largest task sizes its buffers, which shrink when they
// hold far more than its share (an earlier single call or autotuning may
// have sized them for the plan alone).
kx_status prepare_batched(const kx_task* tasks, int ntasks) {
  std::vector<kx_plan> plans;
  std::vector<size_t> need;
  std::vector<int> big;  // task with the largest need, per plan
  for (int i = 0; i < ntasks; ++i) {
    const kx_task& t = tasks[i];
    if (t.n_occ == 0 || t.n_b == 0) continue;
    const kx_plan p = t.plan;
    const size_t nd = (size_t)t.n_b * t.n_occ * p->N * elem_bytes(p->prec) * (p->cplx ? 2 : 1);
    size_t j = 0;
    while (j < plans.size() && plans[j] != p) ++j;
    if (j == plans.size()) {
      plans.push_back(p);
      need.push_back(nd);
      big.push_back(i);
    } else if (nd > need[j]) {
      need[j] = nd;
      big[j] = i;
    }
  }
  std::vector<size_t> limit(plans.size(), 0);
  const char* env = std::getenv("KX_WORKSPACE_MB");
  if (!(env && *env && std::atoll(env) > 0)) {
    size_t free_b = 0, total_b = 0, held = 0, sum = 0;
    for (size_t j = 0; j < plans.size(); ++j) {
      held += plans[j]->ws_bytes;
      sum += need[j];
    }
    size_t budget = (size_t)4 << 30;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) budget = (free_b + held) / 5 * 3;
    for (size_t j = 0; j < plans.size(); ++j)
      limit[j] = std::max<size_t>((size_t)64 << 20,
                                  sum <= budget ? need[j] : (size_t)((double)budget * need[j] / sum));
  }
  // each plan's largest task sizes its buffers: those that shrink first,
  // then those that grow
  for (int grow = 0; grow < 2; ++grow)
    for (size_t j = 0; j < plans.size(); ++j) {
      const kx_task& t = tasks[big[j]];
      const kx_plan p = t.plan;
      const size_t want = (size_t)batch_targets(p, t.n_occ, t.n_b, limit[j]) * t.n_occ * p->N *
                          elem_bytes(p->prec) * (p->cplx ? 2 : 1);
      if ((p->ws_bytes > want) == (grow == 1)) continue;
      kx_status st = prepare_exx(p, t.n_occ, t.n_b, KX_PATH_FUSED, limit[j], limit[j] != 0);
      if (st != KX_OK) return st;
    }
  for (int i = 0; i < ntasks; ++i) {
    const kx_task& t = tasks[i];
    if (t.n_occ == 0 || t.n_b == 0) continue;
    size_t j = 0;
    while (plans[j] != t.plan) ++j;
    if (i == big[j]) continue;
    kx_status st = prepare_exx(t.plan, t.n_occ, t.n_b, KX_PATH_FUSED, limit[j], false);
    if (st != KX_OK) return st;
  }
  return KX_OK;
}

// Shape of the last captured schedule (kx_batched_schedule).
int g_last_sched[4] = {0, 0, 0, 0};

// The work-queue form of a schedule (one persistent launch, kernels_queue.hip):
// its tile shape, or false when a plan needs an element type or a tile count
// it has no instantiation for (the grouped-round form runs then).
bool queue_eligible(const kx_task* tasks, int ntasks, bool* f64, int* nkr, int* nkc) {
  const char* env = std::getenv("KX_BATCHED");
  if (env && std::strcmp(env, "rounds") == 0) return false;
  int nk_real = 1, nk_cplx = 1;
  bool any = false;
  for (int i = 0; i < ntasks; ++i) {
    const kx_plan p = tasks[i].plan;
    if (tasks[i].n_occ == 0 || tasks[i].n_b == 0) continue;
    if (p->prec != KX_PREC_FP64 && p->prec != KX_PREC_FP32) return false;
    const int nk = std::max(p->nk12, p->nk3);
    (p->cplx ? nk_cplx : nk_real) = std::max(p->cplx ? nk_cplx : nk_real, nk);
    *f64 = p->prec == KX_PREC_FP64;
    any = true;
  }
  return any && kx::queue_shape(nk_real, nk_cplx, nkr, nkc);
}

// Tickets and argument tables of the work queue for the batches of `rounds`
// (order and dependencies: queue_plan.h).  Virtual grids: passes A and C
// spread over the queue's grid, pass B over a multiple of its pencil chunks.
struct QueueBuild {
  std::vector<kx::QTicket> tickets;
  std::vector<kx::SliceArgs> sa;
  std::vector<kx::PencilArgs> pa;
  std::vector<kx::AccArgs> ca;
  std::vector<kx::QFin> fa;
  int nctr = 0;
};
QueueBuild build_queue(const kx_task* tasks, const std::vector<std::vector<SubTask>>& rounds, int grid) {
  QueueBuild q;
  std::vector<std::vector<kx::QBatchDesc>> desc;
  std::vector<bool> cplx;
  std::vector<int> fin_index;
  std::vector<const kx_plan_s*> plan_ids;
  for (const auto& round : rounds) {
    desc.emplace_back();
    for (const SubTask& st : round) {
      const kx_task& t = tasks[st.task];
      const kx_plan p = t.plan;
      const size_t vxw = p->cplx ? 2 : 1;
      const double* lo = t.d_vx + (size_t)st.n0 * t.ld_vx * vxw;
      const double* hi = lo + (size_t)(st.cur - 1) * t.ld_vx * vxw + (size_t)p->N * vxw;
      const BatchArgs ba = batch_args(p, t.d_psi, t.ld_psi, t.n_occ, t.d_occ, t.d_phi, t.ld_phi, t.d_vx, t.ld_vx,
                                      t.d_ex != nullptr, st.n0, st.cur);
      // the queue runs the FP64 / FP32 bodies of every pass
      q.sa.push_back(kernel_args_a(p, ba.A, false));
      q.pa.push_back(kernel_args_b(p, ba.B, false));
      q.ca.push_back(kernel_args_c(p, ba.C, false));
      fin_index.push_back(t.d_ex ? (int)q.fa.size() : -1);
      if (t.d_ex) q.fa.push_back(kx::QFin{p->d_part, st.cur, p->n[2], t.d_gphi + st.n0, p->dV, t.d_ex});
      cplx.push_back(p->cplx);
      int pid = 0;
      while (pid < (int)plan_ids.size() && plan_ids[pid] != p) ++pid;
      if (pid == (int)plan_ids.size()) plan_ids.push_back(p);
      const int64_t npairs = (int64_t)st.cur * t.n_occ;
      const int nch = std::max(ba.B.nchunks, 1);
      const int64_t groups = std::max<int64_t>(1, std::min<int64_t>(npairs, grid / nch));
      desc.back().push_back(kx::QBatchDesc{pid, (int)std::min<int64_t>(npairs * p->n[2], grid), (int)(groups * nch),
                                           (int)std::min<int64_t>((int64_t)st.cur * p->n[2], grid), t.d_ex ? 1 : 0,
                                           (uintptr_t)lo, (uintptr_t)hi});
    }
  }
  for (const kx::QTicketDesc& d : kx::queue_tickets(desc)) {
    kx::QTicket t{};
    t.kind = d.pass == 3 ? kx::QK_FINAL : d.pass + (cplx[d.batch] ? kx::QK_CPLX_A : kx::QK_REAL_A);
    t.arg = d.pass == 3 ? fin_index[d.batch] : d.batch;
    t.vb = d.vb;
    t.vg = d.vg;
    t.done = d.done;
    for (int i = 0; i < 3; ++i) {
      t.dep[i] = d.dep[i];
      t.need[i] = d.need[i];
    }
    q.tickets.push_back(t);
  }
  q.nctr = 4 * (int)cplx.size();
  return q;
}

// One launch of the grouped schedule: pass `pass` over the batches `subs`.
struct GroupLaunch {
  int pass;
  std::vector<SubTask> subs;
  size_t args_off = 0, pre_off = 0;  // byte offsets of its table in the device block
};

}  // namespace

}  // extern "C"

namespace {

// Capture the work-queue form (a counter reset, then one persistent launch)
// of a task list whose plans are prepared, cache and launch it.  Called with
// g_graph_mu held.
kx_status capture_queue(const kx_task* tasks, int ntasks, const std::vector<std::vector<SubTask>>& rounds,
                        bool f64, int nkr, int nkc, hipStream_t s) {
  const int grid = kx::queue_grid(f64, nkr, nkc);
  if (grid < 1) return fail(KX_EDEVICE, "exx_apply_batched: no work-queue kernel for this shape");
  const QueueBuild qb = build_queue(tasks, rounds, grid);
  // one device block: tickets | slice args | pencil args | acc args | finalize
  // args | counters | dispenser | error flag
  size_t off = 0;
  auto place = [&](size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    const size_t at = off;
    off += bytes;
    return at;
  };
  const size_t o_t = place(qb.tickets.size() * sizeof(kx::QTicket));
  const size_t o_sa = place(qb.sa.size() * sizeof(kx::SliceArgs));
  const size_t o_pa = place(qb.pa.size() * sizeof(kx::PencilArgs));
  const size_t o_ca = place(qb.ca.size() * sizeof(kx::AccArgs));
  const size_t o_fa = place(std::max<size_t>(1, qb.fa.size()) * sizeof(kx::QFin));
  const size_t o_ctr = place(std::max(1, qb.nctr) * sizeof(unsigned));
  const size_t o_next = place(sizeof(unsigned));
  const size_t o_err = place(sizeof(unsigned));
  const size_t bytes = place(0);
  std::vector<char> h(bytes, 0);
  std::memcpy(h.data() + o_t, qb.tickets.data(), qb.tickets.size() * sizeof(kx::QTicket));
  std::memcpy(h.data() + o_sa, qb.sa.data(), qb.sa.size() * sizeof(kx::SliceArgs));
  std::memcpy(h.data() + o_pa, qb.pa.data(), qb.pa.size() * sizeof(kx::PencilArgs));
  std::memcpy(h.data() + o_ca, qb.ca.data(), qb.ca.size() * sizeof(kx::AccArgs));
  if (!qb.fa.empty()) std::memcpy(h.data() + o_fa, qb.fa.data(), qb.fa.size() * sizeof(kx::QFin));
  char* d = nullptr;
  hipError_t e = hipMalloc((void**)&d, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(KX_ENOMEM, "exx_apply_batched: work-queue tables");
  }
  e = hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(d);
    return dev_fail(e, "exx_apply_batched: work-queue upload");
  }
  kx::QueueArgs qa{};
  qa.tickets = (const kx::QTicket*)(d + o_t);
  qa.ntickets = (int)qb.tickets.size();
  qa.sa = (const kx::SliceArgs*)(d + o_sa);
  qa.pa = (const kx::PencilArgs*)(d + o_pa);
  qa.ca = (const kx::AccArgs*)(d + o_ca);
  qa.fa = (const kx::QFin*)(d + o_fa);
  qa.ctr = (unsigned*)(d + o_ctr);
  qa.next = (unsigned*)(d + o_next);
  qa.err = (unsigned*)(d + o_err);
  qa.nctr = qb.nctr;
  qa.spin_limit = 1 << 24;  // polls of ~2 us: a wait gives up after about half a minute
  if (const char* env = std::getenv("KX_QUEUE_SPIN")) {  // 0: a wait not met at its first poll gives up
    const long long v = std::atoll(env);
    if (v >= 0 && *env) qa.spin_limit = v;
  }
  hipGraph_t graph = nullptr;
  hipStream_t cap = nullptr;
  e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e == hipSuccess) {
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) hipStreamDestroy(cap);
  }
  if (e != hipSuccess) {
    hipFree(d);
    return dev_fail(e, "exx_apply_batched capture");
  }
  e = kx::launch_queue(f64, nkr, nkc, qa, grid, cap);
  hipError_t e2 = hipStreamEndCapture(cap, &graph);
  hipStreamDestroy(cap);
  if (e == hipSuccess) e = e2;
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    hipFree(d);
    return dev_fail(e, "exx_apply_batched capture");
  }
  {
    int nsub = 0;
    for (const auto& r : rounds) nsub += (int)r.size();
    g_last_sched[0] = (int)rounds.size();
    g_last_sched[1] = nsub;
    g_last_sched[2] = 1;
    g_last_sched[3] = nsub;
  }
  std::vector<unsigned> gens(ntasks);
  for (int i = 0; i < ntasks; ++i) gens[i] = tasks[i].plan->gen;
  kx_graph_entry ge{std::vector<kx_task>(tasks, tasks + ntasks), gens, s, graph, exec, d, ++g_graph_clock};
  ge.d_err = qa.err;
  g_graphs.push_back(ge);
  ++g_graph_captures;
  e = hipGraphLaunch(exec, s);
  if (e != hipSuccess) return dev_fail(e, "exx_apply_batched launch");
  g_last_err = qa.err;
  g_last_err_stream = s;
  return KX_OK;
}

}  // namespace

extern "C" {

kx_status exx_apply_batched(const kx_task* tasks, int ntasks, void* stream) {
  if (ntasks < 0 || (ntasks > 0 && !tasks)) return fail(KX_EINVAL, "exx_apply_batched: bad task list");
  if (ntasks == 0) return KX_OK;
  const int prec0 = tasks[0].plan ? tasks[0].plan->prec : -1;
  for (int i = 0; i < ntasks; ++i) {
    const kx_task& t = tasks[i];
    kx_status st = check_exx_args(t.plan, t.d_psi, t.ld_psi, t.n_occ, t.d_occ, t.d_phi, t.ld_phi,
                                  t.n_b, t.d_vx, t.ld_vx, t.d_ex, t.d_gphi, KX_PATH_FUSED);
    if (st != KX_OK) return st;
    if (t.plan->prec != prec0) return fail(KX_EINVAL, "exx_apply_batched: mixed precisions");
  }
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_graph_mu);
  {
    kx_status st = prepare_batched(tasks, ntasks);
    if (st != KX_OK) return st;
  }
  bool qf64 = false;
  int nkr = 0, nkc = 0;
  const bool want_queue = queue_eligible(tasks, ntasks, &qf64, &nkr, &nkc);
  for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it) {
    kx_graph_entry& g = *it;
    if (g.stream != s || (int)g.tasks.size() != ntasks || (g.d_err != nullptr) != want_queue) continue;
    bool same = true;
    for (int i = 0; i < ntasks && same; ++i) same = same_task(g.tasks[i], tasks[i]);
    if (!same) continue;
    bool fresh = true;
    for (int i = 0; i < ntasks; ++i) fresh &= g.generations[i] == tasks[i].plan->gen;
    if (!fresh) {  // a workspace moved or a plan was retuned since capture
      (void)hipDeviceSynchronize();  // an earlier replay may still read its tables
      destroy_graph_entry(g);
      g_graphs.erase(it);
      break;
    }
    g.last_use = ++g_graph_clock;
    hipError_t e = hipGraphLaunch(g.exec, s);
    if (e != hipSuccess) return dev_fail(e, "exx_apply_batched replay");
    g_last_err = g.d_err;
    g_last_err_stream = s;
    return KX_OK;
  }
  if (g_graphs.size() >= kGraphCacheCap) {
    auto lru = g_graphs.begin();
    for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
      if (it->last_use < lru->last_use) lru = it;
    (void)hipDeviceSynchronize();
    destroy_graph_entry(*lru);
    g_graphs.erase(lru);
  }

  const std::vector<std::vector<SubTask>> rounds = schedule_rounds(tasks, ntasks);
  if (want_queue) return capture_queue(tasks, ntasks, rounds, qf64, nkr, nkc, s);
  // Grouped rounds: per round, the batches of each pass are grouped by kernel
  // instantiation; a group of several batches is one persistent launch over
  // a task table, a single batch launches with its own arguments.
  std::vector<GroupLaunch> launches;
  size_t tab_bytes = 0;
  auto arg_size = [](int pass) {
    return pass == 0 ? sizeof(kx::SliceArgs) : pass == 1 ? sizeof(kx::PencilArgs) : sizeof(kx::AccArgs);
  };
  for (const auto& round : rounds) {
    for (int pass = 0; pass < 3; ++pass) {
      std::vector<std::array<int, 6>> keys;
      std::vector<std::vector<SubTask>> groups;
      for (const SubTask& st : round) {
        const std::array<int, 6> k = launch_key(tasks[st.task].plan, pass);
        size_t gi = 0;
        while (gi < keys.size() && keys[gi] != k) ++gi;
        if (gi == keys.size()) {
          keys.push_back(k);
          groups.emplace_back();
        }
        groups[gi].push_back(st);
      }
      for (auto& g : groups) {
        GroupLaunch gl;
        gl.pass = pass;
        gl.subs = g;
        if (g.size() > 1) {
          tab_bytes = (tab_bytes + 255) & ~(size_t)255;
          gl.args_off = tab_bytes;
          tab_bytes += g.size() * arg_size(pass);
          tab_bytes = (tab_bytes + 7) & ~(size_t)7;
          gl.pre_off = tab_bytes;
          tab_bytes += (g.size() + 1) * sizeof(int64_t);
        }
        launches.push_back(std::move(gl));
      }
    }
  }
  {
    int nsub = 0, widest = 0;
    for (const auto& r : rounds) nsub += (int)r.size();
    for (const GroupLaunch& gl : launches) widest = std::max(widest, (int)gl.subs.size());
    g_last_sched[0] = (int)rounds.size();
    g_last_sched[1] = nsub;
    g_last_sched[2] = (int)launches.size();
    g_last_sched[3] = widest;
  }
  void* d_tab = nullptr;
  if (tab_bytes) {
    std::vector<char> h(tab_bytes, 0);
    for (const GroupLaunch& gl : launches) {
      if (gl.subs.size() < 2) continue;
      int64_t* pre = (int64_t*)(h.data() + gl.pre_off);
      pre[0] = 0;
      for (size_t j = 0; j < gl.subs.size(); ++j) {
        const SubTask& st = gl.subs[j];
        const kx_task& t = tasks[st.task];
        const kx_plan p = t.plan;
        const BatchArgs ba = batch_args(p, t.d_psi, t.ld_psi, t.n_occ, t.d_occ, t.d_phi, t.ld_phi, t.d_vx,
                                        t.ld_vx, t.d_ex != nullptr, st.n0, st.cur);
        int64_t items = 0;
        char* dst = h.data() + gl.args_off + j * arg_size(gl.pass);
        if (gl.pass == 0) {
          const kx::SliceArgs a = kernel_args_a(p, ba.A, pass_bf(p, 0));
          std::memcpy(dst, &a, sizeof(a));
          items = (int64_t)ba.A.npairs * p->n[2];
        } else if (gl.pass == 1) {
          const kx::PencilArgs b = kernel_args_b(p, ba.B, pass_bf(p, 1));
          std::memcpy(dst, &b, sizeof(b));
          items = (int64_t)ba.B.nchunks * ba.B.npairs;
        } else {
          const kx::AccArgs c = kernel_args_c(p, ba.C, pass_bf(p, 2));
          std::memcpy(dst, &c, sizeof(c));
          items = (int64_t)st.cur * p->n[2];
        }
        pre[j + 1] = pre[j] + items;
      }
    }
    hipError_t e = hipMalloc(&d_tab, tab_bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(KX_ENOMEM, "exx_apply_batched: task tables");
    }
    e = hipMemcpy(d_tab, h.data(), tab_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      hipFree(d_tab);
      return dev_fail(e, "exx_apply_batched: task table upload");
    }
  }

  // Capture on a private stream (capture is not allowed on the legacy default
  // stream); the instantiated graph is launched on the caller's stream.
  hipGraph_t graph = nullptr;
  hipStream_t cap = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e == hipSuccess) {
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) hipStreamDestroy(cap);
  }
  if (e != hipSuccess) {
    if (d_tab) hipFree(d_tab);
    return dev_fail(e, "exx_apply_batched capture");
  }
  size_t li = 0;
  for (size_t r = 0; r < rounds.size() && e == hipSuccess; ++r) {
    for (int pass = 0; pass < 3 && e == hipSuccess; ++pass) {
      for (; li < launches.size() && launches[li].pass == pass && e == hipSuccess; ++li) {
        const GroupLaunch& gl = launches[li];
        const SubTask& st0 = gl.subs[0];
        const kx_task& t0 = tasks[st0.task];
        const kx_plan p0 = t0.plan;
        const BatchArgs ba = batch_args(p0, t0.d_psi, t0.ld_psi, t0.n_occ, t0.d_occ, t0.d_phi, t0.ld_phi,
                                        t0.d_vx, t0.ld_vx, t0.d_ex != nullptr, st0.n0, st0.cur);
        kx::TaskTab tt = kx::kNoTasks;
        int64_t total = 0;
        if (gl.subs.size() > 1) {
          tt.args = (const char*)d_tab + gl.args_off;
          tt.pre = (const int64_t*)((const char*)d_tab + gl.pre_off);
          tt.ntasks = (int)gl.subs.size();
          for (const SubTask& st : gl.subs) {
            const kx_plan p = tasks[st.task].plan;
            const int64_t np = (int64_t)st.cur * tasks[st.task].n_occ;
            total += pass == 0 ? np * p->n[2] : pass == 1 ? (int64_t)((p->n12 + 63) / 64) * np
                                                          : (int64_t)st.cur * p->n[2];
          }
        }
        if (pass == 0) {
          e = launch_pass_a(p0, kx::SF_PAIR12, ba.A, tt.ntasks ? total : (int64_t)ba.A.npairs * p0->n[2], cap, tt);
        } else if (pass == 1) {
          e = launch_pass_b(p0, ba.B, cap, tt, total);
        } else {
          e = launch_pass_c(p0, kx::SI_ACC12, ba.C, tt.ntasks ? total : (int64_t)st0.cur * p0->n[2], cap, tt);
          // E_x of every batch of this launch
          for (size_t j = 0; j < gl.subs.size() && e == hipSuccess; ++j) {
            const SubTask& st = gl.subs[j];
            const kx_task& t = tasks[st.task];
            if (t.d_ex)
              e = kx::launch_ex_finalize(t.plan->d_part, st.cur, t.plan->n[2], t.d_gphi + st.n0, t.plan->dV,
                                         t.d_ex, cap);
          }
        }
      }
    }
  }
  hipError_t e2 = hipStreamEndCapture(cap, &graph);
  hipStreamDestroy(cap);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    if (d_tab) hipFree(d_tab);
    return dev_fail(e, "exx_apply_batched capture");
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(graph);
    if (d_tab) hipFree(d_tab);
    return dev_fail(e, "exx_apply_batched instantiate");
  }
  std::vector<unsigned> gens(ntasks);
  for (int i = 0; i < ntasks; ++i) gens[i] = tasks[i].plan->gen;
  g_graphs.push_back(kx_graph_entry{std::vector<kx_task>(tasks, tasks + ntasks), gens, s, graph, exec, d_tab,
                                    ++g_graph_clock});
  ++g_graph_captures;
  e = hipGraphLaunch(exec, s);
  if (e != hipSuccess) return dev_fail(e, "exx_apply_batched launch");
  return KX_OK;
}

kx_status kx_workspace_bytes(kx_plan p, int n_b, int n_occ, int64_t* bytes) {
  if (!p || !bytes) return fail(KX_EINVAL, "kx_workspace_bytes: NULL argument");
  if (n_b < 0 || n_occ < 0) return fail(KX_EINVAL, "kx_workspace_bytes: negative size");
  if (n_b == 0 || n_occ == 0) {
    *bytes = 0;
    return KX_OK;
  }
  const int nt = batch_targets(p, n_occ, n_b);
  const size_t eb = elem_bytes(p->prec) * (p->cplx ? 2 : 1);
  const size_t part = (size_t)nt * std::max<size_t>(64, (size_t)p->n[2]) * sizeof(double);
  *bytes = (int64_t)((size_t)nt * n_occ * p->N * eb + part);
  return KX_OK;
}

// ---------------------------------------------------------------------------
// ACE construction and application
// ---------------------------------------------------------------------------
namespace {
constexpr int kAceMaxNs = 1024;   // one workgroup factors / inverts the n_s x n_s matrix

struct AceWork {
  size_t part, small, total;
};
// One workspace serves ace_construct (Gram n_s x n_s) and ace_apply (Gram
// n_s x n_phi) for the same sizes.
AceWork ace_work(int64_t N, int n_s, int n_phi, int cplx) {
  const size_t eb = cplx ? 16 : 8;
  const size_t pc = (size_t)kx::ace_gram_part_bytes(cplx, N, n_s, n_s);
  const size_t pa = n_phi > 0 ? (size_t)kx::ace_gram_part_bytes(cplx, N, n_s, n_phi) : 0;
  AceWork w;
  w.part = (std::max(pc, pa) + 255) & ~(size_t)255;
  w.small = ((3 * (size_t)n_s * n_s + (size_t)n_s * std::max(n_phi, 1)) * eb + 255) & ~(size_t)255;
  w.total = w.part + w.small;
  return w;
}

kx_status check_ace(int64_t N, int n_s, int cplx, const void* a, int64_t lda, const void* b, int64_t ldb,
                    const void* c, int64_t ldc, const void* work, int64_t work_bytes, size_t need,
                    const char* who) {
  if (N <= 0 || n_s < 1 || n_s > kAceMaxNs)
    return fail(KX_EINVAL, "%s: need N > 0 and 1 <= n_s <= %d", who, kAceMaxNs);
  if (cplx != 0 && cplx != 1) return fail(KX_EINVAL, "%s: cplx must be 0 or 1", who);
  if (!a || !b || !c || !work) return fail(KX_EINVAL, "%s: NULL pointer", who);
  if (lda < N || ldb < N || ldc < N) return fail(KX_EINVAL, "%s: leading dimension below N", who);
  const size_t eb = cplx ? 16 : 8;
  if (((uintptr_t)a % eb) || ((uintptr_t)b % eb) || ((uintptr_t)c % eb) || ((uintptr_t)work % 256))
    return fail(KX_EINVAL, "%s: misaligned pointer (work needs 256-byte alignment)", who);
  if (work_bytes < 0 || (size_t)work_bytes < need)
    return fail(KX_EINVAL, "%s: workspace of %lld bytes, %zu needed", who, (long long)work_bytes, need);
  return KX_OK;
}
}  // namespace

kx_status kx_ace_workspace_bytes(int64_t N, int n_s, int n_phi, int cplx, int64_t* bytes) {
  if (!bytes) return fail(KX_EINVAL, "kx_ace_workspace_bytes: NULL argument");
  if (N <= 0 || n_s < 1 || n_s > kAceMaxNs || n_phi < 0 || (cplx != 0 && cplx != 1))
    return fail(KX_EINVAL, "kx_ace_workspace_bytes: bad sizes");
  *bytes = (int64_t)ace_work(N, n_s, n_phi, cplx).total;
  return KX_OK;
}

kx_status ace_construct(int64_t N, int n_s, int cplx, double dV, const void* d_psi, int64_t ld_psi,
                        const void* d_w, int64_t ld_w, void* d_xi, int64_t ld_xi, void* d_work,
                        int64_t work_bytes, int* d_info, void* stream) {
  const AceWork aw = ace_work(N > 0 ? N : 1, n_s > 0 ? n_s : 1, 0, cplx == 1);
  kx_status st = check_ace(N, n_s, cplx, d_psi, ld_psi, d_w, ld_w, d_xi, ld_xi, d_work, work_bytes, aw.total,
                           "ace_construct");
  if (st != KX_OK) return st;
  if (!d_info) return fail(KX_EINVAL, "ace_construct: NULL info");
  if (!(dV > 0.0)) return fail(KX_EINVAL, "ace_construct: dV must be positive");
  hipStream_t s = (hipStream_t)stream;
  const size_t eb = cplx ? 16 : 8;
  char* part = (char*)d_work;
  char* S = part + aw.part;
  char* U = S + (size_t)n_s * n_s * eb;
  char* X = U + (size_t)n_s * n_s * eb;
  // S = -M = -dV Psi^H W
  hipError_t e = kx::launch_ace_gram(cplx, N, n_s, n_s, d_psi, ld_psi, d_w, ld_w, -dV, part, S, s);
  // -M = L L^H, U = L^{-H}
  if (e == hipSuccess) e = kx::launch_ace_factor(cplx, n_s, S, U, X, d_info, s);
  if (e == hipSuccess) e = kx::launch_ace_tsmm(cplx, N, n_s, n_s, d_w, ld_w, U, 1.0, 0.0, d_xi, ld_xi, d_info, s);
  if (e != hipSuccess) return dev_fail(e, "ace_construct launch");
  return KX_OK;
}

kx_status ace_apply(int64_t N, int n_s, int cplx, double dV, const void* d_xi, int64_t ld_xi,
                    const void* d_phi, int64_t ld_phi, int n_phi, void* d_vphi, int64_t ld_vphi, void* d_work,
                    int64_t work_bytes, void* stream) {
  if (n_phi < 0) return fail(KX_EINVAL, "ace_apply: negative n_phi");
  if (n_phi == 0) return KX_OK;
  const AceWork aw = ace_work(N > 0 ? N : 1, n_s > 0 ? n_s : 1, n_phi, cplx == 1);
  kx_status st = check_ace(N, n_s, cplx, d_xi, ld_xi, d_phi, ld_phi, d_vphi, ld_vphi, d_work, work_bytes,
                           aw.total, "ace_apply");
  if (st != KX_OK) return st;
  if (!(dV > 0.0)) return fail(KX_EINVAL, "ace_apply: dV must be positive");
  hipStream_t s = (hipStream_t)stream;
  char* part = (char*)d_work;
  char* chi = part + aw.part;
  hipError_t e = kx::launch_ace_gram(cplx, N, n_s, n_phi, d_xi, ld_xi, d_phi, ld_phi, dV, part, chi, s);
  if (e == hipSuccess)
    e = kx::launch_ace_tsmm(cplx, N, n_s, n_phi, d_xi, ld_xi, chi, -1.0, 1.0, d_vphi, ld_vphi, nullptr, s);
  if (e != hipSuccess) return dev_fail(e, "ace_apply launch");
  return KX_OK;
}

kx_status kx_graph_cache_info(int64_t out[3]) {
  if (!out) return fail(KX_EINVAL, "kx_graph_cache_info: NULL argument");
  std::lock_guard<std::mutex> lock(g_graph_mu);
  out[0] = (int64_t)g_graphs.size();
  out[1] = (int64_t)kGraphCacheCap;
  out[2] = (int64_t)g_graph_captures;
  return KX_OK;
}

kx_status kx_batched_check(void* stream) {
  unsigned* err = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_graph_mu);
    err = g_last_err;
  }
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return dev_fail(e, "kx_batched_check");
  if (!err) return KX_OK;
  unsigned v = 0;
  e = hipMemcpy(&v, err, sizeof(v), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return dev_fail(e, "kx_batched_check");
  if (v) return fail(KX_EDEVICE, "exx_apply_batched: a work-queue wait gave up; results are incomplete");
  return KX_OK;
}

kx_status kx_batched_schedule(int out[4]) {
  if (!out) return fail(KX_EINVAL, "kx_batched_schedule: NULL argument");
  std::lock_guard<std::mutex> lock(g_graph_mu);
  for (int i = 0; i < 4; ++i) out[i] = g_last_sched[i];
  return KX_OK;
}

}  // extern "C"
