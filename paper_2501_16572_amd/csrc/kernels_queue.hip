// Work-queue kernel of exx_apply_batched: one persistent launch runs every
// pass of every batch of a batched call (several k-point blocks and systems
// of uneven sizes, the n_c batches of Sec. II.B), in place of rounds of
// grouped launches.
//
// Tickets (kernels.h, QTicket) are taken in order from a counter.  A ticket
// runs one virtual block of a pass body (the same bodies as the standalone
// kernels: pair density + forward modes 1, 2; mode 3 with the f scaling;
// inverse modes 2, 1 with the psi_m product and the Vx accumulation) or the
// fixed-order E_x finalize of a batch.  Before running, the block waits
// until the ticket's dependency counters are full: pass B of a batch after
// its pass A, pass C after B, the finalize after C; the next batch on a
// plan's workspace after the previous one's pass C; overlapping Vx outputs
// in task order; finalizes in ticket order.  All dependencies point to
// smaller ticket numbers, so the tickets waited on are held by running
// blocks and every wait ends; each wait is bounded as well, and one that
// gives up sets the error flag, which ends every block at its next ticket.
//
// Data produced by one block and read by another (possibly on another XCD,
// whose L2 is separate) is published with an agent-scope release fence by
// every thread before the completion count, and acquired with an
// agent-scope fence after the wait.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "kernels.h"
#include "kernels_real.inc"
#include "kernels_cplx.inc"
#include "launch.h"

namespace kx {
namespace {

template <typename T, int NKR, int NKC>
struct QShape {
  static constexpr int PR = Tiles<NKR>::P, PC = CTiles<NKC>::P;
  static constexpr int THREADS = 64 * (Tiles<NKR>::NT > CTiles<NKC>::NT ? Tiles<NKR>::NT : CTiles<NKC>::NT);
  static constexpr size_t lr_slice = (size_t)PR * (PR + 1), lr_pencil = (size_t)64 * (PR + 1);
  static constexpr size_t lc_slice = (size_t)PC * (PC + 1), lc_pencil = (size_t)PC * 65;
  static constexpr size_t m1 = lr_slice > lr_pencil ? lr_slice : lr_pencil;
  static constexpr size_t m2 = 2 * (lc_slice > lc_pencil ? lc_slice : lc_pencil);
  static constexpr size_t elems = m1 > m2 ? m1 : m2;  // LDS elements of T
};

// Orientation of the mode-2 product in the queue's slice passes: the
// transposed one for FP32 (at 120^3 FP32 pass A runs 207 ms per 64-band step
// transposed against 301 ms direct, pass C 354 against 477), the direct one
// for FP64, where the transposed one is the slower.
template <typename T>
constexpr bool kQTr2 = sizeof(T) == 4;

// The fixed-order E_x reduction of k_ex_finalize (256 partial sums, then a
// binary tree) with any block width.
__device__ __forceinline__ void ex_finalize_body(const QFin& f, double* red256) {
  const int total = f.n_t * f.per_target;
  for (int vt = threadIdx.x; vt < 256; vt += blockDim.x) {
    double s = 0.0;
    for (int i = vt; i < total; i += 256) s += f.gphi[i / f.per_target] * f.partials[i];
    red256[vt] = s;
  }
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    for (int vt = threadIdx.x; vt < off; vt += blockDim.x) red256[vt] += red256[vt + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *f.ex += f.dV * red256[0];
}

// Wait until ctr >= need (thread 0).  Returns false if the error flag is set
// or the poll budget runs out (then sets the flag).
__device__ bool wait_counter(const QueueArgs& q, int id, int need) {
  for (long long it = 0;; ++it) {
    const unsigned v = __hip_atomic_load(&q.ctr[id], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((int)v >= need) return true;
    if (__hip_atomic_load(q.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return false;
    if (it >= q.spin_limit) {
      __hip_atomic_fetch_or(q.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(64);
  }
}

template <typename T, int NKR, int NKC>
__global__ void __launch_bounds__((QShape<T, NKR, NKC>::THREADS))
k_queue(QueueArgs q) {
  using Sh = QShape<T, NKR, NKC>;
  __shared__ __align__(16) T lds[Sh::elems];
  __shared__ double red[256];
  __shared__ int s_t, s_go;
  const TaskTab none{nullptr, nullptr, 0};
  // One thread-0 section per iteration (count the finished ticket, take the
  // next one, wait for its dependencies) and a loop exit read back with
  // readfirstlane: the loop is uniform, so every wave meets every barrier
  // with all its lanes (two thread-0 sections around the back edge would
  // let the compiler thread one into the other and split wave 0 at the
  // top barrier).
  int done = -1;  // counter of the ticket this block finished last (thread 0)
  for (;;) {
    if (threadIdx.x == 0) {
      // release: every thread's writes of the last ticket were fenced before
      // the barrier that ended it; then its completion count
      if (done >= 0) __hip_atomic_fetch_add(&q.ctr[done], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned t = atomicAdd(q.next, 1u);
      int go = t < (unsigned)q.ntickets &&
               __hip_atomic_load(q.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
      if (go) {
        const QTicket& d = q.tickets[t];
        for (int i = 0; i < 3 && go; ++i)
          if (d.dep[i] >= 0) go = wait_counter(q, d.dep[i], d.need[i]);
        done = d.done;
      }
      s_t = (int)t;
      s_go = go;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_go) == 0) break;
    const int tk = __builtin_amdgcn_readfirstlane(s_t);
    // acquire: what the tickets waited on wrote is visible from here on
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const QTicket d = q.tickets[tk];
    switch (d.kind) {
      case QK_REAL_A:
        slice_fwd_body<T, NKR, 0, true, true, false, kQTr2<T>>(q.sa[d.arg], none, d.vb, d.vg, lds);
        break;
      case QK_REAL_B:
        pencil_body<T, NKR, true, true, true>(q.pa[d.arg], none, d.vb, d.vg, lds);
        break;
      case QK_REAL_C:
        slice_inv_body<T, NKR, true, true, true, false, kQTr2<T>>(q.ca[d.arg], none, d.vb, d.vg, lds, red);
        break;
      case QK_CPLX_A:
        slice_fwd_c_body<T, NKC, 0>(q.sa[d.arg], none, d.vb, d.vg, lds, lds + Sh::lc_slice);
        break;
      case QK_CPLX_B:
        pencil_c_body<T, NKC>(q.pa[d.arg], none, d.vb, d.vg, lds, lds + Sh::lc_pencil);
        break;
      case QK_CPLX_C:
        slice_inv_c_body<T, NKC, true>(q.ca[d.arg], none, d.vb, d.vg, lds, lds + Sh::lc_slice, red);
        break;
      default:
        ex_finalize_body(q.fa[d.arg], red);
        break;
    }
    // every thread's writes of this ticket, before thread 0 counts it at the
    // top of the next iteration
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
  }
}

// Counters, dispenser and error flag to zero before each replay (a kernel,
// so that a captured graph holds no memset node).
__global__ void k_queue_reset(unsigned* next, unsigned* ctr, int nctr, unsigned* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nctr) ctr[i] = 0u;
  if (i == 0) {
    *next = 0u;
    *err = 0u;
  }
}

template <typename K>
int q_resident(K kernel, int threads) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find((const void*)kernel);
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) nb = 1;
  cache[(const void*)kernel] = nb;
  return nb;
}

// Instantiated tile counts: real plans up to NKR K steps on the slices and
// pencils, complex plans up to NKC.
constexpr int kQReal[] = {12, 24, 30};
constexpr int kQCplx[] = {12, 20};

template <typename T>
void* q_kernel(int nkr, int nkc, int* threads) {
#define KX_Q(R, C)                                  \
  if (nkr == R && nkc == C) {                       \
    *threads = QShape<T, R, C>::THREADS;            \
    return (void*)k_queue<T, R, C>;                 \
  }
  KX_Q(12, 12) KX_Q(12, 20) KX_Q(24, 12) KX_Q(24, 20) KX_Q(30, 12) KX_Q(30, 20)
#undef KX_Q
  return nullptr;
}

}  // namespace

bool queue_shape(int nk_real, int nk_cplx, int* nkr, int* nkc) {
  *nkr = *nkc = -1;
  for (int v : kQReal)
    if (v >= nk_real) {
      *nkr = v;
      break;
    }
  for (int v : kQCplx)
    if (v >= nk_cplx) {
      *nkc = v;
      break;
    }
  return *nkr > 0 && *nkc > 0;
}

int queue_grid(bool f64, int nkr, int nkc) {
  int th = 0;
  void* k = f64 ? q_kernel<double>(nkr, nkc, &th) : q_kernel<float>(nkr, nkc, &th);
  if (!k) return 0;
  const int nb = f64 ? q_resident((void (*)(QueueArgs))k, th) : q_resident((void (*)(QueueArgs))k, th);
  return nb * device_cu_count();
}

hipError_t launch_queue(bool f64, int nkr, int nkc, const QueueArgs& q, int grid, hipStream_t s) {
  int th = 0;
  void* k = f64 ? q_kernel<double>(nkr, nkc, &th) : q_kernel<float>(nkr, nkc, &th);
  if (!k || grid < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_queue_reset, dim3((q.nctr + 255) / 256 > 0 ? (q.nctr + 255) / 256 : 1), dim3(256), 0, s,
                     q.next, q.ctr, q.nctr, q.err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((void (*)(QueueArgs))k, dim3(grid), dim3(th), 0, s, q);
  return hipGetLastError();
}

}  // namespace kx
