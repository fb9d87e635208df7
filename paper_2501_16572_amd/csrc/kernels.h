// Device kernels of the batched Kronecker-product solver for gfx950.
//
// Data layout (Sec. II.A): a grid function is N = n1*n2*n3 contiguous values,
// flat index i1 + n1*(i2 + n2*i3); a frontal slice (fixed i3) is n1*n2
// contiguous values; an x3 pencil (fixed i1, i2) has stride n1*n2.  A batch
// is a set of such functions at a fixed stride (one "pair" each).
//
// The six mode products of the batch solve (Sec. II.B) are dense matrix
// products with the 1D eigenvector matrices.  With x1 fastest they are
// products on strided views, so the reorganizations [1]-[4] of Sec. II.B are
// never materialized:
//   mode 1: per slice, V1^T S (forward) / V1 S (inverse),
//   mode 2: per slice, S V2 (forward) / S V2^T (inverse),
//   mode 3: per chunk of x3 pencils, P V3 (forward) / P V3^T (inverse).
// Each kernel stages one slice (or one pencil chunk) in LDS and runs 16x16
// MFMA tiles over it; the eigenvector operand of every tile is held in
// registers, the data operand is read from LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kx {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// Arguments of the slice kernels (modes 1 and 2).
struct SliceArgs {
  int n1, n2, n3, n12;
  int64_t N;
  int npairs;             // number of batch entries (pairs or right-hand sides)
  int n_occ;              // pairs are (target t, occupied m), p = t*n_occ + m
  // pair-density input: rho_p = conj(psi_m) * phi_t
  const void* psi; int64_t ld_psi;
  const void* phi; int64_t ld_phi;
  // plain input: src + p*ld_src
  const void* src; int64_t ld_src;
  // output: dst + p*ld_dst
  void* dst; int64_t ld_dst;
  const void* V1; const void* V2;  // padded P x P, V[k*P + a], plan element type
  int P;
};

// Arguments of the pencil kernel (mode 3 and the eigen-scaling).
struct PencilArgs {
  int n1, n2, n3, n12;
  int npairs;
  int nchunks;            // ceil(n12 / Q)
  void* T; int64_t ld;    // in place: T + p*ld
  const void* V3;         // padded P3 x P3, V3[k*P3 + c]
  const void* V3T;        // its transpose
  int P3;
  const double* ftab;     // N doubles, f(lambda) in the flat grid order
};

// Arguments of the inverse slice kernel with accumulation into Vx.
struct AccArgs {
  int n1, n2, n3, n12;
  int64_t N;
  int n_t, n_occ;         // targets in this batch, occupied orbitals
  const void* T; int64_t ld_T;       // pair p = t*n_occ + m at T + p*ld_T
  const void* psi; int64_t ld_psi;   // occupied orbitals (for psi_m * phi_mn)
  const double* occ;                 // n_occ weights; the accumulated term is -occ[m]
  const void* phi; int64_t ld_phi;   // targets (for the E_x partials)
  double* vx; int64_t ld_vx;         // target t of this batch at vx + t*ld_vx
  double* partials;                  // n_t * n3 doubles (E_x partials) or null
  void* dst; int64_t ld_dst;         // solve mode: Y stored at dst + p*ld_dst
  const void* V1; const void* V2;    // TRANSPOSED padded matrices V1^T, V2^T
  int P;
};

// Several batches in one persistent launch (the batched entry point): the
// launch's flat item space is the concatenation of the entries' item spaces,
// entry i owning items [pre[i], pre[i+1]); its arguments are args[i], an
// array of the pass's argument struct in device memory.  ntasks = 0: one
// batch, described by the kernel's own argument struct.
struct TaskTab {
  const void* args;
  const int64_t* pre;
  int ntasks;
};

// Work queue of the batched entry point (one persistent launch for a whole
// task list).  A ticket is one virtual block (vb of a virtual grid of vg
// blocks) of one pass of one batch, or the E_x finalize of a batch; blocks
// take tickets in order from a shared counter, wait until the counters named
// in dep[] have reached need[], run the ticket and increment counter `done`.
// Every dependency is on tickets with a smaller number, which were taken by
// running blocks, so every wait ends; each wait is also bounded (spin_limit
// polls), and a wait that gives up sets *err and ends its block.
enum QKind { QK_REAL_A = 0, QK_REAL_B, QK_REAL_C, QK_CPLX_A, QK_CPLX_B, QK_CPLX_C, QK_FINAL };
struct QTicket {
  int kind, arg, vb, vg, done;
  int dep[3], need[3];
};
struct QFin {  // E_x finalize: *ex += dV sum_t gphi[t] sum_j partials[t * per_target + j]
  const double* partials;
  int n_t, per_target;
  const double* gphi;
  double dV;
  double* ex;
};
struct QueueArgs {
  const QTicket* tickets;
  int ntickets;
  const SliceArgs* sa;
  const PencilArgs* pa;
  const AccArgs* ca;
  const QFin* fa;
  unsigned* next;         // ticket dispenser
  unsigned* ctr;          // completion counters
  unsigned* err;          // nonzero once a wait gave up
  int nctr;
  long long spin_limit;   // retries after a wait's first poll (each after a sleep of ~2 us)
};

// Entry of flat item g: its index, a copy of its argument struct, and the
// item's index within it.  The table is read through the constant address
// space (it does not change during a launch), so the loads are scalar and the
// arguments stay in SGPRs as kernel arguments do.  A linear scan: a launch
// holds a few dozen entries at most.
template <typename A>
__device__ __forceinline__ A task_args(const TaskTab& tt, int64_t g, int64_t& item, int& t) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef __attribute__((address_space(4))) const int64_t cpre_t;
  typedef __attribute__((address_space(4))) const A cargs_t;
#else  // the host pass only parses device functions
  typedef const int64_t cpre_t;
  typedef const A cargs_t;
#endif
  cpre_t* pre = (cpre_t*)tt.pre;
  t = 0;
  while (t + 1 < tt.ntasks && pre[t + 1] <= g) ++t;
  item = g - pre[t];
  return ((cargs_t*)tt.args)[t];
}

}  // namespace kx
