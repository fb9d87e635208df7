"""Thin Python binding of ``libkronx.so`` (argument marshalling only).

Every step of the exact-exchange path runs in the library's HIP kernels; this
module converts torch tensors to pointers, leading dimensions and the current
HIP stream, and raises on a non-OK status.  It raises ImportError-like
``RuntimeError`` when the library has not been built: there is no fallback.

Tensor conventions: a set of grid functions is a 2D tensor of shape
(ncols, N) with unit stride along N (one grid function per row, i.e. the
column-major N x ncols matrix of the C interface); the leading dimension is
the row stride.  Real plans take float64 (FP64) or float32 (other precisions);
complex plans take complex128 / complex64.  Vx outputs are float64 /
complex128.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkronx.so")

KX_OK, KX_EINVAL, KX_EUNSUPPORTED, KX_ENOMEM, KX_EDEVICE, KX_ESTATE = range(6)
STATUS_NAMES = {0: "KX_OK", 1: "KX_EINVAL", 2: "KX_EUNSUPPORTED", 3: "KX_ENOMEM",
                4: "KX_EDEVICE", 5: "KX_ESTATE"}
BC = {"periodic": 0, "dirichlet": 1}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
PATH = {"fused": 0, "plain": 1, "slicewise": 2}
FLAG_COMPLEX = 16

# Every symbol declared in include/kronx.h.
EXPORTS = ["kron_setup", "kron_destroy", "kron_solve", "exx_apply", "exx_apply_batched",
           "kx_plan_info", "kx_plan_tables", "kx_host_eig1d", "kx_host_fd_weights",
           "kx_last_error", "kx_trace_enable", "kx_trace_read", "kx_trace_name", "kx_autotune",
           "kx_plan_tuning", "kx_batched_schedule", "kx_workspace_bytes", "kx_ace_workspace_bytes",
           "ace_construct", "ace_apply", "kx_graph_cache_info", "exx_apply_static",
           "kx_static_scratch_bytes", "kx_batched_check"]


class KronxError(RuntimeError):
    def __init__(self, status, where, text):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {text}")
        self.status = status


class _Task(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("d_psi", ctypes.c_void_p), ("ld_psi", ctypes.c_int64),
                ("n_occ", ctypes.c_int), ("d_occ", ctypes.c_void_p), ("d_phi", ctypes.c_void_p),
                ("ld_phi", ctypes.c_int64), ("n_b", ctypes.c_int), ("d_vx", ctypes.c_void_p),
                ("ld_vx", ctypes.c_int64), ("d_ex", ctypes.c_void_p), ("d_gphi", ctypes.c_void_p)]


_lib = None


def load_library(path=None):
    """Load libkronx.so once; raise if it is missing (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libkronx.so not built at {path}: run __graft_entry__.build() "
                           "or python -m paper_2501_16572_amd.build")
    lib = ctypes.CDLL(path)
    vp, i64, ci, cd = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    ip = ctypes.POINTER(ctypes.c_int)
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.kron_setup.argtypes = [ip, dp, ip, ci, cd, dp, ci, ctypes.POINTER(vp)]
    lib.kron_destroy.argtypes = [vp]
    lib.kron_solve.argtypes = [vp, vp, i64, vp, i64, ci, ci, vp]
    lib.exx_apply.argtypes = [vp, vp, i64, ci, vp, vp, i64, ci, vp, i64, vp, vp, ci, vp]
    lib.exx_apply_static.argtypes = [vp, vp, i64, ci, vp, vp, i64, ci, vp, i64, vp, vp, ci, vp]
    lib.kx_static_scratch_bytes.argtypes = []
    lib.exx_apply_batched.argtypes = [ctypes.POINTER(_Task), ci, vp]
    lib.kx_batched_check.argtypes = [vp]
    lib.kx_plan_info.argtypes = [vp, i64p]
    lib.kx_plan_tables.argtypes = [vp, ci, dp, dp, dp]
    lib.kx_host_eig1d.argtypes = [ci, cd, ci, ci, cd, dp, dp, dp]
    lib.kx_host_fd_weights.argtypes = [ci, dp]
    lib.kx_last_error.restype = ctypes.c_char_p
    lib.kx_trace_enable.argtypes = [ci]
    lib.kx_trace_read.argtypes = [dp, i64p, ci]
    lib.kx_trace_name.argtypes = [ci]
    lib.kx_trace_name.restype = ctypes.c_char_p
    lib.kx_autotune.argtypes = [vp, vp, i64, ci, vp, vp, i64, ci, vp]
    lib.kx_plan_tuning.argtypes = [vp, ip]
    lib.kx_batched_schedule.argtypes = [ip]
    lib.kx_graph_cache_info.argtypes = [i64p]
    lib.kx_workspace_bytes.argtypes = [vp, ci, ci, ctypes.POINTER(i64)]
    lib.kx_ace_workspace_bytes.argtypes = [i64, ci, ci, ci, ctypes.POINTER(i64)]
    lib.ace_construct.argtypes = [i64, ci, ci, cd, vp, i64, vp, i64, vp, i64, vp, i64, vp, vp]
    lib.ace_apply.argtypes = [i64, ci, ci, cd, vp, i64, vp, i64, ci, vp, i64, vp, i64, vp]
    for name in EXPORTS:
        if name not in ("kx_last_error", "kx_trace_name", "kx_static_scratch_bytes"):
            getattr(lib, name).restype = ci
    lib.kx_static_scratch_bytes.restype = ctypes.c_size_t
    _lib = lib
    return lib


def kx_last_error():
    return load_library().kx_last_error().decode()


def _check(status, where):
    if status != KX_OK:
        raise KronxError(status, where, kx_last_error())


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """Handle of a kx_plan (kron_setup's output)."""

    def __init__(self, handle, n, h, bc, order, omega, kq, prec, complex_=False):
        self.handle = handle
        self.n, self.h, self.bc = tuple(n), tuple(h), tuple(bc)
        self.order, self.omega, self.kq, self.prec = order, omega, tuple(kq), prec
        self.complex = complex_ or any(k != 0.0 for k in self.kq)
        self.N = int(np.prod(self.n))
        self.dV = float(np.prod(self.h))

    @property
    def real_dtype(self):
        import torch
        return torch.float64 if self.prec == "fp64" else torch.float32

    @property
    def dtype(self):
        import torch
        if self.complex:
            return torch.complex128 if self.prec == "fp64" else torch.complex64
        return self.real_dtype

    def info(self):
        out = (ctypes.c_int64 * 8)()
        _check(load_library().kx_plan_info(self.handle, out), "kx_plan_info")
        return list(out)

    def tables(self, axis):
        """Host FP64 tables: (lam, V) for axis 0..2 (V[k, a]), or the f table for axis 3."""
        lib = load_library()
        if axis == 3:
            f = np.empty(self.N)
            _check(lib.kx_plan_tables(self.handle, 3, _dptr(f), None, None), "kx_plan_tables")
            return f
        nd = self.n[axis]
        lam = np.empty(nd)
        vr = np.empty((nd, nd))
        vi = np.empty((nd, nd))
        _check(lib.kx_plan_tables(self.handle, axis, _dptr(lam), _dptr(vr), _dptr(vi)),
               "kx_plan_tables")
        return lam, (vr + 1j * vi if self.complex else vr)

    def tuning(self):
        """{pass: (variant bits, blocks per CU)} and whether it was autotuned.

        Variant bits: 1 = alternative occupancy target, 2 = transposed mode-2
        product (passes A and C), 4 = eigenvector matrices resident in LDS
        (passes B and C)."""
        out = (ctypes.c_int * 7)()
        _check(load_library().kx_plan_tuning(self.handle, out), "kx_plan_tuning")
        return {"A": (out[0], out[1]), "B": (out[2], out[3]), "C": (out[4], out[5]),
                "tuned": bool(out[6])}

    def destroy(self):
        if self.handle:
            _check(load_library().kron_destroy(self.handle), "kron_destroy")
            self.handle = None


def kron_setup(n, h, bc=("periodic",) * 3, fd_order=12, omega=0.0, kq=None, prec="fp64",
               complex=False):
    """Plan for X = f(L) B.  complex=True forces complex data at k - q = 0."""
    lib = load_library()
    bcs = [BC[b] if isinstance(b, str) else int(b) for b in bc]
    kqv = (ctypes.c_double * 3)(*kq) if kq is not None else None
    handle = ctypes.c_void_p()
    st = lib.kron_setup((ctypes.c_int * 3)(*n), (ctypes.c_double * 3)(*h), (ctypes.c_int * 3)(*bcs),
                        int(fd_order), float(omega), kqv, PREC[prec] | (FLAG_COMPLEX if complex else 0),
                        ctypes.byref(handle))
    _check(st, "kron_setup")
    return Plan(handle, n, h, bc, fd_order, omega, kq if kq is not None else (0.0, 0.0, 0.0), prec,
                complex_=complex)


def kron_destroy(plan):
    plan.destroy()


def _cols(t, N, what):
    if t.dim() != 2 or (t.stride(1) != 1 and t.shape[1] > 1) or t.shape[1] < N:
        raise ValueError(f"{what}: expected a (ncols, >=N) tensor with unit stride along the grid")
    # with a single column the row stride is arbitrary (torch and numpy may
    # report any value for a dimension of size 1): N is a valid leading dimension
    ld = t.stride(0) if t.shape[0] > 1 else max(t.stride(0), N)
    return t.data_ptr(), ld


def _on_device(t, what):
    if not t.is_cuda:
        raise ValueError(f"{what}: must be a GPU tensor (got device {t.device})")


def _grid_set(t, N, dtype, what, rows=None):
    """A (ncols, N) set of grid functions of `dtype` on the GPU, with at least
    `rows` rows when given; returns (pointer, leading dimension)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what}: expected a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{what}: dtype {t.dtype}, the plan needs {dtype}")
    out = _cols(t, N, what)
    if rows is not None and t.shape[0] < rows:
        raise ValueError(f"{what}: {t.shape[0]} rows, at least {rows} needed")
    return out


def _vector(t, n, dtype, what):
    """A contiguous GPU vector of `dtype` with at least n entries; its pointer."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what}: expected a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{what}: dtype {t.dtype}, {dtype} needed")
    if not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"{what}: a contiguous tensor of at least {n} entries is needed "
                         f"(got {tuple(t.shape)})")
    return t.data_ptr()


def _all_on_device(**tensors):
    """After the shape and type checks: every tensor must live on the GPU."""
    for what, t in tensors.items():
        if t is not None:
            _on_device(t, what)


def _vx_dtype(plan):
    import torch
    return torch.complex128 if plan.complex else torch.float64


def _exx_args(plan, psi, occ, phi, vx, ex, gphi):
    """Pointers and leading dimensions of one exx_apply call, every tensor
    checked against the plan before the library sees it."""
    import torch
    N = plan.N
    pp, ldp = _grid_set(psi, N, plan.dtype, "psi")
    pf, ldf = _grid_set(phi, N, plan.dtype, "phi")
    n_occ, n_b = psi.shape[0], phi.shape[0]
    pv, ldv = _grid_set(vx, N, _vx_dtype(plan), "vx", rows=n_b)
    po = _vector(occ, n_occ, torch.float64, "occ")
    pe = pg = None
    if ex is not None:
        pe = _vector(ex, 1, torch.float64, "ex")
        if gphi is None:
            raise ValueError("ex given without gphi")
    if gphi is not None:
        pg = _vector(gphi, n_b, torch.float64, "gphi")
    _all_on_device(psi=psi, phi=phi, vx=vx, occ=occ, ex=ex, gphi=gphi)
    return dict(psi=(pp, ldp, n_occ), phi=(pf, ldf, n_b), vx=(pv, ldv), occ=po, ex=pe, gphi=pg)


def kron_solve(plan, B, X=None, path="fused", stream=None):
    """X = f(L) B for the rows of B (shape (nrhs, N)); returns X.

    path: "fused" (three fused passes), "plain" (one kernel per step, FP64)
    or "slicewise" (the original formalism of Sec. II.A, one GEMM launch per
    frontal slice; FP64 real plans; the comparison point for batching)."""
    import torch
    if X is None:
        X = torch.empty_like(B)
    pb, ldb = _grid_set(B, plan.N, plan.dtype, "B")
    px, ldx = _grid_set(X, plan.N, plan.dtype, "X", rows=B.shape[0])
    _all_on_device(B=B, X=X)
    st = load_library().kron_solve(plan.handle, ctypes.c_void_p(pb), ldb, ctypes.c_void_p(px), ldx,
                                   B.shape[0], PATH[path], _stream(stream))
    _check(st, "kron_solve")
    return X


def exx_apply(plan, psi, occ, phi, vx, ex=None, gphi=None, path="fused", stream=None):
    """vx[n] += -sum_m occ[m] psi[m] * f(L)(conj(psi[m]) * phi[n]); ex += dV sum_n gphi[n] <phi_n, dvx_n>.

    psi: (n_occ, N), occ: (n_occ,) float64, phi: (n_b, N), vx: (n_b, N) float64
    (complex128 for complex plans), ex: (1,) float64 or None, gphi: (n_b,) float64.
    psi and phi have the plan's element type (plan.dtype).  All GPU tensors;
    a tensor that does not fit raises ValueError before the library is called.
    Returns vx.
    """
    a = _exx_args(plan, psi, occ, phi, vx, ex, gphi)
    pp, ldp, n_occ = a["psi"]
    pf, ldf, n_b = a["phi"]
    pv, ldv = a["vx"]
    st = load_library().exx_apply(
        plan.handle, ctypes.c_void_p(pp), ldp, n_occ, ctypes.c_void_p(a["occ"]),
        ctypes.c_void_p(pf), ldf, n_b, ctypes.c_void_p(pv), ldv,
        ctypes.c_void_p(a["ex"]) if a["ex"] is not None else None,
        ctypes.c_void_p(a["gphi"]) if a["gphi"] is not None else None,
        PATH[path], _stream(stream))
    _check(st, "exx_apply")
    return vx


def exx_apply_static(plan, psi, occ, phi, vx, ex=None, gphi=None, path="fused", stream=None):
    """exx_apply without any device allocation: the library's fixed device
    array (kx_static_scratch_bytes()) holds the pair workspace.  Same
    arguments and result as exx_apply; calls that overlap on one GPU race."""
    a = _exx_args(plan, psi, occ, phi, vx, ex, gphi)
    pp, ldp, n_occ = a["psi"]
    pf, ldf, n_b = a["phi"]
    pv, ldv = a["vx"]
    st = load_library().exx_apply_static(
        plan.handle, ctypes.c_void_p(pp), ldp, n_occ, ctypes.c_void_p(a["occ"]),
        ctypes.c_void_p(pf), ldf, n_b, ctypes.c_void_p(pv), ldv,
        ctypes.c_void_p(a["ex"]) if a["ex"] is not None else None,
        ctypes.c_void_p(a["gphi"]) if a["gphi"] is not None else None,
        PATH[path], _stream(stream))
    _check(st, "exx_apply_static")
    return vx


def kx_static_scratch_bytes():
    return int(load_library().kx_static_scratch_bytes())


def kx_autotune(plan, psi, occ, phi, stream=None):
    """Pick the fused passes' launch configuration on this workload (synchronous)."""
    import torch
    pp, ldp = _grid_set(psi, plan.N, plan.dtype, "psi")
    pf, ldf = _grid_set(phi, plan.N, plan.dtype, "phi")
    po = _vector(occ, psi.shape[0], torch.float64, "occ")
    _all_on_device(psi=psi, phi=phi, occ=occ)
    st = load_library().kx_autotune(plan.handle, ctypes.c_void_p(pp), ldp, psi.shape[0],
                                    ctypes.c_void_p(po), ctypes.c_void_p(pf), ldf,
                                    phi.shape[0], _stream(stream))
    _check(st, "kx_autotune")
    return plan.tuning()


def kx_batched_check(stream=None):
    """Wait for the stream; raise if the last work-queue replay ended early."""
    _check(load_library().kx_batched_check(_stream(stream)), "kx_batched_check")


def exx_apply_batched(tasks, stream=None):
    """tasks: list of dicts with keys plan, psi, occ, phi, vx, ex (opt), gphi (opt),
    each checked as exx_apply checks its arguments."""
    arr = (_Task * len(tasks))()
    for i, t in enumerate(tasks):
        plan = t["plan"]
        a = _exx_args(plan, t["psi"], t["occ"], t["phi"], t["vx"], t.get("ex"), t.get("gphi"))
        pp, ldp, n_occ = a["psi"]
        pf, ldf, n_b = a["phi"]
        pv, ldv = a["vx"]
        arr[i] = _Task(plan.handle.value, pp, ldp, n_occ, a["occ"], pf, ldf, n_b, pv, ldv, a["ex"], a["gphi"])
    _check(load_library().exx_apply_batched(arr, len(tasks), _stream(stream)), "exx_apply_batched")


def kx_workspace_bytes(plan, n_b, n_occ):
    """Device bytes exx_apply on `plan` holds for n_b targets x n_occ occupied."""
    out = ctypes.c_int64(0)
    _check(load_library().kx_workspace_bytes(plan.handle, n_b, n_occ, ctypes.byref(out)),
           "kx_workspace_bytes")
    return out.value


def kx_ace_workspace_bytes(N, n_s, n_phi, cplx):
    out = ctypes.c_int64(0)
    _check(load_library().kx_ace_workspace_bytes(N, n_s, n_phi, 1 if cplx else 0, ctypes.byref(out)),
           "kx_ace_workspace_bytes")
    return out.value


def _ace_work(N, n_s, n_phi, cplx, work):
    import torch
    need = kx_ace_workspace_bytes(N, n_s, n_phi, cplx)
    if work is None:
        return torch.empty(need // 8 + 64, dtype=torch.float64, device="cuda")
    if not isinstance(work, torch.Tensor) or not work.is_contiguous():
        raise ValueError("work: expected a contiguous torch tensor")
    if work.numel() * work.element_size() < need:
        raise ValueError(f"work: {work.numel() * work.element_size()} bytes, {need} needed")
    return work


def _ace_dtype(t, what):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype not in (torch.float64, torch.complex128):
        raise ValueError(f"{what}: expected a float64 or complex128 torch tensor")
    return t.dtype


def ace_construct(psi, w, dV, xi=None, work=None, stream=None):
    """xi (n_s, N) of the ACE operator from psi and w = Vx psi (both (n_s, N),
    float64 or complex128, GPU).  Raises if -dV psi^H w is not positive definite."""
    import torch
    dt = _ace_dtype(psi, "psi")
    n_s, N = psi.shape
    cplx = psi.is_complex()
    if xi is None:
        xi = torch.empty_like(w)
    pp, ldp = _grid_set(psi, N, dt, "psi")
    pw, ldw = _grid_set(w, N, dt, "w", rows=n_s)
    px, ldx = _grid_set(xi, N, dt, "xi", rows=n_s)
    work = _ace_work(N, n_s, 0, cplx, work)
    _all_on_device(psi=psi, w=w, xi=xi, work=work)
    info = torch.zeros(1, dtype=torch.int32, device=psi.device)
    st = load_library().ace_construct(N, n_s, 1 if cplx else 0, float(dV), ctypes.c_void_p(pp), ldp,
                                      ctypes.c_void_p(pw), ldw, ctypes.c_void_p(px), ldx,
                                      ctypes.c_void_p(work.data_ptr()),
                                      work.numel() * work.element_size(),
                                      ctypes.c_void_p(info.data_ptr()), _stream(stream))
    _check(st, "ace_construct")
    if int(info.item()) != 0:
        raise KronxError(KX_EINVAL, "ace_construct", f"-M not positive definite at pivot {int(info.item())}")
    return xi


def ace_apply(xi, phi, dV, vphi, work=None, stream=None):
    """vphi += -xi (dV xi^H phi); xi (n_s, N), phi and vphi (n_phi, N), one dtype."""
    dt = _ace_dtype(xi, "xi")
    n_s, N = xi.shape
    cplx = xi.is_complex()
    px, ldx = _grid_set(xi, N, dt, "xi")
    pf, ldf = _grid_set(phi, N, dt, "phi")
    pv, ldv = _grid_set(vphi, N, dt, "vphi", rows=phi.shape[0])
    work = _ace_work(N, n_s, phi.shape[0], cplx, work)
    _all_on_device(xi=xi, phi=phi, vphi=vphi, work=work)
    st = load_library().ace_apply(N, n_s, 1 if cplx else 0, float(dV), ctypes.c_void_p(px), ldx,
                                  ctypes.c_void_p(pf), ldf, phi.shape[0], ctypes.c_void_p(pv), ldv,
                                  ctypes.c_void_p(work.data_ptr()), work.numel() * work.element_size(),
                                  _stream(stream))
    _check(st, "ace_apply")
    return vphi


def kx_batched_schedule():
    """Shape of the last captured exx_apply_batched schedule:
    (rounds, batches, launches of the three passes, most batches in one launch)."""
    out = (ctypes.c_int * 4)()
    _check(load_library().kx_batched_schedule(out), "kx_batched_schedule")
    return tuple(out)


def kx_graph_cache_info():
    """(task lists cached now, cache capacity, captures so far) of exx_apply_batched."""
    out = (ctypes.c_int64 * 3)()
    _check(load_library().kx_graph_cache_info(out), "kx_graph_cache_info")
    return tuple(out)


TRACE_KINDS = 23


def kx_trace_enable(on=True):
    _check(load_library().kx_trace_enable(1 if on else 0), "kx_trace_enable")


def kx_trace_read():
    """{kind name: (total ms, launches)} for every kind launched since enabling."""
    lib = load_library()
    ms = (ctypes.c_double * TRACE_KINDS)()
    cnt = (ctypes.c_int64 * TRACE_KINDS)()
    _check(lib.kx_trace_read(ms, cnt, TRACE_KINDS), "kx_trace_read")
    return {lib.kx_trace_name(k).decode(): (ms[k], cnt[k]) for k in range(TRACE_KINDS) if cnt[k]}


def kx_host_eig1d(n, h, bc, fd_order=12, kappa=0.0):
    """Host-only: (lam, V) of the 1D operator as the plan computes them, V[k, a]."""
    lam = np.empty(n)
    vr = np.empty((n, n))
    vi = np.empty((n, n))
    st = load_library().kx_host_eig1d(n, h, BC[bc] if isinstance(bc, str) else bc, fd_order,
                                      kappa, _dptr(lam), _dptr(vr), _dptr(vi))
    _check(st, "kx_host_eig1d")
    return lam, (vr + 1j * vi if kappa != 0.0 else vr)


def kx_host_fd_weights(fd_order):
    c = np.empty(fd_order // 2 + 1)
    _check(load_library().kx_host_fd_weights(fd_order, _dptr(c)), "kx_host_fd_weights")
    return c
