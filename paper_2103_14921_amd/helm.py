"""Thin Python binding of the C ABI in include/helm.h (ctypes; argument marshalling only).

Every arithmetic step runs in the HIP library ``libhelm.so`` built in-tree by
``paper_2103_14921_amd.build``.  There is no fallback: importing this module
without the built library raises.  Fields may be NumPy arrays (host memory) or
torch tensors on the GPU (device memory); outputs come back as the same kind.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhelm.so")

HELM_OK, HELM_NOT_CONVERGED, HELM_PENDING = 0, 1, 2
HELM_EINVAL, HELM_ENOMEM, HELM_EDEVICE, HELM_EBREAKDOWN = -1, -2, -3, -4
HELM_FP64, HELM_MIXED, HELM_SINGLE_LOCAL, HELM_APPROX_LOCAL = 0, 1, 2, 3
HELM_VEL_COMPLEX128, HELM_VEL_REAL64 = 0, 1
PRECISIONS = {"fp64": HELM_FP64, "mixed": HELM_MIXED, "single_local": HELM_SINGLE_LOCAL,
              "approx_local": HELM_APPROX_LOCAL}


def _precision(name):
    """Library code of a precision name: "fp64" (everything complex FP64), "mixed"
    (fine local solves complex FP32), "single_local" (local solves of both
    levels complex FP32) or "approx_local" (fine local solves approximate: plane
    inverses in complex FP16 on FP16 matrix cores); Krylov, residuals and the
    coarse GMRES stay FP64."""
    try:
        return PRECISIONS[name]
    except KeyError:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}, not {name!r}") from None
HELM_X0 = 1
HELM_BLOCK = 2
HELM_TILE_MARCH = 0x100

EXPORTS = [
    "helm_fit_weights", "helm_setup", "helm_solve", "helm_footprint", "helm_workspace_bytes", "helm_resident_bytes",
    "helm_last_timings", "helm_destroy", "helm_last_error", "helm_set_stream", "helm_apply_A",
    "helm_apply_M", "helm_apply_oras", "helm_restrict", "helm_prolong", "helm_apply_E", "helm_apply_Q",
    "helm_num_subdomains", "helm_subdomain_box", "helm_set_sweep_timing", "helm_sweep_stats", "helm_stencil_stats",
    "helm_sweep_config",
    "helm_local_solve", "helm_release_workspace", "helm_trim_cache", "helm_set_graphs", "helm_graph_stats",
    "helm_set_sweep_policy",
    "helm_set_row_tiling",
    "helm_set_lu_panel",
    "helm_solve_async", "helm_request_query", "helm_request_wait", "helm_solve_bound",
    "helm_device_headroom", "helm_apply_oras_noalloc", "helm_fit_weight_table",
]


class HelmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"helm status {code}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double)]


class PmlT(C.Structure):
    _fields_ = [("npml_x", C.c_int32), ("npml_y", C.c_int32), ("npml_zbot", C.c_int32),
                ("npml_ztop", C.c_int32), ("R", C.c_double)]


class WeightsT(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("w1", "w2", "w3", "wm1", "wm2", "wm3", "wm4")]


class DecompT(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("px", "py", "pz", "overlap", "levels", "coarse_iters",
                                         "precision", "restart", "robin", "nrhs_chunk", "adaptive")]


def _init_torch_runtime_first():
    """PyTorch ships its own HIP runtime; it must initialise before this library's
    runtime in a process that uses both (for device buffers and streams)."""
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except Exception:
        pass


def _load():
    _init_torch_runtime_first()
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2103_14921_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i32 = C.c_int32
    sig = {
        "helm_fit_weights": ([C.c_double, C.c_double, i32, i32, C.POINTER(WeightsT)], C.c_int),
        "helm_setup": ([C.POINTER(Grid), P, i32, C.c_double, C.POINTER(PmlT), C.POINTER(WeightsT),
                        C.POINTER(DecompT), C.POINTER(P)], C.c_int),
        "helm_solve": ([P, i32, P, P, C.c_double, i32, C.c_uint32, P, P, P], C.c_int),
        "helm_footprint": ([C.POINTER(Grid), C.POINTER(DecompT), i32], C.c_size_t),
        "helm_workspace_bytes": ([C.POINTER(Grid), C.POINTER(DecompT), i32], C.c_size_t),
        "helm_resident_bytes": ([P], C.c_size_t),
        "helm_last_timings": ([P, C.POINTER(C.c_double)], C.c_int),
        "helm_destroy": ([P], None),
        "helm_last_error": ([P], C.c_char_p),
        "helm_set_stream": ([P, P], C.c_int),
        "helm_apply_A": ([P, i32, P, P], C.c_int),
        "helm_apply_M": ([P, i32, P, P], C.c_int),
        "helm_apply_oras": ([P, i32, i32, P, P], C.c_int),
        "helm_restrict": ([P, i32, P, P], C.c_int),
        "helm_prolong": ([P, i32, P, P], C.c_int),
        "helm_apply_E": ([P, i32, P, P], C.c_int),
        "helm_apply_Q": ([P, i32, P, P], C.c_int),
        "helm_num_subdomains": ([P, i32], i32),
        "helm_subdomain_box": ([P, i32, i32, C.POINTER(i32)], C.c_int),
        "helm_set_sweep_timing": ([P, i32], C.c_int),
        "helm_sweep_stats": ([P, i32, C.POINTER(C.c_double)], C.c_int),
        "helm_sweep_config": ([P, i32, i32, C.POINTER(C.c_int32)], C.c_int),
        "helm_stencil_stats": ([P, i32, C.POINTER(C.c_double)], C.c_int),
        "helm_local_solve": ([P, i32, i32, i32, P, P], C.c_int),
        "helm_release_workspace": ([P], C.c_int),
        "helm_trim_cache": ([], C.c_size_t),
        "helm_set_graphs": ([P, i32], C.c_int),
        "helm_graph_stats": ([P, C.POINTER(C.c_double)], C.c_int),
        "helm_set_sweep_policy": ([i32], C.c_int),
        "helm_set_row_tiling": ([i32], C.c_int),
        "helm_set_lu_panel": ([i32], C.c_int),
        "helm_solve_async": ([P, i32, P, P, C.c_double, i32, C.c_uint32, P, P, P, P, C.POINTER(C.c_void_p)],
                             C.c_int),
        "helm_request_query": ([P], C.c_int),
        "helm_request_wait": ([P], C.c_int),
        "helm_solve_bound": ([P, C.POINTER(C.c_double)], C.c_int),
        "helm_device_headroom": ([], C.c_size_t),
        "helm_apply_oras_noalloc": ([P, i32, i32, P, P], C.c_int),
        "helm_fit_weight_table": ([C.c_double, C.c_double, i32, i32, C.POINTER(WeightsT)], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def last_error(handle=None):
    """Message of the last failure on the calling thread, or of the last failed call on a handle."""
    return lib.helm_last_error(handle).decode()


def _check(code, ok=(HELM_OK,), handle=None):
    if code not in ok:
        raise HelmError(code, last_error(handle))
    return code


def fit_weights(gmin=4.0, gmax=10.0, ng=7, nang=15):
    w = WeightsT()
    _check(lib.helm_fit_weights(gmin, gmax, ng, nang, C.byref(w)))
    return {k: getattr(w, k) for k, _ in WeightsT._fields_}


def fit_weight_table(g0=3.0, dg=0.25, n=29, nang=15):
    """The adaptive coefficients' weight table (helm_fit_weight_table): a list of n weight dicts."""
    out = (WeightsT * n)()
    _check(lib.helm_fit_weight_table(g0, dg, n, nang, out))
    return [{k: getattr(w, k) for k, _ in WeightsT._fields_} for w in out]


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a, n_expect, real=False):
    """Pointer of a contiguous complex128 (or, with real=True, float64) buffer of n_expect elements."""
    if _is_torch(a):
        import torch
        want = torch.float64 if real else torch.complex128
        if a.dtype != want or not a.is_contiguous() or a.numel() != n_expect:
            raise ValueError("expected a contiguous %s tensor of %d elements" % (want, n_expect))
        return C.c_void_p(a.data_ptr())
    want = np.float64 if real else np.complex128
    if not isinstance(a, np.ndarray) or a.dtype != want or not a.flags.c_contiguous or a.size != n_expect:
        raise ValueError("expected a C-contiguous %s array of %d elements" % (np.dtype(want), n_expect))
    return C.c_void_p(a.ctypes.data)


def trim_cache():
    """Return the library's cached device blocks to the runtime; bytes freed."""
    return lib.helm_trim_cache()


def device_headroom():
    """Device bytes the library leaves to the runtime (helm_device_headroom); other
    allocations beside the library keep the same margin."""
    return lib.helm_device_headroom()


def torch_alloc(fn):
    """Run a PyTorch allocation; on out-of-memory, trim the library's device cache and retry once."""
    import torch
    try:
        return fn()
    except torch.OutOfMemoryError:
        trim_cache()
        torch.cuda.empty_cache()
        return fn()


def _empty_like_kind(a, shape):
    if _is_torch(a):
        import torch
        return torch_alloc(lambda: torch.empty(shape, dtype=torch.complex128, device=a.device))
    return np.empty(shape, dtype=np.complex128)


class Request:
    """An asynchronous solve in flight (Solver.solve_async).  It keeps B, X and the
    result arrays alive until wait() returns."""

    def __init__(self, solver, B, X, nrhs):
        self.solver, self.B, self.X = solver, B, X
        self.its = np.zeros(nrhs, np.int32)
        self.est = np.zeros(nrhs)
        self.tru = np.zeros(nrhs)
        self._h = None
        self._result = None

    def done(self):
        if self._result is not None:
            return True
        return lib.helm_request_query(self._h) != HELM_PENDING

    def wait(self):
        if self._result is None:
            h, self._h = self._h, None
            code = lib.helm_request_wait(h)
            self._result = (code, last_error())
            self.B = None
        code, msg = self._result
        if code not in (HELM_OK, HELM_NOT_CONVERGED):
            raise HelmError(code, msg)
        timings = self.solver.timings() if getattr(self.solver, "_h", None) else None
        return self.X, dict(status=code, iters=self.its, relres_est=self.est, relres_true=self.tru, timings=timings)

    def __del__(self):
        # an abandoned request still owns a library thread: join it
        try:
            if self._result is None and self._h is not None:
                lib.helm_request_wait(self._h)
        except Exception:
            pass


SWEEP_POLICIES = {"auto": 0, "item": 1, "pipelined": 2, "two_per_cu": 3, "pipelined16": 4, "paired": 5,
                  "paired_lds": 6, "lds_solutions": 6}


def set_sweep_policy(policy):
    """Process-wide choice of local-solve sweep: "auto" (tuned), "item", "pipelined" or "two_per_cu"."""
    _check(lib.helm_set_sweep_policy(SWEEP_POLICIES[policy]))


def set_row_tiling(nodes_per_thread):
    """Process-wide schedule of the 27-point products: 0 (autotuned), 2, 4 or 8 (row tiles with that many
    nodes per thread), HELM_TILE_MARCH | 2 or | 3 (plane-marching, batches of 16 k right-hand sides)."""
    _check(lib.helm_set_row_tiling(int(nodes_per_thread)))


def set_lu_panel(columns):
    """Process-wide panel width of the local Gauss-Jordan inversions: 0 (autotuned), 4, 8 or 16."""
    _check(lib.helm_set_lu_panel(int(columns)))


def footprint(shape, parts, overlap=2, levels=1, coarse_iters=10, precision="fp64", restart=30, nrhs_chunk=1):
    g = Grid(*shape, 1.0)
    d = DecompT(*parts, overlap, levels, coarse_iters, _precision(precision),
                restart, 1, nrhs_chunk)
    return lib.helm_footprint(C.byref(g), C.byref(d), nrhs_chunk)


def workspace_bytes(shape, parts, overlap=2, levels=1, coarse_iters=10, precision="fp64", restart=30, nrhs_chunk=1):
    """Device bytes of the Krylov workspace of nrhs_chunk right-hand sides (helm_workspace_bytes)."""
    g = Grid(*shape, 1.0)
    d = DecompT(*parts, overlap, levels, coarse_iters, _precision(precision),
                restart, 1, nrhs_chunk)
    return lib.helm_workspace_bytes(C.byref(g), C.byref(d), nrhs_chunk)


class Solver:
    """A set-up problem (helm_setup); owns the library handle."""

    def __init__(self, shape, h, velocity, freq, pml=(0, 0, 0, 0), weights=None, parts=(1, 1, 1), overlap=2,
                 levels=1, coarse_iters=10, precision="fp64", restart=30, robin=True, nrhs_chunk=0, R=1e-3,
                 adaptive=False):
        self.shape = tuple(int(v) for v in shape)
        nx, ny, nz = self.shape
        self.n = nx * ny * nz
        self.levels = levels
        self.cshape = tuple((v + 1) // 2 for v in self.shape)
        self.nc = int(np.prod(self.cshape))
        g = Grid(nx, ny, nz, float(h))
        p = PmlT(*[int(v) for v in pml], float(R))
        d = DecompT(*[int(v) for v in parts], int(overlap), int(levels), int(coarse_iters),
                    _precision(precision), int(restart), 1 if robin else 0,
                    int(nrhs_chunk), 1 if adaptive else 0)
        w = None
        if weights is not None:
            if not isinstance(weights, dict):
                weights = {k: float(getattr(weights, k)) for k, _ in WeightsT._fields_}
            w = WeightsT(**{k: float(weights[k]) for k, _ in WeightsT._fields_})
        # a real velocity array (float64) is passed as HELM_VEL_REAL64, anything else as complex128
        if _is_torch(velocity):
            import torch
            real = velocity.dtype == torch.float64
            vel = velocity
        else:
            real = np.asarray(velocity).dtype == np.float64
            vel = np.ascontiguousarray(velocity, dtype=np.float64 if real else np.complex128)
        handle = C.c_void_p()
        _check(lib.helm_setup(C.byref(g), _ptr(vel, self.n, real=real),
                              HELM_VEL_REAL64 if real else HELM_VEL_COMPLEX128, float(freq), C.byref(p),
                              C.byref(w) if w is not None else None, C.byref(d), C.byref(handle)))
        self._h = handle

    def close(self):
        if getattr(self, "_h", None):
            lib.helm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, B, tol=1e-8, maxit=500, X0=None, block=False):
        """Solve A X = B, B of shape [nrhs][nz][ny][nx] (or [nrhs][n]); returns (X, info).

        block=True: block FGMRES, one Krylov space per batch of at most 32 right-hand sides."""
        nrhs = B.shape[0]
        X = _empty_like_kind(B, tuple(B.shape)) if X0 is None else X0
        flags = (HELM_X0 if X0 is not None else 0) | (HELM_BLOCK if block else 0)
        its = np.zeros(nrhs, np.int32)
        est = np.zeros(nrhs)
        tru = np.zeros(nrhs)
        code = lib.helm_solve(self._h, nrhs, _ptr(B, nrhs * self.n), _ptr(X, nrhs * self.n), float(tol), int(maxit),
                              flags, its.ctypes.data_as(C.c_void_p), est.ctypes.data_as(C.c_void_p),
                              tru.ctypes.data_as(C.c_void_p))
        _check(code, ok=(HELM_OK, HELM_NOT_CONVERGED), handle=self._h)
        return X, dict(status=code, iters=its, relres_est=est, relres_true=tru, timings=self.timings())

    def solve_async(self, B, tol=1e-8, maxit=500, X0=None, stream=None):
        """Start the solve of A X = B on a library thread; returns a Request (wait() -> (X, info)).

        stream: a torch.cuda.Stream (or raw hipStream_t) that receives the solve's device work, ordered
        after what was already enqueued on it; None = the handle's own stream."""
        nrhs = B.shape[0]
        X = _empty_like_kind(B, tuple(B.shape)) if X0 is None else X0
        req = Request(self, B, X, nrhs)
        h = C.c_void_p()
        sp = None if stream is None else C.c_void_p(getattr(stream, "cuda_stream", stream))
        _check(lib.helm_solve_async(self._h, nrhs, _ptr(B, nrhs * self.n), _ptr(X, nrhs * self.n), float(tol),
                                    int(maxit), HELM_X0 if X0 is not None else 0,
                                    req.its.ctypes.data_as(C.c_void_p), req.est.ctypes.data_as(C.c_void_p),
                                    req.tru.ctypes.data_as(C.c_void_p), sp, C.byref(h)), handle=self._h)
        req._h = h
        return req

    def timings(self):
        out = (C.c_double * 5)()
        _check(lib.helm_last_timings(self._h, out))
        return dict(setup=out[0], solve=out[1], factor=out[2], coarse=out[3], iters_total=out[4])

    def solve_bound(self):
        """Lower bound of the last solve: seconds at the device's peaks, algorithmic bytes and flops."""
        out = (C.c_double * 3)()
        _check(lib.helm_solve_bound(self._h, out))
        return dict(seconds=out[0], bytes=out[1], flops=out[2])

    def set_sweep_timing(self, enable=True):
        _check(lib.helm_set_sweep_timing(self._h, 1 if enable else 0))

    def sweep_stats(self, level=0):
        out = (C.c_double * 4)()
        _check(lib.helm_sweep_stats(self._h, int(level), out))
        return dict(launches=int(out[0]), ms=out[1], flops=out[2], bytes=out[3])

    def sweep_config(self, level=0, nrhs=32):
        """The autotuned local-solve launch of a level at a batch width: group, waves per item, variant
        (numbered as the sweep policy that forces it) and waves per workgroup; zeros if not tuned yet."""
        out = (C.c_int32 * 4)()
        _check(lib.helm_sweep_config(self._h, int(level), int(nrhs), out), handle=self._h)
        return dict(group=out[0], waves_per_item=out[1], variant=out[2], waves=out[3])

    def stencil_stats(self, kind=0):
        """Timed fine 27-point products of the solves: kind 0 y = A x, 1 y = b - A x."""
        out = (C.c_double * 4)()
        _check(lib.helm_stencil_stats(self._h, int(kind), out))
        return dict(launches=int(out[0]), ms=out[1], flops=out[2], bytes=out[3])

    def set_graphs(self, enable=True):
        """Capture outer iterations as HIP graphs (default on) or launch directly."""
        _check(lib.helm_set_graphs(self._h, 1 if enable else 0))

    def graph_stats(self):
        out = (C.c_double * 2)()
        _check(lib.helm_graph_stats(self._h, out))
        return dict(captures=int(out[0]), replays=int(out[1]))

    def release_workspace(self):
        _check(lib.helm_release_workspace(self._h))

    def resident_bytes(self):
        return lib.helm_resident_bytes(self._h)

    def _map(self, fn, X, n_in, n_out, *lead):
        nrhs = X.shape[0]
        Y = _empty_like_kind(X, (nrhs, n_out))
        _check(fn(self._h, *lead, nrhs, _ptr(X, nrhs * n_in), _ptr(Y, nrhs * n_out)), handle=self._h)
        return Y

    def last_error(self):
        """Message of the last failed call on this handle (helm_last_error(h))."""
        return last_error(self._h)

    def apply_A(self, X):
        return self._map(lib.helm_apply_A, X, self.n, self.n)

    def apply_M(self, R):
        return self._map(lib.helm_apply_M, R, self.n, self.n)

    def apply_oras(self, R, level=0):
        n = self.n if level == 0 else self.nc
        return self._map(lib.helm_apply_oras, R, n, n, int(level))

    def apply_oras_noalloc(self, R, Z, level=0):
        """Z = M1^{-1} R without allocating (helm_apply_oras_noalloc): R and Z are device tensors
        [nrhs][n]; the work is enqueued on the handle's stream (the call does not wait for it)."""
        n = self.n if level == 0 else self.nc
        nrhs = R.shape[0]
        _check(lib.helm_apply_oras_noalloc(self._h, int(level), nrhs, _ptr(R, nrhs * n), _ptr(Z, nrhs * n)),
               handle=self._h)
        return Z

    def restrict(self, R):
        return self._map(lib.helm_restrict, R, self.n, self.nc)

    def prolong(self, Cc):
        return self._map(lib.helm_prolong, Cc, self.nc, self.n)

    def apply_E(self, X):
        return self._map(lib.helm_apply_E, X, self.nc, self.nc)

    def apply_Q(self, R):
        return self._map(lib.helm_apply_Q, R, self.n, self.n)

    def local_solve(self, R, s, level=0):
        """A_i^{-1} R for subdomain s (R: [nrhs][ez*ey*ex] in the box's natural order)."""
        nrhs = R.shape[0]
        nloc = R.shape[1] if R.ndim == 2 else int(np.prod(R.shape[1:]))
        X = _empty_like_kind(R, (nrhs, nloc))
        _check(lib.helm_local_solve(self._h, int(level), int(s), nrhs, _ptr(R, nrhs * nloc), _ptr(X, nrhs * nloc)))
        return X

    def num_subdomains(self, level=0):
        return lib.helm_num_subdomains(self._h, int(level))

    def subdomain_box(self, s, level=0):
        box = (C.c_int32 * 12)()
        _check(lib.helm_subdomain_box(self._h, int(level), int(s), box))
        b = list(box)
        return dict(elo=tuple(b[0:3]), ehi=tuple(b[3:6]), lo=tuple(b[6:9]), hi=tuple(b[9:12]))
