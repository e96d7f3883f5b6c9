"""Python binding of librbfgs.so (argument marshalling only).

Every computation runs in the HIP library; this module passes pointers, sizes and
flags through ctypes.  The functions mirror the C ABI of include/rbfgs.h
(rbfgs_create, rbfgs_step, rbfgs_invert, rbfgs_residual, ...); `Solver` wraps a
context.  Device buffers are torch tensors on the current HIP device and stream.

The library must be built (python -m paper_1602_01768_amd.build); importing this
module raises if it is missing -- there is no fallback path.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbfgs.so")

OK, E_INVALID_ARG, E_OOM, E_NOT_SPD, E_NONFINITE, E_NOT_CONVERGED, E_DEVICE, E_CANCELLED = range(8)
STATUS_NAMES = {0: "OK", 1: "E_INVALID_ARG", 2: "E_OOM", 3: "E_NOT_SPD", 4: "E_NONFINITE",
                5: "E_NOT_CONVERGED", 6: "E_DEVICE", 7: "E_CANCELLED"}
SKETCH = {"gauss": 0, "coord": 1, "cols": 1, "partition": 2, "importance": 3}
VARIANT = {"fixed": 0, "adaptive": 1, "ada": 1, "psb": 2, "aip": 3, "kaczmarz": 4, "newton_schulz": 5,
           "mr": 6}
PRECISION = {"fp64": 0, "mixed": 1}
F32, F64 = 0, 1


class RbfgsError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")


class rbfgs_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("q", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("sketch", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("check_every", ctypes.c_int32)]


class rbfgs_job_result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("iters", ctypes.c_int64),
                ("resid", ctypes.c_double), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class rbfgs_server_info(ctypes.Structure):
    _fields_ = [("now", ctypes.c_double), ("queued", ctypes.c_int64), ("running", ctypes.c_int32),
                ("outstanding", ctypes.c_int64), ("active_bytes", ctypes.c_int64), ("peak_bytes", ctypes.c_int64),
                ("peak_running", ctypes.c_int32)]


EXPORTS = {
    "rbfgs_create": (ctypes.c_int, [ctypes.POINTER(rbfgs_params), ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_void_p)]),
    "rbfgs_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "rbfgs_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "rbfgs_invert": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "rbfgs_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "rbfgs_estimate": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "rbfgs_get_x": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_int32]),
    "rbfgs_get_l": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_int32]),
    "rbfgs_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_int64]),
    "rbfgs_get_iter": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "rbfgs_destroy": (None, [ctypes.c_void_p]),
    "rbfgs_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "rbfgs_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "rbfgs_profile_report": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int64]),
    "rbfgs_pcg": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int64,
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "rbfgs_ridge_hessian": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                            ctypes.c_void_p]),
    "rbfgs_ridge_hessian_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                                    ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                                    ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p]),
    "rbfgs_sketch_gauss": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "rbfgs_sketch_coord": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "rbfgs_sample_partition": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                              ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rbfgs_get_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rbfgs_footprint": (ctypes.c_int, [ctypes.POINTER(rbfgs_params), ctypes.POINTER(ctypes.c_int64)]),
    "rbfgs_server_create": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "rbfgs_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rbfgs_params), ctypes.c_void_p,
                                           ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                           ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                           ctypes.c_int32, ctypes.c_uint64]),
    "rbfgs_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rbfgs_job_result), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
    "rbfgs_server_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "rbfgs_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rbfgs_server_info)]),
    "rbfgs_server_destroy": (None, [ctypes.c_void_p]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load librbfgs.so and declare its exports (loading needs no GPU)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1602_01768_amd.build`")
    # torch first: the library then binds the HIP runtime torch has loaded (its own copy of
    # libamdhip64), so that device pointers and streams from torch are valid in the library;
    # loaded the other way round, the process holds two runtimes and every call fails
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check(status, ctx=None):
    if status != OK:
        msg = ""
        if ctx:
            raw = load_library().rbfgs_last_error(ctx)
            msg = raw.decode() if raw else ""
        raise RbfgsError(status, msg)


def _matrix_arg(M):
    """(pointer, dtype code, leading dim, on_device, keepalive) for a 2-D torch tensor or numpy array."""
    try:
        import torch
        is_torch = isinstance(M, torch.Tensor)
    except ImportError:
        is_torch = False
    if is_torch:
        if M.dim() != 2 or M.stride(1) != 1:
            raise ValueError("need a 2-D row-major tensor")
        if M.dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be float32 or float64")
        code = F32 if M.dtype == torch.float32 else F64
        return ctypes.c_void_p(M.data_ptr()), code, M.stride(0), int(M.is_cuda), M
    a = np.ascontiguousarray(M)
    if a.dtype not in (np.float32, np.float64):
        a = a.astype(np.float64)
    code = F32 if a.dtype == np.float32 else F64
    return ctypes.c_void_p(a.ctypes.data), code, a.shape[1], 0, a


# ----------------------------------------------------- same-name C ABI wrappers
def rbfgs_create(A, q, seed, sketch="gauss", variant="fixed", precision="fp64", check_every=16, stream=None):
    lib = load_library()
    ptr, code, ld, on_dev, keep = _matrix_arg(A)
    n = int(A.shape[0])
    p = rbfgs_params(n=n, q=int(q), seed=int(seed), sketch=SKETCH[sketch], variant=VARIANT[variant],
                     precision=PRECISION[precision], check_every=int(check_every))
    out = ctypes.c_void_p()
    st = lib.rbfgs_create(ctypes.byref(p), ptr, code, ld, on_dev, _stream_handle(stream), ctypes.byref(out))
    del keep
    _check(st)
    return out.value


def rbfgs_step(ctx, nsteps=1):
    _check(load_library().rbfgs_step(ctx, int(nsteps)), ctx)


def rbfgs_sync(ctx):
    _check(load_library().rbfgs_sync(ctx), ctx)


def rbfgs_invert(ctx, tol, max_iters):
    it = ctypes.c_int64()
    r = ctypes.c_double()
    st = load_library().rbfgs_invert(ctx, float(tol), int(max_iters), ctypes.byref(it), ctypes.byref(r))
    if st not in (OK, E_NOT_CONVERGED):
        _check(st, ctx)
    return st == OK, it.value, r.value


def rbfgs_residual(ctx):
    r = ctypes.c_double()
    _check(load_library().rbfgs_residual(ctx, ctypes.byref(r)), ctx)
    return r.value


def rbfgs_estimate(ctx):
    r = ctypes.c_double()
    _check(load_library().rbfgs_estimate(ctx, ctypes.byref(r)), ctx)
    return r.value


def _get_matrix(fn, ctx, n, dtype, device):
    import torch
    tdt = torch.float64 if dtype == F64 else torch.float32
    out = torch.empty((n, n), dtype=tdt, device=device)
    _check(fn(ctx, ctypes.c_void_p(out.data_ptr()), dtype, n, int(out.is_cuda)), ctx)
    return out


def rbfgs_get_x(ctx, n, dtype=F64, device="cuda"):
    return _get_matrix(load_library().rbfgs_get_x, ctx, n, dtype, device)


def rbfgs_get_l(ctx, n, dtype=F64, device="cuda"):
    return _get_matrix(load_library().rbfgs_get_l, ctx, n, dtype, device)


def rbfgs_set_state(ctx, M, k):
    ptr, code, ld, on_dev, keep = _matrix_arg(M)
    _check(load_library().rbfgs_set_state(ctx, ptr, code, ld, on_dev, int(k)), ctx)
    del keep


def rbfgs_get_iter(ctx):
    k = ctypes.c_int64()
    _check(load_library().rbfgs_get_iter(ctx, ctypes.byref(k)), ctx)
    return k.value


def rbfgs_destroy(ctx):
    if ctx:
        load_library().rbfgs_destroy(ctx)


def rbfgs_profile(ctx, enable=True):
    """enable: False/0 off, True/1 every phase, 2 the n x n products only."""
    _check(load_library().rbfgs_profile(ctx, int(enable)), ctx)


def rbfgs_profile_report(ctx):
    """{phase: (total_ms, count)} accumulated since profiling was enabled."""
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load_library().rbfgs_profile_report(ctx, buf, len(buf)), ctx)
    return {k: (v[0], v[1]) for k, v in json.loads(buf.value.decode()).items()}


def rbfgs_pcg(ctx, b, precond=True, tol=1e-8, max_iters=10000):
    """Solve A x = b by CG preconditioned with the context's X (or plain CG); b a CUDA
    tensor or numpy vector.  Returns (x as an FP64 CUDA tensor, converged, iters, relres)."""
    import torch
    if isinstance(b, torch.Tensor):
        bt = b.to(device="cuda", dtype=torch.float64).contiguous()
    else:
        import numpy as np
        bt = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64)).cuda()
    x = torch.empty_like(bt)
    it = ctypes.c_int64(0)
    rel = ctypes.c_double(0.0)
    st = load_library().rbfgs_pcg(ctx, ctypes.c_void_p(bt.data_ptr()), F64, 1, ctypes.c_void_p(x.data_ptr()), F64, 1,
                                  1 if precond else 0, float(tol), int(max_iters), ctypes.byref(it), ctypes.byref(rel))
    if st not in (OK, E_NOT_CONVERGED):
        _check(st, ctx)
    return x, st == OK, it.value, rel.value


def rbfgs_ridge_hessian(B, scale, lam, dtype=F32, stream=None):
    """scale * B^T B + lam I (eq. ridgeMatrix) for an m x n B (numpy or torch, FP32/FP64,
    host or device); returns the n x n result as a CUDA tensor of `dtype`."""
    import torch
    on_dev = isinstance(B, torch.Tensor) and B.is_cuda
    if isinstance(B, torch.Tensor):
        Bt = B.contiguous()
        b_dt = F32 if Bt.dtype == torch.float32 else F64
        if Bt.dtype not in (torch.float32, torch.float64):
            raise TypeError("B must be float32 or float64")
        ptr = Bt.data_ptr()
        keep = Bt
    else:
        import numpy as np
        keep = np.ascontiguousarray(B)
        if keep.dtype not in (np.float32, np.float64):
            keep = keep.astype(np.float64)
        b_dt = F32 if keep.dtype == np.float32 else F64
        ptr = keep.ctypes.data
    m, n = keep.shape
    out = torch.empty((n, n), dtype=torch.float32 if dtype == F32 else torch.float64, device="cuda")
    _check(load_library().rbfgs_ridge_hessian(ctypes.c_void_p(ptr), b_dt, m, n, n, 1 if on_dev else 0, float(scale),
                                              float(lam), ctypes.c_void_p(out.data_ptr()), dtype, n, 1,
                                              _stream_handle(stream)))
    del keep
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20  # RBFGS_NOALLOC_SCRATCH_BYTES


def rbfgs_ridge_hessian_noalloc(B, scale, lam, out, stream=None):
    """scale * B^T B + lam I for a CUDA tensor B (m x n, FP32/FP64, contiguous) into the
    caller's CUDA tensor `out` (n x n, FP32/FP64, contiguous), through the library's
    allocation-free entry point (work buffers in its fixed device array; asynchronous)."""
    import torch
    if not (isinstance(B, torch.Tensor) and B.is_cuda and B.is_contiguous() and B.dim() == 2):
        raise TypeError("B must be a contiguous 2-D CUDA tensor")
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.is_contiguous() and out.dim() == 2):
        raise TypeError("out must be a contiguous 2-D CUDA tensor")
    types = {torch.float32: F32, torch.float64: F64}
    if B.dtype not in types or out.dtype not in types:
        raise TypeError("B and out must be float32 or float64")
    m, n = B.shape
    if tuple(out.shape) != (n, n):
        raise ValueError(f"out must be {n} x {n}")
    _check(load_library().rbfgs_ridge_hessian_noalloc(ctypes.c_void_p(B.data_ptr()), types[B.dtype], m, n, n,
                                                      float(scale), float(lam), ctypes.c_void_p(out.data_ptr()),
                                                      types[out.dtype], n, _stream_handle(stream)))
    return out


def rbfgs_sketch_gauss(seed, k, n, q, dtype=F64, stream=None):
    import torch
    out = torch.zeros((q, n), dtype=torch.float64 if dtype == F64 else torch.float32, device="cuda")
    _check(load_library().rbfgs_sketch_gauss(int(seed), int(k), int(n), int(q), ctypes.c_void_p(out.data_ptr()),
                                             dtype, _stream_handle(stream)))
    return out.T  # n x q view of the column-major buffer


def rbfgs_sketch_coord(seed, k, n, q, stream=None):
    import torch
    out = torch.zeros(q, dtype=torch.int32, device="cuda")
    _check(load_library().rbfgs_sketch_coord(int(seed), int(k), int(n), int(q), ctypes.c_void_p(out.data_ptr()),
                                             _stream_handle(stream)))
    return out


def rbfgs_sample_partition(t, q, seed, k, stream=None):
    """Partition draw of iteration k from the FP64 weights t (a CUDA tensor of n):
    returns (the q indices of the drawn block as an int32 CUDA tensor, 1/p_i)."""
    import torch
    tt = t.to(device="cuda", dtype=torch.float64).contiguous()
    idx = torch.zeros(q, dtype=torch.int32, device="cuda")
    ht = torch.zeros(1, dtype=torch.float64, device="cuda")
    _check(load_library().rbfgs_sample_partition(ctypes.c_void_p(tt.data_ptr()), int(tt.numel()), int(q), int(seed),
                                                 int(k), ctypes.c_void_p(idx.data_ptr()),
                                                 ctypes.c_void_p(ht.data_ptr()), _stream_handle(stream)))
    return idx, ht


def rbfgs_get_weights(ctx, n):
    """The n per-coordinate partition weights of the context (numpy FP64)."""
    out = np.empty(int(n), dtype=np.float64)
    _check(load_library().rbfgs_get_weights(ctx, out.ctypes.data_as(ctypes.c_void_p)), ctx)
    return out


def _params(n, q, seed, sketch, variant, precision, check_every):
    return rbfgs_params(n=int(n), q=int(q), seed=int(seed), sketch=SKETCH[sketch], variant=VARIANT[variant],
                        precision=PRECISION[precision], check_every=int(check_every))


def rbfgs_footprint(n, q, sketch="gauss", variant="fixed", precision="fp64"):
    """Device bytes of a context for these parameters (no allocation, no GPU needed)."""
    p = _params(n, q, 1, sketch, variant, precision, 16)
    out = ctypes.c_int64()
    _check(load_library().rbfgs_footprint(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def rbfgs_server_create(budget_bytes, workers):
    out = ctypes.c_void_p()
    _check(load_library().rbfgs_server_create(int(budget_bytes), int(workers), ctypes.byref(out)))
    return out.value


def rbfgs_server_submit(server, A, q, seed, tol, max_iters, tag, sketch="gauss", variant="adaptive",
                        precision="mixed", check_every=16, x_out=None):
    """Queue one inversion.  Returns the objects whose memory the library reads (A, or the
    contiguous copy made of it) and writes (x_out): the caller keeps them alive until the
    job's result is polled.  A numpy x_out must be a C-contiguous float32/float64 array (a
    copy would receive the result instead of it)."""
    ptr, code, ld, on_dev, keep = _matrix_arg(A)
    p = _params(A.shape[0], q, seed, sketch, variant, precision, check_every)
    xp, xcode, xld, xdev, xkeep = None, F64, 0, 0, None
    if x_out is not None:
        if isinstance(x_out, np.ndarray) and not (x_out.flags.c_contiguous and x_out.dtype in (np.float32, np.float64)):
            raise ValueError("x_out must be a C-contiguous float32/float64 array")
        xp, xcode, xld, xdev, xkeep = _matrix_arg(x_out)
    _check(load_library().rbfgs_server_submit(server, ctypes.byref(p), ptr, code, ld, on_dev, float(tol),
                                              int(max_iters), xp, xcode, xld, xdev, int(tag)))
    return keep, xkeep


def rbfgs_server_poll(server, max_results=256, wait_ms=0):
    buf = (rbfgs_job_result * max(1, int(max_results)))()
    n = ctypes.c_int32()
    _check(load_library().rbfgs_server_poll(server, buf, int(max_results), ctypes.byref(n), int(wait_ms)))
    return [dict(tag=r.tag, status=r.status, iters=r.iters, resid=r.resid, t_submit=r.t_submit,
                 t_admit=r.t_admit, t_done=r.t_done) for r in buf[:n.value]]


def rbfgs_server_cancel(server, tag):
    _check(load_library().rbfgs_server_cancel(server, int(tag)))


def rbfgs_server_stats(server):
    info = rbfgs_server_info()
    _check(load_library().rbfgs_server_stats(server, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in info._fields_}


def rbfgs_server_destroy(server):
    if server:
        load_library().rbfgs_server_destroy(server)


class Server:
    """Many inversions sharing the GPU under a device-memory budget (see rbfgs.h)."""

    def __init__(self, budget_bytes, workers=8):
        self.handle = rbfgs_server_create(budget_bytes, workers)
        self._keep = {}  # tag -> what the library reads and writes, one entry per job with that tag
        self._done = {}  # tag -> results polled so far

    def submit(self, A, q, seed, tol, max_iters, tag, x_out=None, **kw):
        # keep what the library reads and writes (possibly a converted copy of A) until polled
        keep = rbfgs_server_submit(self.handle, A, q, seed, tol, max_iters, tag, x_out=x_out, **kw)
        self._keep.setdefault(int(tag), []).append(keep)

    def poll(self, max_results=256, wait_ms=0):
        res = rbfgs_server_poll(self.handle, max_results, wait_ms)
        for r in res:
            # jobs sharing a tag may finish in any order: their buffers are all kept until the
            # last of them has been polled
            t = int(r["tag"])
            if t in self._keep:
                self._done[t] = self._done.get(t, 0) + 1
                if self._done[t] == len(self._keep[t]):
                    del self._keep[t], self._done[t]
        return res

    def cancel(self, tag):
        """Cancel the earliest outstanding job with this tag (rbfgs_server_cancel)."""
        rbfgs_server_cancel(self.handle, tag)

    def stats(self):
        return rbfgs_server_stats(self.handle)

    def close(self):
        if self.handle:
            rbfgs_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()
            self._done.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Solver:
    """One inversion context (library-owned device state for A and X or L)."""

    def __init__(self, A, q, seed, sketch="gauss", variant="fixed", precision="fp64", check_every=16,
                 stream=None):
        self.n = int(A.shape[0])
        self.q, self.seed = int(q), int(seed)
        self.sketch, self.variant, self.precision = sketch, variant, precision
        self.ctx = rbfgs_create(A, q, seed, sketch, variant, precision, check_every, stream)

    def step(self, nsteps=1):
        rbfgs_step(self.ctx, nsteps)
        return self

    def sync(self):
        rbfgs_sync(self.ctx)

    def invert(self, tol=1e-3, max_iters=20000):
        """(converged, iterations, ||I - AX||_F / sqrt(n))"""
        return rbfgs_invert(self.ctx, tol, max_iters)

    def pcg(self, b, precond=True, tol=1e-8, max_iters=10000):
        """Solve A x = b by CG preconditioned with the current X: (x, converged, iters, relres)."""
        return rbfgs_pcg(self.ctx, b, precond, tol, max_iters)

    def residual(self):
        return rbfgs_residual(self.ctx)

    def weights(self):
        """Partition weights: the diagonal of A (fixed) or of L_k^T A L_k (AdaRBFGS); with
        importance sampling each block's weight of the last draw on its first coordinate."""
        return rbfgs_get_weights(self.ctx, self.n)

    def estimate(self):
        return rbfgs_estimate(self.ctx)

    def x(self, dtype=F64, device="cuda"):
        return rbfgs_get_x(self.ctx, self.n, dtype, device)

    def factor(self, dtype=F64, device="cuda"):
        return rbfgs_get_l(self.ctx, self.n, dtype, device)

    def set_state(self, M, k):
        rbfgs_set_state(self.ctx, M, k)

    def profile(self, enable=True):
        rbfgs_profile(self.ctx, enable)

    def profile_report(self):
        return rbfgs_profile_report(self.ctx)

    @property
    def iteration(self):
        return rbfgs_get_iter(self.ctx)

    def close(self):
        if self.ctx:
            rbfgs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def relative_residual(fro, n):
    return fro / math.sqrt(n)
