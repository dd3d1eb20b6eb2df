"""Python binding of the gpbo C ABI (``include/gpbo.h``), argument marshalling only.

Every step of fit and scoring runs in the HIP library ``libgpbo.so``; this
module passes torch tensors' device pointers and torch's current stream to it,
and gives the library torch's caching allocator for its own device buffers.
If the library is missing, importing :func:`lib` raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpbo.so")

OK, E_INVALID_ARG, E_NOT_PD, E_NONFINITE, E_OOM, E_HIP, E_UNSUPPORTED = range(7)
KERNEL_SE, KERNEL_MATERN52 = 0, 1
FP64, FP32, BF16 = 0, 1, 2
NSTATS = 8
ESCALATE_KINV = 8.0
PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16}
PATH_AUTO, PATH_FUSED, PATH_LARGE = 0, 1, 2
PATHS = {"auto": PATH_AUTO, "fused": PATH_FUSED, "large": PATH_LARGE}


class GpboError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gpbo status {status}: {msg}")
        self.status = status


class HyperOpts(C.Structure):
    _fields_ = [("starts", C.c_int32), ("steps", C.c_int32), ("lr", C.c_double),
                ("jitter0", C.c_double), ("retries", C.c_int32)]


class Problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("d", C.c_int32), ("X", C.c_void_p), ("y", C.c_void_p),
                ("kernel", C.c_int32), ("lengthscale", C.POINTER(C.c_double)),
                ("signal_var", C.c_double), ("noise_var", C.c_double),
                ("normalize_y", C.c_int32), ("refine_alpha", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


_lib = None

# Every symbol the header declares, with its ctypes signature.
_SIGS = {
    "gpbo_status_string": (C.c_char_p, [C.c_int]),
    "gpbo_last_error": (C.c_char_p, [C.c_void_p]),
    "gpbo_version": (C.c_int32, []),
    "gpbo_ctx_create": (C.c_int, [C.c_int32, C.c_void_p, C.POINTER(Allocator), C.POINTER(C.c_void_p)]),
    "gpbo_ctx_destroy": (C.c_int, [C.c_void_p]),
    "gpbo_ctx_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gpbo_ctx_enable_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "gpbo_ctx_timing": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "gpbo_ctx_set_score_path": (C.c_int, [C.c_void_p, C.c_int]),
    "gpbo_fit": (C.c_int, [C.c_void_p, C.POINTER(Problem), C.POINTER(C.c_void_p),
                           C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "gpbo_fit_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Problem), C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "gpbo_fit_async": (C.c_int, [C.c_void_p, C.POINTER(Problem), C.POINTER(C.c_void_p)]),
    "gpbo_fit_batched_async": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Problem),
                                         C.POINTER(C.c_void_p), C.POINTER(C.c_int32)]),
    "gpbo_model_status_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p),
                                            C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "gpbo_model_status": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double)]),
    "gpbo_model_free": (C.c_int, [C.c_void_p]),
    "gpbo_next_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p),
                                    C.POINTER(C.c_int64), C.POINTER(C.c_void_p), C.c_int, C.c_void_p,
                                    C.c_int32, C.c_void_p]),
    "gpbo_lml_grad_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_int32,
                                        C.c_void_p, C.c_void_p]),
    "gpbo_fit_hyper_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Problem),
                                         C.POINTER(HyperOpts), C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.POINTER(C.c_void_p), C.POINTER(C.c_int32)]),
    "gpbo_ens_select": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int32,
                                  C.c_double, C.c_int64, C.c_void_p, C.c_void_p]),
    "gpbo_mlp_set_occupancy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "gpbo_append_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_void_p,
                                      C.c_int32, C.c_void_p]),
    "gpbo_model_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "gpbo_model_shape": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "gpbo_model_factors": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gpbo_score": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gpbo_score_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_void_p), C.c_int,
                                     C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p]),
    "gpbo_score_prepare_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p),
                                             C.c_int]),
    "gpbo_topk": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "gpbo_topk_noalloc": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "gpbo_topk_set": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "gpbo_score_subset": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                    C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gpbo_score_bound": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p]),
    "gpbo_gather_rows": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p,
                                   C.c_void_p]),
    "gpbo_sensitivity": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "gpbo_plan_searches": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_double,
                                     C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gpbo_mlp_create": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                  C.POINTER(C.c_void_p)]),
    "gpbo_mlp_free": (C.c_int, [C.c_void_p]),
    "gpbo_mlp_nparams": (C.c_int64, [C.c_int32, C.c_int32]),
    "gpbo_mlp_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gpbo_mlp_grads": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p]),
    "gpbo_mlp_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                 C.c_int32, C.c_double, C.c_void_p]),
    "gpbo_mlp_train_model": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double,
                                       C.c_void_p]),
    "gpbo_mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "gpbo_mlp_prescreen": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_double,
                                     C.c_int64, C.c_void_p, C.c_void_p]),
    "gpbo_mlp_prescreen_lcb": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                         C.c_double, C.c_int64, C.c_void_p, C.c_void_p]),
}


def lib():
    """Load ``libgpbo.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"gpbo HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """A gpbo context on one device and torch's current stream (at creation,
    or at the last :meth:`sync_stream`).

    The library's own buffers come from torch's caching allocator through the
    allocator callbacks below, allocated on the context's stream so that the
    allocator reuses them in that stream's order."""

    def __init__(self, device=0, use_torch_allocator=True):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self._children = weakref.WeakSet()  # models and MLPs, freed before the context
        self._held = {}
        self._alloc = None
        self._tstream = torch.cuda.current_stream(self.device)
        if use_torch_allocator:
            def _a(nbytes, stream, user):
                with torch.cuda.stream(self._tstream):
                    t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
                p = t.data_ptr()
                self._held[p] = t
                return p

            def _f(ptr, stream, user):
                self._held.pop(ptr, None)

            self._afn = ALLOC_FN(_a)
            self._ffn = FREE_FN(_f)
            self._alloc = Allocator(self._afn, self._ffn, None)
        h = C.c_void_p()
        st = lib().gpbo_ctx_create(self.device.index or 0, _stream_handle(self.device),
                                   C.byref(self._alloc) if self._alloc else None, C.byref(h))
        if st != OK:
            raise GpboError(st, lib().gpbo_last_error(None).decode())
        self.h = h

    def check(self, st):
        if st != OK:
            raise GpboError(st, lib().gpbo_last_error(self.h).decode())

    def sync_stream(self):
        """Move the context to torch's current stream (the library first waits
        for the work queued on the previous one)."""
        self._tstream = torch.cuda.current_stream(self.device)
        self.check(lib().gpbo_ctx_set_stream(self.h, _stream_handle(self.device)))

    def enable_timing(self, on=True):
        self.check(lib().gpbo_ctx_enable_timing(self.h, 1 if on else 0))

    def set_score_path(self, path="auto"):
        """gpbo_ctx_set_score_path: "auto", "fused" or "large"."""
        self.check(lib().gpbo_ctx_set_score_path(self.h, PATHS[path] if isinstance(path, str) else int(path)))

    def timing(self):
        """(launches, total_ms) of the scoring kernels since the last call."""
        n = C.c_int64()
        ms = C.c_double()
        self.check(lib().gpbo_ctx_timing(self.h, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def close(self):
        if getattr(self, "h", None):
            for ch in list(self._children):
                ch.free()
            lib().gpbo_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """A fitted Gaussian process (owns device copies of X, L, L^-1, alpha)."""

    def __init__(self, ctx: Context, handle, n, d):
        self.ctx = ctx
        self.h = handle
        ctx._children.add(self)
        self.n = n
        self.d = d

    def stats(self):
        s = (C.c_double * NSTATS)()
        self.ctx.check(lib().gpbo_model_stats(self.h, s))
        keys = ("ymean", "ystd", "fbest", "lml", "logdet", "res0", "res1", "kinv")
        return dict(zip(keys, list(s)))

    def factors(self):
        dev = self.ctx.device
        L = torch.empty((self.n, self.n), dtype=torch.float64, device=dev)
        Li = torch.empty_like(L)
        a = torch.empty(self.n, dtype=torch.float64, device=dev)
        self.ctx.check(lib().gpbo_model_factors(self.ctx.h, self.h, _ptr(L), _ptr(Li), _ptr(a)))
        return L, Li, a

    def status(self):
        """gpbo_model_status: raises GpboError (with .bad_pivot on NOT_PD) if
        the fit failed; returns the log marginal likelihood otherwise."""
        bad = C.c_int32(-1)
        lml = C.c_double()
        st = lib().gpbo_model_status(self.ctx.h, self.h, C.byref(bad), C.byref(lml))
        if st != OK:
            err = GpboError(st, lib().gpbo_last_error(self.ctx.h).decode())
            err.bad_pivot = bad.value
            raise err
        return lml.value

    def free(self):
        if self.h:
            lib().gpbo_model_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _problem(X, y, lengthscale, kernel, signal_var, noise_var, normalize_y, refine_alpha):
    assert X.dtype == torch.float64 and y.dtype == torch.float64 and X.is_cuda and y.is_cuda
    assert X.is_contiguous() and y.is_contiguous()
    n, d = X.shape
    ls = (C.c_double * d)(*[float(v) for v in lengthscale])
    p = Problem(n, d, X.data_ptr(), y.data_ptr(), int(kernel), ls, float(signal_var),
                float(noise_var), 1 if normalize_y else 0, 1 if refine_alpha else 0)
    return p, ls


def fit(ctx: Context, X, y, lengthscale, kernel=KERNEL_SE, signal_var=1.0, noise_var=1e-4,
        normalize_y=True, refine_alpha=False):
    """gpbo_fit: returns a :class:`Model`; raises GpboError (with .bad_pivot on NOT_PD)."""
    p, _keep = _problem(X, y, lengthscale, kernel, signal_var, noise_var, normalize_y, refine_alpha)
    h = C.c_void_p()
    lml = C.c_double()
    bad = C.c_int32(-1)
    st = lib().gpbo_fit(ctx.h, C.byref(p), C.byref(h), C.byref(lml), C.byref(bad))
    if st != OK:
        err = GpboError(st, lib().gpbo_last_error(ctx.h).decode())
        err.bad_pivot = bad.value
        raise err
    return Model(ctx, h, X.shape[0], X.shape[1])


def fit_async(ctx: Context, X, y, lengthscale, kernel=KERNEL_SE, signal_var=1.0, noise_var=1e-4,
              normalize_y=True, refine_alpha=False):
    """gpbo_fit_async: queues the fit without synchronising and returns the
    :class:`Model` at once; call ``Model.status()`` (which synchronises)
    before trusting its scores.  X and y must stay unchanged until the stream
    has run the fit."""
    p, _keep = _problem(X, y, lengthscale, kernel, signal_var, noise_var, normalize_y, refine_alpha)
    h = C.c_void_p()
    ctx.check(lib().gpbo_fit_async(ctx.h, C.byref(p), C.byref(h)))
    return Model(ctx, h, X.shape[0], X.shape[1])


class ProblemBatch:
    """Problems marshalled once into the C array gpbo_fit_batched reads, for
    repeated batched fits of the same observations and hyperparameters (a
    benchmark, or a search refitted in place): holds the array and keeps the
    tensors and lengthscale arrays it points to alive."""

    def __init__(self, problems):
        self.B = len(problems)
        self.arr = (Problem * self.B)()
        self._keep = []
        self.shapes = []
        for b, pr in enumerate(problems):
            p, ls = _problem(pr["X"], pr["y"], pr["lengthscale"], pr.get("kernel", KERNEL_SE),
                             pr.get("signal_var", 1.0), pr.get("noise_var", 1e-4),
                             pr.get("normalize_y", True), pr.get("refine_alpha", False))
            self.arr[b] = p
            self._keep.append((pr["X"], pr["y"], ls))
            self.shapes.append(tuple(pr["X"].shape))


def fit_batched(ctx: Context, problems, sync=True):
    """gpbo_fit_batched on a list of dicts with the :func:`fit` arguments (or
    a :class:`ProblemBatch`).  With sync=False, gpbo_fit_batched_async: the
    statuses returned are those of the checks made before queueing
    (``Model.status()`` gives the factorisation's) and the LML list is empty."""
    if not isinstance(problems, ProblemBatch):
        problems = ProblemBatch(problems)
    B = problems.B
    arr = problems.arr
    hs = (C.c_void_p * B)()
    lml = (C.c_double * B)()
    status = (C.c_int32 * B)()
    if sync:
        st = lib().gpbo_fit_batched(ctx.h, B, arr, hs, lml, status)
    else:
        st = lib().gpbo_fit_batched_async(ctx.h, B, arr, hs, status)
        lml = []
    models = [Model(ctx, C.c_void_p(hs[b]), sh[0], sh[1]) if status[b] == OK else None
              for b, sh in enumerate(problems.shapes)]
    return st, models, list(status), list(lml)


def append_batched(ctx: Context, models, x_new, y_new):
    """gpbo_append_batched: add row b of ``x_new`` (device float64, B x ldx,
    ldx >= every model's d) with value ``y_new[b]`` (device float64, B) to
    model b, queued without synchronising (``Model.status()`` reports the
    outcome).  x_new and y_new must stay unchanged until the stream has run
    the update."""
    B = len(models)
    assert x_new.dtype == torch.float64 and y_new.dtype == torch.float64
    assert x_new.is_cuda and y_new.is_cuda and x_new.is_contiguous() and y_new.is_contiguous()
    assert x_new.dim() == 2 and x_new.shape[0] == B and y_new.numel() == B
    hs = (C.c_void_p * B)(*[mo.h.value if isinstance(mo.h, C.c_void_p) else mo.h for mo in models])
    ctx.check(lib().gpbo_append_batched(ctx.h, B, hs, _ptr(x_new), int(x_new.shape[1]), _ptr(y_new)))
    for mo in models:
        mo.n += 1


def next_batched(ctx: Context, models, Xcs, prec, argmax, out):
    """gpbo_next_batched: row argmax[b] of pool Xcs[b] into row b of ``out``
    (device float64, B x ldx), queued on the context's stream."""
    pr = PREC[prec] if isinstance(prec, str) else int(prec)
    B = len(models)
    assert out.dtype == torch.float64 and out.is_contiguous() and out.shape[0] == B
    assert argmax.dtype == torch.int64 and argmax.is_cuda
    hs = (C.c_void_p * B)(*[mo.h.value if isinstance(mo.h, C.c_void_p) else mo.h for mo in models])
    ms = (C.c_int64 * B)(*[x.shape[0] for x in Xcs])
    xs = (C.c_void_p * B)(*[x.data_ptr() for x in Xcs])
    ctx.check(lib().gpbo_next_batched(ctx.h, B, hs, ms, xs, pr, _ptr(argmax), int(out.shape[1]),
                                      _ptr(out)))


def lml_grad_batched(ctx: Context, models):
    """gpbo_lml_grad_batched: (grad (B x ldg device float64, ldg = max d + 2),
    lml (B device float64))."""
    B = len(models)
    ldg = max(mo.d for mo in models) + 2
    grad = torch.empty((B, ldg), dtype=torch.float64, device=ctx.device)
    lml = torch.empty(B, dtype=torch.float64, device=ctx.device)
    hs = (C.c_void_p * B)(*[mo.h.value if isinstance(mo.h, C.c_void_p) else mo.h for mo in models])
    ctx.check(lib().gpbo_lml_grad_batched(ctx.h, B, hs, ldg, _ptr(grad), _ptr(lml)))
    return grad, lml


def fit_hyper_batched(ctx: Context, problems, theta0, lo, hi, steps=100, lr=0.05, jitter0=1e-8,
                      retries=4, want_models=True):
    """gpbo_fit_hyper_batched.  problems: dicts with X, y (device float64) and
    optionally kernel, normalize_y, refine_alpha; theta0: (B, S, ldt) host
    array of starts; lo, hi: (B, ldt).  Returns (status, statuses, theta
    (B, ldt), lml (B,), jitter (B,), models or None)."""
    import numpy as np
    B = len(problems)
    theta0 = np.ascontiguousarray(theta0, dtype=np.float64)
    S, ldt = theta0.shape[1], theta0.shape[2]
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    arr = (Problem * B)()
    for b, pr in enumerate(problems):
        X, y = pr["X"], pr["y"]
        assert X.dtype == torch.float64 and y.dtype == torch.float64 and X.is_contiguous()
        arr[b] = Problem(X.shape[0], X.shape[1], X.data_ptr(), y.data_ptr(),
                         int(pr.get("kernel", KERNEL_SE)), None, 1.0, 0.0,
                         1 if pr.get("normalize_y", True) else 0,
                         1 if pr.get("refine_alpha", False) else 0)
    o = HyperOpts(S, int(steps), float(lr), float(jitter0), int(retries))
    th = np.zeros((B, ldt))
    lml = np.zeros(B)
    jit = np.zeros(B)
    hs = (C.c_void_p * B)()
    status = (C.c_int32 * B)()
    st = lib().gpbo_fit_hyper_batched(ctx.h, B, arr, C.byref(o), theta0.ctypes.data, lo.ctypes.data,
                                      hi.ctypes.data, ldt, th.ctypes.data, lml.ctypes.data,
                                      jit.ctypes.data, hs if want_models else None, status)
    models = None
    if want_models:
        models = [Model(ctx, C.c_void_p(hs[b]), pr["X"].shape[0], pr["X"].shape[1]) if hs[b]
                  else None for b, pr in enumerate(problems)]
    return st, list(status), th, lml, jit, models


SELECT_EI, SELECT_LCB = 0, 1


def ens_select(ctx: Context, outs, rule, arg, k, want_score=False):
    """gpbo_ens_select on member outputs (device float32, E x m): the k best
    indices by ensemble EI (rule SELECT_EI, arg = f_best) or negated LCB
    (SELECT_LCB, arg = kappa); returns (idx, score or None)."""
    assert outs.dtype == torch.float32 and outs.is_contiguous() and outs.dim() == 2
    E, m = outs.shape
    idx = torch.empty(k, dtype=torch.int64, device=ctx.device)
    sc = torch.empty(m, dtype=torch.float32, device=ctx.device) if want_score else None
    ctx.check(lib().gpbo_ens_select(ctx.h, E, m, _ptr(outs), int(rule), float(arg), int(k),
                                    _ptr(idx), _ptr(sc)))
    return idx, sc


def status_batched(ctx: Context, models):
    """gpbo_model_status_batched: (first failing status, statuses, LMLs)."""
    B = len(models)
    hs = (C.c_void_p * B)(*[mo.h.value if isinstance(mo.h, C.c_void_p) else mo.h for mo in models])
    status = (C.c_int32 * B)()
    lml = (C.c_double * B)()
    st = lib().gpbo_model_status_batched(ctx.h, B, hs, status, lml)
    return st, list(status), list(lml)


def score(ctx: Context, model: Model, Xc, prec="fp32", want=("mu", "sigma", "ei"), reduce=True,
          host_argmax=False):
    """gpbo_score: posterior mean, sd, EI (device tensors) and the argmax.

    host_argmax=True passes host buffers for argmax and ei_max (the library
    then synchronises and fills them): out["argmax"] is an int and
    out["ei_max"] a float."""
    pr = PREC[prec] if isinstance(prec, str) else int(prec)
    odt = torch.float64 if pr == FP64 else torch.float32
    assert Xc.dtype == odt and Xc.is_contiguous() and Xc.shape[1] == model.d
    m = Xc.shape[0]
    out = {k: torch.empty(m, dtype=odt, device=ctx.device) for k in want}
    if reduce and host_argmax:
        am_h, em_h = C.c_int64(-2), C.c_double(0.0)
        ctx.check(lib().gpbo_score(ctx.h, model.h, m, _ptr(Xc), pr, _ptr(out.get("mu")),
                                   _ptr(out.get("sigma")), _ptr(out.get("ei")), C.byref(am_h),
                                   C.byref(em_h)))
        out["argmax"] = am_h.value
        out["ei_max"] = em_h.value
        return out
    am = torch.empty(1, dtype=torch.int64, device=ctx.device) if reduce else None
    emax = torch.empty(1, dtype=torch.float64, device=ctx.device) if reduce else None
    ctx.check(lib().gpbo_score(ctx.h, model.h, m, _ptr(Xc), pr, _ptr(out.get("mu")),
                               _ptr(out.get("sigma")), _ptr(out.get("ei")), _ptr(am), _ptr(emax)))
    if reduce:
        out["argmax"] = am
        out["ei_max"] = emax
    return out


def _ptr_array(ts):
    if ts is None:
        return None
    return (C.c_void_p * len(ts))(*[None if t is None else t.data_ptr() for t in ts])


def score_batched(ctx: Context, models, Xcs, prec="bf16", want=("ei",), host_argmax=False):
    """gpbo_score_batched: per problem the outputs named in ``want`` (any of
    "mu", "sigma", "ei"; float32 device tensors) and the argmax / EI maximum
    of every problem (device tensors, or numpy arrays with host_argmax).
    Returns (outs, argmax, ei_max) with outs a dict of per-problem lists."""
    pr = PREC[prec] if isinstance(prec, str) else int(prec)
    B = len(models)
    hs = (C.c_void_p * B)(*[mo.h.value if isinstance(mo.h, C.c_void_p) else mo.h for mo in models])
    ms = (C.c_int64 * B)(*[x.shape[0] for x in Xcs])
    xs = (C.c_void_p * B)(*[x.data_ptr() for x in Xcs])
    odt = torch.float64 if pr == FP64 else torch.float32
    outs = {k: [torch.empty(x.shape[0], dtype=odt, device=ctx.device) for x in Xcs] for k in want}
    if host_argmax:
        import numpy as np
        am = np.empty(B, dtype=np.int64)
        emax = np.empty(B, dtype=np.float64)
        amp, emp = C.c_void_p(am.ctypes.data), C.c_void_p(emax.ctypes.data)
    else:
        am = torch.empty(B, dtype=torch.int64, device=ctx.device)
        emax = torch.empty(B, dtype=torch.float64, device=ctx.device)
        amp, emp = _ptr(am), _ptr(emax)
    ctx.check(lib().gpbo_score_batched(ctx.h, B, hs, ms, xs, pr, _ptr_array(outs.get("mu")),
                                       _ptr_array(outs.get("sigma")), _ptr_array(outs.get("ei")),
                                       amp, emp))
    return outs, am, emax


def score_prepare_batched(ctx: Context, models, prec="bf16"):
    """gpbo_score_prepare_batched: build the scoring operands of all the
    models for a precision now (one launch pair), so that later scoring
    calls on them skip that step."""
    pr = PREC[prec] if isinstance(prec, str) else int(prec)
    B = len(models)
    hs = (C.c_void_p * B)(*[mo.h.value if isinstance(mo.h, C.c_void_p) else mo.h for mo in models])
    ctx.check(lib().gpbo_score_prepare_batched(ctx.h, B, hs, pr))


def topk(ctx: Context, v, k):
    """gpbo_topk: indices of the k largest entries of a float32 device vector
    (descending value, ascending index among ties)."""
    assert v.dtype == torch.float32 and v.is_contiguous()
    idx = torch.empty(k, dtype=torch.int64, device=ctx.device)
    ctx.check(lib().gpbo_topk(ctx.h, v.shape[0], _ptr(v), int(k), _ptr(idx)))
    return idx


def topk_set(ctx: Context, v, k):
    """gpbo_topk_set: the top-k entries of a float32 device vector as a set,
    in ascending index order (any k <= len(v))."""
    assert v.dtype == torch.float32 and v.is_contiguous()
    idx = torch.empty(k, dtype=torch.int64, device=ctx.device)
    ctx.check(lib().gpbo_topk_set(ctx.h, v.shape[0], _ptr(v), int(k), _ptr(idx)))
    return idx


def score_bound(ctx: Context, model: Model, Xc, want=("mu", "sigma_ub", "ei_ub")):
    """gpbo_score_bound: posterior mean and the nearest-observation upper
    bounds of sigma and EI (float32 device tensors)."""
    assert Xc.dtype == torch.float32 and Xc.is_contiguous() and Xc.shape[1] == model.d
    m = Xc.shape[0]
    out = {k: torch.empty(m, dtype=torch.float32, device=ctx.device) for k in want}
    ctx.check(lib().gpbo_score_bound(ctx.h, model.h, m, _ptr(Xc), _ptr(out.get("mu")),
                                     _ptr(out.get("sigma_ub")), _ptr(out.get("ei_ub"))))
    return out


def score_subset(ctx: Context, model: Model, Xc, idx, k2):
    """gpbo_score_subset with host outputs (synchronises): (pool index of the
    best candidate of the subset, its EI, certified)."""
    assert Xc.dtype == torch.float32 and Xc.is_contiguous() and idx.dtype == torch.int64
    nxt, em, cert = C.c_int64(-2), C.c_double(0.0), C.c_int32(-1)
    ctx.check(lib().gpbo_score_subset(ctx.h, model.h, Xc.shape[0], _ptr(Xc), idx.shape[0], _ptr(idx),
                                      int(k2), C.byref(nxt), C.byref(em), C.byref(cert)))
    return nxt.value, em.value, bool(cert.value)


def topk_noalloc(ctx: Context, v, k, idx=None):
    """gpbo_topk_noalloc: gpbo_topk with the library's static scratch; the
    output buffer may be passed in (idx, device int64 of k entries)."""
    assert v.dtype == torch.float32 and v.is_contiguous()
    if idx is None:
        idx = torch.empty(k, dtype=torch.int64, device=ctx.device)
    ctx.check(lib().gpbo_topk_noalloc(ctx.h, v.shape[0], _ptr(v), int(k), _ptr(idx)))
    return idx


def gather_rows(ctx: Context, idx, Xc):
    assert Xc.dtype == torch.float32 and Xc.is_contiguous() and idx.dtype == torch.int64
    out = torch.empty((idx.shape[0], Xc.shape[1]), dtype=torch.float32, device=ctx.device)
    ctx.check(lib().gpbo_gather_rows(ctx.h, idx.shape[0], _ptr(idx), Xc.shape[1], _ptr(Xc), _ptr(out)))
    return out


def sensitivity(base, out):
    """gpbo_sensitivity on host arrays: base (R,), out (P, V, R) -> S (R, P)."""
    import numpy as np
    base = np.ascontiguousarray(base, dtype=np.float64)
    out = np.ascontiguousarray(out, dtype=np.float64)
    P, V, R = out.shape
    S = np.empty((R, P))
    st = lib().gpbo_sensitivity(P, R, V, base.ctypes.data, out.ctypes.data, S.ctypes.data)
    if st != OK:
        raise GpboError(st, "gpbo_sensitivity")
    return S


def plan_searches(S, owner, cutoff=0.25, max_dims=10):
    """gpbo_plan_searches: (routine_search (R,), param_search (P,), n_searches)."""
    import numpy as np
    S = np.ascontiguousarray(S, dtype=np.float64)
    R, P = S.shape
    own = np.ascontiguousarray(owner, dtype=np.int32)
    rs = np.empty(R, dtype=np.int32)
    ps = np.empty(P, dtype=np.int32)
    n = C.c_int32()
    st = lib().gpbo_plan_searches(P, R, S.ctypes.data, own.ctypes.data, float(cutoff), int(max_dims),
                                  rs.ctypes.data, ps.ctypes.data, C.byref(n))
    if st != OK:
        raise GpboError(st, "gpbo_plan_searches")
    return rs, ps, n.value


class Mlp:
    """An MLP ensemble on the device (gpbo_mlp_*); params are float32 master
    weights in the per-member layout W1, b1, W2, b2, w3, b3."""

    @staticmethod
    def pack(W1, b1, W2, b2, w3, b3, device=None):
        """Per-member arrays (W1 (E,H,D), b1 (E,H), W2 (E,H,H), b2 (E,H),
        w3 (E,H), b3 (E,)) -> the (E, P) float32 device tensor the library
        takes, in its documented per-member order."""
        E = W1.shape[0]
        parts = [torch.as_tensor(a, dtype=torch.float32).reshape(E, -1)
                 for a in (W1, b1, W2, b2, w3, b3)]
        return torch.cat(parts, dim=1).contiguous().to(device or torch.device("cuda", 0))

    def __init__(self, ctx: Context, init, members, d_in, hidden=256):
        assert init.dtype == torch.float32 and init.is_cuda and init.is_contiguous()
        self.ctx = ctx
        self.E, self.D, self.H = members, d_in, hidden
        self.P = int(lib().gpbo_mlp_nparams(d_in, hidden))
        assert init.numel() == members * self.P
        h = C.c_void_p()
        ctx.check(lib().gpbo_mlp_create(ctx.h, members, d_in, hidden, _ptr(init), C.byref(h)))
        self.h = h
        ctx._children.add(self)

    def params(self):
        out = torch.empty((self.E, self.P), dtype=torch.float32, device=self.ctx.device)
        self.ctx.check(lib().gpbo_mlp_params(self.ctx.h, self.h, _ptr(out)))
        return out

    def grads(self, X, y):
        g = torch.empty((self.E, self.P), dtype=torch.float32, device=self.ctx.device)
        loss = torch.empty(self.E, dtype=torch.float32, device=self.ctx.device)
        self.ctx.check(lib().gpbo_mlp_grads(self.ctx.h, self.h, X.shape[0], _ptr(X), _ptr(y),
                                            _ptr(g), _ptr(loss)))
        return g, loss

    def train(self, X, y, steps, lr=1e-3, history=True):
        hist = torch.empty((steps, self.E), dtype=torch.float32, device=self.ctx.device) if history else None
        self.ctx.check(lib().gpbo_mlp_train(self.ctx.h, self.h, X.shape[0], _ptr(X), _ptr(y),
                                            int(steps), float(lr), _ptr(hist)))
        return hist

    def train_on_model(self, model, steps, lr=1e-3, history=True):
        """gpbo_mlp_train_model: train on a fitted model's X and normalised y."""
        hist = torch.empty((steps, self.E), dtype=torch.float32, device=self.ctx.device) if history else None
        self.ctx.check(lib().gpbo_mlp_train_model(self.ctx.h, self.h, model.h, int(steps), float(lr),
                                                  _ptr(hist)))
        return hist

    def forward(self, Xc):
        out = torch.empty((self.E, Xc.shape[0]), dtype=torch.float32, device=self.ctx.device)
        self.ctx.check(lib().gpbo_mlp_forward(self.ctx.h, self.h, Xc.shape[0], _ptr(Xc), _ptr(out)))
        return out

    def prescreen(self, Xc, f_best, k, want_ei=False):
        idx = torch.empty(k, dtype=torch.int64, device=self.ctx.device)
        ei = torch.empty(Xc.shape[0], dtype=torch.float32, device=self.ctx.device) if want_ei else None
        self.ctx.check(lib().gpbo_mlp_prescreen(self.ctx.h, self.h, Xc.shape[0], _ptr(Xc),
                                                float(f_best), int(k), _ptr(idx), _ptr(ei)))
        return idx, ei

    def set_occupancy(self, workgroups_per_cu):
        """gpbo_mlp_set_occupancy: 0 = fill the GPU; k > 0 = k workgroups per
        compute unit for the pass over a pool."""
        self.ctx.check(lib().gpbo_mlp_set_occupancy(self.ctx.h, self.h, int(workgroups_per_cu)))

    def prescreen_lcb(self, Xc, kappa, k, want_score=False):
        """gpbo_mlp_prescreen_lcb: top-k by -(ensemble mean - kappa * sd)."""
        assert Xc.dtype == torch.float32 and Xc.is_contiguous() and Xc.shape[1] == self.D
        idx = torch.empty(k, dtype=torch.int64, device=self.ctx.device)
        sc = torch.empty(Xc.shape[0], dtype=torch.float32, device=self.ctx.device) if want_score else None
        self.ctx.check(lib().gpbo_mlp_prescreen_lcb(self.ctx.h, self.h, Xc.shape[0], _ptr(Xc),
                                                    float(kappa), int(k), _ptr(idx), _ptr(sc)))
        return idx, sc

    def free(self):
        if getattr(self, "h", None):
            lib().gpbo_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
