"""Python bindings of the float64 CPU oracle (``gp_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The product path
(``paper_2403_08131_amd``) never imports it, and the two share no code: the
oracle is a plain transcription of the textbook definitions (see the header
of ``gp_oracle.c``) in float64 loops.

Parity status: every function here is pinned by tests in
``tests/test_oracle_pins.py`` against closed forms, brute force at tiny sizes,
library special cases, Monte Carlo, and finite differences.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SE = 0
MATERN52 = 1
OK = 0
NOT_PD = 2
INVALID = 1


def build(force=False):
    """Compile the oracle with gcc (-O2, IEEE float64, OpenMP)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("GPBO_ORACLE_LIB")  # a deliberately altered build, for the mutation tests
        if not path:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            path = _LIB
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        ip = C.POINTER(C.c_int)
        L.oracle_kernel.restype = C.c_double
        L.oracle_kernel.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_double]
        L.oracle_gram.restype = None
        L.oracle_gram.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_double, C.c_double, dp]
        L.oracle_cholesky.restype = C.c_int
        L.oracle_cholesky.argtypes = [C.c_int, dp, dp, ip]
        L.oracle_forward_sub.restype = None
        L.oracle_forward_sub.argtypes = [C.c_int, dp, dp, dp]
        L.oracle_back_sub.restype = None
        L.oracle_back_sub.argtypes = [C.c_int, dp, dp, dp]
        L.oracle_chol_append.restype = C.c_int
        L.oracle_chol_append.argtypes = [C.c_int, dp, dp, C.c_double, dp, ip]
        L.oracle_lml_grad.restype = C.c_int
        L.oracle_lml_grad.argtypes = [C.c_int, C.c_int, dp, dp, C.c_int, dp, C.c_double,
                                      C.c_double, C.c_int, dp, dp]
        L.oracle_fit.restype = C.c_int
        L.oracle_fit.argtypes = [C.c_int, C.c_int, dp, dp, C.c_int, dp, C.c_double,
                                 C.c_double, C.c_int, dp, dp, dp, ip]
        L.oracle_ei.restype = C.c_double
        L.oracle_ei.argtypes = [C.c_double, C.c_double, C.c_double]
        L.oracle_score.restype = None
        L.oracle_score.argtypes = [C.c_int, C.c_int, dp, C.c_int, dp, C.c_double, dp, dp,
                                   dp, C.c_int64, dp, dp, dp, dp, C.c_int]
        L.oracle_score_bound.restype = None
        L.oracle_score_bound.argtypes = [C.c_int, C.c_int, dp, C.c_int, dp, C.c_double, C.c_double,
                                         dp, dp, C.c_int64, dp, dp, dp, dp, C.c_int]
        L.oracle_max_threads.restype = C.c_int
        L.oracle_max_threads.argtypes = []
        L.oracle_argmax.restype = C.c_int64
        L.oracle_argmax.argtypes = [C.c_int64, dp]
        L.oracle_topk.restype = None
        L.oracle_topk.argtypes = [C.c_int64, dp, C.c_int64, i64p]
        L.oracle_mlp_nparams.restype = C.c_int64
        L.oracle_mlp_nparams.argtypes = [C.c_int, C.c_int]
        L.oracle_bf16.restype = C.c_double
        L.oracle_bf16.argtypes = [C.c_double]
        L.oracle_gelu.restype = C.c_double
        L.oracle_gelu.argtypes = [C.c_double]
        L.oracle_gelu_grad.restype = C.c_double
        L.oracle_gelu_grad.argtypes = [C.c_double]
        L.oracle_mlp_forward.restype = None
        L.oracle_mlp_forward.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.c_int64, dp,
                                         C.c_int, dp, C.c_int]
        L.oracle_mlp_loss_grad.restype = None
        L.oracle_mlp_loss_grad.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.c_int, dp, dp,
                                           C.c_int, dp, dp]
        L.oracle_adam.restype = None
        L.oracle_adam.argtypes = [C.c_int64, dp, dp, dp, dp, C.c_int, C.c_double,
                                  C.c_double, C.c_double, C.c_double]
        L.oracle_ens_ei.restype = None
        L.oracle_ens_ei.argtypes = [C.c_int, C.c_int64, dp, C.c_double, dp, dp, dp]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _null():
    return C.POINTER(C.c_double)()


# --------------------------------------------------------------------------
# GP
# --------------------------------------------------------------------------

def kernel(kind, a, b, ls, sf2=1.0):
    a, pa = _d(a)
    b, pb = _d(b)
    ls, pl = _d(ls)
    return lib().oracle_kernel(int(kind), a.shape[-1], pa, pb, pl, float(sf2))


def gram(kind, X, ls, sf2=1.0, sn2=0.0):
    X, px = _d(X)
    ls, pl = _d(ls)
    n, d = X.shape
    K = np.empty((n, n))
    lib().oracle_gram(int(kind), n, d, px, pl, float(sf2), float(sn2),
                      K.ctypes.data_as(C.POINTER(C.c_double)))
    return K


def cholesky(K):
    """Returns (status, L, bad_pivot)."""
    K, pk = _d(K)
    n = K.shape[0]
    L = np.empty((n, n))
    bad = C.c_int(-1)
    st = lib().oracle_cholesky(n, pk, L.ctypes.data_as(C.POINTER(C.c_double)), C.byref(bad))
    return st, L, bad.value


def forward_sub(L, b):
    L, pl = _d(L)
    b, pb = _d(b)
    z = np.empty_like(b)
    lib().oracle_forward_sub(L.shape[0], pl, pb, z.ctypes.data_as(C.POINTER(C.c_double)))
    return z


def back_sub(L, z):
    L, pl = _d(L)
    z, pz = _d(z)
    x = np.empty_like(z)
    lib().oracle_back_sub(L.shape[0], pl, pz, x.ctypes.data_as(C.POINTER(C.c_double)))
    return x


def chol_append(L, k, kappa):
    """Factor of the bordered matrix [[K, k], [k^T, kappa]] from the factor L
    of K (see oracle_chol_append).  Returns (status, L', bad_pivot)."""
    L, pL = _d(L)
    k, pk = _d(k)
    n = L.shape[0]
    out = np.empty((n + 1, n + 1))
    bad = C.c_int(-1)
    st = lib().oracle_chol_append(n, pL, pk, float(kappa),
                                  out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(bad))
    return st, out, bad.value


def lml_grad(X, y, ls, kind=SE, sf2=1.0, sn2=1e-4, normalize_y=True):
    """Gradient of the log marginal likelihood with respect to (log l_1..d,
    log sf2, log sn2) and the LML itself (see oracle_lml_grad).  Returns
    (status, grad, lml)."""
    X, px = _d(X)
    y, py = _d(y)
    n, d = X.shape
    ls, pl = _d(np.broadcast_to(np.asarray(ls, dtype=np.float64), (d,)))
    g = np.zeros(d + 2)
    lml = C.c_double(np.nan)
    st = lib().oracle_lml_grad(n, d, px, py, int(kind), pl, float(sf2), float(sn2),
                               1 if normalize_y else 0, g.ctypes.data_as(C.POINTER(C.c_double)),
                               C.byref(lml))
    return st, g, lml.value


class Fit:
    """Result of :func:`fit`: L, alpha and the scalar statistics."""

    def __init__(self, status, bad, X, kind, ls, sf2, sn2, L, alpha, stats):
        self.status = status
        self.bad_pivot = bad
        self.X = X
        self.kernel = kind
        self.ls = ls
        self.sf2 = sf2
        self.sn2 = sn2
        self.L = L
        self.alpha = alpha
        self.stats = stats

    ymean = property(lambda s: s.stats[0])
    ystd = property(lambda s: s.stats[1])
    fbest = property(lambda s: s.stats[2])
    lml = property(lambda s: s.stats[3])
    logdet = property(lambda s: s.stats[4])


def fit(X, y, ls, kind=SE, sf2=1.0, sn2=1e-4, normalize_y=True):
    X, px = _d(X)
    y, py = _d(y)
    ls, pl = _d(np.broadcast_to(np.asarray(ls, dtype=np.float64), (X.shape[1],)))
    n, d = X.shape
    L = np.zeros((n, n))
    alpha = np.zeros(n)
    stats = np.zeros(5)
    bad = C.c_int(-1)
    st = lib().oracle_fit(n, d, px, py, int(kind), pl, float(sf2), float(sn2),
                          1 if normalize_y else 0,
                          L.ctypes.data_as(C.POINTER(C.c_double)),
                          alpha.ctypes.data_as(C.POINTER(C.c_double)),
                          stats.ctypes.data_as(C.POINTER(C.c_double)), C.byref(bad))
    return Fit(st, bad.value, X, kind, ls, sf2, sn2, L, alpha, stats)


def score(f: Fit, Xc, nthreads=0, want=("mu", "sigma", "ei")):
    """Posterior mean, standard deviation and EI at the rows of Xc."""
    Xc, pc = _d(Xc)
    m = Xc.shape[0]
    out = {}
    ptrs = []
    for k in ("mu", "sigma", "ei"):
        if k in want:
            out[k] = np.empty(m)
            ptrs.append(out[k].ctypes.data_as(C.POINTER(C.c_double)))
        else:
            ptrs.append(_null())
    X, px = _d(f.X)
    ls, pl = _d(f.ls)
    L, pL = _d(f.L)
    a, pa = _d(f.alpha)
    s, ps = _d(f.stats)
    lib().oracle_score(X.shape[0], X.shape[1], px, int(f.kernel), pl, float(f.sf2), pL, pa,
                       ps, m, pc, ptrs[0], ptrs[1], ptrs[2], int(nthreads))
    return out


def score_bound(f: Fit, Xc, nthreads=0):
    """Posterior mean, the nearest-observation upper bound of the standard
    deviation and the EI upper bound it implies (see gp_oracle.c)."""
    Xc, pc = _d(Xc)
    m = Xc.shape[0]
    out = {k: np.empty(m) for k in ("mu", "sigma_ub", "ei_ub")}
    X, px = _d(f.X)
    ls, pl = _d(f.ls)
    a, pa = _d(f.alpha)
    s, ps = _d(f.stats)
    dp = C.POINTER(C.c_double)
    lib().oracle_score_bound(X.shape[0], X.shape[1], px, int(f.kernel), pl, float(f.sf2),
                             float(f.sn2), pa, ps, m, pc, out["mu"].ctypes.data_as(dp),
                             out["sigma_ub"].ctypes.data_as(dp), out["ei_ub"].ctypes.data_as(dp),
                             int(nthreads))
    return out


def ei(mu, sigma, fbest):
    return lib().oracle_ei(float(mu), float(sigma), float(fbest))


def max_threads():
    return lib().oracle_max_threads()


def argmax(v):
    v, pv = _d(v)
    return int(lib().oracle_argmax(v.shape[0], pv))


def topk(v, k):
    v, pv = _d(v)
    idx = np.empty(k, dtype=np.int64)
    lib().oracle_topk(v.shape[0], pv, int(k), idx.ctypes.data_as(C.POINTER(C.c_int64)))
    return idx


# --------------------------------------------------------------------------
# MLP ensemble
# --------------------------------------------------------------------------

def mlp_nparams(D, H):
    return int(lib().oracle_mlp_nparams(D, H))


def bf16(x):
    return lib().oracle_bf16(float(x))


def gelu(u):
    return lib().oracle_gelu(float(u))


def gelu_grad(u):
    return lib().oracle_gelu_grad(float(u))


def mlp_pack(W1, b1, W2, b2, w3, b3):
    """Per-member flat parameter vectors, (E, P) float64, in the oracle layout."""
    E = W1.shape[0]
    parts = [np.asarray(W1, np.float64).reshape(E, -1), np.asarray(b1, np.float64).reshape(E, -1),
             np.asarray(W2, np.float64).reshape(E, -1), np.asarray(b2, np.float64).reshape(E, -1),
             np.asarray(w3, np.float64).reshape(E, -1), np.asarray(b3, np.float64).reshape(E, 1)]
    return np.ascontiguousarray(np.concatenate(parts, axis=1))


def mlp_forward(params, D, H, X, bf16=False, nthreads=0):
    params, pp = _d(params)
    X, px = _d(X)
    E = params.shape[0]
    n = X.shape[0]
    out = np.empty((E, n))
    lib().oracle_mlp_forward(E, D, H, pp, n, px, 1 if bf16 else 0,
                             out.ctypes.data_as(C.POINTER(C.c_double)), int(nthreads))
    return out


def mlp_loss_grad(params, D, H, X, yt, bf16=False):
    params, pp = _d(params)
    X, px = _d(X)
    yt, py = _d(yt)
    E = params.shape[0]
    g = np.empty_like(params)
    loss = np.empty(E)
    lib().oracle_mlp_loss_grad(E, D, H, pp, X.shape[0], px, py, 1 if bf16 else 0,
                               g.ctypes.data_as(C.POINTER(C.c_double)),
                               loss.ctypes.data_as(C.POINTER(C.c_double)))
    return loss, g


def adam_step(w, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In place on contiguous float64 arrays w, m, v."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g, pg = _d(g)
    lib().oracle_adam(w.size, w.ctypes.data_as(C.POINTER(C.c_double)),
                      m.ctypes.data_as(C.POINTER(C.c_double)),
                      v.ctypes.data_as(C.POINTER(C.c_double)), pg, int(t), float(lr),
                      float(beta1), float(beta2), float(eps))


def ens_ei(out, fbest):
    out, po = _d(out)
    E, n = out.shape
    mu = np.empty(n)
    sd = np.empty(n)
    e = np.empty(n)
    lib().oracle_ens_ei(E, n, po, float(fbest), mu.ctypes.data_as(C.POINTER(C.c_double)),
                        sd.ctypes.data_as(C.POINTER(C.c_double)),
                        e.ctypes.data_as(C.POINTER(C.c_double)))
    return mu, sd, e


def ens_lcb(out, kappa):
    """Prescreen score from the ensemble's lower confidence bound, larger is
    better for minimisation: -(mean - kappa * sd), with the member mean and
    population standard deviation of ens_ei."""
    mu, sd, _ = ens_ei(out, 0.0)
    return -(mu - kappa * sd)


def mlp_train(params, D, H, X, yt, steps, lr=1e-3, bf16=False, master_f32=False):
    """Full-batch Adam training of every member; returns (params, losses per step).

    With master_f32 the master weights and Adam moments are rounded to float32
    after every step (the device keeps them in float32)."""
    w = np.ascontiguousarray(params, dtype=np.float64).copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    hist = []
    for t in range(1, steps + 1):
        loss, g = mlp_loss_grad(w, D, H, X, yt, bf16=bf16)
        hist.append(loss)
        for e in range(w.shape[0]):
            we, me, ve = w[e].copy(), m[e].copy(), v[e].copy()
            adam_step(we, me, ve, g[e], t, lr)
            w[e], m[e], v[e] = we, me, ve
        if master_f32:
            w = w.astype(np.float32).astype(np.float64)
            m = m.astype(np.float32).astype(np.float64)
            v = v.astype(np.float32).astype(np.float64)
    return w, np.array(hist)
