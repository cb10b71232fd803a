"""CPU float64 oracle of the cost-model hot path (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
use this package. It is a ctypes wrapper over ``oracle.c`` (plain C, float64,
no BLAS), built with gcc on first use, plus the synthetic runtime model that
stands in for measured runtimes. It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_LIBRARY names another build of oracle.c to load (the sanitizer run)
_LIB = os.environ.get("ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
NFEAT = 32

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no fast-math,
    no FMA contraction, OpenMP over kernels in the rank routine)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out: str) -> str:
    """oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer (ROCm's
    clang, shared sanitizer runtime), for a CPU run of the tests with that
    runtime preloaded."""
    cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
           "-fPIC", "-shared", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-shared-libsan", _SRC, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def _load():
    global _lib
    if _lib is None:
        if not os.environ.get("ORACLE_LIBRARY"):
            build()
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        i64 = C.c_int64
        lib.oracle_featurize.argtypes = [P, P, i64, i64, P, P]
        lib.oracle_featurize.restype = None
        lib.oracle_zscore_fit.argtypes = [P, i64, P, P]
        lib.oracle_zscore_fit.restype = None
        lib.oracle_normalize.argtypes = [P, i64, P, P, P]
        lib.oracle_normalize.restype = None
        lib.oracle_forward.argtypes = [P, C.c_int, P, C.c_int, P, i64, P]
        lib.oracle_forward.restype = C.c_int
        lib.oracle_argmin.argtypes = [P, P, P, i64, P]
        lib.oracle_argmin.restype = None
        lib.oracle_topn.argtypes = [P, P, P, i64, C.c_int, P]
        lib.oracle_topn.restype = None
        lib.oracle_mse.argtypes = [P, P, i64]
        lib.oracle_mse.restype = C.c_double
        lib.oracle_loss_grad.argtypes = [P, C.c_int, P, C.c_int, P, P, i64, P, P]
        lib.oracle_loss_grad.restype = C.c_int
        lib.oracle_l2norm.argtypes = [P, i64]
        lib.oracle_l2norm.restype = C.c_double
        lib.oracle_adam.argtypes = [P, P, P, P, i64, i64, C.c_double, C.c_double, C.c_double,
                                    C.c_double]
        lib.oracle_adam.restype = None
        lib.oracle_rmsprop.argtypes = [P, P, P, i64, C.c_double, C.c_double, C.c_double,
                                       C.c_double]
        lib.oracle_rmsprop.restype = None
        lib.oracle_enumerate.argtypes = [C.c_int, C.c_int, P]
        lib.oracle_enumerate.restype = i64
        lib.oracle_lower_variants.argtypes = [P, P, i64, i64, i64, P]
        lib.oracle_lower_variants.restype = None
        lib.oracle_map_class.argtypes = [C.c_int]
        lib.oracle_map_class.restype = C.c_int
        lib.oracle_classify.argtypes = [P, P, P, i64, P, P, P, P]
        lib.oracle_classify.restype = None
        lib.oracle_rank.argtypes = [P, P, P, i64, i64, P, C.c_int, P, P, P, P, P, C.c_int]
        lib.oracle_rank.restype = C.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = C.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


ACT = {"relu": 0, "identity": 1}


def featurize(kdesc, vdesc):
    kd, vd = _c(kdesc, np.int64), _c(vdesc, np.int64)
    n = vd.shape[0]
    feat = np.zeros((n, NFEAT), dtype=np.int64)
    inv = np.zeros(n, dtype=np.uint8)
    _load().oracle_featurize(_p(kd), _p(vd), kd.shape[0], n, _p(feat), _p(inv))
    return feat, inv


def zscore_fit(feat):
    f = _c(feat, np.int64)
    mu = np.zeros(NFEAT)
    sd = np.zeros(NFEAT)
    _load().oracle_zscore_fit(_p(f), f.shape[0], _p(mu), _p(sd))
    return mu, sd


def normalize(feat, mu, sigma):
    f = _c(feat, np.int64)
    x = np.zeros((f.shape[0], NFEAT))
    _load().oracle_normalize(_p(f), f.shape[0], _p(_c(mu, np.float64)),
                             _p(_c(sigma, np.float64)), _p(x))
    return x


def _widths(widths):
    return _c(widths, np.int32)


def forward(widths, params, x, act="relu"):
    w = _widths(widths)
    p = _c(params, np.float64)
    xx = _c(x, np.float64)
    y = np.zeros(xx.shape[0])
    rc = _load().oracle_forward(_p(w), w.size, _p(p), ACT[act], _p(xx), xx.shape[0], _p(y))
    if rc:
        raise ValueError("oracle_forward: bad widths (%d)" % rc)
    return y


def argmin(pred, offsets, invalid=None):
    pr = _c(pred, np.float64)
    off = _c(offsets, np.int64)
    inv = None if invalid is None else _c(invalid, np.uint8)
    best = np.zeros(off.size - 1, dtype=np.int64)
    _load().oracle_argmin(_p(pr), _p(inv), _p(off), off.size - 1, _p(best))
    return best


def topn(pred, offsets, N, invalid=None):
    pr = _c(pred, np.float64)
    off = _c(offsets, np.int64)
    inv = None if invalid is None else _c(invalid, np.uint8)
    out = np.zeros((off.size - 1, N), dtype=np.int64)
    _load().oracle_topn(_p(pr), _p(inv), _p(off), off.size - 1, int(N), _p(out))
    return out


def mse(pred, y):
    a, b = _c(pred, np.float64), _c(y, np.float64)
    return _load().oracle_mse(_p(a), _p(b), a.size)


def rmse(pred, y):
    """Root mean square error between predicted and true runtimes."""
    return float(np.sqrt(mse(pred, y)))


def nrmse(pred, y, y_min=None, y_max=None):
    """RMSE divided by the range of the true values (the paper's
    normalization; the range may be given explicitly)."""
    y = np.asarray(y, dtype=np.float64)
    lo = float(np.min(y)) if y_min is None else float(y_min)
    hi = float(np.max(y)) if y_max is None else float(y_max)
    return rmse(pred, y) / (hi - lo)


def loss_grad(widths, params, x, y, act="relu"):
    w = _widths(widths)
    p = _c(params, np.float64)
    xx, yy = _c(x, np.float64), _c(y, np.float64)
    g = np.zeros_like(p)
    loss = C.c_double(0.0)
    rc = _load().oracle_loss_grad(_p(w), w.size, _p(p), ACT[act], _p(xx), _p(yy), xx.shape[0],
                                  _p(g), C.byref(loss))
    if rc:
        raise ValueError("oracle_loss_grad failed (%d)" % rc)
    return loss.value, g


def l2norm(g):
    gg = _c(g, np.float64)
    return _load().oracle_l2norm(_p(gg), gg.size)


def adam(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays w, m, v."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    gg = _c(g, np.float64)
    _load().oracle_adam(_p(w), _p(m), _p(v), _p(gg), w.size, int(t), lr, b1, b2, eps)


def rmse_loss_grad(widths, params, x, y, act="relu"):
    """The RMSE loss of section 5.3 (eq. rmse: the square root of the mean
    squared error) and its gradient by the chain rule, d sqrt(L) = dL / (2
    sqrt(L)), taken as 0 where the error is exactly 0."""
    mse, g = loss_grad(widths, params, x, y, act)
    r = float(np.sqrt(mse))
    return r, (g / (2.0 * r) if r > 0.0 else np.zeros_like(g))


def rmsprop(w, v, g, lr=1e-2, alpha=0.99, eps=1e-8, weight_decay=0.0):
    """In-place RMSprop step with coupled weight decay on float64 arrays w, v."""
    for a in (w, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    gg = _c(g, np.float64)
    _load().oracle_rmsprop(_p(w), _p(v), _p(gg), w.size, lr, alpha, eps, weight_decay)


def step_lr(epoch, lr0=1e-2, gamma=0.1, every=30):
    """The learning-rate schedule of section 5.3: lr0, multiplied by gamma
    after every `every` epochs."""
    return lr0 * gamma ** (int(epoch) // int(every))


def map_class(bits):
    """Section 4.1.2's map class of one variable from its access bits."""
    return _load().oracle_map_class(int(bits))


def classify(access, nbytes, var_offsets):
    """(class [n_vars] uint8, enter, exit, naive bytes [n_k] int64)."""
    acc = _c(access, np.uint8)
    b = _c(nbytes, np.int64)
    off = _c(var_offsets, np.int64)
    nk = off.size - 1
    cls = np.zeros(acc.size, dtype=np.uint8)
    e, x, nv = (np.zeros(nk, dtype=np.int64) for _ in range(3))
    _load().oracle_classify(_p(acc), _p(b), _p(off), nk, _p(cls), _p(e), _p(x), _p(nv))
    return cls, e, x, nv


def enumerate_variants(n_loops, sched_mask=7):
    """Section 4.1.3's variants of kernels with the given loop counts:
    (offsets [n_k + 1], rows [n_v, 6] = kernel, x, d, c, schedule, data)."""
    nl = np.asarray(n_loops, dtype=np.int64).ravel()
    L = _load()
    counts = np.array([L.oracle_enumerate(int(n) if -2**31 < n < 2**31 else 0, int(sched_mask),
                                          None) for n in nl], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    rows = np.zeros((int(off[-1]), 6), dtype=np.int64)
    for k, n in enumerate(nl):
        if counts[k] == 0:
            continue
        blk = np.zeros((int(counts[k]), 5), dtype=np.int64)
        L.oracle_enumerate(int(n), int(sched_mask), _p(blk))
        rows[off[k]:off[k + 1], 0] = k
        rows[off[k]:off[k + 1], 1:] = blk
    return off, rows


def lower_variants(kdesc, gen_rows, teams, threads):
    """Generated variants (rows [k, x, d, c, schedule, data] of
    enumerate_variants) as cost-model descriptor rows [n_v, 8]: the parallel
    structure c + 8x + 64d + 512 schedule, the given default launch, and map
    clauses from the data option (0: each array's analysed class, 1: tofrom)."""
    kd, g = _c(kdesc, np.int64), _c(gen_rows, np.int64)
    out = np.zeros((g.shape[0], 8), dtype=np.int64)
    _load().oracle_lower_variants(_p(kd), _p(g), g.shape[0], int(teams), int(threads), _p(out))
    return out


def rank(kdesc, vdesc, offsets, widths, params, mu, sigma, n_threads=0, want_pred=True):
    kd, vd, off = _c(kdesc, np.int64), _c(vdesc, np.int64), _c(offsets, np.int64)
    w = _widths(widths)
    p = _c(params, np.float64)
    best = np.zeros(off.size - 1, dtype=np.int64)
    pred = np.zeros(vd.shape[0]) if want_pred else None
    rc = _load().oracle_rank(_p(kd), _p(vd), _p(off), off.size - 1, vd.shape[0], _p(w), w.size,
                             _p(p), _p(_c(mu, np.float64)), _p(_c(sigma, np.float64)),
                             _p(best), _p(pred), int(n_threads))
    if rc:
        raise ValueError("oracle_rank failed (%d)" % rc)
    return best, pred


def max_threads():
    return _load().oracle_max_threads()
