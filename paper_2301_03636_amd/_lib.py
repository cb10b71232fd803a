"""ctypes binding of libadvisor.so: argument marshalling only.

Every function here has the name of the C entry point it calls and checks
nothing that the library does not check itself beyond tensor placement,
dtype and contiguity (the library sees raw pointers). Device buffers are
torch tensors on the current HIP device; work is enqueued on torch's current
stream. There is no fallback: if the library is missing, loading fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# ADVISOR_LIBRARY names another build of the library to load (the sanitizer run)
LIB_PATH = os.environ.get("ADVISOR_LIBRARY") or os.path.join(_HERE, "libadvisor.so")

FP32, BF16, FP8_E4M3, BF16X3 = 0, 1, 2, 3
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp8": FP8_E4M3, "bf16x3": BF16X3}
NFEAT = 32

_lib = None


class AdvisorError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__("%s failed (%d): %s" % (where, code, msg))
        self.code = code


def lib():
    """Load libadvisor.so (built by paper_2301_03636_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libadvisor.so is not built (%s); run "
                              "paper_2301_03636_amd/build.py or __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        P, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        sig = {
            "advisor_last_error": ([], C.c_char_p),
            "advisor_version": ([], C.c_char_p),
            "advisor_model_create": ([P, i32, i32, C.POINTER(C.c_void_p)], i32),
            "advisor_model_destroy": ([P], None),
            "advisor_model_param_count": ([P], i64),
            "advisor_model_set_params": ([P, P, P, P], i32),
            "advisor_model_get_params": ([P, P, P, P], i32),
            "advisor_model_get_adam": ([P, P, P, C.POINTER(C.c_int64)], i32),
            "advisor_model_set_adam": ([P, P, P, i64], i32),
            "advisor_model_set_zscore": ([P, P, P, P], i32),
            "advisor_featurize": ([P, P, i64, i64, P, P, P], i32),
            "advisor_zscore_fit": ([P, i64, P, P, P], i32),
            "advisor_predict": ([P, P, i64, P, P], i32),
            "advisor_rank": ([P, P, P, P, i64, i64, P, P, P], i32),
            "advisor_rank_preds": ([P, P, i64, i64, P, P], i32),
            "advisor_rank_refined": ([P, P, P, P, P, i64, i64, i32, P, P, P], i32),
            "advisor_rank_cascade": ([P, P, i32, P, P, P, i64, i64, P, P, P], i32),
            "advisor_rank_cascade_noalloc": ([P, P, i32, P, P, P, i64, i64, P, P, P], i32),
            "advisor_mlp_saved_bytes": ([P, i64], i64),
            "advisor_mlp_forward": ([P, P, i64, P, P, P], i32),
            "advisor_mlp_backward": ([P, P, P, i64, P, P], i32),
            "advisor_train_step": ([P, P, P, i64, C.c_float, C.c_float, C.c_float, C.c_float, P, P,
                                    P], i32),
            "advisor_model_load_params": ([P, P, P], i32),
            "advisor_model_grads": ([P, P, P], i32),
            "advisor_model_calibrate_fp8": ([P, P, i64, P], i32),
            "advisor_model_get_fp8_scales": ([P, P, P], i32),
            "advisor_rank_plan_create": ([P, P, P, P, i64, i64, P, P, C.POINTER(C.c_void_p)], i32),
            "advisor_train_plan_create": ([P, P, P, i64, C.c_float, C.c_float, C.c_float,
                                           C.c_float, P, P, C.POINTER(C.c_void_p)], i32),
            "advisor_plan_launch": ([P, P], i32),
            "advisor_plan_destroy": ([P], None),
            "advisor_autotune": ([P, P, P, P, i64, i64, i32, P, i32, C.POINTER(C.c_int), P], i32),
            "advisor_model_set_tile_variant": ([P, i32], i32),
            "advisor_model_get_tile_variant": ([P], i32),
            "advisor_profile_enable": ([i32], i32),
            "advisor_profile_read": ([C.POINTER(C.c_int64), C.POINTER(C.c_double)], i32),
            "advisor_profile_read_each": ([C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_int64)],
                                          i32),
            "advisor_mfma_peak": ([i32, i64, i32, C.POINTER(C.c_double), P], i32),
            "advisor_validate_offsets": ([P, i64, i64, C.POINTER(C.c_int64), P], i32),
            "advisor_train_step_rmsprop": ([P, P, P, i64, C.c_float, C.c_float, C.c_float,
                                            C.c_float, i32, P, P, P], i32),
            "advisor_train_plan_create_rmsprop": ([P, P, P, i64, C.c_float, C.c_float, C.c_float,
                                                   C.c_float, i32, P, P, C.POINTER(C.c_void_p)],
                                                  i32),
            "advisor_train_plan_create_rmsprop_multi": ([P, P, P, P, i32, C.c_float, C.c_float,
                                                         C.c_float, C.c_float, i32, P, P,
                                                         C.POINTER(C.c_void_p)], i32),
            "advisor_rank_multi": ([P, i32, P, P, P, i64, i64, P, P, P], i32),
            "advisor_classify_maps": ([P, P, P, i64, i64, P, P, P, P, P], i32),
            "advisor_count_variants": ([P, i64, i32, P, P], i32),
            "advisor_enumerate_variants": ([P, P, i64, i64, i32, P, P], i32),
            "advisor_topn_preds": ([P, P, i64, i64, i32, P, P, P], i32),
            "advisor_rank_topn": ([P, P, P, P, i64, i64, i32, P, P, P, P], i32),
            "advisor_step_lr": ([i64, C.c_double, C.c_double, i64], C.c_double),
            "advisor_lower_variants": ([P, P, i64, i64, i64, i64, P, P], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def last_error() -> str:
    return lib().advisor_last_error().decode()


def _check(rc: int, where: str):
    if rc != 0:
        raise AdvisorError(rc, where, last_error())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s tensor on the GPU" % (name, dtype))
    return t


# --------------------------------------------------------------------------- model


def advisor_model_create(widths, precision) -> C.c_void_p:
    w = np.ascontiguousarray(widths, dtype=np.int32)
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    h = C.c_void_p()
    _check(lib().advisor_model_create(w.ctypes.data_as(C.c_void_p), w.size, p, C.byref(h)),
           "advisor_model_create")
    return h


def advisor_model_destroy(h):
    lib().advisor_model_destroy(h)


def advisor_model_param_count(h) -> int:
    return int(lib().advisor_model_param_count(h))


def advisor_model_set_params(h, w_master, mu, sigma):
    w = np.ascontiguousarray(w_master, dtype=np.float32)
    m = np.ascontiguousarray(mu, dtype=np.float64)
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    if w.size != advisor_model_param_count(h) or m.size != NFEAT or s.size != NFEAT:
        raise ValueError("parameter or statistics size mismatch")
    _check(lib().advisor_model_set_params(h, w.ctypes.data_as(C.c_void_p),
                                          m.ctypes.data_as(C.c_void_p),
                                          s.ctypes.data_as(C.c_void_p)),
           "advisor_model_set_params")


def advisor_model_get_params(h):
    n = advisor_model_param_count(h)
    w = np.zeros(n, dtype=np.float32)
    mu = np.zeros(NFEAT)
    sd = np.zeros(NFEAT)
    _check(lib().advisor_model_get_params(h, w.ctypes.data_as(C.c_void_p),
                                          mu.ctypes.data_as(C.c_void_p),
                                          sd.ctypes.data_as(C.c_void_p)),
           "advisor_model_get_params")
    return w, mu, sd


def advisor_model_get_adam(h):
    n = advisor_model_param_count(h)
    m = np.zeros(n, dtype=np.float32)
    v = np.zeros(n, dtype=np.float32)
    step = C.c_int64(0)
    _check(lib().advisor_model_get_adam(h, m.ctypes.data_as(C.c_void_p),
                                        v.ctypes.data_as(C.c_void_p), C.byref(step)),
           "advisor_model_get_adam")
    return m, v, step.value


def advisor_model_set_adam(h, m, v, step):
    mm = np.ascontiguousarray(m, dtype=np.float32)
    vv = np.ascontiguousarray(v, dtype=np.float32)
    _check(lib().advisor_model_set_adam(h, mm.ctypes.data_as(C.c_void_p),
                                        vv.ctypes.data_as(C.c_void_p), int(step)),
           "advisor_model_set_adam")


def advisor_model_set_zscore(h, mu, sigma):
    _dev(mu, torch.float64, "mu")
    _dev(sigma, torch.float64, "sigma")
    _check(lib().advisor_model_set_zscore(h, _ptr(mu), _ptr(sigma), _stream()),
           "advisor_model_set_zscore")


def advisor_model_calibrate_fp8(h, feat):
    _dev(feat, torch.int64, "feat")
    _check(lib().advisor_model_calibrate_fp8(h, _ptr(feat), feat.shape[0], _stream()),
           "advisor_model_calibrate_fp8")


def advisor_model_get_fp8_scales(h, n_hidden):
    w = np.zeros(n_hidden, dtype=np.float32)
    a = np.zeros(n_hidden, dtype=np.float32)
    _check(lib().advisor_model_get_fp8_scales(h, w.ctypes.data_as(C.c_void_p),
                                              a.ctypes.data_as(C.c_void_p)),
           "advisor_model_get_fp8_scales")
    return w, a


# --------------------------------------------------------------------------- hot path


def advisor_featurize(kdesc, vdesc, n_kernels=None, feat_out=None, invalid_out=None):
    _dev(kdesc, torch.int64, "kdesc")
    _dev(vdesc, torch.int64, "vdesc")
    nk = kdesc.shape[0] if n_kernels is None else int(n_kernels)
    nv = vdesc.shape[0]
    if feat_out is None:
        feat_out = torch.empty((nv, NFEAT), dtype=torch.int64, device=vdesc.device)
    if invalid_out is None:
        invalid_out = torch.empty(nv, dtype=torch.uint8, device=vdesc.device)
    _dev(feat_out, torch.int64, "feat_out")
    _dev(invalid_out, torch.uint8, "invalid_out")
    _check(lib().advisor_featurize(_ptr(kdesc), _ptr(vdesc), nk, nv, _ptr(feat_out),
                                   _ptr(invalid_out), _stream()), "advisor_featurize")
    return feat_out, invalid_out


def advisor_zscore_fit(feat):
    _dev(feat, torch.int64, "feat")
    mu = torch.empty(NFEAT, dtype=torch.float64, device=feat.device)
    sd = torch.empty(NFEAT, dtype=torch.float64, device=feat.device)
    _check(lib().advisor_zscore_fit(_ptr(feat), feat.shape[0], _ptr(mu), _ptr(sd), _stream()),
           "advisor_zscore_fit")
    return mu, sd


def advisor_predict(h, feat, pred_out=None):
    _dev(feat, torch.int64, "feat")
    n = feat.shape[0]
    if pred_out is None:
        pred_out = torch.empty(n, dtype=torch.float32, device=feat.device)
    _dev(pred_out, torch.float32, "pred_out")
    _check(lib().advisor_predict(h, _ptr(feat), n, _ptr(pred_out), _stream()), "advisor_predict")
    return pred_out


def advisor_rank(h, kdesc, vdesc, offsets, best_out=None, pred_out=None, want_pred=False):
    for t, nm in ((kdesc, "kdesc"), (vdesc, "vdesc"), (offsets, "offsets")):
        _dev(t, torch.int64, nm)
    nk = offsets.shape[0] - 1
    nv = vdesc.shape[0]
    if best_out is None:
        best_out = torch.empty(nk, dtype=torch.int64, device=vdesc.device)
    if pred_out is None and want_pred:
        pred_out = torch.empty(nv, dtype=torch.float32, device=vdesc.device)
    _dev(best_out, torch.int64, "best_out")
    _dev(pred_out, torch.float32, "pred_out")
    _check(lib().advisor_rank(h, _ptr(kdesc), _ptr(vdesc), _ptr(offsets), nk, nv,
                              _ptr(best_out), _ptr(pred_out), _stream()), "advisor_rank")
    return (best_out, pred_out) if want_pred or pred_out is not None else best_out


def advisor_rank_multi(handles, kdesc, vdesc, offsets, best_out=None, pred_out=None,
                       want_pred=False):
    """Rank the same variants by several models (one per target): best
    [n_models, n_k] (and pred [n_models, n_v])."""
    for t, nm in ((kdesc, "kdesc"), (vdesc, "vdesc"), (offsets, "offsets")):
        _dev(t, torch.int64, nm)
    nm_ = len(handles)
    nk = offsets.shape[0] - 1
    nv = vdesc.shape[0]
    if best_out is None:
        best_out = torch.empty((nm_, nk), dtype=torch.int64, device=vdesc.device)
    if pred_out is None and want_pred:
        pred_out = torch.empty((nm_, nv), dtype=torch.float32, device=vdesc.device)
    _dev(best_out, torch.int64, "best_out")
    _dev(pred_out, torch.float32, "pred_out")
    if best_out.numel() != nm_ * nk or (pred_out is not None and pred_out.numel() != nm_ * nv):
        raise ValueError("output sizes do not match n_models x n_kernels / n_variants")
    arr = (C.c_void_p * max(nm_, 1))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    _check(lib().advisor_rank_multi(arr, nm_, _ptr(kdesc), _ptr(vdesc), _ptr(offsets), nk, nv,
                                    _ptr(best_out), _ptr(pred_out), _stream()),
           "advisor_rank_multi")
    return (best_out, pred_out) if want_pred or pred_out is not None else best_out


def advisor_rank_refined(h, refine, kdesc, vdesc, offsets, top_k=8, best_out=None,
                         pred_out=None):
    for t, nm in ((kdesc, "kdesc"), (vdesc, "vdesc"), (offsets, "offsets")):
        _dev(t, torch.int64, nm)
    nk = offsets.shape[0] - 1
    nv = vdesc.shape[0]
    if best_out is None:
        best_out = torch.empty(nk, dtype=torch.int64, device=vdesc.device)
    _dev(best_out, torch.int64, "best_out")
    _dev(pred_out, torch.float32, "pred_out")
    _check(lib().advisor_rank_refined(h, refine, _ptr(kdesc), _ptr(vdesc), _ptr(offsets), nk, nv,
                                      int(top_k), _ptr(best_out), _ptr(pred_out), _stream()),
           "advisor_rank_refined")
    return best_out


def advisor_rank_cascade(handles, keep, kdesc, vdesc, offsets, best_out=None, pred_out=None):
    """Multi-stage ranking: handles [n_stages] model handles (first the
    fastest), keep [n_stages - 1] candidates per kernel handed on by each cut."""
    return _cascade("advisor_rank_cascade", handles, keep, kdesc, vdesc, offsets, best_out,
                    pred_out)


def advisor_rank_cascade_noalloc(handles, keep, kdesc, vdesc, offsets, best_out, pred_out=None):
    """advisor_rank_cascade on the library's fixed static workspace: the call
    allocates no device memory (best_out must be given)."""
    if best_out is None:
        raise ValueError("advisor_rank_cascade_noalloc: best_out must be given")
    return _cascade("advisor_rank_cascade_noalloc", handles, keep, kdesc, vdesc, offsets, best_out,
                    pred_out)


def _cascade(name, handles, keep, kdesc, vdesc, offsets, best_out, pred_out):
    for t, nm in ((kdesc, "kdesc"), (vdesc, "vdesc"), (offsets, "offsets")):
        _dev(t, torch.int64, nm)
    nk = offsets.shape[0] - 1
    nv = vdesc.shape[0]
    if best_out is None:
        best_out = torch.empty(nk, dtype=torch.int64, device=vdesc.device)
    _dev(best_out, torch.int64, "best_out")
    _dev(pred_out, torch.float32, "pred_out")
    ns = len(handles)
    arr = (C.c_void_p * max(ns, 1))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    kp = (C.c_int * max(len(keep), 1))(*[int(k) for k in keep])
    _check(getattr(lib(), name)(arr, kp, ns, _ptr(kdesc), _ptr(vdesc), _ptr(offsets), nk, nv,
                                _ptr(best_out), _ptr(pred_out), _stream()), name)
    return best_out


def advisor_validate_offsets(offsets, n_variants):
    """-1 when offsets (device int64 [n_k + 1]) segments n_variants rows,
    else the lowest offending index (the library also reports ADVISOR_ESHAPE,
    which this wrapper turns into the index rather than an exception)."""
    _dev(offsets, torch.int64, "offsets")
    bad = C.c_int64(-1)
    rc = lib().advisor_validate_offsets(_ptr(offsets), offsets.shape[0] - 1, int(n_variants),
                                        C.byref(bad), _stream())
    if rc not in (0, -2):
        _check(rc, "advisor_validate_offsets")
    return bad.value


def advisor_rank_preds(pred, offsets, best_out=None):
    _dev(pred, torch.float32, "pred")
    _dev(offsets, torch.int64, "offsets")
    nk = offsets.shape[0] - 1
    if best_out is None:
        best_out = torch.empty(nk, dtype=torch.int64, device=pred.device)
    _dev(best_out, torch.int64, "best_out")
    _check(lib().advisor_rank_preds(_ptr(pred), _ptr(offsets), nk, pred.shape[0], _ptr(best_out),
                                    _stream()), "advisor_rank_preds")
    return best_out


def advisor_classify_maps(access, nbytes, var_offsets):
    """(class [n_vars] uint8, enter, exit, naive bytes [n_k] int64) of
    section 4.1.2's data analysis."""
    _dev(access, torch.uint8, "access")
    _dev(nbytes, torch.int64, "nbytes")
    _dev(var_offsets, torch.int64, "var_offsets")
    nk = var_offsets.shape[0] - 1
    nv = access.shape[0]
    if nbytes.shape[0] != nv:
        raise ValueError("access and nbytes differ in length")
    dev = access.device
    cls = torch.empty(nv, dtype=torch.uint8, device=dev)
    e, x, n = (torch.empty(nk, dtype=torch.int64, device=dev) for _ in range(3))
    _check(lib().advisor_classify_maps(_ptr(access), _ptr(nbytes), _ptr(var_offsets), nk, nv,
                                       _ptr(cls), _ptr(e), _ptr(x), _ptr(n), _stream()),
           "advisor_classify_maps")
    return cls, e, x, n


def advisor_count_variants(n_loops, sched_mask=7, offsets_out=None):
    _dev(n_loops, torch.int64, "n_loops")
    nk = n_loops.shape[0]
    if offsets_out is None:
        offsets_out = torch.empty(nk + 1, dtype=torch.int64, device=n_loops.device)
    _dev(offsets_out, torch.int64, "offsets_out")
    if offsets_out.numel() != nk + 1:
        raise ValueError("offsets_out must hold n_kernels + 1 elements")
    _check(lib().advisor_count_variants(_ptr(n_loops), nk, int(sched_mask), _ptr(offsets_out),
                                        _stream()), "advisor_count_variants")
    return offsets_out


def advisor_enumerate_variants(n_loops, sched_mask=7, offsets=None, variants_out=None):
    """(offsets [n_k + 1], variants [n_v, 6]) of section 4.1.3's variant
    generation; counts first (one host synchronization to size the rows)."""
    _dev(n_loops, torch.int64, "n_loops")
    if offsets is None:
        offsets = advisor_count_variants(n_loops, sched_mask)
    _dev(offsets, torch.int64, "offsets")
    nk = n_loops.shape[0]
    nv = int(offsets[-1].item())
    if variants_out is None:
        variants_out = torch.empty((nv, 6), dtype=torch.int64, device=n_loops.device)
    _dev(variants_out, torch.int64, "variants_out")
    if variants_out.numel() != nv * 6:
        raise ValueError("variants_out must hold offsets[-1] rows of 6")
    _check(lib().advisor_enumerate_variants(_ptr(n_loops), _ptr(offsets), nk, nv, int(sched_mask),
                                            _ptr(variants_out), _stream()),
           "advisor_enumerate_variants")
    return offsets, variants_out


def advisor_lower_variants(kdesc, variants, teams, threads, vdesc_out=None):
    """Generated variants (rows of advisor_enumerate_variants) as cost-model
    descriptor rows [n_v, 8] under the given default launch."""
    _dev(kdesc, torch.int64, "kdesc")
    _dev(variants, torch.int64, "variants")
    nv = variants.shape[0]
    if vdesc_out is None:
        vdesc_out = torch.empty((nv, 8), dtype=torch.int64, device=variants.device)
    _dev(vdesc_out, torch.int64, "vdesc_out")
    _check(lib().advisor_lower_variants(_ptr(kdesc), _ptr(variants), kdesc.shape[0], nv,
                                        int(teams), int(threads), _ptr(vdesc_out), _stream()),
           "advisor_lower_variants")
    return vdesc_out


def _topn_outputs(nk, top_n, idx_out, val_out, device):
    if idx_out is None:
        idx_out = torch.empty((nk, top_n), dtype=torch.int64, device=device)
    if val_out is None:
        val_out = torch.empty((nk, top_n), dtype=torch.float32, device=device)
    _dev(idx_out, torch.int64, "idx_out")
    _dev(val_out, torch.float32, "val_out")
    if idx_out.numel() != nk * top_n or val_out.numel() != nk * top_n:
        raise ValueError("idx_out and val_out must hold n_kernels * top_n elements")
    return idx_out, val_out


def advisor_topn_preds(pred, offsets, top_n, idx_out=None, val_out=None):
    """(idx [n_k, top_n] int64, val [n_k, top_n] float32): each kernel's
    variants by ascending prediction, -1 / NaN past the eligible ones."""
    _dev(pred, torch.float32, "pred")
    _dev(offsets, torch.int64, "offsets")
    nk = offsets.shape[0] - 1
    idx_out, val_out = _topn_outputs(nk, int(top_n), idx_out, val_out, pred.device)
    _check(lib().advisor_topn_preds(_ptr(pred), _ptr(offsets), nk, pred.shape[0], int(top_n),
                                    _ptr(idx_out), _ptr(val_out), _stream()),
           "advisor_topn_preds")
    return idx_out, val_out


def advisor_rank_topn(h, kdesc, vdesc, offsets, top_n, idx_out=None, val_out=None, pred_out=None):
    """The fused prediction flow with a top-N list per kernel: (idx, val)
    as for advisor_topn_preds."""
    for t, name in ((kdesc, "kdesc"), (vdesc, "vdesc"), (offsets, "offsets")):
        _dev(t, torch.int64, name)
    nk = offsets.shape[0] - 1
    nv = vdesc.shape[0]
    idx_out, val_out = _topn_outputs(nk, int(top_n), idx_out, val_out, vdesc.device)
    if pred_out is not None:
        _dev(pred_out, torch.float32, "pred_out")
    _check(lib().advisor_rank_topn(h, _ptr(kdesc), _ptr(vdesc), _ptr(offsets), nk, nv, int(top_n),
                                   _ptr(idx_out), _ptr(val_out), _ptr(pred_out), _stream()),
           "advisor_rank_topn")
    return idx_out, val_out


# --------------------------------------------------------------------------- measurement


def advisor_profile_enable(on: bool):
    _check(lib().advisor_profile_enable(1 if on else 0), "advisor_profile_enable")


def advisor_profile_read():
    """(launches, summed milliseconds) of the tile-kernel launches bracketed
    since profiling was enabled or last read."""
    n = C.c_int64(0)
    ms = C.c_double(0.0)
    _check(lib().advisor_profile_read(C.byref(n), C.byref(ms)), "advisor_profile_read")
    return n.value, ms.value


def advisor_profile_read_each(cap=4096):
    """Durations (ms, launch order) of the tile-kernel launches bracketed
    since profiling was enabled or last read (at most `cap` of them)."""
    n = C.c_int64(0)
    buf = (C.c_double * max(int(cap), 1))()
    _check(lib().advisor_profile_read_each(buf, int(cap), C.byref(n)), "advisor_profile_read_each")
    return [buf[i] for i in range(min(n.value, int(cap)))]


def advisor_mfma_peak(precision, iters=20000, workgroups_per_cu=2) -> float:
    """Sustained dense matrix-core TFLOP/s of the current device for
    'fp32', 'bf16' or 'fp8' (register operands, no memory traffic)."""
    code = {"fp32": 0, "bf16": 1, "fp8": 2}[precision]
    out = C.c_double(0.0)
    _check(lib().advisor_mfma_peak(code, int(iters), int(workgroups_per_cu), C.byref(out),
                                   _stream()), "advisor_mfma_peak")
    return out.value


# --------------------------------------------------------------------------- training


def advisor_mlp_saved_bytes(h, n) -> int:
    return int(lib().advisor_mlp_saved_bytes(h, int(n)))


def advisor_mlp_forward(h, feat, y_out=None, saved=None):
    _dev(feat, torch.int64, "feat")
    n = feat.shape[0]
    if y_out is None:
        y_out = torch.empty(n, dtype=torch.float32, device=feat.device)
    if saved is None:
        saved = torch.empty(advisor_mlp_saved_bytes(h, n), dtype=torch.uint8, device=feat.device)
    _dev(y_out, torch.float32, "y_out")
    _dev(saved, torch.uint8, "saved")
    if saved.numel() < advisor_mlp_saved_bytes(h, n):
        raise ValueError("saved buffer too small")
    _check(lib().advisor_mlp_forward(h, _ptr(feat), n, _ptr(y_out), _ptr(saved), _stream()),
           "advisor_mlp_forward")
    return y_out, saved


def advisor_mlp_backward(h, dy, saved, n, grads_out=None):
    _dev(dy, torch.float32, "dy")
    _dev(saved, torch.uint8, "saved")
    if grads_out is None:
        grads_out = torch.empty(advisor_model_param_count(h), dtype=torch.float32, device=dy.device)
    _dev(grads_out, torch.float32, "grads_out")
    _check(lib().advisor_mlp_backward(h, _ptr(dy), _ptr(saved), int(n), _ptr(grads_out), _stream()),
           "advisor_mlp_backward")
    return grads_out


def advisor_train_step(h, feat, y, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, loss_out=None,
                       gnorm_out=None):
    _dev(feat, torch.int64, "feat")
    _dev(y, torch.float64, "y")
    if loss_out is None:
        loss_out = torch.empty(1, dtype=torch.float64, device=feat.device)
    if gnorm_out is None:
        gnorm_out = torch.empty(1, dtype=torch.float64, device=feat.device)
    _check(lib().advisor_train_step(h, _ptr(feat), _ptr(y), feat.shape[0], lr, beta1, beta2, eps,
                                    _ptr(loss_out), _ptr(gnorm_out), _stream()),
           "advisor_train_step")
    return loss_out, gnorm_out


LOSSES = {"mse": 0, "rmse": 1}


def advisor_step_lr(epoch, lr0=1e-2, gamma=0.1, every=30):
    r = lib().advisor_step_lr(int(epoch), float(lr0), float(gamma), int(every))
    if r != r:
        raise AdvisorError(-1, "advisor_step_lr", last_error())
    return r


def advisor_train_step_rmsprop(h, feat, y, lr=1e-2, alpha=0.99, eps=1e-8, weight_decay=1e-4,
                               loss="rmse", loss_out=None, gnorm_out=None):
    _dev(feat, torch.int64, "feat")
    _dev(y, torch.float64, "y")
    if loss not in LOSSES:
        raise ValueError("loss must be one of %s" % sorted(LOSSES))
    if loss_out is None:
        loss_out = torch.empty(1, dtype=torch.float64, device=feat.device)
    if gnorm_out is None:
        gnorm_out = torch.empty(1, dtype=torch.float64, device=feat.device)
    _check(lib().advisor_train_step_rmsprop(h, _ptr(feat), _ptr(y), feat.shape[0], lr, alpha, eps,
                                            weight_decay, LOSSES[loss], _ptr(loss_out),
                                            _ptr(gnorm_out), _stream()),
           "advisor_train_step_rmsprop")
    return loss_out, gnorm_out


def advisor_model_load_params(h, w_master):
    _dev(w_master, torch.float32, "w_master")
    if w_master.numel() != advisor_model_param_count(h):
        raise ValueError("parameter count mismatch")
    _check(lib().advisor_model_load_params(h, _ptr(w_master), _stream()),
           "advisor_model_load_params")


def advisor_model_grads(h, grads_out):
    _dev(grads_out, torch.float32, "grads_out")
    _check(lib().advisor_model_grads(h, _ptr(grads_out), _stream()), "advisor_model_grads")
    return grads_out


# --------------------------------------------------------------------------- captured plans


def advisor_rank_plan_create(h, kdesc, vdesc, offsets, best_out, pred_out=None):
    for t, nm in ((kdesc, "kdesc"), (vdesc, "vdesc"), (offsets, "offsets"), (best_out, "best_out")):
        _dev(t, torch.int64, nm)
    _dev(pred_out, torch.float32, "pred_out")
    p = C.c_void_p()
    _check(lib().advisor_rank_plan_create(h, _ptr(kdesc), _ptr(vdesc), _ptr(offsets),
                                          offsets.shape[0] - 1, vdesc.shape[0], _ptr(best_out),
                                          _ptr(pred_out), C.byref(p)), "advisor_rank_plan_create")
    return p


def advisor_train_plan_create(h, feat, y, loss_out, gnorm_out, lr=1e-3, beta1=0.9, beta2=0.999,
                              eps=1e-8):
    _dev(feat, torch.int64, "feat")
    for t, nm in ((y, "y"), (loss_out, "loss_out"), (gnorm_out, "gnorm_out")):
        _dev(t, torch.float64, nm)
    p = C.c_void_p()
    _check(lib().advisor_train_plan_create(h, _ptr(feat), _ptr(y), feat.shape[0], lr, beta1, beta2,
                                           eps, _ptr(loss_out), _ptr(gnorm_out), C.byref(p)),
           "advisor_train_plan_create")
    return p


def advisor_train_plan_create_rmsprop(h, feat, y, loss_out, gnorm_out, lr=1e-2, alpha=0.99,
                                      eps=1e-8, weight_decay=1e-4, loss="rmse"):
    _dev(feat, torch.int64, "feat")
    for t, nm in ((y, "y"), (loss_out, "loss_out"), (gnorm_out, "gnorm_out")):
        _dev(t, torch.float64, nm)
    if loss not in LOSSES:
        raise ValueError("loss must be one of %s" % sorted(LOSSES))
    p = C.c_void_p()
    _check(lib().advisor_train_plan_create_rmsprop(h, _ptr(feat), _ptr(y), feat.shape[0], lr, alpha,
                                                   eps, weight_decay, LOSSES[loss], _ptr(loss_out),
                                                   _ptr(gnorm_out), C.byref(p)),
           "advisor_train_plan_create_rmsprop")
    return p


def advisor_train_plan_create_rmsprop_multi(handles, feats, ys, loss_out=None, gnorm_out=None,
                                            lr=1e-2, alpha=0.99, eps=1e-8, weight_decay=1e-4,
                                            loss="rmse"):
    n = len(handles)
    if not (len(feats) == len(ys) == n):
        raise ValueError("one batch per model")
    for f, y in zip(feats, ys):
        _dev(f, torch.int64, "feat")
        _dev(y, torch.float64, "y")
        if y.shape[0] != f.shape[0]:
            raise ValueError("feat and y differ in rows")
    for t, nm in ((loss_out, "loss_out"), (gnorm_out, "gnorm_out")):
        _dev(t, torch.float64, nm)
        if t is not None and t.numel() < n:
            raise ValueError("%s needs one entry per model" % nm)
    if loss not in LOSSES:
        raise ValueError("loss must be one of %s" % sorted(LOSSES))
    hs = (C.c_void_p * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    fp = (C.c_void_p * n)(*[f.data_ptr() for f in feats])
    yp = (C.c_void_p * n)(*[y.data_ptr() for y in ys])
    ns = (C.c_int64 * n)(*[f.shape[0] for f in feats])
    p = C.c_void_p()
    _check(lib().advisor_train_plan_create_rmsprop_multi(hs, fp, yp, ns, n, lr, alpha, eps,
                                                         weight_decay, LOSSES[loss],
                                                         _ptr(loss_out), _ptr(gnorm_out),
                                                         C.byref(p)),
           "advisor_train_plan_create_rmsprop_multi")
    return p


def advisor_plan_launch(p):
    _check(lib().advisor_plan_launch(p, _stream()), "advisor_plan_launch")


def advisor_plan_destroy(p):
    lib().advisor_plan_destroy(p)


# --------------------------------------------------------------------------- autotuner


def advisor_autotune(h, kdesc, vdesc, offsets, reps=5, max_variants=4):
    for t, nm in ((kdesc, "kdesc"), (vdesc, "vdesc"), (offsets, "offsets")):
        _dev(t, torch.int64, nm)
    times = np.zeros(max_variants)
    chosen = C.c_int(-1)
    _check(lib().advisor_autotune(h, _ptr(kdesc), _ptr(vdesc), _ptr(offsets), offsets.shape[0] - 1,
                                  vdesc.shape[0], int(reps), times.ctypes.data_as(C.c_void_p),
                                  max_variants, C.byref(chosen), _stream()), "advisor_autotune")
    return chosen.value, times


def advisor_model_set_tile_variant(h, v):
    _check(lib().advisor_model_set_tile_variant(h, int(v)), "advisor_model_set_tile_variant")


def advisor_model_get_tile_variant(h):
    return int(lib().advisor_model_get_tile_variant(h))
