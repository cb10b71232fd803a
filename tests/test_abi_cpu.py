"""The C ABI without a GPU: the library loads, exports every entry point its
header declares, and rejects bad arguments on the host with the documented
status codes before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2301_03636_amd as adv
from paper_2301_03636_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "advisor.h")

OK, EINVAL, ESHAPE, EHIP, ENOMEM, EUNSUP = 0, -1, -2, -3, -4, -5


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(advisor_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_version_and_error_text():
    L = _lib.lib()
    assert b"gfx950" in L.advisor_version()
    rc = L.advisor_featurize(None, None, -1, 5, None, None, None)
    assert rc == ESHAPE and "negative" in _lib.last_error()


@pytest.mark.parametrize("args,code", [
    ((None, None, 1, 10, None, None, None), EINVAL),
    ((None, None, -1, 10, None, None, None), ESHAPE),
    ((C.c_void_p(8), C.c_void_p(8), 1, 1 << 32, C.c_void_p(8), C.c_void_p(8), None), ESHAPE),
    ((None, None, 0, 0, None, None, None), OK),
])
def test_featurize_argument_checks(args, code):
    assert _lib.lib().advisor_featurize(*args) == code


def test_rank_preds_argument_checks():
    L = _lib.lib()
    assert L.advisor_rank_preds(None, None, 1, 4, None, None) == EINVAL
    assert L.advisor_rank_preds(None, None, -1, 4, None, None) == ESHAPE
    assert L.advisor_rank_preds(C.c_void_p(8), C.c_void_p(8), 1, 1 << 32, C.c_void_p(8),
                                None) == ESHAPE
    assert L.advisor_rank_preds(None, None, 0, 0, None, None) == OK


def test_model_create_argument_checks():
    L = _lib.lib()
    h = C.c_void_p()

    def create(widths, prec):
        w = np.ascontiguousarray(widths, dtype=np.int32)
        return L.advisor_model_create(w.ctypes.data_as(C.c_void_p), w.size, prec, C.byref(h))
    assert create([32, 64, 1], 7) == EINVAL
    assert create([31, 64, 1], 0) == ESHAPE
    assert create([32, 64, 2], 0) == ESHAPE
    assert create([32, 2048, 1], 1) == ESHAPE
    assert create([32, 1], 0) == ESHAPE
    assert create([32] + [64] * 9 + [1], 0) == ESHAPE
    assert L.advisor_model_create(None, 3, 0, C.byref(h)) == EINVAL
    assert L.advisor_model_create(None, 3, 0, None) == EINVAL


def test_entry_points_reject_null_model():
    L = _lib.lib()
    assert L.advisor_predict(None, None, 4, None, None) == EINVAL
    assert L.advisor_rank(None, None, None, None, 1, 4, None, None, None) == EINVAL
    assert L.advisor_rank_refined(None, None, None, None, None, 1, 4, 8, None, None, None) == EINVAL
    assert L.advisor_model_set_params(None, None, None, None) == EINVAL
    assert L.advisor_model_param_count(None) == -1
    L.advisor_model_destroy(None)


def test_cascade_argument_checks():
    L = _lib.lib()
    null2 = (C.c_void_p * 3)(None, None, None)

    def call(n_stages, keep, nk=1, nv=4, models=null2):
        kp = None if keep is None else (C.c_int * len(keep))(*keep)
        return L.advisor_rank_cascade(models, kp, n_stages, None, None, None, nk, nv, None, None,
                                      None)
    assert call(0, [8]) == EINVAL
    assert call(5, [8, 4, 2, 1]) == EINVAL
    assert call(2, None) == EINVAL
    assert call(2, [3]) == EINVAL            # not a power of two
    assert call(2, [64]) == EINVAL           # more than 32
    assert call(3, [4, 8]) == EINVAL         # a later cut keeps more
    assert call(2, [8], nk=-1) == ESHAPE
    assert call(2, [8], nv=1 << 32) == ESHAPE
    assert call(2, [8], nk=1 << 26) == ESHAPE
    assert call(2, [8]) == EINVAL            # null models
    assert call(1, None, models=None) == EINVAL


def test_zscore_argument_checks():
    L = _lib.lib()
    assert L.advisor_zscore_fit(None, 0, None, None, None) == ESHAPE
    assert L.advisor_zscore_fit(None, 5, None, None, None) == EINVAL


def test_python_binding_names_match_c():
    for n in declared_symbols():
        if n in ("advisor_last_error", "advisor_version"):
            continue
        assert hasattr(_lib, n), n
    assert adv.PRECISIONS == {"fp32": 0, "bf16": 1, "fp8": 2, "bf16x3": 3}
    # the codes are the header's enum values
    hdr = open(os.path.join(ROOT, "include", "advisor.h")).read()
    for name, code in (("ADVISOR_FP32", 0), ("ADVISOR_BF16", 1), ("ADVISOR_FP8_E4M3", 2),
                       ("ADVISOR_BF16X3", 3)):
        assert re.search(r"\b%s = %d\b" % (name, code), hdr), name


def test_profile_read_each_argument_checks():
    L = _lib.lib()
    n = C.c_int64(-5)
    assert L.advisor_profile_read_each(None, -1, C.byref(n)) == EINVAL
    # nothing bracketed (profiling never enabled): no launches, no device work
    buf = (C.c_double * 4)(7.0, 7.0, 7.0, 7.0)
    assert L.advisor_profile_read_each(buf, 4, C.byref(n)) == 0
    assert n.value == 0 and list(buf) == [7.0] * 4
    assert _lib.advisor_profile_read_each(8) == []


def test_mfma_peak_argument_checks():
    L = _lib.lib()
    out = C.c_double(0.0)
    assert L.advisor_mfma_peak(0, 10, 1, None, None) == EINVAL
    assert L.advisor_mfma_peak(7, 10, 1, C.byref(out), None) == EINVAL
    assert L.advisor_mfma_peak(1, 0, 1, C.byref(out), None) == EINVAL
    assert L.advisor_mfma_peak(1, (1 << 24) + 1, 1, C.byref(out), None) == EINVAL
    assert L.advisor_mfma_peak(2, 10, 0, C.byref(out), None) == EINVAL
    assert L.advisor_mfma_peak(2, 10, 9, C.byref(out), None) == EINVAL


def test_validate_offsets_argument_checks():
    L = _lib.lib()
    bad = C.c_int64(7)
    assert L.advisor_validate_offsets(None, 3, 10, C.byref(bad), None) == EINVAL
    assert bad.value == -1
    assert L.advisor_validate_offsets(C.c_void_p(8), -1, 10, C.byref(bad), None) == ESHAPE


def test_topn_argument_checks():
    L = _lib.lib()
    v = C.c_void_p(8)
    assert L.advisor_topn_preds(v, v, 1, 4, 0, v, None, None) == EINVAL
    assert L.advisor_topn_preds(v, v, 1, 4, 33, v, None, None) == EINVAL
    assert L.advisor_topn_preds(None, None, 1, 4, 10, None, None, None) == EINVAL
    assert L.advisor_topn_preds(v, v, -1, 4, 10, v, None, None) == ESHAPE
    assert L.advisor_topn_preds(v, v, 1, 1 << 32, 10, v, None, None) == ESHAPE
    assert L.advisor_topn_preds(None, None, 0, 0, 10, None, None, None) == OK
    assert L.advisor_rank_topn(None, v, v, v, 1, 4, 10, v, None, None, None) == EINVAL
    assert "null model" in _lib.last_error()


def test_rmsprop_argument_checks():
    L = _lib.lib()
    v = C.c_void_p(8)
    f = C.c_float
    assert L.advisor_train_step_rmsprop(None, v, v, 16, f(1e-2), f(0.99), f(1e-8), f(1e-4), 1,
                                        None, None, None) == EINVAL
    assert "null" in _lib.last_error() or "model" in _lib.last_error()


def test_variant_generation_argument_checks():
    L = _lib.lib()
    v = C.c_void_p(8)
    assert L.advisor_count_variants(v, 4, 0, v, None) == EINVAL
    assert L.advisor_count_variants(v, 4, 8, v, None) == EINVAL
    assert L.advisor_count_variants(None, 4, 7, v, None) == EINVAL
    assert L.advisor_count_variants(v, -1, 7, v, None) == ESHAPE
    assert L.advisor_count_variants(v, 4, 7, None, None) == EINVAL
    assert L.advisor_enumerate_variants(v, v, 4, -1, 7, v, None) == ESHAPE
    assert L.advisor_enumerate_variants(v, None, 4, 10, 7, v, None) == EINVAL
    assert L.advisor_enumerate_variants(v, v, 0, 0, 7, None, None) == OK


def test_classify_maps_argument_checks():
    L = _lib.lib()
    v = C.c_void_p(8)
    assert L.advisor_classify_maps(v, v, None, 2, 5, None, None, None, None, None) == EINVAL
    assert L.advisor_classify_maps(None, v, v, 2, 5, None, None, None, None, None) == EINVAL
    assert L.advisor_classify_maps(v, v, v, -1, 5, None, None, None, None, None) == ESHAPE
    assert L.advisor_classify_maps(None, None, None, 0, 0, None, None, None, None, None) == OK


def test_rank_multi_argument_checks():
    L = _lib.lib()
    assert L.advisor_rank_multi(None, 0, None, None, None, 1, 1, None, None, None) == EINVAL
    arr = (C.c_void_p * 1)(None)
    assert L.advisor_rank_multi(arr, 1, None, None, None, 1, 1, None, None, None) == EINVAL


def test_multi_train_plan_argument_checks():
    L = _lib.lib()
    out = C.c_void_p()
    assert L.advisor_train_plan_create_rmsprop_multi(None, None, None, None, 0, C.c_float(1e-2),
                                                     C.c_float(0.99), C.c_float(1e-8),
                                                     C.c_float(1e-4), 1, None, None,
                                                     C.byref(out)) == EINVAL


def test_missing_library_fails_loudly(monkeypatch):
    """No fallback: without the built library every entry point raises."""
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libadvisor.so")
    with pytest.raises(ImportError):
        _lib.lib()
    with pytest.raises(ImportError):
        adv.Model((32, 8, 1), "fp32")


def test_step_lr_schedule_from_the_library():
    """Section 5.3's schedule as the library computes it (host only): 0.01
    for epochs 0-29, divided by ten every 30 epochs; bad arguments raise."""
    assert adv.step_lr(0) == 1e-2 and adv.step_lr(29) == 1e-2
    assert np.isclose(adv.step_lr(30), 1e-3, rtol=1e-15, atol=0)
    assert np.isclose(adv.step_lr(149), 1e-6, rtol=1e-14, atol=0)
    assert adv.step_lr(59, lr0=0.5, gamma=0.5, every=20) == 0.125
    import oracle
    assert all(adv.step_lr(e) == oracle.step_lr(e) for e in range(300))
    for bad in ((-1, 1e-2, 0.1, 30), (0, 0.0, 0.1, 30), (0, 1e-2, 1.5, 30), (0, 1e-2, 0.1, 0)):
        with pytest.raises(adv.AdvisorError):
            adv.step_lr(*bad)
