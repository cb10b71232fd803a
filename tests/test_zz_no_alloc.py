"""advisor_rank_cascade_noalloc (the multi-stage ranking on the library's
fixed static workspace, for callers that cannot allocate) against
advisor_rank_cascade on the same inputs: identical picks and first-stage
predictions, on two calls in a row, the second smaller than the first, and
the size limit rejected with ADVISOR_ESHAPE. Called through the C ABI."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import paper_2301_03636_amd as adv
import workload
from gpu_util import host, say, to_dev
from paper_2301_03636_amd import _lib

pytestmark = pytest.mark.gpu

ESHAPE = -2
SCRATCH = 96 << 20


def _models(widths, precs, p, f_cal, mu, sd):
    ms = []
    for pr in precs:
        m = adv.Model(widths, pr)
        m.set_params(p, mu, sd)
        if pr == "fp8":
            m.calibrate_fp8(to_dev(f_cal))
        ms.append(m)
    return ms


def _call(name, handles, keep, K, V, O, best, pred):
    arr = (C.c_void_p * len(handles))(*handles)
    kp = (C.c_int * max(len(keep), 1))(*[int(k) for k in keep])
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
    return getattr(_lib.lib(), name)(arr, kp, len(handles), ptr(K), ptr(V), ptr(O),
                                     O.shape[0] - 1, V.shape[0], ptr(best), ptr(pred), stream)


@pytest.mark.parametrize("precs, keep", [(("fp8", "bf16", "fp32"), (32, 4)),
                                         (("bf16", "fp32"), (8,)),
                                         (("fp32",), ())])
def test_noalloc_cascade_matches_allocating_call(precs, keep):
    widths = (32, 256, 256, 256, 1)
    kd, vd, off = workload.make_descriptors(2000, 16, 1024, seed=931, invalid_frac=0.03)
    f, inv = oracle.featurize(kd, vd[:65536])
    mu, sd = oracle.zscore_fit(f[inv == 0])
    p = workload.he_init(widths, 932, bias_scale=0.2)
    ms = _models(widths, precs, p, f[inv == 0][:4096], mu, sd)
    hs = [m.handle.value for m in ms]
    # two calls in a row, the second on the first 700 kernels only
    for nk in (2000, 700):
        K, V, O = to_dev(kd), to_dev(vd[:off[nk]]), to_dev(off[:nk + 1])
        say("noalloc cascade %s keep %s: %d kernels, %d variants" % ("/".join(precs), keep, nk,
                                                                     V.shape[0]))
        ref_b = torch.full((nk,), -7, dtype=torch.int64, device="cuda")
        ref_p = torch.zeros(V.shape[0], dtype=torch.float32, device="cuda")
        assert _call("advisor_rank_cascade", hs, keep, K, V, O, ref_b, ref_p) == 0
        for give_pred in (True, False):
            b = torch.full((nk,), -9, dtype=torch.int64, device="cuda")
            pr = torch.full((V.shape[0],), 5.0, dtype=torch.float32, device="cuda") if give_pred else None
            rc = _call("advisor_rank_cascade_noalloc", hs, keep, K, V, O, b, pr)
            assert rc == 0, _lib.last_error()
            assert np.array_equal(host(b), host(ref_b))
            if give_pred:
                assert np.array_equal(host(pr).view(np.uint32), host(ref_p).view(np.uint32))
        assert (host(ref_b) >= -1).all()
    for m in ms:
        m.close()


def test_noalloc_cascade_rejects_workspace_above_the_limit():
    """A last cut takes 72 bytes per candidate: 50,000 kernels x 32
    candidates (110 MiB) is above the 96 MiB array; the call fails before
    any device work and leaves best_out untouched."""
    widths = (32, 64, 64, 1)
    p = workload.he_init(widths, 941)
    ms = _models(widths, ("bf16", "fp32"), p, None, np.zeros(32), np.ones(32))
    hs = [m.handle.value for m in ms]
    nk = 50000
    kd, vd, off = workload.make_descriptors(nk, 1, 2, seed=942)
    K, V, O = to_dev(kd), to_dev(vd), to_dev(off)
    b = torch.full((nk,), -9, dtype=torch.int64, device="cuda")
    pr = torch.empty(V.shape[0], dtype=torch.float32, device="cuda")
    assert _call("advisor_rank_cascade_noalloc", hs, (32,), K, V, O, b, pr) == ESHAPE
    assert "workspace" in _lib.last_error()
    assert (host(b) == -9).all()
    # the same call with fewer candidates per kernel fits and matches
    ref = torch.empty(nk, dtype=torch.int64, device="cuda")
    assert _call("advisor_rank_cascade", hs, (4,), K, V, O, ref, None) == 0
    assert _call("advisor_rank_cascade_noalloc", hs, (4,), K, V, O, b, None) == 0
    assert np.array_equal(host(b), host(ref))
    for m in ms:
        m.close()
