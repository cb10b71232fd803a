"""FP8 (OCP e4m3) inference with calibrated per-tensor scales.

Two checks: the kernel against a numpy model of exactly the quantized
arithmetic it is meant to perform (bf16 first layer, e4m3 weights and
activations with the library's scales, fp32 accumulation), which must agree
closely; and the fp8 predictions against the float64 oracle, whose error is
bounded by e4m3's 3-bit mantissa and whose argmin agreement is reported.
"""
import numpy as np
import pytest

import oracle
import paper_2301_03636_amd as adv
import workload
from gpu_util import host, rel_err, say, segment_argmin, to_dev

def e4m3_table():
    """All non-negative finite OCP e4m3 values, indexed by their code."""
    vals = []
    for code in range(0x7F):          # 0x7f is NaN
        e, m = code >> 3, code & 7
        vals.append(m * 2.0 ** -9 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 7))
    return np.array(vals)


E4M3 = e4m3_table()


def to_e4m3(x):
    """Round to the nearest e4m3 value, ties to the even code, saturating."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), 448.0)
    i = np.clip(np.searchsorted(E4M3, a), 1, E4M3.size - 1)
    lo, hi = E4M3[i - 1], E4M3[i]
    pick_hi = (a - lo > hi - a) | ((a - lo == hi - a) & (i % 2 == 0))
    q = np.where(pick_hi, hi, lo)
    q = np.where(a >= E4M3[-1], E4M3[-1], q)
    return np.sign(x) * q


def to_bf16(x):
    f = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((f + 0x7FFF + ((f >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_e4m3_table_is_the_ocp_format():
    assert E4M3[0] == 0.0 and E4M3[1] == 2.0 ** -9 and E4M3[8] == 2.0 ** -6
    assert E4M3[-1] == 448.0 and np.all(np.diff(E4M3) > 0)
    assert to_e4m3(1000.0) == 448.0 and to_e4m3(-0.0) == 0.0
    assert to_e4m3(1.0625) == 1.0 and to_e4m3(1.1875) == 1.25   # ties to even


def emulate(widths, p, x, wscale, ascale):
    """The quantized network the fp8 kernels implement, in float64."""
    off = 0
    h = to_bf16(x)
    L = len(widths) - 2
    for l in range(L + 1):
        fin, fout = widths[l], widths[l + 1]
        W = p[off:off + fout * fin].reshape(fout, fin)
        off += fout * fin
        b = p[off:off + fout]
        off += fout
        if l == L:
            return h @ W[0] + b[0]
        if l == 0:
            z = h @ to_bf16(W).T + b
        else:
            qa = to_e4m3(h / ascale[l])
            qw = to_e4m3(W / wscale[l])
            z = (qa @ qw.T) * (np.float32(wscale[l]) * np.float32(ascale[l])) + b
        h = np.maximum(z, 0.0)


@pytest.mark.gpu
@pytest.mark.parametrize("widths", [(32, 256, 256, 256, 1), (32, 1024, 1024, 1), (32, 64, 1)])
def test_fp8_kernel_matches_quantized_model_and_oracle(widths):
    kd, vd, off = workload.make_descriptors(60, 16, 600, seed=401)
    f, inv = oracle.featurize(kd, vd)
    p = workload.he_init(widths, 402, bias_scale=0.1)
    mu, sd = oracle.zscore_fit(f[inv == 0])
    m = adv.Model(widths, "fp8")
    m.set_params(p, mu, sd)
    with pytest.raises(adv.AdvisorError):
        m.predict(to_dev(f))                       # not calibrated yet
    cal = f[workload.sample_rows(f.shape[0], 4096, 403)]
    m.calibrate_fp8(to_dev(cal))
    wscale, ascale = m.fp8_scales()
    assert np.all(wscale > 0) and np.all(ascale > 0)
    pred = host(m.predict(to_dev(f)))
    x = oracle.normalize(f, mu, sd)
    emu = emulate(widths, p.astype(np.float64), x, wscale, ascale)
    e_emu = rel_err(pred, emu)
    ref = oracle.forward(widths, p.astype(np.float64), x)
    e_ref = rel_err(pred, ref)
    say("fp8 %s: vs quantized model median %.2e p99 %.2e; vs oracle median %.3f max %.3f" %
        (widths, np.median(e_emu), np.percentile(e_emu, 99), np.median(e_ref), e_ref.max()))
    # the same quantized arithmetic: only fp32 summation order differs, which
    # can move a value across an e4m3 rounding boundary in a later layer
    assert np.median(e_emu) < 1e-5
    assert np.mean(e_emu < 1e-3) > 0.97
    # against float64: 3 mantissa bits per operand
    assert np.median(e_ref) < 0.05
    # rank gives the same bits as predict, and an exact argmin on them
    best, pr = m.rank(to_dev(kd), to_dev(vd), to_dev(off), want_pred=True)
    pr = host(pr)
    ok = inv == 0
    assert np.array_equal(pr[ok], pred[ok])
    assert host(best).tolist() == segment_argmin(pr, off).tolist()
    best_ref, _ = oracle.rank(kd, vd, off, widths, p.astype(np.float64), mu, sd)
    say("  argmin agreement with the oracle: %.3f" % np.mean(host(best) == best_ref))
