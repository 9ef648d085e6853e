"""Batched form: many uneven series through m2n_batch_psd (one t check, the
lattice tapers of all series in one set of launches, one NuFFT launch set per
band count) give the same tapers bit for bit and the same P / Ehat within the
NuFFT tolerance as the per-series calls, and match the CPU FP64 oracle.
Calls on the same t buffers reuse the last t-check records and confirm them
at the end: in-place changes of t (span, lattice, validity) give a fresh
context's results (tapers bitwise) or its error."""
import numpy as np
import pytest

import workloads as W
from tests.metrics import align_signs, normwise_rows, psd_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m2n():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_01943_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(m2n):
    c = m2n.Context(0)
    yield c
    c.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _say(msg):
    print(msg, flush=True)


def _spec(s, want_E=True):
    return {"t": _dev(s.t), "x": _dev(s.x), "fmax": s.fmax, "fw": s.fw, "K": s.K,
            "f_lo": s.f_lo, "df": s.df, "I": s.I, "want_E": want_E}


def _single(m2n, ctx, s, prec, want_E=True):
    t, x = _dev(s.t), _dev(s.x)
    w, lam = m2n.gpss_tapers(ctx, t, s.fmax, s.fw, s.K)
    out = m2n.m2nufft_psd(ctx, t, x, w, lam, s.fmax, s.fw, s.f_lo, s.df, s.I, prec=prec,
                          want_E=want_E)
    return w, lam, out["P"], out["E"]


def _compare(m2n, ctx, series, flags, prec):
    specs = [_spec(s, e) for s, e in zip(series, flags)]
    outs = m2n.m2n_batch_psd(ctx, specs, prec=prec)
    torch.cuda.synchronize()
    for s, e, o in zip(series, flags, outs):
        w, lam, P, E = _single(m2n, ctx, s, prec, e)
        dP = psd_err(o["P"].double().cpu().numpy(), P.double().cpu().numpy())
        _say(f"  {s.name} N={s.N} K={s.K} I={s.I}: batch-vs-single P {dP:.2e}")
        assert torch.equal(o["w"], w) and torch.equal(o["lam"], lam)
        assert dP < (2e-6 if prec == m2n.M2N_FP32 else 1e-12)
        if e:
            assert torch.allclose(o["E"].double(), E.double(), rtol=0, atol=1e-7)


def test_batch_matches_single_series(m2n, ctx):
    series = [W.batched_series(s) for s in range(10)]
    _say(f"case batched_series 0..9, N {[s.N for s in series]}")
    _compare(m2n, ctx, series, [True] * len(series), m2n.M2N_FP32)


def test_batch_mixed_paths_and_band_counts(m2n, ctx):
    # single-workgroup NuFFT (I = 512), a dense (jittered) GEP, two lattice
    # series with I = 2^16, in one batch
    series = [W.small_gapped(), W.jitter_stress(n=300, seed=42, K=5), W.batched_series(3),
              W.batched_series(7)]
    series[1].I, series[1].df = 4096, 1.0 / 4096
    _say("case mixed: small_gapped, jitter_stress(300), batched_series 3 and 7")
    _compare(m2n, ctx, series, [True, False, True, True], m2n.M2N_FP32)
    _compare(m2n, ctx, series[:2], [True, False], m2n.M2N_FP64)


def test_batch_512_series_bitwise_tapers(m2n, ctx):
    # the batched form's size (512 uneven series, more than 4,096 Gram chunks in
    # all): every series' tapers and eigenvalues are bitwise those of its call
    # alone, P within the FP32 NuFFT tolerance
    series = [W.batched_series(s) for s in range(512)]
    _say(f"case 512 batched_series: {sum(s.N for s in series)} samples, "
         f"{sum((s.N + 63) // 64 for s in series)} Gram chunks")
    outs = m2n.m2n_batch_psd(ctx, [_spec(s) for s in series], prec=m2n.M2N_FP32)
    torch.cuda.synchronize()
    worst = 0.0
    for s, o in zip(series, outs):
        w, lam, P, _ = _single(m2n, ctx, s, m2n.M2N_FP32, False)
        assert torch.equal(o["w"], w) and torch.equal(o["lam"], lam), s.name
        worst = max(worst, psd_err(o["P"].double().cpu().numpy(), P.double().cpu().numpy()))
    _say(f"  tapers bitwise for all 512; P batch-vs-single max {worst:.2e}")
    assert worst < 2e-6


def test_batch_against_oracle(m2n, ctx, orc):
    picks = [s for s in (W.batched_series(i) for i in range(40)) if s.N < 2500][:2]
    assert len(picks) == 2
    outs = m2n.m2n_batch_psd(ctx, [_spec(s) for s in picks], prec=m2n.M2N_FP32)
    for s, o in zip(picks, outs):
        _say(f"case oracle {s.name} N={s.N} K={s.K}")
        w_o, lam_o = orc.gpss_tapers(s.t, s.fmax, s.fw, s.K)
        lam = o["lam"].cpu().numpy()
        w, sgn = align_signs(o["w"].cpu().numpy(), w_o)
        assert np.abs(lam - lam_o).max() < 1e-12
        assert normwise_rows(w, w_o) < 1e-9
        # the sign rule applied inside the eigen-solver agrees with the oracle's
        assert np.all(sgn == 1.0)
        bands = np.linspace(0, s.I - 1, 512).round().astype(np.int64)
        P_o = orc.psd(orc.nudft(s.t, s.x, w_o, s.f_lo, s.df, bands=bands))
        P = o["P"].double().cpu().numpy()[bands]
        e = float(np.max(np.abs(P - P_o)) / np.max(P_o))
        _say(f"  lambda {np.abs(lam - lam_o).max():.2e}  P sampled {e:.2e}")
        assert e < 1e-5


def test_batch_error_names_series(m2n, ctx):
    good = W.small_gapped()
    bad = W.small_gapped()
    bad.t = bad.t.copy()
    bad.t[[3, 4]] = bad.t[[4, 3]]
    with pytest.raises(m2n.M2NError) as ei:
        m2n.m2n_batch_psd(ctx, [_spec(good), _spec(bad)], prec=m2n.M2N_FP32)
    assert ei.value.code == m2n.M2N_ERR_T_ORDER
    assert "series 1" in str(ei.value)


def _same_result(got, ref, label):
    # tapers and eigenvalues bit for bit; P and Ehat within the FP32 NuFFT
    # tolerance (the spreading sums points in an order set by LDS atomics)
    assert torch.equal(got["w"], ref["w"]) and torch.equal(got["lam"], ref["lam"]), label
    dP = psd_err(got["P"].double().cpu().numpy(), ref["P"].double().cpu().numpy())
    assert dP < 2e-6, (label, dP)
    assert torch.allclose(got["E"].double(), ref["E"].double(), rtol=0, atol=1e-7), label


def _run_on(m2n, c, spec, prec):
    o = m2n.m2n_batch_psd(c, [spec], prec=prec)[0]
    torch.cuda.synchronize()
    return {k: (v.clone() if v is not None else None) for k, v in o.items()}


@pytest.mark.parametrize("name", ["small_gapped", "batched_series_3"])
def test_batch_check_records_reused_and_confirmed(m2n, ctx, name):
    # Calls on the same t buffer queue their tapers on the previous call's
    # t-check records and compare them with the real check at the end.  Each
    # case below changes the buffer in place between calls: results must
    # equal those of a fresh context (which has no records to reuse), and an
    # invalid t must still be reported.
    s = W.small_gapped() if name == "small_gapped" else W.batched_series(3)
    t0 = s.t.copy()
    t, x = _dev(t0), _dev(s.x)
    spec = {"t": t, "x": x, "fmax": s.fmax, "fw": s.fw, "K": s.K, "f_lo": s.f_lo, "df": s.df,
            "I": s.I, "want_E": True}
    prec = m2n.M2N_FP32
    cases = [("same contents", t0),
             ("t shifted by 7 (t_1, t_N change)", t0 + 7.0),
             ("one sample off the integers (dense path)", t0 + np.where(np.arange(s.N) == 5, 0.5, 0.0)),
             ("back to the first contents", t0)]
    _run_on(m2n, ctx, spec, prec)   # leaves the records of t0
    for label, tv in cases:
        t.copy_(torch.from_numpy(tv))
        torch.cuda.synchronize()
        got = _run_on(m2n, ctx, spec, prec)
        c2 = m2n.Context(0)
        ref = _run_on(m2n, c2, spec, prec)
        c2.close()
        _say(f"case {name}: {label}")
        _same_result(got, ref, label)
    # an invalid t after valid records: the real check wins
    bad = t0.copy()
    bad[[3, 4]] = bad[[4, 3]]
    t.copy_(torch.from_numpy(bad))
    torch.cuda.synchronize()
    with pytest.raises(m2n.M2NError) as ei:
        m2n.m2n_batch_psd(ctx, [spec], prec=prec)
    assert ei.value.code == m2n.M2N_ERR_T_ORDER
    t.copy_(torch.from_numpy(t0))
    torch.cuda.synchronize()
    got = _run_on(m2n, ctx, spec, prec)
    c2 = m2n.Context(0)
    ref = _run_on(m2n, c2, spec, prec)
    c2.close()
    _same_result(got, ref, "valid again after the error")


def test_gpss_tapers_check_records_reused_and_confirmed(m2n, ctx):
    # the per-series taper call follows the same scheme: in-place changes of
    # t between calls give a fresh context's tapers bit for bit, and an
    # invalid t is still reported
    s = W.batched_series(5)
    t0 = s.t.copy()
    t = _dev(t0)
    w = torch.empty((s.K, s.N), dtype=torch.float64, device="cuda")
    lam = torch.empty((s.K,), dtype=torch.float64, device="cuda")
    cases = [("same contents", t0), ("t shifted by 3", t0 + 3.0), ("same again", t0 + 3.0),
             ("one sample off the integers (dense path)", t0 + np.where(np.arange(s.N) == 7, 0.25, 0.0)),
             ("the first contents", t0)]
    m2n.gpss_tapers(ctx, t, s.fmax, s.fw, s.K, out=(w, lam))
    for label, tv in cases:
        t.copy_(torch.from_numpy(tv))
        torch.cuda.synchronize()
        m2n.gpss_tapers(ctx, t, s.fmax, s.fw, s.K, out=(w, lam))
        torch.cuda.synchronize()
        c2 = m2n.Context(0)
        w2, lam2 = m2n.gpss_tapers(c2, t, s.fmax, s.fw, s.K)
        torch.cuda.synchronize()
        c2.close()
        _say(f"case gpss_tapers: {label}")
        assert torch.equal(w, w2) and torch.equal(lam, lam2), label
    bad = t0.copy()
    bad[[10, 11]] = bad[[11, 10]]
    t.copy_(torch.from_numpy(bad))
    torch.cuda.synchronize()
    with pytest.raises(m2n.M2NError) as ei:
        m2n.gpss_tapers(ctx, t, s.fmax, s.fw, s.K, out=(w, lam))
    assert ei.value.code == m2n.M2N_ERR_T_ORDER
