"""Replayable batches (m2n_batch_create / launch): the batched form captured
into a HIP graph, with and without the NuFFT schedule autotuner, against
m2n_batch_psd on the same series.  Tapers and eigenvalues bitwise; P and Ehat
within the NuFFT tolerance (the tuner may choose another grid split, which
changes only the rounding).  The graph is replayed several times with the
program's own eager work and synchronisations between replays, every replay
checked; x is changed between launches (new data on the same sampling); the
tuner's choice is read back from its file by a second batch of the same size
class; a series off the lattice path is refused."""
import os

import numpy as np
import pytest

import workloads as W
from tests.metrics import psd_err

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


def _specs(series):
    return [{"t": _dev(s.t), "x": _dev(s.x), "fmax": s.fmax, "fw": s.fw, "K": s.K, "f_lo": s.f_lo,
             "df": s.df, "I": s.I, "want_E": True} for s in series]


def _reference(m2n, ctx, specs, prec):
    ref = m2n.m2n_batch_psd(ctx, [dict(sp) for sp in specs], prec=prec)
    torch.cuda.synchronize()
    return [{k: (v.clone() if v is not None else None) for k, v in o.items()} for o in ref]


def _check(outs, ref, tol):
    worst = 0.0
    for o, r in zip(outs, ref):
        assert torch.equal(o["w"], r["w"]) and torch.equal(o["lam"], r["lam"])
        worst = max(worst, psd_err(o["P"].double().cpu().numpy(), r["P"].double().cpu().numpy()))
        assert torch.allclose(o["E"].double(), r["E"].double(), rtol=0, atol=tol)
    assert worst < tol
    return worst


@pytest.mark.parametrize("prec,tune", [(1, True), (1, False), (2, False)])
def test_graph_replays_match_batch(m2n, ctx, tmp_path, prec, tune):
    os.environ["M2N_TUNE_CACHE"] = str(tmp_path / "schedules.txt")
    series = [W.batched_series(s) for s in range(12)] + [W.small_gapped()]
    specs = _specs(series)
    tol = 2e-6 if prec == 1 else 1e-12
    ref = _reference(m2n, ctx, specs, prec)
    _say(f"graph batch prec={prec} tune={tune}: {len(series)} series, N {[s.N for s in series]}")
    b = m2n.Batch(ctx, specs, prec=prec, graph=True, tune=tune)
    info = b.info()
    _say(f"  info {info}")
    assert info["graph"] == 1 and info["graph_nodes"] > 0 and info["band_counts"] == 2
    assert info["tuned"] == (1 if tune else 0)
    torch.cuda.synchronize()
    _check(b.outputs, ref, tol)              # the warm-up pass
    for rep in range(4):
        for o in b.outputs:                  # eager work between replays
            o["P"].zero_()
            o["w"].zero_()
        torch.cuda.synchronize()
        outs = b.launch()
        torch.cuda.synchronize()
        worst = _check(outs, ref, tol)
        _say(f"  replay {rep}: P max rel {worst:.2e}")
    b.close()


def test_graph_new_data_between_launches(m2n, ctx):
    series = [W.batched_series(s) for s in range(6)]
    specs = _specs(series)
    b = m2n.Batch(ctx, specs, prec=m2n.M2N_FP32, graph=True)
    for k in range(3):
        rng = np.random.default_rng(900 + k)
        for sp in specs:
            sp["x"].copy_(torch.from_numpy(rng.standard_normal(sp["x"].shape[0])))
        torch.cuda.synchronize()
        outs = b.launch()
        torch.cuda.synchronize()
        ref = _reference(m2n, ctx, specs, m2n.M2N_FP32)
        worst = _check(outs, ref, 2e-6)
        _say(f"  new data {k}: P max rel {worst:.2e}")
    b.close()


def test_tuner_choice_read_back_from_file(m2n, ctx, tmp_path):
    path = tmp_path / "schedules.txt"
    os.environ["M2N_TUNE_CACHE"] = str(path)
    specs = _specs([W.batched_series(s) for s in range(8)])
    b1 = m2n.Batch(ctx, specs, graph=False, tune=True)
    i1 = b1.info()
    b1.close()
    assert i1["tuned"] == 1 and i1["from_cache"] == 0 and i1["candidates"] >= 2
    assert i1["nufft_ms_tuned"] <= i1["nufft_ms_default"]
    assert path.exists() and " -> " in path.read_text()
    b2 = m2n.Batch(ctx, specs, graph=True, tune=True)
    i2 = b2.info()
    _say(f"  tuned {i1}; from file {i2}")
    assert i2["from_cache"] == 1 and (i2["l1"], i2["B"], i2["M"]) == (i1["l1"], i1["B"], i1["M"])
    ref = _reference(m2n, ctx, specs, m2n.M2N_FP32)
    _check(b2.launch(), ref, 2e-6)
    b2.close()


def test_batch_refuses_series_off_the_lattice_path(m2n, ctx):
    specs = _specs([W.small_gapped(), W.jitter_stress(n=300, seed=3, K=4, I=512)])
    with pytest.raises(m2n.M2NError) as ei:
        m2n.Batch(ctx, specs)
    assert ei.value.code == m2n.M2N_ERR_UNSUPPORTED
    assert "series 1" in str(ei.value)


def test_graph_launch_in_sync_mode(m2n, ctx, monkeypatch):
    # a batch made from a context in synchronous mode: each launch waits and
    # returns the device-side error its kernels flagged (a non-finite sample
    # written into x between launches), and launches cleanly once it is gone
    monkeypatch.setenv("M2N_SYNC", "1")
    sctx = m2n.Context(0)
    monkeypatch.delenv("M2N_SYNC")
    try:
        series = [W.batched_series(s) for s in range(120, 124)]
        specs = _specs(series)
        ref = _reference(m2n, ctx, specs, m2n.M2N_FP32)
        b = m2n.Batch(sctx, specs, prec=m2n.M2N_FP32, graph=True)
        _check(b.launch(), ref, 2e-6)
        x0 = specs[2]["x"][7].item()
        specs[2]["x"][7] = float("nan")
        torch.cuda.synchronize()
        with pytest.raises(m2n.M2NError) as ei:
            b.launch()
        assert ei.value.code == m2n.M2N_ERR_ARG
        specs[2]["x"][7] = x0
        torch.cuda.synchronize()
        _check(b.launch(), ref, 2e-6)
        _say("case graph batch in sync mode: the flagged launch returned M2N_ERR_ARG, the next one clean")
        b.close()
    finally:
        sctx.close()
