"""Served form: requests through the m2n_queue (continuous batching) give the
same tapers bit for bit, and P / Ehat within the NuFFT tolerance, as the
same series alone; a failing request does not fail the others; a tiny HBM
budget serialises the batches."""
import threading

import numpy as np
import pytest

import workloads as W

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


def _say(msg):
    print(msg, flush=True)


def _alone(m2n, ctx, s, prec):
    dev = torch.device("cuda:0")
    t = torch.from_numpy(s.t).to(dev)
    x = torch.from_numpy(s.x).to(dev)
    w, lam = m2n.gpss_tapers(ctx, t, s.fmax, s.fw, s.K)
    out = m2n.m2nufft_psd(ctx, t, x, w, lam, s.fmax, s.fw, s.f_lo, s.df, s.I, prec=prec)
    return w.cpu().numpy(), lam.cpu().numpy(), out["P"].cpu().numpy(), out["E"].cpu().numpy()


def _submit(q, s):
    return q.submit(s.t, s.x, s.fmax, s.fw, s.K, s.f_lo, s.df, s.I)


WAIT_US = 60_000_000   # a request not done within a minute fails the test


def _wait(q, ticket):
    r = q.wait(ticket, timeout_us=WAIT_US)
    assert r is not None, f"ticket {ticket} not done within {WAIT_US / 1e6:.0f} s"
    return r


def _check(m2n, ctx, s, r, prec):
    w, lam, P, E = _alone(m2n, ctx, s, prec)
    assert r["status"] == m2n.M2N_OK
    assert np.array_equal(r["w"], w) and np.array_equal(r["lam"], lam)
    dP = float(np.max(np.abs(r["P"].astype(np.float64) - P)) / np.max(np.abs(P)))
    assert dP < 2e-6, dP
    assert np.max(np.abs(r["E"].astype(np.float64) - E)) < 1e-7
    return dP


def test_queue_same_alone_and_in_mix(m2n, ctx):
    series = [W.batched_series(s) for s in range(24)]
    q = m2n.Queue(ctx, slots=2, prec=m2n.M2N_FP32)
    tickets = {}
    # two submitting threads: the mix depends on timing, the results must not
    def sub(part):
        for i in part:
            tickets[i] = _submit(q, series[i])
    th = threading.Thread(target=sub, args=(range(0, 24, 2),))
    th.start()
    sub(range(1, 24, 2))
    th.join()
    res = {i: _wait(q, tk) for i, tk in tickets.items()}
    sizes = sorted(r["batch_size"] for r in res.values())
    _say(f"case 24 requests, batch sizes seen {sizes[0]}..{sizes[-1]}")
    assert sizes[-1] > 1
    worst = max(_check(m2n, ctx, series[i], res[i], m2n.M2N_FP32) for i in res)
    _say(f"  worst P difference alone vs in the mix {worst:.2e}")
    q.close()


def test_queue_fp64(m2n, ctx):
    # the FP64 queue: the same tapers bit for bit, and P and Ehat within the
    # FP64 NuFFT tolerance, as the series alone
    series = [W.batched_series(s) for s in range(110, 118)]
    q = m2n.Queue(ctx, slots=2, prec=m2n.M2N_FP64)
    tk = [_submit(q, s) for s in series]
    res = [_wait(q, t) for t in tk]
    worst = 0.0
    for s, r in zip(series, res):
        w, lam, P, E = _alone(m2n, ctx, s, m2n.M2N_FP64)
        assert r["status"] == m2n.M2N_OK and r["P"].dtype == np.float64
        assert np.array_equal(r["w"], w) and np.array_equal(r["lam"], lam)
        dP = float(np.max(np.abs(r["P"] - P)) / np.max(np.abs(P)))
        assert dP < 1e-11, dP
        assert np.max(np.abs(r["E"] - E)) < 1e-12
        worst = max(worst, dP)
    _say(f"case FP64 queue: 8 requests, batch sizes {sorted(r['batch_size'] for r in res)}, worst P {worst:.2e}")
    q.close()


def test_queue_pinned_outputs(m2n, ctx):
    # results copied from the device straight into pinned host buffers: the
    # same as alone; requests without tapers leave w out
    series = [W.batched_series(s) for s in range(60, 76)]
    q = m2n.Queue(ctx, slots=2, prec=m2n.M2N_FP32, pinned_outputs=True)
    tk = [q.submit(s.t, s.x, s.fmax, s.fw, s.K, s.f_lo, s.df, s.I, want_w=(i % 2 == 0))
          for i, s in enumerate(series)]
    res = [_wait(q, t) for t in tk]
    worst = 0.0
    for i, (s, r) in enumerate(zip(series, res)):
        if i % 2 == 0:
            worst = max(worst, _check(m2n, ctx, s, r, m2n.M2N_FP32))
        else:
            assert r["w"] is None
            w, lam, P, E = _alone(m2n, ctx, s, m2n.M2N_FP32)
            assert np.array_equal(r["lam"], lam)
            assert float(np.max(np.abs(r["P"].astype(np.float64) - P)) / np.max(np.abs(P))) < 2e-6
    _say(f"case pinned outputs: 16 requests, batch sizes {sorted(r['batch_size'] for r in res)}, "
         f"worst P {worst:.2e}")
    q.close()


@pytest.mark.parametrize("borrow", [False, True])
def test_queue_pinned_pool_merged_copies(m2n, ctx, borrow):
    # outputs as back-to-back views of one pinned pool (P, E of each request
    # in turn; eigenvalues and tapers in pools of their own), so that the
    # copies of a batch merge; requests without E, without tapers and one
    # band count whose P is not a multiple of 256 bytes break the runs; the
    # inputs copied at submit or borrowed until the results are collected
    series = [W.batched_series(s) for s in range(80, 92)]
    series[5].I = 1000
    want_E = [i % 4 != 3 for i in range(len(series))]
    want_w = [i % 3 == 0 for i in range(len(series))]
    pin = dict(pin_memory=True)
    pe = torch.empty(sum((2 if e else 1) * s.I for s, e in zip(series, want_E)), dtype=torch.float32, **pin)
    lp = torch.empty(sum(s.K for s in series), dtype=torch.float64, **pin)
    wp = torch.empty(sum(s.K * s.N for s, f in zip(series, want_w) if f), dtype=torch.float64, **pin)
    pe, lp, wp = pe.numpy(), lp.numpy(), wp.numpy()
    outs, o, ol, ow = [], 0, 0, 0
    for s, e, f in zip(series, want_E, want_w):
        ob = {"P": pe[o:o + s.I], "E": None, "lam": lp[ol:ol + s.K], "w": None}
        o += s.I
        if e:
            ob["E"] = pe[o:o + s.I]
            o += s.I
        if f:
            ob["w"] = wp[ow:ow + s.K * s.N].reshape(s.K, s.N)
            ow += s.K * s.N
        ol += s.K
        outs.append(ob)
    q = m2n.Queue(ctx, slots=1, prec=m2n.M2N_FP32, pinned_outputs=True, borrow_inputs=borrow)
    # fresh copies of t and x, referenced by nothing but the queue object:
    # a borrowed input must be kept alive by it until its result is taken
    tk = [q.submit(s.t.copy(), s.x.copy(), s.fmax, s.fw, s.K, s.f_lo, s.df, s.I, out=ob)
          for s, ob in zip(series, outs)]
    res = [_wait(q, t) for t in tk]
    worst = 0.0
    for i, (s, r) in enumerate(zip(series, res)):
        assert r["status"] == m2n.M2N_OK and "_inputs" not in r
        w, lam, P, E = _alone(m2n, ctx, s, m2n.M2N_FP32)
        assert np.array_equal(r["lam"], lam), i
        if want_w[i]:
            assert np.array_equal(r["w"], w), i
        dP = float(np.max(np.abs(r["P"].astype(np.float64) - P)) / np.max(np.abs(P)))
        assert dP < 2e-6, (i, dP)
        worst = max(worst, dP)
        if want_E[i]:
            assert np.max(np.abs(r["E"].astype(np.float64) - E)) < 1e-7, i
    _say(f"case pinned pool (borrowed inputs {borrow}): 12 requests, batch sizes {sorted(r['batch_size'] for r in res)}, "
         f"worst P {worst:.2e}")
    q.close()


@pytest.mark.parametrize("borrow", [False, True])
def test_queue_failing_request_is_isolated(m2n, ctx, borrow):
    # the batch holding the bad request fails and is rerun one request at a
    # time (with borrowed inputs, from the callers' arrays again)
    good = [W.batched_series(s) for s in (30, 31, 32)]
    bad = W.batched_series(33)
    bad.x = bad.x.copy()
    bad.x[5] = np.nan
    q = m2n.Queue(ctx, slots=1, prec=m2n.M2N_FP32, borrow_inputs=borrow)
    tk = [_submit(q, s) for s in good[:2]] + [_submit(q, bad)] + [_submit(q, good[2])]
    out = []
    for t in tk:
        try:
            out.append(_wait(q, t))
        except m2n.M2NError as e:
            out.append(e.code)
    assert out[2] == m2n.M2N_ERR_ARG
    for s, r in zip(good, [out[0], out[1], out[3]]):
        _check(m2n, ctx, s, r, m2n.M2N_FP32)
    q.close()


def test_queue_budget_serialises(m2n, ctx):
    series = [W.batched_series(s) for s in (40, 41, 42)]
    q = m2n.Queue(ctx, hbm_budget_bytes=1, slots=2, prec=m2n.M2N_FP32)
    tk = [_submit(q, s) for s in series]
    res = [_wait(q, t) for t in tk]
    assert all(r["batch_size"] == 1 for r in res)
    for s, r in zip(series, res):
        _check(m2n, ctx, s, r, m2n.M2N_FP32)
    q.close()


def test_queue_destroy_with_pending_requests(m2n, ctx):
    q = m2n.Queue(ctx, slots=1, prec=m2n.M2N_FP32)
    for s in range(6):
        _submit(q, W.batched_series(50 + s))
    q.close()   # pending ones are cancelled, running batches complete
