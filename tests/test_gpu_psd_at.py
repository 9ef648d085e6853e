"""Eigencoefficients and P at an arbitrary list of band centres on the GPU
against the oracle's direct sum: the direct FP64 summation within 1e-11 of the
largest value (also with more than 16 tapers), the type-3 NuFFT within 1e-10
(FP64) and 1e-5 (FP32) at a few hundred and at 2^17 centres; both against the
type-1 NuFFT path at equally spaced centres (1e-10)."""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("name,nf", [("small_gapped", 300), ("jitter", 1000), ("arithmetic", 77)])
def test_psd_at_random_centres(m2n, ctx, orc, name, nf):
    s = W.by_name(name) if name != "jitter" else W.scheme_jitter(n=700)
    K = 4
    w, _ = orc.gpss_tapers(s.t, s.fmax, s.fw, K, method="jacobi") if s.N <= 600 else \
        orc.gpss_tapers(s.t, s.fmax, s.fw, K)
    rng = np.random.default_rng(nf)
    freqs = rng.uniform(-0.5, 0.5, nf)
    freqs[:5] = freqs[5:10]                     # repeats
    print(f"psd_at {name} N={s.N} I={nf}", flush=True)
    out = m2n.m2nufft_psd_at(ctx, _dev(s.t), _dev(s.x), _dev(w), _dev(freqs), want_J=True)
    J = out["J"].cpu().numpy()
    P = out["P"].cpu().numpy()
    Jo = orc.nudft_freqs(s.t, s.x, w, freqs)
    Po = orc.psd(Jo)
    assert np.abs(J - Jo).max() < 1e-11 * np.abs(Jo).max()
    assert np.abs(P - Po).max() < 1e-11 * Po.max()


def test_psd_at_equals_nufft_on_a_progression(m2n, ctx):
    s = W.small_gapped()
    t, x = _dev(s.t), _dev(s.x)
    w, lam = m2n.gpss_tapers(ctx, t, s.fmax, s.fw, s.K)
    ref = m2n.m2nufft_psd(ctx, t, x, w, lam, s.fmax, s.fw, s.f_lo, s.df, s.I, prec=m2n.M2N_FP64, want_E=False)
    freqs = s.f_lo + s.df * np.arange(s.I)
    out = m2n.m2nufft_psd_at(ctx, t, x, w, _dev(freqs))
    P, Pr = out["P"].cpu().numpy(), ref["P"].cpu().numpy()
    assert np.abs(P - Pr).max() < 1e-10 * Pr.max()


def test_psd_at_errors(m2n, ctx):
    s = W.small_gapped()
    w = torch.zeros((65, s.N), dtype=torch.float64, device="cuda")
    with pytest.raises(m2n.M2NError) as ei:
        m2n.m2nufft_psd_at(ctx, _dev(s.t), _dev(s.x), w, _dev(np.zeros(4)))
    assert ei.value.code == m2n.M2N_ERR_ARG


@pytest.mark.parametrize("name,nf", [("small_gapped", 300), ("jitter", 1000), ("arithmetic", 77)])
@pytest.mark.parametrize("prec,tol", [(2, 1e-10), (1, 1e-5)])
def test_psd_freqs_type3_random_centres(m2n, ctx, orc, name, nf, prec, tol):
    # the type-3 NuFFT against the oracle's direct sum at random centres
    # (negative, repeated), both precisions, within tol of the largest value
    s = W.by_name(name) if name != "jitter" else W.scheme_jitter(n=700)
    K = 4
    w, _ = orc.gpss_tapers(s.t, s.fmax, s.fw, K, method="jacobi") if s.N <= 600 else \
        orc.gpss_tapers(s.t, s.fmax, s.fw, K)
    rng = np.random.default_rng(nf + 5)
    freqs = rng.uniform(-0.5, 0.5, nf)
    freqs[:5] = freqs[5:10]
    print(f"psd_freqs {name} N={s.N} I={nf} prec={prec}", flush=True)
    out = m2n.m2nufft_psd_freqs(ctx, _dev(s.t), _dev(s.x), _dev(w), _dev(freqs), prec=prec, want_J=True)
    J = out["J"].cpu().numpy().astype(np.complex128)
    P = out["P"].cpu().numpy().astype(np.float64)
    Jo = orc.nudft_freqs(s.t, s.x, w, freqs)
    Po = orc.psd(Jo)
    eJ = np.abs(J - Jo).max() / np.abs(Jo).max()
    eP = np.abs(P - Po).max() / Po.max()
    print(f"  J {eJ:.2e}  P {eP:.2e}", flush=True)
    assert eJ < tol and eP < tol


def test_psd_freqs_many_centres_sampled(m2n, ctx, orc):
    # 2^17 random centres on the 20,480-sample gapped series with its GPU
    # tapers; the oracle's direct sum on 512 of them
    s = W.gapped_20k()
    t, x = _dev(s.t), _dev(s.x)
    w, lam = m2n.gpss_tapers(ctx, t, s.fmax, s.fw, s.K)
    freqs = np.random.default_rng(17).uniform(-0.5, 0.5, 2 ** 17)
    pick = np.random.default_rng(18).choice(freqs.shape[0], 512, replace=False)
    wn = w.cpu().numpy()
    Jo = orc.nudft_freqs(s.t, s.x, wn, freqs[pick])
    Po = orc.psd(Jo)
    for prec, tol in ((2, 1e-10), (1, 1e-5)):
        out = m2n.m2nufft_psd_freqs(ctx, t, x, w, _dev(freqs), prec=prec, want_J=True)
        J = out["J"].cpu().numpy().astype(np.complex128)[:, pick]
        P = out["P"].cpu().numpy().astype(np.float64)[pick]
        eJ = np.abs(J - Jo).max() / np.abs(Jo).max()
        eP = np.abs(P - Po).max() / Po.max()
        print(f"psd_freqs 2^17 centres prec={prec}: J {eJ:.2e}  P {eP:.2e}", flush=True)
        assert eJ < tol and eP < tol


def test_psd_freqs_equals_nufft_and_any_sample_order(m2n, ctx):
    # on an arithmetic progression of centres the type-3 path equals the
    # type-1 path; shuffling the samples changes nothing
    s = W.small_gapped()
    t, x = _dev(s.t), _dev(s.x)
    w, lam = m2n.gpss_tapers(ctx, t, s.fmax, s.fw, s.K)
    ref = m2n.m2nufft_psd(ctx, t, x, w, lam, s.fmax, s.fw, s.f_lo, s.df, s.I, prec=m2n.M2N_FP64, want_E=False)
    freqs = _dev(s.f_lo + s.df * np.arange(s.I))
    P = m2n.m2nufft_psd_freqs(ctx, t, x, w, freqs)["P"].cpu().numpy()
    Pr = ref["P"].cpu().numpy()
    assert np.abs(P - Pr).max() < 1e-10 * Pr.max()
    perm = torch.from_numpy(np.random.default_rng(3).permutation(s.N)).cuda()
    P2 = m2n.m2nufft_psd_freqs(ctx, t[perm], x[perm], w[:, perm].contiguous(), freqs)["P"].cpu().numpy()
    assert np.abs(P2 - Pr).max() < 1e-10 * Pr.max()


def test_psd_at_more_than_16_tapers(m2n, ctx, orc):
    # the direct sum in groups of 16 tapers (K = 20), against the oracle
    s = W.scheme_jitter(n=400)
    w = np.random.default_rng(19).standard_normal((20, s.N)) * 0.05
    freqs = np.random.default_rng(20).uniform(-0.5, 0.5, 333)
    out = m2n.m2nufft_psd_at(ctx, _dev(s.t), _dev(s.x), _dev(w), _dev(freqs), want_J=True)
    Jo = orc.nudft_freqs(s.t, s.x, w, freqs)
    assert np.abs(out["J"].cpu().numpy() - Jo).max() < 1e-11 * np.abs(Jo).max()
    Po = orc.psd(Jo)
    assert np.abs(out["P"].cpu().numpy() - Po).max() < 1e-11 * Po.max()
