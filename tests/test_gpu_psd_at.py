"""Eigencoefficients and P at an arbitrary list of band centres on the GPU
(direct FP64 summation) against the oracle's direct sum: within 1e-11 of the
largest value; and against the NuFFT path at equally spaced centres within its
FP64 tolerance (1e-10)."""
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
    w = torch.zeros((17, s.N), dtype=torch.float64, device="cuda")
    with pytest.raises(m2n.M2NError) as ei:
        m2n.m2nufft_psd_at(ctx, _dev(s.t), _dev(s.x), w, _dev(np.zeros(4)))
    assert ei.value.code == m2n.M2N_ERR_ARG
