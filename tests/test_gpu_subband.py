"""One sub-band of the multiband partition on the GPU against the oracle
(Sec. 2.4 sub-band matrix; Sec. 3.1-3.2 nominal band at fc0, relative
eigencoefficients).

Tapers: lambda within 1e-12; the complex tapers, under the same phase reading
on both sides, within 1e-9 of the oracle's largest entry (the eigenvalue gaps
of these cases are >= 1e-3, so both eigen-solvers fix the vectors to near
rounding level).  Eigencoefficients and P: within 1e-10 (FP64 path) and 1e-5
(FP32 path) of the largest oracle value, as for the full band."""
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


def _say(msg):
    print(msg, flush=True)


def _tapers(m2n, ctx, t, fmin, fmax, fw, fc0, K):
    w, lam = m2n.gpss_tapers_subband(ctx, _dev(t), fmin, fmax, fw, fc0, K)
    torch.cuda.synchronize()
    return m2n.as_complex(w).cpu().numpy(), lam.cpu().numpy()


def _check_tapers(w, lam, wo, lo):
    el = np.abs(lam - lo).max()
    ew = np.abs(w - wo).max() / np.abs(wo).max()
    _say(f"  lambda err {el:.2e}  taper err {ew:.2e}")
    assert el < 1e-12 and ew < 1e-9


@pytest.mark.parametrize("n", [512, 1000])
def test_subband_tapers_multiband(m2n, ctx, orc, n):
    s, sbs = W.multiband(n=n)
    for sb in sbs:
        _say(f"subband tapers n={n} {sb}")
        w, lam = _tapers(m2n, ctx, s.t, sb.fmin, sb.fmax, s.fw, sb.fc0, s.K)
        wo, lo = orc.subband_tapers(s.t, sb.fmin, sb.fmax, s.fw, sb.fc0, s.K)
        _check_tapers(w, lam, wo, lo)


def test_subband_full_band_at_zero_is_gpss(m2n, ctx, orc):
    """f_min = 0, fc0 = 0: real tapers equal to the full-band entry point's."""
    s = W.scheme_jitter(n=300)
    fw = 2.5 / (s.t[-1] - s.t[0])
    _say("subband f_min=0 fc0=0 vs gpss_tapers, jitter n=300")
    w, lam = _tapers(m2n, ctx, s.t, 0.0, 0.5, fw, 0.0, 4)
    w0, l0 = m2n.gpss_tapers(ctx, _dev(s.t), 0.5, fw, 4)
    torch.cuda.synchronize()
    w0, l0 = w0.cpu().numpy(), l0.cpu().numpy()
    assert np.abs(w.imag).max() < 1e-12 * np.abs(w0).max()
    assert np.abs(w.real - w0).max() < 1e-9 * np.abs(w0).max()
    assert np.abs(lam - l0).max() < 1e-12
    wo, lo = orc.subband_tapers(s.t, 0.0, 0.5, fw, 0.0, 4)
    _check_tapers(w, lam, wo, lo)


@pytest.mark.parametrize("fc0", [0.2, -0.31])
def test_subband_lattice_modulated(m2n, ctx, orc, fc0):
    """Integer lattice with R(B) = I: modulated DPSS (oracle pin), through the
    dense sub-band path (a diagonal R(B) whose off-diagonal tiles are skipped)."""
    N = 640
    t = np.arange(N, dtype=np.float64)
    fw = 2.5 / N
    _say(f"subband lattice N={N} fc0={fc0}")
    w, lam = _tapers(m2n, ctx, t, 0.0, 0.5, fw, fc0, 4)
    wo, lo = orc.subband_tapers(t, 0.0, 0.5, fw, fc0, 4)
    _check_tapers(w, lam, wo, lo)


@pytest.mark.parametrize("prec,tol", [(2, 1e-10), (1, 1e-5)])
def test_subband_psd(m2n, ctx, orc, prec, tol):
    s, sbs = W.multiband(n=512, I=1024)
    for sb in sbs:
        _say(f"subband psd prec={prec} {sb}")
        wo, _ = orc.subband_tapers(s.t, sb.fmin, sb.fmax, s.fw, sb.fc0, s.K)
        wp = np.concatenate([wo.real, wo.imag])
        out = m2n.m2nufft_psd_subband(ctx, _dev(s.t), _dev(s.x), _dev(wp), s.f_lo, s.df, s.I,
                                      prec=prec, want_J=True)
        torch.cuda.synchronize()
        J = out["J"].cpu().numpy().astype(np.complex128)
        P = out["P"].cpu().numpy().astype(np.float64)
        Jo = orc.subband_eigcoeffs(s.t, s.x, wo, s.f_lo, s.df, s.I)
        Po = orc.psd(Jo)
        eJ = np.abs(J - Jo).max() / np.abs(Jo).max()
        eP = np.abs(P - Po).max() / Po.max()
        _say(f"  J err {eJ:.2e}  P err {eP:.2e}")
        assert eJ < tol and eP < tol


def test_subband_end_to_end_finds_both_lines(m2n, ctx, orc):
    """Both sub-bands from the GPU tapers: P agrees with the oracle's
    end-to-end result, and each sub-band's peak sits at its sinusoid
    (0.1 in [0, 1/4], 0.41 in [1/4, 1/2]) within the band half-width f_w
    (P integrates the spectrum over |f - f_c| <= f_w, flat across a line)."""
    s, sbs = W.multiband(n=768, I=2048)
    for sb, fline in zip(sbs, (0.1, 0.41)):
        _say(f"subband end-to-end {sb}")
        w, lam = m2n.gpss_tapers_subband(ctx, _dev(s.t), sb.fmin, sb.fmax, s.fw, sb.fc0, s.K)
        P = m2n.m2nufft_psd_subband(ctx, _dev(s.t), _dev(s.x), w, s.f_lo, s.df, s.I)["P"]
        P = P.cpu().numpy()
        wo, _ = orc.subband_tapers(s.t, sb.fmin, sb.fmax, s.fw, sb.fc0, s.K)
        Po = orc.psd(orc.subband_eigcoeffs(s.t, s.x, wo, s.f_lo, s.df, s.I))
        assert np.abs(P - Po).max() / Po.max() < 1e-9
        fpeak = sb.fc0 + s.f_lo + np.argmax(P) * s.df
        assert abs(fpeak - fline) <= s.fw


def test_subband_errors(m2n, ctx):
    t = np.arange(512, dtype=np.float64)
    with pytest.raises(m2n.M2NError) as ei:          # nominal band outside the sub-band
        m2n.gpss_tapers_subband(ctx, _dev(t), 0.25, 0.5, 0.01, 0.1, 4)
    assert ei.value.code == m2n.M2N_ERR_ARG
    with pytest.raises(m2n.M2NError) as ei:          # fmin >= fmax
        m2n.gpss_tapers_subband(ctx, _dev(t), 0.3, 0.3, 0.01, 0.3, 4)
    assert ei.value.code == m2n.M2N_ERR_ARG
    with pytest.raises(m2n.M2NError) as ei:          # K > 32
        m2n.gpss_tapers_subband(ctx, _dev(t), 0.0, 0.5, 0.01, 0.2, 33)
    assert ei.value.code == m2n.M2N_ERR_ARG
    with pytest.raises(m2n.M2NError) as ei:          # complex rank above 32
        m2n.gpss_tapers_subband(ctx, _dev(t), 0.0, 0.5, 6.0 / 512, 0.2, 4)
    assert ei.value.code == m2n.M2N_ERR_UNSUPPORTED
    _say("subband NOT_PD: integer lattice, sub-band [0.1, 0.2]")
    with pytest.raises(m2n.M2NError) as ei:          # oversampled: R(B^q) singular
        m2n.gpss_tapers_subband(ctx, _dev(t), 0.1, 0.2, 2.0 / 512, 0.15, 4)
    assert ei.value.code == m2n.M2N_ERR_NOT_PD
    with pytest.raises(m2n.M2NError) as ei:          # t not increasing
        m2n.gpss_tapers_subband(ctx, _dev(t[::-1].copy()), 0.0, 0.5, 0.01, 0.2, 4)
    assert ei.value.code == m2n.M2N_ERR_T_ORDER


def test_multiband_equals_single_calls(m2n, ctx):
    """All sub-bands at once (child contexts, own streams) give bitwise the
    one-sub-band results."""
    s, sbs = W.multiband(n=700)
    _say("multiband entry, two sub-bands, n=700")
    outs = m2n.gpss_tapers_multiband(ctx, _dev(s.t), [(b.fmin, b.fmax, b.fc0) for b in sbs], s.fw, s.K)
    torch.cuda.synchronize()
    for (w, lam), b in zip(outs, sbs):
        w1, l1 = m2n.gpss_tapers_subband(ctx, _dev(s.t), b.fmin, b.fmax, s.fw, b.fc0, s.K)
        torch.cuda.synchronize()
        assert torch.equal(w, w1) and torch.equal(lam, l1)


def test_multiband_error_names_the_subband(m2n, ctx):
    t = np.arange(512, dtype=np.float64)
    _say("multiband entry, second sub-band not positive definite")
    with pytest.raises(m2n.M2NError) as ei:
        m2n.gpss_tapers_multiband(ctx, _dev(t), [(0.0, 0.5, 0.2), (0.1, 0.2, 0.15)], 2.0 / 512, 4)
    assert ei.value.code == m2n.M2N_ERR_NOT_PD
    assert "sub-band 1" in str(ei.value)
