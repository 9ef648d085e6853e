"""Interpolated-DPSS tapers (Table 3 step 3 for fc0 = 0) on the GPU against the
oracle.  The GPU takes the DPSS from its lattice GEP path, the spline second
derivatives from an exact recursive-filter form, and the R(B) scale from
2 f_max sum w^2 on lattices or an O(N^2) quadratic form elsewhere; the oracle
takes scipy's DPSS and cubic spline and a dense R(B).  Bar: lambda within
1e-12, tapers within 1e-9 of the oracle's largest entry (NW <= 3.5, so the
DPSS eigenvalue gaps fix the vectors to near rounding level: every case uses
NW = f_w (t_N - t_1) = 2.5 to 3 and K = 4); P end to end within 1e-10 (FP64
path)."""
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


def _case(m2n, ctx, orc, t, fmax, fw, K):
    w, lam = m2n.idpss_tapers(ctx, _dev(t), fmax, fw, K)
    torch.cuda.synchronize()
    w, lam = w.cpu().numpy(), lam.cpu().numpy()
    wo, lo = orc.idpss_tapers(t, fmax, fw, K)
    el = np.abs(lam - lo).max()
    ew = np.abs(w - wo).max() / np.abs(wo).max()
    _say(f"  lambda err {el:.2e}  taper err {ew:.2e}")
    assert el < 1e-12 and ew < 1e-9
    return w, lam


def test_idpss_uniform_grid_is_gpss(m2n, ctx, orc):
    t = 3.0 + 1.5 * np.arange(640)
    fmax, fw, K = 1.0 / 3.0, 2.5 / (639 * 1.5), 4
    _say("idpss uniform grid N=640 h=1.5")
    w, lam = _case(m2n, ctx, orc, t, fmax, fw, K)
    w0, l0 = m2n.gpss_tapers(ctx, _dev(t), fmax, fw, K)
    torch.cuda.synchronize()
    assert np.abs(lam - l0.cpu().numpy()).max() < 1e-12
    assert np.abs(w - w0.cpu().numpy()).max() < 1e-9 * np.abs(w).max()


@pytest.mark.parametrize("name", ["small_gapped", "missing"])
def test_idpss_gapped(m2n, ctx, orc, name):
    s = W.by_name(name)
    _say(f"idpss {name} N={s.N}")
    _case(m2n, ctx, orc, s.t, s.fmax, 2.5 / (s.t[-1] - s.t[0]), 4)


@pytest.mark.parametrize("n", [300, 1000, 2100])
def test_idpss_jittered_quadratic_form(m2n, ctx, orc, n):
    s = W.scheme_jitter(n=n, sigma=0.1)
    fw = 2.5 / (s.t[-1] - s.t[0])
    _say(f"idpss jittered N={n}")
    _case(m2n, ctx, orc, s.t, 0.5, fw, 4)


def test_idpss_gapped_grid_spans_tiles(m2n, ctx, orc):
    """A gapped unit grid with 2,600 samples (lattice scale, several tiles of
    the spline and evaluation kernels and a ragged tail)."""
    s = W.gapped_scaled(3264, 5, 4096)
    _say(f"idpss gapped_scaled N={s.N}")
    _case(m2n, ctx, orc, s.t, s.fmax, 2.5 / (s.t[-1] - s.t[0]), 4)


def test_idpss_end_to_end_psd(m2n, ctx, orc):
    s = W.small_gapped()
    K = 4
    fw = 2.5 / (s.t[-1] - s.t[0])
    _say("idpss end to end small_gapped")
    w, lam = m2n.idpss_tapers(ctx, _dev(s.t), s.fmax, fw, K)
    out = m2n.m2nufft_psd(ctx, _dev(s.t), _dev(s.x), w, lam, s.fmax, fw, s.f_lo, s.df, s.I,
                          prec=m2n.M2N_FP64, want_E=False)
    P = out["P"].cpu().numpy()
    wo, _ = orc.idpss_tapers(s.t, s.fmax, fw, K)
    Po = orc.psd(orc.nudft(s.t, s.x, wo, s.f_lo, s.df, s.I))
    assert np.abs(P - Po).max() / Po.max() < 1e-10


def test_idpss_errors(m2n, ctx):
    t = np.arange(64, dtype=np.float64)
    for args in [(t[:1], 0.5, 0.01, 1), (t, 0.5, 0.01, 33), (t, 0.5, 0.6, 2), (2.0 * t, 1.0, 0.3, 2)]:
        with pytest.raises(m2n.M2NError) as ei:
            m2n.idpss_tapers(ctx, _dev(args[0]), *args[1:])
        assert ei.value.code == m2n.M2N_ERR_ARG
    with pytest.raises(m2n.M2NError) as ei:
        m2n.idpss_tapers(ctx, _dev(t[::-1].copy()), 0.5, 0.01, 2)
    assert ei.value.code == m2n.M2N_ERR_T_ORDER


def test_idpss_with_ftest(m2n, ctx, orc):
    """Interpolated tapers are real, so the F-statistic of the full-band path
    applies; its coherence gamma = F / (F + K - 1) against the oracle's."""
    s = W.small_gapped()
    K = 4
    fw = 2.5 / (s.t[-1] - s.t[0])
    _say("idpss with F-test, small_gapped")
    w, lam = m2n.idpss_tapers(ctx, _dev(s.t), s.fmax, fw, K)
    out = m2n.m2nufft_psd(ctx, _dev(s.t), _dev(s.x), w, lam, s.fmax, fw, s.f_lo, s.df, s.I,
                          prec=m2n.M2N_FP64, want_E=False, want_F=True)
    F = out["F"].cpu().numpy()
    wo, _ = orc.idpss_tapers(s.t, s.fmax, fw, K)
    Fo, _ = orc.ftest(orc.nudft(s.t, s.x, wo, s.f_lo, s.df, s.I), wo)
    g = np.where(np.isinf(F), 1.0, F / (F + K - 1))
    go = np.where(np.isinf(Fo), 1.0, Fo / (Fo + K - 1))
    assert np.abs(g - go).max() < 1e-10
