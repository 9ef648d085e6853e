"""Edge cases of the GPU path against the oracle and closed forms: a single
sample and two samples (closed forms of the 1x1 and 2x2 GEPs), one taper,
ragged band counts on both NuFFT paths, arbitrary band grids (f_lo, df not
tied to I), an all-zero signal, and the largest band count of the build
(I = 2^21, sampled bands)."""
import math

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


def test_single_sample_closed_form(m2n, ctx):
    # N = 1: R(B) = 2 f_max, R(A0) = 2 f_w, so lambda = f_w / f_max,
    # w = sqrt(f_w / f_max) (w^T R(B) w = 2 f_w, positive sum) and
    # P = (f_w / f_max) x^2 in every band
    fmax, fw, x0 = 0.5, 0.1, -1.75
    _say("case N=1 K=1")
    t = _dev(np.array([3.0]))
    w, lam = m2n.gpss_tapers(ctx, t, fmax, fw, 1)
    assert abs(float(lam[0]) - fw / fmax) < 1e-14
    assert abs(float(w[0, 0]) - math.sqrt(fw / fmax)) < 1e-14
    # within the gates of the two modes (1e-10 FP64, 1e-5 FP32)
    for prec, tol in ((m2n.M2N_FP64, 1e-10), (m2n.M2N_FP32, 1e-5)):
        out = m2n.m2nufft_psd(ctx, t, _dev(np.array([x0])), w, lam, fmax, fw, -0.5, 1.0 / 64, 64,
                              prec=prec)
        P = out["P"].cpu().numpy().astype(np.float64)
        assert np.abs(P - fw / fmax * x0 * x0).max() < tol * fw / fmax * x0 * x0


def test_two_samples_closed_form(m2n, ctx, orc):
    # N = 2 with equal diagonals: eigenvectors [1, 1] and [1, -1],
    # lambda_pm = (2 f_w + s_A) / (2 f_max + s_B) with the off-diagonals s
    fmax, fw, tau = 0.5, 0.15, 1.3
    _say("case N=2 K=2")
    tt = np.array([0.0, tau])
    sA = math.sin(2 * math.pi * fw * tau) / (math.pi * tau)
    sB = math.sin(2 * math.pi * fmax * tau) / (math.pi * tau)
    lam_p, lam_m = (2 * fw + sA) / (2 * fmax + sB), (2 * fw - sA) / (2 * fmax - sB)
    w, lam = m2n.gpss_tapers(ctx, _dev(tt), fmax, fw, 2)
    w, lam = w.cpu().numpy(), lam.cpu().numpy()
    assert np.abs(np.sort(lam)[::-1] - np.sort([lam_p, lam_m])[::-1]).max() < 1e-13
    for k in range(2):
        v = w[k]
        # each taper is proportional to [1, 1] or [1, -1] and R(B)-normalised
        assert min(abs(v[0] - v[1]), abs(v[0] + v[1])) < 1e-12 * abs(v[0])
    w_o, lam_o = orc.gpss_tapers(tt, fmax, fw, 2)
    assert np.abs(lam - lam_o).max() < 1e-13
    assert normwise_rows(align_signs(w, w_o)[0], w_o) < 1e-12


def test_one_taper(m2n, ctx, orc):
    s = W.gapped_scaled(3000, 1, 2 ** 13, seed=41)
    _say(f"case K=1 N={s.N}")
    t = _dev(s.t)
    w, lam = m2n.gpss_tapers(ctx, t, s.fmax, s.fw, 1)
    w_o, lam_o = orc.gpss_tapers(s.t, s.fmax, s.fw, 1, method="lanczos")
    assert abs(float(lam[0]) - lam_o[0]) < 1e-12
    assert normwise_rows(w.cpu().numpy(), w_o) < 1e-10
    out = m2n.m2nufft_psd(ctx, t, _dev(s.x), w, lam, s.fmax, s.fw, s.f_lo, s.df, s.I, prec=m2n.M2N_FP64)
    P_o = orc.psd(orc.nudft(s.t, s.x, w_o, s.f_lo, s.df, I=s.I))
    assert psd_err(out["P"].cpu().numpy(), P_o) < 1e-10


@pytest.mark.parametrize("I", [1, 3, 1000, 8193, 20000])
def test_ragged_band_counts(m2n, ctx, orc, I):
    # band counts that are not powers of two, on the single-workgroup path
    # (n_f <= 8192) and the two-pass path (I = 8193, 20000)
    s = W.small_gapped()
    w = np.random.default_rng(200 + I).standard_normal((3, s.N)) * 0.1
    df = 1.0 / max(I, 2)
    _say(f"case ragged I={I}")
    J_o = orc.nudft(s.t, s.x, w, -0.5, df, I=I)
    for prec, tol in ((m2n.M2N_FP64, 1e-10), (m2n.M2N_FP32, 1e-5)):
        out = m2n.m2nufft_psd(ctx, _dev(s.t), _dev(s.x), _dev(w), None, s.fmax, s.fw, -0.5, df, I,
                              prec=prec, want_E=False, want_J=True)
        J = out["J"].cpu().numpy().astype(np.complex128)
        assert J.shape == (3, I)
        assert normwise_rows(J, J_o) < tol
        assert psd_err(out["P"].cpu().numpy().astype(np.float64), orc.psd(J_o)) < tol


@pytest.mark.parametrize("f_lo,df_scale", [(0.1, 1.0 / 3.0), (-0.37, 2.5), (0.0, 1.0)])
def test_arbitrary_band_grid(m2n, ctx, orc, f_lo, df_scale):
    s = W.gapped_scaled(3000, 4, 2 ** 13, seed=43)
    I = s.I
    df = df_scale / I
    w = np.random.default_rng(300).standard_normal((4, s.N)) * 0.05
    _say(f"case band grid f_lo={f_lo} df={df:.3e}")
    J_o = orc.nudft(s.t, s.x, w, f_lo, df, I=I)
    for prec, tol in ((m2n.M2N_FP64, 1e-10), (m2n.M2N_FP32, 1e-5)):
        out = m2n.m2nufft_psd(ctx, _dev(s.t), _dev(s.x), _dev(w), None, s.fmax, s.fw, f_lo, df, I,
                              prec=prec, want_E=False, want_J=True)
        J = out["J"].cpu().numpy().astype(np.complex128)
        assert normwise_rows(J, J_o) < tol


def test_zero_signal(m2n, ctx):
    s = W.gapped_scaled(3000, 4, 2 ** 13, seed=44)
    _say("case zero signal")
    t = _dev(s.t)
    w, lam = m2n.gpss_tapers(ctx, t, s.fmax, s.fw, s.K)
    for prec in (m2n.M2N_FP64, m2n.M2N_FP32):
        out = m2n.m2nufft_psd(ctx, t, _dev(np.zeros(s.N)), w, lam, s.fmax, s.fw, s.f_lo, s.df, s.I,
                              prec=prec, want_J=True)
        assert float(out["P"].abs().max()) == 0.0
        assert float(out["J"].abs().max()) == 0.0


def test_largest_band_count_sampled(m2n, ctx, orc):
    # I = 2^21 (n_f = 2^22, the largest split of this build), sampled bands
    s = W.gapped_scaled(6000, 3, 2 ** 21, seed=45)
    w = np.random.default_rng(301).standard_normal((3, s.N)) * 0.05
    _say(f"case I=2^21 N={s.N}")
    out64 = m2n.m2nufft_psd(ctx, _dev(s.t), _dev(s.x), _dev(w), None, s.fmax, s.fw, s.f_lo, s.df,
                            s.I, prec=m2n.M2N_FP64, want_E=False, want_J=True)
    P64 = out64["P"].cpu().numpy()
    # both ends, 4,096 uniform draws and the 256 bands of largest P
    bands = np.unique(np.concatenate([np.arange(0, 32), np.arange(s.I - 32, s.I),
                                      np.random.default_rng(8).integers(0, s.I, 4096),
                                      np.argsort(P64)[-256:]]))
    J_o = orc.nudft(s.t, s.x, w, s.f_lo, s.df, bands=bands)
    for prec, tol in ((m2n.M2N_FP64, 1e-10), (m2n.M2N_FP32, 1e-5)):
        out = out64 if prec == m2n.M2N_FP64 else m2n.m2nufft_psd(
            ctx, _dev(s.t), _dev(s.x), _dev(w), None, s.fmax, s.fw, s.f_lo, s.df, s.I, prec=prec,
            want_E=False, want_J=True)
        J = out["J"].cpu().numpy().astype(np.complex128)[:, bands]
        P = out["P"].cpu().numpy().astype(np.float64)[bands]
        eJ, eP = normwise_rows(J, J_o), psd_err(P, orc.psd(J_o))
        _say(f"  prec={prec}: J sampled {eJ:.3e}  P {eP:.3e}")
        assert eJ < tol and eP < tol
