"""The suboptimality estimate Ehat (Sec. 3.5 with the Appendix B Rayleigh
quotient) on grids where R(B) is not a multiple of the identity, against the
oracle's direct quadratic form D_k(i) = (E_i w_k)^* R(B) (E_i w_k): absolute
1e-10 in FP64 mode and 1e-5 in FP32 mode, on sampled bands (both ends of the
band range, its middle and random ones).

Grids: t = 5n/6 with a sixth of the samples removed (a lattice whose R(B) is
dense because 2 f_max * 5/6 is not an integer), jittered and arithmetic
grids; windows that are whole multiples of the band spacing, windows with a
fractional cell, and windows narrower than one band spacing; single-workgroup
and two-pass NuFFT grids; tapers from the GEP (oracle or GPU) and random
tapers; the batched form against the per-series call."""
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


def _bands(I, seed, n=40):
    rng = np.random.default_rng(seed)
    b = np.concatenate([[0, 1, 2, I // 2, I - 3, I - 2, I - 1], rng.integers(0, I, n)])
    return np.unique(b).astype(np.int64)


def _random_tapers(N, K, fmax, fw, seed):
    # rows scaled so that D_k is near 2 f_w (lambda_hat near lambda)
    w = np.random.default_rng(seed).standard_normal((K, N))
    w *= np.sqrt(fw / fmax / (w * w).sum(axis=1, keepdims=True))
    lam = np.sort(np.random.default_rng(seed + 1).uniform(0.6, 1.0, K))[::-1].copy()
    return w, lam


def _check(m2n, ctx, orc, t, x, w, lam, fmax, fw, f_lo, df, I, label, seed=0):
    bands = _bands(I, seed)
    E_ref, _ = orc.ehat(t, w, lam, fmax, fw, f_lo, df, bands=bands)
    for prec, tol in ((2, 1e-10), (1, 1e-5)):
        _say(f"ehat {label}: N={t.shape[0]} K={w.shape[0]} I={I} 2fmax/df={2 * fmax / df:.3f} prec={prec}")
        out = m2n.m2nufft_psd(ctx, _dev(t), _dev(x), _dev(w), _dev(lam), fmax, fw, f_lo, df, I,
                              prec=prec, want_E=True)
        E = out["E"].cpu().numpy().astype(np.float64)
        err = np.abs(E[bands] - E_ref).max()
        _say(f"  |dE| max {err:.3e} (Ehat range {E_ref.min():.3e} .. {E_ref.max():.3e})")
        assert np.isfinite(E).all()
        assert err < tol


def test_ehat_lattice_5n6_two_pass(m2n, ctx, orc):
    # t = 5n/6: R(B) dense (and numerically singular at this size), random
    # tapers; 2 f_max / df = I: whole cells, two-pass grids
    s = W.scheme_missing(L=2400, n_keep=2000)
    fmax, fw, K, I = 0.5, 4.0 / 2000, 6, 4096
    w, lam = _random_tapers(s.N, K, fmax, fw, 1)
    _check(m2n, ctx, orc, s.t, s.x, w, lam, fmax, fw, -0.5, 1.0 / I, I, "5n/6 whole cells", 1)


def test_ehat_fractional_cell(m2n, ctx, orc):
    # 2 f_max / df = 2457.6: every window ends in a fractional cell
    s = W.scheme_missing(L=2400, n_keep=2000, seed=14)
    fmax, fw, K, I = 0.3, 3.0 / 2000, 5, 4096
    w, lam = _random_tapers(s.N, K, fmax, fw, 2)
    _check(m2n, ctx, orc, s.t, s.x, w, lam, fmax, fw, -0.37, 1.0 / I, I, "fractional cell", 2)


def test_ehat_window_narrower_than_spacing(m2n, ctx, orc):
    # 2 f_max < df: no whole cell, only the fractional one
    s = W.scheme_jitter(n=50)
    fmax, fw, K, I = 0.04, 0.01, 3, 16
    w, lam = _random_tapers(s.N, K, fmax, fw, 3)
    _check(m2n, ctx, orc, s.t, s.x, w, lam, fmax, fw, -0.8, 0.1, I, "window < df", 3)


def test_ehat_paper_scheme_oracle_tapers(m2n, ctx, orc):
    # the paper's 50-point 5n/6 and arithmetic schemes with their GEP tapers
    for s in (W.scheme_missing(), W.scheme_arithmetic()):
        w, lam = orc.gpss_tapers(s.t, s.fmax, s.fw, s.K, method="jacobi")
        _check(m2n, ctx, orc, s.t, s.x, w, lam, s.fmax, s.fw, s.f_lo, s.df, s.I, s.name, 4)


def test_ehat_jitter_gpu_tapers(m2n, ctx, orc):
    # GPU tapers on a jittered grid (dense R(B)), single-workgroup grids
    s = W.jitter_stress(n=600, seed=9, K=5, I=1024)
    t = _dev(s.t)
    w, lam = m2n.gpss_tapers(ctx, t, s.fmax, s.fw, s.K)
    torch.cuda.synchronize()
    _check(m2n, ctx, orc, s.t, s.x, w.cpu().numpy(), lam.cpu().numpy(), s.fmax, s.fw, s.f_lo, s.df,
           s.I, "jitter_600", 5)


def test_ehat_batch_mixed(m2n, ctx, orc):
    # a lattice series (band-constant Ehat) and two dense-R(B) series in one
    # batch: each equal to its per-series call
    specs = [W.small_gapped(), W.scheme_missing(), W.jitter_stress(n=300, seed=4, K=4, I=512)]
    series = [{"t": _dev(s.t), "x": _dev(s.x), "K": s.K, "fmax": s.fmax, "fw": s.fw, "f_lo": s.f_lo,
               "df": s.df, "I": s.I, "want_E": True} for s in specs]
    outs = m2n.m2n_batch_psd(ctx, series, prec=m2n.M2N_FP64)
    torch.cuda.synchronize()
    for s, o in zip(specs, outs):
        _say(f"batch ehat {s.name}: N={s.N}")
        t, x = _dev(s.t), _dev(s.x)
        w, lam = m2n.gpss_tapers(ctx, t, s.fmax, s.fw, s.K)
        one = m2n.m2nufft_psd(ctx, t, x, w, lam, s.fmax, s.fw, s.f_lo, s.df, s.I, prec=2, want_E=True)
        Eb, Es = o["E"].cpu().numpy(), one["E"].cpu().numpy()
        assert np.abs(Eb - Es).max() < 1e-12
        E_ref, _ = orc.ehat(s.t, w.cpu().numpy(), lam.cpu().numpy(), s.fmax, s.fw, s.f_lo, s.df,
                            bands=_bands(s.I, 6))
        assert np.abs(Es[_bands(s.I, 6)] - E_ref).max() < 1e-10


def test_ehat_needs_increasing_t(m2n, ctx):
    t = _dev(np.array([0.0, 2.5, 1.0, 3.0]))
    x = _dev(np.ones(4))
    w = _dev(np.ones((1, 4)))
    lam = _dev(np.ones(1))
    with pytest.raises(m2n.M2NError) as ei:
        m2n.m2nufft_psd(ctx, t, x, w, lam, 0.5, 0.1, -0.5, 1 / 64, 64, want_E=True)
    assert ei.value.code == m2n.M2N_ERR_T_ORDER
