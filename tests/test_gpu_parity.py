"""GPU parity: the HIP path through the C-ABI against the CPU FP64 oracle.

Tolerances (normwise, after per-taper sign alignment):
  FP64 mode: J and P within 1e-10, lambda within 1e-12 absolute, Ehat 1e-10 abs.
  FP32 mode: J and P within 1e-5 (NuFFT tolerance 1e-6, kernel width 7).
"""
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


# ------------------------------------------------------------- NuFFT alone
def _nufft_case(m2n, ctx, orc, s, w, prec, tol_J, tol_P):
    _say(f"case {s.name} N={s.N} K={w.shape[0]} I={s.I} prec={prec}")
    ref_J = orc.nudft(s.t, s.x, w, s.f_lo, s.df, I=s.I)
    ref_P = orc.psd(ref_J)
    out = m2n.m2nufft_psd(ctx, _dev(s.t), _dev(s.x), _dev(w), None, s.fmax, s.fw, s.f_lo,
                          s.df, s.I, prec=prec, want_E=False, want_J=True)
    J = out["J"].cpu().numpy().astype(np.complex128)
    P = out["P"].cpu().numpy().astype(np.float64)
    eJ, eP = normwise_rows(J, ref_J), psd_err(P, ref_P)
    _say(f"  J normwise {eJ:.3e}  P {eP:.3e}")
    assert eJ < tol_J and eP < tol_P
    J2 = m2n.m2nufft_eigcoeffs(ctx, _dev(s.t), _dev(s.x), _dev(w), s.f_lo, s.df, s.I, prec=prec)
    assert normwise_rows(J2.cpu().numpy().astype(np.complex128), ref_J) < tol_J


@pytest.mark.parametrize("prec,tol", [(2, 1e-10), (1, 1e-5)])
def test_nufft_single_workgroup(m2n, ctx, orc, prec, tol):
    s = W.small_gapped()
    w = np.random.default_rng(100).standard_normal((s.K, s.N)) * 0.1
    _nufft_case(m2n, ctx, orc, s, w, prec, tol, tol)


@pytest.mark.parametrize("prec,tol", [(2, 1e-10), (1, 1e-5)])
def test_nufft_two_pass(m2n, ctx, orc, prec, tol):
    # I = 2^14 -> nf = 2^15: two passes; a ragged N and a wrap of the points
    s = W.gapped_scaled(3000, 5, 2 ** 14, seed=31)
    w = np.random.default_rng(101).standard_normal((5, s.N)) * 0.05
    _nufft_case(m2n, ctx, orc, s, w, prec, tol, tol)


@pytest.mark.parametrize("prec,tol", [(2, 1e-10), (1, 1e-5)])
def test_nufft_two_pass_k9(m2n, ctx, orc, prec, tol):
    # K = 9 > 8 tapers per pass-2 chunk: the average spans two chunks
    s = W.gapped_scaled(4000, 9, 2 ** 13, seed=34)
    w = np.random.default_rng(104).standard_normal((9, s.N)) * 0.05
    _nufft_case(m2n, ctx, orc, s, w, prec, tol, tol)


@pytest.mark.parametrize("prec,tol", [(2, 1e-10), (1, 1e-5)])
def test_nufft_large_grid_sampled(m2n, ctx, orc, prec, tol):
    # I = 2^17 (nf = 2^18, 512 x 512 split); the oracle evaluates a sample of
    # bands: both ends, 4,096 uniform draws and the 256 bands of largest P, so
    # that the sampled norms stand for the full-band ones and carry the peaks
    s = W.gapped_scaled(12000, 5, 2 ** 17, seed=35)
    w = np.random.default_rng(105).standard_normal((5, s.N)) * 0.02
    _say(f"case sampled N={s.N} I={s.I} prec={prec}")
    out = m2n.m2nufft_psd(ctx, _dev(s.t), _dev(s.x), _dev(w), None, s.fmax, s.fw, s.f_lo,
                          s.df, s.I, prec=prec, want_E=False, want_J=True)
    Pall = out["P"].cpu().numpy().astype(np.float64)
    bands = np.unique(np.concatenate([np.arange(0, 64), np.arange(s.I - 64, s.I),
                                      np.random.default_rng(7).integers(0, s.I, 4096),
                                      np.argsort(Pall)[-256:]]))
    ref_J = orc.nudft(s.t, s.x, w, s.f_lo, s.df, bands=bands)
    J = out["J"].cpu().numpy().astype(np.complex128)[:, bands]
    eJ = normwise_rows(J, ref_J)
    eP = psd_err(Pall[bands], orc.psd(ref_J))
    _say(f"  J sampled {eJ:.3e}  P {eP:.3e}")
    assert eJ < tol and eP < tol


@pytest.mark.parametrize("I,K,weighted,prec,tol_P,tol_E", [
    (2 ** 16, 5, False, 1, 1e-5, 1e-6), (2 ** 17, 9, True, 1, 1e-5, 1e-6), (2 ** 18, 7, False, 1, 1e-5, 1e-6),
    (2 ** 16, 5, True, 2, 1e-10, 1e-12), (2 ** 18, 9, False, 2, 1e-10, 1e-12),
    (2 ** 20, 7, False, 1, 1e-5, 1e-6), (2 ** 20, 9, True, 1, 1e-5, 1e-6)])
def test_psd_only_wavefront_rows(m2n, ctx, orc, I, K, weighted, prec, tol_P, tol_E):
    # P and E without J or F: rows of 512 (I = 2^16, 2^17), 1024 (I = 2^18)
    # or 2048 (I = 2^20, FP32) take the pass-2 form with one wavefront per
    # taper row; with
    # K = 9 a wavefront takes two tapers (and their weights).  P against the
    # oracle's direct NUDFT on sampled bands (both ends, uniform draws, the
    # largest-P bands); E, band-constant on a lattice, against the oracle's
    # Ehat for tapers and lambda that do not solve the GEP, so that it is not
    # zero and every taper's norm enters it.
    s = W.gapped_scaled(12000, K, I, seed=37)
    rng = np.random.default_rng(106)
    w = rng.standard_normal((K, s.N)) * 0.02
    lam = rng.uniform(0.5, 1.0, K)
    d = rng.uniform(0.5, 1.5, K) / K if weighted else None
    _say(f"case psd-only N={s.N} K={K} I={I} weighted={weighted} prec={prec}")
    out = m2n.m2nufft_psd(ctx, _dev(s.t), _dev(s.x), _dev(w), _dev(lam), s.fmax, s.fw, s.f_lo,
                          s.df, s.I, prec=prec, weights=None if d is None else _dev(d), want_E=True,
                          want_J=False)
    P = out["P"].cpu().numpy().astype(np.float64)
    E = out["E"].cpu().numpy().astype(np.float64)
    bands = np.unique(np.concatenate([np.arange(0, 32), np.arange(s.I - 32, s.I),
                                      np.random.default_rng(8).integers(0, s.I, 2048),
                                      np.argsort(P)[-128:]]))
    ref_P = orc.psd(orc.nudft(s.t, s.x, w, s.f_lo, s.df, bands=bands), weights=d)
    eP = psd_err(P[bands], ref_P)
    eb = bands[[0, 1, len(bands) // 2, -1]]
    E_ref, _ = orc.ehat(s.t, w, lam, s.fmax, s.fw, s.f_lo, s.df, bands=eb)
    eE = float(np.abs(E[eb] - E_ref).max() / np.abs(E_ref).max())
    _say(f"  P sampled {eP:.3e}  E {eE:.3e} (E_ref {E_ref[0]:.4e})")
    assert eP < tol_P and eE < tol_E
    assert np.all(E == E[0])


def test_ehat_two_pass_lattice(m2n, ctx, orc):
    # Ehat through the two-pass path on a lattice (R(B) = I): identically ~0
    s = W.gapped_scaled(3000, 5, 2 ** 14, seed=36)
    w, lam = orc.gpss_tapers(s.t, s.fmax, s.fw, 5, method="lanczos")
    bands = np.array([0, 1, 777, 8192, 16383], dtype=np.int64)
    E_ref, _ = orc.ehat(s.t, w, lam, s.fmax, s.fw, s.f_lo, s.df, bands=bands)
    out = m2n.m2nufft_psd(ctx, _dev(s.t), _dev(s.x), _dev(w), _dev(lam), s.fmax, s.fw, s.f_lo,
                          s.df, s.I, prec=2, want_E=True)
    E = out["E"].cpu().numpy()
    assert np.abs(E[bands] - E_ref).max() < 1e-10
    assert np.abs(E).max() < 1e-10


@pytest.mark.parametrize("name", ["jitter", "arithmetic", "missing"])
def test_nufft_nonlattice_times(m2n, ctx, orc, name):
    s = W.by_name(name)
    s.I = 4096
    s.df = 1.0 / 4096
    w = np.random.default_rng(102).standard_normal((s.K, s.N))
    _nufft_case(m2n, ctx, orc, s, w, 2, 1e-10, 1e-10)


def test_nufft_wrapped_grid(m2n, ctx, orc):
    # df * span > 1: the points wrap around the periodic grid several times
    s = W.gapped_scaled(3000, 3, 2 ** 14, seed=33)
    s.I = 8192            # two-pass grid (nf = 16384)
    s.df = 1.0 / 1777.0
    s.f_lo = -0.31
    w = np.random.default_rng(103).standard_normal((3, s.N))
    _nufft_case(m2n, ctx, orc, s, w, 2, 1e-10, 1e-10)


# ---------------------------------------------------------------- the GEP
def _gep_case(m2n, ctx, orc, t, fmax, fw, K, tol_w=1e-9):
    _say(f"gep N={len(t)} fw={fw} K={K}")
    w_ref, lam_ref = orc.gpss_tapers(t, fmax, fw, K)
    w, lam = m2n.gpss_tapers(ctx, _dev(t), fmax, fw, K)
    w, lam = w.cpu().numpy(), lam.cpu().numpy()
    el = np.abs(lam - lam_ref).max()
    wa, _ = align_signs(w, w_ref)
    ew = normwise_rows(wa, w_ref)
    _say(f"  lambda {el:.3e}  w {ew:.3e}")
    assert el < 1e-12
    assert ew < tol_w
    return w, lam


def test_gep_lattice_small(m2n, ctx, orc):
    s = W.small_gapped()
    _gep_case(m2n, ctx, orc, s.t, s.fmax, s.fw, s.K)


@pytest.mark.parametrize("name", ["jitter", "missing", "arithmetic", "uniform"])
def test_gep_dense_small(m2n, ctx, orc, name):
    s = W.by_name(name)
    _gep_case(m2n, ctx, orc, s.t, s.fmax, 0.0125 if name != "uniform" else s.fw, s.K)


def test_gep_lattice_medium(m2n, ctx, orc):
    s = W.gapped_scaled(2048, 6, 4096, seed=41)
    _gep_case(m2n, ctx, orc, s.t, s.fmax, s.fw, 6)


def test_gep_lattice_two_pass_fft(m2n, ctx, orc):
    # span ~ 6000 -> convolution grid M = 16384 > 4096: two-pass FP64 FFT
    s = W.gapped_scaled(6000, 7, 8192, seed=43)
    _say(f"gep lattice two-pass N={s.N}")
    w_ref, lam_ref = orc.gpss_tapers(s.t, s.fmax, s.fw, 7, method="lanczos")
    w, lam = m2n.gpss_tapers(ctx, _dev(s.t), s.fmax, s.fw, 7)
    w, lam = w.cpu().numpy(), lam.cpu().numpy()
    assert np.abs(lam - lam_ref).max() < 1e-12
    wa, _ = align_signs(w, w_ref)
    assert normwise_rows(wa, w_ref) < 1e-8


def _gep_subspace_case(m2n, ctx, orc, s, fw, K, I=4096):
    """Wide band (quadrature rank > 64): block subspace iteration.  Top
    eigenvalues cluster, so tapers are compared through what is unique: the
    eigenvalues and the PSD of a series (invariant to rotations of the span)."""
    _say(f"gep subspace N={s.N} fw={fw} K={K}")
    w_ref, lam_ref = orc.gpss_tapers(s.t, s.fmax, fw, K, method="jacobi" if s.N <= 600 else "lanczos")
    t, x = _dev(s.t), _dev(s.x)
    w, lam = m2n.gpss_tapers(ctx, t, s.fmax, fw, K)
    el = np.abs(lam.cpu().numpy() - lam_ref).max()
    P = m2n.m2nufft_psd(ctx, t, x, w, None, s.fmax, fw, -0.5, 1.0 / I, I, prec=2,
                        want_E=False)["P"].cpu().numpy()
    P_ref = orc.psd(orc.nudft(s.t, s.x, w_ref, -0.5, 1.0 / I, I=I))
    eP = psd_err(P, P_ref)
    G = w.cpu().numpy() @ orc.gpss_matrix(s.t, s.fmax) @ w.cpu().numpy().T
    eG = np.abs(G - 2 * fw * np.eye(K)).max()
    _say(f"  lambda {el:.3e}  P {eP:.3e}  R(B)-orthonormality {eG:.3e}")
    assert el < 1e-12 and eP < 1e-10 and eG < 1e-12


def test_gep_lattice_subspace_fallback(m2n, ctx, orc):
    s = W.gapped_scaled(3000, 14, 4096, seed=44)
    _gep_subspace_case(m2n, ctx, orc, s, 12 / 3000, 14)


def test_gep_dense_subspace_fallback(m2n, ctx, orc):
    s = W.jitter_stress(n=300, seed=45, K=35)
    _gep_subspace_case(m2n, ctx, orc, s, 0.06, 35)


@pytest.mark.parametrize("N,NW,K", [(1200, 4, 7), (1200, 5, 9), (2000, 6, 11)])
def test_gep_lattice_dpss_clusters(m2n, ctx, orc, N, NW, K):
    """Uniform sampling (the DPSS case): the top concentrations crowd
    towards 1.  Smallest gaps 2.7e-8 (NW = 4, eigenvectors from twisted
    factorisations), 7.3e-11 and 1.8e-13 (NW = 5, 6: inverse iteration).
    Within such clusters single eigenvectors are ill-conditioned, so the
    comparison is through the eigenvalues, the PSD of a series and
    R(B)-orthonormality."""
    t = np.arange(N, dtype=np.float64)
    x = np.random.default_rng(N + NW).standard_normal(N)
    fw, fmax, I = NW / N, 0.5, 4096
    _say(f"gep dpss N={N} NW={NW} K={K}")
    w_ref, lam_ref = orc.gpss_tapers(t, fmax, fw, K, method="lanczos")
    w, lam = m2n.gpss_tapers(ctx, _dev(t), fmax, fw, K)
    el = np.abs(lam.cpu().numpy() - lam_ref).max()
    P = m2n.m2nufft_psd(ctx, _dev(t), _dev(x), w, None, fmax, fw, -0.5, 1.0 / I, I, prec=2,
                        want_E=False)["P"].cpu().numpy()
    P_ref = orc.psd(orc.nudft(t, x, w_ref, -0.5, 1.0 / I, I=I))
    eP = psd_err(P, P_ref)
    wn = w.cpu().numpy()
    eG = np.abs(wn @ wn.T - 2 * fw * np.eye(K)).max()     # R(B) = 2 f_max I = I
    _say(f"  lambda {el:.3e}  P {eP:.3e}  orthonormality {eG:.3e}")
    assert el < 1e-12 and eP < 1e-10 and eG < 1e-12


def test_gep_dense_medium(m2n, ctx, orc):
    s = W.jitter_stress(n=300, seed=42, K=5)
    _gep_case(m2n, ctx, orc, s.t, s.fmax, 2.5 / 300, 5)


@pytest.mark.parametrize("n,seed", [(2100, 46), (3200, 47)])
def test_gep_dense_large(m2n, ctx, orc, n, seed):
    # dense R(B) on the jittered grid at 33 and 50 panels of 64 (the tiled
    # Cholesky with look-ahead and the blocked triangular solves over many
    # panels), against the oracle's unblocked Cholesky and Lanczos; and the
    # PSD of the series through both sets of tapers
    s = W.jitter_stress(n=n, seed=seed, K=6)
    w, lam = _gep_case(m2n, ctx, orc, s.t, s.fmax, 4.0 / n, 6, tol_w=1e-7)
    I = 4096
    P = m2n.m2nufft_psd(ctx, _dev(s.t), _dev(s.x), _dev(w), None, s.fmax, 4.0 / n, -0.5, 1.0 / I, I,
                        prec=2, want_E=False)["P"].cpu().numpy()
    w_ref, _ = orc.gpss_tapers(s.t, s.fmax, 4.0 / n, 6)
    bands = np.unique(np.random.default_rng(seed).integers(0, I, 256))
    P_ref = orc.psd(orc.nudft(s.t, s.x, w_ref, -0.5, 1.0 / I, bands=bands))
    eP = psd_err(P[bands], P_ref)
    _say(f"  P {eP:.3e}")
    assert eP < 1e-10


# ------------------------------------------------------------ end to end
@pytest.mark.parametrize("prec,tol", [(2, 1e-10), (1, 1e-5)])
def test_end_to_end_small(m2n, ctx, orc, prec, tol):
    s = W.small_gapped()
    ref = orc.m2nufft(s.t, s.x, s.fmax, s.fw, s.K, s.f_lo, s.df, s.I)
    t, x = _dev(s.t), _dev(s.x)
    w, lam = m2n.gpss_tapers(ctx, t, s.fmax, s.fw, s.K)
    out = m2n.m2nufft_psd(ctx, t, x, w, lam, s.fmax, s.fw, s.f_lo, s.df, s.I, prec=prec,
                          want_E=True, want_J=True)
    P = out["P"].cpu().numpy().astype(np.float64)
    E = out["E"].cpu().numpy().astype(np.float64)
    assert psd_err(P, ref["P"]) < tol
    assert np.abs(E - ref["E"]).max() < tol


def test_errors(m2n, ctx):
    t = _dev(np.array([0.0, 2.0, 1.0, 3.0]))
    with pytest.raises(m2n.M2NError) as ei:
        m2n.gpss_tapers(ctx, t, 0.5, 0.1, 2)
    assert ei.value.code == m2n.M2N_ERR_T_ORDER
    with pytest.raises(m2n.M2NError) as ei:
        m2n.gpss_tapers(ctx, _dev(np.arange(4.0)), 0.5, 0.6, 2)
    assert ei.value.code == m2n.M2N_ERR_ARG
    with pytest.raises(m2n.M2NError) as ei:
        m2n.gpss_tapers(ctx, _dev(np.arange(4.0)), 0.5, 0.1, 2, fc0=0.1)
    assert ei.value.code == m2n.M2N_ERR_UNSUPPORTED
    x = _dev(np.array([1.0, np.nan, 2.0, 3.0]))
    w = _dev(np.ones((1, 4)))
    with pytest.raises(m2n.M2NError) as ei:
        m2n.m2nufft_psd(ctx, _dev(np.arange(4.0)), x, w, None, 0.5, 0.1, -0.5, 1 / 64, 64,
                        want_E=False)
    assert ei.value.code == m2n.M2N_ERR_ARG


def test_sync_mode_returns_device_errors(m2n, ctx, monkeypatch):
    # a context created while M2N_SYNC=1: the call waits and returns the error
    # its kernels flagged (non-finite x); on the default context the same call
    # returns at once and the error surfaces at the next m2n_stream_status
    monkeypatch.setenv("M2N_SYNC", "1")
    sctx = m2n.Context(0)
    monkeypatch.delenv("M2N_SYNC")
    try:
        t = _dev(np.arange(4.0))
        x = _dev(np.array([1.0, np.nan, 2.0, 3.0]))
        w = _dev(np.ones((1, 4)))
        args = (t, x, w, None, 0.5, 0.1, -0.5, 1 / 64, 64)
        with pytest.raises(m2n.M2NError) as ei:
            m2n.m2nufft_psd(sctx, *args, want_E=False, check=False)
        assert ei.value.code == m2n.M2N_ERR_ARG
        sctx.check()                       # reported once, then cleared
        m2n.m2nufft_psd(ctx, *args, want_E=False, check=False)
        with pytest.raises(m2n.M2NError) as ei:
            ctx.check()
        assert ei.value.code == m2n.M2N_ERR_ARG
        ctx.check()
        # a clean series: the same tapers and spectrum bit for bit in both modes
        s = W.small_gapped()
        outs = []
        for c in (ctx, sctx):
            tt, xx = _dev(s.t), _dev(s.x)
            wk, lam = m2n.gpss_tapers(c, tt, s.fmax, s.fw, s.K)
            o = m2n.m2nufft_psd(c, tt, xx, wk, lam, s.fmax, s.fw, s.f_lo, s.df, s.I, prec=2)
            outs.append([wk.cpu().numpy(), lam.cpu().numpy(), o["P"].cpu().numpy(), o["E"].cpu().numpy()])
        for a, b in zip(*outs):
            assert np.array_equal(a, b)
        _say("case sync mode: error returned by the call; results bitwise equal to the default mode")
    finally:
        sctx.close()
