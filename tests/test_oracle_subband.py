"""Pins of the oracle's sub-band functions (Sec. 2.4 sub-band matrix and
Appendix A; Sec. 3.1-3.2 nominal band at fc0 and relative eigencoefficients).

Each pin compares the oracle with something it does not compute itself: a
40-digit integral, the Appendix A decomposition, the full-band oracle (pinned
in test_oracle_pins.py), scipy's DPSS on the integer lattice, or a brute-force
quadrature of the tapers' spectral windows.
"""
import numpy as np
import pytest
import scipy.signal.windows as sw

import workloads as W


def _jittered(n, d, sigma, seed):
    rng = np.random.default_rng(seed)
    t = d * np.arange(n, dtype=np.float64) + rng.normal(0.0, sigma, n)
    t.sort()
    return t


def test_subband_matrix_against_mpmath_integral(orc):
    """R(B^q)_{nm} is the integral of e^{j 2 pi f tau} over f_min <= |f| <= f_max:
    checked against mpmath's quadrature of 2 cos(2 pi f tau) on [f_min, f_max]
    and against the 40-digit difference of the two full-band sincs."""
    import mpmath
    mpmath.mp.dps = 40
    t = _jittered(40, 2.2, 0.4, 1)
    for fmin, fmax in [(0.0, 0.25), (0.25, 0.5), (0.13, 0.31)]:
        R = orc.subband_matrix(t, fmin, fmax)
        assert np.array_equal(R, R.T)
        assert np.all(np.diag(R) == 2.0 * (fmax - fmin))
        rng = np.random.default_rng(2)
        for n, m in rng.integers(0, 40, size=(25, 2)):
            if n == m:
                continue
            tau = mpmath.mpf(float(t[n])) - mpmath.mpf(float(t[m]))
            ref = (mpmath.sin(2 * mpmath.pi * mpmath.mpf(fmax) * tau)
                   - mpmath.sin(2 * mpmath.pi * mpmath.mpf(fmin) * tau)) / (mpmath.pi * tau)
            assert abs(R[n, m] - float(ref)) < 2e-15
        for n, m in [(0, 1), (3, 17), (5, 39)]:
            tau = float(t[n] - t[m])
            q = mpmath.quad(lambda f: 2 * mpmath.cos(2 * mpmath.pi * f * tau), [fmin, fmax])
            assert abs(R[n, m] - float(q)) < 1e-14


def test_subband_matrix_positive_definite_appendix_a(orc):
    """Appendix A: R(B^q) = R(A1) - R(A2) with A1 = {|f| <= f_max},
    A2 = {|f| < f_min}, Hermitian and positive definite for distinct t."""
    t = _jittered(60, 2.2, 0.4, 3)
    for fmin, fmax in [(0.0, 0.25), (0.25, 0.5), (0.1, 0.3)]:
        R = orc.subband_matrix(t, fmin, fmax)
        D = orc.gpss_matrix(t, fmax) - (orc.gpss_matrix(t, fmin) if fmin > 0 else 0.0)
        assert np.abs(R - D).max() < 1e-14
        assert np.linalg.eigvalsh(R)[0] > 0.0


def test_subband_full_band_at_zero_reduces_to_gpss(orc):
    """Q = 1, f_min = 0, fc0 = 0: the sub-band tapers are the full-band GPSS
    tapers (real, same sign reading) and the eigenvalues agree."""
    s = W.scheme_jitter()
    w, lam = orc.subband_tapers(s.t, 0.0, s.fmax, s.fw, 0.0, s.K)
    w0, lam0 = orc.gpss_tapers(s.t, s.fmax, s.fw, s.K, method="jacobi")
    assert np.abs(lam - lam0).max() < 1e-12
    assert np.abs(w.imag).max() < 1e-12
    assert np.abs(w.real - w0).max() < 1e-9 * np.abs(w0).max()


@pytest.mark.parametrize("fc0", [0.1, 0.23, -0.17])
def test_subband_lattice_is_modulated_dpss(orc, fc0):
    """Integer lattice, f_max = 1/2 (R(B) = I): the tapers of the band centred
    at fc0 are the DPSS of N, f_w modulated by e^{j 2 pi fc0 (t - tbar)},
    scaled to norm 2 f_w, and the eigenvalues are the DPSS concentrations
    (scipy).  A wrong sign of the modulation fails the comparison.  NW = 2.5
    keeps the eigenvalue gaps near 1e-3, so both eigen-solvers fix the
    vectors to rounding level."""
    N, NW, K = 128, 2.5, 4
    fw = NW / N
    t = np.arange(N, dtype=np.float64)
    w, lam = orc.subband_tapers(t, 0.0, 0.5, fw, fc0, K)
    v, ratios = sw.dpss(N, NW, Kmax=K, return_ratios=True)
    assert np.abs(lam - ratios).max() < 1e-10
    tbar = 0.5 * (t[0] + t[-1])
    mod = np.exp(2j * np.pi * fc0 * (t - tbar))
    for k in range(K):
        ref = np.sqrt(2 * fw) * mod * v[k]
        err = min(np.abs(w[k] - ref).max(), np.abs(w[k] + ref).max())
        assert err < 1e-9 * np.abs(ref).max()
        demod = w[k] * np.conj(mod)
        assert np.abs(demod.imag).max() < 1e-10 * np.abs(demod).max()


def test_subband_concentration_brute_force(orc):
    """lambda_k = int_{A0} |W_k|^2 / int_{B^q} |W_k|^2 with W_k(f) =
    sum_n w_k(t_n) e^{-j 2 pi f t_n}, both integrals by dense Gauss-Legendre
    over f; also int_{B^q} W_k conj(W_l) = 2 f_w delta_kl (normalisation and
    R(B)-orthogonality written as integrals, not as matrix products)."""
    t = _jittered(90, 2.2, 0.4, 5)
    fmin, fmax, fc0 = 0.25, 0.5, 0.37
    fw = 3.0 / (t[-1] - t[0])
    K = 4
    w, lam = orc.subband_tapers(t, fmin, fmax, fw, fc0, K)

    def integral(a, b, n=4000):
        x, g = np.polynomial.legendre.leggauss(n)
        f = 0.5 * (b - a) * x + 0.5 * (a + b)
        Wf = np.exp(-2j * np.pi * np.outer(f, t)) @ w.T          # [n, K]
        return 0.5 * (b - a) * np.einsum("f,fk,fl->kl", g, Wf, Wf.conj())

    GB = integral(-fmax, -fmin) + integral(fmin, fmax)
    GA = integral(fc0 - fw, fc0 + fw, 600)
    assert np.abs(GB - 2 * fw * np.eye(K)).max() < 1e-11
    assert np.abs(np.diag(GA).real / np.diag(GB).real - lam).max() < 1e-11
    assert lam[0] > 0.5 and np.all(np.diff(lam) <= 0)


def test_subband_psd_equals_full_band_at_absolute_frequency(orc):
    """On the lattice with R(B) = I the sub-band eigencoefficients at the
    relative frequency df_i are, up to a unit phase, the full-band ones at
    fc0 + df_i (full-band oracle: gpss_tapers + nudft), so the PSDs agree.
    A missing conjugate or a sign slip in the relative frequency fails it.
    NW = 2.5 keeps the tapers well separated (see the DPSS pin above)."""
    N, fw, K = 256, 2.5 / 256, 4
    t = np.arange(N, dtype=np.float64)
    x = W.white_noise(N, 7) + np.cos(2 * np.pi * 0.21 * t)
    fc0, f_lo, df, I = 0.2, -0.05, 0.1 / 64, 64
    w, _ = orc.subband_tapers(t, 0.0, 0.5, fw, fc0, K)
    J = orc.subband_eigcoeffs(t, x, w, f_lo, df, I)
    w0, _ = orc.gpss_tapers(t, 0.5, fw, K, method="jacobi")
    J0 = orc.nudft(t, x, w0, fc0 + f_lo, df, I)
    assert np.abs(np.abs(J) - np.abs(J0)).max() < 1e-10 * np.abs(J0).max()
    P, P0 = orc.psd(J), orc.psd(J0)
    assert np.abs(P - P0).max() < 1e-10 * P0.max()
