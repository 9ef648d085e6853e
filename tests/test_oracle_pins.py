"""Pins of the CPU FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own code: each one compares it with a
closed form, a library routine on a special case, an exact rational
computation, a brute force, or an invariant the paper states.  A plausible
slip in the oracle (dropped term, wrong sign or index, transposed operand,
wrong normalisation) fails at least one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.signal.windows as sw

import workloads as W


# --------------------------------------------------------------------------
# sin(pi u) reduction and the GPSS matrices (Sec. 2.1 R(B), Sec. 2.3 R(A))
# --------------------------------------------------------------------------

def test_sinpi_exact_zero_at_integers_and_matches_mpmath(orc):
    import mpmath
    mpmath.mp.dps = 40
    for u in [0.0, 1.0, -1.0, 2.0, 7.0, -12345.0, 2.0 ** 40]:
        assert orc.sinpi(u) == 0.0
    rng = np.random.default_rng(0)
    for u in np.concatenate([rng.uniform(-50, 50, 200), [0.5, -0.5, 1.5, 1e-9, 3.25]]):
        ref = float(mpmath.sin(mpmath.pi * mpmath.mpf(float(u))))
        assert abs(orc.sinpi(u) - ref) <= 4e-16 * max(abs(ref), 1e-300) + 1e-300


def test_gpss_matrix_entries_against_mpmath(orc):
    import mpmath
    mpmath.mp.dps = 40
    s = W.scheme_jitter()
    R = orc.gpss_matrix(s.t, 0.5)
    assert np.array_equal(R, R.T)
    rng = np.random.default_rng(1)
    for _ in range(50):
        n, m = rng.integers(0, s.N, 2)
        tau = mpmath.mpf(float(s.t[n])) - mpmath.mpf(float(s.t[m]))
        tau = mpmath.mpf(float(tau))          # the difference is rounded once, as in FP64
        ref = 1.0 if n == m else float(mpmath.sin(2 * mpmath.pi * 0.5 * tau) / (mpmath.pi * tau))
        assert abs(R[n, m] - ref) <= 1e-15
    np.testing.assert_array_equal(np.diag(R), 1.0)


def test_lattice_signal_band_matrix_is_identity(orc):
    # Appendix B: integer lattice, f_s = 1, f_max = 1/2  =>  R(B) = I exactly
    s = W.small_gapped()
    R = orc.gpss_matrix(s.t, 0.5)
    assert np.array_equal(R, np.eye(s.N))
    # also for a lattice of spacing 2 with f_max = 1/2 (2 f_max beta = 2)
    R2 = orc.gpss_matrix(2.0 * s.t, 0.5)
    assert np.array_equal(R2, np.eye(s.N))


def test_band_matrix_shift_identity(orc):
    # Sec. 3.5: R(A0) = E_i^* R(A_i) E_i with E_i = diag(exp(j 2 pi df_i t_n))
    s = W.scheme_arithmetic()
    fw, fci = 0.05, 0.137
    RA0 = orc.band_matrix(s.t, 0.0, fw)
    RAi = orc.band_matrix(s.t, fci, fw)
    E = np.diag(np.exp(2j * np.pi * fci * s.t))
    np.testing.assert_allclose(E.conj().T @ RAi @ E, RA0, atol=1e-14)
    np.testing.assert_allclose(RA0.imag, 0.0, atol=0)
    np.testing.assert_allclose(RA0.real, orc.gpss_matrix(s.t, fw), atol=0)


def test_apply_sinc_matches_dense(orc):
    s = W.small_gapped()
    V = np.random.default_rng(2).standard_normal((s.N, 3))
    Y = orc.apply_sinc(s.t, s.fw, V)          # integer t: lag-table path
    np.testing.assert_allclose(Y, orc.gpss_matrix(s.t, s.fw) @ V, rtol=0, atol=1e-13)
    j = W.scheme_jitter()
    V = np.random.default_rng(3).standard_normal((j.N, 2))
    np.testing.assert_allclose(orc.apply_sinc(j.t, 0.3, V),
                               orc.gpss_matrix(j.t, 0.3) @ V, rtol=0, atol=1e-13)


# --------------------------------------------------------------------------
# linear algebra against LAPACK (numpy) on the same matrices
# --------------------------------------------------------------------------

def test_cholesky_and_reduce_against_lapack(orc):
    s = W.scheme_jitter()
    RB = orc.gpss_matrix(s.t, 0.5)
    L = orc.cholesky(RB)
    np.testing.assert_allclose(L, np.linalg.cholesky(RB), atol=1e-13)
    RA = orc.gpss_matrix(s.t, 0.05)
    C = orc.reduce(L, RA)
    np.testing.assert_allclose(L @ C @ L.T, RA, atol=1e-13)
    Li = np.linalg.inv(np.linalg.cholesky(RB))
    np.testing.assert_allclose(C, Li @ RA @ Li.T, atol=1e-12)


def test_cholesky_reports_non_pd(orc):
    # duplicated sampling time: R(B) is singular
    t = np.array([0.0, 1.0, 1.0, 2.0])
    with pytest.raises(orc.OracleError):
        orc.cholesky(orc.gpss_matrix(t, 0.5))
    assert orc.validate(t, 0.5, 0.1, 2) == orc.ERR_T_ORDER


def test_jacobi_against_lapack(orc):
    s = W.scheme_missing()
    C = orc.gpss_matrix(s.t, 0.05)
    ev, V = orc.jacobi_eigh(C)
    ref = np.linalg.eigvalsh(C)[::-1]
    np.testing.assert_allclose(ev, ref, atol=1e-14)
    np.testing.assert_allclose(V @ np.diag(ev) @ V.T, C, atol=1e-13)
    np.testing.assert_allclose(V.T @ V, np.eye(s.N), atol=1e-13)


def test_lanczos_matches_jacobi(orc):
    s = W.gapped_scaled(512, 5, 1024, seed=21)
    w_j, lam_j = orc.gpss_tapers(s.t, 0.5, s.fw, 5, method="jacobi")
    w_l, lam_l = orc.gpss_tapers(s.t, 0.5, s.fw, 5, method="lanczos")
    np.testing.assert_allclose(lam_l, lam_j, atol=1e-13)
    np.testing.assert_allclose(w_l, w_j, atol=1e-9)
    # general (dense, non-diagonal R(B)) Lanczos path too
    # (f_w chosen so the top eigenvalues are separated by >= 5e-4: a taper is
    # only determined to ~eps/gap)
    j = W.scheme_jitter(n=200)
    w_j, lam_j = orc.gpss_tapers(j.t, 0.5, 0.0125, 4, method="jacobi")
    w_l, lam_l = orc.gpss_tapers(j.t, 0.5, 0.0125, 4, method="lanczos")
    np.testing.assert_allclose(lam_l, lam_j, atol=1e-13)
    np.testing.assert_allclose(w_l, w_j, atol=1e-9)


def test_oracle_fft_is_the_dft(orc):
    # the oracle's own radix-2 FFT against the DFT written out as a sum
    rng = np.random.default_rng(31)
    for M in (1, 2, 8, 64, 256):
        x = rng.standard_normal(M) + 1j * rng.standard_normal(M)
        jk = np.outer(np.arange(M), np.arange(M)) % M
        for sign in (-1, 1):
            ref = (np.exp(sign * 2j * np.pi * jk / M) * x[None, :]).sum(axis=1)
            assert np.abs(orc.fft(x, sign) - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_toeplitz_matvec_matches_direct_sum(orc):
    # R(f) V on integer lattices by the Toeplitz convolution equals the direct
    # sum of the sinc kernel (N up to 4096; gaps, a shifted origin, several f)
    rng = np.random.default_rng(32)
    for L, seed in ((700, 1), (2000, 2), (5200, 3)):
        s = W.gapped_scaled(L, 3, 1024, seed=seed)
        t = s.t + 17.0
        assert s.N <= 4096
        V = rng.standard_normal((s.N, 3))
        for f in (s.fw, 0.5, 0.37):
            A = orc.apply_sinc(t, f, V)
            B = orc.apply_sinc_toeplitz(t, f, V)
            assert np.abs(A - B).max() <= 1e-13 * np.abs(A).max()
    with pytest.raises(orc.OracleError):
        orc.apply_sinc_toeplitz(np.array([0.0, 1.5, 3.0]), 0.1, np.ones((3, 1)))


def test_lattice_method_matches_jacobi_and_lanczos(orc):
    # the lattice method (no N x N matrix, Toeplitz Lanczos) against the dense
    # Jacobi solve and the direct-sum Lanczos
    s = W.gapped_scaled(700, 4, 4096, seed=5)
    w_j, lam_j = orc.gpss_tapers(s.t, 0.5, s.fw, 4, method="jacobi")
    w_t, lam_t = orc.gpss_tapers(s.t, 0.5, s.fw, 4, method="lattice")
    np.testing.assert_allclose(lam_t, lam_j, atol=1e-13)
    np.testing.assert_allclose(w_t, w_j, atol=1e-9)
    s = W.gapped_scaled(2600, 5, 4096, seed=6)
    w_l, lam_l = orc.gpss_tapers(s.t, 1.0, s.fw, 5, method="lanczos")
    w_t, lam_t = orc.gpss_tapers(s.t, 1.0, s.fw, 5, method="lattice")
    np.testing.assert_allclose(lam_t, lam_l, atol=1e-13)
    np.testing.assert_allclose(w_t, w_l, atol=1e-9)
    with pytest.raises(orc.OracleError):
        orc.gpss_tapers(s.t + 0.5, 0.5, s.fw, 5, method="lattice")


# --------------------------------------------------------------------------
# P1: closed forms at N = 1 and N = 2
# --------------------------------------------------------------------------

def test_tapers_closed_form_n1(orc):
    fmax, fw, x = 0.5, 0.125, 1.7
    w, lam = orc.gpss_tapers(np.array([3.25]), fmax, fw, 1)
    assert abs(lam[0] - fw / fmax) < 1e-16
    assert abs(w[0, 0] - math.sqrt(fw / fmax)) < 1e-16
    J = orc.nudft(np.array([3.25]), np.array([x]), w, -0.5, 1 / 8, I=8)
    np.testing.assert_allclose(orc.psd(J), (fw / fmax) * x * x, rtol=1e-15)


def test_tapers_closed_form_n2(orc):
    t = np.array([0.0, 0.7])
    fmax, fw = 0.5, 0.2
    sB = math.sin(2 * math.pi * fmax * 0.7) / (math.pi * 0.7)
    sA = math.sin(2 * math.pi * fw * 0.7) / (math.pi * 0.7)
    lp, lm = (2 * fw + sA) / (2 * fmax + sB), (2 * fw - sA) / (2 * fmax - sB)
    w, lam = orc.gpss_tapers(t, fmax, fw, 2)
    order = [0, 1] if lp >= lm else [1, 0]
    pairs = [(lp, math.sqrt(fw / (2 * fmax + sB)) * np.array([1.0, 1.0])),
             (lm, math.sqrt(fw / (2 * fmax - sB)) * np.array([1.0, -1.0]))]
    for k, idx in enumerate(order):
        assert abs(lam[k] - pairs[idx][0]) < 1e-15
        np.testing.assert_allclose(w[k], pairs[idx][1], atol=1e-15)


# --------------------------------------------------------------------------
# P2: GPSS on a gap-free unit grid with f_max = 1/2 are the DPSS
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N,NW,K", [(64, 2.5, 4), (128, 3.0, 5)])
def test_gpss_reduce_to_dpss(orc, N, NW, K):
    t = np.arange(N, dtype=np.float64)
    fw = NW / N
    w, lam = orc.gpss_tapers(t, 0.5, fw, K)
    v, ratios = sw.dpss(N, NW, Kmax=K, sym=True, norm=2, return_ratios=True)
    np.testing.assert_allclose(lam, ratios, atol=1e-12)
    # same sign convention as the Slepian sequences: even sum > 0, odd start > 0
    np.testing.assert_allclose(w, math.sqrt(2 * fw) * v, atol=1e-9)


# --------------------------------------------------------------------------
# P3: uniform / lattice closed form of the eigencoefficients by FFT
# --------------------------------------------------------------------------

def test_nudft_lattice_closed_form_fft(orc):
    s = W.small_gapped()
    K, I = 3, s.I
    w = np.random.default_rng(4).standard_normal((K, s.N))
    J = orc.nudft(s.t, s.x, w, s.f_lo, s.df, I=I)
    # f_lo = -1/2, df = 1/I, integer t < I: J = FFT_I of (w x e^{j pi t}) on the grid
    g = np.zeros((K, I), dtype=complex)
    ti = s.t.astype(np.int64)
    g[:, ti] = w * s.x * np.exp(1j * np.pi * s.t)
    np.testing.assert_allclose(J, np.fft.fft(g, axis=1), atol=1e-12)


def test_nudft_phase_is_exact_for_large_times(orc):
    # the phase (f_lo + i df) t_n is evaluated exactly in rationals here
    rng = np.random.default_rng(5)
    t = np.sort(rng.uniform(7.0e4, 8.2e4, 12))
    x = rng.standard_normal(12)
    w = np.ones((1, 12))
    f_lo, df = -0.5 + 1.0 / 3.0, 1.0 / 262144.0
    bands = np.array([0, 1, 12345, 262143], dtype=np.int64)
    J = orc.nudft(t, x, w, f_lo, df, bands=bands)[0]
    for b, i in enumerate(bands):
        acc = 0j
        for n in range(12):
            ph = (Fraction(f_lo) + i * Fraction(df)) * Fraction(float(t[n]))
            r = float(ph - math.floor(ph))
            acc += x[n] * complex(math.cos(2 * math.pi * r), -math.sin(2 * math.pi * r))
        assert abs(J[b] - acc) < 1e-13


# --------------------------------------------------------------------------
# invariants the paper states
# --------------------------------------------------------------------------

def test_eigenvalues_in_unit_interval_and_trace(orc):
    # P5: 0 <= lambda <= 1 (Sec. 3.5); with R(B) = I the full spectrum sums to
    # tr R(A0) = 2 f_w N
    s = W.small_gapped()
    RA = orc.gpss_matrix(s.t, s.fw)
    ev, _ = orc.jacobi_eigh(RA)
    assert ev.min() > -1e-14 and ev.max() < 1 + 1e-14
    assert abs(ev.sum() - 2 * s.fw * s.N) < 1e-12
    j = W.scheme_jitter()
    L = orc.cholesky(orc.gpss_matrix(j.t, 0.5))
    evj, _ = orc.jacobi_eigh(orc.reduce(L, orc.gpss_matrix(j.t, 0.05)))
    assert evj.min() > -1e-13 and evj.max() < 1 + 1e-13


@pytest.mark.parametrize("scheme", ["jitter", "missing", "arithmetic", "uniform"])
def test_normalisation_and_variance_factor(orc, scheme):
    # P6: w_k^T R(B) w_l = 2 f_w delta_kl (Sec. 2.2), so the variance bound
    # factor V = (1/K^2) sum |w_k^T R(B) w_l|^2 = (2 f_w)^2 / K
    s = W.by_name(scheme)
    w, lam = orc.gpss_tapers(s.t, s.fmax, s.fw, s.K)
    G = w @ orc.gpss_matrix(s.t, s.fmax) @ w.T
    np.testing.assert_allclose(G, 2 * s.fw * np.eye(s.K), atol=1e-13)
    V = (G ** 2).sum() / s.K ** 2
    assert abs(V - (2 * s.fw) ** 2 / s.K) < 1e-14
    # and they solve the GEP: R(A0) w = lambda R(B) w
    RA, RB = orc.gpss_matrix(s.t, s.fw), orc.gpss_matrix(s.t, s.fmax)
    np.testing.assert_allclose(RA @ w.T, (RB @ w.T) * lam, atol=1e-12)
    # lambdas are the K largest generalized eigenvalues (LAPACK on the pencil)
    Lc = np.linalg.cholesky(RB)
    Li = np.linalg.inv(Lc)
    ref = np.linalg.eigvalsh(Li @ RA @ Li.T)[::-1][:s.K]
    np.testing.assert_allclose(lam, ref, atol=1e-12)


def test_parseval_on_lattice(orc):
    # P8: integer t, df = 1/M, M >= span: (1/M) sum_i |J_k(i)|^2 = sum_n |w_k x_n|^2
    s = W.small_gapped()
    M = 256
    w = np.random.default_rng(6).standard_normal((2, s.N))
    J = orc.nudft(s.t, s.x, w, -0.5, 1.0 / M, I=M)
    np.testing.assert_allclose((np.abs(J) ** 2).sum(1) / M, ((w * s.x) ** 2).sum(1), rtol=1e-13)


def test_symmetry_real_data(orc):
    # P9: real x and w, f_lo = -1/2, df = 1/I, integer t: P_{I-i} = P_i
    s = W.small_gapped()
    out = orc.m2nufft(s.t, s.x, s.fmax, s.fw, s.K, s.f_lo, s.df, s.I, with_ehat=False)
    P = out["P"]
    np.testing.assert_allclose(P[1:], P[1:][::-1], rtol=1e-12, atol=1e-15)


def test_ehat_zero_on_lattice_and_at_nominal_band(orc):
    # P4 (Appendix B): on the lattice with f_max = 1/2, R(B) = I and Ehat = 0
    s = W.small_gapped()
    out = orc.m2nufft(s.t, s.x, s.fmax, s.fw, s.K, s.f_lo, s.df, s.I)
    assert np.abs(out["E"]).max() < 1e-14
    np.testing.assert_allclose(out["D"], 2 * s.fw, rtol=1e-13)
    # P10: at df_i = 0 the shifted taper is the nominal one, D = 2 f_w, Ehat = 0
    for name in ["jitter", "missing", "arithmetic"]:
        j = W.by_name(name)
        w, lam = orc.gpss_tapers(j.t, j.fmax, j.fw, j.K)
        E, D = orc.ehat(j.t, w, lam, j.fmax, j.fw, -0.5, 1.0 / 64, bands=np.array([32]))
        assert abs(E[0]) < 1e-13
        np.testing.assert_allclose(D[:, 0], 2 * j.fw, rtol=1e-12)
        E_all, _ = orc.ehat(j.t, w, lam, j.fmax, j.fw, -0.5, 1.0 / 64, I=64)
        assert E_all.min() >= 0.0


def test_ehat_equals_exact_suboptimality_on_lattice(orc):
    # P4/P12 brute force: per-band GEP R(A_i) w = lambda R(B) w on a tiny lattice
    # has the same eigenvalues as at A0, so the exact E_i is 0 like Ehat
    s = W.small_gapped()
    t = s.t[:40]
    fw, K = 0.1, 3
    w, lam = orc.gpss_tapers(t, 0.5, fw, K)
    for fci in [0.0, 0.1, -0.23, 0.4]:
        RAi = orc.band_matrix(t, fci, fw)     # R(B) = I here
        ev = np.linalg.eigvalsh(RAi)[::-1][:K]
        np.testing.assert_allclose(ev, lam, atol=1e-13)


def test_ehat_nonlattice_matches_rayleigh_quotient(orc):
    # Appendix B: lambda_hat = (E w)^* R(A_i) (E w) / (E w)^* R(B) (E w), using
    # the complex band matrix directly (independent of the 2 f_w lambda form)
    s = W.scheme_missing()
    w, lam = orc.gpss_tapers(s.t, s.fmax, s.fw, s.K)
    RB = orc.gpss_matrix(s.t, s.fmax)
    bands = np.array([5, 20, 40, 60], dtype=np.int64)
    E, D = orc.ehat(s.t, w, lam, s.fmax, s.fw, -0.5, 1.0 / 64, bands=bands)
    for b, i in enumerate(bands):
        fci = -0.5 + i / 64.0
        Ei = np.exp(2j * np.pi * fci * s.t)
        RAi = orc.band_matrix(s.t, fci, s.fw)
        lh = []
        for k in range(s.K):
            z = Ei * w[k]
            lh.append((z.conj() @ RAi @ z).real / (z.conj() @ RB @ z).real)
        np.testing.assert_allclose(D[:, b], [(Ei * w[k]).conj() @ RB @ (Ei * w[k]) for k in range(s.K)],
                                   rtol=1e-12)
        assert abs(E[b] - np.mean(np.abs(lam - np.array(lh)))) < 1e-12


def test_ehat_d_is_spectral_window_integral(orc):
    # Appendix B with R(B) written as an integral over the signal band:
    # D_k(i) = int_{df_i - f_max}^{df_i + f_max} |W_k(f)|^2 df, W_k the taper's
    # spectral window.  Brute-force quadrature in f (composite Gauss-Legendre,
    # W_k summed directly) against the oracle's quadratic form, on the paper's
    # 5n/6 and arithmetic schemes and at a band count whose window ends inside
    # a band spacing (f_max = 0.3)
    xg, wg = np.polynomial.legendre.leggauss(40)
    for s, fmax in ((W.scheme_missing(), 0.5), (W.scheme_arithmetic(), 0.5), (W.scheme_missing(), 0.3)):
        if fmax == 0.5:
            w, lam = orc.gpss_tapers(s.t, fmax, s.fw, s.K)
        else:   # R(B) of f_max = 0.3 is numerically singular on this grid: any tapers
            w = np.random.default_rng(7).standard_normal((s.K, s.N)) * 0.05
            lam = np.full(s.K, 0.9)
        bands = np.array([0, 17, 40, 63], dtype=np.int64)
        _, D = orc.ehat(s.t, w, lam, fmax, s.fw, -0.5, 1.0 / 64, bands=bands)
        for b, i in enumerate(bands):
            fc = -0.5 + i / 64.0
            edges = np.linspace(fc - fmax, fc + fmax, 201)
            f = (0.5 * (edges[:-1] + edges[1:])[:, None] + 0.5 * np.diff(edges)[:, None] * xg).ravel()
            wt = (0.5 * np.diff(edges)[:, None] * wg).ravel()
            Wf = np.exp(-2j * np.pi * np.outer(f, s.t)) @ w.T          # [nf, K]
            Dq = (wt[:, None] * np.abs(Wf) ** 2).sum(axis=0)
            np.testing.assert_allclose(D[:, b], Dq, rtol=1e-12)


def test_unbiased_for_white_noise(orc):
    # P7 (Sec. 3.3): E[P(A_i)] = 2 f_w sigma^2 for white noise on the lattice
    s = W.small_gapped()
    w, lam = orc.gpss_tapers(s.t, s.fmax, s.fw, s.K)
    bands = np.arange(0, s.I, 8, dtype=np.int64)
    acc = []
    for m in range(300):
        x = W.white_noise(s.N, 7000 + m, sigma=1.3)
        acc.append(orc.psd(orc.nudft(s.t, x, w, s.f_lo, s.df, bands=bands)).mean())
    acc = np.array(acc)
    target = 2 * s.fw * 1.3 ** 2
    se = acc.std(ddof=1) / math.sqrt(len(acc))
    assert abs(acc.mean() - target) < 4 * se


def test_sinusoid_peak_band(orc):
    # P14: the strongest sinusoid (f = 0.05) dominates the bands around +-0.05
    s = W.small_gapped()
    out = orc.m2nufft(s.t, s.x, s.fmax, s.fw, s.K, s.f_lo, s.df, s.I, with_ehat=False)
    top = np.argmax(out["P"])
    fc = s.f_lo + top * s.df
    assert abs(abs(fc) - 0.05) <= s.fw


# --------------------------------------------------------------------------
# Thomson F-test (Sec. 3.6)
# --------------------------------------------------------------------------
def _ftest_levels():
    import os
    rows = []
    path = os.path.join(os.path.dirname(__file__), "golden", "ftest_levels.txt")
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                p, K = line.split()[:2]
                rows.append((float(p), int(K)))
    return rows


def test_f_critical_matches_inverse_f_distribution(orc):
    # the paper's levels (p = 0.05, 0.01, 1/240, 1/688; F(2, 10)) against the
    # library's inverse survival function of the F distribution
    import scipy.stats as ss
    rows = _ftest_levels()
    assert len(rows) == 4
    for p, K in rows:
        Fp = orc.f_critical(p, K)
        assert abs(Fp - ss.f.isf(p, 2, 2 * K - 2)) < 1e-9 * Fp
        assert abs(ss.f.sf(Fp, 2, 2 * K - 2) - p) < 1e-12
    # ordering of the paper's three lines: 0.05 < 0.01 < Rayleigh level
    vals = [orc.f_critical(p, K) for p, K in rows]
    assert vals[0] < vals[1] < vals[2] < vals[3]


def test_ftest_amplitude_and_residual_are_least_squares(orc):
    # C_i is the least-squares amplitude of J_k(i) ~ C W_k(0), and the
    # denominator of F is that fit's residual: checked with lstsq per band
    rng = np.random.default_rng(91)
    K, N, nb = 6, 40, 17
    w = rng.standard_normal((K, N))
    J = rng.standard_normal((K, nb)) + 1j * rng.standard_normal((K, nb))
    F, C = orc.ftest(J, w)
    W0 = w.sum(axis=1).astype(np.complex128)
    for i in range(nb):
        c, res, _, _ = np.linalg.lstsq(W0[:, None], J[:, i], rcond=None)
        assert abs(C[i] - c[0]) < 1e-12 * max(1.0, abs(c[0]))
        ref = abs(c[0]) ** 2 * (K - 1) * np.real(np.vdot(W0, W0)) / res[0]
        assert abs(F[i] - ref) < 1e-10 * ref


def test_ftest_exact_line_and_scale_invariance(orc):
    rng = np.random.default_rng(92)
    K, N = 5, 30
    w = rng.standard_normal((K, N))
    W0 = w.sum(axis=1)
    J = np.outer(W0, [1.5 - 0.5j, -2.0 + 0.25j])    # exactly proportional to W(0)
    F, C = orc.ftest(J, w)
    assert np.all(F > 1e25)                          # residual at rounding level (or exactly 0: inf)
    assert np.allclose(C, [1.5 - 0.5j, -2.0 + 0.25j], rtol=1e-14, atol=0)
    Jn = rng.standard_normal((K, 9)) + 1j * rng.standard_normal((K, 9))
    F1, _ = orc.ftest(Jn, w)
    F2, _ = orc.ftest((3.0 - 4.0j) * Jn, 7.0 * w)   # a complex gain and a taper scale
    assert np.allclose(F1, F2, rtol=1e-12, atol=0)


def test_ftest_detects_a_line_on_the_lattice(orc):
    # a sinusoid on a band centre in white noise: its band is the largest F
    # and exceeds the Rayleigh level 1/N
    N, K, NW = 600, 6, 3.5
    t = np.arange(N, dtype=np.float64)
    fw = NW / N
    w, _ = orc.gpss_tapers(t, 0.5, fw, K)
    I = 1200
    f_lo, df = -0.5, 1.0 / I
    i0 = 900                                          # f = 0.25
    rng = np.random.default_rng(93)
    x = rng.standard_normal(N) + 0.6 * np.cos(2 * np.pi * (f_lo + i0 * df) * t + 0.3)
    bands = np.arange(620, 1180, dtype=np.int64)      # f in (0.017, 0.483): 2 f > f_w
    F, _ = orc.ftest(orc.nudft(t, x, w, f_lo, df, bands=bands), w)
    assert bands[np.argmax(F)] == i0
    assert F.max() > orc.f_critical(1.0 / N, K)


def test_ftest_null_distribution(orc):
    # white Gaussian noise: F ~ F(2, 2K-2) (Sec. 3.6).  Bands 4 f_w apart
    # are nearly independent; the exceedance rate at p = 0.05 and the mean
    # nu / (nu - 2) are checked against binomial and sampling errors
    N, K, NW = 512, 6, 3.5
    t = np.arange(N, dtype=np.float64)
    fw = NW / N
    w, _ = orc.gpss_tapers(t, 0.5, fw, K)
    I = N
    f_lo, df = -0.5, 1.0 / I
    step = int(math.ceil(4 * fw / df))
    bands = np.arange(N // 2 + step, N - step, step, dtype=np.int64)   # 0 < f < 1/2
    rng = np.random.default_rng(94)
    Fs = []
    for _ in range(80):
        x = rng.standard_normal(N)
        Fs.append(orc.ftest(orc.nudft(t, x, w, f_lo, df, bands=bands), w)[0])
    Fs = np.concatenate(Fs)
    n = Fs.size
    rate = np.mean(Fs > orc.f_critical(0.05, K))
    assert abs(rate - 0.05) < 4 * math.sqrt(0.05 * 0.95 / n)
    nu = 2 * K - 2
    mean_ref = nu / (nu - 2)
    sd_ref = math.sqrt(2 * nu ** 2 * (2 + nu - 2) / (2 * (nu - 2) ** 2 * (nu - 4)))
    assert abs(Fs.mean() - mean_ref) < 4 * sd_ref / math.sqrt(n)


def test_nudft_freqs_matches_progression_and_fft(orc):
    """Eigencoefficients at a list of band centres: equal to the pinned
    progression form at the same centres (any order, repeats allowed), and on
    a uniform grid equal to numpy's FFT at the DFT frequencies."""
    s = W.small_gapped()
    w, _ = orc.gpss_tapers(s.t, s.fmax, s.fw, 3, method="jacobi")
    rng = np.random.default_rng(3)
    bands = rng.integers(0, s.I, size=40)
    J0 = orc.nudft(s.t, s.x, w, s.f_lo, s.df, bands=bands)
    J1 = orc.nudft_freqs(s.t, s.x, w, s.f_lo + bands * s.df)
    assert np.abs(J1 - J0).max() < 1e-12 * np.abs(J0).max()
    N = 64
    t = np.arange(N, dtype=np.float64)
    x = rng.standard_normal(N)
    J2 = orc.nudft_freqs(t, x, np.ones((1, N)), np.arange(N) / N)
    assert np.abs(J2[0] - np.fft.fft(x)).max() < 1e-12 * np.abs(np.fft.fft(x)).max()


# --------------------------------------------------------------------------
# Rank-revealing reduction for a numerically singular R(B)
# --------------------------------------------------------------------------

def test_rr_full_rank_is_the_gep(orc):
    # a well-conditioned grid keeps every sample: the plain GEP's tapers
    s = W.jitter_stress(n=200, seed=8, K=4)
    w, lam, S = orc.gpss_tapers_rr(s.t, s.fmax, 4.0 / 200, 4, 1e-12)
    w0, lam0 = orc.gpss_tapers(s.t, s.fmax, 4.0 / 200, 4)
    assert S.shape[0] == s.N
    assert np.array_equal(w, w0) and np.array_equal(lam, lam0)


@pytest.mark.parametrize("tau", [1e-8, 1e-6])
def test_rr_schur_complement_bound(orc, tau):
    # t = 5n/6 (R(B) numerically singular): the kept block is positive
    # definite and the Schur complement of the left-out samples, formed
    # independently with a dense solve, is bounded by the largest remaining
    # pivot, which is below tau * 2 f_max
    s = W.scheme_missing(L=480, n_keep=400, seed=3)
    S, maxrem = orc.rr_select(s.t, s.fmax, tau)
    R = orc.gpss_matrix(s.t, s.fmax)
    out = np.setdiff1d(np.arange(s.N), S)
    assert 0 < S.shape[0] < s.N and maxrem < tau * 2 * s.fmax
    orc.cholesky(R[np.ix_(S, S)])                                 # positive definite
    Sc = R[np.ix_(out, out)] - R[np.ix_(out, S)] @ np.linalg.solve(R[np.ix_(S, S)], R[np.ix_(S, out)])
    assert np.abs(Sc).max() <= maxrem * (1 + 1e-6) + 1e-14
    assert abs(np.diag(Sc).max() - maxrem) <= 1e-6 * maxrem + 1e-14


def test_rr_near_duplicate_sample(orc):
    # a sample repeated 1e-7 later makes R(B) singular to rounding: one of the
    # pair is left out and the result is the GEP of the series without it
    s = W.jitter_stress(n=120, seed=9, K=4)
    t2 = np.sort(np.concatenate([s.t, [s.t[10] + 1e-7]]))
    w, lam, S = orc.gpss_tapers_rr(t2, s.fmax, 4.0 / 120, 4, 1e-8)
    _, lam0 = orc.gpss_tapers(s.t, s.fmax, 4.0 / 120, 4)
    assert S.shape[0] == s.N and (10 not in S or 11 not in S)
    np.testing.assert_allclose(lam, lam0, atol=1e-6)


def test_rr_taper_properties(orc):
    # tapers vanish off the kept samples, are R(B)-orthonormal with the full
    # R(B) (2 f_w delta_kl) and their lambda lie in [0, 1]
    for s in [W.scheme_arithmetic(seed=sd) for sd in (21, 30, 38, 43)]:   # plain GEP: NOT_PD
        w, lam, S = orc.gpss_tapers_rr(s.t, s.fmax, s.fw, s.K, 1e-8)
        out = np.setdiff1d(np.arange(s.N), S)
        assert np.all(w[:, out] == 0.0)
        G = w @ orc.gpss_matrix(s.t, s.fmax) @ w.T
        assert np.abs(G - 2 * s.fw * np.eye(s.K)).max() < 1e-8
        assert lam.min() >= -1e-12 and lam.max() <= 1 + 1e-12
