"""Pins of the oracle's interpolated-DPSS tapers (Table 3 step 3, the branch for
a nominal band centred at 0: uniform-grid DPSS, cubic spline, R(B) scale).

On a gap-free uniform grid the branch must return the GPSS tapers themselves
(the full-band oracle, pinned to scipy's DPSS in test_oracle_pins.py); the
scale is checked as an integral of the spectral window, not as the matrix
product the oracle uses; and on a slightly jittered grid the interpolated
tapers approximate the GPSS tapers of that grid, the paper's premise.
"""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("h,t0,N,NW", [(1.0, 0.0, 160, 2.5), (1.5, 3.0, 200, 3.0), (0.25, -7.0, 96, 2.0)])
def test_idpss_equals_gpss_on_uniform_grids(orc, h, t0, N, NW):
    t = t0 + h * np.arange(N)
    fmax = 0.5 / h
    fw = NW / (N * h)
    K = 4
    w, lam = orc.idpss_tapers(t, fmax, fw, K)
    w0, lam0 = orc.gpss_tapers(t, fmax, fw, K, method="jacobi")
    assert np.abs(lam - lam0).max() < 1e-12
    assert np.abs(w - w0).max() < 1e-9 * np.abs(w0).max()


def test_idpss_scale_as_spectral_window_integral(orc):
    """int_{-f_max}^{f_max} |W_k(f)|^2 df = 2 f_w with W_k(f) = sum_n w_k(t_n)
    e^{-j 2 pi f t_n}, by dense Gauss-Legendre in f; and the sign reading."""
    s = W.scheme_jitter(n=80, sigma=0.2)
    fw = 3.0 / (s.t[-1] - s.t[0])
    w, _ = orc.idpss_tapers(s.t, 0.5, fw, 4)
    x, g = np.polynomial.legendre.leggauss(3000)
    f = 0.5 * x
    Wf = np.exp(-2j * np.pi * np.outer(f, s.t)) @ w.T
    q = 0.5 * (g[:, None] * np.abs(Wf) ** 2).sum(axis=0)
    assert np.abs(q - 2 * fw).max() < 1e-12
    tbar = 0.5 * (s.t[0] + s.t[-1])
    span = s.t[-1] - s.t[0]
    for k in range(4):
        s1, s2 = w[k].sum(), ((tbar - s.t) * w[k]).sum() / span
        assert (s1 if abs(s1) >= abs(s2) else s2) > 0


def test_idpss_approximates_gpss_on_jittered_grids(orc):
    """The interpolated tapers approach the GPSS tapers of the same grid as
    the jitter shrinks (error roughly proportional to the jitter)."""
    errs = []
    for sigma in (0.1, 0.01, 0.001):
        s = W.scheme_jitter(n=120, sigma=sigma)
        fw = 2.5 / (s.t[-1] - s.t[0])
        w, _ = orc.idpss_tapers(s.t, 0.5, fw, 3)
        w0, _ = orc.gpss_tapers(s.t, 0.5, fw, 3, method="jacobi")
        errs.append(np.abs(w - w0).max() / np.abs(w0).max())
    assert errs[2] < 0.02 and errs[2] < errs[1] < errs[0]


def test_natural_spline_end_conditions_and_library(orc):
    # the oracle's natural cubic spline: it interpolates the knots, reproduces
    # linear functions, has zero second derivative at both ends (central
    # second differences of a cubic are exact, extrapolated linearly to the
    # end knot), and equals scipy's natural CubicSpline on non-uniform knots
    from scipy.interpolate import CubicSpline
    rng = np.random.default_rng(77)
    u = np.cumsum(rng.uniform(0.5, 1.5, 40))
    v = rng.standard_normal((3, 40))
    S = lambda x: orc.natural_spline(u, v, np.atleast_1d(np.asarray(x, dtype=np.float64)))
    np.testing.assert_allclose(S(u), v, atol=1e-13)
    lin = 0.3 * u - 1.7
    np.testing.assert_allclose(orc.natural_spline(u, lin, u + 0.1)[0], 0.3 * (u + 0.1) - 1.7, atol=1e-12)
    x = np.linspace(u[0], u[-1], 2001)
    np.testing.assert_allclose(S(x), CubicSpline(u, v.T, bc_type="natural")(x).T, atol=1e-12)
    for a, h in ((u[0], (u[1] - u[0]) / 8), (u[-1], -(u[-1] - u[-2]) / 8)):
        p = S(a + h * np.arange(4)).T            # [4, 3]
        d2_1 = (p[0] - 2 * p[1] + p[2]) / h ** 2  # S'' at a + h
        d2_2 = (p[1] - 2 * p[2] + p[3]) / h ** 2  # S'' at a + 2 h
        assert np.abs(2 * d2_1 - d2_2).max() < 1e-7 * max(1.0, np.abs(d2_1).max())
