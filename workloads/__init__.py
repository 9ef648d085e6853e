"""Seeded synthetic gapped series shared by the oracle tests, the GPU tests and
the benchmark.

This module only draws random numbers and lays out sampling grids; it holds
none of the estimator's arithmetic (no GPSS matrices, tapers, transforms or
averages). Every generator takes an explicit seed and uses numpy's
``Generator(PCG64(seed))`` so that both sides of a parity test see the same
bytes.

Workloads (sizes follow the paper's problem statement, Table 3 step 1:
sampling times t_n, samples x(t_n), signal band B = [-f_max, f_max], K tapers,
nominal half-width f_w and I analysis bands with centres f_lo + i*df):

* ``small_gapped``      256-sample unit grid, exactly 51 indices dropped
                         (Bernoulli-exact 20 %), three sinusoids + white noise,
                         f_w = 4/256, K = 6, I = 512.
* ``gapped_20k``        20,480-sample unit grid, periodic 64-of-320 missing
                         blocks plus 5 % i.i.d. dropouts, AR(2) + 5 sinusoids,
                         f_w = 4/20480, K = 7, I = 2**18.
* ``gapped_82k``        the same scheme on 81,920 samples, K = 9,
                         f_w = 5/81920, I = 2**20.
* ``batched_series(s)`` one series of the 512-series batch: N log-uniform in
                         [1024, 16384], missing fraction U[5 %, 40 %],
                         Bernoulli-exact or periodic-block gaps, K in {3..9},
                         f_w = (K+1)/(2 L), I = 2**16.
* ``scheme_*``          the paper's four 50-point sampling schemes
                         (Section 4: uniform, jitter, missing data on 5n/6,
                         arithmetic) used as small non-lattice test cases.
* ``jitter_stress``     jittered unit grid t_n = n + z_n, z ~ N(0, 0.1^2),
                         whose signal-band matrix is dense.
* ``multiband``         band-pass sampled series for the sub-band partition:
                         t_n = 2.2 n + z_n, z ~ N(0, 0.4^2), f_max = 1/2 split
                         into [0, 1/4] and [1/4, 1/2] with nominal centres
                         1/8 and 3/8, f_w = 3.5 / span, K = 6, I relative band
                         centres per sub-band over |df_i| <= 1/8 - f_w; x is
                         one sinusoid in each sub-band plus white noise.  The
                         grid (density 1/2.2) is sparser than either
                         sub-band's Landau rate (1/2), so both matrices are well
                         conditioned (smallest eigenvalues 4e-2 and 7e-4 at
                         n = 512); aliasing on the coarse grid bounds the
                         concentrations (about 0.98 down to 0.87 for K = 6).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Series", "small_gapped", "gapped_20k", "gapped_82k", "gapped_scaled",
    "batched_series", "served_request", "poisson_arrivals", "scheme_uniform", "scheme_jitter", "scheme_missing",
    "scheme_arithmetic", "jitter_stress", "multiband", "SubBand", "white_noise", "by_name",
]


@dataclasses.dataclass
class Series:
    """One gapped series plus the analysis parameters that go with it."""
    name: str
    t: np.ndarray          # float64 [N], strictly increasing
    x: np.ndarray          # float64 [N]
    fmax: float            # signal band half-width
    fw: float              # nominal analysis band half-width
    K: int                 # number of tapers
    f_lo: float            # first band centre
    df: float              # band-centre spacing
    I: int                 # number of bands
    grid_len: int = 0      # length of the underlying unit grid (0 if none)

    @property
    def N(self) -> int:
        return int(self.t.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _sinusoids(rng, tt, amps, freqs):
    """Sum of A cos(2 pi f t + phi) with phases drawn from U[0, 2 pi)."""
    phases = rng.uniform(0.0, 2.0 * math.pi, size=len(amps))
    out = np.zeros_like(tt)
    for a, f, p in zip(amps, freqs, phases):
        out += a * np.cos(2.0 * math.pi * f * tt + p)
    return out


def _ar2(rng, n, r=0.95, theta=0.6 * math.pi, burn=1000):
    """AR(2) with poles r e^{+-j theta}, unit-variance innovations:
    y_i = a1 y_{i-1} + a2 y_{i-2} + e_i (recursive filter, zero start)."""
    from scipy.signal import lfilter
    a1, a2 = 2.0 * r * math.cos(theta), -r * r
    e = rng.standard_normal(n + burn)
    e[:2] = 0.0
    y = lfilter([1.0], [1.0, -a1, -a2], e)
    return y[burn:]


def _bernoulli_exact_keep(rng, L, n_drop):
    drop = rng.choice(L, size=n_drop, replace=False)
    keep = np.ones(L, dtype=bool)
    keep[drop] = False
    return np.nonzero(keep)[0]


def _periodic_then_random(rng, L, period, block, p_random):
    j = np.arange(L)
    keep = (j % period) < (period - block)
    keep &= rng.random(L) >= p_random
    return np.nonzero(keep)[0]


def small_gapped(seed: int = 0) -> Series:
    """256-point unit grid, 20 % Bernoulli-exact dropouts (205 observed)."""
    rng = _rng(seed)
    L = 256
    idx = _bernoulli_exact_keep(rng, L, int(round(0.2 * L)))
    tt = np.arange(L, dtype=np.float64)
    sig = _sinusoids(rng, tt, [1.0, 0.5, 0.2], [0.05, 0.17, 0.31])
    sig += rng.normal(0.0, 0.1, size=L)
    return Series("small_gapped", tt[idx].copy(), sig[idx].copy(), 0.5,
                  4.0 / L, 6, -0.5, 1.0 / 512, 512, L)


def _gapped_periodic(name, seed, L, K, fw, I):
    rng = _rng(seed)
    idx = _periodic_then_random(rng, L, 320, 64, 0.05)
    tt = np.arange(L, dtype=np.float64)
    sig = _ar2(rng, L)
    amps = 10.0 ** rng.uniform(-3.0, 0.0, size=5)
    freqs = rng.uniform(0.0, 0.5, size=5)
    sig += _sinusoids(rng, tt, amps, freqs)
    return Series(name, tt[idx].copy(), sig[idx].copy(), 0.5, fw, K, -0.5,
                  1.0 / I, I, L)


def gapped_20k(seed: int = 1) -> Series:
    return _gapped_periodic("gapped_20k", seed, 20480, 7, 4.0 / 20480, 2 ** 18)


def gapped_82k(seed: int = 2) -> Series:
    return _gapped_periodic("gapped_82k", seed, 81920, 9, 5.0 / 81920, 2 ** 20)


def gapped_scaled(L: int, K: int, I: int, seed: int = 11) -> Series:
    """The gapped_20k scheme at another grid length (smaller parity cases)."""
    return _gapped_periodic(f"gapped_{L}", seed, L, K, 4.0 / L, I)


def _batched_from_rng(rng, name, n_obs=None, I=2 ** 16) -> Series:
    if n_obs is None:
        n_obs = int(round(math.exp(rng.uniform(math.log(1024), math.log(16384)))))
    p = rng.uniform(0.05, 0.40)
    if rng.random() < 0.5:
        L = int(math.ceil(n_obs / (1.0 - p)))
        idx = _bernoulli_exact_keep(rng, L, L - n_obs)
    else:
        period = int(rng.integers(128, 1025))
        block = max(1, int(round(p * period)))
        L0 = int(math.ceil(n_obs * period / (period - block))) + period
        j = np.arange(L0)
        keep = np.nonzero((j % period) < (period - block))[0]
        surplus = keep.shape[0] - n_obs
        if surplus > 0:
            drop = rng.choice(keep.shape[0], size=surplus, replace=False)
            mask = np.ones(keep.shape[0], dtype=bool)
            mask[drop] = False
            keep = keep[mask]
        idx = keep
        L = int(idx[-1]) + 1
    K = int(rng.integers(3, 10))
    tt = np.arange(L, dtype=np.float64)
    sig = _ar2(rng, L)
    amps = 10.0 ** rng.uniform(-3.0, 0.0, size=5)
    freqs = rng.uniform(0.0, 0.5, size=5)
    sig += _sinusoids(rng, tt, amps, freqs)
    return Series(name, tt[idx].copy(), sig[idx].copy(), 0.5,
                  (K + 1) / (2.0 * L), K, -0.5, 1.0 / I, I, L)


def batched_series(s: int) -> Series:
    """Series s of the 512-series batch (seed 3,000,000 + s)."""
    return _batched_from_rng(_rng(3_000_000 + s), f"batched_{s}")


def served_request(r: int) -> Series:
    """Request r of the served workload (seed 4,000,000 + r): with
    probability 0.02 a long series (N_obs = 65,536, I = 2**20), otherwise a
    series of the batched distribution."""
    rng = _rng(4_000_000 + r)
    if rng.random() < 0.02:
        return _batched_from_rng(rng, f"served_{r}_long", n_obs=65536, I=2 ** 20)
    return _batched_from_rng(rng, f"served_{r}")


def poisson_arrivals(rate: float, seconds: float, seed: int = 4) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate on [0, seconds)."""
    rng = _rng(seed)
    n = int(rate * seconds * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    return t[t < seconds]


# --- the paper's four 50-point sampling schemes (Section 4) ----------------

def _scheme(name, t, seed, fw=0.05, K=4, I=64):
    rng = _rng(seed)
    x = rng.standard_normal(t.shape[0])
    return Series(name, t, x, 0.5, fw, K, -0.5, 1.0 / I, I, 0)


def scheme_uniform(seed: int = 10) -> Series:
    return _scheme("uniform", np.arange(1, 51, dtype=np.float64), seed)


def scheme_jitter(seed: int = 11, n: int = 50, sigma: float = 0.1) -> Series:
    rng = _rng(seed + 1000)
    t = np.arange(1, n + 1, dtype=np.float64) + rng.normal(0.0, sigma, n)
    t.sort()
    return _scheme("jitter", t, seed)


def scheme_missing(seed: int = 12, L: int = 60, n_keep: int = 50) -> Series:
    """t_n = 5n/6 for n = 1..L with L - n_keep samples removed at random
    (the paper's scheme has L = 60, n_keep = 50)."""
    rng = _rng(seed + 1000)
    n = np.arange(1, L + 1, dtype=np.float64)
    keep = np.sort(rng.choice(L, size=n_keep, replace=False))
    return _scheme("missing", 5.0 * n[keep] / 6.0, seed)


def scheme_arithmetic(seed: int = 13, n: int = 50) -> Series:
    """t_n = 1 + a (n-1) + b (n-1)(n-2)/2 with a ~ U[0.5, 1], b ~ U[0, 0.02].

    The paper leaves the law of a and b open; this draw keeps the 50 points
    inside roughly the same 50 s span as the other schemes.
    """
    rng = _rng(seed + 1000)
    a = rng.uniform(0.5, 1.0)
    b = rng.uniform(0.0, 0.02)
    m = np.arange(n, dtype=np.float64)
    t = 1.0 + a * m + b * m * (m - 1.0) / 2.0
    return _scheme("arithmetic", t, seed)


def jitter_stress(n: int = 16384, seed: int = 5, K: int = 7,
                  I: int = 2 ** 15) -> Series:
    rng = _rng(seed)
    t = np.arange(n, dtype=np.float64) + rng.normal(0.0, 0.1, n)
    t.sort()
    x = rng.standard_normal(n)
    return Series(f"jitter_{n}", t, x, 0.5, 4.0 / n, K, -0.5, 1.0 / I, I, 0)


@dataclasses.dataclass
class SubBand:
    """One sub-band f_min <= |f| <= f_max with its nominal band centre."""
    fmin: float
    fmax: float
    fc0: float


def multiband(n: int = 1024, seed: int = 21, I: int = 4096):
    """(Series, [SubBand]) of the band-pass sampled workload; the Series'
    f_lo, df, I are the relative band centres shared by both sub-bands."""
    rng = _rng(seed)
    t = 2.2 * np.arange(n, dtype=np.float64) + rng.normal(0.0, 0.4, n)
    t.sort()
    span = t[-1] - t[0]
    fw = 3.5 / span
    half = 0.125 - fw
    x = (np.cos(2.0 * np.pi * 0.1 * t + 0.3) + np.cos(2.0 * np.pi * 0.41 * t + 1.1)
         + rng.standard_normal(n))
    s = Series(f"multiband_{n}", t, x, 0.5, fw, 6, -half, 2.0 * half / I, I, 0)
    return s, [SubBand(0.0, 0.25, 0.125), SubBand(0.25, 0.5, 0.375)]


def white_noise(n: int, seed: int, sigma: float = 1.0) -> np.ndarray:
    return _rng(seed).normal(0.0, sigma, n)


def by_name(name: str) -> Series:
    table = {
        "small_gapped": small_gapped, "gapped_20k": gapped_20k,
        "gapped_82k": gapped_82k, "uniform": scheme_uniform,
        "jitter": scheme_jitter, "missing": scheme_missing,
        "arithmetic": scheme_arithmetic,
    }
    return table[name]()
