"""CPU FP64 oracle of the M2NuFFT estimator (arXiv 2407.01943).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
package and shares no code with it.

The arithmetic lives in ``m2n_oracle.c`` (plain C, FP64, OpenMP), built into
``liboracle.so`` by ``oracle/build.py``; this module marshals numpy arrays and
adds the two one-line steps that are clearer in numpy:

* ``psd``: P(A_i) = sum_k d_k |J_k(A_i)|^2 with d_k = 1/K (Sec. 3.2, the
  estimator of the integrated spectrum; Table 3 step 5);
* ``ftest``, ``f_critical``: the Thomson F-statistic from the eigencoefficients
  and the critical value of F(2, 2K-2) (Sec. 3.6);
* ``m2nufft``: Table 3 steps 3 (GEP branch), 4 and 5 in order;
* ``nudft_freqs``: eigencoefficients at an arbitrary list of band centres;
* ``idpss_tapers``: the interpolated-DPSS tapers of Table 3 step 3 (fc0 = 0):
  uniform-grid DPSS (this oracle's GEP on the gap-free lattice), natural cubic
  spline to t (or_natural_spline), R(B) normalisation;
* ``subband_tapers``, ``subband_eigcoeffs``, ``fix_phase``: one sub-band of
  the multiband partition (Sec. 2.4, Sec. 3.1-3.2): complex tapers of the
  nominal band at fc0 (or_reduce_herm, Hermitian Lanczos with or_jacobi on
  the tridiagonal) and their eigencoefficients on relative frequencies.

No eigen-solver, factorisation or triangular solve of a library is used: the
GEPs are the oracle's own Cholesky, Jacobi and Lanczos; numpy serves for
matrix products, sums and the elementwise steps.

Parity pins: tests/test_oracle_pins.py.  Readings where the paper is silent
(sign of a taper, the suboptimality estimate) are stated at each function.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, ERR_ARG, ERR_T_ORDER, ERR_NOT_PD, ERR_NO_CONVERGE = 0, -1, -2, -3, -4

_d = ctypes.POINTER(ctypes.c_double)
_l = ctypes.POINTER(ctypes.c_long)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_num_threads.restype = ctypes.c_int
        L.or_num_threads.argtypes = []
        L.or_set_threads.restype = None
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_validate.restype = ctypes.c_int
        L.or_validate.argtypes = [_d, ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.or_sinpi.restype = ctypes.c_double
        L.or_sinpi.argtypes = [ctypes.c_double]
        L.or_gpss_matrix.restype = None
        L.or_gpss_matrix.argtypes = [_d, ctypes.c_long, ctypes.c_double, _d]
        L.or_band_matrix.restype = None
        L.or_band_matrix.argtypes = [_d, ctypes.c_long, ctypes.c_double, ctypes.c_double, _d, _d]
        L.or_subband_matrix.restype = None
        L.or_subband_matrix.argtypes = [_d, ctypes.c_long, ctypes.c_double, ctypes.c_double, _d]
        L.or_apply_sinc.restype = None
        L.or_apply_sinc.argtypes = [_d, ctypes.c_long, ctypes.c_double, _d, ctypes.c_long, _d]
        L.or_cholesky.restype = ctypes.c_long
        L.or_cholesky.argtypes = [_d, ctypes.c_long]
        L.or_reduce.restype = None
        L.or_reduce.argtypes = [_d, _d, ctypes.c_long, _d]
        L.or_jacobi.restype = ctypes.c_int
        L.or_jacobi.argtypes = [_d, ctypes.c_long, _d, _d, ctypes.c_int]
        L.or_lanczos.restype = ctypes.c_int
        L.or_lanczos.argtypes = [_d, ctypes.c_long, ctypes.c_double, _d, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_double, _d, _d,
                                 ctypes.c_uint64, ctypes.c_int]
        L.or_reduce_herm.restype = None
        L.or_reduce_herm.argtypes = [_d, _d, _d, ctypes.c_long, _d, _d]
        L.or_solve_LT.restype = None
        L.or_solve_LT.argtypes = [_d, ctypes.c_long, _d, ctypes.c_long]
        L.or_natural_spline.restype = None
        L.or_natural_spline.argtypes = [_d, ctypes.c_long, _d, ctypes.c_long, _d, ctypes.c_long, _d]
        L.or_rr_select.restype = ctypes.c_long
        L.or_rr_select.argtypes = [_d, ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_int), _d]
        L.or_fft.restype = None
        L.or_fft.argtypes = [_d, _d, ctypes.c_long, ctypes.c_int]
        L.or_apply_sinc_toeplitz.restype = ctypes.c_int
        L.or_apply_sinc_toeplitz.argtypes = [_d, ctypes.c_long, ctypes.c_double, _d, ctypes.c_long, _d]
        L.or_gpss_tapers.restype = ctypes.c_long
        L.or_gpss_tapers.argtypes = [_d, ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, _d, _d]
        L.or_nudft.restype = None
        L.or_nudft.argtypes = [_d, _d, _d, ctypes.c_long, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, _l, ctypes.c_long, _d, _d]
        L.or_ehat_direct.restype = None
        L.or_ehat_direct.argtypes = [_d, _d, _d, ctypes.c_long, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double, _l,
                                     ctypes.c_long, _d, _d]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_d)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    """OpenMP threads for the oracle's parallel loops (timing only)."""
    lib().or_set_threads(int(n))


def validate(t, fmax, fw, K):
    t = _f64(t)
    return lib().or_validate(_p(t), t.shape[0], fmax, fw, K)


def sinpi(u: float) -> float:
    """sin(pi u) with exact zeros at integers (argument reduction by 2)."""
    return lib().or_sinpi(float(u))


def gpss_matrix(t, f):
    """R_{nm} = sin(2 pi f (t_n - t_m)) / (pi (t_n - t_m)); diagonal 2 f.

    With f = f_max this is R(B) (Sec. 2.1); with f = f_w it is R(A0) for a
    band centred at 0 (Sec. 3.2).
    """
    t = _f64(t)
    N = t.shape[0]
    R = np.empty((N, N))
    lib().or_gpss_matrix(_p(t), N, float(f), _p(R))
    return R


def band_matrix(t, fc, fw):
    """Complex R(A) of the band |f - fc| <= fw (Sec. 2.3)."""
    t = _f64(t)
    N = t.shape[0]
    re, im = np.empty((N, N)), np.empty((N, N))
    lib().or_band_matrix(_p(t), N, float(fc), float(fw), _p(re), _p(im))
    return re + 1j * im


def subband_matrix(t, fmin, fmax):
    """Real R(B^q) of the sub-band f_min <= |f| <= f_max (Sec. 2.4): the
    integral of e^{j 2 pi f tau} over [-f_max, -f_min] and [f_min, f_max]."""
    t = _f64(t)
    N = t.shape[0]
    R = np.empty((N, N))
    lib().or_subband_matrix(_p(t), N, float(fmin), float(fmax), _p(R))
    return R


def apply_sinc(t, f, V):
    """R(f) @ V without storing R(f) (V is N x nv)."""
    t = _f64(t)
    V = _f64(V)
    squeeze = V.ndim == 1
    if squeeze:
        V = V[:, None].copy()
    Y = np.empty_like(V)
    lib().or_apply_sinc(_p(t), t.shape[0], float(f), _p(V), V.shape[1], _p(Y))
    return Y[:, 0] if squeeze else Y


def cholesky(A):
    A = _f64(A).copy()
    st = lib().or_cholesky(_p(A), A.shape[0])
    if st < 0:
        raise OracleError(ERR_NOT_PD, f"cholesky (pivot {-st - 1})")
    return A


def reduce(L, RA):
    L, RA = _f64(L), _f64(RA)
    C = np.empty_like(RA)
    lib().or_reduce(_p(L), _p(RA), L.shape[0], _p(C))
    return C


def jacobi_eigh(A, max_sweeps=100):
    """Eigen-decomposition by cyclic Jacobi; eigenvalues descending."""
    A = _f64(A).copy()
    N = A.shape[0]
    ev, V = np.empty(N), np.empty((N, N))
    st = lib().or_jacobi(_p(A), N, _p(ev), _p(V), max_sweeps)
    if st < 0:
        raise OracleError(st, "jacobi")
    return ev, V


def is_lattice(t, fmax):
    """Every t_n an integer and 2 f_max a positive integer (R(B) = 2 f_max I)."""
    t = np.asarray(t, dtype=np.float64)
    c = 2.0 * float(fmax)
    return bool(np.all(t == np.rint(t)) and np.all(np.abs(t) <= 1e15) and c == round(c) and c >= 1.0)


def fft(x, sign=-1):
    """The oracle's own radix-2 FFT (length a power of two)."""
    x = np.asarray(x, dtype=np.complex128)
    re, im = _f64(x.real.copy()), _f64(x.imag.copy())
    lib().or_fft(_p(re), _p(im), x.shape[0], int(sign))
    return re + 1j * im


def apply_sinc_toeplitz(t, f, V):
    """R(f) @ V for integer t through the lattice Toeplitz convolution."""
    t = _f64(t)
    V = _f64(np.atleast_2d(V.T).T) if V.ndim == 1 else _f64(V)
    N, nv = V.shape
    Y = np.empty((N, nv))
    st = lib().or_apply_sinc_toeplitz(_p(t), N, float(f), _p(V), nv, _p(Y))
    if st < 0:
        raise OracleError(st, "apply_sinc_toeplitz")
    return Y


def gpss_tapers(t, fmax, fw, K, method="auto"):
    """The K largest solutions of R(A0) w = lambda R(B) w (Sec. 3.2), with
    w_k^T R(B) w_k = 2 f_w (Sec. 2.2) and the sign reading of fix_sign.

    method: "jacobi" (dense reduction + cyclic Jacobi), "lanczos", "lattice"
    (integer t and integer 2 f_max: R(B) = 2 f_max I, Lanczos with the
    Toeplitz operator, no N x N matrix) or "auto" (Jacobi up to N = 600, then
    "lattice" where it applies, else "lanczos").  Returns (w [K, N], lam [K]).
    """
    t = _f64(t)
    N = t.shape[0]
    if method == "auto" and N > 600 and is_lattice(t, fmax):
        method = "lattice"
    m = {"jacobi": 0, "lanczos": 1, "lattice": 2}.get(method, 0 if N <= 600 else 1)
    w, lam = np.empty((K, N)), np.empty(K)
    st = lib().or_gpss_tapers(_p(t), N, float(fmax), float(fw), int(K), m, _p(w), _p(lam))
    if st < 0:
        raise OracleError(st, "gpss_tapers")
    return w, lam


def rr_select(t, fmax, tau):
    """The samples a rank-revealing (diagonally pivoted) Cholesky of R(B)
    takes before every remaining Schur diagonal is below tau * 2 f_max
    (or_rr_select).  Returns (sorted indices, largest remaining diagonal)."""
    t = _f64(t)
    N = t.shape[0]
    sel = np.zeros(N, dtype=np.int32)
    mr = np.zeros(1)
    lib().or_rr_select(_p(t), N, float(fmax), float(tau), sel.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                       _p(mr))
    return np.nonzero(sel)[0], float(mr[0])


def gpss_tapers_rr(t, fmax, fw, K, tau, method="auto"):
    """GPSS tapers when R(B) may be numerically singular (the paper assumes it
    positive definite): the rank-revealing reduction keeps the samples S that
    a diagonally pivoted Cholesky of R(B) takes down to tau * 2 f_max, and
    solves the GEP of the sub-series t_S (R(B)_SS is positive definite with
    its pivots >= tau * 2 f_max; sign reading on t_S); the tapers are zero on
    the other samples.  Returns (w [K, N], lam [K], S)."""
    t = _f64(t)
    S, _ = rr_select(t, fmax, tau)
    if S.shape[0] < K:
        raise OracleError(ERR_ARG, "gpss_tapers_rr (rank below K)")
    wS, lam = gpss_tapers(t[S], fmax, fw, K, method=method)
    w = np.zeros((K, t.shape[0]))
    w[:, S] = wS      # the sign reading is that of the sub-series t_S
    return w, lam, S


def fix_sign(t, w):
    """The sign reading of the full-band tapers, for rows of w [K, N]: the larger
    in magnitude of sum w and sum (tbar - t) w / (t_N - t_1) is made positive."""
    t = _f64(t)
    tbar = 0.5 * (t[0] + t[-1])
    span = t[-1] - t[0] if t.shape[0] > 1 else 1.0
    out = np.array(w, dtype=np.float64)
    for k in range(out.shape[0]):
        s1 = out[k].sum()
        s2 = ((tbar - t) * out[k]).sum() / span
        if (s1 if abs(s1) >= abs(s2) else s2) < 0.0:
            out[k] = -out[k]
    return out


def natural_spline(u, v, x):
    """Natural cubic spline through (u_m, v_m) (rows of v share the knots),
    evaluated at x (or_natural_spline)."""
    u, x = _f64(u), _f64(x)
    v = _f64(np.atleast_2d(v))
    out = np.empty((v.shape[0], x.shape[0]))
    lib().or_natural_spline(_p(u), u.shape[0], _p(v), v.shape[0], _p(x), x.shape[0], _p(out))
    return out


def idpss_tapers(t, fmax, fw, K):
    """Interpolated-DPSS tapers (Table 3 step 3, the branch for fc0 = 0):
    (a) the DPSS of length N and half-bandwidth f_w D on the uniform grid
    u_m = t_1 + m D, D = (t_N - t_1) / (N - 1): the unit-norm GPSS tapers of
    the gap-free lattice 0..N-1 with f_max = 1/2 (R(B) = I there, so the GEP
    is the standard eigenproblem of the sinc matrix of half-bandwidth f_w D,
    whose eigenvectors are the DPSS), from this oracle's own GEP; (b) the
    natural cubic spline from u to t (``natural_spline``); (c) the scale that
    makes w^T R(B) w = 2 f_w, with R(B) from or_gpss_matrix; sign by
    ``fix_sign``.  Returns (w [K, N], lam [K]), lam the concentrations of the
    uniform-grid DPSS."""
    t = _f64(t)
    N = t.shape[0]
    D = (t[-1] - t[0]) / (N - 1)
    u = t[0] + D * np.arange(N)
    fwD = fw * D
    g, lam = gpss_tapers(np.arange(N, dtype=np.float64), 0.5, fwD, K)
    v = g / np.sqrt(2.0 * fwD)                  # unit-norm DPSS
    w = natural_spline(u, v, t)
    q = np.einsum("kn,nm,km->k", w, gpss_matrix(t, fmax), w)
    w = w * np.sqrt(2.0 * fw / q)[:, None]
    return fix_sign(t, w), np.atleast_1d(lam).copy()


def herm_lanczos(C, K, mmax=400, tol=1e-14, seed=0x5EED):
    """The K largest eigenpairs of a complex Hermitian matrix C by Lanczos
    with full re-orthogonalisation (two classical Gram-Schmidt passes), the
    Ritz pairs from or_jacobi on the real tridiagonal T (Hermitian Lanczos
    keeps alpha and beta real).  Convergence: |beta_m s_{m,k}| <= tol for
    the K wanted Ritz pairs, checked every 8 steps.  Returns (theta [K]
    descending, Z [N, K])."""
    C = np.asarray(C, dtype=np.complex128)
    N = C.shape[0]
    mmax = min(mmax, N)
    rng = np.random.default_rng(seed)
    q = rng.uniform(-1, 1, N) + 1j * rng.uniform(-1, 1, N)
    Q = np.zeros((mmax + 1, N), dtype=np.complex128)
    Q[0] = q / np.linalg.norm(q)
    alpha, beta = np.zeros(mmax), np.zeros(mmax)
    for j in range(mmax):
        z = C @ Q[j]
        alpha[j] = float(np.real(np.vdot(Q[j], z)))
        for _ in range(2):
            z -= Q[:j + 1].T @ (Q[:j + 1].conj() @ z)
        b = float(np.linalg.norm(z))
        beta[j] = b
        m = j + 1
        if m >= K and (m % 8 == 0 or m == mmax or b < 1e-300):
            T = np.diag(alpha[:m]) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
            th, S = jacobi_eigh(T)
            if np.max(np.abs(b * S[m - 1, :K])) <= tol or b < 1e-300 or m == mmax:
                return th[:K].copy(), Q[:m].T @ S[:, :K]
        if b < 1e-300:
            break
        Q[j + 1] = z / b
    raise OracleError(-4, "herm_lanczos")


def fix_phase(t, fc0, w):
    """Phase reading for complex tapers (the paper leaves it open): with
    v_n = w_n e^{-j 2 pi fc0 (t_n - tbar)}, tbar = (t_1 + t_N)/2,
    a = sum_n v_n and b = sum_n (tbar - t_n) v_n / (t_N - t_1), the one of
    larger modulus is made real and positive.  For fc0 = 0 and real tapers it
    is the sign reading of the full-band tapers.  w is [K, N] complex."""
    t = _f64(t)
    N = t.shape[0]
    tbar = 0.5 * (t[0] + t[-1])
    span = t[-1] - t[0] if N > 1 else 1.0
    u = fc0 * (t - tbar)
    demod = np.exp(-2j * np.pi * (u - np.round(u)))
    out = np.array(w, dtype=np.complex128)
    for k in range(out.shape[0]):
        v = out[k] * demod
        a = v.sum()
        b = ((tbar - t) * v).sum() / span
        key = a if abs(a) >= abs(b) else b
        if abs(key) > 0.0:
            out[k] *= np.conj(key) / abs(key)
    return out


def subband_tapers(t, fmin, fmax, fw, fc0, K):
    """The K largest solutions of R(A0) w = lambda R(B^q) w for the nominal
    band |f - fc0| <= fw inside the sub-band f_min <= |f| <= f_max (Sec. 2.4
    sub-band matrix; Sec. 3.2 GEP at the nominal band), scaled to
    w^* R(B^q) w = 2 f_w, phase by ``fix_phase``.

    Steps: R(B^q) = L L^T (real Cholesky, or_cholesky); R(A0) is complex
    Hermitian (Sec. 3.2, e^{j 2 pi fc0 tau} times the sinc of f_w), and
    C = L^{-1} R(A0) L^{-T} by triangular solves on its real and imaginary
    parts (or_reduce_herm; L is real, so L^{-T} is also L^{-*}); the top
    eigenpairs of C by Hermitian Lanczos (``herm_lanczos``);
    w = sqrt(2 f_w) L^{-T} z (or_solve_LT).  Returns (w [K, N] complex, lam [K]).
    """
    t = _f64(t)
    N = t.shape[0]
    L = cholesky(subband_matrix(t, fmin, fmax))
    RA = band_matrix(t, fc0, fw)
    Ar, Ai = _f64(RA.real.copy()), _f64(RA.imag.copy())
    Cr, Ci = np.empty((N, N)), np.empty((N, N))
    lib().or_reduce_herm(_p(L), _p(Ar), _p(Ai), N, _p(Cr), _p(Ci))
    th, Z = herm_lanczos(Cr + 1j * Ci, K)
    Xr, Xi = _f64(Z.real.copy()), _f64(Z.imag.copy())
    lib().or_solve_LT(_p(L), N, _p(Xr), K)
    lib().or_solve_LT(_p(L), N, _p(Xi), K)
    w = np.sqrt(2.0 * fw) * (Xr + 1j * Xi)
    return fix_phase(t, fc0, w.T), np.asarray(th, dtype=np.float64).copy()


def subband_eigcoeffs(t, x, w, f_lo, df, I=None, bands=None):
    """J_k(A_i) = sum_n conj(w_k(t_n)) x(t_n) e^{-j 2 pi df_i t_n} on the
    relative frequencies df_i = f_lo + i df of a sub-band (Sec. 3.2
    eigencoefficients with the shift of the nominal band; the NuFFT runs on
    the frequencies relative to fc0).  Direct summation; the phase df_i t_n
    is reduced modulo 1 before the exponential.  w is [K, N] complex."""
    t, x = _f64(t), _f64(x)
    w = np.atleast_2d(np.asarray(w, dtype=np.complex128))
    if bands is None:
        bands = np.arange(I, dtype=np.int64)
    bands = np.asarray(bands, dtype=np.int64)
    y = np.conj(w) * x[None, :]
    J = np.empty((w.shape[0], bands.shape[0]), dtype=np.complex128)
    for j, i in enumerate(bands):
        u = (f_lo + i * df) * t
        J[:, j] = y @ np.exp(-2j * np.pi * (u - np.round(u)))
    return J


def nudft_freqs(t, x, w, freqs):
    """J_k(i) = sum_n w_k(t_n) x(t_n) e^{-j 2 pi f_i t_n} at an arbitrary list
    of band centres f_i (Sec. 3.2 eigencoefficients; the band centres of an
    analysis need not be equally spaced), by direct summation with the phase
    f_i t_n reduced modulo 1 before the exponential.  Real tapers [K, N]."""
    t, x = _f64(t), _f64(x)
    w = np.atleast_2d(_f64(w))
    freqs = _f64(np.atleast_1d(freqs))
    y = w * x[None, :]
    J = np.empty((w.shape[0], freqs.shape[0]), dtype=np.complex128)
    for i, f in enumerate(freqs):
        u = f * t
        J[:, i] = y @ np.exp(-2j * np.pi * (u - np.round(u)))
    return J


def nudft(t, x, w, f_lo, df, I=None, bands=None):
    """J_k(i) = sum_n w_k(t_n) x_n exp(-j 2 pi (f_lo + i df) t_n) by direct
    summation (Sec. 3.2 eigencoefficients; Table 3 step 4).  Real tapers, so
    w^* = w.  Returns complex [K, len(bands)]."""
    t, x, w = _f64(t), _f64(x), _f64(np.atleast_2d(w))
    K, N = w.shape
    if bands is None:
        bands = np.arange(I, dtype=np.int64)
    bands = np.ascontiguousarray(bands, dtype=np.int64)
    nb = bands.shape[0]
    re, im = np.empty((K, nb)), np.empty((K, nb))
    lib().or_nudft(_p(t), _p(x), _p(w), N, K, float(f_lo), float(df),
                   bands.ctypes.data_as(_l), nb, _p(re), _p(im))
    return re + 1j * im


def psd(J, weights=None):
    """P(A_i) = sum_k d_k |J_k(A_i)|^2, d_k = 1/K unless given (Sec. 3.2)."""
    K = J.shape[0]
    d = np.full(K, 1.0 / K) if weights is None else np.asarray(weights, dtype=np.float64)
    return (d[:, None] * np.abs(J) ** 2).sum(axis=0)


def ftest(J, w):
    """Thomson F-statistic of every band (Sec. 3.6, "Thomson F-test for
    Nonuniform Signal", Eq. (f_stat) and the amplitude estimate after it):
        W_k(0) = sum_n w_k(t_n)               (the tapers' DC gains),
        C_i    = sum_k J_k(i) W_k(0) / sum_k W_k(0)^2,
        F_i    = |C_i|^2 (K - 1) sum_k W_k(0)^2 / sum_k |J_k(i) - C_i W_k(0)|^2.
    J: K x nb complex eigencoefficients, w: K x N real tapers.  Returns
    (F, C).  A band whose eigencoefficients are exactly proportional to
    W(0) has a zero denominator and F = inf."""
    J = np.asarray(J, dtype=np.complex128)
    w = np.asarray(w, dtype=np.float64)
    K = J.shape[0]
    W0 = w.sum(axis=1)
    sww = float((W0 ** 2).sum())
    C = (J * W0[:, None]).sum(axis=0) / sww
    num = np.abs(C) ** 2 * (K - 1) * sww
    den = (np.abs(J - C[None, :] * W0[:, None]) ** 2).sum(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        F = np.where(den > 0.0, num / np.where(den > 0.0, den, 1.0), np.inf)
    return F, C


def f_critical(p, K):
    """Critical value of F(2, 2K - 2) at upper-tail probability p (Sec. 3.6:
    F_s follows F(2, 2K-2); the level is chosen as p, for instance the
    Rayleigh level 1/N).  With nu = 2K - 2 the upper tail of F(2, nu) is
    (1 + 2 F / nu)^(-nu / 2), so F_p = (nu / 2)(p^(-2 / nu) - 1)."""
    nu = 2.0 * K - 2.0
    return 0.5 * nu * (float(p) ** (-2.0 / nu) - 1.0)


def ehat(t, w, lam, fmax, fw, f_lo, df, I=None, bands=None):
    """Suboptimality estimate (Appendix B with Sec. 3.5):
    D_k(i) = (E_i w_k)^* R(B) (E_i w_k), lambda_hat = 2 f_w lambda_k / D_k(i),
    Ehat_i = (1/K) sum_k |lambda_k - lambda_hat_k(i)|.
    Returns (E [nb], D [K, nb])."""
    t, w, lam = _f64(t), _f64(np.atleast_2d(w)), _f64(lam)
    K, N = w.shape
    if bands is None:
        bands = np.arange(I, dtype=np.int64)
    bands = np.ascontiguousarray(bands, dtype=np.int64)
    nb = bands.shape[0]
    D, E = np.empty((K, nb)), np.empty(nb)
    lib().or_ehat_direct(_p(t), _p(w), _p(lam), N, K, float(fmax), float(fw),
                         float(f_lo), float(df), bands.ctypes.data_as(_l), nb,
                         _p(D), _p(E))
    return E, D


def lanczos(t, fw, K, L=None, cdiag=1.0, mmax=400, tol=1e-14, seed=0x5EED, toeplitz=False):
    """Top-K eigenpairs of L^{-1} R(A0) L^{-T} (L None: R(B) = cdiag I).
    toeplitz: apply R(A0) as the lattice Toeplitz convolution (integer t)."""
    t = _f64(t)
    N = t.shape[0]
    ev, y = np.empty(K), np.empty((N, K))
    Lp = _p(_f64(L)) if L is not None else ctypes.cast(None, _d)
    st = lib().or_lanczos(_p(t), N, float(fw), Lp, float(cdiag), K, int(mmax),
                          float(tol), _p(ev), _p(y), seed, 1 if toeplitz else 0)
    if st < 0:
        raise OracleError(st, "lanczos")
    return ev, y


def m2nufft(t, x, fmax, fw, K, f_lo, df, I, bands=None, method="auto",
            with_ehat=True):
    """Table 3 with one sub-band and the GEP branch at f_c0 = 0:
    step 3 tapers, step 4 eigencoefficients, step 5 average; plus Ehat."""
    w, lam = gpss_tapers(t, fmax, fw, K, method=method)
    J = nudft(t, x, w, f_lo, df, I=I, bands=bands)
    P = psd(J)
    out = {"w": w, "lam": lam, "J": J, "P": P}
    if with_ehat:
        out["E"], out["D"] = ehat(t, w, lam, fmax, fw, f_lo, df, I=I, bands=bands)
    return out
