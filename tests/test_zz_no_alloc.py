"""The allocation-free entry point m2nufft_psd_at_noalloc against
m2nufft_psd_at, through the C-ABI: two calls in a row on one context, the
second with a smaller input.  The first call is large enough that its partial
sums are regrouped into fewer chunks to fit the fixed scratch array (FP64
rounding only: within 1e-12 of the largest value); the second keeps the
chunking of the allocating call, so its results are bitwise equal.  The
context's workspace stays empty throughout (nothing was allocated for the
calls)."""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _case(seed, N, K, I):
    rng = np.random.default_rng(seed)
    s = W.scheme_jitter(n=N)
    w = rng.standard_normal((K, s.N)) / np.sqrt(s.N)
    freqs = rng.uniform(-0.5, 0.5, I)
    return s, w, freqs


def test_noalloc_matches_allocating_call_twice(m2n):
    ctx_na = m2n.Context(0)
    ctx_ref = m2n.Context(0)
    try:
        for seed, (N, K, I, bitwise) in enumerate([(2000, 16, 65536, False), (700, 4, 300, True)]):
            s, w, freqs = _case(seed, N, K, I)
            t, x, wd, fd = _dev(s.t), _dev(s.x), _dev(w), _dev(freqs)
            P = torch.empty((I,), dtype=torch.float64, device="cuda")
            J = torch.empty((K, I), dtype=torch.complex128, device="cuda")
            torch.cuda.synchronize()
            print(f"no_alloc call {seed}: N={s.N} K={K} I={I}", flush=True)
            m2n.m2nufft_psd_at_noalloc(ctx_na, t, x, wd, fd, P, J)
            torch.cuda.synchronize()
            assert ctx_na.workspace_bytes() == 0
            ref = m2n.m2nufft_psd_at(ctx_ref, t, x, wd, fd, want_J=True)
            torch.cuda.synchronize()
            Pn, Jn = P.cpu().numpy(), J.cpu().numpy()
            Pr, Jr = ref["P"].cpu().numpy(), ref["J"].cpu().numpy()
            if bitwise:
                assert np.array_equal(Pn, Pr) and np.array_equal(Jn, Jr)
            else:
                assert np.abs(Pn - Pr).max() <= 1e-12 * Pr.max()
                assert np.abs(Jn - Jr).max() <= 1e-12 * np.abs(Jr).max()
    finally:
        ctx_na.close()
        ctx_ref.close()


def test_noalloc_rejects_oversize(m2n):
    ctx = m2n.Context(0)
    try:
        s, w, freqs = _case(5, 300, 16, 65537)
        P = torch.empty((65537,), dtype=torch.float64, device="cuda")
        with pytest.raises(m2n.M2NError) as ei:
            m2n.m2nufft_psd_at_noalloc(ctx, _dev(s.t), _dev(s.x), _dev(w), _dev(freqs), P)
        assert ei.value.code == m2n.M2N_ERR_ARG
    finally:
        ctx.close()
