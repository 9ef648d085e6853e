"""Error metrics used by the parity tests (normwise, after sign alignment)."""
import numpy as np


def align_signs(w_test, w_ref):
    """Flip each row of w_test to best match the corresponding row of w_ref."""
    s = np.sign(np.sum(w_test * w_ref, axis=1))
    s[s == 0] = 1.0
    return w_test * s[:, None], s


def normwise_rows(a, b):
    """max_k ||a_k - b_k|| / ||b_k|| over rows."""
    num = np.linalg.norm(a - b, axis=1)
    den = np.linalg.norm(b, axis=1)
    return float(np.max(num / np.maximum(den, 1e-300)))


def psd_err(p, ref):
    """max_i |p_i - ref_i| / max_i ref_i."""
    return float(np.max(np.abs(p - ref)) / np.max(np.abs(ref)))


def per_band_rel(p, ref):
    r = np.abs(p - ref) / np.maximum(np.abs(ref), 1e-300)
    return {"median": float(np.median(r)), "p99": float(np.quantile(r, 0.99)), "max": float(r.max())}
