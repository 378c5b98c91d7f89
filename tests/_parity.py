"""Element-wise comparison used by the GPU parity tests.

A result matches its reference to `tol` when every element does:
|got_i - ref_i| <= tol |ref_i| + tol max_j |ref_j|.  The second term keeps entries near zero
(whose relative error is meaningless) at the scale of the vector; an error of tol in the
largest entries, or of tol max|ref| in small ones, fails.
"""
import numpy as np


def to_np(a):
    return np.asarray(a.cpu() if hasattr(a, "cpu") else a, dtype=np.float64)


def assert_close(got, ref, tol, what=""):
    got, ref = to_np(got), to_np(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    scale = float(np.abs(ref).max()) if ref.size else 0.0
    np.testing.assert_allclose(got, ref, rtol=tol, atol=tol * scale, err_msg=what)


def rel(a, b):
    """Norm-wise relative difference, for the diagnostic prints."""
    a, b = to_np(a), to_np(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
