"""Element-wise comparison used by the GPU parity tests."""
import numpy as np


def max_rel_err(x, ref):
    """max_i |x_i - ref_i| / max_i |ref_i|."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert x.shape == ref.shape, (x.shape, ref.shape)
    if ref.size == 0:
        return 0.0
    scale = np.abs(ref).max()
    return float(np.abs(x - ref).max() / (scale if scale > 0 else 1.0))


def assert_elementwise(x, ref, tol, what=""):
    """Every entry within tol * max|ref| of the reference."""
    e = max_rel_err(x, ref)
    assert e <= tol, f"{what}: max|x - x*| / max|x*| = {e:.3e} > {tol:.1e}"
    return e
