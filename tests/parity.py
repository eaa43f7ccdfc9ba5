"""Element-wise comparison helpers of the GPU parity tests (no arithmetic of
the method: plain checks of |got - want| against a stated tolerance)."""

import numpy as np


def assert_close(got, want, rtol, atol_frac, what=""):
    """|got - want| <= atol + rtol |want| for every entry, with atol =
    atol_frac times the largest |want| of the entry's column (2-D arrays: a
    factor's columns carry their own scale) or of the whole array (1-D)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if want.size == 0:
        return
    if want.ndim == 2:
        scale = np.max(np.abs(want), axis=0, keepdims=True)
    else:
        scale = np.max(np.abs(want))
    atol = atol_frac * scale
    err = np.abs(got - want)
    bad = err > atol + rtol * np.abs(want)
    if np.any(bad):
        where = np.argwhere(bad)[:5]
        worst = float(np.max(err / (atol + rtol * np.abs(want) + 1e-300)))
        raise AssertionError(
            f"{what}: {int(bad.sum())} of {want.size} entries outside rtol {rtol}, atol "
            f"{atol_frac} x column max (worst {worst:.3g} x the bound); first at "
            f"{where.tolist()}: got {got[tuple(where[0])]!r} want {want[tuple(where[0])]!r}")


def max_rel_err(got, want):
    """Largest |got - want| / max|want| per column (2-D) or overall (1-D)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    if want.ndim == 2:
        scale = np.max(np.abs(want), axis=0, keepdims=True)
    else:
        scale = np.max(np.abs(want))
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(got - want) / scale))
