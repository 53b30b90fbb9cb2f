"""Shared helpers of the GPU parity tests (tolerances and reporting)."""
import numpy as np

import oracle as O

# FP64 path: relative tolerance on top of the rounding floor of each output.
REL_FP64 = 1e-10


def fp64_tolerance(ref, v):
    """|delta| <= 1e-10 |ref| + 64 u v, v the magnitude of the cancelling terms
    (oracle.c_error_floor)."""
    return REL_FP64 * np.abs(ref) + O.FLOOR_FACTOR * O.U64 * v


def assert_within(got, ref, tol, what):
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, what
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    err = np.abs(got - ref)
    bad = np.nonzero(err > tol)[0]
    if len(bad):
        i = bad[np.argmax(err[bad] / np.maximum(tol[bad], 1e-300))]
        raise AssertionError(f"{what}: {len(bad)}/{len(ref)} outside tolerance; worst index {i}: "
                             f"got {got[i]!r} ref {ref[i]!r} tol {tol[i]!r}")
    return err


def rel_stats(got, ref):
    rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
    return {"median": float(np.median(rel)), "p99": float(np.quantile(rel, 0.99)),
            "max": float(rel.max())}
