"""Shared helpers of the GPU parity tests (tolerances and reporting).

FP64 tolerance (the click reading of the cumulant tolerance, with the parity
scale documented beside it):

    |delta| <= 1e-10 * max(|ref|, 1e-4 * scale)

* click cumulants: scale(S) = sum over set partitions pi of S of
  |w(pi)| prod_{B in pi} |mu(B)| (the magnitude of the terms of the partition
  sum of Eq. cumulant_corr_main that cancel);
* parity cumulants: the parity correlators c(B) are themselves small
  differences of terms 2^|T| p(T), so the rounding that matters is carried in
  from them: scale(S) = sum_pi |w(pi)| sum_{B in pi} V(B) prod_{B' != B} |c(B')|,
  V(B) = sum_{T subset B} 2^|T| p(T) (oracle.c_error_floor); the partition
  scale above is exceeded by the FP64 oracle's own error against a 40-digit
  evaluation at orders 4 and 5 in this convention;
* correlators: scale(S) = sum_{T subset S} |w_T| p(T); for click correlators
  the relative term always dominates (mu(S) is a probability), for parity
  correlators, which can pass through zero, the floor keeps the bound finite.

tests/test_tolerance_pins.py pins every scale against the 40-digit arbiter.
"""
import numpy as np

import oracle as O

# FP64 path: relative tolerance and the fraction of the summand scale below
# which it stops shrinking.
REL_FP64 = 1e-10
FLOOR_REL = 1e-4


def fp64_scales(sigma, d, ranks, conv=O.CLICK, mu=None):
    """(scale of each correlator, scale of each cumulant) of the sampled
    order-d subsets, for fp64_tolerance."""
    smu, skap = O.c_tolerance_scale(sigma, d, ranks, conv, mu=mu)
    if conv == O.PARITY:
        _, skap = O.c_error_floor(sigma, d, ranks, conv, mu=mu)
    return smu, skap


def fp64_tolerance(ref, scale):
    """1e-10 * max(|ref|, 1e-4 * scale)."""
    return REL_FP64 * np.maximum(np.abs(ref), FLOOR_REL * np.asarray(scale))


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
