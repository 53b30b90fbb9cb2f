"""Shared helpers of the GPU parity tests (tolerances and reporting).

FP64 tolerances, derived from the arithmetic of a plain FP64 evaluation:

* correlators: |delta| <= 1e-10 max(|ref|, 1e-4 scale), scale(S) = sum over
  T subset S of |w_T| p(T), the magnitude of the inclusion-exclusion terms
  (for click correlators the relative term always dominates: mu(S) is a
  probability; parity correlators can pass through zero, and the floor keeps
  the bound finite);
* cumulants: |delta| <= 1e-10 max(|ref|, 1e-4 S_pi) + CARRY u V,
  - S_pi(S) = sum over set partitions pi of S of |w(pi)| prod_{B in pi} |m(B)|,
    the magnitude of the terms of the partition sum of Eq. cumulant_corr_main
    (m = mu click, c parity): the rounding of the partition sum itself;
  - V(S) = sum_pi |w(pi)| sum_{B in pi} V_m(B) prod_{B' != B} |m(B')|, with
    V_m(B) = sum_{T subset B} |w_T| p(T): the first-order propagation of the
    rounding that every correlator m(B) carries in from its own
    inclusion-exclusion (oracle.c_error_floor).  Without it the bound fails for
    weakly illuminated modes, where m(B) is a small difference of
    probabilities near one: there the FP64 oracle itself misses 1e-10 max(|ref|,
    1e-4 S_pi) against a 40-digit evaluation by a factor of ten, while its error
    stays below u V.

tests/test_tolerance_pins.py pins both terms against the 40-digit arbiter: the
FP64 oracle's error fits in half of the tolerance, and the tolerance is not
more than a stated factor above the measured error.
"""
import numpy as np

import oracle as O

# FP64 path: relative tolerance, the fraction of the summand scale below which
# it stops shrinking, and the multiple of u V allowed for the rounding carried
# in from the correlators.
REL_FP64 = 1e-10
FLOOR_REL = 1e-4
CARRY = 4.0
U = 2.0 ** -53


def fp64_scales(sigma, d, ranks, conv=O.CLICK, mu=None):
    """(scale of each correlator, scales of each cumulant) of the sampled
    order-d subsets, for fp64_tolerance; the cumulant entry is a 2 x n array,
    row 0 the partition-sum magnitude S_pi, row 1 the carried-in magnitude V."""
    smu, spi = O.c_tolerance_scale(sigma, d, ranks, conv, mu=mu)
    _, vk = O.c_error_floor(sigma, d, ranks, conv, mu=mu)
    return smu, np.stack([spi, vk])


def fp64_tolerance(ref, scale):
    """Correlators (1-D scale): 1e-10 max(|ref|, 1e-4 scale).  Cumulants
    (2 x n scale from fp64_scales): 1e-10 max(|ref|, 1e-4 S_pi) + CARRY u V."""
    scale = np.asarray(scale)
    if scale.ndim == 2:
        return (REL_FP64 * np.maximum(np.abs(ref), FLOOR_REL * scale[0]) +
                CARRY * U * scale[1])
    return REL_FP64 * np.maximum(np.abs(ref), FLOOR_REL * scale)


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
