"""CPU oracle of the chain-rule sampler (TEST INFRASTRUCTURE).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this module; it shares no code with the GPU library.

The sampler draws x_1, x_2, ..., x_M one bit at a time from the conditional
p(x_n | x_{n-1}, ..., x_1) = p(x_n, ..., x_1) / p(x_{n-1}, ..., x_1), where the
joint probability is expanded in the parity cumulants kappa(S) of the bits
(Sec. II "The sampling algorithm", Eq. samplecumulant; App. B, Eqs.
probs_corr_cumulants_3 and delta_bias), truncated at order K, and the marginal
probabilities the expansion needs are replaced by approximations kept in tables
that are updated after every bit:

* single elision, K = 3 (Methods, "Marginals approximations"): Eq. methprob
  for p, Eq. b for the one-elided marginals p1, Eq. a for the partial marginals
  p+;
* double elision, K = 5 (App. C.1): Eq. probade for p, Eq. probpartialade for
  p+, Eq. probelidedade for p1 and Eq. probdoubleelidedade for the two-elided
  marginals p2.

Notation follows the paper: bits are numbered 1..M in sampling order (bit n is
mode n-1 of the covariance), gamma_A = kappa(A) chi(A) with the parity
function chi(A) = (-1)^(sum_{i in A} x_i).  Marginals:

  p(a)        = p(x_a, ..., x_1)                         (p(0) = 1)
  p1(a, e)    = p(x_a, ..., ~x_e, ..., x_1), e <= a      (variable e traced out)
  p2(a, e, d) = p(x_a, ..., ~x_e, ..., ~x_d, ..., x_1), d < e <= a
  pp(b, a)    = p+(x_b, ..., x_a)                        (1 when b < a)

A marginal whose top variable is traced out is the marginal with the next top:
p1(a, a) = p(a - 1) and p2(a, a, d) = p1(a - 1, d).

Bit decision: with u_n ~ U[0, 1) supplied by the caller, x_n = 1 when
u_n < p(x_n = 1 | x_{<n}) = p(x_n = 1, x_{n-1}, ..., x_1) / p(n - 1), the
expansion's value over the previously computed p(n - 1).  The expansion may
leave [0, 1]: the comparison then clamps it; when p(n - 1) is not positive the
conditional is undefined and 1/2 is used (the paper fixes neither case; both
are readings of it).
All arithmetic is FP64.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _c, _dptr, colex_rank, order_offset

SINGLE = 3  # single elision, K = 3
DOUBLE = 5  # double elision, K = 5


def kappa_lookup(cum: np.ndarray, M: int, K: int):
    """kappa(bits...) from the library layout of parity cumulants (order blocks
    d = 1..K, colex inside a block); bit b is mode b - 1."""
    offs = [0] + [order_offset(M, d) for d in range(1, K + 1)]

    def kap(*bits):
        modes = sorted(b - 1 for b in bits)
        return float(cum[offs[len(modes)] + colex_rank(modes)])
    return kap


class _Tables:
    """The marginal tables of one sample (dictionaries keyed as in the module
    docstring)."""

    def __init__(self):
        self.P0 = {0: 1.0}
        self.P1 = {}
        self.P2 = {}
        self.PP = {}

    def p(self, a):
        return self.P0[a]

    def p1(self, a, e):
        if e == a:
            return self.p(a - 1)
        return self.P1[(a, e)]

    def p2(self, a, e, d):
        assert d < e <= a
        if e == a:
            return self.p1(a - 1, d)
        return self.P2[(a, e, d)]

    def pp(self, b, a):
        if b < a:
            return 1.0
        return self.PP[(b, a)]


def _ord(*idx):
    """The indices rearranged in decreasing order (the paper's ord(...))."""
    return tuple(sorted(idx, reverse=True))


class _Step:
    """gamma_A for the bits sampled so far and a trial value of x_n."""

    def __init__(self, kap, x):
        self.kap = kap
        self.x = x  # dict bit -> value

    def chi(self, *bits):
        return -1.0 if sum(self.x[b] for b in bits) % 2 else 1.0

    def gamma(self, *bits):
        return self.kap(*bits) * self.chi(*bits)


# ---------------------------------------------------------------------------
# single elision, K = 3 (Methods)


def _single_p(t: _Tables, g: _Step, n: int) -> float:
    """Eq. methprob: p(x_n, ..., x_1)."""
    s1 = 0.5 * (1.0 + g.gamma(n)) * t.p(n - 1)
    s2 = math.fsum(0.25 * g.gamma(i, n) * t.p1(n - 1, i) for i in range(1, n))
    s3 = math.fsum(0.125 * g.gamma(i, j, n) * t.pp(n - 1, i + 1) * t.p1(i - 1, j)
                   for i in range(1, n) for j in range(1, i))
    return math.fsum([s1, s2, s3])


def _single_update(t: _Tables, g: _Step, n: int, pn: float):
    """Tables of top n after x_n is fixed: Eq. b (p1) and Eq. a (p+)."""
    for e in range(1, n):
        terms = [0.5 * (1.0 + g.gamma(n)) * t.p1(n - 1, e)]
        for i in range(1, n):
            if i == e:
                continue
            a, b = min(i, e), max(i, e)
            terms.append(0.25 * g.gamma(i, n) * t.pp(n - 1, b + 1) * t.p1(b - 1, a))
        t.P1[(n, e)] = math.fsum(terms)
    for ell in range(1, n + 1):
        terms = [0.5 * (1.0 + g.gamma(n)) * t.pp(n - 1, ell)]
        for i in range(ell, n):
            terms.append(0.25 * g.gamma(i, n) * t.pp(n - 1, i + 1) * t.pp(i - 1, ell))
        t.PP[(n, ell)] = math.fsum(terms)
    t.P0[n] = pn


# ---------------------------------------------------------------------------
# double elision, K = 5 (App. C.1)


def _double_p(t: _Tables, g: _Step, n: int) -> float:
    """Eq. probade: p(x_n, ..., x_1)."""
    terms = [0.5 * (1.0 + g.gamma(n)) * t.p(n - 1)]
    for i in range(1, n):
        terms.append(0.25 * g.gamma(i, n) * t.p1(n - 1, i))
    for i in range(2, n):
        for j in range(1, i):
            terms.append(0.125 * g.gamma(i, j, n) * t.p2(n - 1, i, j))
    for i in range(3, n):
        for j in range(2, i):
            for k in range(1, j):
                terms.append(g.gamma(i, j, k, n) * t.pp(n - 1, i + 1) * t.p2(i - 1, j, k) / 16.0)
    for i in range(4, n):
        for j in range(3, i):
            for k in range(2, j):
                for l in range(1, k):
                    terms.append(g.gamma(i, j, k, l, n) * t.pp(n - 1, i + 1) * t.pp(i - 1, j + 1)
                                 * t.p2(j - 1, k, l) / 32.0)
    return math.fsum(terms)


def _double_update(t: _Tables, g: _Step, n: int, pn: float):
    """Tables of top n after x_n is fixed: Eqs. probpartialade (p+),
    probelidedade (p1) and probdoubleelidedade (p2)."""
    for ell in range(1, n + 1):
        terms = [0.5 * (1.0 + g.gamma(n)) * t.pp(n - 1, ell)]
        for i in range(ell, n):
            terms.append(0.25 * g.gamma(i, n) * t.pp(n - 1, i + 1) * t.pp(i - 1, ell))
        for i in range(ell + 1, n):
            for j in range(ell, i):
                terms.append(0.125 * g.gamma(i, j, n) * t.pp(n - 1, i + 1) * t.pp(i - 1, j + 1)
                             * t.pp(j - 1, ell))
        t.PP[(n, ell)] = math.fsum(terms)
    for e in range(1, n):
        terms = [0.5 * (1.0 + g.gamma(n)) * t.p1(n - 1, e)]
        others = [i for i in range(1, n) if i != e]
        for i in others:
            a, b = _ord(i, e)
            terms.append(0.25 * g.gamma(i, n) * t.p2(n - 1, a, b))
        for i in others:
            for j in others:
                if not i > j:
                    continue
                a, b, c = _ord(i, j, e)
                terms.append(0.125 * g.gamma(i, j, n) * t.pp(n - 1, a + 1) * t.p2(a - 1, b, c))
        t.P1[(n, e)] = math.fsum(terms)
    for e in range(2, n):
        for d in range(1, e):
            terms = [0.5 * (1.0 + g.gamma(n)) * t.p2(n - 1, e, d)]
            for i in range(1, n):
                if i in (e, d):
                    continue
                a, b, c = _ord(i, e, d)
                terms.append(0.25 * g.gamma(i, n) * t.pp(n - 1, a + 1) * t.p2(a - 1, b, c))
            t.P2[(n, e, d)] = math.fsum(terms)
    t.P0[n] = pn


# ---------------------------------------------------------------------------


def conditional_one(p_one: float, p_prev: float) -> float:
    """p(x_n = 1 | x_{<n}) as used for the decision (see module docstring)."""
    if not p_prev > 0.0:
        return 0.5
    return p_one / p_prev


def sample(cum: np.ndarray, M: int, method: int, u=None, forced=None):
    """One sample of M bits.

    cum     parity cumulants kappa, orders 1..K (K = method), library layout
    method  SINGLE (K = 3) or DOUBLE (K = 5)
    u       M uniforms in [0, 1): x_n = 1 iff u[n-1] < p(x_n = 1 | x_{<n})
    forced  alternatively, M bits to follow (the probabilities of a given path)

    Returns (bits, cond, p): the bits (uint8, length M), the conditionals
    p(x_n = 1 | x_{<n}) of every step, and p(x_M, ..., x_1) of the path.
    """
    kap = kappa_lookup(cum, M, method)
    t = _Tables()
    x = {}
    bits = np.zeros(M, dtype=np.uint8)
    cond = np.zeros(M)
    step_p = _single_p if method == SINGLE else _double_p
    update = _single_update if method == SINGLE else _double_update
    for n in range(1, M + 1):
        x[n] = 1
        g = _Step(kap, x)
        p_one = step_p(t, g, n)
        q = conditional_one(p_one, t.p(n - 1))
        cond[n - 1] = q
        if forced is not None:
            xn = int(forced[n - 1])
        else:
            xn = 1 if u[n - 1] < q else 0
        x[n] = xn
        bits[n - 1] = xn
        pn = p_one if xn == 1 else step_p(t, _Step(kap, x), n)
        update(t, _Step(kap, x), n, pn)
    return bits, cond, t.p(M)


def pattern_probability(cum: np.ndarray, M: int, method: int, bits) -> float:
    """The sampler's p(x_M, ..., x_1) for a given pattern (teacher-forced)."""
    return sample(cum, M, method, forced=bits)[2]


def c_sample(cum: np.ndarray, M: int, method: int, u=None, forced=None, threads: int = 0):
    """C tier (oracle/gbs_sampler_oracle.c): n samples at once.

    u       (M, n) uniforms, u[m, s] for bit m + 1 of sample s; or
    forced  (n, M) bits to follow.
    Returns (bits (n, M) uint8, prob (n,), cond (M, n)).
    """
    lib = _c()
    if not hasattr(lib, "_sample_ready"):
        lib.oracle_sample.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                      ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_int32]
        lib.oracle_sample.restype = ctypes.c_int32
        lib._sample_ready = True
    cum = np.ascontiguousarray(cum, dtype=np.float64)
    if forced is not None:
        forced = np.ascontiguousarray(forced, dtype=np.uint8)
        n = forced.shape[0]
        u = np.zeros((M, n))
    else:
        u = np.ascontiguousarray(u, dtype=np.float64)
        n = u.shape[1]
    bits = np.zeros((n, M), dtype=np.uint8)
    prob = np.zeros(n)
    cond = np.zeros((M, n))
    rc = lib.oracle_sample(M, _dptr(cum), method, n, _dptr(u), n,
                           forced.ctypes.data if forced is not None else None,
                           bits.ctypes.data, _dptr(prob), _dptr(cond), threads)
    if rc != 0:
        raise RuntimeError(f"oracle_sample failed ({rc})")
    return bits, prob, cond
