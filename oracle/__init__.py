"""CPU oracle for the click-correlator / cumulant path (TEST INFRASTRUCTURE).

This package is test infrastructure only.  It may be imported or executed only
by ``tests/``, by ``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of
``bench.py``.  The product path (the HIP library and its Python binding) never
imports, calls or links anything here, and nothing here imports the product.

Everything is plain FP64 and follows the paper's definitions directly:

* vacuum probability of a mode subset T: p(T) = det(Q_T)^(-1/2), Q = sigma + I/2,
  Q_T keeping rows/columns k and k+M for k in T (App. D.1, Eqs.
  vacuum_gaussian_prob and correlator_sum_cov with hbar = 1; the reduced-state
  rule is stated in the paragraph before Eq. vacuum_gaussian_prob);
  for a displaced state with first moments mu (xxpp, length 2M) the same
  equation gives p(T) = exp(-mu_T^T Q_T^{-1} mu_T / 2) det(Q_T)^(-1/2), mu_T
  keeping entries k and k+M for k in T; every function taking ``mu`` uses it
  (``mu=None`` is the zero-mean state);
* click correlator (joint click moment) mu(S) = sum_{T subset S} (-1)^|T| p(T):
  the probability that every mode of S clicks (App. A.2, Eq. joint_moments_def,
  expanded with the threshold POVM of App. D.1);
* parity correlator c(S) = (-1)^|S| sum_{T subset S} (-2)^|T| p(T)
  (Sec. I.A, Eq. corre_cov_main; App. D.1, Eq. correlator_sum_cov);
* cumulant of either kind by the moment-to-cumulant sum over set partitions,
  weight (-1)^(|pi|-1) (|pi|-1)! (Sec. I.A, Eq. cumulant_corr_main; App. A.2,
  Eq. joint_cumulants_def).

Output layout shared with the GPU library: for d = 1..K an order block of
C(M, d) values, subsets in colexicographic order inside a block (rank of
{s_0 < ... < s_{d-1}} is sum_j C(s_j, j+1)).

``oracle/gbs_oracle.c`` is the same definition in plain C with OpenMP over
subsets, for the large workloads; it is checked against this module.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
from functools import lru_cache

import numpy as np

CLICK = 0
PARITY = 1

# ----------------------------------------------------------------------------
# layout: colexicographic ranks


def num_subsets(M: int, d: int) -> int:
    return math.comb(M, d)


def total_outputs(M: int, K: int) -> int:
    return sum(math.comb(M, d) for d in range(1, K + 1))


def order_offset(M: int, d: int) -> int:
    """Start of the order-d block in the concatenated layout."""
    return sum(math.comb(M, e) for e in range(1, d))


def colex_rank(S) -> int:
    s = sorted(S)
    return sum(math.comb(x, j + 1) for j, x in enumerate(s))


def colex_unrank(d: int, r: int) -> tuple:
    """Inverse of colex_rank: the d-subset of rank r (largest element first)."""
    out = []
    for j in range(d, 0, -1):
        x = j - 1
        while math.comb(x + 1, j) <= r:
            x += 1
        out.append(x)
        r -= math.comb(x, j)
    return tuple(reversed(out))


def subsets_colex(M: int, d: int):
    """All d-subsets of range(M) in colex order."""
    if d == 0:
        yield ()
        return
    for top in range(d - 1, M):
        for rest in subsets_colex(top, d - 1):
            yield rest + (top,)


# ----------------------------------------------------------------------------
# set partitions and their weights (Sec. III, "partition patterns")


@lru_cache(maxsize=None)
def set_partitions(n: int) -> tuple:
    """All partitions of {0..n-1} as tuples of blocks (each a tuple of indices),
    generated from restricted growth strings."""
    out = []

    def rec(i, labels, nblocks):
        if i == n:
            blocks = [[] for _ in range(nblocks)]
            for k, b in enumerate(labels):
                blocks[b].append(k)
            out.append(tuple(tuple(b) for b in blocks))
            return
        for b in range(nblocks + 1):
            rec(i + 1, labels + [b], max(nblocks, b + 1))

    rec(0, [], 0)
    return tuple(out)


def partition_weight(nblocks: int) -> int:
    """w(pi) = (-1)^(|pi|-1) (|pi|-1)!  (Eq. cumulant_corr_main)."""
    return (-1) ** (nblocks - 1) * math.factorial(nblocks - 1)


def cumulant_from_moments(S: tuple, moment) -> float:
    """sum over partitions pi of S of w(pi) prod_{B in pi} moment(B).

    ``moment`` maps a sorted tuple of modes to its correlator/joint moment.
    """
    terms = []
    for pi in set_partitions(len(S)):
        prod = float(partition_weight(len(pi)))
        for block in pi:
            prod *= moment(tuple(S[k] for k in block))
        terms.append(prod)
    return math.fsum(terms)


# ----------------------------------------------------------------------------
# vacuum probabilities and correlators


def q_matrix(sigma: np.ndarray) -> np.ndarray:
    """Q = sigma + I/2 (hbar = 1): the matrix whose principal minors give the
    vacuum probabilities."""
    sigma = np.asarray(sigma, dtype=np.float64)
    return sigma + 0.5 * np.eye(sigma.shape[0])


def principal_block(Q: np.ndarray, T) -> np.ndarray:
    """Q_T: rows and columns k and k+M for k in T (xxpp)."""
    M = Q.shape[0] // 2
    idx = [t for t in T] + [t + M for t in T]
    return Q[np.ix_(idx, idx)]


def principal_mean(mu: np.ndarray, T) -> np.ndarray:
    """mu_T: entries k and k+M for k in T (xxpp), the first moments of the
    reduced state (paragraph before Eq. vacuum_gaussian_prob)."""
    M = len(mu) // 2
    idx = [t for t in T] + [t + M for t in T]
    return np.asarray(mu, dtype=np.float64)[idx]


def mean_quadratic_form(Q: np.ndarray, mu: np.ndarray, T) -> float:
    """mu_T^T Q_T^{-1} mu_T (library linear solve)."""
    m = principal_mean(mu, T)
    return float(m @ np.linalg.solve(principal_block(Q, T), m))


def vacuum_probability(Q: np.ndarray, T, mu=None) -> float:
    """p(T) = exp(-mu_T^T Q_T^{-1} mu_T / 2) det(Q_T)^(-1/2); p(empty) = 1
    (Eq. vacuum_gaussian_prob, hbar = 1; mu=None is the zero-mean state).  The
    determinant is the squared product of the Cholesky diagonal (library
    Cholesky)."""
    if len(T) == 0:
        return 1.0
    L = np.linalg.cholesky(principal_block(Q, T))
    p = 1.0 / float(np.prod(np.diag(L)))
    if mu is not None:
        p *= math.exp(-0.5 * mean_quadratic_form(Q, mu, T))
    return p


def _vacuum_fn(Q, mu):
    """T -> p(T) for the zero-mean (mu None) or the displaced state."""
    if mu is None:
        return lambda T: vacuum_probability(Q, T)
    mu = np.asarray(mu, dtype=np.float64)
    return lambda T: vacuum_probability(Q, T, mu)


def all_subsets(S):
    for k in range(len(S) + 1):
        for T in itertools.combinations(S, k):
            yield T


def click_correlator(Q: np.ndarray, S, p=None) -> float:
    """mu(S) = sum_{T subset S} (-1)^|T| p(T): probability that all of S click."""
    p = p or (lambda T: vacuum_probability(Q, T))
    return math.fsum((-1) ** len(T) * p(T) for T in all_subsets(tuple(S)))


def parity_correlator(Q: np.ndarray, S, p=None) -> float:
    """c(S) = (-1)^|S| sum_{T subset S} (-2)^|T| p(T)  (Eq. corre_cov_main)."""
    p = p or (lambda T: vacuum_probability(Q, T))
    s = math.fsum((-2.0) ** len(T) * p(T) for T in all_subsets(tuple(S)))
    return (-1) ** len(S) * s


def subset_values(sigma: np.ndarray, S, convention: int = CLICK, mu=None) -> tuple:
    """(correlator, cumulant) of one subset S, computed from scratch."""
    Q = q_matrix(sigma)
    S = tuple(sorted(S))
    pcache = {}
    vac = _vacuum_fn(Q, mu)

    def p(T):
        if T not in pcache:
            pcache[T] = vac(T)
        return pcache[T]

    corr_fn = click_correlator if convention == CLICK else parity_correlator
    mcache = {}

    def moment(B):
        if B not in mcache:
            mcache[B] = corr_fn(Q, B, p)
        return mcache[B]

    return moment(S), cumulant_from_moments(S, moment)


def correlators_and_cumulants(sigma: np.ndarray, K: int, convention: int = CLICK,
                              mu=None) -> tuple:
    """Full layout (all subsets of order 1..K) -> (corr, cum) FP64 arrays.

    Plain enumeration; p(T) of each distinct subset is evaluated once and
    memoised, which changes nothing in the arithmetic of any single output.
    Intended for small M (seconds at M=16, K=3).
    """
    Q = q_matrix(sigma)
    M = Q.shape[0] // 2
    N = total_outputs(M, K)
    corr = np.empty(N)
    cum = np.empty(N)
    pcache = {}
    vac = _vacuum_fn(Q, mu)

    def p(T):
        if T not in pcache:
            pcache[T] = vac(T)
        return pcache[T]

    corr_fn = click_correlator if convention == CLICK else parity_correlator
    mcache = {}

    def moment(B):
        if B not in mcache:
            mcache[B] = corr_fn(Q, B, p)
        return mcache[B]

    pos = 0
    for d in range(1, K + 1):
        for S in subsets_colex(M, d):
            corr[pos] = moment(S)
            cum[pos] = cumulant_from_moments(S, moment)
            pos += 1
    return corr, cum


def sampled_values(sigma: np.ndarray, d: int, ranks, convention: int = CLICK, mu=None) -> tuple:
    """(corr, cum) for the order-d subsets with the given colex ranks."""
    ranks = np.asarray(ranks, dtype=np.int64)
    corr = np.empty(len(ranks))
    cum = np.empty(len(ranks))
    for i, r in enumerate(ranks):
        corr[i], cum[i] = subset_values(sigma, colex_unrank(d, int(r)), convention, mu)
    return corr, cum


def cumulant_scale(sigma: np.ndarray, S, convention: int = CLICK) -> float:
    """sum over partitions of |w(pi)| prod |moment(B)|: the magnitude of the
    terms that cancel in the cumulant of S (used to state tolerances)."""
    Q = q_matrix(sigma)
    S = tuple(sorted(S))
    corr_fn = click_correlator if convention == CLICK else parity_correlator
    m = {}

    def moment(B):
        if B not in m:
            m[B] = corr_fn(Q, B)
        return m[B]

    tot = []
    for pi in set_partitions(len(S)):
        prod = float(abs(partition_weight(len(pi))))
        for block in pi:
            prod *= abs(moment(tuple(S[k] for k in block)))
        tot.append(prod)
    return math.fsum(tot)


def vacuum_mass(sigma: np.ndarray, S) -> float:
    """sum_{T subset S} p(T): the magnitude of the terms that cancel in mu(S)."""
    Q = q_matrix(sigma)
    return math.fsum(vacuum_probability(Q, T) for T in all_subsets(tuple(sorted(S))))


# ----------------------------------------------------------------------------
# independent brute force: pattern probabilities by the Torontonian
# (App. F, Eqs. ground_truth_prob_tor and torontonian_def)


def complex_basis_covariance(sigma: np.ndarray) -> np.ndarray:
    """Sigma = I/2 + R sigma R^dagger (hbar = 1), R = [[I, iI], [I, -iI]]/sqrt(2)."""
    M = sigma.shape[0] // 2
    I = np.eye(M)
    R = np.block([[I, 1j * I], [I, -1j * I]]) / math.sqrt(2.0)
    return 0.5 * np.eye(2 * M) + R @ sigma @ R.conj().T


def torontonian(A: np.ndarray) -> complex:
    """tor(A) = sum_{R subset [n]} (-1)^(n-|R|) / sqrt(det(I - A_R)).

    The sign printed in Eq. torontonian_def, (-1)^|R|, gives probabilities that
    do not sum to one; (-1)^(n-|R|) is the standard form (it reduces to the
    single-mode click probability 1 - det(Sigma)^(-1/2) for n = 1).
    """
    n = A.shape[0] // 2
    total = 0.0 + 0.0j
    for k in range(n + 1):
        for R in itertools.combinations(range(n), k):
            idx = list(R) + [x + n for x in R]
            sub = A[np.ix_(idx, idx)]
            det = np.linalg.det(np.eye(2 * k) - sub) if k else 1.0
            total += (-1) ** (n - k) / np.sqrt(det + 0j)
    return total


def pattern_probabilities(sigma: np.ndarray) -> np.ndarray:
    """p(x) for every click pattern x in {0,1}^M (bit k of the index is x_k).

    p(x) = tor(O_(x)) / sqrt(det Sigma), O = I - Sigma^{-1}, O_(x) keeping the
    rows/columns of the clicked modes.  Cost 3^M determinants: M <= 10 or so.
    """
    M = sigma.shape[0] // 2
    Sig = complex_basis_covariance(sigma)
    O = np.eye(2 * M) - np.linalg.inv(Sig)
    norm = np.sqrt(np.linalg.det(Sig) + 0j)
    probs = np.empty(1 << M)
    for x in range(1 << M):
        clicked = [k for k in range(M) if (x >> k) & 1]
        idx = clicked + [k + M for k in clicked]
        sub = O[np.ix_(idx, idx)] if clicked else np.zeros((0, 0))
        probs[x] = (torontonian(sub) / norm).real
    return probs


# ----------------------------------------------------------------------------
# high-precision arbiter (mpmath, 40 digits)


def arbiter_values(sigma: np.ndarray, S, convention: int = CLICK, dps: int = 40,
                   mu=None) -> tuple:
    """(correlator, cumulant) of S with every step in dps-digit arithmetic.

    sigma (and mu) are taken as exact (their FP64 values); the result is
    accurate to far better than FP64 rounding, so it settles disagreements
    between FP64 evaluations that round differently.  For a displaced state
    the quadratic form is |z|^2 with z = L^{-1} mu_T, L the Cholesky factor.
    """
    import mpmath as mp

    ctx = mp.mp.clone()
    ctx.dps = dps
    M = sigma.shape[0] // 2
    S = tuple(sorted(S))
    Q = [[ctx.mpf(float(sigma[i, j])) + (ctx.mpf(1) / 2 if i == j else 0)
          for j in range(2 * M)] for i in range(2 * M)]

    pc = {}

    def p(T):
        if T in pc:
            return pc[T]
        if not T:
            pc[T] = ctx.mpf(1)
            return pc[T]
        idx = [t for t in T] + [t + M for t in T]
        n = len(idx)
        A = [[Q[i][j] for j in idx] for i in idx]
        det = ctx.mpf(1)
        # textbook Cholesky in high precision
        L = [[ctx.mpf(0)] * n for _ in range(n)]
        for i in range(n):
            for j in range(i + 1):
                s = A[i][j] - ctx.fsum(L[i][k] * L[j][k] for k in range(j))
                if i == j:
                    L[i][i] = ctx.sqrt(s)
                    det *= L[i][i]
                else:
                    L[i][j] = s / L[j][j]
        pc[T] = 1 / det
        if mu is not None:
            # forward substitution L z = mu_T
            z = []
            for i in range(n):
                v = ctx.mpf(float(mu[idx[i]])) - ctx.fsum(L[i][k] * z[k] for k in range(i))
                z.append(v / L[i][i])
            pc[T] *= ctx.exp(-ctx.fsum(v * v for v in z) / 2)
        return pc[T]

    def moment(B):
        terms = []
        for T in all_subsets(B):
            if convention == CLICK:
                terms.append((-1) ** len(T) * p(T))
            else:
                terms.append(ctx.mpf(-2) ** len(T) * p(T))
        s = ctx.fsum(terms)
        return s if convention == CLICK else (-1) ** len(B) * s

    mc = {}

    def mom(B):
        if B not in mc:
            mc[B] = moment(B)
        return mc[B]

    cum_terms = []
    for pi in set_partitions(len(S)):
        prod = ctx.mpf(partition_weight(len(pi)))
        for block in pi:
            prod *= mom(tuple(S[k] for k in block))
        cum_terms.append(prod)
    return float(mom(S)), float(ctx.fsum(cum_terms))


# ----------------------------------------------------------------------------
# gradient of the cumulant-matching loss (hand-written reverse mode, FP64)


def cumulant_loss_and_grad(sigma: np.ndarray, K: int, target: np.ndarray) -> tuple:
    """L = sum_S (kappa~(S) - target(S))^2 over all |S| <= K (click cumulants),
    and dL/dsigma with the entries of sigma treated as independent (symmetric).

    Reverse mode of the definition:
      kbar(S)  = 2 (kappa~(S) - target(S))
      mubar(B) = sum_{S >= B} kbar(S) d kappa~(S)/d mu(B),
                 d kappa~(S)/d mu(B) = sum_{pi of S, B in pi} w(pi) prod_{B' in pi, B' != B} mu(B')
      pbar(T)  = sum_{B >= T} (-1)^|T| mubar(B)
      d p(T)/d Q_T = -p(T) Q_T^{-1} / 2   (d log det A = tr(A^{-1} dA))
    The gradient with respect to Q equals the one with respect to sigma.
    Plain enumeration: small M only (tests); the C oracle covers M = 144.
    """
    Q = q_matrix(sigma)
    M = Q.shape[0] // 2
    subsets = [S for d in range(1, K + 1) for S in subsets_colex(M, d)]
    p = {(): 1.0}
    for S in subsets:
        p[S] = vacuum_probability(Q, S)
    mu = {(): 1.0}
    for S in subsets:
        mu[S] = math.fsum((-1) ** len(T) * p[T] for T in all_subsets(S))
    kap = {S: cumulant_from_moments(S, lambda B: mu[B]) for S in subsets}
    target = np.asarray(target, dtype=np.float64)
    loss_terms = []
    kbar = {}
    for i, S in enumerate(subsets):
        diff = kap[S] - target[i]
        loss_terms.append(diff * diff)
        kbar[S] = 2.0 * diff
    mubar = {S: 0.0 for S in subsets}
    for S in subsets:
        for pi in set_partitions(len(S)):
            blocks = [tuple(S[k] for k in b) for b in pi]
            w = partition_weight(len(pi))
            for bi, B in enumerate(blocks):
                prod = float(w)
                for bj, B2 in enumerate(blocks):
                    if bj != bi:
                        prod *= mu[B2]
                mubar[B] += kbar[S] * prod
    pbar = {}
    for T in subsets:
        acc = []
        for B in subsets:
            if set(T) <= set(B):
                acc.append(mubar[B])
        pbar[T] = (-1) ** len(T) * math.fsum(acc)
    grad = np.zeros_like(Q)
    for T in subsets:
        idx = [t for t in T] + [t + M for t in T]
        QTinv = np.linalg.inv(principal_block(Q, T))
        grad[np.ix_(idx, idx)] += -0.5 * pbar[T] * p[T] * QTinv
    return math.fsum(loss_terms), 0.5 * (grad + grad.T)


def covariance_param_grad(U: np.ndarray, r: np.ndarray, eta: np.ndarray,
                          grad_sigma: np.ndarray) -> tuple:
    """Chain dL/dsigma to (dL/deta_k, dL/dr_k) through the input model
    sigma = V D(sq) V^T + (I - V V^T)/2, V = symplectic(U diag(sqrt(eta))).

    With W = symplectic(U) and Pk the projector on quadratures k, k+M:
      d sigma/d eta_k = W [ (sq_k - I/2) on block k ] W^T
      d sigma/d r_k   = W [ eta_k * d sq_k/d r_k on block k ] W^T
    where sq_k = diag(e^{-2r_k}, e^{2r_k})/2.
    """
    M = U.shape[0]
    W = np.block([[U.real, -U.imag], [U.imag, U.real]])
    G = W.T @ grad_sigma @ W  # gradient with respect to the pre-interferometer covariance
    gx = np.diag(G)[:M]
    gp = np.diag(G)[M:]
    ex, ep = 0.5 * np.exp(-2.0 * r), 0.5 * np.exp(2.0 * r)
    d_eta = gx * (ex - 0.5) + gp * (ep - 0.5)
    d_r = eta * (gx * (-2.0 * ex) + gp * (2.0 * ep))
    return d_eta, d_r


# ----------------------------------------------------------------------------
# C tier (plain C + OpenMP), same definition


_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def c_oracle_available() -> bool:
    return os.path.exists(_LIB_PATH)


def _c():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("oracle/liboracle.so is not built (run oracle/build.py)")
        lib = ctypes.CDLL(_LIB_PATH)
        i32, i64, dp, lp = ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), \
            ctypes.POINTER(ctypes.c_int64)
        lib.oracle_forward.argtypes = [i32, dp, i32, i32, dp, dp, i32]
        lib.oracle_forward.restype = i32
        lib.oracle_forward_sample.argtypes = [i32, dp, i32, lp, i64, i32, dp, dp, i32]
        lib.oracle_forward_sample.restype = i32
        lib.oracle_loss_grad.argtypes = [i32, dp, i32, dp, dp, dp, i32]
        lib.oracle_loss_grad.restype = i32
        lib.oracle_error_floor.argtypes = [i32, dp, i32, lp, i64, i32, dp, dp, i32]
        lib.oracle_error_floor.restype = i32
        lib.oracle_forward_mu.argtypes = [i32, dp, dp, i32, i32, dp, dp, i32]
        lib.oracle_forward_mu.restype = i32
        lib.oracle_forward_sample_mu.argtypes = [i32, dp, dp, i32, lp, i64, i32, dp, dp, i32]
        lib.oracle_forward_sample_mu.restype = i32
        lib.oracle_error_floor_mu.argtypes = [i32, dp, dp, i32, lp, i64, i32, dp, dp, i32]
        lib.oracle_error_floor_mu.restype = i32
        lib.oracle_forward_range_mu.argtypes = [i32, dp, dp, i32, i64, i64, i32, dp, dp, dp, dp,
                                                i32]
        lib.oracle_forward_range_mu.restype = i32
        lib.oracle_tolerance_scale_mu.argtypes = [i32, dp, dp, i32, lp, i64, i32, dp, dp, i32]
        lib.oracle_tolerance_scale_mu.restype = i32
        lib.oracle_threads.argtypes = [i32]
        lib.oracle_threads.restype = i32
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _mu_arg(mu, M):
    """(array kept alive, pointer) for an optional mean vector of length 2M."""
    if mu is None:
        return None, ctypes.POINTER(ctypes.c_double)()
    mu = np.ascontiguousarray(mu, dtype=np.float64).reshape(-1)
    if mu.shape[0] != 2 * M:
        raise ValueError("mu must have 2M entries")
    return mu, _dptr(mu)


def c_threads(requested: int = 0) -> int:
    return int(_c().oracle_threads(requested))


def c_forward(sigma: np.ndarray, K: int, convention: int = CLICK, threads: int = 0,
              mu=None) -> tuple:
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    M = sigma.shape[0] // 2
    N = total_outputs(M, K)
    corr = np.empty(N)
    cum = np.empty(N)
    keep, mptr = _mu_arg(mu, M)
    rc = _c().oracle_forward_mu(M, _dptr(sigma), mptr, K, convention, _dptr(corr), _dptr(cum),
                                threads)
    if rc != 0:
        raise RuntimeError(f"oracle_forward failed ({rc})")
    return corr, cum


def c_forward_sample(sigma: np.ndarray, d: int, ranks, convention: int = CLICK,
                     threads: int = 0, mu=None) -> tuple:
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    M = sigma.shape[0] // 2
    ranks = np.ascontiguousarray(ranks, dtype=np.int64)
    corr = np.empty(len(ranks))
    cum = np.empty(len(ranks))
    keep, mptr = _mu_arg(mu, M)
    rc = _c().oracle_forward_sample_mu(M, _dptr(sigma), mptr, d,
                                    ranks.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    len(ranks), convention, _dptr(corr), _dptr(cum), threads)
    if rc != 0:
        raise RuntimeError(f"oracle_forward_sample failed ({rc})")
    return corr, cum


def c_loss_grad(sigma: np.ndarray, K: int, target: np.ndarray, threads: int = 0) -> tuple:
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    M = sigma.shape[0] // 2
    target = np.ascontiguousarray(target, dtype=np.float64)
    loss = np.zeros(1)
    grad = np.zeros_like(sigma)
    rc = _c().oracle_loss_grad(M, _dptr(sigma), K, _dptr(target), _dptr(loss), _dptr(grad), threads)
    if rc != 0:
        raise RuntimeError(f"oracle_loss_grad failed ({rc})")
    return float(loss[0]), grad


# Unit roundoff of FP64 and the multiple of it used in stated tolerances.
U64 = 2.0 ** -53
FLOOR_FACTOR = 64.0


def c_error_floor(sigma: np.ndarray, d: int, ranks, convention: int = CLICK,
                  threads: int = 0, mu=None) -> tuple:
    """(vmu, vkap): magnitudes of the cancelling terms of each sampled output.

    An FP64 evaluation of mu(S) (or c(S)) sums terms of total magnitude vmu(S),
    so its rounding error is a small multiple of U64 * vmu(S); vkap(S) carries
    those errors through the partition sum to first order.  Tolerances are
    stated as |delta| <= rel * |ref| + FLOOR_FACTOR * U64 * v.
    """
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    M = sigma.shape[0] // 2
    ranks = np.ascontiguousarray(ranks, dtype=np.int64)
    vmu = np.empty(len(ranks))
    vkap = np.empty(len(ranks))
    keep, mptr = _mu_arg(mu, M)
    rc = _c().oracle_error_floor_mu(M, _dptr(sigma), mptr, d,
                                 ranks.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 len(ranks), convention, _dptr(vmu), _dptr(vkap), threads)
    if rc != 0:
        raise RuntimeError(f"oracle_error_floor failed ({rc})")
    return vmu, vkap


def c_forward_range(sigma: np.ndarray, d: int, rank0: int, count: int,
                    convention: int = CLICK, threads: int = 0, mu=None, scales: bool = False):
    """(corr, cum) of the order-d subsets with colex ranks rank0 .. rank0+count-1;
    with ``scales`` also (smu, skap) of ``c_tolerance_scale`` for the same subsets."""
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    M = sigma.shape[0] // 2
    corr = np.empty(count)
    cum = np.empty(count)
    smu = np.empty(count) if scales else None
    skap = np.empty(count) if scales else None
    null = ctypes.POINTER(ctypes.c_double)()
    keep, mptr = _mu_arg(mu, M)
    rc = _c().oracle_forward_range_mu(M, _dptr(sigma), mptr, d, int(rank0), int(count),
                                      convention, _dptr(corr), _dptr(cum),
                                      _dptr(smu) if scales else null,
                                      _dptr(skap) if scales else null, threads)
    if rc != 0:
        raise RuntimeError(f"oracle_forward_range failed ({rc})")
    return (corr, cum, smu, skap) if scales else (corr, cum)


def c_tolerance_scale(sigma: np.ndarray, d: int, ranks, convention: int = CLICK,
                      threads: int = 0, mu=None) -> tuple:
    """(smu, skap): the summand magnitudes of the two sums of each sampled output.

    smu(S) = sum_{T subset S} |w_T| p(T) for the correlator (inclusion-exclusion,
    w_T = (-1)^|T| click or (-2)^|T| parity); skap(S) = sum over set partitions of
    |w(pi)| prod_{B in pi} |m(B)| for the cumulant (the partition sum of Eq.
    cumulant_corr_main).  An FP64 evaluation of either sum is accurate to a
    small multiple of u times that scale, however much the terms cancel, so the
    stated tolerance is |delta| <= 1e-10 max(|ref|, 1e-4 scale).
    """
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    M = sigma.shape[0] // 2
    ranks = np.ascontiguousarray(ranks, dtype=np.int64)
    smu = np.empty(len(ranks))
    skap = np.empty(len(ranks))
    keep, mptr = _mu_arg(mu, M)
    rc = _c().oracle_tolerance_scale_mu(M, _dptr(sigma), mptr, d,
                                        ranks.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        len(ranks), convention, _dptr(smu), _dptr(skap), threads)
    if rc != 0:
        raise RuntimeError(f"oracle_tolerance_scale failed ({rc})")
    return smu, skap
