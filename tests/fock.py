"""Truncated Fock-basis simulator of a few modes (pure states), test-only.

Independent of the Gaussian formulas: gates are matrix exponentials of their
generators, moments and probabilities are sums over Fock amplitudes.
"""
import math

import numpy as np
from scipy.linalg import expm


def _lowering(N):
    return np.diag(np.sqrt(np.arange(1, N, dtype=np.float64)), 1).astype(complex)


class FockState:
    """Pure state of m modes as an amplitude tensor psi[n_0, ..., n_{m-1}]."""

    def __init__(self, m, N):
        self.m, self.N = m, N
        self.psi = np.zeros((N,) * m, dtype=complex)
        self.psi[(0,) * m] = 1.0
        self.a = _lowering(N)

    def _apply1(self, U, k):
        self.psi = np.moveaxis(np.tensordot(U, self.psi, axes=([1], [k])), 0, k)

    def squeeze(self, k, r):
        a = self.a
        self._apply1(expm(0.5 * r * (a @ a - a.conj().T @ a.conj().T)), k)

    def displace(self, k, alpha):
        a = self.a
        self._apply1(expm(alpha * a.conj().T - np.conj(alpha) * a), k)

    def rotate(self, k, phi):
        self._apply1(np.diag(np.exp(1j * phi * np.arange(self.N))), k)

    def beamsplitter(self, j, k, theta, phi):
        N = self.N
        a = self.a
        I = np.eye(N)
        aj, ak = np.kron(a, I), np.kron(I, a)
        H = theta * (np.exp(1j * phi) * aj.conj().T @ ak - np.exp(-1j * phi) * aj @ ak.conj().T)
        U = expm(H).reshape(N, N, N, N)
        self.psi = np.moveaxis(np.tensordot(U, self.psi, axes=([2, 3], [j, k])), [0, 1], [j, k])

    # -- observables -------------------------------------------------------

    def tail_weight(self, width=3):
        """Probability of any mode at one of the top `width` Fock levels."""
        w = np.abs(self.psi) ** 2
        tot = 0.0
        for k in range(self.m):
            tot += np.moveaxis(w, k, 0)[self.N - width:].sum()
        return tot

    def _quadratures(self):
        a = self.a
        x = (a + a.conj().T) / math.sqrt(2.0)
        p = (a - a.conj().T) / (1j * math.sqrt(2.0))
        return x, p

    def _apply_op(self, op, k, psi):
        return np.moveaxis(np.tensordot(op, psi, axes=([1], [k])), 0, k)

    def moments(self):
        """(sigma, mu) in xxpp order, hbar = 1: mu_i = <R_i>,
        sigma_ij = <R_i R_j + R_j R_i>/2 - mu_i mu_j."""
        x, p = self._quadratures()
        ops = [(x, k) for k in range(self.m)] + [(p, k) for k in range(self.m)]
        Rpsi = [self._apply_op(op, k, self.psi) for op, k in ops]
        n = 2 * self.m
        mu = np.array([np.vdot(self.psi, Rp).real for Rp in Rpsi])
        sig = np.empty((n, n))
        for i in range(n):
            for j in range(n):
                sig[i, j] = np.vdot(Rpsi[i], Rpsi[j]).real - mu[i] * mu[j]
        return 0.5 * (sig + sig.T), mu

    def vacuum_probability(self, T):
        """Probability that every mode of T is in vacuum (others traced out)."""
        w = np.abs(self.psi) ** 2
        idx = tuple(0 if k in T else slice(None) for k in range(self.m))
        return float(w[idx].sum())

    def click_correlator(self, S):
        """Probability that every mode of S holds at least one photon."""
        w = np.abs(self.psi) ** 2
        idx = tuple(slice(1, None) if k in S else slice(None) for k in range(self.m))
        return float(w[idx].sum())

    def parity_correlator(self, S):
        """<prod_{k in S} (2 |0><0|_k - 1)>: +1 for no photon, -1 otherwise,
        the product form of Eq. corre_cov_main's expansion."""
        w = np.abs(self.psi) ** 2
        sign = np.ones_like(w)
        for k in S:
            shape = [1] * self.m
            shape[k] = self.N
            s = -np.ones(self.N)
            s[0] = 1.0
            sign = sign * s.reshape(shape)
        return float((sign * w).sum())


def fock_cumulant(S, moment):
    """Partition sum over the Fock-basis moments (the definition, written
    out independently of the oracle's partition generator)."""
    S = tuple(S)
    if len(S) == 1:
        return moment(S)
    if len(S) == 2:
        return moment(S) - moment(S[:1]) * moment(S[1:])
    if len(S) == 3:
        a, b, c = [(s,) for s in S]
        m = moment
        return (m(S) - m(a) * m(tuple(sorted(b + c))) - m(b) * m(tuple(sorted(a + c)))
                - m(c) * m(tuple(sorted(a + b))) + 2 * m(a) * m(b) * m(c))
    raise ValueError("order > 3 not needed")


def two_mode_state():
    st = FockState(2, 40)
    st.squeeze(0, 0.45)
    st.squeeze(1, -0.3)
    st.displace(0, 0.6 + 0.3j)
    st.displace(1, -0.4 + 0.5j)
    st.beamsplitter(0, 1, 0.7, 0.4)
    st.rotate(1, 1.1)
    return st


def three_mode_state():
    st = FockState(3, 22)
    st.squeeze(0, 0.25)
    st.squeeze(1, -0.2)
    st.squeeze(2, 0.15)
    st.displace(0, 0.5 - 0.2j)
    st.displace(1, 0.3j)
    st.displace(2, -0.45 + 0.1j)
    st.beamsplitter(0, 1, 0.8, 0.3)
    st.beamsplitter(1, 2, 0.6, -0.9)
    st.rotate(2, 0.7)
    st.beamsplitter(0, 2, 0.5, 1.3)
    return st
