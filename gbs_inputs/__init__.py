"""Seeded synthetic Gaussian-boson-sampling inputs.

This module is the only code shared by the CPU oracle and the GPU path.  It
draws covariance matrices and random subset samples; it holds none of the
method's arithmetic (no vacuum probabilities, correlators or cumulants).

Physical model (paper, App. F "Benchmarking theory and implementation",
Eqs. jiuzhang_input_cov, symplectic_inter and ground_truth_cov): M single-mode
squeezed vacua enter a lossy linear interferometer; the output state is a
zero-mean Gaussian state with 2M x 2M quadrature covariance sigma in ``xxpp``
order (index k is x_k, index k+M is p_k), hbar = 1 so that the vacuum is I/2.

Conventions fixed here (the paper leaves them open):

* Haar unitary by QR of a complex Ginibre matrix with the phases of R's
  diagonal divided out (Mezzadri's recipe); draw order: real part, imaginary
  part of the Ginibre matrix, then squeezing r, then transmissions eta.
* Each input mode k is x-squeezed: its covariance is diag(e^{-2 r_k}, e^{2 r_k})/2.
* Loss eta_k acts on input k before the interferometer, i.e. the transmission
  matrix is T = U diag(sqrt(eta)).  With uniform eta this is exactly
  sigma = eta S S^T / 2 + (1 - eta) I / 2 with S the squeezed interferometer.
* Displaced inputs (first moments mu != 0, paper App. D.1 before Eq.
  vacuum_gaussian_prob): input k is D(alpha_k) S(r_k)|0>, with |alpha_k|^2 drawn
  uniformly from a stated range and a uniform phase; its mean is
  sqrt(2) (Re alpha_k, Im alpha_k) (hbar = 1), and the lossy interferometer maps
  input means linearly, mu = V mu_in with V the symplectic form of T.  The
  covariance is unchanged by the displacement.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "haar_unitary",
    "interferometer_symplectic",
    "lossy_squeezed_covariance",
    "Instance",
    "WORKLOADS",
    "make_instance",
    "make_batch",
    "vacuum_covariance",
    "product_state_covariance",
    "tmsv_covariance",
    "random_ranks",
    "local_phase_rotation",
    "mode_permutation",
    "input_displacement",
    "sampler_uniforms",
    "pseudo_pnr_covariance",
    "synthetic_parity_cumulants",
    "DISPLACEMENT_SEED",
    "DISPLACEMENT_AMP2",
]


def haar_unitary(M: int, rng: np.random.Generator) -> np.ndarray:
    """M x M Haar-random unitary (QR of a complex Ginibre matrix, phase-fixed)."""
    re = rng.standard_normal((M, M))
    im = rng.standard_normal((M, M))
    z = (re + 1j * im) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def interferometer_symplectic(T: np.ndarray) -> np.ndarray:
    """Real 2M x 2K matrix [[Re T, -Im T], [Im T, Re T]] acting on xxpp vectors
    (paper, Eq. symplectic_inter)."""
    return np.block([[T.real, -T.imag], [T.imag, T.real]])


def lossy_squeezed_covariance(U: np.ndarray, r: np.ndarray, eta: np.ndarray) -> np.ndarray:
    """Output covariance (xxpp, hbar=1) of M x-squeezed vacua with input-side
    transmissions ``eta`` sent through the unitary ``U``.

    sigma = V sigma_sq V^T + (I - V V^T)/2 with V the symplectic form of
    T = U diag(sqrt(eta)) (paper, Eq. ground_truth_cov with hbar = 1).
    """
    M = U.shape[0]
    r = np.asarray(r, dtype=np.float64).reshape(M)
    eta = np.broadcast_to(np.asarray(eta, dtype=np.float64), (M,))
    T = U * np.sqrt(eta)[None, :]
    V = interferometer_symplectic(T)
    sq = 0.5 * np.concatenate([np.exp(-2.0 * r), np.exp(2.0 * r)])
    sigma = (V * sq[None, :]) @ V.T + 0.5 * (np.eye(2 * M) - V @ V.T)
    return 0.5 * (sigma + sigma.T)


@dataclass(frozen=True)
class Workload:
    name: str
    M: int
    K: int
    r_range: tuple
    eta: object  # float (uniform) or (lo, hi) per-mode range
    seed: int
    precision: str = "fp64"
    note: str = ""


# The five workloads of the build.  Sizes and distributions follow the stated
# configurations; the paper's Jiuzhang squeezing/transmission data are not
# available, so Haar interferometers with squeezing in the same brightness range
# (mean photon number per mode 0.47-0.71; the paper's runs span 0.093-0.975)
# stand in for them.
WORKLOADS = {
    "m16_k3": Workload("m16_k3", 16, 3, (0.4, 1.2), 0.5, 2511_0001,
                       note="plain FP64, M=16, orders 1..3"),
    "m100_k4": Workload("m100_k4", 100, 4, (0.6, 1.4), 0.3, 2511_0002,
                        note="plain FP64, M=100, orders 1..4"),
    "m144_k5": Workload("m144_k5", 144, 5, (0.6, 1.6), (0.25, 0.4), 2511_0003,
                        precision="mixed+fp64", note="M=144, orders 1..5"),
    "batch48_k4": Workload("batch48_k4", 0, 4, (0.6, 1.6), (0.25, 0.4), 2511_0004,
                           note="48 instances, M ~ U{40..144}, orders 1..4"),
    "grad_m144_k3": Workload("grad_m144_k3", 144, 3, (0.6, 1.6), (0.25, 0.4), 2511_0005,
                             note="adjoint, M=144, orders 1..3"),
}
GRAD_TARGET_SEED = 2511_1005
# Displaced variant of a workload: same covariance, input amplitudes with
# |alpha|^2 ~ U[0.05, 0.5] (0.02-0.2 displaced photons per mode after the
# workloads' losses, small beside the squeezed photons).
DISPLACEMENT_SEED = 2511_0006
DISPLACEMENT_AMP2 = (0.05, 0.5)
BATCH_COUNT = 48
BATCH_M_RANGE = (40, 144)


@dataclass
class Instance:
    M: int
    U: np.ndarray
    r: np.ndarray
    eta: np.ndarray
    sigma: np.ndarray = field(repr=False)


def _draw_params(rng, M, r_range, eta_spec):
    U = haar_unitary(M, rng)
    r = rng.uniform(r_range[0], r_range[1], size=M)
    if isinstance(eta_spec, tuple):
        eta = rng.uniform(eta_spec[0], eta_spec[1], size=M)
    else:
        eta = np.full(M, float(eta_spec))
    return U, r, eta


def make_instance(name: str, M: int | None = None, seed: int | None = None) -> Instance:
    """Instance of a named workload (optionally overriding M or the seed)."""
    w = WORKLOADS[name]
    M = w.M if M is None else M
    rng = np.random.default_rng(w.seed if seed is None else seed)
    U, r, eta = _draw_params(rng, M, w.r_range, w.eta)
    return Instance(M, U, r, eta, lossy_squeezed_covariance(U, r, eta))


def make_grad_target(inst: Instance) -> tuple:
    """Second (r*, eta*) draw on the same interferometer, for the cumulant-matching loss."""
    w = WORKLOADS["grad_m144_k3"]
    rng = np.random.default_rng(GRAD_TARGET_SEED)
    r_t = rng.uniform(w.r_range[0], w.r_range[1], size=inst.M)
    eta_t = rng.uniform(w.eta[0], w.eta[1], size=inst.M)
    return r_t, eta_t, lossy_squeezed_covariance(inst.U, r_t, eta_t)


def make_batch(count: int = BATCH_COUNT, seed: int | None = None,
               m_range: tuple = BATCH_M_RANGE) -> list:
    """Independent instances with M ~ U{m_range} (inclusive), r, eta as M=144."""
    w = WORKLOADS["batch48_k4"]
    rng = np.random.default_rng(w.seed if seed is None else seed)
    Ms = rng.integers(m_range[0], m_range[1] + 1, size=count)
    out = []
    for M in Ms:
        U, r, eta = _draw_params(rng, int(M), w.r_range, w.eta)
        out.append(Instance(int(M), U, r, eta, lossy_squeezed_covariance(U, r, eta)))
    return out


def vacuum_covariance(M: int) -> np.ndarray:
    return 0.5 * np.eye(2 * M)


def product_state_covariance(r: np.ndarray, eta: np.ndarray) -> np.ndarray:
    """Identity interferometer: independent lossy squeezed modes."""
    M = len(r)
    return lossy_squeezed_covariance(np.eye(M, dtype=complex), r, eta)


def tmsv_covariance(r: float, M: int = 2, i: int = 0, j: int = 1) -> np.ndarray:
    """Pure two-mode squeezed vacuum on modes (i, j), vacuum elsewhere (xxpp, hbar=1).

    x-quadrature block [[ch, sh], [sh, ch]]/2, p-quadrature block
    [[ch, -sh], [-sh, ch]]/2 with ch = cosh 2r, sh = sinh 2r (the form of the
    paper's Eq. jiuzhang_input_cov, with its squeezing parameter read as 2r).
    """
    s = 0.5 * np.eye(2 * M)
    ch, sh = math.cosh(2 * r), math.sinh(2 * r)
    for (a, b) in ((i, i), (j, j)):
        s[a, b] = 0.5 * ch
        s[a + M, b + M] = 0.5 * ch
    s[i, j] = s[j, i] = 0.5 * sh
    s[i + M, j + M] = s[j + M, i + M] = -0.5 * sh
    return s


def local_phase_rotation(sigma: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Apply an independent phase rotation to every mode (xxpp)."""
    M = sigma.shape[0] // 2
    c, s = np.cos(theta), np.sin(theta)
    R = np.zeros((2 * M, 2 * M))
    R[np.arange(M), np.arange(M)] = c
    R[np.arange(M) + M, np.arange(M) + M] = c
    R[np.arange(M), np.arange(M) + M] = -s
    R[np.arange(M) + M, np.arange(M)] = s
    out = R @ sigma @ R.T
    return 0.5 * (out + out.T)


def mode_permutation(sigma: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """Relabel modes: new mode k is old mode perm[k]."""
    M = sigma.shape[0] // 2
    idx = np.concatenate([perm, perm + M])
    return sigma[np.ix_(idx, idx)].copy()


def random_ranks(count_total: int, n: int, seed: int) -> np.ndarray:
    """``n`` distinct sorted ranks drawn uniformly from [0, count_total)."""
    rng = np.random.default_rng(seed)
    n = min(n, count_total)
    if count_total <= 4 * n:
        return np.sort(rng.permutation(count_total)[:n]).astype(np.int64)
    picks = set()
    while len(picks) < n:
        picks.update(int(x) for x in rng.integers(0, count_total, size=n - len(picks)))
    return np.array(sorted(picks), dtype=np.int64)


def input_displacement(inst: Instance, seed: int = DISPLACEMENT_SEED,
                       amp2_range: tuple = DISPLACEMENT_AMP2) -> np.ndarray:
    """Output first moments (xxpp, hbar = 1, length 2M) when input k of ``inst``
    is displaced by alpha_k, |alpha_k|^2 ~ U[amp2_range], phase ~ U[0, 2 pi);
    draw order: all |alpha|^2, then all phases."""
    rng = np.random.default_rng(seed)
    amp2 = rng.uniform(amp2_range[0], amp2_range[1], size=inst.M)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=inst.M)
    alpha = np.sqrt(amp2) * np.exp(1j * phase)
    mu_in = math.sqrt(2.0) * np.concatenate([alpha.real, alpha.imag])
    V = interferometer_symplectic(inst.U * np.sqrt(inst.eta)[None, :])
    return V @ mu_in


def sampler_uniforms(M: int, n: int, seed: int) -> np.ndarray:
    """(M, n) uniforms in [0, 1) for n samples of M bits (row m: bit m + 1)."""
    return np.random.default_rng(seed).random((M, n))


def synthetic_parity_cumulants(M: int, K: int, seed: int) -> np.ndarray:
    """A seeded array in the cumulant layout (orders 1..K, colex inside an
    order), cheap at any M: order 1 ~ U[0.2, 0.7] (parity correlators of modes
    that click with probability 0.15-0.4), order d >= 2 ~ N(0, (0.1 / 2^d)^2).
    Not the cumulants of any particular state: a stand-in input for sampler
    parity tests at sizes where exact cumulants are too slow to compute on a CPU."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(0.2, 0.7, size=M)]
    for d in range(2, K + 1):
        parts.append(rng.normal(0.0, 0.1 / 2 ** d, size=math.comb(M, d)))
    return np.concatenate(parts)


def pseudo_pnr_covariance(sigma: np.ndarray, k: int = 8) -> np.ndarray:
    """Covariance (xxpp, hbar = 1) after every mode of ``sigma`` is split evenly
    over k threshold detectors (pseudo-photon-number resolution): mode g and
    k - 1 vacua enter a k x k discrete Fourier transform whose outputs are
    modes g k .. g k + k - 1.  M modes become M k (144 -> 1152 for k = 8)."""
    M0 = sigma.shape[0] // 2
    M = M0 * k
    sin = 0.5 * np.eye(2 * M)
    sig_idx = np.arange(M0) * k  # input index of signal g: g k + 0
    idx = np.concatenate([sig_idx, sig_idx + M])
    sin[np.ix_(idx, idx)] = sigma
    F = np.exp(2j * math.pi * np.outer(np.arange(k), np.arange(k)) / k) / math.sqrt(k)
    U = np.kron(np.eye(M0), F)
    W = interferometer_symplectic(U)
    out = W @ sin @ W.T
    return 0.5 * (out + out.T)
