"""GPU parity of the stage-2 sampler (gbs_sample) against the sampler oracle,
through the C ABI.

Both sides consume the same cumulants and uniforms.  A bit decision compares a
uniform with a floating-point conditional, so the two sides may legitimately
part ways where u lies within rounding of the conditional; each sample is
therefore compared up to its first differing bit, which must be such a near
tie, and the oracle's probabilities are evaluated on the GPU's path."""
import math
import sys

import numpy as np
import pytest

import gbs_inputs as G
import oracle as O
from oracle import sampler as S

pytestmark = pytest.mark.gpu

TIE = 1e-12  # |u - conditional| within which either decision is correct


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2511_14923_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.lib()
    return P


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _gpu_sample(P, cum, M, K, u, batch=0):
    import torch
    bits, prob, cond = P.gbs_sample(M, _dev(cum), K, _dev(u), batch=batch, want_cond=True)
    torch.cuda.synchronize()
    return bits.cpu().numpy(), prob.cpu().numpy(), cond.cpu().numpy()


def _compare(cum, M, K, u, bits, prob, cond, what):
    """Oracle on the GPU's paths (teacher-forced) and with the same uniforms."""
    fb, fprob, fcond = S.c_sample(cum, M, K, forced=bits)
    rb, _, _ = S.c_sample(cum, M, K, u=u)
    n = u.shape[1]
    # conditionals and probabilities along the GPU's own path
    assert np.allclose(cond, fcond, rtol=1e-11, atol=1e-14), f"{what}: conditionals"
    assert np.all(np.abs(prob - fprob) <= 1e-11 * np.abs(fprob)), f"{what}: pattern probabilities"
    # decisions: identical, or the first difference is a near tie
    ties = 0
    for s in range(n):
        diff = np.nonzero(bits[s] != rb[s])[0]
        if len(diff):
            m = diff[0]
            assert abs(u[m, s] - fcond[m, s]) <= TIE, f"{what}: sample {s} bit {m + 1}"
            ties += 1
        assert np.array_equal(bits[s], (u[:, s] < cond[:, s]).astype(np.uint8))
    return ties


@pytest.mark.parametrize("K,M,n,batch", [(3, 20, 300, 64), (3, 3, 70, 0), (5, 12, 200, 64),
                                         (5, 5, 65, 0), (5, 7, 1, 0)])
def test_small_gaussian(P, K, M, n, batch):
    _say("case: sampler small", K, M, n, batch)
    inst = G.make_instance("m144_k5", M=M, seed=200 + M)
    _, cum = O.c_forward(inst.sigma, K, O.PARITY)
    u = G.sampler_uniforms(M, n, 300 + M)
    bits, prob, cond = _gpu_sample(P, cum, M, K, u, batch)
    assert _compare(cum, M, K, u, bits, prob, cond, f"K={K} M={M}") <= 1


def test_k3_m144_gaussian(P):
    """Single elision at the workload's size: M = 144, the oracle's K = 3 parity
    cumulants of the M = 144 covariance, 512 samples (8 workgroups)."""
    _say("case: sampler K=3 M=144")
    inst = G.make_instance("m144_k5")
    _, cum = O.c_forward(inst.sigma, 3, O.PARITY)
    u = G.sampler_uniforms(144, 512, 7)
    bits, prob, cond = _gpu_sample(P, cum, 144, 3, u)
    assert _compare(cum, 144, 3, u, bits, prob, cond, "K=3 M=144") <= 2
    assert 0.2 < bits.mean() < 0.6


def test_k5_m60_gaussian(P):
    """Double elision with the oracle's K = 5 parity cumulants of an M = 60
    covariance, 130 samples (ragged last workgroup), two launches."""
    _say("case: sampler K=5 M=60")
    inst = G.make_instance("m144_k5", M=60, seed=61)
    _, cum = O.c_forward(inst.sigma, 5, O.PARITY)
    u = G.sampler_uniforms(60, 130, 8)
    bits, prob, cond = _gpu_sample(P, cum, 60, 5, u, batch=64)
    assert _compare(cum, 60, 5, u, bits, prob, cond, "K=5 M=60") <= 1


def test_k5_m144_synthetic(P):
    """Double elision at M = 144 in the benchmark's launch shape, on a seeded
    synthetic cumulant array (exact K = 5 cumulants of the M = 144 state take
    minutes on a CPU); 24 samples checked against the C oracle."""
    _say("case: sampler K=5 M=144 synthetic")
    cum = G.synthetic_parity_cumulants(144, 5, 9)
    u = G.sampler_uniforms(144, 24, 10)
    bits, prob, cond = _gpu_sample(P, cum, 144, 5, u)
    assert _compare(cum, 144, 5, u, bits, prob, cond, "K=5 M=144") <= 1


@pytest.mark.parametrize("K", [3, 5])
def test_frequencies_of_independent_pairs(P, K):
    """200,000 samples of a distribution both methods represent exactly
    (independent consecutive bit pairs): chi-square against the closed form."""
    _say("case: sampler pair frequencies", K)
    M = 8
    rng = np.random.default_rng(40 + K)
    blocks = [(list(range(k, k + 2)), rng.dirichlet(np.full(4, 2.0))) for k in range(0, M, 2)]
    cum = np.zeros(O.total_outputs(M, K))
    for modes, w in blocks:
        ez0 = w[0] - w[1] + w[2] - w[3]
        ez1 = w[0] + w[1] - w[2] - w[3]
        ez01 = w[0] - w[1] - w[2] + w[3]
        cum[modes[0]] = ez0
        cum[modes[1]] = ez1
        cum[O.order_offset(M, 2) + O.colex_rank(tuple(modes))] = ez01 - ez0 * ez1
    n = 200_000
    u = G.sampler_uniforms(M, n, 50 + K)
    bits, _, _ = _gpu_sample(P, cum, M, K, u)
    idx = (bits.astype(np.int64) << np.arange(M)).sum(axis=1)
    counts = np.bincount(idx, minlength=1 << M)
    expect = np.array([math.prod(w[((x >> m[0]) & 1) | (((x >> m[1]) & 1) << 1)] for m, w in blocks)
                       for x in range(1 << M)]) * n
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    from scipy.stats import chi2 as dist
    assert dist.sf(chi2, (1 << M) - 1) > 1e-4


def test_zero_samples_and_null_outputs(P):
    import torch
    _say("case: sampler edge")
    inst = G.make_instance("m144_k5", M=6, seed=5)
    _, cum = O.c_forward(inst.sigma, 3, O.PARITY)
    kd = _dev(cum)
    u0 = torch.empty((6, 0), dtype=torch.float64, device="cuda:0")
    bits, prob, cond = P.gbs_sample(6, kd, 3, u0)
    assert bits.shape == (0, 6)
    u = G.sampler_uniforms(6, 40, 3)
    b1, _, _ = P.gbs_sample(6, kd, 3, _dev(u), want_prob=False)
    b2, p2, c2 = P.gbs_sample(6, kd, 3, _dev(u), want_cond=True)
    torch.cuda.synchronize()
    assert torch.equal(b1, b2)
