"""GPU parity of the sample statistics (gbs_sample_cumulants, gbs_pearson)
against the oracle (oracle/estimators.py, exact rational arithmetic), and the
stage-1 -> sampler -> estimator loop at M = 144 against the oracle's ground
truth.  Parity inputs are seeded host-side bit arrays; the loop test consumes
the GPU sampler's own output and asserts only properties of it."""
import sys

import numpy as np
import pytest

import gbs_inputs as G
import oracle as O
from oracle import estimators as E

pytestmark = pytest.mark.gpu


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


def _bits(N, M, seed):
    rng = np.random.default_rng(seed)
    base = rng.random((N, 1)) < 0.3
    return ((rng.random((N, M)) < 0.35) | (base & (rng.random((N, M)) < 0.4))).astype(np.uint8)


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.mark.parametrize("M,K,N", [(1, 1, 1), (5, 5, 5), (10, 5, 500), (24, 4, 2000),
                                   (17, 3, 64), (40, 3, 4097)])
def test_sample_cumulants_match_oracle(P, M, K, N):
    import torch
    _say("case: estimator", M, K, N)
    b = _bits(N, M, 100 + M + N)
    got = P.gbs_sample_cumulants(_dev(b), K)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    ref = E.sample_cumulants(b, K)
    scale = max(1.0, float(np.abs(ref).max()))
    # exact rational reference; the FP64 partition sum cancels terms of size ~1
    tol = 1e-13 * scale if N >= 64 else 1e-11 * scale
    assert np.max(np.abs(got - ref)) <= tol, (np.max(np.abs(got - ref)), tol)


def test_pearson_matches_oracle(P):
    import torch
    _say("case: pearson")
    rng = np.random.default_rng(7)
    for n in (2, 3, 1000, 300_001):
        x = rng.normal(size=n)
        y = 0.4 * x + rng.normal(size=n) + 5.0
        r = P.gbs_pearson(_dev(x), _dev(y))
        torch.cuda.synchronize()
        assert abs(float(r.item()) - E.pearson(x, y)) <= 1e-13


def test_stage1_sampler_estimator_loop(P):
    """M = 144: ground truth of orders 1..3 from the oracle; 262,144 samples from
    the single-elision sampler on the GPU's own parity cumulants; the GPU
    estimator's click cumulants correlate with the ground truth order by order."""
    import torch
    _say("case: validation loop M=144")
    inst = G.make_instance("m144_k5")
    sig = _dev(inst.sigma)
    _, kap = P.gbs_cumulants(144, sig, 3, P.GBS_PARITY, want_corr=False)
    u = _dev(G.sampler_uniforms(144, 262_144, 11))
    bits, _, _ = P.gbs_sample(144, kap, 3, u, want_prob=False)
    est = P.gbs_sample_cumulants(bits, 3)
    _, truth = O.c_forward(inst.sigma, 3, O.CLICK)
    tdev = _dev(truth)
    rs = []
    for d in (1, 2, 3):
        a, b = O.order_offset(144, d), O.order_offset(144, d + 1)
        r = P.gbs_pearson(est[a:b].contiguous(), tdev[a:b].contiguous())
        rs.append(float(r.item()))
    torch.cuda.synchronize()
    _say("pearson by order", rs)
    # Sampling noise alone limits r at this N: with the ground truth's spread and
    # the estimator's variance (about prod mu(1 - mu) / N) the expected values
    # are 0.9974, 0.865 and 0.115 for orders 1-3.
    assert rs[0] > 0.99 and rs[1] > 0.8 and rs[2] > 0.03
    # standardised residuals of orders 1 and 2: mean ~ 0, spread ~ 1
    e = est.cpu().numpy()
    n = 262_144
    mu1 = truth[:144]
    z1 = (e[:144] - mu1) / np.sqrt(mu1 * (1 - mu1) / n)
    a, b = O.order_offset(144, 2), O.order_offset(144, 3)
    pairs = np.array(list(O.subsets_colex(144, 2)))
    v2 = mu1[pairs[:, 0]] * (1 - mu1[pairs[:, 0]]) * mu1[pairs[:, 1]] * (1 - mu1[pairs[:, 1]]) / n
    z2 = (e[a:b] - truth[a:b]) / np.sqrt(v2)
    _say("z1 mean/std", z1.mean(), z1.std(), "z2 mean/std", z2.mean(), z2.std())
    assert abs(z1.mean()) < 0.5 and 0.6 < z1.std() < 1.6
    assert abs(z2.mean()) < 0.2 and 0.7 < z2.std() < 1.4
