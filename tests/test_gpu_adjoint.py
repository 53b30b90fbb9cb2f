"""GPU parity of the adjoint (gbs_cumulant_grad) and of the torch.autograd chain
to per-mode transmissions and squeezings."""
import math
import sys

import numpy as np
import pytest

import gbs_inputs as G
import oracle as O

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2511_14923_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _grad(P, sigma, K, gcorr=None, gcum=None, flags=0):
    import torch
    M = sigma.shape[0] // 2
    g = P.gbs_cumulant_grad(M, _dev(sigma), K, flags,
                            grad_corr=_dev(gcorr) if gcorr is not None else None,
                            grad_cum=_dev(gcum) if gcum is not None else None)
    torch.cuda.synchronize()
    return g.cpu().numpy()


def _normwise(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_loss_gradient_matches_python_oracle(P):
    _say("case: adjoint vs python oracle M=7 K=3")
    inst = G.make_instance("grad_m144_k3", M=7, seed=51)
    _, _, sig_t = G.make_grad_target(inst)
    _, target = O.correlators_and_cumulants(sig_t, 3)
    _, kap = O.correlators_and_cumulants(inst.sigma, 3)
    _, ref = O.cumulant_loss_and_grad(inst.sigma, 3, target)
    got = _grad(P, inst.sigma, 3, gcum=2.0 * (kap - target))
    assert _normwise(got, ref) < 1e-10
    assert np.allclose(got, got.T, rtol=0, atol=0)


@pytest.mark.parametrize("K,conv", [(1, 0), (2, 0), (3, 0), (4, 0), (3, 1), (4, 1)])
def test_vjp_against_finite_differences(P, K, conv):
    """<grad, D> against central differences of the oracle's forward:
    f(sigma) = sum gc * corr(sigma) + sum gk * cum(sigma)."""
    _say("case: adjoint FD", K, conv)
    inst = G.make_instance("grad_m144_k3", M=6, seed=60 + K)
    N = O.total_outputs(6, K)
    rng = np.random.default_rng(K + 10 * conv)
    gc = rng.standard_normal(N)
    gk = rng.standard_normal(N)
    got = _grad(P, inst.sigma, K, gcorr=gc, gcum=gk, flags=conv)

    def f(s):
        c, k = O.correlators_and_cumulants(s, K, conv)
        return math.fsum(gc * c) + math.fsum(gk * k)

    h = 1e-6
    for _ in range(3):
        D = rng.standard_normal(inst.sigma.shape)
        D = 0.5 * (D + D.T)
        fd = (f(inst.sigma + h * D) - f(inst.sigma - h * D)) / (2 * h)
        an = float(np.sum(got * D))
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-9 * max(1.0, abs(fd)))


def test_grad_m144_k3_matches_c_oracle(P, c_oracle):
    """The M = 144, K = 3 gradient workload against the C oracle's reverse mode."""
    _say("case: adjoint M=144 K=3 vs C oracle")
    inst = G.make_instance("grad_m144_k3")
    _, _, sig_t = G.make_grad_target(inst)
    _, target = O.c_forward(sig_t, 3)
    _, kap = O.c_forward(inst.sigma, 3)
    loss_ref, ref = O.c_loss_grad(inst.sigma, 3, target)
    got = _grad(P, inst.sigma, 3, gcum=2.0 * (kap - target))
    err = _normwise(got, ref)
    _say("normwise |grad - oracle| / max|oracle|", err)
    assert err < 1e-10
    # bitwise reproducible
    again = _grad(P, inst.sigma, 3, gcum=2.0 * (kap - target))
    assert np.array_equal(got, again)


def test_autograd_chain_to_eta_and_r(P, c_oracle):
    """dL/d(eta, r) through GBSCumulants + the torch covariance model, against
    (a) the oracle's gradient chained analytically and (b) central differences
    (h = 1e-6) of the GPU forward along random directions in the 288 parameters."""
    import torch
    _say("case: autograd chain M=144 K=3")
    inst = G.make_instance("grad_m144_k3")
    _, _, sig_t = G.make_grad_target(inst)
    _, target = O.c_forward(sig_t, 3)
    W = P.interferometer_symplectic(torch.from_numpy(inst.U).to("cuda:0"))
    r = torch.tensor(inst.r, device="cuda:0", requires_grad=True)
    eta = torch.tensor(inst.eta, device="cuda:0", requires_grad=True)
    tgt = _dev(target)
    sigma_t = P.lossy_squeezed_covariance(W, r, eta)
    assert np.allclose(sigma_t.detach().cpu().numpy(), inst.sigma, rtol=1e-13, atol=1e-14)
    loss = P.cumulant_matching_loss(W, r, eta, tgt, 3)
    loss.backward()
    g_eta, g_r = eta.grad.cpu().numpy(), r.grad.cpu().numpy()
    # (a) oracle
    loss_ref, gsig_ref = O.c_loss_grad(inst.sigma, 3, target)
    d_eta, d_r = O.covariance_param_grad(inst.U, inst.r, inst.eta, gsig_ref)
    assert float(loss.detach()) == pytest.approx(loss_ref, rel=1e-10)
    assert _normwise(np.concatenate([g_eta, g_r]), np.concatenate([d_eta, d_r])) < 1e-9
    # (b) finite differences of the GPU forward
    rng = np.random.default_rng(7)
    h = 1e-6
    with torch.no_grad():
        for _ in range(2):
            v_eta = _dev(rng.standard_normal(144))
            v_r = _dev(rng.standard_normal(144))
            lp = P.cumulant_matching_loss(W, r + h * v_r, eta + h * v_eta, tgt, 3)
            lm = P.cumulant_matching_loss(W, r - h * v_r, eta - h * v_eta, tgt, 3)
            fd = float((lp - lm) / (2 * h))
            an = float((eta.grad * v_eta).sum() + (r.grad * v_r).sum())
            _say("directional derivative: analytic", an, "fd", fd)
            assert an == pytest.approx(fd, rel=1e-6)
