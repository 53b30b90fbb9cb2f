"""The torch covariance model used by the autograd chain agrees with the seeded
input generator (CPU; no GPU or library call)."""
import numpy as np
import torch

import gbs_inputs as G
import paper_2511_14923_amd as P


def test_torch_model_matches_generator():
    inst = G.make_instance("grad_m144_k3", M=10, seed=3)
    W = P.interferometer_symplectic(torch.from_numpy(inst.U))
    s = P.lossy_squeezed_covariance(W, torch.from_numpy(inst.r), torch.from_numpy(inst.eta))
    assert np.allclose(s.numpy(), inst.sigma, rtol=1e-13, atol=1e-14)


def test_uniform_loss_closed_form():
    """With uniform eta the model is eta S S^T / 2 + (1 - eta) I / 2."""
    inst = G.make_instance("m16_k3", M=8, seed=4)
    W = G.interferometer_symplectic(inst.U)
    Sq = W @ np.diag(np.concatenate([np.exp(-inst.r), np.exp(inst.r)]))
    eta = inst.eta[0]
    ref = eta * Sq @ Sq.T / 2 + (1 - eta) * np.eye(16) / 2
    assert np.allclose(inst.sigma, ref, rtol=1e-12, atol=1e-14)
