"""The Python binding checks every buffer's size, dtype, layout and device
before it calls into libgbs (whose C ABI sees bare pointers and cannot): each
bad call below raises ValueError or TypeError without launching anything.  CPU
tensors serve as stand-ins, so no GPU is needed; the size checks come before
the device check, and a right-sized CPU tensor fails the device check."""
import pytest
import torch

import paper_2511_14923_amd as P

f64 = torch.float64


def z(*shape, dtype=f64):
    return torch.zeros(*shape, dtype=dtype)


def test_sigma_size_shape_dtype_layout():
    M, K = 6, 3
    with pytest.raises(ValueError, match="sigma: 144 elements"):
        P.gbs_cumulants(M, z(10, 10), K)
    with pytest.raises(ValueError, match="sigma: shape"):
        P.gbs_cumulants(M, z(6, 24), K)
    with pytest.raises(ValueError, match="float64"):
        P.gbs_cumulants(M, z(12, 12, dtype=torch.float32), K)
    with pytest.raises(ValueError, match="contiguous"):
        P.gbs_cumulants(M, z(24, 12)[::2], K)
    with pytest.raises(TypeError):
        P.gbs_cumulants(M, [[0.0] * 12] * 12, K)


def test_bad_orders_rejected():
    with pytest.raises(ValueError, match="invalid M"):
        P.gbs_cumulants(4, z(8, 8), 5)
    with pytest.raises(ValueError, match="invalid M"):
        P.gbs_correlators(0, z(0), 1)


def test_output_sizes():
    M, K = 6, 3
    n = P.gbs_total_outputs(M, K)
    with pytest.raises(ValueError, match=f"corr: {n} elements"):
        P.gbs_correlators(M, z(12, 12), K, corr=z(n - 1))
    with pytest.raises(ValueError, match=f"cum: {n} elements"):
        P.gbs_cumulants(M, z(12, 12), K, corr=z(n), cum=z(n + 1))
    with pytest.raises(ValueError, match=f"corr: {n} elements"):
        P.gbs_cumulants(M, z(12, 12), K, corr=z(5), cum=z(n))
    # right sizes, host tensors: the device check fires
    with pytest.raises(ValueError, match="device tensor required"):
        P.gbs_cumulants(M, z(12, 12), K, corr=z(n), cum=z(n))


def test_displaced_mean_size():
    M, K = 6, 3
    n = P.gbs_total_outputs(M, K)
    with pytest.raises(ValueError, match="mu: 12 elements"):
        P.gbs_cumulants_displaced(M, z(12, 12), z(6), K, corr=z(n), cum=z(n))


def test_shard_range_and_sizes():
    M = 10
    with pytest.raises(ValueError, match="rank range"):
        P.gbs_cumulants_shard(M, z(20, 20), 3, 100, 21)
    with pytest.raises(ValueError, match="rank range"):
        P.gbs_cumulants_shard(M, z(20, 20), 3, -1, 5)
    with pytest.raises(ValueError, match="invalid M"):
        P.gbs_cumulants_shard(M, z(20, 20), 6, 0, 1)
    with pytest.raises(ValueError, match="cum: 7 elements"):
        P.gbs_cumulants_shard(M, z(20, 20), 3, 0, 7, corr=z(7), cum=z(8))


def test_gradient_sizes():
    M, K = 6, 3
    n = P.gbs_total_outputs(M, K)
    with pytest.raises(ValueError, match="grad_cum"):
        P.gbs_cumulant_grad(M, z(12, 12), K, grad_cum=z(n - 2))
    with pytest.raises(ValueError, match="grad_corr"):
        P.gbs_cumulant_grad(M, z(12, 12), K, grad_corr=z(n + 2), grad_cum=z(n))
    with pytest.raises(ValueError, match="grad_sigma"):
        P.gbs_cumulant_grad(M, z(12, 12), K, grad_cum=z(n), grad_sigma=z(11, 11))


def test_batched_instance_sizes():
    n6 = P.gbs_total_outputs(6, 3)
    n9 = P.gbs_total_outputs(9, 3)
    good = (6, z(12, 12), None, z(n6))
    with pytest.raises(ValueError, match="at least one"):
        P.gbs_cumulants_batched([], 3)
    with pytest.raises(ValueError, match="instance 1 cum"):
        P.gbs_cumulants_batched([good, (9, z(18, 18), None, z(n6))], 3)
    with pytest.raises(ValueError, match="instance 1 sigma"):
        P.gbs_cumulants_batched([good, (9, z(12, 12), None, z(n9))], 3)
    with pytest.raises(ValueError, match="instance 0 corr"):
        P.gbs_autotune_batched([(6, z(12, 12), z(3), z(n6))], 3)


def test_sampler_sizes():
    M, K, n = 8, 3, 64
    nk = P.gbs_total_outputs(M, K)
    with pytest.raises(ValueError, match="kappa"):
        P.gbs_sample(M, z(nk - 1), K, z(M, n))
    with pytest.raises(ValueError, match="uniforms: shape"):
        P.gbs_sample(M, z(nk), K, z(M + 1, n))
    with pytest.raises(ValueError, match="multiple of M"):
        P.gbs_sample(M, z(nk), K, z(M * n + 3))
    with pytest.raises(ValueError, match="bits"):
        P.gbs_sample(M, z(nk), K, z(M, n), bits=z(n, M - 1, dtype=torch.uint8))
    with pytest.raises(ValueError, match="uint8"):
        P.gbs_sample(M, z(nk), K, z(M, n), bits=z(n, M))
    with pytest.raises(ValueError, match="prob"):
        P.gbs_sample(M, z(nk), K, z(M, n), prob=z(n - 1))
    with pytest.raises(ValueError, match="cond"):
        P.gbs_sample(M, z(nk), K, z(M, n), cond=z(M, n - 1))


def test_estimator_sizes():
    with pytest.raises(ValueError, match="shape"):
        P.gbs_sample_cumulants(z(100, dtype=torch.uint8), 2)
    nk = P.gbs_total_outputs(5, 2)
    with pytest.raises(ValueError, match="cum"):
        P.gbs_sample_cumulants(z(100, 5, dtype=torch.uint8), 2, cum=z(nk + 1))
    with pytest.raises(ValueError, match="y: 10 elements"):
        P.gbs_pearson(z(10), z(9))
    with pytest.raises(ValueError, match="r: 1 elements"):
        P.gbs_pearson(z(10), z(10), r=z(2))
