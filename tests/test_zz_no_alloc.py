"""The allocation-free entry point gbs_cumulants_noalloc against gbs_cumulants,
through the C ABI: the same kernels on the same inputs, so the outputs must be
identical bit for bit; two calls in a row with the second smaller, a return to
the first layout (tile plans copied in again), the other flag combinations,
the scratch limit, asynchronous status, a non-SPD input, and device memory
unchanged across calls."""
import sys

import numpy as np
import pytest

import gbs_inputs as G
from parity import assert_within, fp64_scales, fp64_tolerance

gpu = pytest.mark.gpu


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


def _pair(P, M, K, flags, sigma, with_corr=True):
    """(reference outputs of gbs_cumulants, outputs of gbs_cumulants_noalloc)."""
    import torch
    s = torch.from_numpy(np.ascontiguousarray(sigma)).to("cuda:0")
    n = P.gbs_total_outputs(M, K)
    rc, rk = P.gbs_cumulants(M, s, K, flags, want_corr=with_corr)
    corr = torch.full((n,), np.nan, dtype=torch.float64, device="cuda:0") if with_corr else None
    cum = torch.full((n,), np.nan, dtype=torch.float64, device="cuda:0")
    P.gbs_cumulants_noalloc(M, s, K, flags, corr, cum)
    torch.cuda.synchronize()
    ref = (rc.cpu().numpy() if with_corr else None, rk.cpu().numpy())
    got = (corr.cpu().numpy() if with_corr else None, cum.cpu().numpy())
    return ref, got


def _same(ref, got, what):
    for r, g, name in ((ref[0], got[0], "corr"), (ref[1], got[1], "cum")):
        if r is None:
            continue
        assert np.all(np.isfinite(g)), f"{what} {name}: unwritten outputs"
        assert np.array_equal(r, g), f"{what} {name}: max |delta| {np.abs(r - g).max():.3e}"


@gpu
def test_two_calls_second_smaller(P):
    big = G.make_instance("m144_k5")
    small = G.make_instance("m144_k5", M=40, seed=5)
    _say("case: noalloc M=144 K=5 then M=40 K=4 then M=144 K=5")
    ref, got = _pair(P, 144, 5, 0, big.sigma)
    _same(ref, got, "M=144 K=5")
    ref2, got2 = _pair(P, 40, 4, 0, small.sigma)
    _same(ref2, got2, "M=40 K=4")
    # back to the first layout: its tile plans are copied in again
    _, got3 = _pair(P, 144, 5, 0, big.sigma)
    _same(ref, got3, "M=144 K=5 again")


@gpu
def test_against_the_oracle(P, c_oracle):
    """The same bar as the other parity tests: sampled outputs of the smaller
    call against the FP64 oracle."""
    import oracle as O
    inst = G.make_instance("m144_k5", M=40, seed=5)
    _say("case: noalloc M=40 K=4 vs oracle")
    _, got = _pair(P, 40, 4, 0, inst.sigma)
    for d in range(1, 5):
        cnt = O.num_subsets(40, d)
        ranks = G.random_ranks(cnt, min(cnt, 2000), seed=60 + d)
        rc, rk = O.c_forward_sample(inst.sigma, d, ranks)
        smu, skap = fp64_scales(inst.sigma, d, ranks)
        off = O.order_offset(40, d)
        assert_within(got[0][off + ranks], rc, fp64_tolerance(rc, smu), f"corr d={d}")
        assert_within(got[1][off + ranks], rk, fp64_tolerance(rk, skap), f"cum d={d}")


@gpu
@pytest.mark.parametrize("flags,with_corr", [(1, True), (2, True), (16, True), (0, False), (3, False)],
                         ids=["parity", "mixed", "all_minors", "corr_null", "mixed_parity_corr_null"])
def test_flag_combinations(P, flags, with_corr):
    inst = G.make_instance("m144_k5", M=33, seed=8)
    _say(f"case: noalloc M=33 K=5 flags={flags} corr={'given' if with_corr else 'NULL'}")
    ref, got = _pair(P, 33, 5, flags, inst.sigma, with_corr)
    _same(ref, got, f"flags={flags}")


@gpu
def test_scratch_limit_and_unsupported(P):
    import torch
    inst = G.make_instance("m144_k5")
    s = torch.from_numpy(inst.sigma).to("cuda:0")
    n = P.gbs_total_outputs(144, 5)
    cum = torch.empty(n, dtype=torch.float64, device="cuda:0")
    _say("case: noalloc scratch limit (M=144 K=5, corr NULL)")
    with pytest.raises(P.GBSError) as ei:  # the correlator tables would not fit
        P.gbs_cumulants_noalloc(144, s, 5, 0, None, cum)
    assert ei.value.status == P.GBS_E_SCRATCH_LIMIT
    small = torch.from_numpy(G.make_instance("m144_k5", M=12, seed=2).sigma).to("cuda:0")
    c12 = torch.empty(P.gbs_total_outputs(12, 3), dtype=torch.float64, device="cuda:0")
    with pytest.raises(P.GBSError) as ei:
        P.gbs_cumulants_noalloc(12, small, 3, P.GBS_TIMING, None, c12)
    assert ei.value.status == P.GBS_E_UNSUPPORTED


@gpu
def test_async_status_and_not_spd(P):
    import torch
    M = 6
    _say("case: noalloc async and not SPD")
    good = torch.from_numpy(G.vacuum_covariance(M)).to("cuda:0")
    cum = torch.empty(P.gbs_total_outputs(M, 3), dtype=torch.float64, device="cuda:0")
    P.gbs_cumulants_noalloc(M, good, 3, P.GBS_ASYNC, None, cum)
    torch.cuda.synchronize()
    assert P.gbs_last_error()[0] == P.GBS_OK
    bad = G.vacuum_covariance(M)
    bad[2, 2] = bad[2 + M, 2 + M] = -0.9  # mode 2: Q_22 has negative pivots
    with pytest.raises(P.GBSError) as ei:
        P.gbs_cumulants_noalloc(M, torch.from_numpy(bad).to("cuda:0"), 3, 0, None, cum)
    assert ei.value.status == P.GBS_E_NOT_SPD
    st, order, rank = P.gbs_last_error()
    assert st == P.GBS_E_NOT_SPD and 1 <= order <= 3
    assert 2 in P.gbs_colex_unrank(order, rank)
    P.gbs_cumulants_noalloc(M, torch.from_numpy(bad).to("cuda:0"), 3, P.GBS_ASYNC, None, cum)
    torch.cuda.synchronize()
    assert P.gbs_last_error()[0] == P.GBS_E_NOT_SPD
    P.gbs_cumulants_noalloc(M, good, 3, 0, None, cum)
    assert P.gbs_last_error()[0] == P.GBS_OK


@gpu
def test_device_memory_unchanged(P):
    """After set-up, calls change neither the device's free memory nor
    torch's allocations."""
    import torch
    inst = G.make_instance("m144_k5", M=60, seed=3)
    s = torch.from_numpy(inst.sigma).to("cuda:0")
    n = P.gbs_total_outputs(60, 5)
    corr = torch.empty(n, dtype=torch.float64, device="cuda:0")
    cum = torch.empty(n, dtype=torch.float64, device="cuda:0")
    _say("case: noalloc device memory")
    P.gbs_cumulants_noalloc(60, s, 5, 0, corr, cum)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    alloc0 = torch.cuda.memory_allocated()
    for flags in (0, P.GBS_MIXED, P.GBS_PARITY, 0):
        P.gbs_cumulants_noalloc(60, s, 5, flags, corr, cum)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    # an allocation would lower the free memory (a late trim of earlier calls'
    # stream-ordered frees could only raise it)
    assert free1 >= free0 and torch.cuda.memory_allocated() == alloc0


def test_host_checks_before_any_launch():
    """Rejections that happen on the host, before the device is touched (the
    pointers are never dereferenced): argument errors, the scratch limit and
    GBS_TIMING."""
    import ctypes
    import paper_2511_14923_amd as P
    L = P.lib()
    fake = ctypes.c_void_p(0x1000)
    f = L.gbs_cumulants_noalloc
    assert f(144, fake, 5, 0, None, fake, None) == P.GBS_E_SCRATCH_LIMIT      # corr NULL: too large
    assert f(200, fake, 5, 0, fake, fake, None) == P.GBS_E_SCRATCH_LIMIT      # p tables too large
    assert f(12, fake, 3, P.GBS_TIMING, None, fake, None) == P.GBS_E_UNSUPPORTED
    assert f(0, fake, 1, 0, None, fake, None) == P.GBS_E_INVALID_ARG
    assert f(12, None, 3, 0, None, fake, None) == P.GBS_E_INVALID_ARG
    assert f(12, fake, 3, 0, fake, None, None) == P.GBS_E_INVALID_ARG
    assert f(12, fake, 6, 0, None, fake, None) == P.GBS_E_INVALID_ARG
    assert f(12, fake, 3, 64, None, fake, None) == P.GBS_E_INVALID_ARG
    assert "GBS_NOALLOC_SCRATCH_BYTES" in P.gbs_status_string(P.GBS_E_SCRATCH_LIMIT)
