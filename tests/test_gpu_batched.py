"""GPU tests of the batched persistent launch (gbs_cumulants_batched), its HIP
graph replay and the autotuner."""
import math
import sys

import numpy as np
import pytest

import gbs_inputs as G
import oracle as O
from parity import assert_within, fp64_scales, fp64_tolerance

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


def _alloc(batch, K, want_corr=True):
    import torch
    out = []
    for inst in batch:
        s = torch.from_numpy(inst.sigma).to("cuda:0")
        n = O.total_outputs(inst.M, K)
        corr = torch.empty(n, dtype=torch.float64, device="cuda:0") if want_corr else None
        cum = torch.empty(n, dtype=torch.float64, device="cuda:0")
        out.append((inst.M, s, corr, cum))
    return out


def _singles(P, bufs, K, flags):
    """Single-instance calls of the same kernels: the default ones (the batched
    launch runs the group kernel at orders >= 3, FP64 or mixed), the all-minors
    kernel for GBS_ALL_MINORS."""
    return [P.gbs_cumulants(M, s, K, flags) for (M, s, _, _) in bufs]


def _agree(a, b):
    """Same FP64 arithmetic compiled into two kernels: equal up to the last few
    ulps of the terms that cancel (|terms| <= 2^K)."""
    import torch
    return bool(torch.allclose(a, b, rtol=1e-12, atol=1e-13))


@pytest.mark.parametrize("flags", [0, 1, 2, 16, 18],
                         ids=["fp64", "parity", "mixed", "all_minors", "mixed_all_minors"])
def test_batch48_equals_single_calls(P, flags):
    """The 48-instance M ~ U{40..144}, K = 4 workload: every instance's output
    agrees with a separate gbs_cumulants call.  FP64 runs the same arithmetic
    on both sides; the mixed form's orders 1 and 2 take their FP32 roundings in
    other orders in the two paths (all minors per subset against the
    order-recursive kernels), so there the two differ, order by order and
    normwise over all instances, by at most twice the mixed form's stated
    bound (each side is within it of the exact value)."""
    import torch
    _say("case: batch48", flags)
    batch = G.make_batch()
    bufs = _alloc(batch, 4)
    P.gbs_cumulants_batched(bufs, 4, flags)
    torch.cuda.synchronize()
    singles = _singles(P, bufs, 4, flags)
    mixed = bool(flags & P.GBS_MIXED)
    worst = 0.0
    num = {d: [0.0, 0.0] for d in range(1, 5)}
    den = {d: [0.0, 0.0] for d in range(1, 5)}
    for (M, _, corr, cum), (c1, k1) in zip(bufs, singles):
        worst = max(worst, float((corr - c1).abs().max()), float((cum - k1).abs().max()))
        if not mixed or flags & P.GBS_ALL_MINORS:
            assert _agree(corr, c1), M
            assert _agree(cum, k1), M
            continue
        for d in range(1, 5):
            lo, hi = O.order_offset(M, d), O.order_offset(M, d + 1)
            for j, (x, y) in enumerate(((corr, c1), (cum, k1))):
                num[d][j] = max(num[d][j], float((x[lo:hi] - y[lo:hi]).abs().max()))
                den[d][j] = max(den[d][j], float(y[lo:hi].abs().max()))
    if mixed and not flags & P.GBS_ALL_MINORS:
        for d in range(1, 5):
            ec, ek = num[d][0] / den[d][0], num[d][1] / den[d][1]
            _say(f"batched vs single mixed order {d}: corr {ec:.2e} cum {ek:.2e}")
            assert ec <= 2 * MIXED_NORM_CORR[d] and ek <= 2 * MIXED_NORM_CUM[d], (d, ec, ek)
    _say("max |batched - single|", worst)


# Mixed form: the normwise bounds stated for the M = 144, K = 5 workload
# (tests/test_gpu_forward.py), per order; every instance here has M <= 144.
MIXED_NORM_CORR = [0, 1e-13, 3e-8, 1e-7, 4e-7]
MIXED_NORM_CUM = [0, 1e-13, 6e-7, 2e-5, 2e-4]


@pytest.mark.parametrize("flags", [0, 2], ids=["fp64", "mixed"])
def test_batch48_against_oracle(P, c_oracle, flags):
    """Sampled outputs of every instance against the C oracle: the FP64
    tolerance, or the mixed form's stated normwise bounds over all instances."""
    import torch
    _say("case: batch48 vs oracle", flags)
    batch = G.make_batch()
    bufs = _alloc(batch, 4)
    P.gbs_cumulants_batched(bufs, 4, flags)
    torch.cuda.synchronize()
    mixed = bool(flags & P.GBS_MIXED)
    num = {d: [0.0, 0.0] for d in range(1, 5)}
    den = {d: [0.0, 0.0] for d in range(1, 5)}
    for i, (inst, (M, _, corr, cum)) in enumerate(zip(batch, bufs)):
        corr, cum = corr.cpu().numpy(), cum.cpu().numpy()
        for d in range(1, 5):
            n = math.comb(M, d)
            ranks = G.random_ranks(n, 400, seed=1000 * i + d)
            rc, rk = O.c_forward_sample(inst.sigma, d, ranks)
            off = O.order_offset(M, d)
            gc, gk = corr[off + ranks], cum[off + ranks]
            assert np.all(np.isfinite(gc)) and np.all(np.isfinite(gk))
            if mixed:
                num[d][0] = max(num[d][0], float(np.abs(gc - rc).max()))
                num[d][1] = max(num[d][1], float(np.abs(gk - rk).max()))
                den[d][0] = max(den[d][0], float(np.abs(rc).max()))
                den[d][1] = max(den[d][1], float(np.abs(rk).max()))
                continue
            smu, skap = fp64_scales(inst.sigma, d, ranks)
            assert_within(gc, rc, fp64_tolerance(rc, smu), f"inst {i} corr d={d}")
            assert_within(gk, rk, fp64_tolerance(rk, skap), f"inst {i} cum d={d}")
    if mixed:
        for d in range(1, 5):
            ec, ek = num[d][0] / den[d][0], num[d][1] / den[d][1]
            _say(f"batched mixed order {d}: corr normwise {ec:.2e} cum normwise {ek:.2e}")
            assert ec <= MIXED_NORM_CORR[d] and ek <= MIXED_NORM_CUM[d], (d, ec, ek)


def test_graph_replay_sees_new_inputs(P):
    """Second and third calls replay the captured graph; the covariances are
    rewritten in place between replays (with eager work in between) and every
    replay matches fresh single-instance calls."""
    import torch
    _say("case: graph replay")
    batch = G.make_batch(count=6, seed=77, m_range=(8, 30))
    bufs = _alloc(batch, 3)
    for rep in range(3):
        if rep:
            for (M, s, _, _) in bufs:  # new values, same buffers
                s.add_(torch.eye(2 * M, dtype=torch.float64, device="cuda:0") * 0.01 * rep)
        _ = torch.randn(1000, device="cuda:0").sum().item()  # eager work between replays
        P.gbs_cumulants_batched(bufs, 3, 0)
        torch.cuda.synchronize()
        for (M, s, corr, cum) in bufs:
            c1, k1 = P.gbs_cumulants(M, s, 3, P.GBS_ALL_MINORS)
            assert _agree(corr, c1) and _agree(cum, k1), (rep, M)


def test_uneven_and_tiny_instances(P):
    import torch
    _say("case: uneven tiny")
    Ms = [5, 1, 2, 40, 3, 17]
    batch = [G.make_instance("m144_k5", M=m, seed=m) for m in Ms]
    # K = 1 for all (M = 1 allowed), then K = 2 without the M = 1 instance
    b1 = _alloc(batch, 1, want_corr=False)
    P.gbs_cumulants_batched(b1, 1, 0)
    for (M, s, _, cum) in b1:
        _, k1 = P.gbs_cumulants(M, s, 1, P.GBS_ALL_MINORS)
        assert _agree(cum, k1)
    b2 = _alloc([x for x in batch if x.M >= 2], 2)
    P.gbs_cumulants_batched(b2, 2, 0)
    for (M, s, corr, cum) in b2:
        c1, k1 = P.gbs_cumulants(M, s, 2, P.GBS_ALL_MINORS)
        assert _agree(corr, c1) and _agree(cum, k1)


def test_autotune_and_set_tuning(P):
    import torch
    _say("case: autotune")
    batch = G.make_batch(count=8, seed=5, m_range=(20, 60))
    bufs = _alloc(batch, 3)
    best = P.gbs_autotune_batched(bufs, 3, 0)
    _say("autotuned", best)
    assert best["block"] in (64, 128, 256) and best["unroll"] in (1, 2, 4)
    assert best["tile"] % (best["block"] * best["unroll"]) == 0
    P.gbs_cumulants_batched(bufs, 3, 0)
    torch.cuda.synchronize()
    ref = [(c.clone(), k.clone()) for (_, _, c, k) in bufs]
    P.gbs_set_tuning(3, 0, {"block": 64, "unroll": 2, "tile": 128, "waves_per_cu": 1})
    P.gbs_cumulants_batched(bufs, 3, 0)
    torch.cuda.synchronize()
    for (_, _, c, k), (c0, k0) in zip(bufs, ref):
        assert torch.equal(c, c0) and torch.equal(k, k0)
    with pytest.raises(P.GBSError):
        P.gbs_set_tuning(3, 0, {"block": 96, "unroll": 1, "tile": 96, "waves_per_cu": 1})
    P.gbs_set_tuning(3, 0, None)


def test_batched_timing_entries(P):
    import torch
    _say("case: batched timing")
    batch = G.make_batch(count=3, seed=9, m_range=(10, 20))
    bufs = _alloc(batch, 3)
    P.gbs_cumulants_batched(bufs, 3, P.GBS_TIMING)
    torch.cuda.synchronize()
    stages = [t[0] for t in P.gbs_last_timings()]
    assert "batched" in stages and "build_q" in stages
    for (M, s, corr, cum) in bufs:
        c1, k1 = P.gbs_cumulants(M, s, 3, P.GBS_ALL_MINORS)
        assert _agree(corr, c1) and _agree(cum, k1)


@pytest.mark.parametrize("conv", [0, 1], ids=["click", "parity"])
def test_order5_tables_scratch_and_fallback(P, c_oracle, conv):
    """K = 5 over instances of uneven M, some without correlator outputs (the
    group kernel then keeps the lower-order correlators in plan scratch), and
    one of M = 150, whose order 5 (more than 2^29 subsets) falls back to the
    all-minors launch while orders 3 and 4 run on the group kernel; sampled
    outputs of every order against the C oracle."""
    import torch
    _say("case: batch K=5 scratch + fallback", conv)
    Ms = [150, 23, 9, 31, 5]
    batch = [G.make_instance("m144_k5", M=m, seed=300 + m) for m in Ms]
    bufs = []
    for j, inst in enumerate(batch):
        s = torch.from_numpy(inst.sigma).to("cuda:0")
        n = O.total_outputs(inst.M, 5)
        corr = torch.empty(n, dtype=torch.float64, device="cuda:0") if j % 2 == 0 else None
        bufs.append((inst.M, s, corr, torch.empty(n, dtype=torch.float64, device="cuda:0")))
    P.gbs_cumulants_batched(bufs, 5, conv)
    torch.cuda.synchronize()
    for i, (inst, (M, _, corr, cum)) in enumerate(zip(batch, bufs)):
        for d in range(1, 6):
            n = math.comb(M, d)
            ranks = G.random_ranks(n, 300 if M > 100 else 2000, seed=700 * i + d)
            rc, rk = O.c_forward_sample(inst.sigma, d, ranks, conv)
            smu, skap = fp64_scales(inst.sigma, d, ranks, conv)
            idx = torch.from_numpy(O.order_offset(M, d) + ranks.astype(np.int64)).to("cuda:0")
            if corr is not None:
                got = corr[idx].cpu().numpy()
                assert_within(got, rc, fp64_tolerance(rc, smu), f"M={M} corr d={d}")
            got = cum[idx].cpu().numpy()
            assert_within(got, rk, fp64_tolerance(rk, skap), f"M={M} cum d={d}")
    # the small instances also agree with single calls everywhere
    for (M, s, corr, cum) in bufs[1:]:
        c1, k1 = P.gbs_cumulants(M, s, 5, conv)
        assert _agree(cum, k1), M
        if corr is not None:
            assert _agree(corr, c1), M


@pytest.mark.parametrize("flags", [0, 2], ids=["fp64", "mixed"])
def test_group_launches_in_timing(P, flags):
    """K = 4, FP64 or mixed: one all-minors launch (orders 1, 2) and one group
    launch per order 3, 4 appear as 'batched' stages."""
    import torch
    _say("case: batched group timing", flags)
    batch = G.make_batch(count=4, seed=19, m_range=(12, 40))
    bufs = _alloc(batch, 4)
    P.gbs_cumulants_batched(bufs, 4, P.GBS_TIMING | flags)
    torch.cuda.synchronize()
    orders = sorted(o for st, o, _ in P.gbs_last_timings() if st == "batched")
    assert orders == [0, 3, 4], orders
