#!/usr/bin/env python3
"""Benchmark: click correlators and cumulants of all subsets of order <= 5 at M = 144.

One step = one full pass of the path on the resident covariance: Q = sigma + I/2
(and, for the mixed form, its per-mode normalisation), then orders 1..5 of
vacuum probabilities -> correlators -> cumulants, every output written to HBM.
498,685,188 subsets per step.  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--precision fp64|mixed]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M = 144
K = 5
# algorithmic flops per order-d subset: one new 2d x 2d factorisation, (2d)^3/3,
# plus 2^(d+1) for inclusion-exclusion and the cumulant recursion
FLOPS_PER_SUBSET = {d: (2 * d) ** 3 / 3 + 2 ** (d + 1) for d in range(1, 6)}
# displaced states add one triangular solve of the mean, (2d)^2
FLOPS_PER_SUBSET_DISP = {d: FLOPS_PER_SUBSET[d] + (2 * d) ** 2 for d in range(1, 6)}
PEAK_VALU_TFLOPS = 78.6  # one non-packed FMA per lane per clock: 256 CU x 64 lanes x 2 x 2.4 GHz
WORKLOAD = ("m144_k5: M=144 modes, subsets of order 1..5 (498,685,188), Haar interferometer, "
            "x-squeezing r~U[0.6,1.6], input loss eta~U[0.25,0.4], xxpp, hbar=1")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_forward_order5_m144.json")
SAMPLER_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sampler_m144.json")
PEAK_HBM_BYTES = 8e12


# the sources the order-5 kernel of the headline path is compiled from
TRAFFIC_SOURCES = ("gbs_device.h", "gbs_subset.h", "gbs_forward_group.hip", "gbs_group_tile.inc")


def kernel_source_hash(sources=TRAFFIC_SOURCES) -> str:
    """Hash of a kernel's sources (default: the order-5 kernel's) with comments
    and whitespace removed, so that the stored counter readings stay valid
    across comment-only edits and edits of other kernels."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_14923_amd", "csrc")
    for name in sources:
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        text = " ".join(text.split())
        h.update(name.encode() + text.encode())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_precision(P, torch, sigma, corr, cum, flags, steps, warmup, label, mu=None):
    """Time `steps` calls of gbs_cumulants (or, with a mean vector mu,
    gbs_cumulants_displaced) on resident buffers: back to back (GBS_ASYNC)
    between two device synchronisations, then the status of the last call;
    then `steps` more calls with a HIP event pair around every launch
    (GBS_TIMING) for the per-order kernel durations."""
    def call(fl):
        if mu is None:
            P.gbs_cumulants(M, sigma, K, fl, corr=corr, cum=cum)
        else:
            P.gbs_cumulants_displaced(M, sigma, mu, K, fl, corr=corr, cum=cum)

    for i in range(warmup):
        call(flags)
        log(f"[bench] {label} warmup {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        call(flags | P.GBS_ASYNC)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    st, order, rank = P.gbs_last_error()
    if st != P.GBS_OK:
        raise P.GBSError(st, f"{label}: failing subset at order {order}, rank {rank}")
    log(f"[bench] {label}: {steps} steps in {t:.3f} s")
    kern = {d: [] for d in range(1, K + 1)}
    for i in range(steps):
        call(flags | P.GBS_TIMING)
        for stage, order, ms in P.gbs_last_timings():
            if stage == "forward":
                kern[order].append(ms)
    ms_step = 1e3 * t / steps
    n = sum(math.comb(M, d) for d in range(1, K + 1))
    k5 = sum(kern[5]) / len(kern[5])
    flops5 = math.comb(M, 5) * (FLOPS_PER_SUBSET if mu is None else FLOPS_PER_SUBSET_DISP)[5]
    return {
        "ms_per_step": ms_step,
        "subsets_per_s": n / (ms_step * 1e-3),
        "kernel_ms": {d: sum(v) / len(v) for d, v in kern.items()},
        "kernel_ms_median": {d: sorted(v)[len(v) // 2] for d, v in kern.items()},
        "order5_kernel_ms": k5,
        "order5_tflops": flops5 / (k5 * 1e-3) / 1e12,
    }


def traffic_entry(label):
    """HBM bytes per order-5 launch from the committed rocprofv3 counter runs,
    or None when missing or taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(label)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def precision_errors(torch, P, corr64, cum64, corrmx, cummx):
    out = {}
    for d in range(1, K + 1):
        a, b = P.gbs_order_offset(M, d), P.gbs_order_offset(M, d + 1)
        for name, x, y in (("corr", corrmx, corr64), ("cum", cummx, cum64)):
            dx = (x[a:b] - y[a:b]).abs()
            ref = y[a:b].abs()
            rel = dx / ref.clamp_min(1e-300)
            q = torch.quantile(rel[:: max(1, rel.numel() // 1_000_000)].float(),
                               torch.tensor([0.5, 0.99], device=rel.device)).tolist()
            out[f"{name}_d{d}"] = {"normwise": float(dx.max() / ref.max()),
                                   "rel_median": q[0], "rel_p99": q[1], "rel_max": float(rel.max())}
    return out


def fp64_tolerance(np, ref, scale, carried=None):
    """The FP64 parity tolerance: 1e-10 max(|ref|, 1e-4 scale), scale the
    summand magnitude of the sum that gives the output
    (oracle.c_tolerance_scale), plus, for a cumulant, 4 u times the rounding
    its correlators carry in (oracle.c_error_floor)."""
    tol = 1e-10 * np.maximum(np.abs(ref), 1e-4 * scale)
    if carried is not None:
        tol = tol + 4.0 * 2.0 ** -53 * carried
    return tol


def fp64_parity_sample(np, O, G, inst, corr, cum, n=3000, mu=None):
    """Sampled FP64 outputs against the oracle (displaced when mu is given):
    worst |delta| / tolerance."""
    worst = 0.0
    for d in range(1, K + 1):
        cnt = math.comb(M, d)
        ranks = G.random_ranks(cnt, min(n, cnt), seed=900 + d)
        rc, rk = O.c_forward_sample(inst.sigma, d, ranks, mu=mu)
        smu, skap = O.c_tolerance_scale(inst.sigma, d, ranks, mu=mu)
        _, vk = O.c_error_floor(inst.sigma, d, ranks, mu=mu)
        off = O.order_offset(M, d)
        gc = corr[off + ranks]
        gk = cum[off + ranks]
        for got, ref, v, c in ((gc, rc, smu, None), (gk, rk, skap, vk)):
            worst = max(worst, float(np.max(np.abs(got - ref) / fp64_tolerance(np, ref, v, c))))
    return worst


def batched_and_adjoint(P, torch, G, steps):
    """The two other launch shapes of the path, measured beside the headline:
    the 48-instance batched launch (M ~ U{40..144}, K = 4, one persistent
    kernel) and the adjoint at M = 144, K = 3 (vector-Jacobian product of the
    cumulants with respect to sigma)."""
    out = {}
    batch = G.make_batch()
    bufs = []
    n_sub = 0
    flops = 0.0
    for inst in batch:
        s = torch.from_numpy(inst.sigma).to("cuda:0")
        n = P.gbs_total_outputs(inst.M, 4)
        bufs.append((inst.M, s, torch.empty(n, dtype=torch.float64, device="cuda:0"),
                     torch.empty(n, dtype=torch.float64, device="cuda:0")))
        n_sub += n
        flops += sum(math.comb(inst.M, d) * FLOPS_PER_SUBSET[d] for d in range(1, 5))
    for label, fl in (("batched48_k4", 0), ("batched48_k4_mixed", P.GBS_MIXED)):
        # launch shapes from the autotuner (all-minors shape, then the group
        # launches' workgroups per CU), cached in the library for later calls
        t0 = time.perf_counter()
        tuned = P.gbs_autotune_batched(bufs, 4, fl)
        t_tune = time.perf_counter() - t0
        P.gbs_cumulants_batched(bufs, 4, fl)  # plan, graph capture
        torch.cuda.synchronize()
        walls, kern = [], []
        for _ in range(steps):
            t0 = time.perf_counter()
            P.gbs_cumulants_batched(bufs, 4, fl)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            P.gbs_cumulants_batched(bufs, 4, fl | P.GBS_TIMING)
            kern.append(sum(ms for st, _, ms in P.gbs_last_timings() if st == "batched"))
        wall = sorted(walls)[len(walls) // 2]
        kms = sorted(kern)[len(kern) // 2]
        out[label] = {
            "instances": len(batch), "subsets": n_sub, "ms_per_call": 1e3 * wall,
            "subsets_per_s": n_sub / wall, "kernel_ms": kms,
            "kernel_tflops": flops / (kms * 1e-3) / 1e12,
            "frac_of_fp64_peak": flops / (kms * 1e-3) / 1e12 / PEAK_VALU_TFLOPS,
            "tuned_shape": tuned, "autotune_seconds": t_tune,
            "kernel": ("persistent work lists: orders 1-2 all-minors, orders 3-4 the group "
                       "kernel, one launch per order" + ("" if fl == 0 else
                       " (FP32 deviations of the normalised Q, FP64 probabilities and sums)"))}
        log(f"[bench] {label}: {1e3 * wall:.2f} ms per call, kernels {kms:.2f} ms, tuned {tuned}")
    del bufs
    inst = G.make_instance("grad_m144_k3")
    s = torch.from_numpy(inst.sigma).to("cuda:0")
    n = P.gbs_total_outputs(144, 3)
    gk = torch.randn(n, dtype=torch.float64, device="cuda:0", generator=torch.Generator("cuda:0").manual_seed(5))
    P.gbs_cumulant_grad(144, s, 3, 0, grad_cum=gk)
    torch.cuda.synchronize()
    walls, stages = [], None
    for _ in range(steps):
        t0 = time.perf_counter()
        P.gbs_cumulant_grad(144, s, 3, 0, grad_cum=gk)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    P.gbs_cumulant_grad(144, s, 3, P.GBS_TIMING, grad_cum=gk)
    stages = {}
    for st, order, ms in P.gbs_last_timings():
        key = f"{st}{order}" if st != "build_q" else st
        stages[key] = stages.get(key, 0.0) + ms
    wall = sorted(walls)[len(walls) // 2]
    # algorithmic work of one gradient: the forward tables, then per subset T of
    # order d the inverse of Q_T ((2d)^3) weighted into the covariance gradient
    # (2 (2d)^2), and two flops per (subset, proper superset) pair for the
    # correlator and probability adjoints
    K3 = 3
    fl = sum(math.comb(144, d) * (FLOPS_PER_SUBSET[d] + (2 * d) ** 3 + 2 * (2 * d) ** 2)
             for d in range(1, K3 + 1))
    fl += 2 * 2 * sum(math.comb(144, d) * sum(math.comb(144 - d, j) for j in range(1, K3 - d + 1))
                      for d in range(1, K3))
    out["grad_m144_k3"] = {"subsets": n, "ms_per_call": 1e3 * wall,
                           "gradients_per_s": 1.0 / wall, "stage_ms": stages,
                           "roofline": {"bound": "alu", "achieved": fl / wall / 1e12,
                                        "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                                        "frac": fl / wall / 1e12 / PEAK_VALU_TFLOPS,
                                        "algorithmic_flops": fl,
                                        "note": "wall time per call, nine launches of "
                                                "small grids: launch and latency bound"}}
    return out


def config_lines(P, torch, np, G, steps):
    """Throughput on the two smaller plain-FP64 workloads (M = 16, K = 3 and
    M = 100, K = 4) with the C oracle timed on the identical workload, and the
    gradient workload (M = 144, K = 3): the adjoint against the oracle's
    gradient and against central differences (h = 1e-6) of the GPU loss in all
    288 parameters (576 forward evaluations), each timed."""
    import oracle as O
    out = {}
    for name, K_ in (("m16_k3", 3), ("m100_k4", 4)):
        inst = G.make_instance(name)
        M_ = inst.M
        s = torch.from_numpy(inst.sigma).to("cuda:0")
        n = P.gbs_total_outputs(M_, K_)
        corr = torch.empty(n, dtype=torch.float64, device="cuda:0")
        cum = torch.empty(n, dtype=torch.float64, device="cuda:0")
        for _ in range(3):
            P.gbs_cumulants(M_, s, K_, 0, corr=corr, cum=cum)
        reps = max(steps, 20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            P.gbs_cumulants(M_, s, K_, P.GBS_ASYNC, corr=corr, cum=cum)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        st, _, _ = P.gbs_last_error()
        if st != P.GBS_OK:
            raise P.GBSError(st, name)
        t1 = time.perf_counter()
        rc, rk = O.c_forward(inst.sigma, K_)
        dto = time.perf_counter() - t1
        gc, gk = corr.cpu().numpy(), cum.cpu().numpy()
        worst = 0.0
        for d in range(1, K_ + 1):
            a, b = O.order_offset(M_, d), O.order_offset(M_, d + 1)
            ranks = np.arange(b - a, dtype=np.int64)
            smu, spi = O.c_tolerance_scale(inst.sigma, d, ranks)
            _, vk = O.c_error_floor(inst.sigma, d, ranks)
            worst = max(worst, float(np.max(np.abs(gc[a:b] - rc[a:b]) / fp64_tolerance(np, rc[a:b], smu))),
                        float(np.max(np.abs(gk[a:b] - rk[a:b]) / fp64_tolerance(np, rk[a:b], spi, vk))))
        out[name] = {"M": M_, "max_order": K_, "subsets": n, "ms_per_call": 1e3 * dt,
                     "subsets_per_s": n / dt,
                     "cpu_oracle": {"seconds": dto, "subsets_per_s": n / dto,
                                    "cores": O.c_threads(0), "kind": "oracle",
                                    "sample": "the whole workload"},
                     "worst_err_over_tol_all_outputs": worst}
        log(f"[bench] {name}: {1e3 * dt:.3f} ms per call, oracle {dto:.2f} s, worst err/tol {worst:.3g}")
    # gradient workload: adjoint vs the oracle's gradient and finite differences
    from paper_2511_14923_amd import autograd as A
    inst = G.make_instance("grad_m144_k3")
    _, _, sig_t = G.make_grad_target(inst)
    _, target = O.c_forward(sig_t, 3)
    t1 = time.perf_counter()
    loss_ref, gsig_ref = O.c_loss_grad(inst.sigma, 3, target)
    t_oracle = time.perf_counter() - t1
    d_eta, d_r = O.covariance_param_grad(inst.U, inst.r, inst.eta, gsig_ref)
    ref = np.concatenate([d_eta, d_r])
    W = A.interferometer_symplectic(torch.from_numpy(inst.U).to("cuda:0"))
    r = torch.tensor(inst.r, device="cuda:0", requires_grad=True)
    eta = torch.tensor(inst.eta, device="cuda:0", requires_grad=True)
    tgt = torch.from_numpy(target).to("cuda:0")
    loss = A.cumulant_matching_loss(W, r, eta, tgt, 3)
    loss.backward()
    got = np.concatenate([eta.grad.cpu().numpy(), r.grad.cpu().numpy()])
    h = 1e-6
    fd = np.empty(288)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    with torch.no_grad():
        for i in range(288):
            e = torch.zeros(288, dtype=torch.float64, device="cuda:0")
            e[i] = h
            lp = A.cumulant_matching_loss(W, r + e[144:], eta + e[:144], tgt, 3)
            lm = A.cumulant_matching_loss(W, r - e[144:], eta - e[:144], tgt, 3)
            fd[i] = float((lp - lm) / (2 * h))
    t_fd = time.perf_counter() - t1

    def normwise(a, b):
        return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))

    out["grad_m144_k3_checks"] = {
        "params": 288, "loss": float(loss.detach()), "loss_oracle": loss_ref,
        "adjoint_vs_oracle_normwise": normwise(got, ref),
        "adjoint_vs_fd_normwise": normwise(got, fd),
        "oracle_gradient_seconds": t_oracle, "oracle_cores": O.c_threads(0),
        "fd_forward_evaluations": 576, "fd_seconds": t_fd}
    log(f"[bench] gradient: oracle {t_oracle:.2f} s, 576 FD evaluations {t_fd:.2f} s, "
        f"adjoint vs oracle {out['grad_m144_k3_checks']['adjoint_vs_oracle_normwise']:.2e}, "
        f"vs FD {out['grad_m144_k3_checks']['adjoint_vs_fd_normwise']:.2e}")
    return out


def full_parity(np, O, inst, bufs, chunk=8_000_000):
    """Every output of the M = 144, K = 5 workload against the C oracle, streamed
    in rank blocks: the FP64 form to its tolerance (the carried-in term is
    computed only for the outputs outside 1e-10 max(|ref|, 1e-4 S_pi)), the
    mixed form's relative error per order.  Returns the oracle's time on the
    whole workload (with the tolerance scales) and the worst ratios."""
    threads = O.c_threads(0)
    res = {"cores": threads, "orders": {}}
    t_all = 0.0
    worst = 0.0
    for d in range(1, K + 1):
        cnt = math.comb(M, d)
        off = O.order_offset(M, d)
        od = {"outputs": cnt, "worst_corr_err_over_tol": 0.0, "worst_cum_err_over_tol": 0.0,
              "carried_term_needed": 0}
        mixed_num = {"corr": 0.0, "cum": 0.0}
        mixed_den = {"corr": 0.0, "cum": 0.0}
        rel_all = []
        for r0 in range(0, cnt, chunk):
            n = min(chunk, cnt - r0)
            t0 = time.perf_counter()
            rc, rk, smu, spi = O.c_forward_range(inst.sigma, d, r0, n, scales=True, threads=threads)
            t_all += time.perf_counter() - t0
            gc = bufs["fp64"][0][off + r0: off + r0 + n].cpu().numpy()
            gk = bufs["fp64"][1][off + r0: off + r0 + n].cpu().numpy()
            ec = np.abs(gc - rc) / fp64_tolerance(np, rc, smu)
            od["worst_corr_err_over_tol"] = max(od["worst_corr_err_over_tol"], float(ec.max()))
            cheap = fp64_tolerance(np, rk, spi)
            ek = np.abs(gk - rk)
            out_idx = np.nonzero(ek > cheap)[0]
            ratio = ek / cheap
            if len(out_idx):
                od["carried_term_needed"] += int(len(out_idx))
                ranks = (r0 + out_idx).astype(np.int64)
                _, vk = O.c_error_floor(inst.sigma, d, ranks, threads=threads)
                ratio[out_idx] = ek[out_idx] / fp64_tolerance(np, rk[out_idx], spi[out_idx], vk)
            od["worst_cum_err_over_tol"] = max(od["worst_cum_err_over_tol"], float(ratio.max()))
            worst = max(worst, float(ec.max()), float(ratio.max()))
            if "mixed" in bufs:
                mc = bufs["mixed"][0][off + r0: off + r0 + n].cpu().numpy()
                mk = bufs["mixed"][1][off + r0: off + r0 + n].cpu().numpy()
                mixed_num["corr"] = max(mixed_num["corr"], float(np.abs(mc - rc).max()))
                mixed_num["cum"] = max(mixed_num["cum"], float(np.abs(mk - rk).max()))
                mixed_den["corr"] = max(mixed_den["corr"], float(np.abs(rc).max()))
                mixed_den["cum"] = max(mixed_den["cum"], float(np.abs(rk).max()))
                rel_all.append((np.abs(mk - rk) / np.maximum(np.abs(rk), 1e-300))[:: max(1, n // 200000)])
            if (r0 // chunk) % 10 == 0:
                log(f"[bench] full parity: order {d}, ranks {r0 + n}/{cnt}, oracle {t_all:.0f} s")
        if rel_all:
            rel = np.concatenate(rel_all)
            od["mixed_vs_oracle"] = {
                "corr_normwise": mixed_num["corr"] / mixed_den["corr"],
                "cum_normwise": mixed_num["cum"] / mixed_den["cum"],
                "cum_rel_median": float(np.median(rel)), "cum_rel_p99": float(np.quantile(rel, 0.99)),
                "cum_rel_max_sampled": float(rel.max())}
        res["orders"][str(d)] = od
    res["oracle_seconds_all_outputs"] = t_all
    res["oracle_subsets_per_s"] = sum(math.comb(M, d) for d in range(1, K + 1)) / t_all
    res["worst_err_over_tol"] = worst
    return res


def sampler_terms(M_, K_):
    """Expansion terms one sample evaluates (the sums of Eqs. methprob, b, a for
    K = 3; Eqs. probade, probpartialade, probelidedade, probdoubleelidedade for
    K = 5), each one product with one per-sample table value."""
    def c(a, b):
        return math.comb(a, b) if a >= 0 else 0
    tot = 0
    for n in range(1, M_ + 1):
        if K_ == 3:
            tot += 1 + (n - 1) + c(n - 1, 2)                              # p
            tot += (n - 1) * (n - 1)                                      # p1
            tot += sum(1 + (n - l) for l in range(1, n + 1))              # p+
        else:
            tot += 1 + (n - 1) + c(n - 1, 2) + c(n - 1, 3) + c(n - 1, 4)  # p
            tot += sum(1 + (n - l) + c(n - l, 2) for l in range(1, n + 1))  # p+
            tot += (n - 1) * (1 + (n - 2) + c(n - 2, 2))                  # p1
            tot += c(n - 1, 2) * (n - 2)                                  # p2
    return tot


def sampler_table_bytes(M_, K_):
    """Algorithmic bytes per sample: at every step n each live entry of the
    per-sample FP64 tables (p: n + 1, p1: C(n, 2), p+: C(n + 1, 2) and, for
    double elision, p2: C(n, 3)) read once, the least any evaluation of the
    step's sums must touch."""
    tot = 0
    for n in range(1, M_ + 1):
        tot += (n + 1) + math.comb(n, 2) + math.comb(n + 1, 2)
        if K_ == 5:
            tot += math.comb(n, 3)
    return 8 * tot


def sampler_traffic(K_):
    """HBM bytes per sample of the sampler kernel from the committed rocprofv3
    counter runs (FETCH_SIZE and WRITE_SIZE, scaled by the copy calibration),
    or None when missing or taken on different kernel sources."""
    try:
        with open(SAMPLER_TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(f"k{K_}")
    if not ent or rec.get("source_hash") != kernel_source_hash(("gbs_sampler.hip",)):
        return None
    return ent.get("bytes_per_sample")


def sampler_legs(P, torch, np, G, sigma, counts):
    """Stage 2 on the stage-1 output: parity cumulants of the M = 144 workload
    (gbs_cumulants, GBS_PARITY) -> gbs_sample, single elision (K = 3) and
    double elision (K = 5); uniforms from a seeded device generator."""
    out = {}
    for K_, n in counts:
        _, kap = P.gbs_cumulants(M, sigma, K_, P.GBS_PARITY, want_corr=False)
        g = torch.Generator(device="cuda:0")
        g.manual_seed(2511 + K_)
        u = torch.rand((M, n), dtype=torch.float64, device="cuda:0", generator=g)
        if K_ == 3:  # warm-up: one workgroup (a K = 5 workgroup alone runs for seconds)
            P.gbs_sample(M, kap, K_, u[:, :64].contiguous())
        torch.cuda.synchronize()
        log(f"[bench] sampler K={K_}: {n} samples")
        t0 = time.perf_counter()
        bits, prob, _ = P.gbs_sample(M, kap, K_, u, flags=P.GBS_TIMING)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = sum(ms for st, _, ms in P.gbs_last_timings() if st == "sample")
        terms = sampler_terms(M, K_) * n
        if K_ == 3:
            keep = bits
        per = sampler_traffic(K_)
        hbm = None
        alg = sampler_table_bytes(M, K_) * n
        alg_rate = alg / (kms * 1e-3)
        # frac: algorithmic bytes (every live table entry read once per step);
        # counter_frac: the bytes the counters measured (re-reads included)
        hbm = {"bound": "hbm", "algorithmic_bytes": alg, "achieved_gb_per_s": alg_rate / 1e9,
               "peak_gb_per_s": PEAK_HBM_BYTES / 1e9, "frac": alg_rate / PEAK_HBM_BYTES}
        if per is not None:  # the per-sample tables stream from HBM: bytes grow with n
            rate = per * n / (kms * 1e-3)
            hbm.update({"counter_bytes": per * n, "counter_gb_per_s": rate / 1e9,
                        "counter_frac": rate / PEAK_HBM_BYTES,
                        "source": os.path.relpath(SAMPLER_TRAFFIC_FILE, ROOT)})
        out[f"sample_k{K_}_m144"] = {
            "samples": n, "seconds": wall, "samples_per_s": n / wall, "kernel_ms": kms,
            "terms_per_sample": sampler_terms(M, K_), "terms_per_s": terms / (kms * 1e-3),
            "roofline": hbm,
            "mean_clicks": float(bits.float().mean().item() * M),
            "method": "single elision" if K_ == 3 else "double elision"}
        del kap, u, bits, prob
    # sample statistics on the single-elision samples: unbiased click cumulants
    # of orders 1..5 and their Pearson coefficient with the stage-1 ground truth
    out["validate_m144"] = estimator_leg(P, torch, sigma, keep)
    del keep
    # the C oracle on the host cores, same sizes, seeded synthetic cumulants
    import oracle as O
    from oracle import sampler as S
    for K_, n in ((3, 512), (5, 16)):
        cum = G.synthetic_parity_cumulants(M, K_, 7)
        uu = G.sampler_uniforms(M, n, 8)
        t0 = time.perf_counter()
        S.c_sample(cum, M, K_, u=uu)
        dt = time.perf_counter() - t0
        out[f"sample_k{K_}_m144"]["cpu_oracle"] = {
            "samples": n, "seconds": dt, "samples_per_s": n / dt, "cores": O.c_threads(0),
            "kind": "oracle"}
        log(f"[bench] sampler K={K_} cpu oracle: {n} samples in {dt:.1f} s")
    return out


def estimator_leg(P, torch, sigma, bits):
    n = bits.shape[0]
    P.gbs_sample_cumulants(bits[:64].contiguous(), 2)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    est = P.gbs_sample_cumulants(bits, K, flags=P.GBS_TIMING)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = sum(ms for st, _, ms in P.gbs_last_timings() if st == "estimate")
    truth = P.gbs_cumulants(M, sigma, K, 0, want_corr=False)[1]
    rs = {}
    for d in range(1, K + 1):
        a, b = P.gbs_order_offset(M, d), P.gbs_order_offset(M, d + 1)
        rs[str(d)] = float(P.gbs_pearson(est[a:b].contiguous(), truth[a:b].contiguous()).item())
    log(f"[bench] estimator: {n} samples, orders 1..{K} in {wall:.3f} s; pearson {rs}")
    N = P.gbs_total_outputs(M, K)
    return {"samples": n, "subsets": N, "seconds": wall, "kernel_ms": kms,
            "subset_samples_per_s": N * n / wall,
            "pearson_vs_ground_truth": rs,
            "note": "unbiased click cumulants of the single-elision samples vs stage-1 click cumulants"}


def shard_leg(P, torch, G, inst):
    """One GPU's share of the pseudo-photon-number-resolving workload: M = 1152
    (each of the 144 modes split over 8 detectors), order-5 outputs of a colex
    rank range as large as the whole M = 144 order-5 launch, by the T-shared
    kernel from Q alone.  The first call of a range builds its T list (host) and
    keeps it; after three warm-up calls the median of five is reported."""
    M_ = 1152
    sig = torch.from_numpy(G.pseudo_pnr_covariance(inst.sigma, 8)).to("cuda:0")
    total = math.comb(M_, 5)
    cnt = math.comb(M, 5)
    r0 = total // 2
    corr = torch.empty(cnt, dtype=torch.float64, device="cuda:0")
    cum = torch.empty(cnt, dtype=torch.float64, device="cuda:0")
    t0 = time.perf_counter()
    P.gbs_cumulants_shard(M_, sig, 5, r0, cnt, 0, corr=corr, cum=cum)  # builds the T list
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    for _ in range(2):  # further warm-up: the first calls of a process run slower
        P.gbs_cumulants_shard(M_, sig, 5, r0, cnt, 0, corr=corr, cum=cum)
    torch.cuda.synchronize()
    kms_all, walls = [], []
    for _ in range(5):
        t0 = time.perf_counter()
        P.gbs_cumulants_shard(M_, sig, 5, r0, cnt, P.GBS_TIMING, corr=corr, cum=cum)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        kms_all.append(sum(ms for st, order, ms in P.gbs_last_timings() if st == "forward"))
    kms = sorted(kms_all)[2]
    wall = sorted(walls)[2]
    rate = cnt / (kms * 1e-3)
    log(f"[bench] shard M=1152 order 5: {cnt} subsets in {kms:.2f} ms")
    # the same shard by the all-minors kernel, for comparison
    P.gbs_cumulants_shard(M_, sig, 5, r0, cnt, P.GBS_TIMING | P.GBS_ALL_MINORS, corr=corr, cum=cum)
    torch.cuda.synchronize()
    kms_am = sum(ms for st, order, ms in P.gbs_last_timings() if st == "forward")
    flops = cnt * FLOPS_PER_SUBSET[5]
    return {"M": M_, "order": 5, "rank0": r0, "subsets": cnt, "seconds": wall,
            "first_call_seconds": first, "kernel_ms": kms, "kernel_ms_calls": kms_all,
            "subsets_per_s": rate, "order5_total": total,
            "full_order5_one_gpu_s": total / rate, "full_order5_eight_gpus_s": total / rate / 8,
            "frac_of_fp64_peak": flops / (kms * 1e-3) / 1e12 / PEAK_VALU_TFLOPS,
            "all_minors_kernel_ms": kms_am,
            "kernel": "T-shared kernel (one T per workgroup: its 64 a's keep their (T, a) "
                      "factors in registers, its b_0's their (B) factors in LDS), one shard of "
                      "the colex rank range"}


def cpu_baseline(np, O, G, inst, seconds):
    """The C oracle on the host cores over a random sample of the workload's
    subsets (all orders, in proportion to their counts)."""
    threads = O.c_threads(0)
    counts = [math.comb(M, d) for d in range(1, K + 1)]
    total = sum(counts)

    def run(n, seed):
        rng = np.random.default_rng(seed)
        picks = np.sort(rng.integers(0, total, size=n))
        done = 0
        t0 = time.perf_counter()
        for d in range(1, K + 1):
            a = sum(counts[: d - 1])
            sel = picks[(picks >= a) & (picks < a + counts[d - 1])] - a
            if len(sel):
                O.c_forward_sample(inst.sigma, d, np.unique(sel), threads=threads)
                done += len(np.unique(sel))
        return done, time.perf_counter() - t0

    # calibrate on a sample large enough that thread start-up does not skew the rate
    n0, t0 = run(500000, 1)
    n = int(min(1e8, max(20000, n0 / max(t0, 1e-3) * seconds)))
    done, t = run(n, 2)
    log(f"[bench] cpu oracle: {done} subsets in {t:.2f} s on {threads} threads")
    return {"value": done / t, "unit": "subsets/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} subsets drawn uniformly from all 498,685,188 of the M=144 K=5 "
                      f"workload (C oracle, OpenMP, {t:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="which form gives the headline value (both are measured)")
    ap.add_argument("--only", choices=["fp64", "mixed", "fp64_all_minors", "mixed_all_minors",
                                       "displaced", "sampler", "batched", "shard"],
                    default=None, help="measure one form only (profiling runs)")
    ap.add_argument("--all-minors", action="store_true",
                    help="also measure the all-minors kernel (GBS_ALL_MINORS) of both precisions")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--full-parity", action="store_true",
                    help="compare every output of the workload with the C oracle (minutes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and adjoint measurements")
    ap.add_argument("--no-sampler", action="store_true", help="skip the stage-2 sampler legs")
    ap.add_argument("--samples-k3", type=int, default=262144)
    ap.add_argument("--samples-k5", type=int, default=16384)
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device-to-device copy of GIB GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: every figure here is per GPU.  The path needs "
              "no communication; on several GPUs each would take a contiguous slice of every "
              "order's colex ranks (gbs_cumulants_shard) after one broadcast of sigma",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gbs_inputs as G
    import paper_2511_14923_amd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration > 0:
        n = int(args.copy_calibration * (1 << 30)) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n}), flush=True)
        return
    P.lib()
    if args.only == "batched":  # profiling runs of the batched and adjoint launches only
        print(json.dumps(batched_and_adjoint(P, torch, G, args.steps)), flush=True)
        return
    if args.only == "shard":  # profiling runs of the M = 1152 shard only
        print(json.dumps(shard_leg(P, torch, G, G.make_instance("m144_k5"))), flush=True)
        return
    inst = G.make_instance("m144_k5")
    sigma = torch.from_numpy(inst.sigma).to("cuda:0")
    N = P.gbs_total_outputs(M, K)
    log(f"[bench] M={M} K={K} outputs={N}")

    forms = [args.only] if args.only and args.only != "sampler" else ["fp64", "mixed"]
    if args.only == "sampler":
        forms = ["fp64"]
    if args.all_minors and not args.only:
        forms += ["fp64_all_minors", "mixed_all_minors"]
    res, bufs = {}, {}
    mu = None
    if args.only == "displaced" or (not args.only and not args.no_extras):
        # displaced variant of the same workload (seeded input amplitudes)
        mu = torch.from_numpy(G.input_displacement(inst)).to("cuda:0")
        if "displaced" not in forms:
            forms.append("displaced")
    for form in forms:
        corr = torch.empty(N, dtype=torch.float64, device="cuda:0")
        cum = torch.empty(N, dtype=torch.float64, device="cuda:0")
        flags = (P.GBS_MIXED if form.startswith("mixed") else 0) | \
            (P.GBS_ALL_MINORS if form.endswith("all_minors") else 0)
        res[form] = run_precision(P, torch, sigma, corr, cum, flags, args.steps, args.warmup, form,
                                  mu=mu if form == "displaced" else None)
        if form in ("fp64", "mixed", "displaced"):
            bufs[form] = (corr, cum)
        else:
            del corr, cum

    primary = args.precision if args.precision in res else forms[0]
    r = res[primary]
    extra = {}
    if not args.no_check:
        import oracle as O
        if "fp64" in bufs:
            c64 = bufs["fp64"][0].cpu().numpy()
            k64 = bufs["fp64"][1].cpu().numpy()
            extra["fp64_worst_err_over_tol"] = fp64_parity_sample(np, O, G, inst, c64, k64)
            del c64, k64
        if "fp64" in bufs and "mixed" in bufs:
            extra["mixed_error_vs_fp64"] = precision_errors(torch, P, *bufs["fp64"], *bufs["mixed"])
        if "displaced" in bufs:
            cd = bufs["displaced"][0].cpu().numpy()
            kd = bufs["displaced"][1].cpu().numpy()
            extra["displaced_worst_err_over_tol"] = fp64_parity_sample(
                np, O, G, inst, cd, kd, mu=G.input_displacement(inst))
            del cd, kd
    if args.full_parity:
        extra["full_parity"] = full_parity(np, __import__("oracle"), inst, bufs)
    if not args.no_extras and not args.only:
        extra["extras"] = batched_and_adjoint(P, torch, G, 5)
        extra["extras"].update(config_lines(P, torch, np, G, args.steps))
        for form in list(bufs):
            del bufs[form]
        torch.cuda.empty_cache()
        extra["extras"]["shard_m1152_k5"] = shard_leg(P, torch, G, inst)
    if args.only == "sampler" or (not args.only and not args.no_extras and not args.no_sampler):
        extra.setdefault("extras", {}).update(
            sampler_legs(P, torch, np, G, sigma, ((3, args.samples_k3), (5, args.samples_k5))))
    base = None
    if not args.no_cpu_baseline:
        import oracle as O
        base = cpu_baseline(np, O, G, inst, args.cpu_seconds)

    flops5 = math.comb(M, 5) * FLOPS_PER_SUBSET[5]
    traffic = traffic_entry(primary)
    line = {
        "metric": "order-<=5 cumulants/sec at M=144 (FP32-mixed vs FP64) at stated rel. error",
        "value": r["subsets_per_s"],
        "unit": "subsets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if primary == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "M": M, "max_order": K,
                   "subsets": N, "precision": primary, "convention": "click"},
        "roofline": {
            "bound": "alu",
            "kernel": f"forward order 5 ({primary})",
            "achieved": r["order5_tflops"],
            "peak": PEAK_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": r["order5_tflops"] / PEAK_VALU_TFLOPS,
            "traffic": traffic,
            "algorithmic_flops_per_launch": flops5,
            "kernel_ms": r["order5_kernel_ms"],
        },
        "cpu_baseline": base,
        "forms": res,
    }
    if "fp64" in res and "mixed" in res:
        line["mixed_speedup_over_fp64"] = res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"]
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
