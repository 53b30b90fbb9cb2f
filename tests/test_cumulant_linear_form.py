"""The kernels' assembly of a subset's correlator and cumulant (the cumulant as a
linear form in the vacuum probabilities p({a} + V), with coefficients from the
inverse of the B-only correlators under subset convolution; csrc/gbs_subset.h,
cumulant_coefficients) against the oracle's plain definitions: inclusion-
exclusion for the correlator and the explicit partition sum for the cumulant
(Eqs. corre_cov_main, cumulant_corr_main). The product helper is compiled for
the host (tests/coeff_check.hip); its inputs, the correlators of the subsets of
B and the probabilities p({a} + V), come from the oracle. No GPU needed."""
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

import gbs_inputs as G
import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not found")
    d = tmp_path_factory.mktemp("coeff")
    exe = str(d / "coeff_check")
    obj = exe + ".o"
    csrc = os.path.join(ROOT, "paper_2511_14923_amd", "csrc")
    flags = ["-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", csrc]
    subprocess.run([HIPCC] + flags + ["-c", os.path.join(HERE, "coeff_check.hip"), "-o", obj],
                   check=True, capture_output=True)
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-o", exe, obj], check=True, capture_output=True)
    return exe


def _cases(conv, n_per_order=12):
    """Seeded subsets of the M = 16 workload: (line for the checker, oracle
    correlator, oracle cumulant, cumulant scale) per subset, orders 2..5."""
    inst = G.make_instance("m16_k3")
    Q = O.q_matrix(inst.sigma)
    corr_fn = O.click_correlator if conv == O.CLICK else O.parity_correlator
    rng = np.random.default_rng(2511 + conv)
    out = []
    for d in range(2, 6):
        for _ in range(n_per_order):
            S = tuple(sorted(rng.choice(16, size=d, replace=False).tolist()))
            a, B = S[0], S[1:]
            nb = len(B)
            subs = [tuple(B[j] for j in range(nb) if (u >> j) & 1) for u in range(1 << nb)]
            mu = [1.0 if not U else corr_fn(Q, U) for U in subs]
            pa = [O.vacuum_probability(Q, (a,) + U) for U in subs]
            ref_m, ref_k = O.subset_values(inst.sigma, S, conv)
            scale = O.cumulant_scale(inst.sigma, S, conv)
            line = f"{1 if conv == O.PARITY else 0} {nb} " + " ".join(f"{x:.17g}" for x in mu + pa)
            out.append((line, ref_m, ref_k, scale))
    return out


@pytest.mark.parametrize("conv", [O.CLICK, O.PARITY])
def test_linear_form_matches_partition_sum(checker, conv):
    cases = _cases(conv)
    r = subprocess.run([checker], input="\n".join(c[0] for c in cases) + "\n",
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    got = [tuple(map(float, ln.split())) for ln in r.stdout.strip().splitlines()]
    assert len(got) == len(cases)
    for (line, ref_m, ref_k, scale), (m, k) in zip(cases, got):
        assert abs(m - ref_m) <= 1e-13 * max(abs(ref_m), 1.0), (line, m, ref_m)
        # FP64 rounding of sums whose terms are of the size of the partition-sum terms
        assert abs(k - ref_k) <= 1e-13 * max(scale, 1e-300) + 1e-15, (line, k, ref_k, scale)


def test_linear_form_detects_a_wrong_coefficient(checker):
    """A planted mistake (one probability scaled by 1 + 1e-6) moves the result
    beyond the bound, so the comparison above has power."""
    (line, ref_m, ref_k, scale), = _cases(O.CLICK, n_per_order=1)[-1:]
    parts = line.split()
    nb = int(parts[1])
    parts[2 + (1 << nb)] = f"{float(parts[2 + (1 << nb)]) * (1 + 1e-6):.17g}"
    r = subprocess.run([checker], input=" ".join(parts) + "\n", capture_output=True, text=True,
                       timeout=60)
    m, k = map(float, r.stdout.split())
    assert abs(k - ref_k) > 1e-13 * scale + 1e-15
