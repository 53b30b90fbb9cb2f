"""Write the stored expected values under tests/golden/.

Calls only the oracle and the seeded input generator; nothing here touches the
HIP path.  Re-run after any change to the oracle's arithmetic:
    python tests/golden/make_golden.py
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gbs_inputs as G  # noqa: E402
import oracle as O  # noqa: E402


def main():
    inst = G.make_instance("m16_k3")
    for conv, tag in ((O.CLICK, "click"), (O.PARITY, "parity")):
        corr, cum = O.correlators_and_cumulants(inst.sigma, 3, conv)
        np.savez(os.path.join(HERE, f"m16_k3_{tag}.npz"), sigma=inst.sigma, corr=corr, cum=cum)
    # closed forms: TMSV pair (r -> tanh^2 r, tanh^2 r sech^2 r)
    with open(os.path.join(HERE, "closed_forms.txt"), "w") as f:
        f.write("# closed-form values (tests/golden/README.md gives the passages they follow)\n")
        f.write("# kind r eta mu kappa\n")
        for r in (0.3, 0.8, 1.3):
            t2 = math.tanh(r) ** 2
            f.write(f"tmsv {r!r} 1.0 {t2!r} {t2 / math.cosh(r) ** 2!r}\n")
        for r, eta in ((0.3, 1.0), (0.7, 0.4), (1.1, 0.9), (1.5, 0.25)):
            det = (1 - eta * (1 - math.exp(-2 * r)) / 2) * (1 + eta * (math.exp(2 * r) - 1) / 2)
            mu = 1 - det ** -0.5
            f.write(f"single {r!r} {eta!r} {mu!r} {mu!r}\n")


if __name__ == "__main__":
    main()
