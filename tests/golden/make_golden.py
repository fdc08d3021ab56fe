"""Writes the stored expected values under tests/golden/ from the oracle only.

  small_theory.json -- closed forms for the 2000 x 1000 workload with
      sigma_i = 0.9^i (i = 1..1000), r = 50, l = 25: the optimal error
      ||A - A_50||_F and the expectation bounds of Theorems 3.1 and 3.2.
  tiny_exact.json   -- an 8 x 6 integer A with integer sketches X (6 x 3) and
      Y (8 x 5) and the exact rational plain-GN approximant AX (Y^T A X)^+ Y^T A
      (Section 2, eq. (3)), computed over fractions by oracle.exact.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact, gn as G  # noqa: E402


def main():
    sig = 0.9 ** np.arange(1, 1001, dtype=np.float64)
    theory = {
        "workload": "2000x1000, sigma_i = 0.9^i, r = 50, l = 25",
        "optimal_error_r50": G.optimal_error(sig, 50),
        "thm3_1_bound": G.hmt_bound(sig, 50),
        "thm3_2_bound": G.gn_bound(sig, 50, 25),
        "gn_over_hmt_factor": G.gn_over_hmt_factor(50, 25),
        "frobenius_norm_A": float(np.sqrt(np.sum(sig ** 2))),
    }
    with open(os.path.join(HERE, "small_theory.json"), "w") as f:
        json.dump(theory, f, indent=1)

    rng = np.random.default_rng(2009)
    A = rng.integers(-3, 4, size=(8, 6))
    X = rng.integers(-2, 3, size=(6, 3))
    Y = rng.integers(-2, 3, size=(8, 5))
    Ahat = exact.gn_exact(A, X, Y)
    tiny = {"source": "oracle.exact.gn_exact (fractions), Section 2 eq. (3)",
            "A": A.tolist(), "X": X.tolist(), "Y": Y.tolist(),
            "A_hat": [[str(v) for v in row] for row in Ahat]}
    with open(os.path.join(HERE, "tiny_exact.json"), "w") as f:
        json.dump(tiny, f, indent=1)


if __name__ == "__main__":
    main()
