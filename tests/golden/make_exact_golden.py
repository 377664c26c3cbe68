"""Writes exact_ccg_n6_p2.json: an exact-rational cCG run on a tiny integer system.

Calls only the oracle's exact-arithmetic routine and the seeded input generator.
Run from the repository root:  python tests/golden/make_exact_golden.py
"""
import json
import os
import sys

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))

import ccg_inputs  # noqa: E402
from oracle import exact  # noqa: E402


def frac_str(v):
    return f"{v.numerator}/{v.denominator}"


def main():
    n, p, seed = 6, 2, 7
    A, b, X0 = ccg_inputs.integer_system(n, p, seed)
    run = exact.ccg(A, b, X0, steps=n // p)
    doc = {
        "what": "exact cCG (Alg. 2, sign convention R = B - A X) on an integer SPD system; "
                "n/p steps, after which R must be exactly zero (Theorem 3, genericity)",
        "n": n, "p": p, "seed": seed, "A": A, "b": b, "X0": X0,
        "alphas": [[[frac_str(v) for v in row] for row in a] for a in run["alphas"]],
        "betas": [[[frac_str(v) for v in row] for row in bt] for bt in run["betas"]],
        "X_final": [[frac_str(v) for v in row] for row in run["Xs"][-1]],
    }
    out = os.path.join(os.path.dirname(__file__), "exact_ccg_n6_p2.json")
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
