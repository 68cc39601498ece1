"""Write margin_lambda0.json: the smallest eigenvalue of the unshifted
conditioning-sweep matrix (N = 4096, n = 64, seed 11 of the input recipe),
found by the oracle-based bisection of tests/margin.py.  The benchmark's
conditioning-sweep leg reads it to shift the diagonal so that
lambda_min(Psi) = c exactly (the margin reading of the shift).

    python tests/golden/make_margin_lambda0.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.dirname(HERE)]

from margin import lambda0_bisect  # noqa: E402
from paper_2601_03754_amd import inputs  # noqa: E402

N, n, SEED, NRHS = 4096, 64, 11, 4


def main():
    GG, E, _ = inputs.unshifted(N, n, seed=SEED, nrhs=NRHS)
    lam0 = lambda0_bisect(GG, E)
    out = {"N": N, "n": n, "seed": SEED, "nrhs": NRHS, "lambda0": lam0, "tol": 1e-7,
           "method": "bisection on the success of the oracle's block Cholesky (Algorithm 1) of the shifted matrix"}
    with open(os.path.join(HERE, "margin_lambda0.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(out)


if __name__ == "__main__":
    main()
