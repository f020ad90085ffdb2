"""Write exact expectations of the Monte Carlo row estimator for tiny matrices.

The estimator of eq. (2) (Section III-A) averages, over chains started at row r,
the sum of the chain weights W_j at the states s_j it visits. For a matrix whose
entries are dyadic rationals the transition probabilities p = |c| / sum|c| and the
weights c / p are exact rationals, so the expectation of every entry, and of its
square, can be enumerated over all paths with Python's ``fractions``. This script
uses no oracle code and no floating point for the expectations.

Conventions (the readings of the paper this implementation takes):
* the start state contributes W_0 = 1 (the identity term of the Neumann series);
* before each draw the chain stops if the row of C is empty or the next weight
  |W * sum_k |c_sk|| is strictly below delta;
* at most L_max transitions.

Run:  python tests/golden/make_golden.py   (rewrites tests/golden/*.json)
"""
from __future__ import annotations

import json
import os
from fractions import Fraction as F

HERE = os.path.dirname(os.path.abspath(__file__))


def enumerate_row(C, r, delta, lmax):
    """Exact E[X_c] and E[X_c^2] for one chain from row r (X_c = sum of W_j at c)."""
    n = len(C)
    mean = [F(0)] * n
    second = [F(0)] * n

    def rec(s, w, prob, j, acc):
        row = [(k, C[s][k]) for k in range(n) if C[s][k] != 0]
        S = sum(abs(v) for _, v in row)
        stop = (not row) or j >= lmax or abs(w * S) < delta
        if stop:
            for c in range(n):
                mean[c] += prob * acc[c]
                second[c] += prob * acc[c] * acc[c]
            return
        for k, v in row:
            p = abs(v) / S
            wn = w * S * (1 if v > 0 else -1)
            acc2 = list(acc)
            acc2[k] += wn
            rec(k, wn, prob * p, j + 1, acc2)

    acc0 = [F(0)] * n
    acc0[r] = F(1)
    rec(r, F(1), F(1), 0, acc0)
    return mean, second


CASES = {
    # 3x3, dyadic |c| with both signs; delta = 1/8 is reached exactly by some paths,
    # so the strict "< delta" test matters.
    "tiny3_signed": {
        "diag": [2, -4, 1],
        "C": [[0, F(1, 2), F(-1, 4)],
              [F(1, 4), 0, F(1, 4)],
              [F(-1, 2), F(1, 8), 0]],
        "delta": F(1, 8),
        "lmax": 64,
    },
    # 4x4 with an empty row (state 3 absorbs) and a long tail; delta small.
    "tiny4_absorbing": {
        "diag": [1, 2, 4, 8],
        "C": [[0, F(1, 4), F(1, 4), 0],
              [F(1, 2), 0, 0, F(1, 4)],
              [0, F(-1, 2), 0, F(1, 8)],
              [0, 0, 0, 0]],
        "delta": F(1, 1024),
        "lmax": 64,
    },
}


def main():
    for name, case in CASES.items():
        C = case["C"]
        n = len(C)
        rows = []
        for r in range(n):
            mean, second = enumerate_row(C, r, case["delta"], case["lmax"])
            rows.append({"mean": [str(x) for x in mean], "second": [str(x) for x in second]})
        # B = D (I - C): b_ii = d_i, b_ij = -d_i c_ij
        B = [[(case["diag"][i] if i == j else -case["diag"][i] * C[i][j]) for j in range(n)]
             for i in range(n)]
        out = {
            "cite": "eq. (2), Section III-A: row estimate = mean over chains of the summed "
                    "weights at each visited state; exact expectation by path enumeration",
            "B": [[str(x) for x in row] for row in B],
            "diag": [str(x) for x in case["diag"]],
            "delta": str(case["delta"]),
            "lmax": case["lmax"],
            "rows": rows,
        }
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f, indent=1)
        print("wrote", name)


if __name__ == "__main__":
    main()
