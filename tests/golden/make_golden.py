"""Writes the stored expected values under tests/golden/ from the oracle only.

zolotarev_inv_sqrt_n8.json: Zolotarev's x^(-1/2) coefficients for 8 poles on
[1e-4, 50] (the spectrum interval of the 48^3 x 12, m = 0.005 workload, rounded)
as computed by oracle.rational; the test-suite checks that the library's host
routine reproduces them and that the oracle still does.

Run from the repository root: python tests/golden/make_golden.py
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import rational  # noqa: E402


def main():
    lmin, lmax, n = 1e-4, 50.0, 8
    a0, al, sh, delta = rational.zolotarev_inv_sqrt(lmin, lmax, n)
    rec = {"source": "oracle.rational.zolotarev_inv_sqrt", "lmin": lmin, "lmax": lmax, "npole": n,
           "alpha0": a0, "alpha": [float(v) for v in al], "shift": [float(v) for v in sh], "delta": delta}
    with open(os.path.join(HERE, "zolotarev_inv_sqrt_n8.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
