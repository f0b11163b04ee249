"""Write workloads/mu_table.json: chemical potential versus hole doping.

Input preparation for the synthetic workloads (App. A: mu is the Lagrange
multiplier fixing the electron number).  For each doping on a grid, bisect mu
so that the uniform zero-field d-wave state (chi = 0.2, Delta = +/-0.1,
t = 1, t' = -0.3, J = 0.3, T = 0.005) on a 128 x 128 k-grid has
n = 1 - doping, using the oracle's k-space reference only.

Run from the repository root:  python -m oracle.gen_mu_table
"""
import json
import os

import numpy as np

from .kspace import mu_for_doping


def main():
    grid = np.round(np.arange(0.05, 0.2500001, 0.005), 6)
    chi = [0.2, 0.2, 0.0, 0.0]
    dlt = [0.1, -0.1, 0.0, 0.0]
    mus = [mu_for_doping(float(d), chi, dlt, 1.0, -0.3, 0.3, 0.005, L=128, tol=1e-11) for d in grid]
    path = os.path.join(os.path.dirname(__file__), "..", "workloads", "mu_table.json")
    with open(path, "w") as fh:
        json.dump({"source": "oracle/gen_mu_table.py (uniform state, 128x128 k-grid)",
                   "doping": [float(d) for d in grid], "mu": mus}, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
