"""Write the stored reference spectra under tests/golden/ using only the oracle.

Run from the repository root:  python tests/golden/make_golden.py

Outputs
-------
two_phase_n8.json   n = 8 two-phase cell (radius 0.35, seed 0): the 12 lowest
                    (non-zero at Gamma) eigenvalues of the full pencil and of each
                    parity block, dense LAPACK, at kappa = (0.15, 0.05, 0.10) and Gamma.
two_phase_n16.json  n = 16, same cell recipe: 10 lowest eigenvalues of each block at
                    kappa = (0.15, 0.05, 0.10) by ARPACK shift-invert (SuperLU).
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import eigen as E, solve as S  # noqa: E402
from oracle.discretization import default_shift  # noqa: E402
from synth import two_phase_cell  # noqa: E402

KAPPA = (0.15, 0.05, 0.10)


def n8():
    dims = (8, 8, 8)
    C21, rho, _ = two_phase_cell(dims, radius=0.35, seed=0)
    out = {"dims": dims, "radius": 0.35, "seed": 0, "delta": default_shift(C21), "points": {}}
    for name, kap in (("k", KAPPA), ("gamma", (0.0, 0.0, 0.0))):
        full = E.full_spectrum(dims, kap, C21, rho)
        blocks = [E.block_spectrum(dims, kap, C21, rho, b) for b in range(4)]
        out["points"][name] = {
            "kappa": list(kap),
            "full_lowest": [float(v) for v in full[:24]],
            "block_lowest": [[float(v) for v in bl[:12]] for bl in blocks],
        }
    return out


def n16():
    dims = (16, 16, 16)
    C21, rho, _ = two_phase_cell(dims, radius=0.35, seed=0)
    blocks = [S.shift_invert_lowest(dims, KAPPA, C21, rho, 10, sigma=-1.0, block=b)
              for b in range(4)]
    return {"dims": dims, "radius": 0.35, "seed": 0, "kappa": list(KAPPA),
            "delta": default_shift(C21),
            "block_lowest": [[float(v) for v in bl] for bl in blocks]}


if __name__ == "__main__":
    with open(os.path.join(HERE, "two_phase_n8.json"), "w") as f:
        json.dump(n8(), f, indent=1)
    with open(os.path.join(HERE, "two_phase_n16.json"), "w") as f:
        json.dump(n16(), f, indent=1)
    print("written")
