"""Write the stored reference spectra under tests/golden/ using only the oracle.

Run from the repository root:  python tests/golden/make_golden.py

Outputs
-------
two_phase_n8.json   n = 8 two-phase cell (radius 0.35, seed 0): the 12 lowest
                    (non-zero at Gamma) eigenvalues of the full pencil and of each
                    parity block, dense LAPACK, at kappa = (0.15, 0.05, 0.10) and Gamma.
two_phase_n16.json  n = 16, same cell recipe: 10 lowest eigenvalues of each block at
                    kappa = (0.15, 0.05, 0.10) by ARPACK shift-invert (SuperLU).
two_phase_n32.json  n = 32, same cell recipe: the 10 lowest (non-zero at Gamma)
                    eigenvalues of each parity block at kappa = (0.15, 0.05, 0.10) and
                    at Gamma by ARPACK shift-invert (SuperLU; Sec. 6.1, Corollary 4.2),
                    and the 20 lowest of their union, certified: every block's 10th
                    value lies at or above the union's 20th, so no block can hide a
                    smaller one (about 100 s per block solve; four processes).

Usage: python tests/golden/make_golden.py [n8] [n16] [n32]   (default: all)
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


def _n32_block(args):
    name, kap, b = args
    dims = (32, 32, 32)
    C21, rho, _ = two_phase_cell(dims, radius=0.35, seed=0)
    gamma = name == "gamma"
    nz = 3 if gamma else 0  # Gamma: 3 zero modes per block (Appendix C)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=2):  # four processes on the host's cores
        vals = S.shift_invert_lowest(dims, kap, C21, rho, 10 + nz, sigma=-1.0, block=b)
    if gamma:
        assert np.all(np.abs(vals[:3]) < 1e-8), vals[:4]
        assert vals[3] > 1e-3, vals[:4]
    return name, b, [float(v) for v in vals[nz:]]


def n32():
    from multiprocessing import Pool
    dims = (32, 32, 32)
    C21, _, _ = two_phase_cell(dims, radius=0.35, seed=0)
    points = {"k": KAPPA, "gamma": (0.0, 0.0, 0.0)}
    jobs = [(name, kap, b) for name, kap in points.items() for b in range(4)]
    with Pool(4) as pool:
        res = pool.map(_n32_block, jobs)
    out = {"dims": dims, "radius": 0.35, "seed": 0, "delta": default_shift(C21),
           "solver": "scipy eigsh shift-invert, sigma = -1, tol 1e-13, per block",
           "points": {}}
    for name, kap in points.items():
        blocks = [next(v for nm, bb, v in res if nm == name and bb == b) for b in range(4)]
        union = np.sort(np.concatenate(blocks))[:20]
        assert all(bl[-1] >= union[-1] for bl in blocks), "union not certified"
        out["points"][name] = {"kappa": list(kap),
                               "block_lowest": blocks,
                               "merged_lowest": [float(v) for v in union]}
    return out


if __name__ == "__main__":
    which = sys.argv[1:] or ["n8", "n16", "n32"]
    for name in which:
        with open(os.path.join(HERE, f"two_phase_{name}.json"), "w") as f:
            json.dump({"n8": n8, "n16": n16, "n32": n32}[name](), f, indent=1)
        print("written", name)
