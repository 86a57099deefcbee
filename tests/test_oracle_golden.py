"""Stored reference spectra (written by tests/golden/make_golden.py from the oracle).

Checks that the files are consistent with the paper's structure (the merged block
spectrum is the full spectrum) and that the oracle still reproduces them.
"""

import json
import os

import numpy as np

from oracle import eigen as E
from synth import two_phase_cell

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_n8_golden_block_union():
    g = _load("two_phase_n8.json")
    for pt in g["points"].values():
        full = np.array(pt["full_lowest"])
        merged = np.sort(np.concatenate([np.array(b) for b in pt["block_lowest"]]))[:full.size]
        assert np.abs(full - merged).max() <= 1e-12 * full.max()


def test_n8_golden_reproduces():
    g = _load("two_phase_n8.json")
    dims = tuple(g["dims"])
    C21, rho, _ = two_phase_cell(dims, radius=g["radius"], seed=g["seed"])
    pt = g["points"]["k"]
    ev = E.block_spectrum(dims, pt["kappa"], C21, rho, 1)[:12]
    assert np.allclose(ev, pt["block_lowest"][1], rtol=1e-12, atol=0)


def test_n16_golden_one_block_dense():
    """The ARPACK values of one n=16 block agree with dense eigh of that block."""
    g = _load("two_phase_n16.json")
    dims = tuple(g["dims"])
    C21, rho, _ = two_phase_cell(dims, radius=g["radius"], seed=g["seed"])
    ev = E.block_spectrum(dims, g["kappa"], C21, rho, 2)[:10]
    assert np.allclose(ev, g["block_lowest"][2], rtol=1e-10, atol=0)


def test_n32_golden_structure():
    """The n=32 file: per-block values ascending and positive (non-zero ones at
    Gamma), the merged list the lowest 20 of their union, and every block's
    10th value at or above the merged 20th (the certification of the cut)."""
    g = _load("two_phase_n32.json")
    assert tuple(g["dims"]) == (32, 32, 32)
    for pt in g["points"].values():
        blocks = [np.array(b) for b in pt["block_lowest"]]
        merged = np.array(pt["merged_lowest"])
        for b in blocks:
            assert b.size == 10 and np.all(np.diff(b) >= 0) and b[0] > 1e-3
        union = np.sort(np.concatenate(blocks))[:20]
        assert np.array_equal(union, merged)
        assert all(b[-1] >= merged[-1] for b in blocks)
