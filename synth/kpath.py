"""Bloch wave-vector paths in reduced reciprocal coordinates.

A reduced vector kappa gives the boundary phases phi_l = 2*pi*kappa_l.  For the
simple-cubic unit cell the high-symmetry points are Gamma=(0,0,0),
X=(1/2,0,0), M=(1/2,1/2,0), R=(1/2,1/2,1/2), and the path is
Gamma-X-M-Gamma-R.  ``npts`` points split ``npts-1`` intervals across the
segments in proportion to segment length (largest remainder; ties go to the
earlier segment).  The endpoints of every segment are included exactly once.
"""

from __future__ import annotations

import numpy as np

SC_POINTS = {
    "G": (0.0, 0.0, 0.0),
    "X": (0.5, 0.0, 0.0),
    "M": (0.5, 0.5, 0.0),
    "R": (0.5, 0.5, 0.5),
}

SC_ROUTE = ("G", "X", "M", "G", "R")


def split_intervals(lengths, total: int):
    """Largest-remainder apportionment of ``total`` intervals to segments."""
    lengths = np.asarray(lengths, dtype=np.float64)
    quota = total * lengths / lengths.sum()
    base = np.floor(quota).astype(int)
    rem = quota - base
    left = total - int(base.sum())
    # stable sort on -remainder keeps earlier segments first on ties
    order = sorted(range(len(lengths)), key=lambda s: (-round(rem[s], 12), s))
    for s in order[:left]:
        base[s] += 1
    return [int(b) for b in base]


def sc_path(npts: int, route=SC_ROUTE, points=SC_POINTS):
    """Return ``(kappas, labels)``: an ``(npts, 3)`` array of reduced Bloch
    vectors and a dict mapping path index -> high-symmetry label."""
    if npts < len(route):
        raise ValueError("need at least one point per high-symmetry vertex")
    P = [np.asarray(points[s], dtype=np.float64) for s in route]
    lens = [float(np.linalg.norm(P[s + 1] - P[s])) for s in range(len(P) - 1)]
    counts = split_intervals(lens, npts - 1)
    ks = [P[0]]
    labels = {0: route[0]}
    for s, c in enumerate(counts):
        for t in range(1, c + 1):
            ks.append(P[s] + (P[s + 1] - P[s]) * (t / c))
        labels[len(ks) - 1] = route[s + 1]
    return np.array(ks), labels
