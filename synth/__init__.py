"""Seeded synthetic inputs for the parity-blocked Bloch eigensolver.

This package only *generates inputs*: material fields, Bloch wave vectors and
random test vectors.  It holds none of the method's arithmetic (no shifts, no
derivatives, no stiffness operator), so both the CPU oracle and the GPU path can
draw from it without sharing any computation.
"""

from .materials import (
    cubic_stiffness,
    haar_orthogonal,
    random_spd_stiffness,
    pack_c21,
    two_phase_cell,
    homogeneous_cell,
    random_spd_field,
    batch_cells,
)
from .kpath import SC_POINTS, sc_path, split_intervals
from .fcc import (
    FCC_POINTS,
    fcc_lattice,
    fcc_path,
    fcc_point,
    fcc_quartz_si_cell,
    frequency_hz,
    quartz_stiffness,
    silicon_stiffness,
)
from .vectors import complex_gaussian

__all__ = [
    "cubic_stiffness",
    "haar_orthogonal",
    "random_spd_stiffness",
    "pack_c21",
    "two_phase_cell",
    "homogeneous_cell",
    "random_spd_field",
    "batch_cells",
    "SC_POINTS",
    "sc_path",
    "split_intervals",
    "complex_gaussian",
    "FCC_POINTS",
    "fcc_lattice",
    "fcc_path",
    "fcc_point",
    "fcc_quartz_si_cell",
    "frequency_hz",
    "quartz_stiffness",
    "silicon_stiffness",
]
