"""Continuum elastic plane waves (textbook Christoffel equation), used as a pin.

For a homogeneous medium with fourth-order stiffness C_ijkl and density rho, a
plane wave exp(i q.x) has omega^2 rho u = Gamma(q) u with the Christoffel matrix
Gamma_ik = sum_{j,l} C_ijkl q_j q_l.  The Voigt matrix maps to C_ijkl by the
index pairs 11->1, 22->2, 33->3, 23->4, 13->5, 12->6 (Sec. 2, Eqs. 2.4-2.6; with
engineering shear strains the Voigt stiffness entries equal the tensor
entries).  The discrete eigenvalues approach these values for small q (the
low-frequency consistency of Remark 3.1).
"""

from __future__ import annotations

import numpy as np

_PAIR = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (1, 2): 3, (2, 1): 3, (0, 2): 4,
         (2, 0): 4, (0, 1): 5, (1, 0): 5}


def voigt_to_tensor(C6):
    C = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    C[i, j, k, l] = C6[_PAIR[(i, j)], _PAIR[(k, l)]]
    return C


def christoffel_eigs(C6, rho, q):
    """omega^2 of the three plane waves with physical wave vector q."""
    C = voigt_to_tensor(np.asarray(C6, float))
    q = np.asarray(q, float)
    G = np.einsum("ijkl,j,l->ik", C, q, q)
    return np.sort(np.linalg.eigvalsh(G)) / rho
