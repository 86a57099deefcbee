"""The paper's FCC workload: a low-quartz matrix with a silicon sphere (Sec. 7,
Sec. 7.1), as deterministic inputs (no random numbers).

* Lattice: a_1 = (0, a0/2, a0/2), a_2 = (a0/2, 0, a0/2), a_3 = (a0/2, a0/2, 0)
  (columns of A_lat), a0 = 3.0e-2 m.
* Matrix (low quartz): rho_1 = 2650 kg/m^3 and the Voigt stiffness listed in
  Sec. 7.1 (GPa); inclusion (silicon): rho_2 = 2329 kg/m^3, cubic stiffness
  C11 = 166.0, C12 = 64.0, C44 = 79.6 GPa.  Voigt order [11,22,33,23,13,12],
  engineering shear; unlisted entries by symmetry or zero.
* Geometry: sphere centred at the reduced point (1/2, 1/2, 1/2), radius
  R = 0.25 a0.
* Subpixel rule: a node's parameters are (1 - theta) P_1 + theta P_2 with theta
  the silicon volume fraction of its cell.  The paper does not say how theta is
  computed; here the node-centred cell r + [-h/2, h/2)^3 (reduced coordinates) is
  sampled at s^3 midpoints mapped through A_lat, and theta is the fraction
  inside the sphere.
* Units: the grid works in dimensionless variables x = a0 x~, C = C_s C~,
  rho = rho_s rho~ with C_s = 1 GPa, rho_s = 1000 kg/m^3; the dimensionless
  eigenvalue lambda~ gives omega^2 = lambda~ C_s / (rho_s a0^2), f = omega/(2 pi).
* Path: Gamma-X-W-K-Gamma-L-U-W-L-K with the high-symmetry points listed in
  Sec. 7 and 10 intervals per segment (91 points).  The text calls the listed
  triples reduced coordinates (q . a_l = 2 pi kappa_l), but the frequencies the
  paper prints for X, W, Gamma and L (its COMSOL comparison table) are
  reproduced only when the triples are read as Cartesian wave vectors in units
  of 2 pi / a0, kappa = A_lat^T q (the two readings agree at Gamma and L).  The
  default ``reading="cartesian"`` follows the printed results; ``"reduced"``
  takes the text literally.
"""

from __future__ import annotations

import numpy as np

from .materials import pack_c21

A0 = 3.0e-2          # lattice constant (m)
C_SCALE = 1.0e9      # Pa
RHO_SCALE = 1.0e3    # kg / m^3
RHO_QUARTZ = 2650.0
RHO_SILICON = 2329.0
SPHERE_RADIUS = 0.25  # in units of a0

FCC_POINTS = {
    "G": (0.0, 0.0, 0.0),
    "X": (0.0, 0.5, 0.5),
    "W": (0.25, 0.5, 0.75),
    "K": (0.375, 0.375, 0.75),
    "L": (0.5, 0.5, 0.5),
    "U": (0.25, 0.625, 0.625),
}
FCC_ROUTE = ("G", "X", "W", "K", "G", "L", "U", "W", "L", "K")


def fcc_lattice(a0: float = 1.0) -> np.ndarray:
    """A_lat with the basis vectors as columns (a0 = 1: dimensionless)."""
    h = 0.5 * a0
    return np.array([[0.0, h, h], [h, 0.0, h], [h, h, 0.0]])


def quartz_stiffness() -> np.ndarray:
    """Voigt matrix of low quartz in GPa (Sec. 7.1)."""
    C = np.zeros((6, 6))
    C[0, 0] = C[1, 1] = 86.6
    C[0, 1] = 6.9
    C[0, 2] = C[1, 2] = 13.6
    C[2, 2] = 106.7
    C[0, 3] = -17.7
    C[1, 3] = 17.7
    C[3, 3] = C[4, 4] = 57.7
    C[4, 5] = -17.7
    C[5, 5] = 39.85
    return np.triu(C) + np.triu(C, 1).T


def silicon_stiffness() -> np.ndarray:
    """Voigt matrix of silicon in GPa (Sec. 7.1)."""
    C = np.zeros((6, 6))
    C[:3, :3] = 64.0
    for a in range(3):
        C[a, a] = 166.0
        C[3 + a, 3 + a] = 79.6
    return C


def silicon_fraction(dims, supersample: int = 4, radius: float = SPHERE_RADIUS):
    """theta per node (natural order): silicon volume fraction of the node's cell,
    from supersample^3 midpoints."""
    n1, n2, n3 = dims
    A = fcc_lattice(1.0)
    s = int(supersample)
    sub = (np.arange(s) + 0.5) / s - 0.5  # midpoints in units of one cell
    k, j, i = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    base = np.stack([i.ravel() / n1, j.ravel() / n2, k.ravel() / n3], axis=1)  # (n, 3)
    inside = np.zeros(base.shape[0])
    for a in sub:
        for b in sub:
            for c in sub:
                r = base + np.array([a / n1, b / n2, c / n3]) - 0.5
                x = r @ A.T
                inside += (np.einsum("ij,ij->i", x, x) < radius * radius)
    return inside / s ** 3


def fcc_quartz_si_cell(dims, supersample: int = 4):
    """(C21~, rho~, A_lat~, theta): dimensionless stiffness (n x 21) and density
    (n,), the dimensionless lattice matrix and the silicon fraction."""
    if isinstance(dims, int):
        dims = (dims, dims, dims)
    theta = silicon_fraction(dims, supersample)
    c1 = pack_c21(quartz_stiffness())
    c2 = pack_c21(silicon_stiffness())
    C21 = (1.0 - theta)[:, None] * c1[None, :] + theta[:, None] * c2[None, :]
    rho = ((1.0 - theta) * RHO_QUARTZ + theta * RHO_SILICON) / RHO_SCALE
    return C21, rho, fcc_lattice(1.0), theta


def frequency_hz(lam):
    """f = omega / (2 pi) in Hz from the dimensionless eigenvalue."""
    lam = np.asarray(lam, dtype=np.float64)
    return np.sqrt(np.maximum(lam, 0.0) * C_SCALE / (RHO_SCALE * A0 * A0)) / (2.0 * np.pi)


def fcc_point(label: str, reading: str = "cartesian") -> np.ndarray:
    """Reduced Bloch vector kappa of a listed high-symmetry point."""
    p = np.asarray(FCC_POINTS[label], dtype=np.float64)
    if reading == "cartesian":
        return fcc_lattice(1.0).T @ p
    if reading == "reduced":
        return p
    raise ValueError("reading must be 'cartesian' or 'reduced'")


def fcc_path(intervals: int = 10, reading: str = "cartesian"):
    """(kappas (9*intervals + 1, 3), labels) along Gamma-X-W-K-Gamma-L-U-W-L-K."""
    P = [fcc_point(s, reading) for s in FCC_ROUTE]
    ks = [P[0]]
    labels = {0: FCC_ROUTE[0]}
    for s in range(len(P) - 1):
        for t in range(1, intervals + 1):
            ks.append(P[s] + (P[s + 1] - P[s]) * (t / intervals))
        labels[len(ks) - 1] = FCC_ROUTE[s + 1]
    return np.array(ks), labels
