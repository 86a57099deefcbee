"""Index-formula construction of A_h(k) + s*M_h (independent of the Kronecker build).

A grid function v is extended to all integer points by the Bloch condition
(Sec. 3.1, Eq. 3.2): v(x + n_l e_l) = e^{i phi_l} v(x).  A shift by an integer
step d then reads the extended field, (S_d v)(x) = v(x + d), and its adjoint is
the shift by -d.  From this single rule:

  D~_s v (x)   = sum_d c_{s,d} v(x + d)          (Eq. 3.11 written per node)
  D~_s^H v (x) = sum_d c_{s,d} v(x - d)

with d in {0, d1, d2, d3, d4}, d1=(1,1,1), d2=(1,1,-1), d3=(1,-1,1), d4=(1,-1,-1)
(the steps of Eq. 3.9), c_{1,0} = -1/h1, c_{1,l} = 1/(4 h1), c_{2,l} = (+,+,-,-)/(4 h2),
c_{3,l} = (+,-,+,-)/(4 h3) and c_{2,0} = c_{3,0} = 0.  The Cartesian operators are
D_m = -i sum_s (A_lat^-1)_{sm} D~_s (Eqs. 3.12-3.13), strains are B_h^H v and the
result is B_h (C (B_h^H v)) (Eq. 3.14-3.15), written here component by component.

Arrays on the grid are shaped (n3, n2, n1) (i fastest in memory), matching the
node index i + n1*(j + n2*k).

Pinned against the Kronecker build element by element (tests/test_oracle_operator.py).
"""

from __future__ import annotations

import numpy as np

from .discretization import as_dims, phases, spacings, unpack_c21

STEPS = ((1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1))


def stencil_coefficients(dims):
    """c[s, d] for s = 0..2 (D~_1..3) and d = 0..4 (identity, d1..d4)."""
    h, _ = spacings(dims)
    c = np.zeros((3, 5))
    c[0, 0] = -1.0 / h[0]
    c[0, 1:] = 1.0 / (4 * h[0])
    c[1, 1:] = np.array([1, 1, -1, -1]) / (4 * h[1])
    c[2, 1:] = np.array([1, -1, 1, -1]) / (4 * h[2])
    return c


def extended_read(f, d, dims, kappa):
    """g(x) = f_ext(x + d) for a grid array f shaped (n3, n2, n1[, ...])."""
    n1, n2, n3 = as_dims(dims)
    ph = phases(kappa)
    g = f
    for axis_grid, (n, dl, p) in enumerate(((n3, d[2], ph[2]), (n2, d[1], ph[1]),
                                            (n1, d[0], ph[0]))):
        idx = np.arange(n) + dl
        wrap = np.floor_divide(idx, n)
        src = np.mod(idx, n)
        g = np.take(g, src, axis=axis_grid)
        fac = np.exp(1j * p * wrap)
        shape = [1] * g.ndim
        shape[axis_grid] = n
        g = g * fac.reshape(shape)
    return g


def _grid(vec, dims):
    n1, n2, n3 = as_dims(dims)
    return np.asarray(vec).reshape(3, n3, n2, n1)


def strains(v, dims, kappa, A_lat=None):
    """B_h^H v as six grid arrays (eps1..eps6), v component-major (3n,)."""
    dims = as_dims(dims)
    V = _grid(v, dims)
    c = stencil_coefficients(dims)
    Ainv = np.eye(3) if A_lat is None else np.linalg.inv(np.asarray(A_lat, float))
    steps = [(0, 0, 0)] + list(STEPS)
    # Dt_adj[s][a] = D~_s^H v_a
    Dt_adj = [[0.0 for _ in range(3)] for _ in range(3)]
    for dd, d in enumerate(steps):
        back = (-d[0], -d[1], -d[2])
        for a in range(3):
            shifted = extended_read(V[a], back, dims, kappa)
            for s in range(3):
                if c[s, dd] != 0.0:
                    Dt_adj[s][a] = Dt_adj[s][a] + c[s, dd] * shifted
    # D_m^H = +i sum_s (A_lat^-1)_{sm} D~_s^H
    G = [[1j * sum(Ainv[s, m] * Dt_adj[s][a] for s in range(3)) for a in range(3)]
         for m in range(3)]
    # Rows of B_h^H (transpose of Eq. 3.14 blocks): strain components.
    e1 = G[0][0]
    e2 = G[1][1]
    e3 = G[2][2]
    e4 = G[2][1] + G[1][2]
    e5 = G[2][0] + G[0][2]
    e6 = G[1][0] + G[0][1]
    return [e1, e2, e3, e4, e5, e6]


def stresses(eps, C21):
    """tau = C(x) eps(x) nodewise."""
    C = unpack_c21(C21)  # (n, 6, 6)
    shape = eps[0].shape
    E = np.stack([e.ravel() for e in eps], axis=1)  # (n, 6)
    T = np.einsum("nab,nb->na", C, E)
    return [T[:, a].reshape(shape) for a in range(6)]


def divergence(tau, dims, kappa, A_lat=None):
    """B_h tau (Eq. 3.14) from six grid arrays; returns (3n,) component-major."""
    dims = as_dims(dims)
    c = stencil_coefficients(dims)
    Ainv = np.eye(3) if A_lat is None else np.linalg.inv(np.asarray(A_lat, float))
    steps = [(0, 0, 0)] + list(STEPS)
    Dt = [[0.0 for _ in range(6)] for _ in range(3)]  # Dt[s][b] = D~_s tau_b
    for dd, d in enumerate(steps):
        for b in range(6):
            shifted = extended_read(tau[b], d, dims, kappa)
            for s in range(3):
                if c[s, dd] != 0.0:
                    Dt[s][b] = Dt[s][b] + c[s, dd] * shifted
    D = [[-1j * sum(Ainv[s, m] * Dt[s][b] for s in range(3)) for b in range(6)]
         for m in range(3)]
    y1 = D[0][0] + D[2][4] + D[1][5]
    y2 = D[1][1] + D[2][3] + D[0][5]
    y3 = D[2][2] + D[1][3] + D[0][4]
    return np.concatenate([y1.ravel(), y2.ravel(), y3.ravel()])


def apply_A(v, dims, kappa, C21, rho=None, s=0.0, A_lat=None):
    """y = (A_h(k) + s M_h) v for a full-space vector v (3n,)."""
    dims = as_dims(dims)
    v = np.asarray(v, dtype=np.complex128)
    y = divergence(stresses(strains(v, dims, kappa, A_lat), C21), dims, kappa, A_lat)
    if s != 0.0:
        r = np.asarray(rho, dtype=np.float64)
        y = y + s * np.concatenate([r, r, r]) * v
    return y


# ----------------------------------------------------------------------------
# Single-node evaluation (for sampled checks on grids too large to sweep)
# ----------------------------------------------------------------------------

def _node(x, dims):
    n1, n2, n3 = dims
    return x[0] + n1 * (x[1] + n2 * x[2])


def _ext(x, d, dims, ph):
    """Node index of x + d and the Bloch phase picked up by the wrap."""
    idx, fac = [], 1.0 + 0j
    for l in range(3):
        q, r = divmod(x[l] + d[l], dims[l])
        idx.append(r)
        fac *= np.exp(1j * ph[l] * q)
    return tuple(idx), fac


def apply_A_at(points, v, dims, kappa, C21, rho=None, s=0.0, A_lat=None):
    """y(x) for each grid point x=(i,j,k) in ``points``; returns (len, 3)."""
    dims = as_dims(dims)
    n = dims[0] * dims[1] * dims[2]
    ph = phases(kappa)
    v = np.asarray(v, dtype=np.complex128).reshape(3, n)
    c = stencil_coefficients(dims)
    Ainv = np.eye(3) if A_lat is None else np.linalg.inv(np.asarray(A_lat, float))
    steps = [(0, 0, 0)] + list(STEPS)
    C21 = np.asarray(C21)

    def tau_at(z):
        # D~_s^H v_a at z, then Cartesian mix and strain, then C.
        g = np.zeros((3, 3), dtype=np.complex128)  # g[s, a]
        for dd, d in enumerate(steps):
            nb, fac = _ext(z, (-d[0], -d[1], -d[2]), dims, ph)
            vv = v[:, _node(nb, dims)] * fac
            for sdir in range(3):
                g[sdir] += c[sdir, dd] * vv
        G = 1j * (Ainv.T @ g)  # G[m, a] = i sum_s Ainv[s, m] g[s, a]
        eps = np.array([G[0, 0], G[1, 1], G[2, 2], G[2, 1] + G[1, 2],
                        G[2, 0] + G[0, 2], G[1, 0] + G[0, 1]])
        Cz = unpack_c21(C21[_node(z, dims)])
        return Cz @ eps

    out = np.zeros((len(points), 3), dtype=np.complex128)
    for t, x in enumerate(points):
        x = tuple(int(u) for u in x)
        Dt = np.zeros((3, 6), dtype=np.complex128)  # D~_s tau_b at x
        for dd, d in enumerate(steps):
            nb, fac = _ext(x, d, dims, ph)
            tz = tau_at(nb) * fac
            for sdir in range(3):
                Dt[sdir] += c[sdir, dd] * tz
        D = -1j * (Ainv.T @ Dt)  # D[m, b]
        y = np.array([D[0, 0] + D[2, 4] + D[1, 5],
                      D[1, 1] + D[2, 3] + D[0, 5],
                      D[2, 2] + D[1, 3] + D[0, 4]])
        if s != 0.0:
            y = y + s * float(np.asarray(rho)[_node(x, dims)]) * v[:, _node(x, dims)]
        out[t] = y
    return out
