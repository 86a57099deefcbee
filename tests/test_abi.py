"""C-ABI checks that need no GPU: the library loads, exports every function the
headers declare, and its host-side logic (Rayleigh-Ritz eigensolver, merge
certification, argument validation that fails before touching a device) works.
"""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2606_03599_amd import pbr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(pbr_\w+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    return pbr.lib()


def test_every_declared_symbol_exported(L):
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    # and the binding wraps each of them under the same name
    for n in names:
        assert n in pbr._SIGS, n


def test_opts_defaults(L):
    o = pbr.pbr_opts_default()
    assert o.tol == 1e-12 and o.tol_inner == 1e-12
    assert o.maxit_outer == 300 and o.maxit_inner == 200
    assert o.precond == 1 and o.ncv == 0
    assert o.concurrent == 1 and o.graphs == 1 and o.warm_start == 1


def test_create_rejects_bad_sizes(L):
    with pytest.raises(pbr.PbrError) as e:
        pbr.pbr_create(0, 4, 4)
    assert e.value.status == pbr.PBR_EINVAL
    with pytest.raises(pbr.PbrError) as e:
        pbr.pbr_create(4, 4, 4, A_lat=np.zeros((3, 3)))
    assert e.value.status == pbr.PBR_EINVAL
    assert "singular" in pbr.pbr_last_error(None)


def test_null_context_calls_fail_cleanly(L):
    assert L.pbr_block_dim(None, 0) == -1
    assert L.pbr_default_shift(None) < 0
    assert L.pbr_material_palette(None) == -1
    assert L.pbr_set_palette(None, 1) == -1  # PBR_EINVAL
    assert L.pbr_set_stencil_shape(None, 16, 13) == -1
    assert L.pbr_set_solve_width(None, 16) == -1
    assert L.pbr_set_precond_passes(None, 3) == -1
    L.pbr_destroy(None)


def test_band_paths_rejects_bad_arguments(L):
    """pbr_band_paths validates its arguments before any cell starts (no GPU)."""
    from paper_2606_03599_amd import pbr
    L.pbr_band_paths.restype = ctypes.c_int
    assert L.pbr_band_paths(0, None, None, None, 4, 1, 0.0, None, None, None) == pbr.PBR_EINVAL
    assert L.pbr_band_paths(65, None, None, None, 4, 1, 0.0, None, None, None) == pbr.PBR_EINVAL
    hs = (ctypes.c_void_p * 2)(None, None)
    nk = (ctypes.c_int * 2)(1, 1)
    assert L.pbr_band_paths(2, hs, nk, None, 4, 1, 0.0, None, None, None) == pbr.PBR_EINVAL


@pytest.mark.parametrize("m", [1, 2, 5, 17, 40])
def test_host_heev_matches_numpy(L, m):
    rng = np.random.default_rng(m)
    G = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    A = G + G.conj().T
    w, V = pbr.pbr_host_heev(A)
    assert np.allclose(w, np.linalg.eigvalsh(A), rtol=0, atol=1e-12 * np.abs(w).max())
    assert np.allclose(V.conj().T @ V, np.eye(m), atol=1e-12)
    assert np.allclose(A @ V, V * w, atol=1e-11 * np.abs(w).max())


def test_host_heev_degenerate(L):
    Q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((6, 6)) + 0j)
    A = Q @ np.diag([1, 1, 1, 2, 2, 5.0]) @ Q.conj().T
    w, V = pbr.pbr_host_heev(A)
    assert np.allclose(w, [1, 1, 1, 2, 2, 5], atol=1e-13)
    assert np.allclose(A @ V, V * w, atol=1e-12)


def test_host_merge_rule(L):
    vals = [[1.0, 4.0], [2.0, 3.0], [0.5, 6.0], [7.0, 8.0]]
    mask, merged = pbr.pbr_host_merge(4, vals)
    assert np.allclose(merged, [0.5, 1.0, 2.0, 3.0])
    # cut = 3.0: block 1's largest (3.0) is not below the cut -> certified;
    # blocks 0, 2, 3 have largest 4, 6, 8 >= 3 -> certified
    assert mask == 0
    mask, merged = pbr.pbr_host_merge(6, vals)
    # cut = 6.0: block 0 largest 4 < 6 and block 1 largest 3 < 6 -> recompute both
    assert mask == 0b0011
    assert np.allclose(merged, [0.5, 1, 2, 3, 4, 6])
    assert pbr.pbr_host_merge(20, vals)[0] == -1
