"""Host side of the material's palette form (pbr_host_palette): the distinct
(C21, rho) rows compared bit for bit, numbered in order of first appearance, and
each node's row.  Checked without a GPU against the definition: every node's row
reproduces its 22 doubles bit for bit, the rows are distinct, the numbering
follows first appearance, and more than 256 distinct rows is reported as such."""

import numpy as np
import pytest

from paper_2606_03599_amd import pbr
from synth import two_phase_cell
from synth.materials import pack_c21, random_spd_stiffness


def labelled(n, K, seed):
    rng = np.random.default_rng(seed)
    rows = np.stack([pack_c21(random_spd_stiffness(rng)) for _ in range(K)])
    rhos = rng.uniform(0.5, 4.0, K)
    lab = rng.integers(0, K, n)
    lab[rng.permutation(n)[:K]] = np.arange(K)
    return rows[lab], rhos[lab]


def check(C21, rho, rows, idx):
    full = np.concatenate([C21, rho[:, None]], axis=1)
    assert np.array_equal(rows[idx].view(np.uint64), full.view(np.uint64))
    k = rows.shape[0]
    assert len({r.tobytes() for r in rows}) == k
    first = [int(np.argmax(idx == r)) for r in range(k)]
    assert first == sorted(first) and first[0] == 0


@pytest.mark.parametrize("K", [1, 7, 256])
def test_palette_rows_reproduce_every_node(K):
    C21, rho = labelled(3000, K, seed=K)
    out = pbr.pbr_host_palette(C21, rho)
    assert out is not None
    rows, idx = out
    assert rows.shape == (K, 22)
    check(C21, rho, rows, idx)


def test_more_than_256_rows_is_reported():
    C21, rho = labelled(3000, 257, seed=3)
    assert pbr.pbr_host_palette(C21, rho) is None


def test_two_phase_cell_and_bitwise_rows():
    C21, rho, _ = two_phase_cell((16, 16, 16), radius=0.35, seed=0)
    rows, idx = pbr.pbr_host_palette(C21, rho)
    assert rows.shape[0] == 2 and idx[0] == 0 and rho[0] == rows[0, 21]
    check(C21, rho, rows, idx)
    # +0.0 and -0.0, or one ulp, make rows of their own
    C2 = C21.copy()
    C2[5, 3] = -0.0 if C2[5, 3] == 0.0 else np.nextafter(C2[5, 3], np.inf)
    rows2, idx2 = pbr.pbr_host_palette(C2, rho)
    assert rows2.shape[0] == 3 and idx2[5] == 1  # second row to appear (node 5)
    check(C2, rho, rows2, idx2)


def test_bad_arguments():
    with pytest.raises(pbr.PbrError):
        pbr.pbr_host_palette(np.zeros((0, 21)), np.zeros(0))
