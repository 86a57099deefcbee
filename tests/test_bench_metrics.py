"""Host-side metric of the grid-refinement study (bench.grouped_errors, the
grouped relative frequency error of Sec. 7.5), checked on hand-made spectra."""

import numpy as np

from bench import grouped_errors


def test_grouped_errors_plain():
    ref = np.arange(1.0, 41.0) ** 2          # frequencies 1..40
    lam = (np.arange(1.0, 41.0) * 1.01) ** 2  # every frequency 1 % high
    e = grouped_errors(lam, ref, 0, 40)
    assert len(e) == 10 and np.allclose(e, 0.01)


def test_grouped_errors_group_means_and_gamma_exclusion():
    # Gamma: 12 zero modes are not passed in; groups 0..2 hold only zero modes
    ref = np.arange(1.0, 29.0) ** 2
    f = np.arange(1.0, 29.0).copy()
    f[0] *= 1.04   # first non-zero band: group 3 (bands 12..15) sees one 4 % error
    f[27] *= 0.98  # last band: group 9 sees one 2 % error
    e = grouped_errors(f ** 2, ref, 12, 40)
    assert e[:3] == [None, None, None]
    assert abs(e[3] - 0.04 / 4) < 1e-15 and abs(e[9] - 0.02 / 4) < 1e-15
    assert all(abs(x) < 1e-15 for x in e[4:9])


def test_grouped_errors_partial_zero_group():
    # 2 zero modes: group 0 averages its 2 non-zero members only
    ref = np.ones(6)
    lam = np.array([1.21, 1.0, 1.0, 1.0, 1.0, 1.0])  # 10 % frequency error on band 2
    e = grouped_errors(lam, ref, 2, 8)
    assert abs(e[0] - 0.05) < 1e-15 and e[1] == 0.0
