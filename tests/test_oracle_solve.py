"""Pins of the oracle's error control and outer iteration (paper Sec. 2.6)."""
import math

import numpy as np
import pytest

from paper_2105_09644_amd import workloads as W


def test_delta_cell_hand_values(orc):
    old = np.array([0.0, 1.0, 2.0, 4.0, 8.0])          # lower median 2
    new = np.array([0.5, 1.5, 2.0, 2.0, 12.0])
    # |new-old| / max(old, 2): 0.25, 0.25, 0, 0.5, 0.5
    assert orc.delta_cell(new, old) == pytest.approx(0.5)
    old = np.array([0.0, 0.0, 0.0, 3.0])               # lower median 0
    assert orc.delta_cell(np.array([0.0, 0.0, 0.0, 6.0]), old) == pytest.approx(1.0)
    assert math.isinf(orc.delta_cell(np.array([1e-30, 0.0, 0.0, 3.0]), old))
    assert orc.delta_cell(old, old) == 0.0
    # even count: lower median of (1, 2, 3, 4) is 2
    assert orc.delta_cell(np.array([1.0, 2.0, 3.0, 4.0]) + 1.0, np.array([1.0, 2.0, 3.0, 4.0])) == pytest.approx(0.5)


def test_delta_tot(orc):
    old = np.array([1.0, 2.0, 3.0])
    new = np.array([2.0, 2.0, 4.0])
    dv = np.array([1.0, 2.0, 3.0])
    a, b = (new * dv).sum(), (old * dv).sum()
    assert orc.delta_tot(new, old, dv) == pytest.approx(2 * (a - b) / (a + b))


@pytest.mark.slow
def test_stromgren_trend_with_opening_angle(orc):
    # Uniform gas around one source (16^3, Q = 1e48, n_H = 100): the converged
    # ionised volume approaches the Stromgren sphere as the opening angle
    # shrinks (the convergence claim of the paper, Sec. 6).  The front recedes
    # monotonically from the optically thin start: a cell once dark keeps
    # zeta_d = 2, so it is not re-ionised.
    P = W.small_uniform(16)
    dom = P.domains[0]
    dx = dom.finest_dx_cm()
    RS = (3 * 1e48 / (4 * math.pi * W.ALPHA_B * 1e4)) ** (1 / 3)
    out = {}
    for th in (0.5, 0.25):
        f, ion, it, dl = orc.solve(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], eps_lim=1e-3,
                                   max_iter=40, theta=th, zeta_g=False)
        out[th] = (3 * ion.sum() / (4 * math.pi)) ** (1 / 3) * dx / RS
    assert 0.8 < out[0.5] < 1.0
    assert abs(out[0.25] - 1) < abs(out[0.5] - 1)
