"""Pins of the oracle's finite-radius sources (paper Sec. 2.7: sources mapped
as uniform spheres): the volume of a ball cut by a box against closed forms
(whole ball, spherical cap, half and quarter balls, symmetric splits) and a
Monte Carlo estimate, and the deposit's conservation and symmetry."""
import math

import numpy as np
import pytest

from paper_2105_09644_amd import workloads as W


def vball(r):
    return 4.0 / 3.0 * math.pi * r ** 3


def cap(r, h):
    """volume of the part of a ball of radius r beyond a plane at distance h from its centre"""
    if h >= r:
        return 0.0
    if h <= -r:
        return vball(r)
    return math.pi * (r - h) ** 2 * (2 * r + h) / 3.0


BIG = 1e3


def test_whole_ball_and_caps(orc):
    c = (0.3, -0.2, 0.1)
    r = 0.7
    assert orc.ball_box_volume(c, r, [-BIG] * 3, [BIG] * 3) == pytest.approx(vball(r), rel=1e-13)
    for h in (-0.65, -0.3, 0.0, 0.25, 0.6, 0.69):
        for axis in range(3):
            lo = [-BIG] * 3
            lo[axis] = c[axis] + h
            assert orc.ball_box_volume(c, r, lo, [BIG] * 3) == pytest.approx(cap(r, h), rel=1e-12, abs=1e-15)
            hi = [BIG] * 3
            hi[axis] = c[axis] - h
            assert orc.ball_box_volume(c, r, [-BIG] * 3, hi) == pytest.approx(cap(r, h), rel=1e-12, abs=1e-15)


def test_symmetric_pieces(orc):
    r = 1.3
    c = (0.0, 0.0, 0.0)
    half = orc.ball_box_volume(c, r, [0, -BIG, -BIG], [BIG] * 3)
    quarter = orc.ball_box_volume(c, r, [0, 0, -BIG], [BIG] * 3)
    eighth = orc.ball_box_volume(c, r, [0, 0, 0], [BIG] * 3)
    assert half == pytest.approx(vball(r) / 2, rel=1e-13)
    assert quarter == pytest.approx(vball(r) / 4, rel=1e-13)
    assert eighth == pytest.approx(vball(r) / 8, rel=1e-13)
    # a slab through the centre, and its complement: the pieces add up
    s = orc.ball_box_volume(c, r, [-0.4, -BIG, -BIG], [0.9, BIG, BIG])
    assert s == pytest.approx(vball(r) - cap(r, 0.4) - cap(r, 0.9), rel=1e-12)


def test_tiling_adds_up_and_monte_carlo(orc):
    rng = np.random.default_rng(5)
    for _ in range(5):
        c = rng.uniform(2.0, 3.0, 3)
        r = rng.uniform(0.3, 1.9)
        tot = 0.0
        for i in range(6):
            for j in range(6):
                for k in range(6):
                    tot += orc.ball_box_volume(c, r, [i, j, k], [i + 1, j + 1, k + 1])
        assert tot == pytest.approx(vball(r), rel=1e-11)
    # one irregular box against Monte Carlo
    c = (0.1, 0.2, -0.1)
    r = 1.0
    lo, hi = np.array([-0.35, -0.8, -0.2]), np.array([0.55, 0.4, 1.3])
    v = orc.ball_box_volume(c, r, lo, hi)
    p = rng.uniform(lo, hi, (1_000_000, 3))
    mc = np.mean(np.sum((p - c) ** 2, axis=1) <= r * r) * np.prod(hi - lo)
    sig = np.prod(hi - lo) * math.sqrt(0.25 / 1e6)
    assert abs(v - mc) < 5 * sig


def test_sphere_deposit(orc):
    n = 16
    dom = W.uniform_domain(n)
    dx = dom.finest_dx_cm()
    # centred on a cell vertex with a radius below a cell: eight equal shares
    nd = orc.deposit(dom, [[8 * dx, 8 * dx, 8 * dx]], [8e48], radius_cm=0.6 * dx)
    idx = np.nonzero(nd)[0]
    assert len(idx) == 8 and np.allclose(nd[idx], 1e48, rtol=1e-12)
    # a larger sphere: the rate is conserved and follows the cell volumes
    xyz = np.array([[5.3 * dx, 7.9 * dx, 8.45 * dx]])
    nd = orc.deposit(dom, xyz, [1e49], radius_cm=2.2 * dx)
    assert nd.sum() == pytest.approx(1e49, rel=1e-13)
    lo, size = orc.cell_geometry(dom)
    for c in np.nonzero(nd)[0][:10]:
        v = orc.ball_box_volume(xyz[0] / dx, 2.2, lo[c], lo[c] + size[c])
        assert nd[c] == pytest.approx(1e49 * v / vball(2.2), rel=1e-11)
    # a sphere cut by the domain boundary keeps its whole rate inside
    nd = orc.deposit(dom, [[0.5 * dx, 3 * dx, 3 * dx]], [1e49], radius_cm=1.5 * dx)
    assert nd.sum() == pytest.approx(1e49, rel=1e-13)
    # AMR grid: conservation
    P = W.small_amr(2, seed=4)
    nd = orc.deposit(P.domains[0], P.src_xyz[0], P.src_q[0], radius_cm=1.3 * P.domains[0].finest_dx_cm())
    assert nd.sum() == pytest.approx(P.src_q[0].sum(), rel=1e-12)
