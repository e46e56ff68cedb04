"""Pins of the oracle's radial kernels and evaluation points (paper App. A, Sec. 2.2)."""
import math

import numpy as np
import pytest

from paper_2105_09644_amd import workloads as W

XE = math.sqrt(3) / 2


def test_wp_shape_constraints(orc):
    # W(0) = M, W'(0) = 0, continuous at 1/2 with value A, W(sqrt3/2) = 0 = W'(sqrt3/2)
    h = 1e-6
    assert orc.wp(0.0) == pytest.approx(1.184, abs=1e-15)
    assert (orc.wp(h) - orc.wp(0.0)) / h == pytest.approx(0.0, abs=1e-4)
    assert orc.wp(0.5 - 1e-12) == pytest.approx(0.408, abs=1e-9)
    assert orc.wp(0.5) == pytest.approx(0.408, abs=1e-12)
    assert orc.wp(XE - 1e-9) == pytest.approx(0.0, abs=1e-12)
    assert (orc.wp(XE - 1e-6) - orc.wp(XE - 2e-6)) / 1e-6 == pytest.approx(0.0, abs=1e-4)
    assert orc.wp(XE) == 0.0 and orc.wp(1.0) == 0.0
    xs = np.linspace(0, XE - 1e-9, 500)
    w = np.array([orc.wp(x) for x in xs])
    assert np.all(w > 0) and np.all(np.diff(w) < 0)   # positive and falling


def test_wp_matches_mean_cube_line_intersection(orc):
    # W_p was fitted to the mean cross-section of a uniform unit cube cut by
    # randomly oriented, randomly placed lines: the density of t = u.p for p
    # uniform in the cube and u uniform on the sphere (App. A.2).  This pins
    # the constants, including the printed A = 4.08 that must read 0.408.
    rng = np.random.default_rng(11)
    n = 4_000_000
    p = rng.uniform(-0.5, 0.5, size=(n, 3))
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    t = np.abs(np.einsum("ij,ij->i", p, u))
    hist, edges = np.histogram(t, bins=43, range=(0, XE))
    dens = hist / (n * np.diff(edges)) / 2.0        # density of the signed t
    mid = 0.5 * (edges[1:] + edges[:-1])
    w = np.array([orc.wp(x) for x in mid])
    assert np.max(np.abs(w - dens)) < 0.03
    # and the integral over the support is close to one
    xs = np.linspace(-XE, XE, 20001)
    assert np.trapezoid([orc.wp(x) for x in xs], xs) == pytest.approx(1.0, abs=0.01)


def test_wf3_conditions(orc):
    # eq. kernCond0 and the sum condition: u_i + u_{i+1} = 1,
    # u_i / r_i^2 + u_{i+1} / r_{i+1}^2 = 1 / d^2, u >= 0
    r = np.array([(i / 31.0) ** 2 * 55.4 for i in range(32)])
    rng = np.random.default_rng(5)
    for d in rng.uniform(r[1], r[-1] * 0.999, 2000):
        u = orc.wf3_weights(r, d)
        assert np.all(u >= 0)
        assert np.count_nonzero(u) <= 2
        assert u.sum() == pytest.approx(1.0, abs=1e-14)
        assert np.sum(u[1:] / r[1:] ** 2) == pytest.approx(1.0 / d ** 2, rel=1e-12)
    # beyond the last point everything goes there; before r_1, to r_1
    assert orc.wf3_weights(r, r[-1] * 1.5)[-1] == 1.0
    assert orc.wf3_weights(r, r[1] * 0.5)[1] == 1.0


def test_wp_weights(orc):
    r = np.array([(i / 31.0) ** 2 * 55.4 for i in range(32)])
    rng = np.random.default_rng(6)
    for _ in range(500):
        d = rng.uniform(0.5, 50)
        h = 2.0 ** rng.integers(0, 5)
        v = orc.wp_weights(r, d, h)
        assert v.sum() == pytest.approx(1.0, abs=1e-13)
        assert np.all(v >= 0)
        inside = np.abs(r - d) / h < XE
        if inside.any():
            assert np.all(v[~inside] == 0)
            ref = np.array([orc.wp((x - d) / h) for x in r])
            assert np.allclose(v, ref / ref.sum(), rtol=1e-13, atol=1e-16)
        else:   # linear split over the bracket
            i = np.searchsorted(r, d, side="right") - 1
            assert v[i] == pytest.approx((r[i + 1] - d) / (r[i + 1] - r[i]))


def test_radial_points(orc):
    # eq. (Nr): N_R = eta_R floor(sqrt(2 L_ray / dx)) + 1 with L_ray the 3-D diagonal
    for n, nr in [(32, 21), (48, 25), (64, 29), (96, 37), (128, 43)]:
        dom = W.uniform_domain(n)
        r = orc.radial_points(dom, W.Params(n_radial=0, eta_r=2.0))
        assert len(r) == nr
        dx = dom.finest_dx_cm()
        assert np.allclose(r, dx * np.arange(nr) ** 2 / 8.0, rtol=1e-14)
        assert r[-1] <= n * math.sqrt(3) * dx
    # prescribed count: quadratic spacing ending at L_ray
    dom = W.uniform_domain(32)
    r = orc.radial_points(dom, W.Params(n_radial=32))
    L = 32 * math.sqrt(3) * dom.finest_dx_cm()
    assert r[0] == 0 and r[-1] == pytest.approx(L, rel=1e-15)
    assert np.allclose(np.sqrt(r / L) * 31, np.arange(32), atol=1e-9)
