"""Pins of the emission and smoothing kernel variants of the paper's App. A:
the flux-conserving W_f,1, W_f,2, W_f,3 (two-point and N-point) by their
defining conditions, W_g by its shape, and the thin sweep's flux
conservation for the flux-conserving kernels."""
import math

import numpy as np
import pytest

from paper_2105_09644_amd import workloads as W

R = np.array([i * i / 8.0 for i in range(30)])   # eq. etaR with eta_R = 2, unit cell


@pytest.mark.parametrize("d", [1.3, 2.05, 5.5, 17.2, 60.0, 107.9])
def test_two_point_flux_kernels(orc, d):
    i = np.searchsorted(R, d, side="right") - 1
    if d >= R[-1] or d < R[1]:   # the W_f,3 fall-backs: everything on one point
        for kind in (orc.K_F1, orc.K_F2):
            assert np.array_equal(orc.eps_weights(kind, R, d, 1.0), orc.eps_weights(orc.K_F3, R, d, 1.0))
        return
    u1 = orc.eps_weights(orc.K_F1, R, d, 1.0)
    nz = np.nonzero(u1)[0]
    assert set(nz) <= {i, i + 1}
    assert np.sum(u1[nz] / R[nz] ** 2) == pytest.approx(1 / d ** 2, rel=1e-13)
    if len(nz) == 2:
        assert u1[i + 1] / u1[i] == pytest.approx((d - R[i]) / (R[i + 1] - d), rel=1e-12)
    u2 = orc.eps_weights(orc.K_F2, R, d, 1.0)
    nz2 = np.nonzero(u2)[0]
    assert np.sum(u2[nz2] / R[nz2] ** 2) == pytest.approx(1 / d ** 2, rel=1e-12)
    if i >= 2 and not np.allclose(u2, orc.eps_weights(orc.K_F3, R, d, 1.0)):
        p = R[i - 1]   # the flux is also exact at r_{i-1}
        assert np.sum(u2[nz2] / (R[nz2] - p) ** 2) == pytest.approx(1 / (d - p) ** 2, rel=1e-10)
    assert np.array_equal(orc.eps_weights(orc.K_F3, R, d, 1.0), orc.eps_weights(orc.K_DEFAULT, R, d, 1.0))


@pytest.mark.parametrize("d,h", [(12.3, 4.0), (30.0, 16.0), (55.5, 8.0), (3.3, 2.0)])
def test_n_point_flux_kernel(orc, d, h):
    u = orc.eps_weights(orc.K_F3N, R, d, h)
    nz = np.nonzero(u)[0]
    assert np.all(u >= 0)
    assert u.sum() == pytest.approx(1.0, rel=1e-13)
    assert np.sum(u[nz] / R[nz] ** 2) == pytest.approx(1 / d ** 2, rel=1e-12)
    span = [k for k in range(1, len(R)) if abs(R[k] - d) < math.sqrt(3) / 2 * h]
    if len(nz) > 2:   # the N-point form: linear in the point index over the node's extent
        assert list(nz) == span
        assert np.allclose(np.diff(u[nz], 2), 0.0, atol=1e-14)


def test_gaussian_kernel(orc):
    assert orc.wg(0.0) == 1.0
    assert orc.wg(0.5) == pytest.approx(math.exp(-0.25), rel=1e-15)
    assert orc.wg(0.87) == 0.0 and orc.wg(-0.3) == orc.wg(0.3)
    v = orc.mass_weights(orc.K_G, R, 20.0, 6.0)
    assert v.sum() == pytest.approx(1.0, rel=1e-14)
    x = (R - 20.0) / 6.0
    ref = np.where(np.abs(x) < math.sqrt(3) / 2, np.exp(-x * x), 0.0)
    assert np.allclose(v, ref / ref.sum(), rtol=1e-13, atol=0)
    assert np.array_equal(orc.mass_weights(orc.K_P, R, 20.0, 6.0), orc.wp_weights(R, 20.0, 6.0))


@pytest.mark.parametrize("kind", [1, 2, 4])
def test_thin_flux_conserved_by_flux_kernels(orc, kind):
    # thin limit: F = sum over accepted nodes of eps_n / (4 pi d_n^2) for every kernel
    # that satisfies eq. kernCond0 (the W_f family), plus the self term
    P = W.small_lognormal(16, n_src=3, seed=31)
    dom = P.domains[0]
    dx = dom.finest_dx_cm()
    args = (dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0])
    f, _, _ = orc.sweep(*args, alpha_b=0.0, eps_kernel=kind)
    nd = orc.deposit(dom, P.src_xyz[0], P.src_q[0])
    lo, size = orc.cell_geometry(dom)
    checked = 0
    for t in (0, 1111, 2222, 4095, 3000, 500):
        ls, mom = orc.accepted(*args, t, alpha_b=0.0)
        xt = (lo[t] + 0.5 * size[t]).astype(float)
        d = np.linalg.norm(mom[:, 5:8] - xt, axis=1) * dx
        # nodes closer than r_1 or beyond the last point are not flux-exact: skip targets that have them
        r = orc.radial_points(dom, P.params)
        em = mom[:, 0] > 0
        if np.any(d[em] < r[1]) or np.any(d[em] >= r[-1]):
            continue
        expect = np.sum(mom[em, 0] / (4 * math.pi * d[em] ** 2))
        rtp = 0.5 * size[t] * dx
        expect += 3 * nd[t] / (4 * math.pi * rtp ** 2)
        assert f[t] == pytest.approx(expect, rel=1e-11)
        checked += 1
    assert checked >= 3
