"""Pins of the oracle's periodic boundaries (paper Sec. 2.8: each node is used
through its periodic copy closest to the target)."""
import math

import numpy as np
import pytest

from paper_2105_09644_amd import workloads as W


def test_theta0_thin_flux_uses_nearest_copies(orc):
    # theta = 0: every other cell is its own node; in the thin limit the flux is
    # the sum over emitting cells of eps / (4 pi d^2) with d the distance to the
    # nearest periodic copy, plus the self term
    n = 16
    P = W.small_lognormal(n, n_src=3, seed=41)
    dom = P.domains[0]
    dx = dom.finest_dx_cm()
    nd = orc.deposit(dom, P.src_xyz[0], P.src_q[0])
    tg = np.array([0, 7, 255, 1000, 2047, 4095])
    f, _, _ = orc.sweep(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], targets=tg, alpha_b=0.0, theta=0.0,
                        periodic=True)
    f_iso, _, _ = orc.sweep(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], targets=tg, alpha_b=0.0,
                            theta=0.0)
    ijk = np.stack(np.unravel_index(np.arange(n ** 3), (n, n, n)), 1).astype(float)
    em = np.nonzero(nd)[0]
    r = orc.radial_points(dom, P.params)
    changed = 0
    for t, ft, fi in zip(tg, f, f_iso):
        off = ijk[em] - ijk[t]
        off = off + n * np.floor((0.5 * n - off) / n)
        d = np.linalg.norm(off, axis=1) * dx
        keep = d > 0
        assert np.all((d[keep] >= r[1]) & (d[keep] < r[-1]))
        ref = np.sum(nd[em][keep] / (4 * math.pi * d[keep] ** 2)) + 3 * nd[t] / (4 * math.pi * (0.5 * dx) ** 2)
        assert ft == pytest.approx(ref, rel=1e-12)
        changed += abs(ft - fi) > 1e-6 * fi
    assert changed > 0   # the copies matter for some targets


def test_half_period_translation(orc):
    # rolling the gas and the sources by half the period maps every node below
    # the root's children onto a node: the absorbing flux rolls with them
    n = 16
    P = W.small_lognormal(n, n_src=3, seed=42)
    dom = P.domains[0]
    L = n * dom.finest_dx_cm()
    f0, _, _ = orc.sweep(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], alpha_b=0.0, periodic=True)
    a, _, _ = orc.sweep(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], f_prev=f0, periodic=True)
    nh = np.roll(P.n_h[0].reshape(n, n, n), n // 2, axis=0).ravel()
    xyz = P.src_xyz[0].copy()
    xyz[:, 0] = np.mod(xyz[:, 0] + 0.5 * L, L)
    g0 = np.roll(f0.reshape(n, n, n), n // 2, axis=0).ravel()
    b, _, _ = orc.sweep(dom, P.params, nh, xyz, P.src_q[0], f_prev=g0, periodic=True)
    b = np.roll(b.reshape(n, n, n), -(n // 2), axis=0).ravel()
    sel = a > 1e-6 * a.max()
    assert np.max(np.abs(a[sel] - b[sel]) / a[sel]) < 1e-12
    assert np.array_equal(a > 0, b > 0)
