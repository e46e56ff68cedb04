"""Pins of the oracle's source deposit, octree, node moments and tree walk
(paper Sec. 2.1, 2.3, 2.4, 2.7).

Independent references are built here in numpy from the inputs alone: cell
centres of a uniform grid, painted occupancy grids, brute-force sums over all
cells.
"""
import math

import numpy as np
import pytest

from paper_2105_09644_amd import workloads as W

FOURPI = 4 * math.pi


def centres_uniform(n, dx):
    a = (np.arange(n) + 0.5) * dx
    x, y, z = np.meshgrid(a, a, a, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def test_deposit(orc):
    n = 16
    dom = W.uniform_domain(n)
    dx = dom.finest_dx_cm()
    box = n * dx
    # centre of the box: a vertex shared by 8 cells
    nd = orc.deposit(dom, [[box / 2] * 3], [8e48])
    idx = np.nonzero(nd)[0]
    assert len(idx) == 8 and np.allclose(nd[idx], 1e48, rtol=1e-15)
    ijk = np.stack(np.unravel_index(idx, (n, n, n)), 1)
    assert set(map(tuple, ijk)) == {(i, j, k) for i in (7, 8) for j in (7, 8) for k in (7, 8)}
    # inside a cell, on a face, on an edge
    for pos, m in [([3.3, 4.6, 5.1], 1), ([3.0, 4.6, 5.1], 2), ([3.0, 4.0, 5.1], 4)]:
        nd = orc.deposit(dom, [[p * dx for p in pos]], [1e47])
        assert np.count_nonzero(nd) == m
        assert nd.sum() == pytest.approx(1e47, rel=1e-15)
    # several sources: the totals add up
    rng = np.random.default_rng(1)
    xyz = rng.uniform(0, box, (50, 3))
    q = 10 ** rng.uniform(46, 49, 50)
    assert orc.deposit(dom, xyz, q).sum() == pytest.approx(q.sum(), rel=1e-13)


def test_deposit_amr(orc):
    P = W.small_amr(2, seed=1)
    dom = P.domains[0]
    nd = orc.deposit(dom, P.src_xyz[0], P.src_q[0])
    assert nd.sum() == pytest.approx(P.src_q[0].sum(), rel=1e-13)


def paint(ext, nodes):
    g = np.zeros(ext, np.int32)
    for lo0, lo1, lo2, s in nodes:
        g[lo0:lo0 + s, lo1:lo1 + s, lo2:lo2 + s] += 1
    return g


@pytest.mark.parametrize("case", ["uniform16", "padded24", "amr"])
def test_accepted_nodes_tile_the_domain(orc, case):
    if case == "uniform16":
        P = W.small_uniform(16)
    elif case == "padded24":
        P = W.small_lognormal(24, seed=2)
    else:
        P = W.small_amr(2, seed=3)
    dom = P.domains[0]
    lo, sz = orc.cell_geometry(dom)
    ext = dom.extent_finest()
    rng = np.random.default_rng(4)
    for t in list(rng.choice(len(sz), 6, replace=False)) + [0, len(sz) - 1]:
        ls, mom = orc.accepted(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], int(t))
        g = paint(ext, list(map(tuple, ls)) + [(*lo[t], sz[t])])
        assert np.all(g == 1), "accepted nodes plus the target must cover every cell once"


def test_theta_zero_accepts_every_other_cell(orc):
    P = W.small_lognormal(16, seed=5)
    dom = P.domains[0]
    ls, mom = orc.accepted(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], 100, theta=0.0)
    assert len(ls) == 16 ** 3 - 1
    assert np.all(ls[:, 3] == 1)


def test_opening_angle_counts(orc):
    # regression against an independent count of accepted nodes for the
    # central target of a 32^3 grid (777) and a corner (161) at theta = 0.5
    P = W.small_uniform(32)
    dom = P.domains[0]
    t = 16 * 32 * 32 + 16 * 32 + 16
    assert len(orc.accepted(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], t)[0]) == 777
    assert len(orc.accepted(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], 0)[0]) == 161


def test_node_moments_are_sums_over_their_cells(orc):
    P = W.small_lognormal(16, n_src=4, seed=6)
    dom = P.domains[0]
    dx = dom.finest_dx_cm()
    n_h = P.n_h[0]
    lo, sz = orc.cell_geometry(dom)
    ndot = orc.deposit(dom, P.src_xyz[0], P.src_q[0])
    dv = (sz * dx) ** 3
    s = ndot - W.ALPHA_B * n_h ** 2 * dv
    eps_c, alp_c, m_c = np.maximum(s, 0), np.maximum(-s, 0), n_h * dv
    fprev = np.random.default_rng(1).uniform(0, 1e9, len(sz))
    ctr = lo + 0.5 * sz[:, None]
    for t in (0, 777, 2000):
        ls, mom = orc.accepted(dom, P.params, n_h, P.src_xyz[0], P.src_q[0], t, f_prev=fprev, theta=2.0)
        for (x0, y0, z0, h), mm in zip(ls, mom):
            inn = ((lo[:, 0] >= x0) & (lo[:, 0] < x0 + h) & (lo[:, 1] >= y0) & (lo[:, 1] < y0 + h) &
                   (lo[:, 2] >= z0) & (lo[:, 2] < z0 + h))
            assert mm[0] == pytest.approx(eps_c[inn].sum(), rel=1e-12, abs=1e-300)
            assert mm[1] == pytest.approx(alp_c[inn].sum(), rel=1e-12)
            assert mm[2] == pytest.approx((fprev * dv)[inn].sum(), rel=1e-12)
            assert mm[3] == pytest.approx(dv[inn].sum(), rel=1e-14)
            assert mm[4] == pytest.approx(m_c[inn].sum(), rel=1e-12)
            com = (m_c[inn, None] * ctr[inn]).sum(0) / m_c[inn].sum()
            assert np.allclose(mm[5:8], com, rtol=1e-12)


def test_thin_theta_zero_equals_direct_sum(orc):
    # theta = 0 opens the tree down to the cells; with alpha_B = 0 the flux at
    # a target is the sum of eps_c / (4 pi d_c^2) over all other cells plus
    # the centre flux of its own emission, 3 eps_t / (4 pi r_tp^2).
    n = 16
    P = W.small_uniform(n, q=1e48)
    dom = P.domains[0]
    dx = dom.finest_dx_cm()
    xyz = np.vstack([P.src_xyz[0], [[3.3 * dx, 11.6 * dx, 5.2 * dx]]])
    q = np.array([8e48, 3e47])
    ndot = orc.deposit(dom, xyz, q)
    ctr = centres_uniform(n, dx)
    rng = np.random.default_rng(8)
    tg = np.concatenate([rng.choice(n ** 3, 40, replace=False), np.nonzero(ndot)[0]])
    f, ion, st = orc.sweep(dom, P.params, P.n_h[0], xyz, q, targets=tg, alpha_b=0.0, theta=0.0)
    for t, ft in zip(tg, f):
        d2 = np.sum((ctr - ctr[t]) ** 2, axis=1)
        d2[t] = np.inf
        ref = np.sum(ndot / (FOURPI * d2)) + 3 * ndot[t] / (FOURPI * (0.5 * dx) ** 2)
        assert ft == pytest.approx(ref, rel=1e-12)


def test_thin_flux_of_point_source(orc):
    # theta = 0, one point source inside a cell: F -> Q / (4 pi r^2) up to the
    # O((dx/r)^2) offset between the source and its cell centre
    n = 16
    P = W.small_uniform(n)
    dom = P.domains[0]
    dx = dom.finest_dx_cm()
    src = np.array([[8.5 * dx, 8.5 * dx, 8.5 * dx]])
    ctr = centres_uniform(n, dx)
    tg = np.arange(0, n ** 3, 97)
    f, ion, st = orc.sweep(dom, P.params, P.n_h[0], src, [1e48], targets=tg, alpha_b=0.0, theta=0.0)
    r = np.linalg.norm(ctr[tg] - src[0], axis=1)
    far = r > 4 * dx
    rel = f[far] / (1e48 / (FOURPI * r[far] ** 2)) - 1
    assert np.all(np.abs(rel) < 1e-12)   # the source sits at a cell centre here


@pytest.mark.parametrize("case", ["lognormal16", "padded24", "amr"])
def test_thin_flux_equals_sum_over_accepted_nodes(orc, case):
    # flux conservation of W_f,3 and unit angular weights: with alpha_B = 0,
    # F = sum over accepted nodes of eps_n / (4 pi d_n^2) + F_self exactly
    if case == "lognormal16":
        P = W.small_lognormal(16, n_src=5, seed=9)
    elif case == "padded24":
        P = W.small_lognormal(24, n_src=3, seed=10)
    else:
        P = W.small_amr(2, seed=11)
    dom = P.domains[0]
    dx = dom.finest_dx_cm()
    lo, sz = orc.cell_geometry(dom)
    ndot = orc.deposit(dom, P.src_xyz[0], P.src_q[0])
    r = orc.radial_points(dom, P.params)
    rng = np.random.default_rng(12)
    tg = np.concatenate([rng.choice(len(sz), 10, replace=False), np.nonzero(ndot)[0][:3]])
    f, ion, st = orc.sweep(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], targets=tg, alpha_b=0.0)
    for t, ft in zip(tg, f):
        ls, mom = orc.accepted(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], int(t), alpha_b=0.0)
        xt = lo[t] + 0.5 * sz[t]
        d = np.linalg.norm(mom[:, 5:8] - xt, axis=1) * dx
        e = mom[:, 0] > 0
        assert np.all((d[e] >= r[1]) & (d[e] < r[-1]))
        ref = np.sum(mom[e, 0] / (FOURPI * d[e] ** 2)) + 3 * ndot[t] / (FOURPI * (0.5 * sz[t] * dx) ** 2)
        assert ft == pytest.approx(ref, rel=1e-12)
