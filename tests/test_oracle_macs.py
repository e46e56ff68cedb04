"""Pins of the oracle's IF MAC and Src MAC (paper Sec. 2.4).

The ionised mass of a node, the emitting nodes and the tiling of the domain
by the accepted nodes are rebuilt here by brute force from the cells."""
import numpy as np
import pytest

from paper_2105_09644_amd import workloads as W

DIF = 1e-8   # delta_IF of Sec. 2.4


def cell_mass_ion(orc, P, f_prev):
    dom = P.domains[0]
    lo, size = orc.cell_geometry(dom)
    dv = (size * dom.finest_dx_cm()) ** 3
    m = P.n_h[0] * dv
    return lo, size, m, np.where(f_prev > 0, m, 0.0)


def painted_sums(lo, size, values, node_lo, node_size):
    inside = np.all((lo >= node_lo) & (lo + size[:, None] <= node_lo + node_size), axis=1)
    return values[inside].sum(), inside


def test_equal_angles_change_nothing(orc):
    P = W.small_lognormal(16, n_src=3, seed=21)
    dom = P.domains[0]
    f0, _, _ = orc.sweep(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], alpha_b=0.0)
    a, _, st_a = orc.sweep(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], f_prev=f0)
    b, _, st_b = orc.sweep(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], f_prev=f0,
                           theta_if=P.params.theta, theta_src=P.params.theta)
    assert np.array_equal(a, b)
    assert st_a.nodes_accepted == st_b.nodes_accepted


def test_src_mac_resolves_emission_to_cells(orc):
    # optically thin: the flux is sum eps_n / (4 pi d_n^2) over accepted nodes, so
    # opening every emitting node down to its cells reproduces theta = 0 exactly
    P = W.small_lognormal(16, n_src=3, seed=22)
    dom = P.domains[0]
    args = (dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0])
    f_src, _, st_src = orc.sweep(*args, alpha_b=0.0, theta_src=1e-6)
    f_all, _, st_all = orc.sweep(*args, alpha_b=0.0, theta=0.0)
    f_bh, _, st_bh = orc.sweep(*args, alpha_b=0.0)
    sel = f_all > 1e-6 * f_all.max()
    assert np.max(np.abs(f_src[sel] - f_all[sel]) / f_all[sel]) < 1e-12
    assert np.max(np.abs(f_bh[sel] - f_all[sel]) / f_all[sel]) > 1e-6   # the plain walk differs
    assert st_bh.nodes_accepted < st_src.nodes_accepted < st_all.nodes_accepted
    # no accepted node above cell size holds emission
    for t in (0, 1234, 4095):
        ls, mom = orc.accepted(*args, t, theta_src=1e-6)
        leaf = np.array([orc_is_leaf(ls[q], dom) for q in range(len(ls))])
        assert np.all(mom[~leaf, 0] == 0)


def orc_is_leaf(row, dom):
    return row[3] == 1   # uniform grids: every leaf cell has size 1


def test_if_mac_opens_front_nodes(orc):
    P = W.small_lognormal(16, n_src=2, seed=23)
    dom = P.domains[0]
    args = (dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0])
    # previous flux with an ionisation front: the absorbing sweep after the thin one
    f0, _, _ = orc.sweep(*args, alpha_b=0.0)
    f1, _, _ = orc.sweep(*args, f_prev=f0)
    assert 0 < np.count_nonzero(f1 > 0) < len(f1)
    lo, size, m, mion = cell_mass_ion(orc, P, f1)
    ext = dom.extent_finest()
    n_if_open = 0
    for t in (0, 777, 2048, 4000):
        ls_bh, mom_bh = orc.accepted(*args, t, f_prev=f1)
        ls, mom = orc.accepted(*args, t, f_prev=f1, theta_if=1e-6)
        # the accepted nodes and the target tile the domain
        vol = np.sum(ls[:, 3].astype(np.float64) ** 3) + 1
        assert vol == ext[0] * ext[1] * ext[2]
        for q in range(len(ls)):
            tm, _ = painted_sums(lo, size, m, ls[q, :3], ls[q, 3])
            ti, _ = painted_sums(lo, size, mion, ls[q, :3], ls[q, 3])
            assert mom[q, 4] == pytest.approx(tm, rel=1e-12)
            assert mom[q, 8] == pytest.approx(ti, rel=1e-12, abs=0.0)
            if ls[q, 3] > 1:   # a node above cell size never straddles the front
                assert not (DIF * tm < ti < (1 - DIF) * tm)
        # the plain walk does accept front nodes here, which the IF MAC opened
        front = [(DIF * mom_bh[q, 4] < mom_bh[q, 8] < (1 - DIF) * mom_bh[q, 4]) and ls_bh[q, 3] > 1
                 for q in range(len(ls_bh))]
        n_if_open += sum(front)
        assert len(ls) >= len(ls_bh)
    assert n_if_open > 0


def test_if_mac_without_previous_flux_is_plain(orc):
    # no ionised gas in the thin first sweep: no node holds a front
    P = W.small_lognormal(16, n_src=2, seed=24)
    dom = P.domains[0]
    args = (dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0])
    a, _, st_a = orc.sweep(*args, alpha_b=0.0)
    b, _, st_b = orc.sweep(*args, alpha_b=0.0, theta_if=1e-6)
    assert np.array_equal(a, b) and st_a.nodes_accepted == st_b.nodes_accepted
