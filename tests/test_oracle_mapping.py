"""Pins of the oracle's node -> ray mapping (paper Sec. 2.3 "Mapping nodes onto
rays", App. A) through the ray buffers of single targets and the angular
weights of single nodes.

The expected values come from the inputs alone: cell totals summed in numpy,
the medium's own per-volume rates, the HEALPix pixel of a single direction
(pinned in test_oracle_healpix.py), and Monte Carlo volume fractions of a box
inside each HEALPix cone.
"""
import math

import numpy as np
import pytest

from paper_2105_09644_amd import workloads as W


def cell_totals(orc, P, f_prev):
    """Per-cell emission, recombination, radiation and volume totals of the
    first domain from the inputs (eqs. os:ems, os:abs, os:erd with the
    per-cell netting of the emission and recombination)."""
    dom = P.domains[0]
    lo, size = W.cell_lo_size(dom)
    dv = (size * dom.finest_dx_cm()) ** 3
    ndot = orc.deposit(dom, P.src_xyz[0], P.src_q[0])
    s = ndot - P.params.alpha_b * P.n_h[0] ** 2 * dv
    return np.maximum(s, 0.0), np.maximum(-s, 0.0), f_prev * dv, dv


@pytest.mark.parametrize("make", [lambda: W.small_lognormal(16, n_src=3, seed=5),
                                  lambda: W.small_lognormal(24, n_src=2, seed=6, nside=1),
                                  lambda: W.small_amr(2, seed=7)])
def test_ray_buffers_conserve_cell_totals(orc, make):
    """Every cell enters a target's ray buffers exactly once, either inside an
    accepted node or as the target's own self term, and the angular and
    radial weights of each node sum to one: the buffer totals of eps, A, E and
    V are the domain's cell totals (uniform, padded and adaptive grids)."""
    P = make()
    dom = P.domains[0]
    n = dom.n_cells()
    rng = np.random.default_rng(11)
    f_prev = 1e9 * np.exp(rng.standard_normal(n))
    eps, alpha, erad, dv = cell_totals(orc, P, f_prev)
    for t in rng.choice(n, 4, replace=False):
        b = orc.target_rays(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], int(t), f_prev=f_prev)
        for got, want, name in zip(b, (eps.sum(), alpha.sum(), erad.sum(), dv.sum()), "eps A E V".split()):
            assert got.sum() == pytest.approx(want, rel=1e-12), f"target {t}: {name}"
        assert np.all(b[3] >= 0) and np.all(b[1] >= 0)


def test_uniform_medium_per_volume_values_are_exact(orc):
    """In a medium of uniform density and uniform previous flux without sources
    every node's recombination and radiation are the same multiples of its
    volume, so A_i/V_i and E_i/V_i must equal the medium's values at every
    point of every ray, whichever support each quantity is spread over."""
    n = 16
    P = W.small_uniform(n, q=0.0)
    dom = P.domains[0]
    fbar = 3.7e10
    f_prev = np.full(n ** 3, fbar)
    alpha_pv = P.params.alpha_b * 100.0 ** 2
    for t in (0, 7 * n * n + 7 * n + 7, 3 * n * n + 15 * n + 9):
        eps, A, E, V = orc.target_rays(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], t, f_prev=f_prev)
        assert np.all(eps == 0)
        m = V > 0
        assert m.sum() > 0.25 * V.size
        assert np.all(np.abs(A[m] / V[m] - alpha_pv) <= 1e-12 * alpha_pv)
        assert np.all(np.abs(E[m] / V[m] - fbar) <= 1e-12 * fbar)
        assert np.all(A[~m] == 0) and np.all(E[~m] == 0)


def test_innermost_point_holds_only_the_target(orc):
    """At theta 0.5 no node other than the target reaches r_0 = 0 with its
    W_p support (accepted neighbours lie at d >= h); so every ray's volume at
    r_0 is the target's volume times the W_p weight of d = 0, shared equally
    by the N_PIX rays (the self term)."""
    P = W.small_lognormal(16, n_src=2, seed=8)
    dom = P.domains[0]
    dx = dom.finest_dx_cm()
    r = orc.radial_points(dom, P.params)
    wself = orc.wp_weights(r, 0.0, dx)
    npix = 12 * P.params.nside ** 2
    for t in (0, 1000, 2345):
        _, A, _, V = orc.target_rays(dom, P.params, P.n_h[0], P.src_xyz[0], P.src_q[0], t)
        assert np.allclose(V[:, 0], dx ** 3 * wself[0] / npix, rtol=1e-13, atol=0)


@pytest.mark.parametrize("nside", [1, 2, 4, 8])
def test_far_tiny_node_falls_in_one_pixel(orc, nside):
    """A node far from the target compared with its size, whose direction is
    away from every pixel edge, puts all its sub-points in the pixel of its
    centre's direction: w_k = delta(k, pix(g_n - x_t))."""
    rng = np.random.default_rng(nside)
    done = 0
    while done < 40:
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        size = int(rng.choice([1, 2, 4, 8]))
        ext = np.array([size, size, size]) if done % 2 == 0 else rng.integers(1, size + 1, 3)
        xt = rng.integers(-50, 50, 3) + 0.5
        lo = np.floor(xt + 2e5 * u).astype(np.int64)
        hi = lo + ext
        # away from edges: every corner of the box and its centre in the same pixel
        corners = np.array([[lo[0] if i == 0 else hi[0], lo[1] if j == 0 else hi[1], lo[2] if k == 0 else hi[2]]
                            for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=np.float64) - xt
        g = 0.5 * (lo + hi) - xt
        pix = orc.ang2pix(nside, np.vstack([corners, g]))
        if np.any(pix != pix[-1]):
            continue
        w = orc.node_pixels(nside, 4, lo, hi, xt)
        assert w == {int(pix[-1]): 64}
        done += 1


@pytest.mark.parametrize("lo,hi,nside", [((3, -2, 1), (7, 1, 3), 2),        # a box beside the target
                                         ((-5, -5, 2), (5, 4, 4), 1),       # a slab over it
                                         ((2, 2, 2), (3, 3, 3), 4)])        # one cell off the diagonal
def test_angular_weights_tend_to_cone_volume_fractions(orc, lo, hi, nside):
    """As the sub-point lattice is refined the angular weights of a box tend to
    the fraction of its volume inside each HEALPix cone from the target
    (Monte Carlo over the box with 2e6 uniform points); at s = 4 they are
    within the lattice's resolution of it."""
    xt = np.array([0.5, 0.5, 0.5])
    lo, hi = np.array(lo, np.int64), np.array(hi, np.int64)
    rng = np.random.default_rng(3)
    pts = lo + (hi - lo) * rng.random((2_000_000, 3)) - xt
    pix = orc.ang2pix(nside, pts)
    npix = 12 * nside ** 2
    mc = np.bincount(pix, minlength=npix) / len(pix)
    err = {}
    for s in (4, 16, 48):
        w = orc.node_pixels(nside, s, lo, hi, xt)
        ws = np.zeros(npix)
        for k, c in w.items():
            ws[k] = c / s ** 3
        assert ws.sum() == pytest.approx(1.0, abs=1e-15)
        err[s] = np.abs(ws - mc).max()
    assert err[48] < 0.006          # Monte Carlo noise ~ 3.5e-4 per pixel, lattice ~ 1/48
    assert err[16] < 0.03
    assert err[4] < 0.12
    assert err[48] < err[4]


def test_angular_weights_depend_on_the_offset_alone(orc):
    """A node's sub-point directions are taken from its exact integer offset to
    the target (plus the sub-box fraction), so its angular weights are the
    same wherever the pair sits in the domain and at any power-of-two cell
    size: the property that lets the sweep tabulate them by offset."""
    rng = np.random.default_rng(17)
    for nside in (2, 4):
        for _ in range(200):
            size = int(rng.choice([1, 2, 4]))
            xt = rng.integers(-6, 6, 3) + 0.5
            lo = rng.integers(-14, 14, 3)
            hi = lo + size
            w = orc.node_pixels(nside, 4, lo, hi, xt)
            shift = rng.integers(-10 ** 6, 10 ** 6, 3)
            assert orc.node_pixels(nside, 4, lo + shift, hi + shift, xt + shift) == w
            k = int(rng.choice([2, 4, 8]))
            assert orc.node_pixels(nside, 4, lo * k, hi * k, xt * k) == w
