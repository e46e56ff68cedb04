"""The absorbing sweep of the oracle against a long-characteristics brute force.

One point source in uniform hydrogen: along the straight line from the source
to a target, the On-the-Spot photon rate per steradian falls from the
source's (netted) emission over 4 pi by the recombinations in the cone of that
line, alpha_B n^2 s^2 ds at distance s from the source, so

    Phi(r) = eps_src / (4 pi) - alpha_B sum_c n_c^2 (s_out^3 - s_in^3) / 3

over the cells c the line crosses (entry and exit distances s_in, s_out), and
the flux at the target is max(Phi(r), 0) / r^2.  The integral is exact cell by
cell here; nothing of the tree, the rays or the radial kernels is used.

TreeRay approximates this (paper Sec. 2.5; its summary states convergence to
long characteristics with angular resolution).  One absorbing sweep fed with
the brute-force flux as previous flux (so that zeta_d of eq. Rcorr:d is close
to one, as at convergence) must approach it as theta_lim falls, as N_side
grows and as the radial resolution eta_R (eq. etaR) grows.  On this 16^3 grid
the source cell subtends several pixels beyond N_side 4, which splits its
photons over several cones, each against the full recombination column, so
the N_side trend is taken up to 4.
"""
import math

import numpy as np
import pytest

from paper_2105_09644_amd import workloads as W

pytestmark = pytest.mark.slow

N = 16
Q = 1e48                                  # Stroemgren radius about 5.8 cells at n_H = 100
SRC = np.array([7.5, 7.5, 7.5])           # a cell centre: the whole rate goes to one cell


def long_characteristics(n, dx_cm, nh, src, q, alpha):
    nh3 = nh.reshape(n, n, n)
    isrc = tuple(int(v) for v in np.floor(src))
    eps0 = q - alpha * nh3[isrc] ** 2 * dx_cm ** 3      # the source cell's own recombinations are netted
    out = np.full(n ** 3, np.nan)
    for idx, (i, j, k) in enumerate(np.ndindex(n, n, n)):
        xt = np.array([i, j, k]) + 0.5
        dvec = xt - src
        r = float(np.linalg.norm(dvec))
        if r == 0.0:
            continue
        ts = [0.0, 1.0]
        for a in range(3):
            if dvec[a] != 0.0:
                lo, hi = sorted((src[a], xt[a]))
                ts += [(p - src[a]) / dvec[a] for p in range(int(math.floor(lo)) + 1, int(math.ceil(hi)))]
        ts = np.unique(np.clip(ts, 0.0, 1.0))
        loss = 0.0
        for t0, t1 in zip(ts[:-1], ts[1:]):
            c = tuple(int(v) for v in np.floor(src + 0.5 * (t0 + t1) * dvec))
            if c == isrc:
                continue
            s0, s1 = t0 * r * dx_cm, t1 * r * dx_cm
            loss += alpha * nh3[c] ** 2 * (s1 ** 3 - s0 ** 3) / 3.0
        out[idx] = max(eps0 / (4.0 * math.pi) - loss, 0.0) / (r * dx_cm) ** 2
    return out


@pytest.fixture(scope="module")
def setup():
    P = W.small_uniform(N, q=Q)
    dom = P.domains[0]
    dx = dom.finest_dx_cm()
    xyz = (SRC * dx)[None, :]
    flc = long_characteristics(N, dx, P.n_h[0], SRC, Q, P.params.alpha_b)
    src_cell = int(np.ravel_multi_index(tuple(int(v) for v in SRC), (N, N, N)))
    return P, xyz, flc, src_cell


_cache = {}


def median_error(orc, setup, **kw):
    key = tuple(sorted(kw.items()))
    if key not in _cache:
        _cache[key] = _median_error(orc, setup, **kw)
    return _cache[key]


def _median_error(orc, setup, **kw):
    P, xyz, flc, src_cell = setup
    f_prev = np.nan_to_num(flc)
    f, ion, _ = orc.sweep(P.domains[0], P.params, P.n_h[0], xyz, np.array([Q]), f_prev=f_prev, n_radial=0, **kw)
    both = (f_prev > 0) & (f > 0)
    both[src_cell] = False
    rel = np.abs(f[both] - f_prev[both]) / f_prev[both]
    lit_or = int(np.count_nonzero(f > 0))
    return float(np.median(rel)), lit_or


def test_brute_force_is_the_stroemgren_profile(setup):
    """The brute force itself.  Along a grid axis through the source the line
    stays in one row of cells, so the flux is the closed form of a uniform
    Stroemgren sphere at its first instant (Sec. 3.1, eq. erSpitzer at t = 0),
    (Q/(4 pi r^2)) (1 - r^3/R_S^3), with the source cell's recombinations netted
    from its emission instead of integrated: r^3 -> r^3 + (3/(4 pi) - 1/8) dx^3.
    The lit volume is the Stroemgren sphere's to within a shell of one cell."""
    P, xyz, flc, src_cell = setup
    dx = P.domains[0].finest_dx_cm()
    rs = (3 * Q / (4 * math.pi * 100.0 ** 2 * P.params.alpha_b)) ** (1 / 3) / dx
    i0 = np.array([int(v) for v in SRC])
    for axis in range(3):
        for sign in (-1, 1):
            for m in range(1, 6):
                c = i0.copy()
                c[axis] += sign * m
                f = flc[np.ravel_multi_index(tuple(c), (N, N, N))]
                x = (m ** 3 + 3 / (4 * math.pi) - 1 / 8) / rs ** 3
                want = Q / (4 * math.pi * (m * dx) ** 2) * max(1.0 - x, 0.0)
                assert f == pytest.approx(want, rel=1e-11, abs=1e-30)
    lit = np.count_nonzero(np.nan_to_num(flc) > 0) + 1
    assert 4 / 3 * math.pi * (rs - 1) ** 3 < lit < 4 / 3 * math.pi * (rs + 1) ** 3


def test_converges_with_opening_angle(orc, setup):
    e = [median_error(orc, setup, theta=t, nside=4, eta_r=8.0)[0] for t in (0.7, 0.5, 0.35, 0.25)]
    print("median error vs theta 0.7 0.5 0.35 0.25:", e)
    assert e[0] > e[1] > e[2] > e[3]
    assert e[3] < 0.02


def test_converges_with_angular_resolution(orc, setup):
    e = [median_error(orc, setup, theta=0.25, nside=ns, eta_r=8.0)[0] for ns in (1, 2, 4)]
    print("median error vs N_side 1 2 4:", e)
    assert e[0] > e[1] > e[2]
    assert e[2] < 0.02


def test_converges_with_radial_resolution(orc, setup):
    e = [median_error(orc, setup, theta=0.25, nside=4, eta_r=er)[0] for er in (2.0, 4.0, 8.0)]
    print("median error vs eta_R 2 4 8:", e)
    assert e[0] > e[1] > e[2]
