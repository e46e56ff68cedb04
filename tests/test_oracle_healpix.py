"""Pins of the oracle's HEALPix pixelisation (paper Sec. 2.2; Gorski et al. 2005).

The map is pinned by (i) the inverse map: every pixel centre, computed from
the ring/pixel formulas, lands in its own pixel; (ii) equal area: uniform
random directions fall into every pixel with probability 1/N_PIX; (iii) the
symmetries of the tessellation (rotation by pi/2 about z, reflections z -> -z
and x -> -x permute the pixels); (iv) a few directions whose pixels follow
from the base-pixel layout alone.
"""
import numpy as np
import pytest


@pytest.mark.parametrize("nside", [1, 2, 4, 8])
def test_centres_map_to_themselves(orc, nside):
    npix = 12 * nside * nside
    cen = np.array([orc.pix2vec(nside, p) for p in range(npix)])
    assert np.allclose(np.linalg.norm(cen, axis=1), 1.0)
    assert np.array_equal(orc.ang2pix(nside, cen), np.arange(npix))
    # ring structure: pixels of a ring share z
    z = cen[:, 2]
    assert len(np.unique(np.round(z, 12))) == 4 * nside - 1


@pytest.mark.parametrize("nside", [2, 4])
def test_equal_area(orc, nside):
    rng = np.random.default_rng(7)
    n = 2_000_000
    v = rng.standard_normal((n, 3))
    pix = orc.ang2pix(nside, v)
    npix = 12 * nside * nside
    cnt = np.bincount(pix, minlength=npix)
    assert cnt.size == npix
    expect = n / npix
    # binomial spread; 5 sigma
    assert np.all(np.abs(cnt - expect) < 5 * np.sqrt(expect))


@pytest.mark.parametrize("nside", [1, 2, 4])
def test_symmetries(orc, nside):
    npix = 12 * nside * nside
    cen = np.array([orc.pix2vec(nside, p) for p in range(npix)])
    rng = np.random.default_rng(3)
    v = rng.standard_normal((20000, 3))
    p0 = orc.ang2pix(nside, v)
    ops = [np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]]),   # rotation by pi/2 about z
           np.diag([1, 1, -1]),                            # z -> -z
           np.diag([-1, 1, 1])]                            # x -> -x
    for S in ops:
        perm = orc.ang2pix(nside, cen @ S.T)
        assert np.array_equal(np.sort(perm), np.arange(npix))   # a permutation
        assert np.array_equal(orc.ang2pix(nside, v @ S.T), perm[p0])


def test_base_pixels(orc):
    # N_side = 1: four polar pixels centred at phi = pi/4 + k pi/2, four
    # equatorial ones centred on the +x, +y, -x, -y axes, four southern ones.
    v = np.array([[1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0],
                  [1, 1, 1.5], [-1, 1, 1.5], [-1, -1, 1.5], [1, -1, 1.5],
                  [1, 1, -1.5], [-1, 1, -1.5], [-1, -1, -1.5], [1, -1, -1.5]], float)
    assert list(orc.ang2pix(1, v)) == [4, 5, 6, 7, 0, 1, 2, 3, 8, 9, 10, 11]


def test_near_pole_directions(orc):
    # 1 - |z| is formed without cancellation: a direction 1e-9 rad from the
    # pole still resolves its quadrant
    for ns in (1, 2, 4, 8):
        for k, (x, y) in enumerate([(1, 1), (-1, 1), (-1, -1), (1, -1)]):
            assert orc.ang2pix(ns, [[1e-9 * x, 1e-9 * y, 1.0]])[0] == k
            assert orc.ang2pix(ns, [[1e-9 * x, 1e-9 * y, -1.0]])[0] == 12 * ns * ns - 4 + k
