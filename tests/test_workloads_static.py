"""The static set-ups of the paper's accuracy tests (Sec. 3.2.1 rabbit hole,
Sec. 3.4 cloud irradiated by two sources): geometry and symmetry of the
generated inputs."""
import numpy as np
import pytest

from paper_2105_09644_amd import workloads as W


def test_two_source_cloud_geometry():
    n = 32
    P = W.two_source_cloud(n)
    dom = P.domains[0]
    assert dom.extent_finest() == (n, n, n)
    assert dom.finest_dx_cm() * n == pytest.approx(6.0 * W.PC_CM)
    nh = P.n_h[0].reshape(n, n, n)
    # symmetric about the plane x = y, sources swapped by it
    assert np.array_equal(nh, np.transpose(nh, (1, 0, 2)))
    s = P.src_xyz[0] / W.PC_CM
    assert np.allclose(s[0], [0, 2, 3]) and np.allclose(s[1], [2, 0, 3])
    # cloud of radius 0.5 pc: its volume and density
    dense = nh > 100
    vol = dense.sum() * (6.0 / n) ** 3
    assert vol == pytest.approx(4 / 3 * np.pi * 0.5 ** 3, rel=0.25)
    assert nh.max() == pytest.approx(0.7 * 2.6e-21 / W.M_P)
    assert nh.min() == pytest.approx(0.7 * 1e-24 / W.M_P)


@pytest.mark.parametrize("axis", [0, 2])
def test_rabbit_hole_geometry(axis):
    P = W.rabbit_hole(0.5, 96, axis)
    dom = P.domains[0]
    e = dom.extent_finest()
    assert e[axis] == 96 and all(e[a] == 32 for a in range(3) if a != axis)
    nh = P.n_h[0].reshape(e)
    hole = nh < 1.0
    # a straight hole through the whole length, square cross-section of 0.5 pc
    sec = hole.take(0, axis=axis)
    assert np.all(hole == np.expand_dims(sec, axis))
    dx = 6.0 / 96
    assert sec.sum() * dx * dx == pytest.approx(0.5 * 0.5, rel=0.3)
    # the source sits at the entrance, the centre of the hole's face
    s = P.src_xyz[0][0] / W.PC_CM
    want = np.array([1.0, 1.0, 1.0]); want[axis] = 0.0
    assert np.allclose(s, want)
