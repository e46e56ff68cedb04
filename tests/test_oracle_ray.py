"""Pins of the oracle's On-the-Spot ray integration (paper Sec. 2.5).

Each case has a closed form that follows from the recurrence and the segment
volume of eq. (dV) without running the recurrence: the cone volumes of the
segments between a source and the target telescope to (r_j^3 - ...)/3, the
correction factors are constants on the chosen rays, and so on.
"""
import math

import numpy as np
import pytest

FOURPI = 4 * math.pi


def ray(n, L=50.0):
    return L * (np.arange(n) / (n - 1.0)) ** 2


def test_thin_ray_sums_point_fluxes(orc):
    r = ray(20)
    eps = np.zeros(20)
    eps[[3, 9, 17]] = [2.0, 5.0, 1.0]
    z = np.zeros(20)
    f = orc.integrate_ray(r, eps, z, z, np.ones(20), 2)
    assert f == pytest.approx(sum(eps[j] / (FOURPI * r[j] ** 2) for j in (3, 9, 17)), rel=1e-14)
    # emission at the target point itself never reaches it (F_0 sums j >= 1)
    eps0 = np.zeros(20)
    eps0[0] = 7.0
    assert orc.integrate_ray(r, eps0, z, z, np.ones(20), 2) == 0.0


def test_single_source_uniform_absorber(orc):
    # uniform alpha, no previous flux (zeta_d = 2 except in the segment next to
    # the source, where zeta_s = zeta_d = 1), zeta_g off:
    # Phi_0 = eps/4pi - alpha [dV_{j-1,j} + 2 (r_j^3 - (r_j - r_{j-1})^3)/3]
    n, j = 30, 22
    r = ray(n)
    alpha = 1e-6
    eps = np.zeros(n)
    eps[j] = 1.0
    V = np.ones(n)
    A = alpha * V
    E = np.zeros(n)
    f = orc.integrate_ray(r, eps, A, E, V, 2, zeta_g=False)
    rj = r[j]
    adj = (rj - r[j - 1]) ** 3 / 3.0
    phi0 = eps[j] / FOURPI - alpha * (adj + 2 * (rj ** 3 - adj * 3) / 3.0)
    assert phi0 > 0
    assert f == pytest.approx(phi0 / rj ** 2, rel=1e-10)
    # a strong absorber kills the source: truncation at zero, no negative flux
    assert orc.integrate_ray(r, eps, A * 1e3, E, V, 2, zeta_g=False) == 0.0


def test_zeta_d_from_previous_flux(orc):
    # absorption only at point a (alpha_a), so the segments [a-1,a] and [a,a+1]
    # each see alpha_a/2; the previous flux at a+1 and a is set to give
    # zeta_d = c1 and c2 there (the ray's flux there is known in closed form).
    n, j, a = 30, 25, 12
    r = ray(n)
    eps = np.zeros(n)
    eps[j] = 1.0
    V = np.ones(n)
    A = np.zeros(n)
    alpha = 3e-5
    A[a] = alpha
    c1, c2 = 0.37, 1.6
    phi_j = 1.0 / FOURPI
    dv = lambda i: ((r[j] - r[i]) ** 3 - (r[j] - r[i + 1]) ** 3) / 3.0
    F_a1 = phi_j / (r[j] - r[a + 1]) ** 2
    phi_a = phi_j - 0.5 * alpha * dv(a) * c1
    F_a = phi_a / (r[j] - r[a]) ** 2
    phi_am1 = phi_a - 0.5 * alpha * dv(a - 1) * c2
    E = np.full(n, 1e30)            # everywhere else zeta_d is ~0 (no alpha there anyway)
    E[a + 1] = F_a1 / c1
    E[a] = F_a / c2
    f = orc.integrate_ray(r, eps, A, E, V, 2, zeta_g=False)
    assert f == pytest.approx(phi_am1 / r[j] ** 2, rel=1e-12)
    # the cap at 2
    E[a + 1] = F_a1 / 7.0
    E[a] = F_a / 9.0
    phi_a2 = phi_j - 0.5 * alpha * dv(a) * 2.0
    F_a2 = phi_a2 / (r[j] - r[a]) ** 2
    zd = min(2.0, F_a2 / E[a])
    phi_c = phi_a2 - 0.5 * alpha * dv(a - 1) * zd
    assert orc.integrate_ray(r, eps, A, E, V, 2, zeta_g=False) == pytest.approx(phi_c / r[j] ** 2, rel=1e-12)


def test_zeta_s_shares_absorption(orc):
    # two sources j1 < j2, absorption only at point a (well inside both), no
    # previous flux (zeta_d = 2): source j gets the fraction F_j / (F_1 + F_2)
    # of the segment's loss, evaluated with the unabsorbed rates.
    n, j1, j2, a = 30, 20, 26, 9
    r = ray(n)
    eps = np.zeros(n)
    eps[j1], eps[j2] = 2.0, 5.0
    V = np.ones(n)
    A = np.zeros(n)
    alpha = 1e-5
    A[a] = alpha
    E = np.zeros(n)
    dv = lambda i, j: ((r[j] - r[i]) ** 3 - (r[j] - r[i + 1]) ** 3) / 3.0
    phi = {j1: eps[j1] / FOURPI, j2: eps[j2] / FOURPI}
    for i in (a, a - 1):                    # segments [a, a+1] then [a-1, a]
        F = {j: phi[j] / (r[j] - r[i + 1]) ** 2 for j in phi}
        tot = sum(F.values())
        phi = {j: phi[j] - 0.5 * alpha * dv(i, j) * 2.0 * F[j] / tot for j in phi}
    expect = sum(phi[j] / r[j] ** 2 for j in phi)
    assert orc.integrate_ray(r, eps, A, E, V, 2, zeta_g=False) == pytest.approx(expect, rel=1e-12)


@pytest.mark.parametrize("nside,frac", [(0, 1.0 / 3.0), (2, 1.0 / 4.0), (4, 31.0 / 96.0)])
def test_zeta_g_continuum_limit(orc, nside, frac):
    # fine ray, one source at distance R, uniform alpha, zeta_d = 2: the total
    # loss tends to 2 alpha int_0^R zeta_g(s) s^2 ds with
    # zeta_g(s) = min(1, N_side s / (2R)) (s = distance from the source):
    # R^3/3 without the correction, R^3/4 for N_side 2, 31 R^3/96 for N_side 4.
    n = 6000
    r = np.linspace(0, 10.0, n)
    j = n - 1
    R = r[j]
    alpha = 1e-4
    eps = np.zeros(n)
    eps[j] = 1.0
    V = np.ones(n)
    A = alpha * V
    E = np.zeros(n)
    f = orc.integrate_ray(r, eps, A, E, V, max(nside, 2), zeta_g=nside > 0)
    expect = (1.0 / FOURPI - 2 * alpha * frac * R ** 3) / R ** 2
    assert f == pytest.approx(expect, rel=2e-3)
