"""The freely falling camera of Appendix C ("Position"), the seeded camera path of the
request generators, pinned to closed forms of Schwarzschild geodesics (r_s = 1):
circular orbits (dr/dtau = 0), radial infall from rest (a cycloid in proper time),
the first integral of the radial equation, the relativistic precession of a nearly
circular orbit, and the initial speed and direction the constants are built from."""
import math

import numpy as np
import pytest

from paper_2010_08735_amd import scenes


def circular_speed(r):
    u = 1.0 / r
    return math.sqrt(u / (2.0 * (1.0 - u)))


@pytest.mark.parametrize("r0", [2.0, 3.0, 6.0, 15.0, 400.0])
def test_circular_orbit_constants(r0):
    """With dr/dtau = 0: l^2 = 1 / (u (2 - 3u)) and e^2 = 2 (1 - u)^2 / (2 - 3u), reached at
    the static observer's speed sqrt(u / (2 (1 - u))) (r = 6: 0.3162c; r = 3: 0.5c)."""
    u = 1.0 / r0
    e, l = scenes.orbit_constants(r0, math.pi / 2, circular_speed(r0))
    assert l * l == pytest.approx(1.0 / (u * (2.0 - 3.0 * u)), rel=1e-12)
    assert e * e == pytest.approx(2.0 * (1.0 - u) ** 2 / (2.0 - 3.0 * u), rel=1e-12)
    if r0 == 6.0:
        assert circular_speed(r0) == pytest.approx(math.sqrt(0.1), rel=1e-12)
    if r0 == 3.0:
        assert circular_speed(r0) == pytest.approx(0.5, rel=1e-12)


@pytest.mark.parametrize("r0", [4.0, 10.0, 30.0])
def test_circular_orbit_keeps_its_radius_at_the_kepler_rate(r0):
    """A circular orbit (stable for r0 > 3) keeps r = r0 over several turns and advances at
    dpsi/dt = sqrt(u^3 / 2), Kepler's rate in Schwarzschild coordinate time."""
    u = 1.0 / r0
    omega = math.sqrt(u ** 3 / 2.0)
    e, _ = scenes.orbit_constants(r0, math.pi / 2, circular_speed(r0))
    period_tau = 2.0 * math.pi / omega * (1.0 - u) / e
    st = scenes.camera_orbit(r0, math.pi / 2, circular_speed(r0),
                             np.linspace(0.0, 3.0 * period_tau, 7), step=0.1)
    assert np.abs(st.r - r0).max() < 1e-8 * r0
    assert np.allclose(st.psi[1:] / st.t[1:], omega, rtol=1e-9)
    assert st.psi[-1] == pytest.approx(6.0 * math.pi, rel=1e-9)


@pytest.mark.parametrize("r0", [5.0, 20.0])
def test_radial_infall_from_rest_is_a_cycloid(r0):
    """Released at rest (v0 = 0, so l = 0): r = (r0/2)(1 + cos eta) at proper time
    tau = (r0^(3/2) / 2)(eta + sin eta), whatever the direction delta0."""
    etas = np.array([0.3, 0.9, 1.5, 2.0])
    taus = 0.5 * r0 ** 1.5 * (etas + np.sin(etas))
    for delta0 in (0.0, 1.0, math.pi):
        st = scenes.camera_orbit(r0, delta0, 0.0, taus, step=0.05)
        assert np.allclose(st.r, 0.5 * r0 * (1.0 + np.cos(etas)), rtol=1e-9)
        assert np.all(st.psi == 0.0)


def test_radial_first_integral_holds_along_a_precessing_orbit():
    """(dr/dtau)^2 = e^2 + l^2 u^3 - l^2 u^2 + u - 1 along the integrated orbit, and the
    4-velocity stays unit timelike: -(1-u) tdot^2 + rdot^2 / (1-u) + r^2 psidot^2 = -1."""
    r0, d0, v0 = 12.0, 1.2, 0.26
    e, l = scenes.orbit_constants(r0, d0, v0)
    st = scenes.camera_orbit(r0, d0, v0, np.linspace(0.0, 4000.0, 41))
    u = 1.0 / st.r
    assert st.r.max() > 3.0 * st.r.min() and st.r.min() > 9.0   # eccentric, bound
    rhs = e * e + l * l * u ** 3 - l * l * u ** 2 + u - 1.0
    assert np.abs(st.dr ** 2 - rhs).max() < 1e-9
    norm = -(1.0 - u) * st.dt ** 2 + st.dr ** 2 / (1.0 - u) + st.r ** 2 * st.dpsi ** 2
    assert np.abs(norm + 1.0).max() < 1e-9


@pytest.mark.parametrize("r0", [10.0, 40.0])
def test_nearly_circular_orbit_precesses_by_the_epicyclic_ratio(r0):
    """A slightly eccentric orbit's angle advances by 2 pi / sqrt(1 - 3/r_g) between
    successive pericentres (radial epicyclic frequency Omega sqrt(1 - 6M/r), M = 1/2, at
    the guiding radius r_g midway between peri- and apocentre), against 2 pi for a
    Newtonian ellipse.  The correction is second order in the eccentricity (about 1e-3
    here), hence the tolerance."""
    u = 1.0 / r0
    v0 = circular_speed(r0) * 1.0005
    taus = np.linspace(0.0, 2.2 * 2.0 * math.pi / math.sqrt(u ** 3 / 2.0) / math.sqrt(1 - 3 * u),
                       200001)
    st = scenes.camera_orbit(r0, math.pi / 2, v0, taus)
    # pericentres: sign changes of dr/dtau from negative to positive (linear interpolation)
    k = np.nonzero((st.dr[:-1] < 0.0) & (st.dr[1:] >= 0.0))[0]
    assert len(k) >= 2
    w = -st.dr[k] / (st.dr[k + 1] - st.dr[k])
    psi = st.psi[k] + w * (st.psi[k + 1] - st.psi[k])
    ratio = (psi[1] - psi[0]) / (2.0 * math.pi)
    rg = 0.5 * (st.r.min() + st.r.max())
    assert ratio == pytest.approx(1.0 / math.sqrt(1.0 - 3.0 / rg), rel=2e-6)
    assert ratio > 1.03   # well away from the Newtonian 1


@pytest.mark.parametrize("r0,delta0,v0,chi", [(8.0, 0.7, 0.3, 0.4), (25.0, 2.3, 0.15, -1.1),
                                               (3.5, 1.5707963, 0.45, 2.0)])
def test_initial_speed_and_direction(r0, delta0, v0, chi):
    """At tau = 0 the static observer measures speed v0, in the orbital plane of inclination
    chi, at the angle atan(sqrt(1 - u0) tan(delta0)) from the outward radial direction
    (delta0 is the coordinate angle, tan(delta) = r dpsi / dr); the position lies on that
    plane at angle psi = 0, and the Schwarzschild angles theta = acos(cos psi sin chi),
    phi = atan2(sin psi, cos chi cos psi) give the same point."""
    st = scenes.camera_orbit(r0, delta0, v0, [0.0, 3.0])
    pos, vel = scenes.orbit_position_velocity(st, chi)
    assert np.allclose(pos[0], r0 * np.array([math.cos(chi), 0.0, math.sin(chi)]), atol=1e-12)
    assert np.linalg.norm(vel[0]) == pytest.approx(v0, rel=1e-12)
    rhat = pos[0] / r0
    local = math.atan2(math.sqrt(1.0 - 1.0 / r0) * math.sin(delta0), math.cos(delta0))
    assert float(vel[0] @ rhat) == pytest.approx(v0 * math.cos(local), abs=1e-12)
    assert st.dr[0] * math.tan(delta0) == pytest.approx(st.r[0] * st.dpsi[0], rel=1e-12)
    nrm = np.array([-math.sin(chi), 0.0, math.cos(chi)])
    for p, v in zip(pos, vel):
        assert abs(p @ nrm) < 1e-9 * r0 and abs(v @ nrm) < 1e-12
    for k in range(2):
        th = math.acos(math.cos(st.psi[k]) * math.sin(chi))
        ph = math.atan2(math.sin(st.psi[k]), math.cos(chi) * math.cos(st.psi[k]))
        sph = st.r[k] * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph),
                                  math.cos(th)])
        assert np.allclose(sph, pos[k], atol=1e-12 * r0)


def test_orbit_views_and_bad_inputs():
    """Frames along an orbit carry the camera's coordinate time; invalid constants and a
    camera that falls in are refused."""
    vs = scenes.orbit_views(10.0, 1.4, 0.3, 0.5, [0.0, 50.0, 100.0], 64, 48)
    assert [v.time for v in vs][0] == 0.0 and vs[1].time > 50.0 and vs[2].time > vs[1].time
    assert all(math.hypot(*v.cam_vel) < 1.0 for v in vs)
    for bad in ((1.0, 1.0, 0.1), (5.0, 1.0, 1.0), (5.0, -0.1, 0.1), (5.0, 1.0, -0.1)):
        with pytest.raises(ValueError):
            scenes.orbit_constants(*bad)
    with pytest.raises(ValueError):
        scenes.camera_orbit(3.0, math.pi, 0.2, [0.0, 100.0])
    with pytest.raises(ValueError):
        scenes.camera_orbit(5.0, 1.0, 0.1, [2.0, 1.0])
