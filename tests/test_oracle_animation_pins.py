"""Pins of the oracle's animated-disc functions: coordinate time along rays (retarded times,
Algorithm 1 and Section 3.3.3) and the procedural disc particles (Appendix B).

Expected values come from closed forms (straight-line distance, radial light travel time,
the weak-field time delay, Kepler's law), the defining integrals evaluated with mpmath,
scipy's elliptic functions, and the orbit equation itself."""
import math

import mpmath
import numpy as np
import pytest
import scipy.special as ss

M = 0.5  # mass in units of the Schwarzschild radius (r_s = 2M = 1)


def test_exact_time_is_the_straight_line_distance_in_flat_space(orc):
    """gr = 0: rays are straight lines and the coordinate time from the camera to a crossing
    is the Euclidean distance between them (law of cosines in the beam plane)."""
    n = 0
    for rc, delta, alpha in [(15, 1.2, 0.7), (40, 2.0, 0.3), (8, 0.5, 2.5), (25, 2.6, 1.9),
                             (6, 1.0, 0.2)]:
        r = orc.trace_exact(1.0 / rc, delta, alpha, 1.0 / 3.0, 1e-6, gr=0.0)
        for k in range(r["n_cross"]):
            rk, psi = 1.0 / r["u"][k], r["phi"][k]
            dist = math.sqrt(rc * rc + rk * rk - 2 * rc * rk * math.cos(psi))
            assert abs(r["t"][k] - dist) < 1e-8 * dist
            n += 1
    assert n >= 3


def test_singular_part_is_the_radial_light_travel_time(orc):
    """For e -> infinity the ray is radial and dt/dr = 1/(1 - 1/r): t = r + ln(r - 1).
    The regularised time then vanishes and S(u) carries the whole travel time."""
    e2 = 1e12
    for ra, rb in [(50.0, 3.0), (1e4, 10.0), (7.5, 1.5)]:
        ua, ub = 1.0 / ra, 1.0 / rb
        t = (orc.tau_in(e2, ub) + orc.time_singular(ub)) - (orc.tau_in(e2, ua) + orc.time_singular(ua))
        expect = (ra - rb) + math.log((ra - 1.0) / (rb - 1.0))
        assert abs(t - expect) < 1e-9 * max(1.0, expect)
        assert abs(orc.tau_in(e2, ub)) < 1e-10


@pytest.mark.parametrize("e2,u", [(0.01, 0.05), (0.1, 0.2), (0.14, 0.3), (0.2, 0.5),
                                  (1.0, 0.9), (0.0009, 0.02)])
def test_regularised_time_is_the_defining_integral(orc, e2, u):
    """tau(u) = integral_0^u [e / (v^2 (1 - v) w) - 1/v^2 - 1/v - 1/(1 - v)] dv with
    w = sqrt(e^2 - v^2 (1 - v)): the rate dt/du of Algorithm 1 minus the derivative of
    S(u) = ln(u/(1-u)) - 1/u, evaluated with 60 digits and Gauss-Legendre nodes (the two
    terms cancel near v = 0)."""
    ua = orc.apsis(e2) if e2 < orc.MU else 2.0
    assert u < ua
    with mpmath.workdps(60):
        e2m = mpmath.mpf(e2)
        e = mpmath.sqrt(e2m)

        def f(v):
            w = mpmath.sqrt(e2m - v * v * (1 - v))
            return e / (v * v * (1 - v) * w) - 1 / v ** 2 - 1 / v - 1 / (1 - v)

        pts = [mpmath.mpf(0), mpmath.mpf(u) / 2, mpmath.mpf(u)]
        expect = float(mpmath.quad(f, pts, method="gauss-legendre"))
    assert abs(orc.tau_in(e2, u) - expect) < 1e-9 * max(1.0, abs(expect))


@pytest.mark.parametrize("b", [300.0, 1000.0, 10000.0])
def test_time_through_periapsis_matches_the_weak_field_delay(orc, b):
    """A ray with large impact parameter from r1 in to its periapsis r0 and back out to r1:
    t = 2 [sqrt(r1^2 - r0^2) + 2M ln((r1 + sqrt(r1^2 - r0^2)) / r0) + M sqrt((r1 - r0)/(r1 + r0))]
    to first order in M / r0 (coordinate time in Schwarzschild coordinates, the classic
    time-delay formula); the remainder is second order, below 25 M^2 / r0."""
    e2 = 1.0 / (b * b)
    ua = orc.apsis(e2)
    r0 = 1.0 / ua
    for r1 in (5 * b, 20 * b):
        u1 = 1.0 / r1
        ta = orc.tau_in(e2, ua) + orc.time_singular(ua)
        t1 = orc.tau_in(e2, u1) + orc.time_singular(u1)
        dt = 2.0 * (ta - t1)
        w = math.sqrt(r1 * r1 - r0 * r0)
        weak = 2.0 * (w + 2 * M * math.log((r1 + w) / r0) + M * math.sqrt((r1 - r0) / (r1 + r0)))
        assert abs(dt - weak) < 25.0 * M * M / r0
        assert abs(dt - weak) > 0.0


def _random_rays(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        yield (1 / rng.uniform(2.5, 50), rng.uniform(0.01, math.pi - 0.01),
               rng.uniform(0, math.pi), 1 / rng.uniform(3, 6), 1 / rng.uniform(10, 30))


def test_table_retarded_times_agree_with_exact_integration(orc):
    """Algorithm 1's retarded times (s (t_0 - t) and 2 t_a - t - t_1 from the time channels)
    against coordinate time integrated along the exact geodesic.  The method places a
    crossing within du ~ 1e-3 of the truth, i.e. dr = du / u^2 along the beam, so its time
    error is of that order; the beam-plane angle of the crossing is exact."""
    tab = orc.Tables(512, 64, 32, time=True)
    errs, scaled = [], []
    for u, d, a, uic, uoc in _random_rays(3000, 5):
        e2 = (u / math.tan(d)) ** 2 + u * u * (1 - u)
        if abs(e2 / orc.MU - 1) < 1e-3:
            continue
        x = orc.trace_exact(u, d, a, uic, uoc)
        t = tab.trace(u, d, a, uic, uoc)
        if x["n_cross"] != t["n_cross"] or x["captured"] != t["captured"]:
            continue
        for k in range(t["n_cross"]):
            assert abs(x["phi"][k] - t["phi"][k]) < 1e-9
            err = abs(x["t"][k] - t["t"][k])
            errs.append(err)
            scaled.append(err * x["u"][k] ** 2 / max(abs(x["u"][k] - t["u"][k]), 1e-6))
    errs = np.array(errs)
    assert len(errs) > 300
    assert np.median(errs) < 0.05
    # the large errors are those of the crossing's position along the beam
    assert np.percentile(scaled, 95) < 10.0


def test_complete_elliptic_integral_matches_scipy(orc):
    for k in (0.0, 0.05, 0.3, 0.7, 0.95):
        assert abs(orc.ellipk(k) - ss.ellipk(k * k)) < 1e-12 * ss.ellipk(k * k)


def _orbit_roots(r_peri, r_apo):
    u2, u1 = 1.0 / r_peri, 1.0 / r_apo
    return u1, u2, 1.0 - u1 - u2


def test_sn_orbit_solves_the_massive_particle_orbit_equation():
    """Appendix B's orbit u = u1 + (u2 - u1) sn^2(phi sqrt(u3 - u1) / 2, kappa) with
    u3 = 1 - u1 - u2 satisfies (du/dphi)^2 = (u - u1)(u - u2)(u - u3), i.e. the geodesic
    equation u'' = 3/2 u^2 - u + const of a massive particle (scipy's sn)."""
    for r_peri, r_apo in [(9.0, 11.0), (5.0, 8.0), (14.0, 14.5)]:
        u1, u2, u3 = _orbit_roots(r_peri, r_apo)
        m = (u2 - u1) / (u3 - u1)
        c = math.sqrt(u3 - u1) / 2
        phi = np.linspace(0.1, 12.0, 40)
        sn, cn, dn, _ = ss.ellipj(phi * c, m)
        u = u1 + (u2 - u1) * sn ** 2
        du = (u2 - u1) * 2 * sn * cn * dn * c
        assert np.allclose(du ** 2, (u - u1) * (u - u2) * (u - u3), rtol=1e-9, atol=1e-15)
        h = 1e-4
        up = u1 + (u2 - u1) * ss.ellipj((phi + h) * c, m)[0] ** 2
        um = u1 + (u2 - u1) * ss.ellipj((phi - h) * c, m)[0] ** 2
        upp = (up - 2 * u + um) / (h * h)
        const = upp - 1.5 * u * u + u
        assert np.ptp(const) < 1e-6 * abs(const).max()


def test_quasi_circular_approximation_and_keplerian_rate(orc):
    """The oracle's particle points turn at Kepler's rate about the mean radius (Omega^2 =
    M / r^3 in coordinate time, r = 1 / ubar): advancing time by dt equals advancing the
    point parameter a by Omega dt; u stays close to the exact sn orbit for a nearly circular
    orbit; and the radial period in phi is the exact one, 4K / sqrt(u3 - u1)."""
    r_peri, r_apo, phi0 = 9.8, 10.2, 0.4
    part = [r_peri, r_apo, phi0]
    u1, u2, u3 = _orbit_roots(r_peri, r_apo)
    ubar = 0.5 * (u1 + u2)
    omega = math.sqrt(M * ubar ** 3)
    for a, t, dt in [(0.3, 10.0, 7.0), (2.0, 400.0, 55.0)]:
        assert abs(orc.particle_u(part, a, t + dt) - orc.particle_u(part, a + omega * dt, t)) < 1e-14
    m = (u2 - u1) / (u3 - u1)
    c = math.sqrt(u3 - u1) / 2
    period = 4 * ss.ellipk(m) / math.sqrt(u3 - u1)
    for t in (0.0, 37.0, 500.0):
        ph = omega * t + phi0
        exact = u1 + (u2 - u1) * ss.ellipj(ph * c, m)[0] ** 2
        approx = orc.particle_u(part, 0.0, t)
        assert abs(approx - exact) < 1e-3 * (u2 - u1)
        assert abs(orc.particle_u(part, period, t) - approx) < 1e-12


def test_density_of_one_particle(orc):
    """f(d) = (1 - d^2)^2 inside d < 1: 1 at the particle centre (a = pi at the orbit's
    radius), 9/16 half way along the arc or half a unit off radially, 0 at the arc's ends."""
    part = [12.0, 12.0, 0.3]            # circular: u is constant
    r, t = 12.0, 123.0
    phi_t = math.sqrt((1 / r) ** 3 / 2) * t + 0.3
    centre = phi_t + math.pi
    assert abs(orc.disc_density(part, t, r, centre) - 1.0) < 1e-12
    assert abs(orc.disc_density(part, t, r, centre + 0.5 * math.pi) - 0.5625) < 1e-12
    assert abs(orc.disc_density(part, t, r + 0.5, centre) - 0.5625) < 1e-12
    assert orc.disc_density(part, t, r, phi_t + 1e-9) < 1e-8
    assert orc.disc_density(part, t, r + 1.01, centre) == 0.0
    # two particles add up
    two = [part, [12.0, 12.0, 0.3 + math.pi]]
    assert abs(orc.disc_density(two, t, r, centre) - 1.0) < 1e-12
