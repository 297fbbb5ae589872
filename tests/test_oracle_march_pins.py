"""Pins of the oracle's ray marcher, the foil of the paper's ablation (Section 5, method M3
of Table 1: TraceRay replaced by numerical integration of the orbit equation).

Expected values come from the closed-form one-step map of the Runge-Kutta method on the
flat-space equation u'' = -u, straight rays in flat space, the exact-mode integrator
(itself pinned by the weak-field and photon-sphere pins), cubic polynomials that a cubic
Hermite interpolant must reproduce, and the fourth order of the method."""
import math

import numpy as np
import pytest


def test_flat_space_step_is_the_truncated_exponential(orc):
    """For y' = A y with A = [[0, 1], [-1, 0]] (u'' = -u) one classic RK4 step multiplies by
    I + hA + (hA)^2/2 + (hA)^3/6 + (hA)^4/24 = (1 - h^2/2 + h^4/24) I + (h - h^3/6) A."""
    A = np.array([[0.0, 1.0], [-1.0, 0.0]])
    for u0, w0, h, k in [(0.1, -0.3, 0.2, 37), (0.02, 0.5, 0.7, 9), (1.0, 0.0, 0.05, 400)]:
        M = (1 - h * h / 2 + h ** 4 / 24) * np.eye(2) + (h - h ** 3 / 6) * A
        want = np.linalg.matrix_power(M, k) @ np.array([u0, w0])
        got = orc.march_state(u0, w0, h, k, gr=0.0)
        assert np.allclose(got, want, rtol=1e-13, atol=1e-15)


def test_one_step_of_the_full_equation_agrees_with_its_taylor_series(orc):
    """One step of size h of u'' = 3/2 u^2 - u from (u0, w0) differs from the Taylor
    polynomial of the solution through h^4 by O(h^5): the derivatives are u'' = 3/2 u^2 - u,
    u''' = (3u - 1) w, u'''' = 3 w^2 + (3u - 1) u''."""
    u0, w0 = 0.3, -0.2
    u2 = 1.5 * u0 * u0 - u0
    u3 = (3 * u0 - 1) * w0
    u4 = 3 * w0 * w0 + (3 * u0 - 1) * u2
    errs = []
    for h in (0.1, 0.05, 0.025):
        taylor = u0 + h * w0 + h ** 2 / 2 * u2 + h ** 3 / 6 * u3 + h ** 4 / 24 * u4
        u, _ = orc.march_state(u0, w0, h, 1)
        errs.append(abs(u - taylor))
    assert errs[0] / errs[1] > 25 and errs[1] / errs[2] > 25  # fifth order (32)


def test_hermite_interpolant_reproduces_cubics_and_finds_the_first_root(orc):
    """p(s) = -(s - 0.2)(s - 0.5)(s - 0.9) on [0, 1] has three roots; the interpolant of its
    end values and slopes is p itself and the first root is 0.2.  With h = 2 the same cubic
    in s/2 has its first root at 0.4."""
    def p(s):
        return -(s - 0.2) * (s - 0.5) * (s - 0.9)

    def dp(s):
        return -((s - 0.5) * (s - 0.9) + (s - 0.2) * (s - 0.9) + (s - 0.2) * (s - 0.5))

    for s in np.linspace(0, 1, 11):
        assert abs(orc.hermite(p(0), dp(0), p(1), dp(1), 1.0, s) - p(s)) < 1e-15
    assert abs(orc.hermite_first_root(p(0), dp(0), p(1), dp(1), 1.0) - 0.2) < 1e-14
    assert abs(orc.hermite_first_root(p(0), dp(0) / 2, p(1), dp(1) / 2, 2.0) - 0.4) < 1e-14
    # a line: the root of the secant
    assert abs(orc.hermite_first_root(0.3, -1.0, -0.2, -1.0, 0.5) - 0.3) < 1e-15


@pytest.mark.parametrize("rc,delta,alpha", [(15, 1.2, 0.7), (40, 2.0, 0.3), (8, 0.5, 2.5),
                                            (25, 2.6, 1.9), (6, 1.0, 0.2)])
def test_straight_rays_in_flat_space(orc, rc, delta, alpha):
    """gr = 0: the ray is the straight line u(phi) = u_c sin(delta - phi) / sin(delta), which
    leaves at phi = delta; crossings lie at alpha + m pi on that line."""
    uc = 1.0 / rc
    r = orc.march(uc, delta, alpha, 1.0, 0.0, 2048, gr=0.0)
    assert not r["captured"]
    assert abs(r["delta_prime"] - delta) < 1e-11
    want = [alpha + m * math.pi for m in range(3) if alpha + m * math.pi < delta]
    assert len(r["u"]) == len(want)
    for phi, u in zip(want, r["u"]):
        assert abs(u - uc * math.sin(delta - phi) / math.sin(delta)) < 1e-12


def _rays(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        yield (1 / rng.uniform(2.5, 50), rng.uniform(0.01, math.pi - 0.01),
               rng.uniform(0, math.pi), 1 / rng.uniform(3, 6), 1 / rng.uniform(10, 30))


def test_fourth_order_convergence_to_the_exact_geodesic(orc):
    """The escape angle's error against exact mode falls 16-fold per halving of the step
    (fourth order), for rays whose march takes many steps and whose e^2 is away from the
    photon-sphere value."""
    ratios = []
    for u, d, a, uic, uoc in _rays(200, 11):
        e2 = (u / math.tan(d)) ** 2 + u * u * (1 - u)
        if abs(e2 / orc.MU - 1) < 0.2:
            continue
        ex = orc.trace_exact(u, d, a, uic, uoc)
        if ex["captured"] or ex["delta_prime"] < 1.5:
            continue
        errs = [abs(orc.march(u, d, a, uic, uoc, n)["delta_prime"] - ex["delta_prime"])
                for n in (64, 128, 256)]
        if errs[2] < 1e-12:
            continue
        ratios += [errs[0] / errs[1], errs[1] / errs[2]]
    assert len(ratios) > 40
    assert 13 < np.median(ratios) < 19


def test_march_agrees_with_exact_mode_at_small_steps(orc):
    """With 4096 steps the march reproduces exact mode: same fate, same crossings, escape
    angles within 1e-9 (fourth order at h = 1.5e-3)."""
    n = 0
    for u, d, a, uic, uoc in _rays(300, 12):
        e2 = (u / math.tan(d)) ** 2 + u * u * (1 - u)
        if abs(e2 / orc.MU - 1) < 1e-3:
            continue
        ex = orc.trace_exact(u, d, a, uic, uoc)
        mr = orc.march(u, d, a, uic, uoc, 4096)
        if mr["unfinished"]:
            assert ex["captured"] or ex["delta_prime"] > 2 * math.pi - 1e-6
            continue
        assert mr["captured"] == ex["captured"]
        if not ex["captured"]:
            assert abs(mr["delta_prime"] - ex["delta_prime"]) < 1e-9
        # crossings within 1e-9 of the annulus edges may flip either way
        keep = range(ex["n_cross"])
        if any(min(abs(x - uic), abs(x - uoc)) < 1e-9 for x in ex["u"]):
            continue
        assert mr["n_cross"] == len(keep)
        for k in keep:
            assert abs(mr["u"][k] - ex["u"][k]) < 1e-10
            assert abs(mr["phi"][k] - ex["phi"][k]) < 1e-12
            assert mr["branch"][k] == ex["branch"][k]
        n += 1
    assert n > 200


def test_capture_and_the_step_budget(orc):
    """An ingoing radial-ish ray is captured within the march; a ray inside the photon
    sphere with e^2 < mu falls in after its apsis; a ray that winds near the photon sphere
    more than once runs out of steps (unfinished, drawn as captured)."""
    r = orc.march(1 / 6, 2.9, 1.0, 1 / 3, 1 / 20, 64)
    assert r["captured"] and not r["unfinished"] and r["steps"] < 64
    # inside the photon sphere moving outward with e^2 < mu: apsis, then the horizon
    u = 0.8
    d = 1.45
    e2 = (u / math.tan(d)) ** 2 + u * u * (1 - u)
    assert e2 < orc.MU
    r = orc.march(u, d, 1.0, 1 / 3, 1 / 20, 256)
    assert r["captured"] and not r["unfinished"]
    # e^2 just above mu from r = 3/2 outward-tangent: many turns near u = 2/3
    uc = 2.0 / 3.0
    d = math.pi / 2 - 1e-7
    r = orc.march(uc, d, 1.0, 1 / 3, 1 / 20, 128)
    assert r["captured"] and r["unfinished"] and r["steps"] == 128


def test_radial_beams_are_not_deflected(orc):
    """A radial beam stays on its radius (u'' and the angle decouple): outward it escapes in
    its own direction, inward it reaches the horizon."""
    for uc in (1 / 40, 1 / 6, 0.9):
        r = orc.march(uc, 1e-8, 1.0, 1 / 3, 1 / 20, 64)
        assert not r["captured"] and r["delta_prime"] == 1e-8 and r["n_cross"] == 0
        assert orc.march(uc, math.pi - 1e-8, 1.0, 1 / 3, 1 / 20, 64)["captured"]


def test_never_a_third_disc_crossing(orc):
    """A beam meets the disc plane at most twice with u <= 1/3 (Section 3.3.3), and the
    march finds no more: the annulus here reaches from r = 3 out to infinity."""
    for u, d, a, uic, uoc in _rays(400, 13):
        r = orc.march(u, d, a, 1.0 / 3.0, 1e-9, 256)
        assert r["n_cross"] <= 2
