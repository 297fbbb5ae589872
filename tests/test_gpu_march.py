"""Ray marching in place of TraceRay (the ablation of Section 5, method M3 of Table 1) on
the GPU, through the C ABI, against the oracle's marcher (same steps, FP64) and against
exact geodesics.

Tolerances.  Both sides run the same fixed-step method, so they differ by FP32 rounding
only: each step rounds u and w at about 2^-24 relative, and the escape angle inherits the
state error divided by |du/dphi| at the escape plus the rounding of phi = n h (2^-24 x 2 pi).
Over n <= 1000 steps the rounding adds up to below 1e-4 relative in the worst case and far
less typically; the bounds below are that worst case, the percentiles the typical one."""
import json
import math

import numpy as np
import pytest

from paper_2010_08735_amd import bh, scenes

import parity

pytestmark = pytest.mark.gpu


def _report(s):
    print("\nPARITY " + json.dumps(s, sort_keys=True))


def _random_rays(n, seed):
    rng = np.random.default_rng(seed)
    u = 1 / rng.uniform(2.5, 50, n)
    d = rng.uniform(0.01, math.pi - 0.01, n)
    a = rng.uniform(0, math.pi, n)
    ric = rng.uniform(3, 6, n)
    roc = rng.uniform(10, 30, n)
    return np.stack([u, d, a, 1 / ric, 1 / roc], axis=1).astype(np.float32)


def _march_gpu(ctx, rays, nsteps):
    import torch
    r = torch.from_numpy(rays).cuda()
    out = torch.zeros((len(rays), 4), dtype=torch.float32, device="cuda")
    bh.bh_march_rays(ctx, r.data_ptr(), len(rays), nsteps, out.data_ptr(), bh.current_stream())
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("nsteps", [25, 100, 1000])
def test_march_rays_match_the_oracle_march(gpu_ctx, orc, nsteps):
    rays = _random_rays(20000 if nsteps < 1000 else 5000, 21)
    g = _march_gpu(gpu_ctx, rays, nsteps)
    bits = g[:, 3].copy().view(np.uint32)
    n = agree = 0
    dd, du = [], []
    for k in range(len(rays)):
        u, d, a, uic, uoc = [float(x) for x in rays[k]]
        e2 = (u / math.tan(d)) ** 2 + u * u * (1 - u)
        if abs(e2 / orc.MU - 1) < 1e-3:
            continue
        o = orc.march(u, d, a, uic, uoc, nsteps)
        cap = bool(bits[k] & bh.BH_AOV_CAPTURED)
        nc = int((bits[k] >> 1) & 1) + int((bits[k] >> 2) & 1)
        n += 1
        same = cap == o["captured"] and nc == o["n_cross"] and \
            bool(bits[k] & bh.BH_AOV_UNFINISHED) == o["unfinished"]
        agree += same
        if not same:
            continue
        for j in range(nc):
            want = bh.BH_AOV_CROSS1 if o["branch"][j] else bh.BH_AOV_CROSS0
            assert bits[k] & want
            du.append(abs(o["u"][j] - g[k, 1 + j]))
        if not cap:
            dd.append(abs(o["delta_prime"] - g[k, 0]) / max(1.0, o["delta_prime"]))
    dd, du = np.array(dd), np.array(du)
    s = {"nsteps": nsteps, "n": n, "agree": agree / n, "dprime_rel_max": float(dd.max()),
         "dprime_rel_p99": float(np.percentile(dd, 99)), "u_max": float(du.max()),
         "u_p99": float(np.percentile(du, 99))}
    _report(s)
    assert s["agree"] > 0.998
    assert s["dprime_rel_max"] < 1e-4 and s["dprime_rel_p99"] < 2e-6
    assert s["u_max"] < 1e-5


def test_radial_rays(gpu_ctx, orc):
    """delta = 0 leaves along the radius (delta' = 0), delta = pi falls in: the GPU keeps a
    finite slope for them, as the render path does, and agrees with the oracle's fates."""
    rays = np.array([[1 / 6, 0.0, 1.0, 1 / 3, 1 / 20], [1 / 6, math.pi, 1.0, 1 / 3, 1 / 20],
                     [1 / 40, 0.0, 0.3, 1 / 3, 1 / 20], [0.9, math.pi, 2.0, 1 / 3, 1 / 20]],
                    np.float32)
    g = _march_gpu(gpu_ctx, rays, 64)
    bits = g[:, 3].copy().view(np.uint32)
    for k in range(len(rays)):
        o = orc.march(*[float(x) for x in rays[k]], 64)
        assert bool(bits[k] & bh.BH_AOV_CAPTURED) == o["captured"]
        assert not bits[k] & bh.BH_AOV_UNFINISHED
        if not o["captured"]:
            assert abs(g[k, 0] - o["delta_prime"]) < 1e-5


def render_march_gpu(ctx, view, stars, nsteps):
    import torch
    W, H = view.width, view.height
    out = torch.full((H, W, 4), float("nan"), dtype=torch.float32, device="cuda")
    a = torch.full((H, W, 4), float("nan"), dtype=torch.float32, device="cuda")
    bh.bh_render_march(ctx, bh.make_view(view, stars), nsteps, out.data_ptr(), a.data_ptr(),
                       bh.current_stream())
    torch.cuda.synchronize()
    return out.cpu().numpy(), a.cpu().numpy()


@pytest.mark.parametrize("nsteps", [32, 256])
def test_march_render_small_view_full_frame(gpu_ctx, orc, small_scene, nsteps):
    """128x128 static camera at r = 15: every pixel against the oracle's marcher with the
    same step budget (pure numerics), and the budget's own accuracy against exact mode."""
    field, n0, h, cube = small_scene
    v = scenes.small_static_view()
    rgb, aov = render_march_gpu(gpu_ctx, v, h, nsteps)
    assert np.all(rgb[..., 3] == 1.0) and np.isfinite(rgb).all()
    quads = scenes.all_quads(v.width, v.height)
    pm = orc.render_quads(v, quads, cube=cube, n0=n0, march=nsteps)
    pe = orc.render_quads(v, quads, cube=cube, n0=n0)
    g = parity.gpu_at(rgb, aov, pm)
    sm, se = parity.compare(pm, g, "march"), parity.compare(pe, g, "exact")
    _report({"nsteps": nsteps, "small_march": sm, "small_exact": se})
    assert sm["masked_fraction"] < 0.02
    assert sm["dprime_max"] < 5e-5 and sm["u_max"] < 1e-5
    assert parity.frac_within(pm, g, 1e-3, "disc") > 0.995
    assert parity.frac_within(pm, g, 2e-2, "star") > 0.99
    assert parity.frac_within(pm, g, 2e-2, "all") > 0.995


def test_march_render_boosted_view_sampled(gpu_ctx, gpu_tables, orc, big_field_scene):
    """1920x1080 camera at r = 6 moving at 0.9c, a seeded 1% of the quads: the march with
    100 steps against the oracle's march, and the accuracy of several step budgets and of
    the tables against exact geodesics on the same pixels (the ablation's comparison)."""
    field, n0, h, cube = big_field_scene
    v = scenes.boosted_orbit_view()
    quads = scenes.sample_quads(v.width, v.height, 0.01, 12)
    pe = orc.render_quads(v, quads, cube=cube, n0=n0)
    rgb, aov = render_march_gpu(gpu_ctx, v, h, 100)
    pm = orc.render_quads(v, quads, cube=cube, n0=n0, march=100)
    g = parity.gpu_at(rgb, aov, pm)
    sm = parity.compare(pm, g, "march100")
    assert sm["masked_fraction"] < 0.02
    # the FP32 beam set-up (aberration at gamma = 2.3) adds to the integrator's own rounding
    assert sm["dprime_max"] < 1e-4 and sm["u_max"] < 5e-5
    assert parity.frac_within(pm, g, 1e-3, "disc") > 0.995
    assert parity.frac_within(pm, g, 2e-2, "star") > 0.99
    acc = {}
    rgb_t, aov_t = parity.render_gpu(gpu_ctx, gpu_tables, v, h)
    runs = [("tables", parity.gpu_at(rgb_t, aov_t, pe))]
    for n in (16, 25, 50, 100, 250, 1000):
        r, a = render_march_gpu(gpu_ctx, v, h, n)
        runs.append(("march%d" % n, parity.gpu_at(r, a, pe)))
    for name, gg in runs:
        s = parity.compare(pe, gg, name)
        acc[name] = {k: s[k] for k in ("masked_fraction", "dprime_max", "dprime_p99", "u_max",
                                       "star_rel_p50", "star_rel_p99", "disc_rel_p99")}
    _report({"boosted_march_vs_oracle_march": sm, "accuracy_vs_exact": acc})
    # fourth order: 16 -> 25 steps divides the error by (25/16)^4 = 6, 25 -> 50 by 16, until
    # the FP32 rounding of the beam set-up (a few 1e-6) is reached from about 100 steps on
    p99 = {n: acc["march%d" % n]["dprime_p99"] for n in (16, 25, 50, 100, 250, 1000)}
    assert p99[16] > 4 * p99[25] and p99[25] > 4 * p99[50]
    assert max(p99[100], p99[250], p99[1000]) < 1e-5
    assert acc["march1000"]["dprime_max"] < 1e-3
    # the 512^2 deflection table sits between 25 and 50 steps
    assert p99[50] < acc["tables"]["dprime_p99"] < 4 * p99[25]


def test_march_rejects_bad_arguments(gpu_ctx):
    import torch
    out = torch.zeros((8, 8, 4), dtype=torch.float32, device="cuda")
    v = scenes.View(**{**scenes.small_static_view().__dict__, "width": 8, "height": 8})
    for n in (0, 2, (1 << 20) + 1):
        with pytest.raises(bh.BhError) as ei:
            bh.bh_render_march(gpu_ctx, bh.make_view(v), n, out.data_ptr())
        assert ei.value.status == bh.BH_EINVAL
    anim = scenes.animated_disc_view(8, 8)
    ph = bh.bh_create_particles(gpu_ctx, anim.particles.as_array())
    with pytest.raises(bh.BhError) as ei:
        bh.bh_render_march(gpu_ctx, bh.make_view(anim, None, ph), 64, out.data_ptr())
    assert ei.value.status == bh.BH_EINVAL
    bh.bh_release_particles(ph)
    rays = torch.zeros((4, 5), dtype=torch.float32, device="cuda")
    with pytest.raises(bh.BhError):
        bh.bh_march_rays(gpu_ctx, rays.data_ptr(), 4, 1, out.data_ptr())
