"""Benchmark of the MI355X beam tracer (one JSON line on stdout).

Workload (the headline metric's configuration): one 1920x1080 frame seen from a camera at
r = 6 r_s, 85 deg from the disc normal, moving at 0.9c along +azimuth; disc r in [3, 20];
1,000,000 seeded stars in a 6x2048x2048 RGBA16F star map; 512x512 / 64x32 tables
integrated on the GPU with the FP64 photon-sphere band; FP32 trace.  A step is one frame of
the whole per-pixel path (beam init, TraceRay, disc, derivatives, star gather, compose) on
device-resident inputs; tables and star map are built once, before timing.

Also reported: the ablation of Section 5 (TraceRay replaced by RK4 ray marching at several
step budgets: frame time and escape-angle accuracy), the bloom pass of Section 3.4.3 on the
rendered frame and the display encoding after it (fused and alone), the batched form (64 uneven views in
one persistent launch) and the served form (Poisson arrivals, continuous batching) against
one launch per frame, the roofline of the render kernel (algorithmic HBM bytes from a
footprint-counting pass, kernel duration from HIP events on the launch stream) and the FP64
CPU oracle on one full frame.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X: 157.3 TFLOP/s published FP32 vector peak (packed FP32, two FMAs per lane); one
# FP32 FMA per lane per clock on 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz gives 78.6 TFLOP/s,
# the rate without packed-FP32 instructions, which this build does not emit.  VALU issue
# reference: one wave64 instruction per CU per clock, 614.4 G/s in all.
FP32_VECTOR_PEAK_TFLOPS = 78.6
FP32_PACKED_PEAK_TFLOPS = 157.3
VALU_ISSUE_REF_G = 256 * 2.4
WAVE_PIXELS = 64
PROFILE = os.path.join(ROOT, "profiles", "k_render_1080p_summary.txt")
KERNEL_SOURCES = ("paper_2010_08735_amd/csrc/render.hip", "paper_2010_08735_amd/csrc/bh_dev.h",
                  "paper_2010_08735_amd/csrc/libbh.cpp", "paper_2010_08735_amd/build.py")


def kernel_profile():
    """Per-unit figures of the render kernel from the committed rocprofv3 summary, if they
    were taken on the current kernel sources (else None)."""
    import hashlib
    if not os.path.exists(PROFILE):
        return None
    vals = {}
    for line in open(PROFILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if vals.get("source_sha256") != h.hexdigest():
        return None
    return {k: float(v) for k, v in vals.items() if k != "source_sha256"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def star_map(bh, ctx, field, n0):
    import torch
    d = torch.from_numpy(field.dirs).cuda()
    i = torch.from_numpy(field.intensity).cuda()
    t = torch.from_numpy(field.temperature).cuda()
    h = bh.bh_build_stars(ctx, d.data_ptr(), i.data_ptr(), t.data_ptr(), len(field), n0,
                          bh.BH_TEXEL_FP16, bh.current_stream())
    torch.cuda.synchronize()
    return h


def warm(fn, seconds=0.2):
    """Untimed calls of fn() for `seconds` of wall time (synchronising every 20 calls), so the
    GPU's clocks have settled when timing starts: after host work the card idles and ramps
    down, and a few warm-up launches time it still ramping up."""
    import torch
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        fn()
        n += 1
        if n % 20 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()


def plain_leg(bh, ctx, tables, view, steps, warmup):
    """One launch per frame, back to back on the launch stream: `warmup` untimed launches
    (long enough for the GPU's clocks to settle; a short warm-up times a card that is still
    ramping up), then `steps` timed launches between two synchronisations (wall clock),
    bracketed by HIP events recorded on the same stream, whose elapsed time over `steps` is
    the kernel's average launch duration."""
    import torch
    out = torch.empty((view.height, view.width, 4), dtype=torch.float32, device="cuda")
    st = bh.current_stream()
    for _ in range(warmup):
        bh.bh_render(ctx, tables, view, out.data_ptr(), None, st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        bh.bh_render(ctx, tables, view, out.data_ptr(), None, st)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / steps, out


def batch_leg(bh, ctx, tables, views, reps):
    """64 uneven views: one launch per frame against one persistent launch (HIP graph)."""
    import torch
    outs = [torch.empty((v.height, v.width, 4), dtype=torch.float32, device="cuda")
            for v in views]
    ptrs = [o.data_ptr() for o in outs]
    st = bh.current_stream()
    px = sum(v.width * v.height for v in views)
    res = {}
    for name in ("plain", "batched"):
        if name == "batched":
            best, ms = bh.bh_autotune(ctx, tables, views, ptrs, reps=2)
            cfg = bh.bh_tile_config_get(best // 2)
            res["autotune"] = {"tile": [cfg.tile_w, cfg.tile_h], "ppt": cfg.ppt,
                               "persistent": best % 2, "ms_per_config": [round(m, 4) for m in ms]}
        def once():
            if name == "plain":
                for v, p in zip(views, ptrs):
                    bh.bh_render(ctx, tables, v, p, None, st)
            else:
                bh.bh_render_batch(ctx, tables, views, ptrs, st)
        warm(once)
        t0 = time.perf_counter()
        for _ in range(reps):
            once()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[name] = {"ms_per_batch": dt * 1e3, "mpx_per_s": px / dt / 1e6}
    res["pixels_per_batch"] = px
    del outs
    return res


def serve_leg(bh, scenes, tables_of, fields, duration, rate, seed, budget, max_tiles,
              inflight, tile_config, orbits="circular"):
    """Poisson arrivals for `duration` seconds through bh_submit/bh_poll (library-allocated
    images inside the HBM budget), then the same requests submitted all at once, twice: the
    first pass allocates the server's images, the second runs on its recycled images.
    Cameras on circular orbits, or freely falling on the orbits of Appendix C."""
    import torch
    if orbits == "freefall":
        reqs = scenes.freefall_requests(rate=rate, duration=duration, seed=seed + 1)
    else:
        reqs = scenes.serve_requests(rate=rate, duration=duration, seed=seed)
    out = {"requests": len(reqs), "rate_per_s": rate, "duration_s": duration, "orbits": orbits,
           "max_tiles_per_launch": max_tiles, "max_inflight_launches": inflight,
           "tile_config": tile_config}
    ctx = bh.bh_create(0, budget)
    try:
        tables = tables_of(ctx)
        smaps = [star_map(bh, ctx, f, 2048) for f in fields]
        bh.bh_set_tile_config(ctx, tile_config)
        bh.bh_serve_start(ctx, 0, inflight, max_tiles)
        for mode in ("poisson", "saturated_first_pass", "saturated"):
            tickets, lat = [], []
            t_start = time.perf_counter()
            px = 0
            for r in reqs:
                if mode == "poisson":
                    wait = t_start + r.arrival - time.perf_counter()
                    if wait > 0:
                        time.sleep(wait)
                v = bh.make_view(r.view, smaps[r.field])
                tickets.append(bh.bh_submit(ctx, tables, v, None))
                px += r.view.width * r.view.height
                # free finished images as we go so the budget admits new frames
                while len(tickets) > 64:
                    done, l = bh.bh_poll(ctx, tickets[0])
                    if not done:
                        break
                    lat.append(l)
                    bh.bh_ticket_free(ctx, tickets.pop(0))
            for t in tickets:
                while True:
                    done, l = bh.bh_poll(ctx, t)
                    if done:
                        break
                    time.sleep(1e-4)
                lat.append(l)
                bh.bh_ticket_free(ctx, t)
            span = time.perf_counter() - t_start
            lat.sort()
            out[mode] = {"mpx_per_s": px / span / 1e6, "makespan_s": span,
                         "latency_p50_ms": 1e3 * lat[len(lat) // 2],
                         "latency_p99_ms": 1e3 * lat[min(len(lat) - 1, int(0.99 * len(lat)))]}
    finally:
        bh.bh_destroy(ctx)
    # the same requests as one plain launch per frame, back to back on one stream
    ctx = bh.bh_create(0, budget)
    try:
        tables = tables_of(ctx)
        smaps = [star_map(bh, ctx, f, 2048) for f in fields]
        imgs = {}
        for r in reqs:
            key = (r.view.width, r.view.height)
            if key not in imgs:
                imgs[key] = torch.empty((key[1], key[0], 4), dtype=torch.float32, device="cuda")
        views = [bh.make_view(r.view, smaps[r.field]) for r in reqs]
        st = bh.current_stream()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        px = 0
        for r, v in zip(reqs, views):
            bh.bh_render(ctx, tables, v, imgs[(r.view.width, r.view.height)].data_ptr(), None, st)
            px += r.view.width * r.view.height
        torch.cuda.synchronize()
        span = time.perf_counter() - t0
        del imgs
    finally:
        bh.bh_destroy(ctx)
    out["plain_per_frame"] = {"mpx_per_s": px / span / 1e6, "makespan_s": span}
    return out


def cpu_baseline(view_obj, field, n0, min_seconds=10.0):
    """The FP64 oracle on whole frames of the same workload, all host cores, repeated until
    at least `min_seconds` of CPU work."""
    import oracle
    from paper_2010_08735_amd import scenes
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cube = oracle.cubemap(field, n0)
    quads = scenes.all_quads(view_obj.width, view_obj.height)
    frames = pixels = 0
    t0 = time.perf_counter()
    while True:
        px = oracle.render_quads(view_obj, quads, cube=cube, n0=n0, nthreads=threads)
        frames += 1
        pixels += len(px)
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    return {"value": pixels / dt / 1e6, "unit": "Mpixels/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d full %dx%d frames (%d pixels each), exact geodesic integration, "
                      "FP64, star map built before timing"
                      % (frames, view_obj.width, view_obj.height, len(px)),
            "seconds": dt}


def march_leg(bh, view, ctx, tables, W, H, reps=100):
    """The ablation of Section 5 (method M3 of Table 1): the same frame with TraceRay
    replaced by RK4 ray marching at several step budgets.  Frame time from HIP events on
    the launch stream; accuracy of the escape angle delta' (from the AOV) of the tables and of
    each budget against a 4096-step march, over pixels that escape on both sides."""
    import numpy as np
    import torch
    st = bh.current_stream()
    out = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")

    def frame_us(fn):
        warm(fn)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return 1e3 * e0.elapsed_time(e1) / reps

    def aov_of(fn):
        a = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
        fn(a.data_ptr())
        torch.cuda.synchronize()
        return a.cpu().numpy().reshape(-1, 4)

    ref = aov_of(lambda a: bh.bh_render_march(ctx, view, 4096, out.data_ptr(), a, st))
    bad = bh.BH_AOV_CAPTURED | bh.BH_AOV_DEGENERATE | bh.BH_AOV_UNFINISHED

    def err(a):
        ok = ((a[:, 3].copy().view(np.uint32) | ref[:, 3].copy().view(np.uint32)) & bad) == 0
        d = np.abs(a[ok, 0].astype(np.float64) - ref[ok, 0])
        return {"dprime_p50": float(np.percentile(d, 50)), "dprime_p99": float(np.percentile(d, 99)),
                "pixels": int(ok.sum())}

    res = {"reference": "4096-step march", "tables": {
        "us_per_frame": frame_us(lambda: bh.bh_render(ctx, tables, view, out.data_ptr(), None, st)),
        **err(aov_of(lambda a: bh.bh_render(ctx, tables, view, out.data_ptr(), a, st)))}}
    for n in (16, 25, 50, 100):
        res["march%d" % n] = {
            "us_per_frame": frame_us(lambda: bh.bh_render_march(ctx, view, n, out.data_ptr(), None, st)),
            **err(aov_of(lambda a: bh.bh_render_march(ctx, view, n, out.data_ptr(), a, st)))}
    for k, v in res.items():
        if isinstance(v, dict):
            v["mpx_per_s"] = W * H / v["us_per_frame"]
    return res


def _event_time_us(fn, reps):
    """HIP-event time per call of fn() on the launch stream, after warm()."""
    import torch
    warm(fn)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return 1e3 * e0.elapsed_time(e1) / reps


def bloom_leg(bh, scenes, ctx, img, W, H, levels=7, reps=200, exposure=4.0):
    """Bloom (Section 3.4.3) of the rendered frame: HIP-event time per pass on the launch
    stream, and the HBM bytes it must move at least: the image read twice (the mipmap pass
    and the output pass) and the output written once, plus the pyramid written and read.
    Then the display encoding that follows it: fused into the glare pass's output (4-byte
    pixels written in place of 16-byte ones) and on its own (16 bytes in, 4 out per pixel)."""
    import torch
    st = bh.current_stream()
    out = torch.empty_like(img)
    disp = torch.empty((H, W), dtype=torch.int32, device=img.device)
    b = bh.bh_bloom_create(ctx, W, H, levels)
    wt = scenes.bloom_weights(levels)
    us = _event_time_us(lambda: bh.bh_bloom_apply(b, wt, img.data_ptr(), out.data_ptr(), st),
                        reps)
    us_fused = _event_time_us(lambda: bh.bh_bloom_apply_display(
        b, wt, exposure, img.data_ptr(), disp.data_ptr(), st), reps)
    bh.bh_bloom_release(b)
    us_tm = _event_time_us(lambda: bh.bh_tonemap(ctx, out.data_ptr(), disp.data_ptr(), W, H,
                                                 exposure, st), reps)
    pyr, w, h = 0, W, H
    for _ in range(levels):
        w, h = (w + 1) // 2, (h + 1) // 2
        pyr += w * h
    alg = 16 * (3 * W * H + 2 * pyr)
    alg_fused = 16 * (2 * W * H + 2 * pyr) + 4 * W * H
    alg_tm = 20 * W * H
    return {"levels": levels, "us_per_frame": us, "mpx_per_s": W * H / us,
            "algorithmic_bytes": alg, "hbm_gbs": alg / us / 1e3,
            "hbm_frac": alg / us / 1e3 / HBM_PEAK_GBS,
            "display": {"exposure": exposure,
                        "fused": {"us_per_frame": us_fused, "algorithmic_bytes": alg_fused,
                                  "hbm_gbs": alg_fused / us_fused / 1e3},
                        "tonemap_alone": {"us_per_frame": us_tm, "algorithmic_bytes": alg_tm,
                                          "hbm_gbs": alg_tm / us_tm / 1e3}}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 2000 warm-up frames (~0.1 s) let the GPU's clocks settle before the 2000 timed ones;
    # 20 warm-up frames time a card still ramping up, ~8% slower at 1080p
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--legs", default="plain,anim,area,march,bloom,batch,serve,cpu",
                    help="comma list of plain, anim, area, march, bloom, batch, serve, cpu")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="seconds of the Poisson arrival stream replayed by the serve leg")
    ap.add_argument("--serve-tiles", type=int, default=262144,
                    help="most tiles (of the serving tile configuration) in one serving launch")
    ap.add_argument("--serve-inflight", type=int, default=6,
                    help="serving launches kept in flight")
    ap.add_argument("--serve-tile-config", type=int, default=0,
                    help="tile configuration index of the serving launches (0: 16x16 "
                         "tiles, the fastest for the mixed stream; -1: the library's default)")
    ap.add_argument("--serve-orbits", choices=("circular", "freefall"), default="circular",
                    help="serve leg cameras: circular orbits, or free fall (Appendix C)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the beam tracer runs on a single MI355X here "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    legs = set(args.legs.split(","))

    import numpy as np
    import torch
    from paper_2010_08735_amd import bh, scenes

    bh.lib()
    ctx = bh.bh_create(0, 0)
    t0 = time.perf_counter()
    tables = bh.bh_precompute_tables(ctx, 512, 64, 32, bh.BH_TAB_FP64_BAND, 0.05)
    t_tab = time.perf_counter() - t0
    field = scenes.star_field(1_000_000, 1)
    t0 = time.perf_counter()
    stars = star_map(bh, ctx, field, 2048)
    t_star = time.perf_counter() - t0
    sv = scenes.boosted_orbit_view()
    view = bh.make_view(sv, stars)
    W, H = sv.width, sv.height
    log("tables %.3f s, star map %.3f s" % (t_tab, t_star))

    # measurement passes of the roofline, before the timed leg: the footprint counting pass
    # (distinct star-map texels visited, bytes requested through the caches) and the L2
    # read-bandwidth probe.  (They also leave the card's clocks up, as a stream of frames
    # would: after host-side set-up the first frames otherwise time a card still ramping up.)
    scratch = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    texels, req = bh.bh_footprint_texels(ctx, tables, view, scratch.data_ptr())
    bw_l2 = bh.bh_probe_l2_read(ctx, 2 << 20, 20)
    del scratch

    wall, kms, out = plain_leg(bh, ctx, tables, view, args.steps, args.warmup)
    img = out.cpu().numpy()
    assert np.isfinite(img).all(), "non-finite pixels"
    ms_step = 1e3 * wall / args.steps
    mpx = W * H * args.steps / wall / 1e6
    kernel_ms = float(kms)
    log("plain: %.4f ms/frame wall, kernel %.4f ms (events), %.0f Mpx/s" % (ms_step, kernel_ms, mpx))

    # roofline of the render kernel: t_roof = max(B_HBM / 8 TB/s, B_L2 / BW_L2) against the
    # live event-timed kernel duration.  B_HBM: the bytes one frame must move at least (the
    # RGBA32F image, 8 B per distinct star-map texel the footprints visit, the tables and the
    # band table, each once).  B_L2: the bytes every pixel requests through the caches
    # (table and band-table fetches, occupancy words, texels, level records, the image), both
    # counted by the counting pass on this frame; BW_L2 from the probe.  The vector-ALU view
    # (FLOPs and instruction issue from the committed rocprofv3 counters, if they were taken
    # on the current kernel sources) is reported beside it: the kernel is bound by VALU issue.
    t_k = kernel_ms * 1e-3
    bytes_out = 16 * W * H
    bytes_tex = 8 * texels
    bytes_tab = 4 * (512 * 512 + 64 * 32) + 16 * 4096
    alg = bytes_out + bytes_tex + bytes_tab
    t_hbm = alg / (HBM_PEAK_GBS * 1e9)
    t_l2 = req / bw_l2
    t_roof = max(t_hbm, t_l2)
    hbm = {"achieved": alg / t_k / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": t_hbm / t_k, "algorithmic_bytes": alg, "bytes_image": bytes_out,
           "bytes_star_texels": bytes_tex, "star_texels_touched": texels,
           "bytes_tables_lut": bytes_tab}
    l2 = {"achieved": req / t_k / 1e9, "peak": bw_l2 / 1e9, "unit": "GB/s", "frac": t_l2 / t_k,
          "requested_bytes": req, "bytes_per_pixel": req / (W * H),
          "probe": "bh_probe_l2_read: streaming 16-byte reads of a 2 MiB buffer held in L2"}
    prof = kernel_profile()
    roof = {"bound": "l2" if t_l2 > t_hbm else "hbm",
            "achieved": (l2 if t_l2 > t_hbm else hbm)["achieved"],
            "peak": (l2 if t_l2 > t_hbm else hbm)["peak"], "unit": "GB/s",
            "frac": t_roof / t_k, "t_roof_us": 1e6 * t_roof, "kernel_us": 1e6 * t_k,
            "traffic": prof["fetch_bytes"] + prof["write_bytes"] if prof else None,
            "kernel": "k_render<8,8,1,0>", "kernel_ms": kernel_ms, "hbm": hbm, "l2": l2}
    if prof is not None:
        flops = prof["fp32_flops_per_pixel"] * W * H
        tf = flops / t_k / 1e12
        # VALU issue: instructions per 8x8-pixel wave (counters) x waves of one launch
        winst = prof["valu_insts_per_wave"] * math.ceil(W / 8) * math.ceil(H / 8)
        gi = winst / t_k / 1e9
        roof["alu"] = {"achieved": tf, "peak": FP32_PACKED_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": tf / FP32_PACKED_PEAK_TFLOPS,
                       "frac_of_non_packed_fp32": tf / FP32_VECTOR_PEAK_TFLOPS,
                       "flops_per_pixel": prof["fp32_flops_per_pixel"],
                       "valu_issue": {"achieved": gi, "unit": "G wave64-instructions/s",
                                      "per_cu_per_clock_at_2_4_ghz": gi / VALU_ISSUE_REF_G,
                                      "insts_per_wave": prof["valu_insts_per_wave"]},
                       "valu_busy_pct": prof["valu_busy_pct"], "l2_hit_pct": prof["l2_hit_pct"]}
    else:
        roof["alu"] = None
        roof["note"] = "counters not taken on the current kernel sources: traffic and alu unset"
    log("roofline: %s frac %.3f (t_roof %.2f us: HBM %.2f us, L2 %.2f us; kernel %.2f us); "
        "L2 probe %.0f GB/s, %.0f B/px requested"
        % (roof["bound"], roof["frac"], 1e6 * t_roof, 1e6 * t_hbm, 1e6 * t_l2, 1e6 * t_k,
           bw_l2 / 1e9, req / (W * H)))

    extra = {}
    if "anim" in legs:
        # the same frame with an animated particle disc (retarded times, Appendix B)
        av = scenes.boosted_orbit_view()
        av.disc_density = scenes.DENSITY_PARTICLES
        av.disc_opacity = 0.5
        av.time = 1000.0
        av.particles = scenes.disc_particles(64, av.disc_r_in, av.disc_r_out, 9)
        ph = bh.bh_create_particles(ctx, av.particles.as_array())
        aview = bh.make_view(av, stars, ph)
        awall, akms, _ = plain_leg(bh, ctx, tables, aview, max(10, args.steps // 4),
                                   args.warmup)
        n_a = max(10, args.steps // 4)
        extra["animated"] = {"particles": len(av.particles), "ms_per_frame": 1e3 * awall / n_a,
                             "kernel_ms": float(akms),
                             "mpx_per_s": W * H * n_a / awall / 1e6}
        bh.bh_release_particles(ph)
        log("animated:", json.dumps(extra["animated"]))
    if "area" in legs:
        # the same frame under an area-source sky (nebulae, Section 3.3.2) read by the
        # anisotropic footprint filter, stars and disc unchanged
        n_area = 512
        tex = torch.from_numpy(scenes.area_map(n_area, 21)).cuda()
        ah = bh.bh_build_area(ctx, tex.data_ptr(), n_area, bh.current_stream())
        torch.cuda.synchronize()
        del tex
        n_ar = max(10, args.steps // 4)
        rwall, rkms, _ = plain_leg(bh, ctx, tables, bh.make_view(sv, stars, None, ah), n_ar,
                                   args.warmup)
        extra["area"] = {"face_size": n_area, "map_bytes": 8 * (8 * n_area * n_area - 2),
                         "ms_per_frame": 1e3 * rwall / n_ar, "kernel_ms": float(rkms),
                         "mpx_per_s": W * H * n_ar / rwall / 1e6}
        bh.bh_release_area(ah)
        # the same sky as band colours (light of any colour, Section 3.4.2): the footprint's
        # (R, G, B) mean, shifted through the colour-shift table (built with the map)
        tex = torch.from_numpy(scenes.area_map_bands(n_area, 21)).cuda()
        t0 = time.perf_counter()
        ah = bh.bh_build_area_bands(ctx, tex.data_ptr(), n_area, bh.current_stream())
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        del tex
        rwall, rkms, _ = plain_leg(bh, ctx, tables, bh.make_view(sv, stars, None, ah), n_ar,
                                   args.warmup)
        extra["area"]["bands"] = {"map_bytes": 16 * (8 * n_area * n_area - 2),
                                  "build_with_color_shift_table_s": build_s,
                                  "ms_per_frame": 1e3 * rwall / n_ar, "kernel_ms": float(rkms),
                                  "mpx_per_s": W * H * n_ar / rwall / 1e6}
        bh.bh_release_area(ah)
        log("area:", json.dumps(extra["area"]))
        # the 1M-star field as stars of any colour (Section 3.4.2): a band-colour star map of
        # the same size, gathered and received through the colour-shift table
        bd, brgb = scenes.star_field_bands(1_000_000, 1)
        d_t, c_t = torch.from_numpy(bd).cuda(), torch.from_numpy(brgb).cuda()
        t0 = time.perf_counter()
        bsh = bh.bh_build_star_bands(ctx, d_t.data_ptr(), c_t.data_ptr(), len(bd), 2048,
                                     bh.BH_TEXEL_FP16, bh.current_stream())
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        del d_t, c_t
        rwall, rkms, _ = plain_leg(bh, ctx, tables, bh.make_view(sv, bsh), n_ar, args.warmup)
        extra["star_bands"] = {"stars": len(bd), "star_map": "6x2048x2048, 16-byte FP16 band texels",
                               "build_s": build_s, "ms_per_frame": 1e3 * rwall / n_ar,
                               "kernel_ms": float(rkms), "mpx_per_s": W * H * n_ar / rwall / 1e6}
        bh.bh_release_stars(bsh)
        log("star bands:", json.dumps(extra["star_bands"]))
    if "bloom" in legs:
        extra["bloom"] = bloom_leg(bh, scenes, ctx, out, W, H)
        log("bloom:", json.dumps(extra["bloom"]))
    if "march" in legs:
        extra["ablation_march"] = march_leg(bh, view, ctx, tables, W, H)
        log("march ablation:", json.dumps(extra["ablation_march"]))
    if "batch" in legs:
        views = [bh.make_view(v, stars) for v in scenes.batch_views(64, 3)]
        extra["batched"] = batch_leg(bh, ctx, tables, views, reps=10)
        log("batch:", json.dumps(extra["batched"]))
    bh.bh_destroy(ctx)
    torch.cuda.synchronize()

    if "serve" in legs:
        fields = [scenes.star_field(n, s) for n, s in scenes.SERVE_FIELDS]
        tab = lambda c: bh.bh_precompute_tables(c, 512, 64, 32, bh.BH_TAB_FP64_BAND, 0.05)
        extra["served"] = serve_leg(bh, scenes, tab, fields, args.serve_seconds, 200.0, 4,
                                    64 << 30, args.serve_tiles, args.serve_inflight,
                                    args.serve_tile_config, args.serve_orbits)
        log("serve:", json.dumps(extra["served"]))

    if "calib" in legs:
        # a plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE counters
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        extra["calib_copy_bytes"] = 4 * (64 << 20)

    cpu = None
    if "cpu" in legs:
        cpu = cpu_baseline(sv, field, 2048)
        log("cpu baseline: %.3f Mpx/s on %d cores (%.1f s)" % (cpu["value"], cpu["cores"], cpu["seconds"]))

    line = {
        "metric": "Mpixels/s at 1080p (plain vs batched/served); p50/p99 frame latency",
        "value": mpx, "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
        "data": "synthetic (seeded star field and camera, no catalog data)",
        "config": {"workload": "1920x1080 frame, camera r=6 at 0.9c tangential, disc [3,20], "
                               "1M stars 6x2048^2 RGBA16F, tables 512^2 + 64x32 (FP64 band)",
                   "width": W, "height": H, "stars": 1_000_000, "star_map": "6x2048x2048 RGBA16F",
                   "tables": "D 512x512, U 64x32, FP32 storage", "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "setup_s": {"tables": t_tab, "star_map": t_star},
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
