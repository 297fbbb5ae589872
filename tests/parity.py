"""GPU-vs-oracle comparison helpers for the parity tests.

Mask (pixels where several answers are legitimately correct, reported as a fraction):
  (i)   the GPU and the oracle disagree on capture or on the number of disc crossings;
  (ii)  another member of the pixel's 2x2 quad is masked by (i) (the star term and the
        screen-space derivatives use every member of the quad);
  (iii) the oracle's lensing factor Omega/Omega' is above 64 (Einstein rings and caustics,
        where the beam's solid angle on the sky goes to zero);
  (iv)  the two sides chose different mip levels;
  (v)   |e^2/mu - 1| < 1e-3 (photon ring) or the beam plane is degenerate.
"""
import numpy as np

from paper_2010_08735_amd import bh


def render_gpu(ctx, tables, view, stars=None, aov=True, particles=None, area=None):
    import torch
    W, H = view.width, view.height
    out = torch.full((H, W, 4), float("nan"), dtype=torch.float32, device="cuda")
    a = torch.full((H, W, 4), float("nan"), dtype=torch.float32, device="cuda") if aov else None
    v = bh.make_view(view, stars, particles, area)
    bh.bh_render(ctx, tables, v, out.data_ptr(), a.data_ptr() if aov else None,
                 bh.current_stream())
    torch.cuda.synchronize()
    return out.cpu().numpy(), (a.cpu().numpy() if aov else None)


def gpu_at(rgb, aov, px):
    y, x = px["y"], px["x"]
    g = aov[y, x]
    bits = g[:, 3].copy().view(np.uint32)
    return {
        "rgb": rgb[y, x, :3].astype(np.float64),
        "alpha": rgb[y, x, 3],
        "dprime": g[:, 0].astype(np.float64),
        "u0": g[:, 1].astype(np.float64),
        "u1": g[:, 2].astype(np.float64),
        "captured": (bits & 1) != 0,
        "ncross": ((bits >> 1) & 1) + ((bits >> 2) & 1),
        "zeroed": ((bits >> 3) & 1) != 0,
        "degenerate": ((bits >> 4) & 1) != 0,
        "mip": (bits >> 8) & 255,
    }


def oracle_as_gpu(px):
    """An oracle rendering in the form gpu_at returns, to compare two oracle modes with the
    same masks and tolerances (the method's own error next to the GPU's)."""
    return {"rgb": px["rgb"], "captured": px["captured"] != 0, "ncross": px["n_cross"],
            "mip": np.where(px["mip_level"] >= 0, px["mip_level"], 255),
            "dprime": px["delta_prime"], "u0": px["u_cross"][:, 0], "u1": px["u_cross"][:, 1]}


def mask_of(px, g):
    cap_o = px["captured"] != 0
    m = (cap_o != g["captured"]) | (px["n_cross"] != g["ncross"])
    m = np.repeat(m.reshape(-1, 4).any(axis=1), 4)
    om = px["omega_ratio"]
    gathered = px["mip_level"] >= 0
    m |= gathered & (om > 64.0)
    m |= gathered & (px["mip_level"] != g["mip"].astype(np.int64))
    m |= np.abs(px["e2_over_mu"] - 1.0) < 1e-3
    m |= px["degenerate"] != 0
    return m


def rel_rgb(o, g, floor):
    """Per-pixel error relative to the pixel's brightest band (with an absolute floor)."""
    den = np.maximum(o.max(axis=1), floor)
    return np.abs(g - o).max(axis=1) / den


def compare(px, g, label=""):
    """Statistics of the GPU against one oracle rendering on the same pixels."""
    m = mask_of(px, g)
    ok = ~m
    s = {"label": label, "pixels": int(len(px)), "masked_fraction": float(m.mean())}
    esc = ok & (px["captured"] == 0)
    dd = np.abs(px["delta_prime"][esc] - g["dprime"][esc])
    s["dprime_max"] = float(dd.max()) if dd.size else 0.0
    s["dprime_p99"] = float(np.percentile(dd, 99)) if dd.size else 0.0
    hit = ok & (px["n_cross"] >= 1)
    du0 = np.abs(px["u_cross"][hit, 0] - g["u0"][hit])
    hit2 = ok & (px["n_cross"] >= 2)
    du1 = np.abs(px["u_cross"][hit2, 1] - g["u1"][hit2])
    s["u_max"] = float(max(du0.max() if du0.size else 0.0, du1.max() if du1.size else 0.0))
    o = px["rgb"]
    floor = 1e-4 * float(np.percentile(o.max(axis=1), 99)) + 1e-30
    r = rel_rgb(o, g["rgb"], floor)
    disc = ok & (px["n_cross"] >= 1)
    star = ok & (px["n_cross"] == 0) & (px["star_A"] > 0)
    for name, sel in (("disc", disc), ("star", star), ("all", ok)):
        v = r[sel]
        s[name + "_n"] = int(sel.sum())
        s[name + "_rel_p50"] = float(np.percentile(v, 50)) if v.size else 0.0
        s[name + "_rel_p99"] = float(np.percentile(v, 99)) if v.size else 0.0
        s[name + "_rel_max"] = float(v.max()) if v.size else 0.0
    s["finite"] = bool(np.isfinite(g["rgb"]).all())
    return s


def frac_within(px, g, tol, sel_name="all"):
    m = mask_of(px, g)
    ok = ~m
    o = px["rgb"]
    floor = 1e-4 * float(np.percentile(o.max(axis=1), 99)) + 1e-30
    r = rel_rgb(o, g["rgb"], floor)
    if sel_name == "disc":
        ok &= px["n_cross"] >= 1
    elif sel_name == "star":
        ok &= (px["n_cross"] == 0) & (px["star_A"] > 0)
    return float((r[ok] <= tol).mean()) if ok.any() else 1.0
