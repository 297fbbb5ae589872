"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline leg may
import this module.  It never touches the GPU library and the GPU library never calls it.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from .build import LIB, build

MU = 4.0 / 27.0


class OrcView(C.Structure):
    _fields_ = [("r_s", C.c_double), ("cam_pos", C.c_double * 3), ("cam_vel", C.c_double * 3),
                ("cam_rot", C.c_double * 9), ("fov_y", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32),
                ("disc_r_in", C.c_double), ("disc_r_out", C.c_double),
                ("disc_T_law", C.c_int32), ("pad0", C.c_int32),
                ("disc_T0", C.c_double), ("disc_T_exp", C.c_double),
                ("disc_opacity", C.c_double), ("k_disc", C.c_double), ("k_star", C.c_double),
                ("time", C.c_double), ("disc_density", C.c_int32), ("n_particles", C.c_int32),
                ("particles", C.POINTER(C.c_double)),
                ("area", C.POINTER(C.c_double)), ("area_n0", C.c_int32),
                ("area_exact", C.c_int32), ("k_area", C.c_double),
                ("area_bands", C.c_int32), ("ct_n", C.c_int32 * 3),
                ("ctable", C.POINTER(C.c_double)), ("star_bands", C.c_int32),
                ("pad1", C.c_int32)]


class OrcRay(C.Structure):
    _fields_ = [("delta_prime", C.c_double), ("captured", C.c_int32), ("n_cross", C.c_int32),
                ("u_cross", C.c_double * 4), ("phi_cross", C.c_double * 4),
                ("branch", C.c_int32 * 4), ("steps", C.c_int32), ("unfinished", C.c_int32),
                ("t_cross", C.c_double * 4)]


PIXEL_DTYPE = np.dtype([
    ("rgb", "<f8", 3), ("disc_rgb", "<f8", 3), ("star_rgb", "<f8", 3),
    ("delta_prime", "<f8"), ("u_cross", "<f8", 2), ("e2_over_mu", "<f8"),
    ("omega_ratio", "<f8"), ("d_cam", "<f8"), ("star_A", "<f8"), ("star_T", "<f8"),
    ("delta", "<f8"), ("alpha", "<f8"), ("zeta", "<f8"),
    ("x", "<i4"), ("y", "<i4"), ("n_cross", "<i4"), ("branch_bits", "<i4"),
    ("captured", "<i4"), ("star_zeroed", "<i4"), ("degenerate", "<i4"), ("mip_level", "<i4"),
    ("pad0", "<i4"), ("pad1", "<i4"), ("t_ret", "<f8", 2), ("hit_az", "<f8", 2), ("density", "<f8", 2),
    ("area_rgb", "<f8", 3), ("area_A", "<f8"), ("area_T", "<f8"), ("area_exact_A", "<f8"),
    ("area_exact_T", "<f8"), ("area_chroma", "<f8", 2),
])

_lib = None


def _check_layout(L):
    """The record layouts above must match the C structs byte for byte."""
    if L.orc_sizeof_pixel() != PIXEL_DTYPE.itemsize or L.orc_sizeof_ray() != C.sizeof(OrcRay) \
            or L.orc_sizeof_view() != C.sizeof(OrcView):
        raise RuntimeError("oracle record layout mismatch")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.orc_apsis.restype = C.c_double
        L.orc_apsis.argtypes = [C.c_double]
        L.orc_deflection.restype = C.c_double
        L.orc_deflection.argtypes = [C.c_double]
        L.orc_u_at_phi.restype = C.c_double
        L.orc_u_at_phi.argtypes = [C.c_double] * 4
        L.orc_trace_exact.argtypes = [C.c_double] * 6 + [C.POINTER(OrcRay)]
        L.orc_trace_table.argtypes = [dp, C.c_int32, dp, C.c_int32, C.c_int32] + \
            [C.c_double] * 5 + [C.POINTER(OrcRay)]
        L.orc_tables.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, dp, C.c_int]
        L.orc_table_entry_D.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, dp, dp]
        L.orc_table_entry_U.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, dp, dp, dp]
        L.orc_band_radiance.argtypes = [C.c_double, dp]
        L.orc_planck.restype = C.c_double
        L.orc_planck.argtypes = [C.c_double, C.c_double]
        L.orc_cubemap_texels.restype = C.c_int64
        L.orc_cubemap_texels.argtypes = [C.c_int32]
        fp = C.POINTER(C.c_float)
        L.orc_cubemap_build.argtypes = [fp, fp, fp, C.c_int64, C.c_int32, dp]
        L.orc_cubemap_build_bands.argtypes = [fp, fp, C.c_int64, C.c_int32, dp]
        L.orc_render_quads.argtypes = [C.POINTER(OrcView), dp, C.c_int32, dp, C.c_int32, dp,
                                       C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.c_int64,
                                       C.c_void_p, C.c_int]
        L.orc_render_quads_t.argtypes = [C.POINTER(OrcView), dp, C.c_int32, dp, dp, C.c_int32,
                                         dp, dp, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                         C.c_int64, C.c_void_p, C.c_int]
        L.orc_tables_time.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, dp, C.c_int]
        L.orc_trace_table_t.argtypes = [dp, dp, C.c_int32, dp, dp, C.c_int32, C.c_int32] + \
            [C.c_double] * 5 + [C.POINTER(OrcRay)]
        L.orc_tau_in.restype = C.c_double
        L.orc_tau_in.argtypes = [C.c_double, C.c_double]
        L.orc_time_singular.restype = C.c_double
        L.orc_time_singular.argtypes = [C.c_double]
        L.orc_ellipk.restype = C.c_double
        L.orc_ellipk.argtypes = [C.c_double]
        L.orc_particle_u.restype = C.c_double
        L.orc_particle_u.argtypes = [dp, C.c_double, C.c_double]
        L.orc_disc_density.restype = C.c_double
        L.orc_disc_density.argtypes = [dp, C.c_int32, C.c_double, C.c_double, C.c_double]
        L.orc_march_ray.argtypes = [C.c_double] * 5 + [C.c_int32, C.c_double, C.POINTER(OrcRay)]
        L.orc_march_state.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32, C.c_double,
                                      dp, dp]
        L.orc_hermite.restype = C.c_double
        L.orc_hermite.argtypes = [C.c_double] * 6
        L.orc_hermite_first_root.restype = C.c_double
        L.orc_hermite_first_root.argtypes = [C.c_double] * 5
        L.orc_render_quads_m.argtypes = [C.POINTER(OrcView), dp, C.c_int32, C.c_int32,
                                         C.POINTER(C.c_int32), C.c_int64, C.c_void_p, C.c_int]
        L.orc_area_texels.restype = C.c_int64
        L.orc_area_texels.argtypes = [C.c_int32]
        L.orc_area_build.argtypes = [fp, C.c_int32, dp]
        L.orc_area_filter.argtypes = [dp, C.c_int32, dp, dp, dp, dp, dp]
        L.orc_area_exact.argtypes = [dp, C.c_int32, dp, dp, dp, dp, dp]
        L.orc_area_build_bands.argtypes = [fp, C.c_int32, dp]
        L.orc_area_filter_bands.argtypes = [dp, C.c_int32, dp, dp, dp, dp]
        L.orc_area_exact_bands.argtypes = [dp, C.c_int32, dp, dp, dp, dp]
        L.orc_absorption.restype = C.c_double
        L.orc_absorption.argtypes = [C.c_int, C.c_double]
        L.orc_chroma_project.argtypes = [C.c_double, C.c_double, dp]
        L.orc_band_cct.restype = C.c_double
        L.orc_band_cct.argtypes = [C.c_double, C.c_double]
        L.orc_spectrum_of.argtypes = [C.c_double, C.c_double, dp]
        L.orc_color_shift.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_cshift_table.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, C.c_int]
        L.orc_cshift_lookup.argtypes = [dp, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                        C.c_double, C.c_double, dp]
        L.orc_bloom.argtypes = [dp, C.c_int32, C.c_int32, C.c_int32, dp, dp]
        L.orc_tonemap.argtypes = [dp, C.c_int64, C.c_double, C.c_void_p, dp]
        for f in ("orc_sizeof_pixel", "orc_sizeof_ray", "orc_sizeof_view"):
            getattr(L, f).restype = C.c_int64
        _check_layout(L)
        L.orc_quad_poly_check.restype = C.c_double
        L.orc_quad_poly_check.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def threads() -> int:
    return os.cpu_count() or 1


def apsis(e2: float) -> float:
    return lib().orc_apsis(e2)


def deflection(e: float) -> float:
    return lib().orc_deflection(e)


def u_at_phi(u0: float, w0: float, phi: float, gr: float = 1.0) -> float:
    return lib().orc_u_at_phi(u0, w0, phi, gr)


def _ray_dict(r: OrcRay):
    n = r.n_cross
    return {"delta_prime": r.delta_prime, "captured": bool(r.captured), "n_cross": n,
            "u": [r.u_cross[k] for k in range(n)], "phi": [r.phi_cross[k] for k in range(n)],
            "branch": [r.branch[k] for k in range(n)], "steps": r.steps,
            "unfinished": bool(r.unfinished),
            "t": [r.t_cross[k] for k in range(n)]}


def trace_exact(u_c, delta, alpha, u_ic, u_oc, gr=1.0):
    r = OrcRay()
    lib().orc_trace_exact(u_c, delta, alpha, u_ic, u_oc, gr, C.byref(r))
    return _ray_dict(r)


def march(u_c, delta, alpha, u_ic, u_oc, nsteps, gr=1.0):
    """Ray marching (fixed-step RK4, h = 2 pi / nsteps) in place of TraceRay."""
    r = OrcRay()
    if lib().orc_march_ray(u_c, delta, alpha, u_ic, u_oc, nsteps, gr, C.byref(r)):
        raise ValueError("bad step count")
    return _ray_dict(r)


def march_state(u0, w0, h, k, gr=1.0):
    u, w = C.c_double(), C.c_double()
    lib().orc_march_state(u0, w0, h, k, gr, C.byref(u), C.byref(w))
    return u.value, w.value


def hermite(p0, m0, p1, m1, h, s):
    return lib().orc_hermite(p0, m0, p1, m1, h, s)


def hermite_first_root(p0, m0, p1, m1, h):
    return lib().orc_hermite_first_root(p0, m0, p1, m1, h)


def bloom(image, levels, weights):
    """Bloom of an (H, W, 4) image with mipmap levels 1..levels and weights w_0..w_levels."""
    img = np.ascontiguousarray(image, np.float64)
    h, w = img.shape[:2]
    wt = np.ascontiguousarray(weights, np.float64)
    if len(wt) != levels + 1:
        raise ValueError("need levels + 1 weights")
    out = np.zeros_like(img)
    if lib().orc_bloom(_dp(img), w, h, levels, _dp(wt), _dp(out)):
        raise ValueError("orc_bloom rejected its arguments")
    return out


def tonemap(image, exposure):
    """Display encoding of an (H, W, 4) linear image: (codes, scaled), codes (H, W, 4) uint8
    (R, G, B, 255) and scaled (H, W, 3) = 255 v + 1/2, the value each code is the floor of."""
    img = np.ascontiguousarray(image, np.float64)
    n = img.size // 4
    out = np.zeros(img.shape[:-1] + (4,), np.uint8)
    sc = np.zeros(img.shape[:-1] + (3,), np.float64)
    if lib().orc_tonemap(_dp(img), n, float(exposure), out.ctypes.data, _dp(sc)):
        raise ValueError("orc_tonemap rejected its arguments")
    return out, sc


class Tables:
    """Quadrature tables at the texel centres; time=True also fills the regularised time
    channels Dt, Ut (same layout)."""

    def __init__(self, d_n=512, u_ne=64, u_nphi=32, nthreads=None, time=False):
        self.d_n, self.u_ne, self.u_nphi = d_n, u_ne, u_nphi
        self.D = np.zeros((d_n, d_n), np.float64)
        self.U = np.zeros((u_nphi, u_ne), np.float64)
        rc = lib().orc_tables(d_n, u_ne, u_nphi, _dp(self.D), _dp(self.U), nthreads or threads())
        if rc:
            raise ValueError("orc_tables failed")
        self.Dt = self.Ut = None
        if time:
            self.Dt = np.zeros((d_n, d_n), np.float64)
            self.Ut = np.zeros((u_nphi, u_ne), np.float64)
            rc = lib().orc_tables_time(d_n, u_ne, u_nphi, _dp(self.Dt), _dp(self.Ut),
                                       nthreads or threads())
            if rc:
                raise ValueError("orc_tables_time failed")

    def trace(self, u_c, delta, alpha, u_ic, u_oc):
        r = OrcRay()
        lib().orc_trace_table_t(_dp(self.D), _dp(self.Dt), self.d_n, _dp(self.U), _dp(self.Ut),
                                self.u_ne, self.u_nphi, u_c, delta, alpha, u_ic, u_oc,
                                C.byref(r))
        return _ray_dict(r)


def tau_in(e2: float, u: float) -> float:
    return lib().orc_tau_in(e2, u)


def time_singular(u: float) -> float:
    return lib().orc_time_singular(u)


def ellipk(kappa: float) -> float:
    return lib().orc_ellipk(kappa)


def particle_u(particle, a: float, t: float) -> float:
    p = np.ascontiguousarray(particle, np.float64)
    return lib().orc_particle_u(_dp(p), a, t)


def disc_density(particles, ht: float, hr: float, hphi: float) -> float:
    p = np.ascontiguousarray(particles, np.float64).reshape(-1, 3)
    return lib().orc_disc_density(_dp(p), len(p), ht, hr, hphi)


def table_entry_D(n, i, j):
    v, e2, u = C.c_double(), C.c_double(), C.c_double()
    if lib().orc_table_entry_D(n, i, j, C.byref(v), C.byref(e2), C.byref(u)):
        raise ValueError("bad entry")
    return v.value, e2.value, u.value


def table_entry_U(ne, nphi, i, j):
    v, e2, phi = C.c_double(), C.c_double(), C.c_double()
    if lib().orc_table_entry_U(ne, nphi, i, j, C.byref(v), C.byref(e2), C.byref(phi)):
        raise ValueError("bad entry")
    return v.value, e2.value, phi.value


def band_radiance(T: float) -> np.ndarray:
    out = np.zeros(3, np.float64)
    lib().orc_band_radiance(float(T), _dp(out))
    return out


def planck(lam: float, T: float) -> float:
    return lib().orc_planck(lam, T)


def cubemap_bands(dirs: np.ndarray, rgb: np.ndarray, n0: int) -> np.ndarray:
    """FP64 band-colour cubemap texels (all mip levels), shape (texels, 5) = (R, G, B, p_u,
    p_v), from star directions (n, 3) and band intensities (n, 3)."""
    d = np.ascontiguousarray(dirs, np.float32).reshape(-1, 3)
    c = np.ascontiguousarray(rgb, np.float32).reshape(-1, 3)
    tex = np.zeros((lib().orc_cubemap_texels(n0), 5), np.float64)
    fp = C.POINTER(C.c_float)
    rc = lib().orc_cubemap_build_bands(d.ctypes.data_as(fp), c.ctypes.data_as(fp), len(d), n0,
                                       _dp(tex))
    if rc:
        raise ValueError("orc_cubemap_build_bands rejected the stars (%d)" % rc)
    return tex


def cubemap_level_bands(tex: np.ndarray, n0: int, level: int) -> np.ndarray:
    """View of one band-map mip level as (6, nL, nL, 5)."""
    off = sum(6 * (n0 >> l) ** 2 for l in range(level))
    nl = n0 >> level
    return tex[off:off + 6 * nl * nl].reshape(6, nl, nl, 5)


def cubemap(field, n0: int) -> np.ndarray:
    """FP64 cubemap texels (all mip levels concatenated), shape (texels, 4)."""
    n = len(field)
    tex = np.zeros((lib().orc_cubemap_texels(n0), 4), np.float64)
    dirs = np.ascontiguousarray(field.dirs, np.float32)
    inten = np.ascontiguousarray(field.intensity, np.float32)
    temp = np.ascontiguousarray(field.temperature, np.float32)
    fp = C.POINTER(C.c_float)
    rc = lib().orc_cubemap_build(dirs.ctypes.data_as(fp), inten.ctypes.data_as(fp),
                                 temp.ctypes.data_as(fp), n, n0, _dp(tex))
    if rc:
        raise ValueError("orc_cubemap_build failed")
    return tex


def cubemap_level(tex: np.ndarray, n0: int, level: int) -> np.ndarray:
    """View of one mip level as (6, nL, nL, 4)."""
    off = sum(6 * (n0 >> l) ** 2 for l in range(level))
    nl = n0 >> level
    return tex[off:off + 6 * nl * nl].reshape(6, nl, nl, 4)


def area_levels(it: np.ndarray) -> np.ndarray:
    """FP64 area-map levels (all mip levels concatenated), shape (texels, 2) = (I, I T), from
    level-0 (I, T) texels shaped (6, n0, n0, 2)."""
    it = np.ascontiguousarray(it, np.float32)
    n0 = it.shape[1]
    out = np.zeros((lib().orc_area_texels(n0), 2), np.float64)
    if lib().orc_area_build(it.ctypes.data_as(C.POINTER(C.c_float)), n0, _dp(out)):
        raise ValueError("orc_area_build rejected the map")
    return out


def area_level(levels: np.ndarray, n0: int, level: int) -> np.ndarray:
    """View of one area-map level as (6, nL, nL, 2)."""
    off = sum(6 * (n0 >> l) ** 2 for l in range(level))
    nl = n0 >> level
    return levels[off:off + 6 * nl * nl].reshape(6, nl, nl, 2)


def _area_call(fn, levels, n0, d, dw, dh):
    a = [np.ascontiguousarray(x, np.float64) for x in (d, dw, dh)]
    A, B = C.c_double(), C.c_double()
    fn(_dp(levels), n0, _dp(a[0]), _dp(a[1]), _dp(a[2]), C.byref(A), C.byref(B))
    return A.value, B.value


def area_filter(levels, n0, d, dw, dh):
    """Anisotropic filter of the footprint d + w dw + h dh, |w|, |h| <= 1/2: (mean I, mean I T)."""
    return _area_call(lib().orc_area_filter, levels, n0, d, dw, dh)


def area_exact(levels, n0, d, dw, dh):
    """Exact mean of the level-0 map over the same footprint: (mean I, mean I T)."""
    return _area_call(lib().orc_area_exact, levels, n0, d, dw, dh)


def area_levels_bands(rgbx: np.ndarray) -> np.ndarray:
    """FP64 band-map levels, shape (texels, 3) = (R, G, B), from level-0 texels shaped
    (6, n0, n0, 4) = (R, G, B, unused)."""
    rgbx = np.ascontiguousarray(rgbx, np.float32)
    n0 = rgbx.shape[1]
    out = np.zeros((lib().orc_area_texels(n0), 3), np.float64)
    if lib().orc_area_build_bands(rgbx.ctypes.data_as(C.POINTER(C.c_float)), n0, _dp(out)):
        raise ValueError("orc_area_build_bands rejected the map")
    return out


def area_level_bands(levels: np.ndarray, n0: int, level: int) -> np.ndarray:
    """View of one band-map level as (6, nL, nL, 3)."""
    off = sum(6 * (n0 >> l) ** 2 for l in range(level))
    nl = n0 >> level
    return levels[off:off + 6 * nl * nl].reshape(6, nl, nl, 3)


def _bands_call(fn, levels, n0, d, dw, dh):
    a = [np.ascontiguousarray(x, np.float64) for x in (d, dw, dh)]
    out = np.zeros(3)
    fn(_dp(levels), n0, _dp(a[0]), _dp(a[1]), _dp(a[2]), _dp(out))
    return out


def area_filter_bands(levels, n0, d, dw, dh):
    """The anisotropic filter on a band map: mean (R, G, B) over the footprint."""
    return _bands_call(lib().orc_area_filter_bands, levels, n0, d, dw, dh)


def area_exact_bands(levels, n0, d, dw, dh):
    """Exact mean (R, G, B) of the level-0 band map over the footprint."""
    return _bands_call(lib().orc_area_exact_bands, levels, n0, d, dw, dh)


# ---- light of any colour under the Doppler shift (Section 3.4.2) ---------------------------

CSHIFT_DIMS = (128, 128, 128)   # nodes in r, g and log2 D (D from 1/8 to 8)


def absorption(k: int, lam: float) -> float:
    return lib().orc_absorption(k, lam)


def chroma_project(r: float, g: float):
    out = np.zeros(2)
    lib().orc_chroma_project(r, g, _dp(out))
    return float(out[0]), float(out[1])


def band_cct(r: float, g: float) -> float:
    return lib().orc_band_cct(r, g)


def spectrum_of(r: float, g: float):
    """(T, a1, a2) of the spectrum B_T (1 - a1 A1 - a2 A2) chosen for chromaticity (r, g)."""
    out = np.zeros(3)
    lib().orc_spectrum_of(r, g, _dp(out))
    return tuple(float(x) for x in out)


def color_shift(r: float, g: float, D: float) -> np.ndarray:
    """C_b(r, g, D): received band radiances per unit emitted band sum."""
    out = np.zeros(3)
    lib().orc_color_shift(r, g, D, _dp(out))
    return out


def cshift_table(nr: int = 128, ng: int = 128, nd: int = 128, nthreads: int = None) -> np.ndarray:
    """log2 C_b at the table's nodes, shape (nr, ng, nd, 3)."""
    out = np.zeros((nr, ng, nd, 3))
    lib().orc_cshift_table(nr, ng, nd, _dp(out), nthreads or threads())
    return out


def cshift_lookup(tab: np.ndarray, r: float, g: float, D: float) -> np.ndarray:
    nr, ng, nd = tab.shape[:3]
    tab = np.ascontiguousarray(tab, np.float64)
    out = np.zeros(3)
    lib().orc_cshift_lookup(_dp(tab), nr, ng, nd, r, g, D, _dp(out))
    return out


def to_orc_view(v) -> OrcView:
    o = OrcView()
    o.r_s = v.r_s
    o.cam_pos[:] = list(v.cam_pos)
    o.cam_vel[:] = list(v.cam_vel)
    o.cam_rot[:] = list(v.cam_rot)
    o.fov_y = v.fov_y
    o.width, o.height = v.width, v.height
    o.disc_r_in, o.disc_r_out = v.disc_r_in, v.disc_r_out
    o.disc_T_law = v.disc_T_law
    o.disc_T0, o.disc_T_exp = v.disc_T0, v.disc_T_exp
    o.disc_opacity, o.k_disc, o.k_star = v.disc_opacity, v.k_disc, v.k_star
    o.time = getattr(v, "time", 0.0)
    o.disc_density = getattr(v, "disc_density", 0)
    parts = getattr(v, "particles", None)
    if parts is not None:
        arr = np.ascontiguousarray(parts.as_array(), np.float64).reshape(-1, 3)
        o._keep = arr  # keeps the triples alive as long as the record
        o.n_particles = len(arr)
        o.particles = _dp(arr)
    return o


def render_quads(view, quads: np.ndarray, cube: np.ndarray = None, n0: int = 0,
                 tables: Tables = None, nthreads: int = None, march: int = 0,
                 area: np.ndarray = None, area_n0: int = 0, area_exact: bool = False,
                 area_bands: bool = False, ctable: np.ndarray = None,
                 star_bands: bool = False) -> np.ndarray:
    """Render the 4 pixels of every quad (x0, y0); returns a PIXEL_DTYPE array (4 per quad).
    march > 0 replaces TraceRay by ray marching with at most that many steps.  area: levels
    from area_levels (area_exact also fills the exact footprint means), or from
    area_levels_bands with area_bands, whose colour shift reads `ctable` (cshift_table) or,
    if None, is computed exactly."""
    q = np.ascontiguousarray(quads, np.int32)
    nq = q.shape[0]
    out = np.zeros(4 * nq, PIXEL_DTYPE)
    ov = to_orc_view(view)
    ov.star_bands = 1 if star_bands else 0
    if ctable is not None and area is None:
        ov._ct = np.ascontiguousarray(ctable, np.float64)
        ov.ct_n[:] = list(ov._ct.shape[:3])
        ov.ctable = _dp(ov._ct)
    if area is not None:
        ov._area = np.ascontiguousarray(area, np.float64)
        ov.area = _dp(ov._area)
        ov.area_n0 = area_n0
        ov.area_exact = 1 if area_exact else 0
        ov.k_area = getattr(view, "k_area", 1.0)
        ov.area_bands = 1 if area_bands else 0
        if ctable is not None:
            ov._ct = np.ascontiguousarray(ctable, np.float64)
            ov.ct_n[:] = list(ov._ct.shape[:3])
            ov.ctable = _dp(ov._ct)
    if march > 0:
        rc = lib().orc_render_quads_m(C.byref(ov), _dp(cube) if cube is not None else None, n0,
                                      march, q.ctypes.data_as(C.POINTER(C.c_int32)), nq,
                                      out.ctypes.data, nthreads or threads())
        if rc:
            raise ValueError("orc_render_quads_m rejected the view")
        return out
    D = U = Dt = Ut = None
    dn = une = unphi = 0
    if tables is not None:
        D, U, dn, une, unphi = tables.D, tables.U, tables.d_n, tables.u_ne, tables.u_nphi
        Dt, Ut = tables.Dt, tables.Ut
    rc = lib().orc_render_quads_t(C.byref(ov), _dp(cube) if cube is not None else None, n0,
                                  _dp(D), _dp(Dt), dn, _dp(U), _dp(Ut), une, unphi,
                                  q.ctypes.data_as(C.POINTER(C.c_int32)), nq,
                                  out.ctypes.data, nthreads or threads())
    if rc:
        raise ValueError("orc_render_quads rejected the view")
    return out
