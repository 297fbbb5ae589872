"""ctypes binding of libbh (include/bh.h).  Argument marshalling only: every step of the
rendering path runs in the library's HIP kernels.  PyTorch supplies device memory and
streams; pointers are passed as plain integers.

The functions mirror the C entry points one for one (bh_create, bh_precompute_tables, ...);
a few helpers at the end wrap them for torch tensors."""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbh.so")

BH_OK, BH_EINVAL, BH_ENOMEM, BH_EDEVICE, BH_EAGAIN, BH_ENOTFOUND, BH_ECANCELED = range(7)
BH_TAB_FP32, BH_TAB_FP64_BAND, BH_TAB_FP64_ALL = 0, 1, 2
BH_TEXEL_FP16, BH_TEXEL_FP32 = 0, 1
BH_T_POWER, BH_T_PAPER = 0, 1
BH_AOV_CAPTURED, BH_AOV_CROSS0, BH_AOV_CROSS1 = 1, 2, 4
BH_AOV_STAR_ZEROED, BH_AOV_DEGENERATE, BH_AOV_UNFINISHED = 8, 16, 32
BH_DENSITY_UNIFORM, BH_DENSITY_PARTICLES = 0, 1

# every symbol include/bh.h declares
EXPORTS = [
    "bh_create", "bh_destroy", "bh_last_error", "bh_bytes_in_use", "bh_release",
    "bh_precompute_tables", "bh_tables_download", "bh_tables_download_time", "bh_release_tables",
    "bh_create_particles", "bh_release_particles",
    "bh_bloom_create", "bh_bloom_apply", "bh_bloom_release", "bh_bloom_apply_display",
    "bh_tonemap",
    "bh_build_stars", "bh_build_star_bands", "bh_stars_download", "bh_release_stars",
    "bh_build_area", "bh_build_area_bands", "bh_color_shift_table_download",
    "bh_area_download", "bh_release_area",
    "bh_render", "bh_render_march", "bh_render_batch", "bh_render_batch_noalloc",
    "bh_tile_config_count", "bh_tile_config_get",
    "bh_set_tile_config", "bh_set_batch_form", "bh_autotune",
    "bh_serve_start", "bh_submit", "bh_poll", "bh_ticket_image", "bh_ticket_free",
    "bh_serve_drain",
    "bh_trace_rays", "bh_trace_rays_timed", "bh_march_rays", "bh_footprint_texels", "bh_probe_l2_read", "bh_band_table_info", "bh_band_table_download", "bh_band_eval",
]


class BhError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libbh status %d: %s" % (status, msg))
        self.status = status


class TableParams(C.Structure):
    _fields_ = [("d_n", C.c_int32), ("u_ne", C.c_int32), ("u_nphi", C.c_int32),
                ("precision", C.c_int32), ("fp64_band", C.c_double), ("step", C.c_double)]


class View(C.Structure):
    _fields_ = [("r_s", C.c_double), ("cam_pos", C.c_double * 3), ("cam_vel", C.c_double * 3),
                ("cam_rot", C.c_double * 9), ("fov_y", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32),
                ("disc_r_in", C.c_double), ("disc_r_out", C.c_double),
                ("disc_T_law", C.c_int32), ("pad0", C.c_int32),
                ("disc_T0", C.c_double), ("disc_T_exp", C.c_double),
                ("disc_opacity", C.c_double), ("k_disc", C.c_double), ("k_star", C.c_double),
                ("stars", C.c_void_p), ("disc_density", C.c_int32), ("pad1", C.c_int32),
                ("time", C.c_double), ("particles", C.c_void_p),
                ("area", C.c_void_p), ("k_area", C.c_double)]


class TileConfig(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("waves", C.c_int32),
                ("ppt", C.c_int32)]


class ServeParams(C.Structure):
    _fields_ = [("max_queue", C.c_int32), ("max_inflight_launches", C.c_int32),
                ("max_tiles_per_launch", C.c_int64)]


_lib = None


def lib():
    """Load libbh.so; raises if the library has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbh.so is not built: run __graft_entry__.build() "
                              "(or python paper_2010_08735_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        sig = {
            "bh_create": ([C.c_int, u64, C.POINTER(vp)], i32),
            "bh_destroy": ([vp], None),
            "bh_last_error": ([vp], C.c_char_p),
            "bh_release": ([vp], i32),
            "bh_bytes_in_use": ([vp], u64),
            "bh_precompute_tables": ([vp, C.POINTER(TableParams), vp, C.POINTER(vp)], i32),
            "bh_tables_download": ([vp, vp, vp], i32),
            "bh_tables_download_time": ([vp, vp, vp], i32),
            "bh_create_particles": ([vp, vp, i32, C.POINTER(vp)], i32),
            "bh_release_particles": ([vp], i32),
            "bh_release_tables": ([vp], i32),
            "bh_build_stars": ([vp, vp, vp, vp, i64, i32, i32, vp, C.POINTER(vp)], i32),
            "bh_build_star_bands": ([vp, vp, vp, i64, i32, i32, vp, C.POINTER(vp)], i32),
            "bh_stars_download": ([vp, i32, vp], i32),
            "bh_release_stars": ([vp], i32),
            "bh_build_area": ([vp, vp, i32, vp, C.POINTER(vp)], i32),
            "bh_build_area_bands": ([vp, vp, i32, vp, C.POINTER(vp)], i32),
            "bh_color_shift_table_download": ([vp, vp], i32),
            "bh_area_download": ([vp, i32, vp], i32),
            "bh_release_area": ([vp], i32),
            "bh_render": ([vp, vp, C.POINTER(View), vp, vp, vp], i32),
            "bh_render_batch": ([vp, vp, C.POINTER(View), i32, C.POINTER(vp), vp], i32),
            "bh_render_batch_noalloc": ([vp, vp, C.POINTER(View), i32, C.POINTER(vp), vp], i32),
            "bh_set_batch_form": ([vp, i32], i32),
            "bh_tile_config_count": ([], i32),
            "bh_tile_config_get": ([i32, C.POINTER(TileConfig)], i32),
            "bh_set_tile_config": ([vp, i32], i32),
            "bh_autotune": ([vp, vp, C.POINTER(View), i32, C.POINTER(vp), i32,
                             C.POINTER(i32), C.POINTER(C.c_float)], i32),
            "bh_serve_start": ([vp, C.POINTER(ServeParams)], i32),
            "bh_submit": ([vp, vp, C.POINTER(View), vp, C.POINTER(u64)], i32),
            "bh_poll": ([vp, u64, C.POINTER(i32), C.POINTER(dp)], i32),
            "bh_ticket_image": ([vp, u64, C.POINTER(vp)], i32),
            "bh_ticket_free": ([vp, u64], i32),
            "bh_serve_drain": ([vp], i32),
            "bh_trace_rays": ([vp, vp, vp, i64, vp, vp], i32),
            "bh_trace_rays_timed": ([vp, vp, vp, i64, vp, vp, vp], i32),
            "bh_march_rays": ([vp, vp, i64, i32, vp, vp], i32),
            "bh_bloom_create": ([vp, i32, i32, i32, C.POINTER(vp)], i32),
            "bh_bloom_apply": ([vp, C.POINTER(C.c_float), vp, vp, vp], i32),
            "bh_bloom_release": ([vp], i32),
            "bh_bloom_apply_display": ([vp, C.POINTER(C.c_float), C.c_float, vp, vp, vp], i32),
            "bh_tonemap": ([vp, vp, vp, i32, i32, C.c_float, vp], i32),
            "bh_render_march": ([vp, C.POINTER(View), i32, vp, vp, vp], i32),
            "bh_footprint_texels": ([vp, vp, C.POINTER(View), vp, C.POINTER(u64), C.POINTER(u64)], i32),
            "bh_probe_l2_read": ([vp, i64, i32, C.POINTER(C.c_double)], i32),
            "bh_band_table_info": ([vp, C.POINTER(i32), C.POINTER(C.c_float),
                                    C.POINTER(C.c_float)], i32),
            "bh_band_table_download": ([vp, vp], i32),
            "bh_band_eval": ([vp, vp, i64, vp, vp], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(status):
    if status != BH_OK:
        msg = lib().bh_last_error(None)
        raise BhError(status, msg.decode() if msg else "")
    return status


# ---- thin wrappers with the C names ------------------------------------------------------

def bh_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    out = C.c_void_p()
    _check(lib().bh_create(device, hbm_budget_bytes, C.byref(out)))
    return out.value


def bh_destroy(ctx: int) -> None:
    lib().bh_destroy(ctx)


def bh_bytes_in_use(ctx: int) -> int:
    return lib().bh_bytes_in_use(ctx)


def bh_precompute_tables(ctx, d_n=512, u_ne=64, u_nphi=32, precision=BH_TAB_FP64_BAND,
                         fp64_band=0.05, step=0.0, stream=None) -> int:
    p = TableParams(d_n, u_ne, u_nphi, precision, fp64_band, step)
    out = C.c_void_p()
    _check(lib().bh_precompute_tables(ctx, C.byref(p), stream, C.byref(out)))
    return out.value


def bh_tables_download(tables, host_D_ptr, host_U_ptr) -> None:
    _check(lib().bh_tables_download(tables, host_D_ptr, host_U_ptr))


def bh_tables_download_time(tables, host_Dt_ptr, host_Ut_ptr) -> None:
    _check(lib().bh_tables_download_time(tables, host_Dt_ptr, host_Ut_ptr))


def bh_release_tables(tables) -> None:
    _check(lib().bh_release_tables(tables))


def bh_create_particles(ctx, triples) -> int:
    """triples: (n, 3) array-like of (r_peri, r_apo, phi0), copied by the library."""
    import numpy as np
    arr = np.ascontiguousarray(triples, np.float64).reshape(-1, 3)
    out = C.c_void_p()
    _check(lib().bh_create_particles(ctx, arr.ctypes.data, len(arr), C.byref(out)))
    return out.value


def bh_release_particles(particles) -> None:
    _check(lib().bh_release_particles(particles))


def bh_release(handle) -> None:
    """Release any handle (tables, star map, area map, particles, bloom pyramid)."""
    _check(lib().bh_release(handle))


def bh_build_stars(ctx, dir_ptr, inten_ptr, temp_ptr, n, face_size, texel_format=BH_TEXEL_FP16,
                   stream=None) -> int:
    out = C.c_void_p()
    _check(lib().bh_build_stars(ctx, dir_ptr, inten_ptr, temp_ptr, n, face_size, texel_format,
                                stream, C.byref(out)))
    return out.value


def bh_build_star_bands(ctx, dir_ptr, rgb_ptr, n, face_size, texel_format=BH_TEXEL_FP16,
                        stream=None) -> int:
    out = C.c_void_p()
    _check(lib().bh_build_star_bands(ctx, dir_ptr, rgb_ptr, n, face_size, texel_format, stream,
                                     C.byref(out)))
    return out.value


def bh_stars_download(stars, level, host_ptr) -> None:
    _check(lib().bh_stars_download(stars, level, host_ptr))


def bh_release_stars(stars) -> None:
    _check(lib().bh_release_stars(stars))


def bh_build_area(ctx, texels_ptr, face_size, stream=None) -> int:
    out = C.c_void_p()
    _check(lib().bh_build_area(ctx, texels_ptr, face_size, stream, C.byref(out)))
    return out.value


def bh_build_area_bands(ctx, rgbx_ptr, face_size, stream=None) -> int:
    out = C.c_void_p()
    _check(lib().bh_build_area_bands(ctx, rgbx_ptr, face_size, stream, C.byref(out)))
    return out.value


BH_CSHIFT_N = 128


def bh_color_shift_table_download(ctx, host_ptr) -> None:
    _check(lib().bh_color_shift_table_download(ctx, host_ptr))


def bh_area_download(area, level, host_ptr) -> None:
    _check(lib().bh_area_download(area, level, host_ptr))


def bh_release_area(area) -> None:
    _check(lib().bh_release_area(area))


def bh_render(ctx, tables, view: View, out_ptr, aov_ptr=None, stream=None) -> None:
    _check(lib().bh_render(ctx, tables, C.byref(view), out_ptr, aov_ptr, stream))


def bh_render_march(ctx, view: View, max_steps: int, out_ptr, aov_ptr=None, stream=None) -> None:
    _check(lib().bh_render_march(ctx, C.byref(view), max_steps, out_ptr, aov_ptr, stream))


def bh_render_batch(ctx, tables, views, out_ptrs, stream=None) -> None:
    n = len(views)
    arr = (View * n)(*views)
    outs = (C.c_void_p * n)(*out_ptrs)
    _check(lib().bh_render_batch(ctx, tables, arr, n, outs, stream))


def bh_render_batch_noalloc(ctx, tables, views, out_ptrs, stream=None) -> None:
    n = len(views)
    arr = (View * n)(*views)
    outs = (C.c_void_p * n)(*out_ptrs)
    _check(lib().bh_render_batch_noalloc(ctx, tables, arr, n, outs, stream))


def bh_set_batch_form(ctx, persistent: int) -> None:
    _check(lib().bh_set_batch_form(ctx, persistent))


def bh_tile_config_count() -> int:
    return lib().bh_tile_config_count()


def bh_tile_config_get(i) -> TileConfig:
    t = TileConfig()
    _check(lib().bh_tile_config_get(i, C.byref(t)))
    return t


def bh_set_tile_config(ctx, i) -> None:
    _check(lib().bh_set_tile_config(ctx, i))


def bh_autotune(ctx, tables, views, out_ptrs, reps=3):
    n = len(views)
    arr = (View * n)(*views)
    outs = (C.c_void_p * n)(*out_ptrs)
    best = C.c_int32()
    ms = (C.c_float * (2 * bh_tile_config_count()))()
    _check(lib().bh_autotune(ctx, tables, arr, n, outs, reps, C.byref(best), ms))
    return best.value, list(ms)


def bh_serve_start(ctx, max_queue=0, max_inflight_launches=0, max_tiles_per_launch=0) -> None:
    p = ServeParams(max_queue, max_inflight_launches, max_tiles_per_launch)
    _check(lib().bh_serve_start(ctx, C.byref(p)))


def bh_submit(ctx, tables, view: View, out_ptr=None) -> int:
    t = C.c_uint64()
    _check(lib().bh_submit(ctx, tables, C.byref(view), out_ptr, C.byref(t)))
    return t.value


def bh_poll(ctx, ticket):
    done, lat = C.c_int32(), C.c_double()
    st = lib().bh_poll(ctx, ticket, C.byref(done), C.byref(lat))
    _check(st)
    return bool(done.value), lat.value


def bh_ticket_image(ctx, ticket) -> int:
    p = C.c_void_p()
    _check(lib().bh_ticket_image(ctx, ticket, C.byref(p)))
    return p.value


def bh_ticket_free(ctx, ticket) -> None:
    _check(lib().bh_ticket_free(ctx, ticket))


def bh_serve_drain(ctx) -> None:
    _check(lib().bh_serve_drain(ctx))


def bh_trace_rays(ctx, tables, rays_ptr, n, out_ptr, stream=None) -> None:
    _check(lib().bh_trace_rays(ctx, tables, rays_ptr, n, out_ptr, stream))


def bh_trace_rays_timed(ctx, tables, rays_ptr, n, out_ptr, out_time_ptr, stream=None) -> None:
    _check(lib().bh_trace_rays_timed(ctx, tables, rays_ptr, n, out_ptr, out_time_ptr, stream))


def bh_bloom_create(ctx, width: int, height: int, levels: int) -> int:
    out = C.c_void_p()
    _check(lib().bh_bloom_create(ctx, width, height, levels, C.byref(out)))
    return out.value


def bh_bloom_apply(b, weights, in_ptr, out_ptr, stream=None) -> None:
    """weights: w_0 .. w_levels (the library reads levels + 1 of them)."""
    _check(lib().bh_bloom_apply(b, _bloom_weights(weights), in_ptr, out_ptr, stream))


def bh_bloom_release(b) -> None:
    _check(lib().bh_bloom_release(b))


def _bloom_weights(weights):
    if len(weights) > 17:
        raise ValueError("at most 17 bloom weights")
    return (C.c_float * 17)(*[float(x) for x in weights])  # zero-padded to the largest count


def bh_bloom_apply_display(b, weights, exposure, in_ptr, out_ptr, stream=None) -> None:
    """Glare pass, then the display encoding of its result into out_ptr (uint32 per pixel)."""
    _check(lib().bh_bloom_apply_display(b, _bloom_weights(weights), float(exposure), in_ptr,
                                        out_ptr, stream))


def bh_tonemap(ctx, in_ptr, out_ptr, width: int, height: int, exposure, stream=None) -> None:
    """Display encoding of a linear RGBA32F image into uint32 pixels (bytes R, G, B, 255)."""
    _check(lib().bh_tonemap(ctx, in_ptr, out_ptr, width, height, float(exposure), stream))


def bh_march_rays(ctx, rays_ptr, n, max_steps, out_ptr, stream=None) -> None:
    _check(lib().bh_march_rays(ctx, rays_ptr, n, max_steps, out_ptr, stream))


def bh_footprint_texels(ctx, tables, view: View, out_ptr):
    """(distinct star-map texels the footprints visit, bytes all pixels request)"""
    n, b = C.c_uint64(), C.c_uint64()
    _check(lib().bh_footprint_texels(ctx, tables, C.byref(view), out_ptr, C.byref(n), C.byref(b)))
    return n.value, b.value


def bh_probe_l2_read(ctx, window_bytes=2 << 20, reps=20) -> float:
    """bytes per second of streaming reads of a buffer held in L2"""
    r = C.c_double()
    _check(lib().bh_probe_l2_read(ctx, window_bytes, reps, C.byref(r)))
    return r.value


def bh_band_table_info(ctx):
    n, x0, dx = C.c_int32(), C.c_float(), C.c_float()
    _check(lib().bh_band_table_info(ctx, C.byref(n), C.byref(x0), C.byref(dx)))
    return n.value, x0.value, dx.value


def bh_band_table_download(ctx, host_ptr) -> None:
    _check(lib().bh_band_table_download(ctx, host_ptr))


def bh_band_eval(ctx, temps_ptr, n, out_ptr, stream=None) -> None:
    _check(lib().bh_band_eval(ctx, temps_ptr, n, out_ptr, stream))


# ---- helpers ------------------------------------------------------------------------------

def make_view(v, stars=None, particles=None, area=None) -> View:
    """bh View record from a scenes.View (same field names); `particles` is the handle from
    bh_create_particles for a view with a particle disc, `area` one from bh_build_area."""
    o = View()
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
    o.stars = stars
    o.disc_density = getattr(v, "disc_density", BH_DENSITY_UNIFORM)
    o.time = getattr(v, "time", 0.0)
    o.particles = particles
    o.area = area
    o.k_area = getattr(v, "k_area", 1.0)
    return o


def current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream
