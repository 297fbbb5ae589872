"""Seeded synthetic inputs for the black-hole beam tracer.

Both the HIP library and the FP64 oracle consume the arrays produced here; this module
only draws random numbers and lays out input records.  It contains none of the
renderer's arithmetic (no geodesics, tables, Doppler factors, shading or filtering).

Units: lengths in Schwarzschild radii (r_s = 1) unless a view says otherwise, speeds in
units of c, angles in radians, temperatures in kelvin.

Input recipes (all RNG draws use numpy's PCG64 ``default_rng(seed)`` in the order listed):

* star field: z ~ U(-1, 1), azimuth ~ U(0, 2 pi), intensity = 10**U(-4, 0),
  temperature ~ U(3000, 12000) K, each drawn as a whole array in that order;
* camera orientation: the camera looks at the apparent direction of the hole centre
  (the hole direction carried from the static frame into the moving camera's frame), with
  the image "up" axis the projection of +z (or +x when the camera looks along z);
* disc particles (animated disc): mid radius ~ U(r_in + 1, r_out - 1), relative
  half-width of the radial excursion ~ U(0, 0.05), initial phase ~ U(0, 2 pi), each drawn
  as a whole array in that order; pericentre = mid (1 - w), apocentre = mid (1 + w);
* area-source sky (nebulae): `blobs` Gaussian patches with centre z ~ U(-1, 1), azimuth
  ~ U(0, 2 pi), angular width sigma ~ U(sigma_lo, sigma_hi) rad, peak radiance
  10**U(-1, 0), temperature ~ U(3000, 15000) K, each drawn as a whole array in that order,
  over a floor of radiance 0.02 at 6000 K; texel (face, x, y) of the level-0 map holds
  the radiance I and the radiance-weighted temperature T at its centre direction (face
  2k + (d_k < 0), U = d_{(k+1)%3} / |d_k|, V = d_{(k+2)%3} / |d_k|, centre at
  U = (x + 1/2) 2 / n0 - 1, V = (y + 1/2) 2 / n0 - 1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

T_LAW_POWER = 0   # T' = T0 * (r' / (3 r_s)) ** T_exp
T_LAW_PAPER = 1   # T'^4 proportional to u^3 (1 - sqrt(3u)), peak value T0
DENSITY_UNIFORM = 0
DENSITY_PARTICLES = 1


@dataclasses.dataclass
class View:
    """One camera + disc configuration (mirrors ``bh_view`` of include/bh.h)."""
    cam_pos: Tuple[float, float, float]
    cam_vel: Tuple[float, float, float]
    cam_rot: Tuple[float, ...]          # 9 values, rows e_w, e_h, e_d (camera looks along -e_d)
    width: int
    height: int
    fov_y: float = math.radians(60.0)
    r_s: float = 1.0
    disc_r_in: float = 3.0
    disc_r_out: float = 12.0
    disc_T_law: int = T_LAW_POWER
    disc_T0: float = 1.0e4
    disc_T_exp: float = -0.75
    disc_opacity: float = 1.0
    k_disc: float = 1.0e-7
    k_star: float = 1.0
    # animated disc: 0 = uniform density, 1 = procedural particles at the camera time
    disc_density: int = DENSITY_UNIFORM
    time: float = 0.0
    particles: Optional["ParticleSet"] = None
    k_area: float = 1.0                 # exposure of an area-source map, when one is given

    def pixels(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class ParticleSet:
    """Disc particles: pericentre and apocentre radii (units of r_s) and initial phase
    (radians), float64 arrays of equal length."""
    r_peri: np.ndarray
    r_apo: np.ndarray
    phi0: np.ndarray
    seed: int

    def __len__(self) -> int:
        return len(self.phi0)

    def as_array(self) -> np.ndarray:
        """(n, 3) triples (r_peri, r_apo, phi0)."""
        return np.stack([self.r_peri, self.r_apo, self.phi0], axis=1)


def disc_particles(n: int, r_in: float, r_out: float, seed: int) -> ParticleSet:
    rng = np.random.default_rng(seed)
    mid = rng.uniform(r_in + 1.0, r_out - 1.0, n)
    w = rng.uniform(0.0, 0.05, n)
    phi0 = rng.uniform(0.0, 2.0 * math.pi, n)
    return ParticleSet(r_peri=mid * (1.0 - w), r_apo=mid * (1.0 + w), phi0=phi0, seed=seed)


@dataclasses.dataclass
class StarField:
    """Point stars: unit directions (n,3), intensities (n,) and temperatures (n,), float32."""
    dirs: np.ndarray
    intensity: np.ndarray
    temperature: np.ndarray
    seed: int

    def __len__(self) -> int:
        return int(self.intensity.shape[0])


def star_field(n: int, seed: int) -> StarField:
    rng = np.random.default_rng(seed)
    z = rng.uniform(-1.0, 1.0, n)
    az = rng.uniform(0.0, 2.0 * math.pi, n)
    inten = 10.0 ** rng.uniform(-4.0, 0.0, n)
    temp = rng.uniform(3000.0, 12000.0, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    dirs = np.stack([s * np.cos(az), s * np.sin(az), z], axis=1)
    return StarField(dirs.astype(np.float32), inten.astype(np.float32),
                     temp.astype(np.float32), seed)


def star_field_bands(n: int, seed: int):
    """A seeded field of stars of any colour: directions (n, 3) and band intensities (n, 3),
    float32.  Directions and the 4-decade log-uniform brightness as `star_field`; each
    star's colour has chromaticity r ~ U(0.2, 0.5), g ~ U(0.22, 0.42), b = 1 - r - g (on
    and off the blackbody locus), so its bands are I (r, g, b)."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(-1.0, 1.0, n)
    az = rng.uniform(0.0, 2.0 * math.pi, n)
    inten = 10.0 ** rng.uniform(-4.0, 0.0, n)
    r = rng.uniform(0.2, 0.5, n)
    g = rng.uniform(0.22, 0.42, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    dirs = np.stack([s * np.cos(az), s * np.sin(az), z], axis=1)
    rgb = inten[:, None] * np.stack([r, g, 1.0 - r - g], axis=1)
    return dirs.astype(np.float32), rgb.astype(np.float32)


def area_map(n0: int, seed: int, blobs: int = 24, sigma_lo: float = 0.10,
             sigma_hi: float = 0.35) -> np.ndarray:
    """Level-0 texels of an area-source cube map, float32 (6, n0, n0, 2) = (I, T)."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(-1.0, 1.0, blobs)
    az = rng.uniform(0.0, 2.0 * math.pi, blobs)
    sig = rng.uniform(sigma_lo, sigma_hi, blobs)
    peak = 10.0 ** rng.uniform(-1.0, 0.0, blobs)
    temp = rng.uniform(3000.0, 15000.0, blobs)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    centres = np.stack([s * np.cos(az), s * np.sin(az), z], axis=1)
    c = (np.arange(n0) + 0.5) * (2.0 / n0) - 1.0
    uu, vv = np.meshgrid(c, c, indexing="xy")          # [y, x]
    out = np.zeros((6, n0, n0, 2), np.float32)
    for f in range(6):
        k, sgn = f // 2, (-1.0 if f % 2 else 1.0)
        d = np.zeros((n0, n0, 3))
        d[..., k] = sgn
        d[..., (k + 1) % 3] = uu
        d[..., (k + 2) % 3] = vv
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        ang = np.arccos(np.clip(d @ centres.T, -1.0, 1.0))  # (n0, n0, blobs)
        g = peak * np.exp(-0.5 * (ang / sig) ** 2)
        I = 0.02 + g.sum(-1)
        IT = 0.02 * 6000.0 + (g * temp).sum(-1)
        out[f, ..., 0] = I
        out[f, ..., 1] = IT / I
    return out


def area_map_bands(n0: int, seed: int, blobs: int = 24, sigma_lo: float = 0.10,
                   sigma_hi: float = 0.35) -> np.ndarray:
    """Level-0 texels of a band-colour sky, float32 (6, n0, n0, 4) = (R, G, B, 0): the same
    Gaussian patches as `area_map`, each with a colour of chromaticity r ~ U(0.2, 0.5),
    g ~ U(0.22, 0.42), b = 1 - r - g (colours on and off the blackbody locus), over a
    floor of 0.02 in each band."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(-1.0, 1.0, blobs)
    az = rng.uniform(0.0, 2.0 * math.pi, blobs)
    sig = rng.uniform(sigma_lo, sigma_hi, blobs)
    peak = 10.0 ** rng.uniform(-1.0, 0.0, blobs)
    r = rng.uniform(0.2, 0.5, blobs)
    g = rng.uniform(0.22, 0.42, blobs)
    col = np.stack([r, g, 1.0 - r - g], axis=1)          # (blobs, 3)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    centres = np.stack([s * np.cos(az), s * np.sin(az), z], axis=1)
    c = (np.arange(n0) + 0.5) * (2.0 / n0) - 1.0
    uu, vv = np.meshgrid(c, c, indexing="xy")          # [y, x]
    out = np.zeros((6, n0, n0, 4), np.float32)
    for f in range(6):
        k, sgn = f // 2, (-1.0 if f % 2 else 1.0)
        d = np.zeros((n0, n0, 3))
        d[..., k] = sgn
        d[..., (k + 1) % 3] = uu
        d[..., (k + 2) % 3] = vv
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        ang = np.arccos(np.clip(d @ centres.T, -1.0, 1.0))  # (n0, n0, blobs)
        gw = peak * np.exp(-0.5 * (ang / sig) ** 2)
        out[f, ..., :3] = 0.02 + gw @ col
    return out


# ----------------------------------------------------------------------------------------
# camera placement helpers (input recipe only)

def spherical_position(r: float, theta: float, phi: float) -> np.ndarray:
    return r * np.array([math.sin(theta) * math.cos(phi),
                         math.sin(theta) * math.sin(phi),
                         math.cos(theta)])


def _unit(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v)


def azimuthal_direction(pos: np.ndarray) -> np.ndarray:
    """Unit vector along increasing azimuth at ``pos`` (z-axis positions fall back to +y)."""
    t = np.array([-pos[1], pos[0], 0.0])
    n = np.linalg.norm(t)
    return t / n if n > 1e-12 else np.array([0.0, 1.0, 0.0])


def apparent_hole_direction(pos: np.ndarray, vel: np.ndarray) -> np.ndarray:
    """Direction of the hole centre as seen in the frame of a camera moving at ``vel``.

    Recipe for aiming views; the renderer and the oracle do their own frame changes."""
    n_s = -_unit(pos)
    v2 = float(vel @ vel)
    if v2 < 1e-30:
        return n_s
    v = math.sqrt(v2)
    vh = vel / v
    g = 1.0 / math.sqrt(1.0 - v2)
    nv = float(n_s @ vh)
    n_c = (n_s + ((g - 1.0) * nv + g * v) * vh) / (g * (1.0 + v * nv))
    return _unit(n_c)


def look_rotation(look: np.ndarray) -> Tuple[float, ...]:
    """Rows e_w, e_h, e_d for a camera looking along ``look`` with +z (else +x) as up."""
    e_d = -_unit(look)
    up = np.array([0.0, 0.0, 1.0])
    if abs(float(up @ e_d)) > 0.999:
        up = np.array([1.0, 0.0, 0.0])
    e_h = _unit(up - (up @ e_d) * e_d)
    e_w = np.cross(e_h, e_d)
    return tuple(float(x) for x in np.concatenate([e_w, e_h, e_d]))


def aimed_view(pos, vel, width, height, **kw) -> View:
    pos = np.asarray(pos, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    rot = look_rotation(apparent_hole_direction(pos, vel))
    return View(cam_pos=tuple(float(x) for x in pos), cam_vel=tuple(float(x) for x in vel),
                cam_rot=rot, width=int(width), height=int(height), **kw)


# ----------------------------------------------------------------------------------------
# freely falling cameras (Appendix C, "Position"); units r_s = 1, u = 1 / r

@dataclasses.dataclass
class OrbitState:
    """Camera on a timelike geodesic in its orbital plane: coordinate time t, radius r,
    in-plane angle psi, and their proper-time rates (Appendix C).  Arrays of one shape."""
    tau: np.ndarray
    t: np.ndarray
    r: np.ndarray
    psi: np.ndarray
    dr: np.ndarray       # dr / dtau
    dt: np.ndarray       # dt / dtau = e / (1 - u)
    dpsi: np.ndarray     # dpsi / dtau = l u^2


def orbit_constants(r0: float, delta0: float, v0: float) -> Tuple[float, float]:
    """Energy e and angular momentum l per unit mass of the geodesic that starts at radius
    r0 with speed v0 (measured by the static observer there) in the direction delta0,
    moving towards increasing psi (Appendix C): e^2 from the Lorentz factor against the
    static observer, l^2 from tan(delta) = r dpsi / dr.  delta is the coordinate angle
    from the outward radial direction; the static observer sees the angle
    atan(sqrt(1 - u) tan(delta)), as radial lengths are stretched by 1 / sqrt(1 - u)."""
    u0 = 1.0 / r0
    if not (r0 > 1.0 and 0.0 <= v0 < 1.0 and 0.0 <= delta0 <= math.pi):
        raise ValueError("need r0 > 1, 0 <= v0 < 1, 0 <= delta0 <= pi")
    e2 = (1.0 - u0) / (1.0 - v0 * v0)
    s = math.sin(delta0)
    if s == 0.0 or v0 == 0.0:
        return math.sqrt(e2), 0.0
    cot = math.cos(delta0) / s
    l2 = (e2 + u0 - 1.0) / (u0 * u0 * (1.0 - u0 + cot * cot))
    return math.sqrt(e2), math.sqrt(l2)


def camera_orbit(r0: float, delta0: float, v0: float, taus, step: float = 0.5) -> OrbitState:
    """States of the Appendix C camera at the proper times `taus` (ascending, from 0).

    r follows the second-order radial equation d2r/dtau2 = (2 l^2 u^3 - 3 l^2 u^4 - u^2)/2,
    t and psi the first integrals dt/dtau = e/(1-u) and dpsi/dtau = l u^2; one classical
    RK4 integration of (t, r, dr/dtau, psi) in proper time, with steps of at most `step`,
    stopped at each requested time.  Raises if the camera reaches r <= 1.05."""
    taus = np.asarray(taus, np.float64)
    if taus.ndim != 1 or (taus.size and (taus[0] < 0 or np.any(np.diff(taus) < 0))):
        raise ValueError("taus must be ascending and non-negative")
    e, l = orbit_constants(r0, delta0, v0)
    u0 = 1.0 / r0
    if l > 0.0:
        dr0 = l * u0 * math.cos(delta0) / math.sin(delta0)   # tan(delta) = r dpsi / dr
    else:
        dr0 = math.copysign(math.sqrt(max(0.0, e * e + u0 - 1.0)), math.cos(delta0))

    def f(y):
        t, r, v, psi = y
        u = 1.0 / r
        return (e / (1.0 - u), v, 0.5 * (2.0 * l * l * u ** 3 - 3.0 * l * l * u ** 4 - u * u),
                l * u * u)

    def rk4(y, h):
        k1 = f(y)
        k2 = f(tuple(a + 0.5 * h * b for a, b in zip(y, k1)))
        k3 = f(tuple(a + 0.5 * h * b for a, b in zip(y, k2)))
        k4 = f(tuple(a + h * b for a, b in zip(y, k3)))
        return tuple(a + h / 6.0 * (p + 2.0 * q + 2.0 * w + z)
                     for a, p, q, w, z in zip(y, k1, k2, k3, k4))

    y, now = (0.0, float(r0), dr0, 0.0), 0.0
    out = np.empty((taus.size, 4))
    for k, target in enumerate(taus):
        while now < target:
            h = min(step, target - now)
            y = rk4(y, h)
            now = target if h == target - now else now + h
            if y[1] <= 1.05:
                raise ValueError("the camera falls into the hole at tau = %.3f" % now)
        out[k] = y
    u = 1.0 / out[:, 1]
    return OrbitState(taus, out[:, 0], out[:, 1], out[:, 3], out[:, 2], e / (1.0 - u),
                      l * u * u)


def orbit_position_velocity(st: OrbitState, chi: float) -> Tuple[np.ndarray, np.ndarray]:
    """Cartesian position r (cos chi cos psi, sin psi, sin chi cos psi) of the orbit of
    inclination chi, and the camera's velocity measured by the static observer, from its
    radial and in-plane components (Appendix C, camera speed in the static orthonormal
    basis) along the radial and psi unit vectors."""
    c, s = math.cos(chi), math.sin(chi)
    cp, sp = np.cos(st.psi), np.sin(st.psi)
    rhat = np.stack([c * cp, sp, s * cp], axis=-1)
    phat = np.stack([-c * sp, cp, -s * sp], axis=-1)
    u = 1.0 / st.r
    v_r = st.dr / ((1.0 - u) * st.dt)
    v_psi = st.dpsi / (u * np.sqrt(1.0 - u) * st.dt)
    return st.r[:, None] * rhat, v_r[:, None] * rhat + v_psi[:, None] * phat


def orbit_views(r0: float, delta0: float, v0: float, chi: float, taus, width: int, height: int,
                **kw) -> List[View]:
    """Frames of a freely falling camera (Appendix C) at proper times `taus`, each aimed at
    the hole's apparent direction; the view's `time` is the camera's coordinate time t,
    which drives the animated disc."""
    st = camera_orbit(r0, delta0, v0, taus)
    pos, vel = orbit_position_velocity(st, chi)
    out = []
    for k in range(len(st.tau)):
        v = aimed_view(pos[k], vel[k], width, height, **kw)
        v.time = float(st.t[k])
        out.append(v)
    return out


# ----------------------------------------------------------------------------------------
# the workloads

def small_static_view() -> View:
    """128x128, static camera at r = 15, 80 deg from the disc normal, disc [3, 12]."""
    pos = spherical_position(15.0, math.radians(80.0), 0.0)
    return aimed_view(pos, np.zeros(3), 128, 128, disc_r_in=3.0, disc_r_out=12.0)


def animated_disc_view(width: int = 128, height: int = 128, n_particles: int = 24,
                       time: float = 1000.0, seed: int = 7) -> View:
    """The small static view with the paper's temperature law and a particle disc seen at
    camera time `time` (disc [4, 12] so particle radii stay outside r = 3)."""
    v = small_static_view()
    v.width, v.height = width, height
    v.disc_r_in, v.disc_r_out = 4.0, 12.0
    v.disc_T_law = T_LAW_PAPER
    v.disc_T0 = 8000.0
    v.disc_density = DENSITY_PARTICLES
    v.disc_opacity = 0.5
    v.time = time
    v.particles = disc_particles(n_particles, v.disc_r_in, v.disc_r_out, seed)
    return v


def boosted_orbit_view(width: int = 1920, height: int = 1080) -> View:
    """Camera at r = 6, 85 deg from the disc normal, moving at 0.9c along +azimuth."""
    pos = spherical_position(6.0, math.radians(85.0), 0.0)
    vel = 0.9 * azimuthal_direction(pos)
    return aimed_view(pos, vel, width, height, disc_r_in=3.0, disc_r_out=20.0)


BATCH_RESOLUTIONS = ((256, 256), (512, 512), (1024, 1024), (1920, 1080), (2048, 2048))


def batch_views(n: int = 64, seed: int = 3) -> List[View]:
    """Uneven views: r ~ U(2.5, 50), inclination ~ U(0, 90 deg), speed ~ U(0, 0.95)."""
    rng = np.random.default_rng(seed)
    res = rng.integers(0, len(BATCH_RESOLUTIONS), n)
    r = rng.uniform(2.5, 50.0, n)
    th = rng.uniform(0.0, math.pi / 2, n)
    ph = rng.uniform(0.0, 2 * math.pi, n)
    sp = rng.uniform(0.0, 0.95, n)
    vz = rng.uniform(-1.0, 1.0, n)
    vaz = rng.uniform(0.0, 2 * math.pi, n)
    r_in = rng.uniform(3.0, 6.0, n)
    r_out = rng.uniform(10.0, 30.0, n)
    views = []
    for k in range(n):
        s = math.sqrt(max(0.0, 1.0 - vz[k] ** 2))
        vdir = np.array([s * math.cos(vaz[k]), s * math.sin(vaz[k]), vz[k]])
        pos = spherical_position(r[k], th[k], ph[k])
        w, h = BATCH_RESOLUTIONS[res[k]]
        views.append(aimed_view(pos, sp[k] * vdir, w, h,
                                disc_r_in=float(r_in[k]), disc_r_out=float(r_out[k])))
    return views


SERVE_RESOLUTIONS = ((512, 512), (1920, 1080), (3840, 2160), (7680, 4320))
SERVE_WEIGHTS = (0.4, 0.3, 0.2, 0.1)
SERVE_FIELDS = ((100_000, 40), (1_000_000, 41), (4_000_000, 42))


@dataclasses.dataclass
class Request:
    arrival: float        # seconds since the start of the stream
    view: View
    field: int            # index into SERVE_FIELDS


def serve_requests(rate: float = 200.0, duration: float = 60.0, seed: int = 4,
                   time_scale: float = 1000.0) -> List[Request]:
    """Poisson arrivals; each request is a frame on a circular orbit of radius U(3, 30).

    The orbit plane normal is uniform on the sphere, the phase advances with the arrival
    time (``time_scale`` r_s/c per second) at the Keplerian rate, and the camera moves
    along the orbit at the local circular-orbit speed sqrt(u / (2 (1 - u)))."""
    rng = np.random.default_rng(seed)
    t = 0.0
    arrivals = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        arrivals.append(t)
    n = len(arrivals)
    res = rng.choice(len(SERVE_RESOLUTIONS), size=n, p=SERVE_WEIGHTS)
    r = rng.uniform(3.0, 30.0, n)
    nz = rng.uniform(-1.0, 1.0, n)
    naz = rng.uniform(0.0, 2 * math.pi, n)
    psi0 = rng.uniform(0.0, 2 * math.pi, n)
    r_in = rng.uniform(3.0, 6.0, n)
    r_out = rng.uniform(10.0, 30.0, n)
    field = rng.integers(0, len(SERVE_FIELDS), n)
    out = []
    for k in range(n):
        s = math.sqrt(max(0.0, 1.0 - nz[k] ** 2))
        nrm = np.array([s * math.cos(naz[k]), s * math.sin(naz[k]), nz[k]])
        a = _unit(np.cross(nrm, [1.0, 0.0, 0.0]) if abs(nrm[0]) < 0.9
                  else np.cross(nrm, [0.0, 1.0, 0.0]))
        b = np.cross(nrm, a)
        u = 1.0 / r[k]
        psi = psi0[k] + math.sqrt(u ** 3 / 2.0) * arrivals[k] * time_scale
        rhat = math.cos(psi) * a + math.sin(psi) * b
        tang = -math.sin(psi) * a + math.cos(psi) * b
        speed = math.sqrt(u / (2.0 * (1.0 - u)))
        w, h = SERVE_RESOLUTIONS[res[k]]
        v = aimed_view(r[k] * rhat, speed * tang, w, h,
                       disc_r_in=float(r_in[k]), disc_r_out=float(r_out[k]))
        out.append(Request(arrivals[k], v, int(field[k])))
    return out


def freefall_requests(rate: float = 200.0, duration: float = 60.0, seed: int = 5,
                      sessions: int = 16, time_scale: float = 100.0,
                      resolutions=SERVE_RESOLUTIONS, weights=SERVE_WEIGHTS) -> List[Request]:
    """Poisson arrivals spread over `sessions` freely falling cameras (Appendix C), each on
    a seeded bound orbit that stays within r in [4, 100]: r0 ~ U(8, 30), coordinate angle
    delta0 ~ U(1.2, 1.9), speed v0 ~ U(0.95, 1.15) times the circular speed at r0,
    inclination chi ~ U(-1.2, 1.2) and the orbital plane turned by a uniform angle about z.
    A request's frame is the camera at proper time (arrival time x `time_scale`), aimed at
    the hole, with the camera's coordinate time as the view's `time`; orbits that leave the
    range are drawn again."""
    rng = np.random.default_rng(seed)
    t, arrivals = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        arrivals.append(t)
    n = len(arrivals)
    owner = rng.integers(0, sessions, n)
    res = rng.choice(len(resolutions), size=n, p=weights)
    field = rng.integers(0, len(SERVE_FIELDS), n)
    out: List[Optional[Request]] = [None] * n
    grid = np.arange(0.0, duration * time_scale + 2.0, 2.0)
    for k in range(sessions):
        mine = np.nonzero(owner == k)[0]
        while True:
            r0 = rng.uniform(8.0, 30.0)
            d0 = rng.uniform(1.2, 1.9)
            u0 = 1.0 / r0
            v0 = math.sqrt(u0 / (2.0 * (1.0 - u0))) * rng.uniform(0.95, 1.15)
            chi, turn = rng.uniform(-1.2, 1.2), rng.uniform(0.0, 2.0 * math.pi)
            r_in, r_out = rng.uniform(3.0, 6.0), rng.uniform(10.0, 30.0)
            taus = np.array([arrivals[j] * time_scale for j in mine])
            both = np.union1d(grid, taus)
            try:
                st = camera_orbit(r0, d0, v0, both)
            except ValueError:
                continue
            if st.r.min() >= 4.0 and st.r.max() <= 100.0:
                break
        pos, vel = orbit_position_velocity(st, chi)
        c, s = math.cos(turn), math.sin(turn)
        rz = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
        pos, vel = pos @ rz.T, vel @ rz.T
        at = np.searchsorted(both, taus)
        for j, i in zip(mine, at):
            w, h = resolutions[res[j]]
            v = aimed_view(pos[i], vel[i], w, h, disc_r_in=float(r_in), disc_r_out=float(r_out))
            v.time = float(st.t[i])
            out[j] = Request(arrivals[j], v, int(field[j]))
    return out


def bloom_weights(levels: int) -> List[float]:
    """Weights w_0 .. w_levels of the bloom's mipmap filters: most light stays in the pixel
    and the halo falls off by half per level (each level's kernel is twice as wide); sum 1."""
    w = [0.0] + [0.5 ** k for k in range(1, levels + 1)]
    halo = sum(w)
    scale = 0.1 / halo if halo > 0 else 0.0
    w = [x * scale for x in w]
    w[0] = 1.0 - sum(w)
    return w


def sample_quads(width: int, height: int, frac: float, seed: int) -> np.ndarray:
    """Sorted unique 2x2-quad origins (even x, even y) covering about ``frac`` of pixels.

    Returns int32 array (m, 2) of (x0, y0)."""
    qw, qh = (width + 1) // 2, (height + 1) // 2
    nq = qw * qh
    m = max(1, int(round(frac * width * height / 4.0)))
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(nq, size=min(m, nq), replace=False))
    return np.stack([2 * (idx % qw), 2 * (idx // qw)], axis=1).astype(np.int32)


def all_quads(width: int, height: int) -> np.ndarray:
    qw, qh = (width + 1) // 2, (height + 1) // 2
    idx = np.arange(qw * qh)
    return np.stack([2 * (idx % qw), 2 * (idx // qw)], axis=1).astype(np.int32)
