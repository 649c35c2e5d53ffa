"""Seeded synthetic inputs for the hybrid depth-of-field pass.

This module produces *data only*: scene triangles, albedos, lights, camera
paths, lens settings and parameter values.  It holds none of the method's
arithmetic (no circle of confusion, no filtering, no ray tracing), so both the
GPU library and the CPU oracle can consume the same inputs without sharing any
of the code under test.

Randomness is SplitMix64 (Steele, Lea & Flood 2014): a 64-bit counter stepped by
the golden-ratio increment and finalised by two xor-shift-multiply rounds.
Uniform floats take the top 24 bits times 2^-24.

The scenes stand in for the paper's test scenes (The Modern Living Room, Sun
Temple, Bistro Exterior; section 4.2), which are not available: a far field of
simple opaque objects and a foreground layer of thin geometry whose blurred
silhouettes are what the ray-traced branch exists for.
"""

from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

BASE_SEED = 2210061580


class SplitMix64:
    """Counter-form SplitMix64; `uniform(n)` draws n floats in [0, 1)."""

    def __init__(self, seed: int):
        self.state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.count = 0

    def next_u64(self, n: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            idx = np.arange(self.count + 1, self.count + n + 1, dtype=np.uint64)
            z = self.state + idx * _GOLDEN
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            z = z ^ (z >> np.uint64(31))
        self.count += n
        return z

    def uniform(self, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        u = (self.next_u64(n) >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)
        return lo + (hi - lo) * u


# ----------------------------------------------------------------------------
# Plain input records (mirrors of the C structs on both sides)
# ----------------------------------------------------------------------------

@dataclass
class Camera:
    pos: tuple
    right: tuple
    up: tuple
    fwd: tuple
    width: int
    height: int
    frame: int = 0
    seed: int = 1
    jitter: tuple = (0.0, 0.0)  # sub-pixel sample offset in full-res pixels (right, down)


@dataclass
class Lens:
    focal: float = 0.050        # metres ("f = 50 mm")
    fnum: float = 1.4           # N; aperture diameter a = f / N
    focus: float = 15.0         # d, distance to the focus plane
    sensor: float = 0.036       # w_s, 36 mm full-frame sensor width
    blades: int = 0             # 0 = circular aperture, 6 = hexagon
    blade_rot: float = 0.0      # radians


MASK_ADAPTIVE, MASK_FIXED, MASK_ALL, MASK_DILATE = 0, 1, 2, 3
TAA_FINAL, TAA_RASTER, TAA_POST = 1, 2, 4     # bits of Params.taa
TAA_ALL = TAA_FINAL | TAA_RASTER | TAA_POST


def jitter_sequence(n: int, seed: int) -> list:
    """n pseudorandom sub-pixel camera offsets in [-0.5, 0.5)^2 (full-res
    pixels), one per frame, from a seeded SplitMix64 stream; binary32 values."""
    u = SplitMix64(seed).uniform(2 * n, -0.5, 0.5).astype(np.float32).reshape(n, 2)
    return [(float(a), float(b)) for a, b in u]


def jittered(cams: list, seed: int) -> list:
    """The camera path with per-frame jitter from jitter_sequence."""
    js = jitter_sequence(len(cams), seed)
    return [dataclasses.replace(c, jitter=j) for c, j in zip(cams, js)]


@dataclass
class Params:
    m: int = 4                  # ray budget per pixel (section 3.2.1)
    s: float = 0.8              # eq. (2) scale (section 4.2)
    var_mask_w: float = 1.0e5   # eq. (4) variance weight
    alpha: float = 0.95         # history weight of the moving average (3.2.3)
    alpha_motion: float = 0.8   # reduced history weight during motion
    var_recon_w: float = 2000.0 # eq. (5)
    b_max: float = 0.9          # eq. (5)
    h_edge: float = 0.3         # eq. (7)
    lod_scale: float = 0.05     # eq. (8)
    lod_max: float = 3.0        # eq. (8)
    depth_range: float = 0.1    # main-filter depth range, 10 cm (4.2)
    r_max: float = 32.0         # largest gather radius in half-res pixels
    tile: int = 16              # tile side for the neighbourhood max CoC
    l_spec: float = 1.0         # luma above which a tap counts as a bright (specular) sample
    mask_mode: int = MASK_ADAPTIVE
    pp_polygon: int = 0         # 1: post-process gather kernel shaped like a bladed aperture
    taa: int = 0                # TAA stages (3.4), bits TAA_FINAL / TAA_RASTER / TAA_POST
    composite_literal: int = 0  # 1: eq. (7)'s far-field blend read literally (high hit ratio -> post-process)


@dataclass
class Scene:
    verts: np.ndarray           # (n, 9) float32: v0 xyz, v1 xyz, v2 xyz
    albedo: np.ndarray          # (n, 3) float32
    light_dir: tuple = (0.0, -1.0, 0.0)   # direction the light travels
    light_rad: tuple = (1.0, 1.0, 1.0)
    ambient: tuple = (0.15, 0.15, 0.15)
    sky: tuple = (0.55, 0.70, 0.95)
    leaf_split: int = 2         # BVH leaves: a long thin triangle becomes 2^leaf_split clipped references

    @property
    def ntri(self) -> int:
        return int(self.verts.shape[0])


def _normalize(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def f32tuple(v):
    return tuple(float(np.float32(x)) for x in v)


def look_camera(pos, yaw: float, pitch: float, width: int, height: int,
                frame: int = 0, seed: int = 1) -> Camera:
    """Orthonormal camera basis: +y up, forward +z at zero yaw/pitch
    (left-handed, right = +x)."""
    cy, sy = math.cos(yaw), math.sin(yaw)
    cp, sp = math.cos(pitch), math.sin(pitch)
    fwd = np.array([sy * cp, sp, cy * cp])
    right = np.array([cy, 0.0, -sy])
    up = np.cross(fwd, right)
    return Camera(f32tuple(pos), f32tuple(right), f32tuple(up), f32tuple(fwd),
                  int(width), int(height), int(frame), int(seed))


def half_fov_tan(lens: Lens) -> float:
    """Horizontal half-field tangent of the sensor at the focused image
    distance; used only to place objects inside the frame."""
    f, d, ws = lens.focal, lens.focus, lens.sensor
    return ws * (d - f) / (2.0 * f * d)


# ----------------------------------------------------------------------------
# Geometry builders
# ----------------------------------------------------------------------------

_BOX_FACES = np.array([
    [0, 2, 1], [0, 3, 2],   # -z
    [4, 5, 6], [4, 6, 7],   # +z
    [0, 1, 5], [0, 5, 4],   # -y
    [3, 7, 6], [3, 6, 2],   # +y
    [0, 4, 7], [0, 7, 3],   # -x
    [1, 2, 6], [1, 6, 5],   # +x
], dtype=np.int64)


def boxes(lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Axis-aligned boxes -> (12 * nbox, 9) triangles."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    n = lo.shape[0]
    corners = np.empty((n, 8, 3))
    for c in range(8):
        x = hi[:, 0] if c in (1, 2, 5, 6) else lo[:, 0]
        y = hi[:, 1] if c in (2, 3, 6, 7) else lo[:, 1]
        z = hi[:, 2] if c >= 4 else lo[:, 2]
        corners[:, c] = np.stack([x, y, z], axis=1)
    tris = corners[:, _BOX_FACES]            # (n, 12, 3, 3)
    return tris.reshape(n * 12, 9).astype(np.float32)


def quad(p0, p1, p2, p3) -> np.ndarray:
    """Two triangles of the quad p0 p1 p2 p3 (in order around the rim)."""
    p = [np.asarray(x, np.float64) for x in (p0, p1, p2, p3)]
    return np.stack([np.concatenate([p[0], p[1], p[2]]),
                     np.concatenate([p[0], p[2], p[3]])]).astype(np.float32)


def uv_spheres(centres: np.ndarray, radii: np.ndarray,
               slices: int = 12, bands: int = 11) -> np.ndarray:
    """UV spheres with `slices` x `bands` cells: 2 * slices * (bands - 1)
    triangles each (240 for 12 x 11)."""
    th = np.linspace(0.0, math.pi, bands + 1)          # polar
    ph = np.linspace(0.0, 2.0 * math.pi, slices + 1)[:-1]
    unit = []
    for b in range(bands):
        t0, t1 = th[b], th[b + 1]
        for s in range(slices):
            p0, p1 = ph[s], ph[(s + 1) % slices]
            a = (math.sin(t0) * math.cos(p0), math.cos(t0), math.sin(t0) * math.sin(p0))
            bb = (math.sin(t0) * math.cos(p1), math.cos(t0), math.sin(t0) * math.sin(p1))
            c = (math.sin(t1) * math.cos(p0), math.cos(t1), math.sin(t1) * math.sin(p0))
            d = (math.sin(t1) * math.cos(p1), math.cos(t1), math.sin(t1) * math.sin(p1))
            if b == 0:
                unit.append((a, d, c))
            elif b == bands - 1:
                unit.append((a, bb, c))
            else:
                unit.append((a, bb, d))
                unit.append((a, d, c))
    unit = np.array(unit, dtype=np.float64)            # (k, 3, 3)
    k = unit.shape[0]
    out = unit[None] * radii[:, None, None, None] + centres[:, None, None, :]
    return out.reshape(-1, 9).astype(np.float32), k


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

def scene_small(seed: int = BASE_SEED + 1000) -> tuple:
    """256x256 workload: ground quad (2 tris), 64 boxes at depth 10-30 with
    uniform albedo (768 tris), 8 thin bars at depth 1.5-2.5 (96 tris);
    Lambert shading with one directional light.  Returns (scene, camera,
    lens, params)."""
    rng = SplitMix64(seed)
    lens = Lens(focal=0.050, fnum=1.4, focus=15.0, sensor=0.036)
    tx = half_fov_tan(lens)
    ground = quad((-60, 0, -1), (-60, 0, 80), (60, 0, 80), (60, 0, -1))
    gal = np.array([[0.45, 0.42, 0.38]] * 2, np.float32)

    nb = 64
    z = rng.uniform(nb, 10.0, 30.0)
    x = rng.uniform(nb, -0.9, 0.9) * z * tx
    fw = rng.uniform(nb, 0.6, 2.4)
    fd = rng.uniform(nb, 0.6, 2.4)
    h = rng.uniform(nb, 0.6, 3.0)
    alb = rng.uniform(nb * 3).reshape(nb, 3)
    lo = np.stack([x - fw / 2, np.zeros(nb), z - fd / 2], 1)
    hi = np.stack([x + fw / 2, h, z + fd / 2], 1)
    bt = boxes(lo, hi)
    bal = np.repeat(alb, 12, axis=0).astype(np.float32)

    nbar = 8
    zb = rng.uniform(nbar, 1.5, 2.5)
    wb = rng.uniform(nbar, 0.01, 0.04)
    xb = (-0.8 + 1.6 * (np.arange(nbar) + rng.uniform(nbar)) / nbar) * zb * tx
    albb = rng.uniform(nbar * 3, 0.2, 0.9).reshape(nbar, 3)
    lo = np.stack([xb - wb / 2, np.zeros(nbar), zb - wb / 2], 1)
    hi = np.stack([xb + wb / 2, np.full(nbar, 3.0), zb + wb / 2], 1)
    bart = boxes(lo, hi)
    baral = np.repeat(albb, 12, axis=0).astype(np.float32)

    verts = np.concatenate([ground, bt, bart]).astype(np.float32)
    albedo = np.concatenate([gal, bal, baral]).astype(np.float32)
    scene = Scene(verts, albedo, light_dir=f32tuple(_normalize((-0.4, -1.0, 0.6))))
    cam = look_camera((0.0, 1.2, 0.0), 0.0, 0.0, 256, 256, frame=0, seed=seed & 0xFFFFFFFF)
    return scene, cam, lens, Params(m=4)


def scene_1080p(seed: int = BASE_SEED + 2000, n_spheres: int = 4096,
                n_blades: int = 50000, width: int = 1920, height: int = 1080) -> tuple:
    """1920x1080 workload: ground quad, 4096 UV spheres of 240 triangles over
    depth 5-80 and a foreground grass band of 50k 4-triangle blades at depth
    0.5-3 (1,183,042 triangles).  Returns (scene, camera_path(60), lens,
    params).  Other sizes and counts give the same kind of scene."""
    rng = SplitMix64(seed)
    lens = Lens(focal=0.050, fnum=1.4, focus=15.0, sensor=0.036)
    tx = half_fov_tan(lens)
    ground = quad((-200, 0, -2), (-200, 0, 200), (200, 0, 200), (200, 0, -2))
    gal = np.array([[0.40, 0.45, 0.30]] * 2, np.float32)

    ns = n_spheres
    zc = rng.uniform(ns, 5.0, 80.0)
    r = rng.uniform(ns, 0.3, 1.5)
    # scattered over a wide field: the frame sees a slice of it (a few near
    # spheres, many distant ones, sky above the horizon)
    xc = rng.uniform(ns, -400.0, 400.0)
    cen = np.stack([xc, r, zc], 1)
    st, per = uv_spheres(cen, r)
    salb = np.repeat(rng.uniform(ns * 3, 0.05, 0.95).reshape(ns, 3), per, axis=0)

    nbld = n_blades
    zg = rng.uniform(nbld, 0.5, 3.0)
    xg = rng.uniform(nbld, -1.0, 1.0) * (zg * tx + 0.5)
    hg = rng.uniform(nbld, 0.1, 0.5)
    wg = rng.uniform(nbld, 0.005, 0.02)
    yaw = rng.uniform(nbld, -0.6, 0.6)
    lean_x = rng.uniform(nbld, -0.25, 0.25)
    lean_z = rng.uniform(nbld, -0.25, 0.25)
    gshade = rng.uniform(nbld, 0.6, 1.0)
    ux, uz = np.cos(yaw), -np.sin(yaw)
    pts = []
    for level, (yf, wf) in enumerate(((0.0, 1.0), (0.5, 0.7), (1.0, 0.15))):
        y = hg * yf
        cx = xg + lean_x * hg * yf * yf
        cz = zg + lean_z * hg * yf * yf
        hw = 0.5 * wg * wf
        pts.append((np.stack([cx - hw * ux, y, cz - hw * uz], 1),
                    np.stack([cx + hw * ux, y, cz + hw * uz], 1)))
    gl = []
    for lv in range(2):
        (a0, a1), (b0, b1) = pts[lv], pts[lv + 1]
        gl.append(np.concatenate([a0, a1, b1], 1))
        gl.append(np.concatenate([a0, b1, b0], 1))
    gt = np.stack(gl, 1).reshape(-1, 9).astype(np.float32)
    galb = np.stack([0.25 * gshade, 0.55 * gshade, 0.12 * gshade], 1)
    galb = np.repeat(galb, 4, axis=0)

    verts = np.concatenate([ground, st, gt]).astype(np.float32)
    albedo = np.concatenate([gal, salb, galb]).astype(np.float32)
    scene = Scene(verts, albedo, light_dir=f32tuple(_normalize((-0.3, -1.0, 0.5))))
    cams = camera_spline(rng, 60, width, height, seed & 0xFFFFFFFF)
    return scene, cams, lens, Params(m=8)


SESSION_SIZES = ((1280, 720), (1920, 1080), (2560, 1440))


def session_specs(n: int, seed: int = BASE_SEED + 4000) -> list:
    """n sessions of the batched workload: resolution uniform over 720p /
    1080p / 1440p, triangle budget uniform in [0.2M, 1M] split between
    spheres and grass in the 1080p scene's proportion.  Returns
    (seed, width, height, n_spheres, n_blades) per session."""
    rng = SplitMix64(seed)
    cls = rng.uniform(n)
    tri = rng.uniform(n, 0.2e6, 1.0e6)
    out = []
    for i in range(n):
        w, h = SESSION_SIZES[min(int(cls[i] * 3), 2)]
        scale = tri[i] / 1183042.0
        out.append((seed + 1 + i, w, h, max(1, int(round(4096 * scale))), max(1, int(round(50000 * scale)))))
    return out


def scene_session(spec: tuple) -> tuple:
    """One session of the batched workload (see session_specs)."""
    sd, w, h, ns, nb = spec
    return scene_1080p(seed=sd, n_spheres=ns, n_blades=nb, width=w, height=h)


def scene_4k(seed: int = BASE_SEED + 3000, n_boxes: int = 130000, n_links: int = 200000) -> tuple:
    """3840x2160 workload: a random-height box city (130k boxes, 1.56M
    triangles, heights 2-40, footprints 2-6) on both sides of a 20 m wide
    street, seen through a chain-link fence of 200k thin quads (400k
    triangles; 5 cm diamonds, 3 mm wire) at depth 1-2; static camera,
    6-blade aperture, N = 2, f = 50 mm, focus pulled linearly from 3 to 40
    over 60 frames; 16 rays per masked pixel.  Returns (scene, cameras(60),
    lenses(60), params)."""
    rng = SplitMix64(seed)
    base = Lens(focal=0.050, fnum=2.0, focus=3.0, sensor=0.036, blades=6, blade_rot=0.0)
    nb = n_boxes
    z = rng.uniform(nb, 5.0, 800.0)
    side = np.where(rng.uniform(nb) < 0.5, -1.0, 1.0)
    x = side * rng.uniform(nb, 10.0, 800.0)
    fw = rng.uniform(nb, 2.0, 6.0)
    fd = rng.uniform(nb, 2.0, 6.0)
    h = rng.uniform(nb, 2.0, 40.0)
    lo = np.stack([x - fw / 2, np.zeros(nb), z - fd / 2], 1)
    hi = np.stack([x + fw / 2, h, z + fd / 2], 1)
    city = boxes(lo, hi)
    calb = np.repeat(rng.uniform(nb * 3, 0.2, 0.9).reshape(nb, 3), 12, axis=0)
    ground = quad((-900, 0, -10), (-900, 0, 900), (900, 0, 900), (900, 0, -10))
    galb = np.array([[0.35, 0.35, 0.38]] * 2)
    # fence: each diamond cell contributes one wire per diagonal, each wire a
    # quad 3 mm wide; gently wavy in depth between 1 and 2
    nl = n_links
    cols = 500
    k = np.arange(nl)
    diag = k % 2
    cell = k // 2
    ci = cell % cols
    cj = cell // cols
    pitch = 0.05
    cx = -12.5 + (ci + 0.5) * pitch
    cy = (cj + 0.5) * pitch
    cz = 1.5 + 0.45 * np.sin(cx * 0.9) + rng.uniform(nl, -0.005, 0.005)
    dx = 0.5 * pitch * np.where(diag == 0, 1.0, -1.0)
    dy = 0.5 * pitch
    p0 = np.stack([cx - dx, cy - dy, cz], 1)
    p1 = np.stack([cx + dx, cy + dy, cz], 1)
    nrm = np.stack([-dy * np.ones(nl), dx, np.zeros(nl)], 1)
    nrm = nrm / np.linalg.norm(nrm, axis=1, keepdims=True) * 0.0015
    a0, a1, b1, b0 = p0 - nrm, p1 - nrm, p1 + nrm, p0 + nrm
    t1 = np.concatenate([a0, a1, b1], 1)
    t2 = np.concatenate([a0, b1, b0], 1)
    fence = np.stack([t1, t2], 1).reshape(-1, 9).astype(np.float32)
    falb = np.tile(np.array([[0.75, 0.75, 0.72]]), (2 * nl, 1))
    verts = np.concatenate([ground, city, fence]).astype(np.float32)
    albedo = np.concatenate([galb, calb, falb]).astype(np.float32)
    scene = Scene(verts, albedo, light_dir=f32tuple(_normalize((0.4, -1.0, 0.3))))
    cam = look_camera((0.0, 1.6, 0.0), 0.0, math.radians(3.0), 3840, 2160, frame=0, seed=seed & 0xFFFFFFFF)
    cams, lenses = [], []
    for fi in range(60):
        cams.append(dataclasses.replace(cam, frame=fi))
        lenses.append(dataclasses.replace(base, focus=float(np.float32(3.0 + 37.0 * fi / 59.0))))
    return scene, cams, lenses, Params(m=16)


def camera_spline(rng: SplitMix64, nframes: int, width: int, height: int,
                  seed: int) -> list:
    """Catmull-Rom path through 8 seeded control points at eye height
    0.8-1.1 with yaw within +-10 degrees and a 5-degree downward pitch, so the
    grass is a foreground band in the lower part of the frame."""
    k = 8
    px = rng.uniform(k, -0.3, 0.3)
    py = rng.uniform(k, 0.8, 1.1)
    pz = rng.uniform(k, -0.3, 0.3)
    yaw = rng.uniform(k, -math.radians(10), math.radians(10))
    ctrl = np.stack([px, py, pz, yaw], 1)
    cams = []
    for fi in range(nframes):
        s = 1.0 + (k - 3) * fi / max(1, nframes - 1)
        i = min(int(math.floor(s)), k - 3)
        t = s - i
        p0, p1, p2, p3 = ctrl[i - 1], ctrl[i], ctrl[i + 1], ctrl[i + 2]
        t2, t3 = t * t, t * t * t
        v = 0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t2
                   + (-p0 + 3 * p1 - 3 * p2 + p3) * t3)
        cams.append(look_camera(v[:3], float(v[3]), math.radians(-5.0), width, height,
                                frame=fi, seed=seed))
    return cams


def shot_cameras(kind: str, nframes: int = 20, width: int = 1920, height: int = 1080, seed: int = 1) -> list:
    """Camera shots of the 1080p scene by foreground coverage, as Table 1
    classes its shots: "BG" at eye height 1.1 pitched 2 degrees down (the
    grass covers about 3 % of the frame), "FG" at 0.12 pitched 8 degrees down
    inside the grass (about 70 %); the 60-frame path is the middle class
    (20-40 %).  A slow dolly along x from -0.2 to 0.2."""
    y, pitch = {"BG": (1.1, -2.0), "FG": (0.12, -8.0)}[kind]
    out = []
    for fi in range(nframes):
        x = -0.2 + 0.4 * fi / max(1, nframes - 1)
        out.append(look_camera((x, y, 0.0), 0.0, math.radians(pitch), width, height, frame=fi, seed=seed))
    return out


def grass_only(scene: Scene, n_blades: int = 50000) -> Scene:
    """The grass of a 1080p-recipe scene (its last 4 n_blades triangles), to
    measure how much of a frame the foreground covers."""
    n = 4 * n_blades
    return Scene(scene.verts[-n:], scene.albedo[-n:])


def pan_camera(cam: Camera, dx: float) -> Camera:
    """The same camera translated by dx along its right axis."""
    p = np.asarray(cam.pos, np.float64) + dx * np.asarray(cam.right, np.float64)
    return dataclasses.replace(cam, pos=f32tuple(p), frame=cam.frame + 1)


def random_triangles(n: int, seed: int, spread: float = 4.0, size: float = 0.6):
    """Small random triangle soups for closest-hit checks."""
    rng = SplitMix64(seed)
    c = rng.uniform(n * 3, -spread, spread).reshape(n, 1, 3)
    off = rng.uniform(n * 9, -size, size).reshape(n, 3, 3)
    v = (c + off).reshape(n, 9).astype(np.float32)
    alb = rng.uniform(n * 3).reshape(n, 3).astype(np.float32)
    return v, alb


def awkward_triangles(seed: int):
    """Thin triangles at awkward places for the leaf split and the traversal:
    three coordinate scales (1, 1e3, 3e6), a vertex exactly on a quarter plane
    of its box, equal x and y extents (a tie for the longest axis), and
    degenerate triangles (collinear, repeated vertices).  Returns (v, albedo,
    rays' origins, rays' directions): 20000 rays aimed near the centroids."""
    rng = SplitMix64(seed)
    tris = []
    for s in (1.0, 1e3, 3e6):
        for _ in range(40):
            c = rng.uniform(3, -2 * s, 2 * s)
            d = rng.uniform(3, -s, s)
            w = rng.uniform(3, -0.01 * s, 0.01 * s)
            tris.append([*c, *(c + d), *(c + d + w)])
    tris.append([0, 0, 0, 2, 0.01, 0, 8, 0.02, 0.01])
    tris.append([0, 0, 0, 4, 4, 0.01, 4.02, 4, 0])
    tris.append([0, 0, 5, 1, 1, 6, 2, 2, 7])
    tris.append([1, 1, 1, 1, 1, 1, 3, 0, 0])
    v = np.array(tris, np.float32)
    n = v.shape[0]
    nr = 20000
    tv = v.reshape(n, 3, 3).astype(np.float64)
    pick = (rng.next_u64(nr) % np.uint64(n)).astype(np.int64)
    bary = rng.uniform(3 * nr, 0.05, 1.0).reshape(nr, 3)
    bary /= bary.sum(1, keepdims=True)
    tgt = np.einsum("rk,rkc->rc", bary, tv[pick])
    scale = np.abs(tv[pick]).max((1, 2)).clip(1.0, None)[:, None]
    o = tgt + rng.uniform(3 * nr, -1, 1).reshape(nr, 3) * scale
    d = tgt - o
    return v, np.ones((n, 3), np.float32), o.astype(np.float32), d.astype(np.float32)
