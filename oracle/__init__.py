"""ctypes binding of the CPU oracle (test infrastructure only).

The oracle is a plain C restatement of the hybrid depth-of-field pass used to
check the GPU library.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_f3 = C.c_float * 3


class OrcCamera(C.Structure):
    _fields_ = [("pos", _f3), ("right", _f3), ("up", _f3), ("fwd", _f3),
                ("width", C.c_int32), ("height", C.c_int32),
                ("frame", C.c_uint32), ("seed", C.c_uint32), ("jitter", C.c_float * 2)]


class OrcLens(C.Structure):
    _fields_ = [("focal", C.c_float), ("fnum", C.c_float), ("focus", C.c_float),
                ("sensor", C.c_float), ("blades", C.c_int32), ("blade_rot", C.c_float)]


class OrcParams(C.Structure):
    _fields_ = [("m", C.c_int32), ("s", C.c_float), ("var_mask_w", C.c_float),
                ("alpha", C.c_float), ("alpha_motion", C.c_float),
                ("var_recon_w", C.c_float), ("b_max", C.c_float), ("h_edge", C.c_float),
                ("lod_scale", C.c_float), ("lod_max", C.c_float),
                ("depth_range", C.c_float), ("r_max", C.c_float), ("tile", C.c_int32),
                ("l_spec", C.c_float), ("mask_mode", C.c_int32), ("pp_polygon", C.c_int32), ("taa", C.c_int32),
                ("composite_literal", C.c_int32)]


class OrcScene(C.Structure):
    _fields_ = [("ntri", C.c_int32), ("verts", C.c_void_p), ("albedo", C.c_void_p),
                ("light_dir", _f3), ("light_rad", _f3), ("ambient", _f3), ("sky", _f3),
                ("leaf_split", C.c_int32)]


class OrcBvh(C.Structure):
    _fields_ = [("nleaf", C.c_int32), ("keys", C.c_void_p), ("refs", C.c_void_p), ("ids", C.c_void_p),
                ("left", C.c_void_p), ("right", C.c_void_p), ("parent", C.c_void_p), ("bounds", C.c_void_p),
                ("leaf_bounds", C.c_void_p)]


class OrcDebug(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in (
        "colr", "zn", "tile_max", "tile_dil", "pre", "gather", "ppmed", "prev_idx",
        "queue", "ray_base", "ray_hit", "ray_t", "ray_col", "ray_pos", "resolve",
        "temporal", "var_blur", "rtmed", "mips", "recon")] + [
        ("n_masked", C.c_int64), ("n_rays", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_threads.restype = C.c_int
        L.orc_coc.restype = C.c_float
        L.orc_coc.argtypes = [C.POINTER(OrcLens), C.c_int32, C.c_float]
        L.orc_zone.argtypes = [C.POINTER(OrcLens), C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.orc_morton.argtypes = [C.POINTER(OrcScene), vp]
        L.orc_build_bvh.argtypes = [C.POINTER(OrcScene), C.POINTER(OrcBvh)]
        L.orc_leaf_refs.argtypes = [C.POINTER(OrcScene), vp]
        L.orc_leaf_refs.restype = C.c_int64
        L.orc_ref_boxes.argtypes = [C.POINTER(OrcScene), vp, vp, vp]
        L.orc_morton_boxes.argtypes = [vp, C.c_int64, vp]
        L.orc_closest_hit.argtypes = [C.POINTER(OrcScene), C.POINTER(OrcBvh), C.c_int64, vp, vp, vp, vp]
        L.orc_lens_sample.argtypes = [C.c_uint32] * 4 + [C.c_int32, C.c_float,
                                                         C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.orc_gbuffer.argtypes = [C.POINTER(OrcScene), C.POINTER(OrcBvh), C.POINTER(OrcCamera),
                                  C.POINTER(OrcLens), vp, vp, vp]
        L.orc_render_frame.argtypes = [C.POINTER(OrcScene), C.POINTER(OrcBvh), C.POINTER(OrcCamera),
                                       C.POINTER(OrcLens), C.POINTER(OrcCamera), C.POINTER(OrcLens),
                                       C.c_int32, C.POINTER(OrcParams), vp, vp, vp, vp, vp, vp, vp,
                                       C.POINTER(OrcDebug)]
        L.orc_pixel_estimate.argtypes = [C.POINTER(OrcScene), C.POINTER(OrcBvh), C.POINTER(OrcCamera),
                                         C.POINTER(OrcLens), C.c_int64, vp, C.c_int32, vp]
        L.orc_lens_integral.argtypes = [C.POINTER(OrcScene), C.POINTER(OrcBvh), C.POINTER(OrcCamera),
                                        C.POINTER(OrcLens), C.c_int64, vp, C.c_int32, vp]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def camera_struct(cam) -> OrcCamera:
    return OrcCamera(_f3(*cam.pos), _f3(*cam.right), _f3(*cam.up), _f3(*cam.fwd),
                     cam.width, cam.height, cam.frame & 0xFFFFFFFF, cam.seed & 0xFFFFFFFF,
                     (C.c_float * 2)(*getattr(cam, "jitter", (0.0, 0.0))))


def lens_struct(lens) -> OrcLens:
    return OrcLens(lens.focal, lens.fnum, lens.focus, lens.sensor, lens.blades, lens.blade_rot)


def gather_rings(lens, params):
    """The post-process gather's taps: (ox, oy, frac) arrays of 81."""
    ox, oy, fr = (np.zeros(81, np.float32) for _ in range(3))
    L = lib()
    L.orc_gather_rings.argtypes = [C.POINTER(OrcLens), C.POINTER(OrcParams), C.c_void_p, C.c_void_p, C.c_void_p]
    rc = L.orc_gather_rings(C.byref(lens_struct(lens)), C.byref(params_struct(params)), _ptr(ox), _ptr(oy), _ptr(fr))
    if rc != 0:
        raise RuntimeError("orc_gather_rings failed")
    return ox, oy, fr


def params_struct(p) -> OrcParams:
    return OrcParams(p.m, p.s, p.var_mask_w, p.alpha, p.alpha_motion, p.var_recon_w, p.b_max,
                     p.h_edge, p.lod_scale, p.lod_max, p.depth_range, p.r_max, p.tile,
                     p.l_spec, p.mask_mode, getattr(p, "pp_polygon", 0), getattr(p, "taa", 0),
                     getattr(p, "composite_literal", 0))


class OracleScene:
    """Holds the scene arrays alive next to their C view."""

    def __init__(self, scene, leaf_split=None):
        self.verts = np.ascontiguousarray(scene.verts, dtype=np.float32)
        self.albedo = np.ascontiguousarray(scene.albedo, dtype=np.float32)
        if leaf_split is None:
            leaf_split = getattr(scene, "leaf_split", 2)
        self.s = OrcScene(self.verts.shape[0], _ptr(self.verts), _ptr(self.albedo),
                          _f3(*scene.light_dir), _f3(*scene.light_rad), _f3(*scene.ambient),
                          _f3(*scene.sky), int(leaf_split))
        self.ntri = self.verts.shape[0]
        self.bvh = None

    def leaf_refs(self):
        """(ref_off[ntri+1], boxes[nleaf, 6], ref_tri[nleaf]) of the leaf references."""
        off = np.zeros(self.ntri + 1, np.uint32)
        n = lib().orc_leaf_refs(C.byref(self.s), _ptr(off))
        if n <= 0:
            raise RuntimeError(f"orc_leaf_refs failed: {n}")
        boxes = np.zeros((n, 6), np.float32)
        tri = np.zeros(n, np.uint32)
        if lib().orc_ref_boxes(C.byref(self.s), _ptr(off), _ptr(boxes), _ptr(tri)) != 0:
            raise RuntimeError("orc_ref_boxes failed")
        return off, boxes, tri

    def build_bvh(self):
        off = np.zeros(self.ntri + 1, np.uint32)
        n = lib().orc_leaf_refs(C.byref(self.s), _ptr(off))
        if n <= 0:
            raise RuntimeError(f"orc_leaf_refs failed: {n}")
        self.nleaf = n
        b = dict(keys=np.zeros(n, np.uint64), refs=np.zeros(n, np.uint32), ids=np.zeros(n, np.uint32),
                 left=np.zeros(max(n - 1, 1), np.uint32),
                 right=np.zeros(max(n - 1, 1), np.uint32), parent=np.zeros(2 * n - 1, np.uint32),
                 bounds=np.zeros((max(n - 1, 1), 6), np.float32),
                 leaf_bounds=np.zeros((n, 6), np.float32))
        st = OrcBvh(n, *(_ptr(b[k]) for k in ("keys", "refs", "ids", "left", "right", "parent", "bounds",
                                                "leaf_bounds")))
        rc = lib().orc_build_bvh(C.byref(self.s), C.byref(st))
        if rc != 0:
            raise RuntimeError(f"orc_build_bvh failed: {rc}")
        self.bvh = b
        self.bvh_struct = st
        return b

    def _bvh_ref(self, use_bvh=True):
        if not use_bvh:
            return None
        if self.bvh is None:
            self.build_bvh()
        return C.byref(self.bvh_struct)


def morton(scene: OracleScene) -> np.ndarray:
    out = np.zeros(scene.ntri, np.uint64)
    rc = lib().orc_morton(C.byref(scene.s), _ptr(out))
    if rc != 0:
        raise RuntimeError("orc_morton failed")
    return out


def morton_boxes(boxes: np.ndarray) -> np.ndarray:
    boxes = np.ascontiguousarray(boxes, np.float32)
    out = np.zeros(boxes.shape[0], np.uint64)
    if lib().orc_morton_boxes(_ptr(boxes), C.c_int64(boxes.shape[0]), _ptr(out)) != 0:
        raise RuntimeError("orc_morton_boxes failed")
    return out


def coc(lens, width: int, z: float) -> float:
    l = lens_struct(lens)
    return float(lib().orc_coc(C.byref(l), int(width), float(z)))


def zone(lens, width: int):
    l = lens_struct(lens)
    a, b = C.c_float(), C.c_float()
    if lib().orc_zone(C.byref(l), int(width), C.byref(a), C.byref(b)) != 0:
        raise ValueError("bad lens")
    return a.value, b.value


def lens_sample(seed, frame, q, k, blades=0, rot=0.0):
    x, y = C.c_float(), C.c_float()
    rc = lib().orc_lens_sample(seed & 0xFFFFFFFF, frame & 0xFFFFFFFF, q & 0xFFFFFFFF,
                               k & 0xFFFFFFFF, blades, rot, C.byref(x), C.byref(y))
    if rc != 0:
        raise ValueError("bad aperture")
    return x.value, y.value


def closest_hit(scene: OracleScene, org: np.ndarray, dirs: np.ndarray, use_bvh=True):
    org = np.ascontiguousarray(org, np.float32).reshape(-1, 3)
    dirs = np.ascontiguousarray(dirs, np.float32).reshape(-1, 3)
    n = org.shape[0]
    hit = np.zeros(n, np.int32)
    t = np.zeros(n, np.float32)
    rc = lib().orc_closest_hit(C.byref(scene.s), scene._bvh_ref(use_bvh), n, _ptr(org), _ptr(dirs),
                               _ptr(hit), _ptr(t))
    if rc != 0:
        raise RuntimeError("orc_closest_hit failed")
    return hit, t


@dataclass
class GBuffer:
    colour: np.ndarray   # (H, W, 4) float32
    depth: np.ndarray    # (H, W) float32
    normal: np.ndarray   # (H, W, 4) float32


def gbuffer(scene: OracleScene, cam, lens, use_bvh=True) -> GBuffer:
    H, W = cam.height, cam.width
    g = GBuffer(np.zeros((H, W, 4), np.float32), np.zeros((H, W), np.float32),
                np.zeros((H, W, 4), np.float32))
    c, l = camera_struct(cam), lens_struct(lens)
    rc = lib().orc_gbuffer(C.byref(scene.s), scene._bvh_ref(use_bvh), C.byref(c), C.byref(l),
                           _ptr(g.colour), _ptr(g.depth), _ptr(g.normal))
    if rc != 0:
        raise RuntimeError("orc_gbuffer failed")
    return g


def taa_offset(width: int, height: int) -> int:
    """Float offset of the final TAA's full-res colour plane in a history
    buffer: after the half-res record (13 floats per half-res pixel), 16-byte
    aligned."""
    return (13 * (width // 2) * (height // 2) + 3) & ~3


def raster_taa_offset(width: int, height: int) -> int:
    """Float offset of the raster TAA's full-res plane (after the final's)."""
    return taa_offset(width, height) + 4 * width * height


def post_taa_offset(width: int, height: int) -> int:
    """Float offset of the post-filter TAA's half-res plane (after the raster's)."""
    return raster_taa_offset(width, height) + 4 * width * height


def history_floats(width: int, height: int) -> int:
    return post_taa_offset(width, height) + 4 * (width // 2) * (height // 2)


def history_zeros(width: int, height: int) -> np.ndarray:
    return np.zeros(history_floats(width, height), np.float32)


def mip_dims(hw: int, hh: int):
    dims = [(hw, hh)]
    for _ in range(3):
        w, h = dims[-1]
        dims.append(((w + 1) >> 1, (h + 1) >> 1))
    return dims


def render_frame(scene: OracleScene, cam, lens, params, gb: GBuffer, hist_in=None,
                 prev_cam=None, prev_lens=None, reset=False, debug=True):
    """One frame of the pass.  Returns a dict with colour, mask, hist_out and
    (when debug) every intermediate stage."""
    W, H = cam.width, cam.height
    hw, hh = W // 2, H // 2
    npx = hw * hh
    T = params.tile
    tw, th = (hw + T - 1) // T, (hh + T - 1) // T
    out = dict(colour=np.zeros((H, W, 4), np.float32), mask=np.zeros((hh, hw), np.uint8),
               hist_out=history_zeros(cam.width, cam.height))
    dbg = None
    if debug:
        rmax = npx * params.m
        mtot = sum(w * h * 4 for w, h in mip_dims(hw, hh))
        arrs = dict(colr=np.zeros((hh, hw, 4), np.float32), zn=np.zeros((hh, hw, 4), np.float32),
                    tile_max=np.zeros((th, tw), np.float32), tile_dil=np.zeros((th, tw), np.float32),
                    pre=np.zeros((hh, hw, 4), np.float32), gather=np.zeros((hh, hw, 4), np.float32),
                    ppmed=np.zeros((hh, hw, 4), np.float32), prev_idx=np.zeros((hh, hw), np.int32),
                    queue=np.zeros(npx, np.uint32), ray_base=np.zeros(npx, np.uint32),
                    ray_hit=np.zeros(rmax, np.int32), ray_t=np.zeros(rmax, np.float32),
                    ray_col=np.zeros((rmax, 4), np.float32), ray_pos=np.zeros((rmax, 4), np.float32),
                    resolve=np.zeros((4, hh, hw, 4), np.float32),
                    temporal=np.zeros((2, hh, hw, 4), np.float32),
                    var_blur=np.zeros((hh, hw), np.float32), rtmed=np.zeros((hh, hw, 4), np.float32),
                    mips=np.zeros(mtot, np.float32), recon=np.zeros((hh, hw, 4), np.float32))
        dbg = OrcDebug(**{k: _ptr(v) for k, v in arrs.items()}, n_masked=0, n_rays=0)
    c, l, p = camera_struct(cam), lens_struct(lens), params_struct(params)
    pc = camera_struct(prev_cam) if prev_cam is not None else None
    pl = lens_struct(prev_lens if prev_lens is not None else lens) if prev_cam is not None else None
    hin = None if hist_in is None else np.ascontiguousarray(hist_in, np.float32)
    colour = np.ascontiguousarray(gb.colour, np.float32)
    depth = np.ascontiguousarray(gb.depth, np.float32)
    normal = np.ascontiguousarray(gb.normal, np.float32)
    rc = lib().orc_render_frame(
        C.byref(scene.s), scene._bvh_ref(True), C.byref(c), C.byref(l),
        C.byref(pc) if pc is not None else None, C.byref(pl) if pl is not None else None,
        1 if (reset or hin is None) else 0, C.byref(p), _ptr(colour), _ptr(depth), _ptr(normal),
        _ptr(hin), _ptr(out["hist_out"]), _ptr(out["colour"]), _ptr(out["mask"]),
        C.byref(dbg) if dbg is not None else None)
    if rc != 0:
        raise RuntimeError(f"orc_render_frame failed: {rc}")
    if debug:
        P, R = int(dbg.n_masked), int(dbg.n_rays)
        arrs["queue"] = arrs["queue"][:P]
        arrs["ray_base"] = arrs["ray_base"][:P]
        for k in ("ray_hit", "ray_t", "ray_col", "ray_pos"):
            arrs[k] = arrs[k][:R]
        out.update(arrs)
        out["n_masked"], out["n_rays"] = P, R
    return out


def pixel_estimate(scene: OracleScene, cam, lens, qlist, spp: int):
    q = np.ascontiguousarray(qlist, np.uint32)
    out = np.zeros((q.size, 3), np.float32)
    c, l = camera_struct(cam), lens_struct(lens)
    rc = lib().orc_pixel_estimate(C.byref(scene.s), scene._bvh_ref(True), C.byref(c), C.byref(l),
                                  q.size, _ptr(q), int(spp), _ptr(out))
    if rc != 0:
        raise RuntimeError("orc_pixel_estimate failed")
    return out


def lens_integral(scene: OracleScene, cam, lens, qlist, grid: int = 64):
    q = np.ascontiguousarray(qlist, np.uint32)
    out = np.zeros((q.size, 3), np.float32)
    c, l = camera_struct(cam), lens_struct(lens)
    rc = lib().orc_lens_integral(C.byref(scene.s), scene._bvh_ref(True), C.byref(c), C.byref(l),
                                 q.size, _ptr(q), int(grid), _ptr(out))
    if rc != 0:
        raise RuntimeError("orc_lens_integral failed")
    return out
