"""Thin ctypes binding of libdof (include/dof.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every stage of the pass runs in the library's HIP kernels.  Loading
fails loudly when libdof.so has not been built -- there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdof.so")

_f3 = C.c_float * 3

DOF_OK, DOF_E_INVALID, DOF_E_NOMEM, DOF_E_DEVICE, DOF_E_STATE, DOF_E_UNSUPPORTED = range(6)
RGBA32F, RGBA16F = 0, 1
MASK_ADAPTIVE, MASK_FIXED, MASK_ALL = 0, 1, 2


class DofCamera(C.Structure):
    _fields_ = [("pos", _f3), ("right", _f3), ("up", _f3), ("fwd", _f3),
                ("width", C.c_int32), ("height", C.c_int32), ("frame", C.c_uint32), ("seed", C.c_uint32),
                ("jitter", C.c_float * 2)]


class DofLens(C.Structure):
    _fields_ = [("focal", C.c_float), ("fnum", C.c_float), ("focus", C.c_float), ("sensor", C.c_float),
                ("blades", C.c_int32), ("blade_rot", C.c_float)]


class DofParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("m", C.c_int32), ("s", C.c_float), ("var_mask_w", C.c_float),
                ("alpha", C.c_float), ("alpha_motion", C.c_float), ("var_recon_w", C.c_float),
                ("b_max", C.c_float), ("h_edge", C.c_float), ("lod_scale", C.c_float), ("lod_max", C.c_float),
                ("depth_range", C.c_float), ("r_max", C.c_float), ("tile", C.c_int32), ("l_spec", C.c_float),
                ("mask_mode", C.c_int32), ("trace_blocks", C.c_int32), ("timing", C.c_int32),
                ("pp_polygon", C.c_int32), ("taa", C.c_int32), ("ray_records", C.c_int32), ("composite_literal", C.c_int32),
                ("gather_window", C.c_int32), ("trace_stack", C.c_int32), ("trace_grab", C.c_int32),
                ("trace_refill", C.c_int32), ("trace_leaf_batch", C.c_int32), ("trace_order", C.c_int32),
                ("trace_steps", C.c_int32)]

# launch-shape knobs of dof_params (0 = library default), set from a dict
KNOBS = ("gather_window", "trace_stack", "trace_grab", "trace_refill", "trace_leaf_batch", "trace_order",
         "trace_steps")


class DofGBuffer(C.Structure):
    _fields_ = [("colour", C.c_void_p), ("colour_format", C.c_int32), ("depth", C.c_void_p),
                ("normal", C.c_void_p), ("normal_format", C.c_int32)]


class DofHistoryIO(C.Structure):
    _fields_ = [("in_", C.c_void_p), ("out", C.c_void_p), ("prev_camera", DofCamera), ("prev_lens", DofLens),
                ("reset", C.c_int32)]


class DofStats(C.Structure):
    _fields_ = [("masked_px", C.c_uint32), ("rays", C.c_uint32), ("node_visits", C.c_uint64),
                ("tri_tests", C.c_uint64), ("reserved", C.c_uint32 * 2)]


class DofFrameOut(C.Structure):
    _fields_ = [("colour", C.c_void_p), ("colour_format", C.c_int32), ("mask", C.c_void_p), ("stats", C.c_void_p)]


class DofBatchItem(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("camera", DofCamera), ("lens", DofLens), ("gbuffer", DofGBuffer),
                ("history", DofHistoryIO), ("out", DofFrameOut), ("scratch", C.c_void_p), ("scratch_bytes", C.c_size_t)]


class DofSceneDesc(C.Structure):
    _fields_ = [("ntri", C.c_int32), ("verts", C.c_void_p), ("albedo", C.c_void_p), ("light_dir", _f3),
                ("light_rad", _f3), ("ambient", _f3), ("sky", _f3), ("leaf_split", C.c_int32)]


class DofBvhView(C.Structure):
    _fields_ = [("ntri", C.c_int32), ("nleaf", C.c_int32), ("keys", C.c_void_p), ("ids", C.c_void_p),
                ("parent", C.c_void_p), ("nodes", C.c_void_p), ("tris", C.c_void_p),
                ("nodes16", C.c_void_p)]


DEBUG_FIELDS = ("colr", "zn", "tile_max", "tile_dil", "pre", "gather", "ppmed", "prev_idx", "queue", "ray_base",
                "ray_hit", "ray_t", "ray_col", "ray_pos", "resolve", "temporal", "var_blur", "rtmed", "mips",
                "recon", "counters")


class DofDebugView(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in DEBUG_FIELDS]


EXPORTS = ("dof_abi_version", "dof_last_error", "dof_default_params", "dof_scene_bytes", "dof_scene_bytes_desc",
           "dof_create_scene",
           "dof_build_bvh", "dof_bvh_view_get", "dof_destroy_scene", "dof_trace_rays", "dof_render_gbuffer",
           "dof_history_bytes", "dof_history_reset", "dof_frame_scratch_bytes", "dof_render_frame",
           "dof_debug_view_get", "dof_stage_times", "dof_batch_bytes", "dof_batch_create", "dof_batch_set",
           "dof_batch_run", "dof_batch_destroy", "dof_reference_scratch_bytes", "dof_render_reference",
           "dof_render_frame_noalloc")
NOALLOC_SCRATCH_BYTES = 64 << 20

STAGES = ("reduce", "dilate", "prefilter", "gather", "median", "mask", "compact", "trace", "resolve", "temporal",
          "blur_median_mips", "recon", "composite")

_lib = None


class DofError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdof error {code}: {msg}")
        self.code = code


def lib():
    """Load libdof.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, P = C.c_void_p, C.POINTER
        L.dof_abi_version.restype = C.c_int32
        L.dof_last_error.restype = C.c_char_p
        L.dof_default_params.argtypes = [P(DofParams)]
        L.dof_default_params.restype = None
        L.dof_scene_bytes.argtypes = [C.c_int32, P(C.c_size_t)]
        L.dof_scene_bytes_desc.argtypes = [P(DofSceneDesc), P(C.c_size_t)]
        L.dof_create_scene.argtypes = [P(DofSceneDesc), vp, C.c_size_t, vp, P(vp)]
        L.dof_build_bvh.argtypes = [vp, vp]
        L.dof_bvh_view_get.argtypes = [vp, P(DofBvhView)]
        L.dof_destroy_scene.argtypes = [vp]
        L.dof_destroy_scene.restype = None
        L.dof_trace_rays.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp]
        L.dof_render_gbuffer.argtypes = [vp, P(DofCamera), P(DofLens), vp, C.c_int32, vp, vp, C.c_int32, vp]
        L.dof_history_bytes.argtypes = [C.c_int32, C.c_int32, P(C.c_size_t)]
        L.dof_history_reset.argtypes = [vp, C.c_int32, C.c_int32, vp]
        L.dof_frame_scratch_bytes.argtypes = [C.c_int32, C.c_int32, P(DofParams), P(C.c_size_t)]
        L.dof_render_frame.argtypes = [vp, P(DofCamera), P(DofLens), P(DofGBuffer), P(DofHistoryIO),
                                       P(DofParams), P(DofFrameOut), vp, C.c_size_t, vp]
        L.dof_debug_view_get.argtypes = [vp, C.c_int32, C.c_int32, P(DofParams), P(DofDebugView)]
        L.dof_stage_times.argtypes = [vp, P(C.c_float), C.c_int32, P(C.c_int32)]
        L.dof_batch_bytes.argtypes = [C.c_int32, P(C.c_size_t)]
        L.dof_batch_create.argtypes = [vp, C.c_size_t, C.c_int32, P(vp)]
        L.dof_batch_set.argtypes = [vp, P(DofBatchItem), C.c_int32, P(DofParams), vp]
        L.dof_batch_run.argtypes = [vp, vp, vp]
        L.dof_reference_scratch_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32, P(C.c_size_t)]
        L.dof_render_reference.argtypes = [vp, P(DofCamera), P(DofLens), C.c_int32, vp, C.c_int32, vp, C.c_size_t, vp]
        L.dof_render_frame_noalloc.argtypes = [vp, P(DofCamera), P(DofLens), P(DofGBuffer), P(DofHistoryIO),
                                               P(DofParams), P(DofFrameOut), vp]
        L.dof_batch_destroy.argtypes = [vp]
        L.dof_batch_destroy.restype = None
        for name in EXPORTS:
            if name not in ("dof_abi_version", "dof_last_error", "dof_default_params", "dof_destroy_scene",
                            "dof_batch_destroy"):
                getattr(L, name).restype = C.c_int32
        if L.dof_abi_version() != 6:
            raise ImportError("libdof ABI version mismatch")
        _lib = L
    return _lib


def check(code: int):
    if code != DOF_OK:
        raise DofError(code, lib().dof_last_error().decode(errors="replace"))


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def camera_struct(cam) -> DofCamera:
    return DofCamera(_f3(*cam.pos), _f3(*cam.right), _f3(*cam.up), _f3(*cam.fwd), cam.width, cam.height,
                     cam.frame & 0xFFFFFFFF, cam.seed & 0xFFFFFFFF, (C.c_float * 2)(*getattr(cam, "jitter", (0.0, 0.0))))


def lens_struct(lens) -> DofLens:
    return DofLens(lens.focal, lens.fnum, lens.focus, lens.sensor, lens.blades, lens.blade_rot)


def params_struct(p, trace_blocks: int = 0, timing: bool = False, ray_records: bool = False,
                  knobs: dict | None = None) -> DofParams:
    s = DofParams()
    lib().dof_default_params(C.byref(s))
    for k in ("m", "s", "var_mask_w", "alpha", "alpha_motion", "var_recon_w", "b_max", "h_edge", "lod_scale",
              "lod_max", "depth_range", "r_max", "tile", "l_spec", "mask_mode"):
        setattr(s, k, getattr(p, k))
    s.pp_polygon = int(getattr(p, "pp_polygon", 0))
    s.taa = int(getattr(p, "taa", 0))
    s.composite_literal = int(getattr(p, "composite_literal", 0))
    s.trace_blocks = trace_blocks
    s.timing = 1 if timing else 0
    s.ray_records = 1 if ray_records else 0
    for k, v in (knobs or {}).items():
        assert k in KNOBS, k
        setattr(s, k, int(v))
    return s


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Scene:
    """A scene resident in a caller-owned (torch) device arena."""

    def __init__(self, scene, device="cuda", leaf_split=None):
        verts = np.ascontiguousarray(scene.verts, np.float32)
        alb = np.ascontiguousarray(scene.albedo, np.float32)
        n = verts.shape[0]
        if leaf_split is None:
            leaf_split = getattr(scene, "leaf_split", 2)
        desc = DofSceneDesc(n, verts.ctypes.data_as(C.c_void_p), alb.ctypes.data_as(C.c_void_p),
                            _f3(*scene.light_dir), _f3(*scene.light_rad), _f3(*scene.ambient), _f3(*scene.sky),
                            int(leaf_split))
        nbytes = C.c_size_t()
        check(lib().dof_scene_bytes_desc(C.byref(desc), C.byref(nbytes)))
        self.arena = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        check(lib().dof_create_scene(C.byref(desc), _ptr(self.arena), nbytes.value, _stream(), C.byref(h)))
        self.handle = h
        self.ntri = n

    def build_bvh(self):
        check(lib().dof_build_bvh(self.handle, _stream()))

    def bvh_view(self):
        v = DofBvhView()
        check(lib().dof_bvh_view_get(self.handle, C.byref(v)))
        n = v.nleaf
        return dict(nleaf=n, keys=self._slice(v.keys, 8 * n, torch.int64), ids=self._slice(v.ids, 4 * n, torch.int32),
                    parent=self._slice(v.parent, 4 * (2 * n - 1), torch.int32),
                    nodes=self._slice(v.nodes, 64 * max(n - 1, 1), torch.float32),
                    nodes16=self._slice(v.nodes16, 32 * max(n - 1, 1), torch.int32),
                    tris=self._slice(v.tris, 48 * n, torch.float32))

    def _slice(self, ptr, nbytes, dtype):
        off = ptr - self.arena.data_ptr()
        return self.arena[off:off + nbytes].view(dtype)

    def trace_rays(self, org: torch.Tensor, dirs: torch.Tensor):
        n = org.shape[0]
        hit = torch.empty(n, dtype=torch.int32, device=org.device)
        t = torch.empty(n, dtype=torch.float32, device=org.device)
        check(lib().dof_trace_rays(self.handle, n, _ptr(org.contiguous()), _ptr(dirs.contiguous()), _ptr(hit),
                                   _ptr(t), _stream()))
        return hit, t

    def render_gbuffer(self, cam, lens, fmt=RGBA32F, device="cuda"):
        H, W = cam.height, cam.width
        dt = torch.float32 if fmt == RGBA32F else torch.float16
        colour = torch.empty((H, W, 4), dtype=dt, device=device)
        normal = torch.empty((H, W, 4), dtype=dt, device=device)
        depth = torch.empty((H, W), dtype=torch.float32, device=device)
        return self.render_gbuffer_into(cam, lens, colour, depth, normal)

    def render_gbuffer_into(self, cam, lens, colour, depth, normal):
        """Pinhole G-buffer into caller tensors (colour/normal FP32 or FP16)."""
        assert colour.shape == (cam.height, cam.width, 4) and normal.shape == colour.shape
        assert depth.shape == (cam.height, cam.width) and depth.dtype == torch.float32
        cf = RGBA32F if colour.dtype == torch.float32 else RGBA16F
        nf = RGBA32F if normal.dtype == torch.float32 else RGBA16F
        c, l = camera_struct(cam), lens_struct(lens)
        check(lib().dof_render_gbuffer(self.handle, C.byref(c), C.byref(l), _ptr(colour), cf, _ptr(depth),
                                       _ptr(normal), nf, _stream()))
        return colour, depth, normal

    def render_reference(self, cam, lens, spp, fmt=RGBA32F, device="cuda"):
        """The fully ray-traced image (spp thin-lens rays per full-res pixel)."""
        nb = C.c_size_t()
        check(lib().dof_reference_scratch_bytes(cam.width, cam.height, spp, C.byref(nb)))
        scratch = torch.empty(nb.value, dtype=torch.uint8, device=device)
        dt = torch.float32 if fmt == RGBA32F else torch.float16
        colour = torch.empty((cam.height, cam.width, 4), dtype=dt, device=device)
        c, l = camera_struct(cam), lens_struct(lens)
        check(lib().dof_render_reference(self.handle, C.byref(c), C.byref(l), spp, _ptr(colour), fmt,
                                         _ptr(scratch), nb.value, _stream()))
        return colour

    def stage_times(self):
        """Per-stage ms of the last frame rendered with timing on."""
        buf = (C.c_float * len(STAGES))()
        n = C.c_int32()
        check(lib().dof_stage_times(self.handle, buf, len(STAGES), C.byref(n)))
        return dict(zip(STAGES, list(buf)[:n.value]))

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.dof_destroy_scene(self.handle)
        except Exception:
            pass


def scene_bytes(ntri) -> int:
    """Arena bound for ntri triangles of any shape."""
    b = C.c_size_t()
    check(lib().dof_scene_bytes(ntri, C.byref(b)))
    return b.value


def scene_bytes_for(scene, leaf_split=None) -> int:
    """The exact arena size of this scene (its split triangles counted)."""
    verts = np.ascontiguousarray(scene.verts, np.float32)
    alb = np.ascontiguousarray(scene.albedo, np.float32)
    if leaf_split is None:
        leaf_split = getattr(scene, "leaf_split", 2)
    desc = DofSceneDesc(verts.shape[0], verts.ctypes.data_as(C.c_void_p), alb.ctypes.data_as(C.c_void_p),
                        _f3(*scene.light_dir), _f3(*scene.light_rad), _f3(*scene.ambient), _f3(*scene.sky),
                        int(leaf_split))
    b = C.c_size_t()
    check(lib().dof_scene_bytes_desc(C.byref(desc), C.byref(b)))
    return b.value


def history_bytes(W, H) -> int:
    b = C.c_size_t()
    check(lib().dof_history_bytes(W, H, C.byref(b)))
    return b.value


def history_alloc(W, H, device="cuda"):
    return torch.zeros(history_bytes(W, H) // 4, dtype=torch.float32, device=device)


def scratch_bytes(W, H, params, ray_records: bool = False) -> int:
    b = C.c_size_t()
    ps = params_struct(params, ray_records=ray_records)
    check(lib().dof_frame_scratch_bytes(W, H, C.byref(ps), C.byref(b)))
    return b.value


class Frame:
    """Per-resolution buffers of the pass: scratch, outputs, stats."""

    def __init__(self, W, H, params, out_format=RGBA32F, device="cuda", trace_blocks=0, timing=False,
                 ray_records=False, knobs=None):
        self.W, self.H = W, H
        self.params = params
        self.ray_records = ray_records
        self.ps = params_struct(params, trace_blocks, timing, ray_records, knobs)
        self.nbytes = scratch_bytes(W, H, params, ray_records)
        self.scratch = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        dt = torch.float32 if out_format == RGBA32F else torch.float16
        self.out_format = out_format
        self.colour = torch.empty((H, W, 4), dtype=dt, device=device)
        self.mask = torch.empty((H // 2, W // 2), dtype=torch.uint8, device=device)
        self.stats = torch.zeros(8, dtype=torch.int32, device=device)

    def item(self, scene: Scene, cam, lens, gb, hist_in, hist_out, prev_cam=None, prev_lens=None, reset=False,
             stats=None):
        """The frame's arguments as one batch item (see Batch).  stats: a device
        int32 tensor of 8 elements for the frame's counters (default: self.stats)."""
        colour, depth, normal = gb
        cf = RGBA32F if colour.dtype == torch.float32 else RGBA16F
        nf = RGBA32F if normal.dtype == torch.float32 else RGBA16F
        g = DofGBuffer(_ptr(colour), cf, _ptr(depth), _ptr(normal), nf)
        hio = DofHistoryIO(_ptr(hist_in) if hist_in is not None else None, _ptr(hist_out),
                           camera_struct(prev_cam if prev_cam is not None else cam),
                           lens_struct(prev_lens if prev_lens is not None else lens),
                           1 if (reset or hist_in is None or prev_cam is None) else 0)
        if stats is None:
            stats = self.stats
        assert stats.dtype == torch.int32 and stats.numel() == 8 and stats.is_contiguous()
        out = DofFrameOut(_ptr(self.colour), self.out_format, _ptr(self.mask), _ptr(stats))
        return DofBatchItem(scene.handle, camera_struct(cam), lens_struct(lens), g, hio, out, _ptr(self.scratch),
                            self.nbytes)

    def render(self, scene: Scene, cam, lens, gb, hist_in, hist_out, prev_cam=None, prev_lens=None, reset=False,
               stats=None):
        it = self.item(scene, cam, lens, gb, hist_in, hist_out, prev_cam, prev_lens, reset, stats)
        check(lib().dof_render_frame(it.scene, C.byref(it.camera), C.byref(it.lens), C.byref(it.gbuffer),
                                     C.byref(it.history), C.byref(self.ps), C.byref(it.out), it.scratch,
                                     it.scratch_bytes, _stream()))

    def render_noalloc(self, scene: Scene, cam, lens, gb, hist_in, hist_out, prev_cam=None, prev_lens=None,
                       reset=False):
        """The same frame through dof_render_frame_noalloc: the library's own
        scratch buffer instead of this frame's (outputs land in this frame's
        colour, mask and stats; debug() does not see that scratch)."""
        it = self.item(scene, cam, lens, gb, hist_in, hist_out, prev_cam, prev_lens, reset)
        check(lib().dof_render_frame_noalloc(it.scene, C.byref(it.camera), C.byref(it.lens), C.byref(it.gbuffer),
                                             C.byref(it.history), C.byref(self.ps), C.byref(it.out), _stream()))

    def debug(self):
        """Host copies of every intermediate plane (synchronises)."""
        v = DofDebugView()
        check(lib().dof_debug_view_get(_ptr(self.scratch), self.W, self.H, C.byref(self.ps), C.byref(v)))
        base = self.scratch.data_ptr()
        hw, hh = self.W // 2, self.H // 2
        np_ = hw * hh
        T = self.params.tile
        tw, th = (hw + T - 1) // T, (hh + T - 1) // T
        cnt = self._view(v.counters - base, 16, torch.int32).cpu().numpy()
        P, R = int(cnt[0]), int(cnt[1])

        def get(name, nbytes, dtype, shape):
            ptr = getattr(v, name)
            if ptr is None:    # a per-ray plane the frame does not keep
                return None
            return self._view(ptr - base, nbytes, dtype).cpu().numpy().reshape(shape)

        dims = [(hw, hh)]
        for _ in range(3):
            w, h = dims[-1]
            dims.append(((w + 1) >> 1, (h + 1) >> 1))
        mtot = sum(w * h * 4 for w, h in dims)
        return dict(
            colr=get("colr", 16 * np_, torch.float32, (hh, hw, 4)), zn=get("zn", 16 * np_, torch.float32, (hh, hw, 4)),
            tile_max=get("tile_max", 4 * tw * th, torch.float32, (th, tw)),
            tile_dil=get("tile_dil", 4 * tw * th, torch.float32, (th, tw)),
            pre=get("pre", 16 * np_, torch.float32, (hh, hw, 4)),
            gather=get("gather", 16 * np_, torch.float32, (hh, hw, 4)),
            ppmed=get("ppmed", 16 * np_, torch.float32, (hh, hw, 4)),
            prev_idx=get("prev_idx", 4 * np_, torch.int32, (hh, hw)),
            queue=get("queue", 4 * P, torch.int32, (P,)).view(np.uint32),
            ray_base=get("ray_base", 4 * P, torch.int32, (P,)).view(np.uint32),
            ray_hit=get("ray_hit", 4 * R, torch.int32, (R,)), ray_t=get("ray_t", 4 * R, torch.float32, (R,)),
            ray_col=get("ray_col", 16 * R, torch.float32, (R, 4)), ray_pos=get("ray_pos", 16 * R, torch.float32, (R, 4)),
            resolve=get("resolve", 64 * np_, torch.float32, (4, hh, hw, 4)),
            temporal=get("temporal", 32 * np_, torch.float32, (2, hh, hw, 4)),
            var_blur=get("var_blur", 4 * np_, torch.float32, (hh, hw)),
            rtmed=get("rtmed", 16 * np_, torch.float32, (hh, hw, 4)),
            mips=get("mips", 4 * mtot, torch.float32, (mtot,)),
            recon=get("recon", 16 * np_, torch.float32, (hh, hw, 4)),
            n_masked=P, n_rays=R)

    def _view(self, off, nbytes, dtype):
        return self.scratch[off:off + nbytes].view(dtype)


class Batch:
    """Frames of several sessions rendered with one launch per stage.

    set() takes Frame.item(...) records (each frame keeps its own scratch and
    outputs) and uploads the item table; run() launches the pass for all of
    them on the current stream and can be captured in a graph.  Totals of
    the last run (frames, rays, node visits, triangle tests) are in stats.
    """

    def __init__(self, max_items, params, device="cuda", trace_blocks=0, ray_records=False, knobs=None):
        nb = C.c_size_t()
        check(lib().dof_batch_bytes(max_items, C.byref(nb)))
        self.table = torch.empty(nb.value, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        check(lib().dof_batch_create(_ptr(self.table), nb.value, max_items, C.byref(h)))
        self.handle = h
        self.max_items = max_items
        # every item's scratch must be laid out with the same ray_records
        self.ps = params_struct(params, trace_blocks, False, ray_records, knobs)
        self.stats = torch.zeros(6, dtype=torch.int32, device=device)
        self._lib = lib()

    def set(self, items):
        arr = (DofBatchItem * len(items))(*items)
        check(lib().dof_batch_set(self.handle, arr, len(items), C.byref(self.ps), _stream()))

    def run(self):
        check(lib().dof_batch_run(self.handle, _ptr(self.stats), _stream()))

    def totals(self):
        """(frames, rays, node visits, triangle tests) of the last run (synchronises)."""
        s = self.stats.cpu().numpy()
        s64 = s.view(np.int64)
        return int(s[0]), int(s[1]), int(s64[1]), int(s64[2])

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self._lib.dof_batch_destroy(h)
            self.handle = None

