"""Python binding of libhair.so (ctypes): argument marshalling only.

Every step of the render runs in the library's HIP kernels; torch supplies device memory
(tensors passed by data pointer) and streams.  The names mirror include/hair.h.  When the
library is missing this module raises at import: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HAIR_LIBRARY may name another build of the same library (e.g. an instrumented one).
LIB_PATH = os.environ.get("HAIR_LIBRARY", os.path.join(HERE, "libhair.so"))

HAIR_OK, HAIR_EINVAL, HAIR_ENOMEM, HAIR_ENOENT, HAIR_EDEVICE, HAIR_ERANGE = 0, -1, -2, -3, -4, -5
HAIR_MAX_LIGHTS = 8
HAIR_PIXEL_CAPACITY = 1536
HAIR_TILE = 16

EXPORTS = [
    "hair_version", "hair_last_error", "hair_device_count", "hair_ctx_create", "hair_ctx_destroy",
    "hair_ctx_memory", "hair_ws_create", "hair_ws_destroy", "hair_ws_estimate", "hair_ws_memory", "hair_ws_set_limit", "hair_ws_trim", "hair_upload", "hair_release",
    "hair_build_lod", "hair_lod_info", "hair_get_lod", "hair_set_lod", "hair_set_cluster_params",
    "hair_select_level", "hair_render", "hair_render_backward", "hair_debug_segments", "hair_debug_bins",
    "hair_debug_fragments", "hair_lod_groups", "hair_lod_init", "hair_render_mixed", "hair_render_shadowed",
    "hair_debug_dom", "hair_render_curved", "hair_render_async", "hair_ws_finish", "hair_render_noalloc",
    "hair_noalloc_scratch_bytes", "hair_debug_issue_rate",
    "hair_render_mixed_shadowed",
]


class HairError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hair error {code}: {msg}")
        self.code = code


MODEL_RTTRT, MODEL_RTTD = 0, 1


class hair_material(C.Structure):
    _fields_ = [("eta", C.c_float), ("alpha", C.c_float), ("beta_m", C.c_float), ("beta_n", C.c_float),
                ("model", C.c_int32), ("beta_r", C.c_float), ("beta_tt", C.c_float), ("gamma_tt", C.c_float),
                ("a_r", C.c_float * 3), ("a_tt", C.c_float * 3), ("a_d", C.c_float * 3)]


def make_material(material) -> hair_material:
    """hair_material from an object with the struct's field names (model defaults to
    R / TT / TRT) or from a sequence (eta, alpha, beta_m, beta_n)."""
    if not hasattr(material, "eta"):
        return hair_material(*[float(v) for v in material])
    m = hair_material(float(material.eta), float(material.alpha), float(material.beta_m), float(material.beta_n),
                      int(getattr(material, "model", MODEL_RTTRT)))
    if m.model == MODEL_RTTD:
        m.beta_r, m.beta_tt, m.gamma_tt = float(material.beta_r), float(material.beta_tt), float(material.gamma_tt)
        for name in ("a_r", "a_tt", "a_d"):
            getattr(m, name)[:] = [float(v) for v in getattr(material, name)]
    return m


class hair_shadow(C.Structure):
    _fields_ = [("resolution", C.c_int32), ("layers", C.c_int32), ("layer_depth", C.c_float)]


class hair_camera(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("rot", C.c_float * 9), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("z_near", C.c_float)]


class hair_light(C.Structure):
    _fields_ = [("kind", C.c_int32), ("vec", C.c_float * 3), ("rgb", C.c_float * 3)]


class hair_stats(C.Structure):
    _fields_ = [("fragments", C.c_uint64), ("pairs", C.c_uint64), ("segments", C.c_uint32),
                ("segments_visible", C.c_uint32), ("segments_culled_long", C.c_uint32),
                ("overflow_pixels", C.c_uint32), ("ms_total", C.c_float), ("ms_project", C.c_float),
                ("ms_bin", C.c_float), ("ms_tile", C.c_float), ("deep_pixels", C.c_uint32),
                ("batches", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    # torch first: its HIP runtime (same soname as the system one) then serves libhair.so too,
    # so device pointers and streams from torch belong to the runtime the library calls
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2405_10565_amd.build.build() (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, U64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_float
    fp = C.POINTER(C.c_float)
    ip = C.POINTER(C.c_int32)
    up = C.POINTER(C.c_uint32)
    sig = {
        "hair_version": ([], C.c_int),
        "hair_last_error": ([], C.c_char_p),
        "hair_device_count": ([], C.c_int),
        "hair_ctx_create": ([I32, U64, C.POINTER(P)], C.c_int),
        "hair_ctx_destroy": ([P], C.c_int),
        "hair_ctx_memory": ([P, C.POINTER(U64), C.POINTER(U64)], C.c_int),
        "hair_ws_create": ([P, U64, C.POINTER(P)], C.c_int),
        "hair_ws_destroy": ([P], C.c_int),
        "hair_ws_estimate": ([I64, I32, I32, I64], U64),
        "hair_ws_memory": ([P, C.POINTER(U64), C.POINTER(U64)], C.c_int),
        "hair_ws_set_limit": ([P, U64], C.c_int),
        "hair_ws_trim": ([P], C.c_int),
        "hair_upload": ([P, I32, I32, fp, fp, fp, C.POINTER(hair_material), P, ip], C.c_int),
        "hair_release": ([P, I32], C.c_int),
        "hair_build_lod": ([P, I32, I32, ip, ip, P], C.c_int),
        "hair_lod_info": ([P, I32, ip, ip, I32, ip], C.c_int),
        "hair_get_lod": ([P, I32, I32, I32, fp, fp, fp, ip, fp, fp], C.c_int),
        "hair_set_lod": ([P, I32, I32, I32, fp, fp, fp, ip, fp, fp, P], C.c_int),
        "hair_set_cluster_params": ([P, I32, I32, P, P, P, P], C.c_int),
        "hair_select_level": ([P, P, I32, C.POINTER(hair_camera), F, P, ip], C.c_int),
        "hair_render": ([P, P, I32, I32, C.POINTER(hair_camera), C.POINTER(hair_light), I32, P, P,
                         C.POINTER(hair_stats)], C.c_int),
        "hair_render_async": ([P, P, I32, I32, C.POINTER(hair_camera), C.POINTER(hair_light), I32, P, P], C.c_int),
        "hair_ws_finish": ([P, C.POINTER(hair_stats)], C.c_int),
        "hair_render_noalloc": ([P, I32, I32, C.POINTER(hair_camera), C.POINTER(hair_light), I32, P, P,
                                 C.POINTER(hair_stats)], C.c_int),
        "hair_noalloc_scratch_bytes": ([], U64),
        "hair_debug_issue_rate": ([P, I32, I32, C.POINTER(C.c_double)], C.c_int),
        "hair_render_backward": ([P, P, I32, I32, C.POINTER(hair_camera), C.POINTER(hair_light), I32, P, P, P, P, P],
                                 C.c_int),
        "hair_lod_groups": ([P, I32, ip], C.c_int),
        "hair_lod_init": ([P, P, I32, C.POINTER(hair_camera), F, P, P], C.c_int),
        "hair_render_mixed": ([P, P, I32, C.POINTER(hair_camera), C.POINTER(hair_light), I32, P, F, P, P,
                               C.POINTER(hair_stats)], C.c_int),
        "hair_render_mixed_shadowed": ([P, P, I32, C.POINTER(hair_camera), C.POINTER(hair_light), I32, P, F,
                                        C.POINTER(hair_shadow), P, P, C.POINTER(hair_stats)], C.c_int),
        "hair_render_shadowed": ([P, P, I32, I32, C.POINTER(hair_camera), C.POINTER(hair_light), I32,
                                  C.POINTER(hair_shadow), P, P, C.POINTER(hair_stats)], C.c_int),
        "hair_debug_dom": ([P, I32, fp, fp], C.c_int),
        "hair_render_curved": ([P, P, I32, I32, C.POINTER(hair_camera), C.POINTER(hair_light), I32, I32, I32, P, P,
                                C.POINTER(hair_stats)], C.c_int),
        "hair_debug_segments": ([P, I64, ip, fp], C.c_int),
        "hair_debug_bins": ([P, I64, up, I64, up], C.c_int),
        "hair_debug_fragments": ([P, P, I32, I32, C.POINTER(hair_camera), C.POINTER(hair_light), I32, I32, I32, I32,
                                  I32, up, I64, up, up, fp, fp, P], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def last_error() -> str:
    return (lib.hair_last_error() or b"").decode()


def check(rc: int):
    if rc != HAIR_OK:
        raise HairError(rc, last_error())
    return rc


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _uptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def make_camera(cam) -> hair_camera:
    """From an object with pos, rot (3x3), fx, fy, cx, cy, width, height, z_near."""
    c = hair_camera()
    c.pos[:] = [float(v) for v in np.asarray(cam.pos, dtype=np.float32)]
    c.rot[:] = [float(v) for v in np.asarray(cam.rot, dtype=np.float32).reshape(9)]
    c.fx, c.fy, c.cx, c.cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    c.width, c.height = int(cam.width), int(cam.height)
    c.z_near = float(np.float32(cam.z_near))
    return c


def make_lights(lights):
    arr = (hair_light * len(lights))()
    for i, l in enumerate(lights):
        arr[i].kind = int(l.kind)
        arr[i].vec[:] = [float(v) for v in np.asarray(l.vec, dtype=np.float32)]
        arr[i].rgb[:] = [float(v) for v in np.asarray(l.rgb, dtype=np.float32)]
    return arr, len(lights)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class Workspace:
    def __init__(self, ctx: "Context", max_bytes: int = 0):
        self.ctx = ctx
        h = C.c_void_p()
        check(lib.hair_ws_create(ctx.handle, max_bytes, C.byref(h)))
        self.handle = h
        self._pending_out = None
        ctx._workspaces.add(self)

    def finish(self, raise_on_error: bool = True):
        """Wait for the frame of Context.render_async (hair_ws_finish): (stats dict, status)."""
        st = hair_stats()
        rc = lib.hair_ws_finish(self.handle, C.byref(st))
        self._pending_out = None
        if raise_on_error:
            check(rc)
        return st.as_dict(), rc

    def memory(self):
        """(bytes held on the device, limit) of the workspace (hair_ws_memory)."""
        h, m = C.c_uint64(), C.c_uint64()
        check(lib.hair_ws_memory(self.handle, C.byref(h), C.byref(m)))
        return h.value, m.value

    def set_limit(self, max_bytes: int):
        check(lib.hair_ws_set_limit(self.handle, int(max_bytes)))

    def trim(self):
        check(lib.hair_ws_trim(self.handle))

    def close(self):
        if self.handle:
            lib.hair_ws_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class LodLevel:
    centers: np.ndarray   # f32 [K, S+1, 3]
    ahat: np.ndarray      # f32 [K, S, 3]
    axes: np.ndarray      # f32 [K, S, 2]
    n_total: np.ndarray   # i32 [K]
    sigma_a: np.ndarray   # f32 [3, K]
    r: np.ndarray         # f32 [K]


class Context:
    """A library context on one device (device=-1: host-only, validation only)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = C.c_void_p()
        check(lib.hair_ctx_create(device, budget_bytes, C.byref(h)))
        self.handle = h
        self.device = device
        self._workspaces = weakref.WeakSet()

    def close(self):
        """Destroy the context's open workspaces, then the context (the C-ABI requires a
        workspace to be destroyed before its context)."""
        if self.handle:
            for ws in list(self._workspaces):
                ws.close()
            lib.hair_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def memory(self):
        u, b = C.c_uint64(), C.c_uint64()
        check(lib.hair_ctx_memory(self.handle, C.byref(u), C.byref(b)))
        return u.value, b.value

    def workspace(self, max_bytes: int = 0) -> Workspace:
        return Workspace(self, max_bytes)

    def upload(self, n_strands, verts_per_strand, xyz_soa, width, sigma_a_soa, material, stream=0) -> int:
        xyz = np.ascontiguousarray(xyz_soa, dtype=np.float32)
        w = np.ascontiguousarray(width, dtype=np.float32)
        sg = np.ascontiguousarray(sigma_a_soa, dtype=np.float32)
        m = make_material(material)
        aid = C.c_int32()
        check(lib.hair_upload(self.handle, int(n_strands), int(verts_per_strand), _fptr(xyz), _fptr(w), _fptr(sg),
                              C.byref(m), C.c_void_p(stream), C.byref(aid)))
        return aid.value

    def upload_asset(self, asset, stream=0) -> int:
        return self.upload(asset.n_strands, asset.verts_per_strand, asset.xyz, asset.width, asset.sigma_a,
                           asset.material, stream)

    def release(self, asset: int):
        check(lib.hair_release(self.handle, asset))

    def build_lod(self, asset: int, assigns, stream=0):
        n_levels = len(assigns)
        if n_levels == 0:
            check(lib.hair_build_lod(self.handle, asset, 0, None, None, C.c_void_p(stream)))
            return
        assign = np.ascontiguousarray(np.stack([np.asarray(a, np.int32) for a in assigns]), dtype=np.int32)
        ncl = np.array([int(a.max()) + 1 for a in assign], dtype=np.int32)
        check(lib.hair_build_lod(self.handle, asset, n_levels, _iptr(ncl), _iptr(assign), C.c_void_p(stream)))

    def lod_info(self, asset: int):
        nl, S = C.c_int32(), C.c_int32()
        counts = np.zeros(65, dtype=np.int32)
        check(lib.hair_lod_info(self.handle, asset, C.byref(nl), _iptr(counts), 65, C.byref(S)))
        return nl.value, counts[: nl.value + 1].tolist(), S.value

    def get_lod(self, asset: int, level: int) -> LodLevel:
        _, counts, S = self.lod_info(asset)
        K = counts[level]
        out = LodLevel(np.zeros((K, S + 1, 3), np.float32), np.zeros((K, S, 3), np.float32),
                       np.zeros((K, S, 2), np.float32), np.zeros(K, np.int32), np.zeros((3, K), np.float32),
                       np.zeros(K, np.float32))
        check(lib.hair_get_lod(self.handle, asset, level, K, _fptr(out.centers), _fptr(out.ahat), _fptr(out.axes),
                               _iptr(out.n_total), _fptr(out.sigma_a), _fptr(out.r)))
        return out

    def set_lod(self, asset: int, level: int, lod, stream=0):
        g = lambda k, dt: np.ascontiguousarray(lod[k] if isinstance(lod, dict) else getattr(lod, k), dtype=dt)
        centers, ahat, axes = g("centers", np.float32), g("ahat", np.float32), g("axes", np.float32)
        n_total, sig, r = g("n_total", np.int32), g("sigma_a", np.float32), g("r", np.float32)
        check(lib.hair_set_lod(self.handle, asset, level, int(n_total.size), _fptr(centers), _fptr(ahat), _fptr(axes),
                               _iptr(n_total), _fptr(sig), _fptr(r), C.c_void_p(stream)))

    def set_cluster_params(self, asset: int, level: int, axes=None, r=None, sigma_a=None, stream=None):
        p = lambda t: C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)
        check(lib.hair_set_cluster_params(self.handle, asset, level, p(axes), p(r), p(sigma_a), _stream_ptr(stream)))

    def select_level(self, asset: int, cam, eps_w: float = 2.0, ws: Workspace | None = None, stream=None) -> int:
        c = make_camera(cam)
        out = C.c_int32()
        check(lib.hair_select_level(self.handle, ws.handle if ws else None, asset, C.byref(c), float(eps_w),
                                    _stream_ptr(stream), C.byref(out)))
        return out.value

    def render(self, asset: int, level: int, cam, lights, out=None, ws: Workspace | None = None, stream=None,
               raise_on_error: bool = True):
        """Render into `out` (torch float32 [H, W, 4] on the context's device; allocated if None).
        Returns (out, stats dict, status code)."""
        import torch
        c = make_camera(cam)
        la, nl = make_lights(lights)
        if out is None:
            out = torch.empty((c.height, c.width, 4), dtype=torch.float32, device=f"cuda:{self.device}")
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
        assert tuple(out.shape) == (c.height, c.width, 4)
        st = hair_stats()
        rc = lib.hair_render(self.handle, ws.handle if ws else None, asset, level, C.byref(c), la, nl,
                             C.c_void_p(out.data_ptr()), _stream_ptr(stream), C.byref(st))
        if raise_on_error:
            check(rc)
        return out, st.as_dict(), rc

    def render_noalloc(self, asset: int, level: int, cam, lights, out, stream=None, raise_on_error: bool = True):
        """hair_render_noalloc into `out` (torch float32 [H, W, 4] on the context's device, given
        by the caller: the call allocates nothing).  Returns (out, stats dict, status code)."""
        import torch
        c = make_camera(cam)
        la, nl = make_lights(lights)
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
        assert tuple(out.shape) == (c.height, c.width, 4)
        st = hair_stats()
        rc = lib.hair_render_noalloc(self.handle, asset, level, C.byref(c), la, nl, C.c_void_p(out.data_ptr()),
                                     _stream_ptr(stream), C.byref(st))
        if raise_on_error:
            check(rc)
        return out, st.as_dict(), rc

    def render_async(self, asset: int, level: int, cam, lights, out, ws: Workspace, stream=None):
        """Enqueue a frame into `out` on `ws` without waiting (hair_render_async); ws.finish()
        returns its (stats dict, status code)."""
        import torch
        c = make_camera(cam)
        la, nl = make_lights(lights)
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
        assert tuple(out.shape) == (c.height, c.width, 4)
        check(lib.hair_render_async(self.handle, ws.handle, asset, level, C.byref(c), la, nl,
                                    C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        ws._pending_out = out      # keeps the output alive until the frame is finished

    def render_shadowed(self, asset: int, level: int, cam, lights, shadow=(512, 4, 0.02), out=None,
                        ws: Workspace | None = None, stream=None, raise_on_error: bool = True):
        """render with deep opacity map shadows; shadow = (resolution, layers, layer_depth)."""
        import torch
        c = make_camera(cam)
        la, nl = make_lights(lights)
        sh = hair_shadow(int(shadow[0]), int(shadow[1]), float(shadow[2]))
        if out is None:
            out = torch.empty((c.height, c.width, 4), dtype=torch.float32, device=f"cuda:{self.device}")
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
        assert tuple(out.shape) == (c.height, c.width, 4)
        st = hair_stats()
        rc = lib.hair_render_shadowed(self.handle, ws.handle if ws else None, asset, level, C.byref(c), la, nl,
                                      C.byref(sh), C.c_void_p(out.data_ptr()), _stream_ptr(stream), C.byref(st))
        if raise_on_error:
            check(rc)
        return out, st.as_dict(), rc

    def render_curved(self, asset: int, level: int, cam, lights, max_px: int = 4, max_sub: int = 16, out=None,
                      ws: Workspace | None = None, stream=None, raise_on_error: bool = True):
        """render a thick-hair level with curved (Catmull-Rom) centre lines tessellated to at
        most max_px pixels per step (at most max_sub steps per segment)."""
        import torch
        c = make_camera(cam)
        la, nl = make_lights(lights)
        if out is None:
            out = torch.empty((c.height, c.width, 4), dtype=torch.float32, device=f"cuda:{self.device}")
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
        assert tuple(out.shape) == (c.height, c.width, 4)
        st = hair_stats()
        rc = lib.hair_render_curved(self.handle, ws.handle if ws else None, asset, level, C.byref(c), la, nl,
                                    int(max_px), int(max_sub), C.c_void_p(out.data_ptr()), _stream_ptr(stream),
                                    C.byref(st))
        if raise_on_error:
            check(rc)
        return out, st.as_dict(), rc

    def lod_groups(self, asset: int) -> int:
        out = C.c_int32()
        check(lib.hair_lod_groups(self.handle, asset, C.byref(out)))
        return out.value

    def lod_init(self, asset: int, cam, eps_w: float, levels, ws: Workspace | None = None, stream=None):
        """Initial per-(group, segment) levels into `levels` (torch int32 [G, S] on the device)."""
        import torch
        assert levels.is_cuda and levels.dtype == torch.int32 and levels.is_contiguous()
        c = make_camera(cam)
        check(lib.hair_lod_init(self.handle, ws.handle if ws else None, asset, C.byref(c), float(eps_w),
                                C.c_void_p(levels.data_ptr()), _stream_ptr(stream)))
        return levels

    def render_mixed(self, asset: int, cam, lights, levels, eps_w: float = 0.0, out=None, ws: Workspace | None = None,
                     stream=None, raise_on_error: bool = True):
        """Mixed-level frame at `levels` (torch int32 [G, S]); eps_w > 0 updates them in place
        for the next frame.  Returns (out, stats dict, status code)."""
        import torch
        assert levels.is_cuda and levels.dtype == torch.int32 and levels.is_contiguous()
        c = make_camera(cam)
        la, nl = make_lights(lights)
        if out is None:
            out = torch.empty((c.height, c.width, 4), dtype=torch.float32, device=f"cuda:{self.device}")
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
        assert tuple(out.shape) == (c.height, c.width, 4)
        st = hair_stats()
        rc = lib.hair_render_mixed(self.handle, ws.handle if ws else None, asset, C.byref(c), la, nl,
                                   C.c_void_p(levels.data_ptr()), float(eps_w), C.c_void_p(out.data_ptr()),
                                   _stream_ptr(stream), C.byref(st))
        if raise_on_error:
            check(rc)
        return out, st.as_dict(), rc

    def render_mixed_shadowed(self, asset: int, cam, lights, levels, shadow=(512, 4, 0.02), eps_w: float = 0.0,
                              out=None, ws: Workspace | None = None, stream=None, raise_on_error: bool = True):
        """Mixed-level frame with deep opacity map shadows; shadow = (resolution, layers,
        layer_depth).  Returns (out, stats dict, status code)."""
        import torch
        assert levels.is_cuda and levels.dtype == torch.int32 and levels.is_contiguous()
        c = make_camera(cam)
        la, nl = make_lights(lights)
        sh = hair_shadow(int(shadow[0]), int(shadow[1]), float(shadow[2]))
        if out is None:
            out = torch.empty((c.height, c.width, 4), dtype=torch.float32, device=f"cuda:{self.device}")
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
        assert tuple(out.shape) == (c.height, c.width, 4)
        st = hair_stats()
        rc = lib.hair_render_mixed_shadowed(self.handle, ws.handle if ws else None, asset, C.byref(c), la, nl,
                                            C.c_void_p(levels.data_ptr()), float(eps_w), C.byref(sh),
                                            C.c_void_p(out.data_ptr()), _stream_ptr(stream), C.byref(st))
        if raise_on_error:
            check(rc)
        return out, st.as_dict(), rc

    def render_backward(self, asset: int, level: int, cam, lights, d_rgba, d_axes, d_r, d_sigma_a,
                        ws: Workspace | None = None, stream=None):
        c = make_camera(cam)
        la, nl = make_lights(lights)
        for t in (d_rgba, d_axes, d_r, d_sigma_a):
            assert t.is_cuda and t.is_contiguous() and t.dtype.is_floating_point
        check(lib.hair_render_backward(self.handle, ws.handle if ws else None, asset, level, C.byref(c), la, nl,
                                       C.c_void_p(d_rgba.data_ptr()), C.c_void_p(d_axes.data_ptr()),
                                       C.c_void_p(d_r.data_ptr()), C.c_void_p(d_sigma_a.data_ptr()),
                                       _stream_ptr(stream)))

    def issue_rate(self, kind: int, iters: int = 4096) -> float:
        """Lane-operations per second of one instruction kind (hair_debug_issue_rate)."""
        v = C.c_double()
        check(lib.hair_debug_issue_rate(self.handle, int(kind), int(iters), C.byref(v)))
        return v.value

    def debug_segments(self, ws: Workspace, n: int):
        ri = np.zeros((n, 6), np.int32)
        rf = np.zeros((n, 3), np.float32)
        check(lib.hair_debug_segments(ws.handle, n, _iptr(ri), _fptr(rf)))
        return ri, rf

    def debug_dom(self, ws: Workspace, light: int, R: int):
        """(texels float32 [R*R, 8], grid float32 [16]) of the last shadowed render on ws."""
        tex = np.zeros((R * R, 8), np.float32)
        grid = np.zeros(16, np.float32)
        check(lib.hair_debug_dom(ws.handle, light, _fptr(tex), _fptr(grid)))
        return tex, grid

    def debug_bins(self, ws: Workspace, n_tiles: int, n_pairs: int):
        ts = np.zeros(n_tiles + 1, np.uint32)
        segs = np.zeros(max(n_pairs, 1), np.uint32)
        check(lib.hair_debug_bins(ws.handle, n_tiles, _uptr(ts), n_pairs, _uptr(segs)))
        return ts, segs[:n_pairs]

    def debug_fragments(self, asset, level, cam, lights, x0, y0, w, h, cap, ws: Workspace | None = None, stream=None):
        c = make_camera(cam)
        la, nl = make_lights(lights)
        counts = np.zeros(w * h, np.uint32)
        keys = np.zeros(cap, np.uint32)
        segs = np.zeros(cap, np.uint32)
        alpha = np.zeros(cap, np.float32)
        hoff = np.zeros(cap, np.float32)
        check(lib.hair_debug_fragments(self.handle, ws.handle if ws else None, asset, level, C.byref(c), la, nl,
                                       x0, y0, w, h, _uptr(counts), cap, _uptr(keys), _uptr(segs), _fptr(alpha),
                                       _fptr(hoff), _stream_ptr(stream)))
        n = int(counts.sum())
        return counts.reshape(h, w), keys[:n], segs[:n], alpha[:n], hoff[:n]


def ws_estimate(n_segments: int, width: int, height: int, pairs_estimate: int = 0) -> int:
    return int(lib.hair_ws_estimate(n_segments, width, height, pairs_estimate))


def device_count() -> int:
    return int(lib.hair_device_count())
