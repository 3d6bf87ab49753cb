"""ctypes binding of libvafr.so with the C names of include/vafr.h.

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Device buffers are torch tensors (memory and streams only); if
the native library is missing, loading fails loudly -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("VAFR_LIB", os.path.join(_PKG, "libvafr.so"))

VAFR_OK = 0
VAFR_E_ARG = -1
VAFR_E_OOM = -2
VAFR_E_HIP = -3
VAFR_E_UNSUPPORTED = -4
VAFR_E_BUDGET = -5
VAFR_E_LATE = -6
VAFR_E_TIMEOUT = -7
ABI_VERSION = 2   # layout of the structures below

VAFR_SHADE_LAMBERT = 0
VAFR_SHADE_PATH = 1
VAFR_LAYOUT_VAFR = 0
VAFR_LAYOUT_LMFR = 1
VAFR_LAYOUT_LAFR = 2

# Symbols declared in include/vafr.h (checked by the CPU test suite).
EXPORTS = (
    "vafr_last_error", "vafr_abi_version", "vafr_lp_layout", "lmfr_lp_layout", "vafr_layout_dims",
    "vafr_layout_tables", "vafr_layout_destroy", "vafr_scene_create", "vafr_scene_get_info",
    "vafr_scene_export", "vafr_scene_destroy", "vafr_shade_lp", "lmfr_shade_lp", "vafr_reconstruct",
    "lmfr_reconstruct", "full_shade", "vafr_count_work", "vafr_batch_create", "vafr_batch_run",
    "vafr_batch_autotune", "vafr_batch_get_config", "vafr_batch_set_config", "vafr_batch_destroy",
    "vafr_batch_set_profiling", "vafr_batch_stage_ms", "vafr_server_create", "vafr_server_add_headset",
    "vafr_server_submit", "vafr_server_poll", "vafr_server_release", "vafr_server_wait_idle", "vafr_server_get_stats",
    "vafr_server_destroy", "vafr_acuity_capped", "vafr_fxaa_lp", "vafr_rep_workspace_bytes", "vafr_shade_lp_rep",
    "lafr_lp_layout", "lafr_shade_lp", "lafr_reconstruct", "vafr_shade_lp_rep_noalloc",
)

VAFR_VIEW_VAFR = 0
VAFR_VIEW_LMFR = 1
VAFR_VIEW_FULL = 2
VAFR_VIEW_LAFR = 3

# LaFR kernel parameters (Sec. 4.1 Eq. (15), Sec. 4.5): a is LMFR's kernel
# exponent in the buffer-to-screen direction; alpha and beta are LaFR's own.
LAFR_A = 0.25
LAFR_ALPHA = 0.85
LAFR_BETA = 0.7


class VafrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class vafr_display(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fov_x_deg", C.c_double), ("fov_y_deg", C.c_double)]


class vafr_acuity(C.Structure):
    _fields_ = [("n_pivots", C.c_int32), ("ecc_deg", C.POINTER(C.c_double)), ("cpd", C.POINTER(C.c_double)),
                ("e_max_deg", C.c_double), ("n_aniso", C.c_int32), ("aniso_ecc_deg", C.POINTER(C.c_double)),
                ("aniso_delta", C.POINTER(C.c_double))]


class vafr_camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("right", C.c_float * 3), ("up", C.c_float * 3), ("forward", C.c_float * 3)]


class vafr_gaze(C.Structure):
    _fields_ = [("x_px", C.c_double), ("y_px", C.c_double)]


class vafr_shading(C.Structure):
    _fields_ = [("light_dir", C.c_float * 3), ("light_rgb", C.c_float * 3), ("ambient", C.c_float * 3),
                ("background", C.c_float * 3), ("shadow_rays", C.c_int32), ("mode", C.c_int32),
                ("bounces", C.c_int32), ("frame", C.c_uint32), ("view", C.c_uint32), ("pad_", C.c_uint32),
                ("seed", C.c_uint64)]


class vafr_dims(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_cols", C.c_int32), ("max_rows", C.c_int32), ("width", C.c_int32),
                ("height", C.c_int32), ("n_texels", C.c_int64)]


class vafr_view(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad_", C.c_int32), ("scene", C.c_void_p), ("layout", C.c_void_p),
                ("display", vafr_display), ("camera", vafr_camera), ("gaze", vafr_gaze), ("shading", vafr_shading),
                ("lp_rgba_dev", C.c_void_p), ("hit_id_dev", C.c_void_p), ("img_rgba_dev", C.c_void_p)]


class vafr_batch_config(C.Structure):
    _fields_ = [("trace_block", C.c_int32), ("recon_rows", C.c_int32), ("use_graph", C.c_int32)]


class vafr_server_config(C.Structure):
    _fields_ = [("max_views_per_launch", C.c_int32), ("max_inflight", C.c_int32), ("n_streams", C.c_int32),
                ("max_queue", C.c_int32), ("hbm_budget_bytes", C.c_int64), ("batch", vafr_batch_config),
                ("simulate", C.c_int32), ("pad_", C.c_int32), ("sim_ms_per_launch", C.c_double),
                ("sim_ms_per_mray", C.c_double), ("sim_ms_per_mpix", C.c_double), ("frame_budget_ms", C.c_double),
                ("latest_only", C.c_int32), ("pad2_", C.c_int32), ("watchdog_ms", C.c_double)]


class vafr_headset(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("layout", C.c_void_p), ("camera", vafr_camera * 2), ("shading", vafr_shading)]


class vafr_request(C.Structure):
    _fields_ = [("headset", C.c_int32), ("frame", C.c_uint32), ("gaze", vafr_gaze), ("deadline_ms", C.c_double),
                ("user_tag", C.c_uint64)]


class vafr_result(C.Structure):
    _fields_ = [("user_tag", C.c_uint64), ("headset", C.c_int32), ("frame", C.c_uint32), ("status", C.c_int32),
                ("slot", C.c_int32), ("submit_ms", C.c_double), ("launch_ms", C.c_double), ("done_ms", C.c_double),
                ("img_rgba_dev", C.c_void_p * 2), ("lp_rgba_dev", C.c_void_p * 2)]


class vafr_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("refused", C.c_int64), ("deferred", C.c_int64),
                ("dropped", C.c_int64), ("launches", C.c_int64), ("views_launched", C.c_int64),
                ("bytes_in_use", C.c_int64), ("waiting", C.c_int32), ("inflight", C.c_int32), ("late", C.c_int64),
                ("superseded", C.c_int64), ("stalled", C.c_int64)]


class vafr_scene_info(C.Structure):
    _fields_ = [("n_tris", C.c_int64), ("n_nodes", C.c_int64), ("n_leaves", C.c_int64), ("max_depth", C.c_int32),
                ("on_device", C.c_int32), ("device_bytes", C.c_int64), ("build_ms", C.c_double),
                ("stack_entries", C.c_int32), ("max_stack", C.c_int32)]


_lib = None
_P = C.c_void_p


def load():
    """Load libvafr.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2503_23410_amd.build`")
    L = C.CDLL(LIB_PATH)
    sig = {
        "vafr_last_error": (C.c_char_p, []),
        "vafr_abi_version": (C.c_int, []),
        "vafr_lp_layout": (C.c_int, [C.POINTER(vafr_display), C.POINTER(vafr_acuity), C.POINTER(_P)]),
        "vafr_fxaa_lp": (C.c_int, [_P, _P, _P, _P]),
        "vafr_rep_workspace_bytes": (C.c_int, [_P, C.POINTER(C.c_int64)]),
        "vafr_shade_lp_rep": (C.c_int, [_P, C.POINTER(vafr_camera), C.POINTER(vafr_camera), vafr_gaze,
                                        C.POINTER(vafr_shading), _P, _P, _P, _P, _P, _P, C.c_int64, _P, _P]),
        "vafr_shade_lp_rep_noalloc": (C.c_int, [_P, C.POINTER(vafr_camera), C.POINTER(vafr_camera), vafr_gaze,
                                                C.POINTER(vafr_shading), _P, _P, _P, _P, _P, _P]),
        "vafr_acuity_capped": (C.c_int, [C.POINTER(vafr_acuity), C.c_double, C.POINTER(C.c_double),
                                         C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32)]),
        "lmfr_lp_layout": (C.c_int, [C.POINTER(vafr_display), C.c_double, C.c_double, C.POINTER(_P)]),
        "lafr_lp_layout": (C.c_int, [C.POINTER(vafr_display), C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.POINTER(_P)]),
        "vafr_layout_dims": (C.c_int, [_P, C.POINTER(vafr_dims)]),
        "vafr_layout_tables": (C.c_int, [_P, C.POINTER(C.POINTER(C.c_int32)), C.POINTER(C.POINTER(C.c_int64)),
                                         C.POINTER(C.POINTER(C.c_float))]),
        "vafr_layout_destroy": (None, [_P]),
        "vafr_scene_create": (C.c_int, [_P, C.c_int64, _P, C.c_int64, C.POINTER(_P)]),
        "vafr_scene_get_info": (C.c_int, [_P, C.POINTER(vafr_scene_info)]),
        "vafr_scene_export": (C.c_int, [_P, _P, _P]),
        "vafr_scene_destroy": (None, [_P]),
        "vafr_shade_lp": (C.c_int, [_P, C.POINTER(vafr_camera), vafr_gaze, C.POINTER(vafr_shading), _P, _P, _P,
                                    _P]),
        "lmfr_shade_lp": (C.c_int, [_P, C.POINTER(vafr_camera), vafr_gaze, C.POINTER(vafr_shading), _P, _P, _P,
                                    _P]),
        "lafr_shade_lp": (C.c_int, [_P, C.POINTER(vafr_camera), vafr_gaze, C.POINTER(vafr_shading), _P, _P, _P,
                                    _P]),
        "vafr_reconstruct": (C.c_int, [_P, vafr_gaze, _P, _P, _P]),
        "lmfr_reconstruct": (C.c_int, [_P, vafr_gaze, _P, _P, _P]),
        "lafr_reconstruct": (C.c_int, [_P, vafr_gaze, _P, _P, _P]),
        "full_shade": (C.c_int, [_P, C.POINTER(vafr_camera), C.POINTER(vafr_display), C.POINTER(vafr_shading), _P,
                                 _P, _P]),
        "vafr_count_work": (C.c_int, [_P, C.POINTER(vafr_camera), vafr_gaze, C.POINTER(vafr_shading), _P, _P, _P]),
        "vafr_batch_create": (C.c_int, [C.c_int32, C.POINTER(vafr_batch_config), C.POINTER(_P)]),
        "vafr_batch_run": (C.c_int, [_P, C.POINTER(vafr_view), C.c_int32, _P]),
        "vafr_batch_autotune": (C.c_int, [_P, C.POINTER(vafr_view), C.c_int32, C.c_int32, _P,
                                          C.POINTER(vafr_batch_config)]),
        "vafr_batch_get_config": (C.c_int, [_P, C.POINTER(vafr_batch_config)]),
        "vafr_batch_set_config": (C.c_int, [_P, C.POINTER(vafr_batch_config)]),
        "vafr_batch_destroy": (None, [_P]),
        "vafr_batch_set_profiling": (C.c_int, [_P, C.c_int32]),
        "vafr_batch_stage_ms": (C.c_int, [_P, C.POINTER(C.c_float), C.POINTER(C.c_int64)]),
        "vafr_server_create": (C.c_int, [C.POINTER(vafr_server_config), C.POINTER(_P)]),
        "vafr_server_add_headset": (C.c_int, [_P, C.POINTER(vafr_headset), C.POINTER(C.c_int32)]),
        "vafr_server_submit": (C.c_int, [_P, C.POINTER(vafr_request)]),
        "vafr_server_poll": (C.c_int, [_P, C.POINTER(vafr_result), C.c_int32, C.POINTER(C.c_int32)]),
        "vafr_server_release": (C.c_int, [_P, C.c_int32]),
        "vafr_server_wait_idle": (C.c_int, [_P, C.c_int32]),
        "vafr_server_get_stats": (C.c_int, [_P, C.POINTER(vafr_server_stats)]),
        "vafr_server_destroy": (None, [_P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    if L.vafr_abi_version() != ABI_VERSION:
        raise ImportError(f"{LIB_PATH} has ABI {L.vafr_abi_version()}, the binding expects {ABI_VERSION}: rebuild it")
    _lib = L
    return L


def last_error() -> str:
    return load().vafr_last_error().decode()


def _check(rc):
    if rc != VAFR_OK:
        raise VafrError(rc, last_error())


# ------------------------------------------------------------------ helpers

def display(width, height, fov=(100.0, 100.0)):
    return vafr_display(int(width), int(height), float(fov[0]), float(fov[1]))


def camera(cam12):
    """cam12 = eye, right, up, forward (12 floats)."""
    c = np.asarray(cam12, np.float32).reshape(4, 3)
    out = vafr_camera()
    for f, row in zip(("eye", "right", "up", "forward"), c):
        getattr(out, f)[:] = [float(x) for x in row]
    return out


def gaze(x, y):
    return vafr_gaze(float(x), float(y))


def shading(light_dir=(0.3, 1.0, -0.5), light_rgb=(1.0, 1.0, 1.0), ambient=(0.1, 0.1, 0.1),
            background=(0.05, 0.05, 0.08), shadow=True, mode=VAFR_SHADE_LAMBERT, bounces=0, frame=0, view=0,
            seed=0):
    """light_dir: toward the light, any non-zero vector (the library
    normalises it)."""
    s = vafr_shading()
    s.light_dir[:] = [float(x) for x in np.float32(light_dir)]
    s.light_rgb[:] = [float(x) for x in np.float32(light_rgb)]
    s.ambient[:] = [float(x) for x in np.float32(ambient)]
    s.background[:] = [float(x) for x in np.float32(background)]
    s.shadow_rays = 1 if shadow else 0
    s.mode = int(mode)
    s.bounces = int(bounces)
    s.frame = int(frame)
    s.view = int(view)
    s.seed = int(seed)
    return s


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ handles

class Layout:
    """Owns a vafr_layout handle (VaFR, LMFR or LaFR)."""

    def __init__(self, handle):
        self._h = handle
        d = vafr_dims()
        _check(load().vafr_layout_dims(self._h, C.byref(d)))
        self.kind = d.kind
        self.n_cols = d.n_cols
        self.max_rows = d.max_rows
        self.width = d.width
        self.height = d.height
        self.n_texels = d.n_texels

    @classmethod
    def vafr(cls, disp: vafr_display, ecc=None, cpd=None, e_max=60.0, aniso=None):
        """ecc/cpd: acuity pivots (None: the paper's); aniso: optional
        (ecc, delta) table of the tangential-to-radial rate Delta(e)."""
        h = C.c_void_p()
        if ecc is None and aniso is None:
            _check(load().vafr_lp_layout(C.byref(disp), None, C.byref(h)))
        else:
            if ecc is None:
                ecc, cpd = (0.0, 10.0, 20.0, 30.0, 60.0), (40.0, 10.0, 6.0, 5.0, 4.0)
            e = np.ascontiguousarray(ecc, np.float64)
            f = np.ascontiguousarray(cpd, np.float64)
            dp = C.POINTER(C.c_double)
            a = vafr_acuity(len(e), e.ctypes.data_as(dp), f.ctypes.data_as(dp), float(e_max), 0, None, None)
            if aniso is not None:
                ae = np.ascontiguousarray(aniso[0], np.float64)
                ad = np.ascontiguousarray(aniso[1], np.float64)
                a.n_aniso, a.aniso_ecc_deg, a.aniso_delta = len(ae), ae.ctypes.data_as(dp), ad.ctypes.data_as(dp)
            _check(load().vafr_lp_layout(C.byref(disp), C.byref(a), C.byref(h)))
        return cls(h)

    @classmethod
    def lmfr(cls, disp: vafr_display, delta=1.8, alpha=4.0):
        h = C.c_void_p()
        _check(load().lmfr_lp_layout(C.byref(disp), float(delta), float(alpha), C.byref(h)))
        return cls(h)

    @classmethod
    def lafr(cls, disp: vafr_display, delta=1.8, a=LAFR_A, alpha=LAFR_ALPHA, beta=LAFR_BETA):
        h = C.c_void_p()
        _check(load().lafr_lp_layout(C.byref(disp), float(delta), float(a), float(alpha), float(beta), C.byref(h)))
        return cls(h)

    @property
    def handle(self):
        return self._h

    def tables(self):
        """Copies of (n_rows, col_off, texel_dxy or None)."""
        nr = C.POINTER(C.c_int32)()
        co = C.POINTER(C.c_int64)()
        dx = C.POINTER(C.c_float)()
        _check(load().vafr_layout_tables(self._h, C.byref(nr), C.byref(co), C.byref(dx)))
        n_rows = np.ctypeslib.as_array(nr, (self.n_cols,)).copy()
        col_off = np.ctypeslib.as_array(co, (self.n_cols + 1,)).copy()
        dxy = np.ctypeslib.as_array(dx, (2 * self.n_texels,)).copy() if dx else None
        return n_rows, col_off, dxy

    def close(self):
        if self._h:
            load().vafr_layout_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Scene:
    """Owns a vafr_scene handle (host BVH + device copy when a GPU exists)."""

    def __init__(self, verts, tris):
        v = np.ascontiguousarray(verts, np.float32).reshape(-1, 3)
        t = np.ascontiguousarray(tris, np.int32).reshape(-1, 3)
        h = C.c_void_p()
        _check(load().vafr_scene_create(v.ctypes.data_as(_P), v.shape[0], t.ctypes.data_as(_P), t.shape[0],
                                        C.byref(h)))
        self._h = h
        self.n_tris = t.shape[0]

    @property
    def handle(self):
        return self._h

    def info(self):
        i = vafr_scene_info()
        _check(load().vafr_scene_get_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in vafr_scene_info._fields_}

    def export(self):
        inf = self.info()
        nodes = np.empty((inf["n_nodes"], 16), np.float32)
        order = np.empty(self.n_tris, np.int32)
        _check(load().vafr_scene_export(self._h, nodes.ctypes.data_as(_P), order.ctypes.data_as(_P)))
        return nodes, order

    def close(self):
        if self._h:
            load().vafr_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------- frame calls

def acuity_capped(cap_cpd, ecc=None, cpd=None):
    """Pivots (ecc, cpd) of the device-adapted curve min(f(e), cap_cpd)."""
    dp = C.POINTER(C.c_double)
    a = None
    if ecc is not None:
        e = np.ascontiguousarray(ecc, np.float64)
        f = np.ascontiguousarray(cpd, np.float64)
        a = vafr_acuity(len(e), e.ctypes.data_as(dp), f.ctypes.data_as(dp), 60.0, 0, None, None)
    eo = np.empty(32, np.float64)
    co = np.empty(32, np.float64)
    n = C.c_int32()
    _check(load().vafr_acuity_capped(None if a is None else C.byref(a), float(cap_cpd), eo.ctypes.data_as(dp),
                                     co.ctypes.data_as(dp), 32, C.byref(n)))
    return eo[:n.value].copy(), co[:n.value].copy()


def vafr_shade_lp(scene, cam, gz, sh, layout, lp_rgba, hit_id=None, stream=None):
    _check(load().vafr_shade_lp(scene.handle, C.byref(cam), gz, C.byref(sh), layout.handle, _dptr(lp_rgba),
                                _dptr(hit_id), _stream(stream)))


def lmfr_shade_lp(scene, cam, gz, sh, layout, lp_rgba, hit_id=None, stream=None):
    _check(load().lmfr_shade_lp(scene.handle, C.byref(cam), gz, C.byref(sh), layout.handle, _dptr(lp_rgba),
                                _dptr(hit_id), _stream(stream)))


def lafr_shade_lp(scene, cam, gz, sh, layout, lp_rgba, hit_id=None, stream=None):
    _check(load().lafr_shade_lp(scene.handle, C.byref(cam), gz, C.byref(sh), layout.handle, _dptr(lp_rgba),
                                _dptr(hit_id), _stream(stream)))


def rep_workspace_bytes(layout):
    n = C.c_int64()
    _check(load().vafr_rep_workspace_bytes(layout.handle, C.byref(n)))
    return n.value


def vafr_shade_lp_rep(scene, cam_left, cam_right, gz, sh, layout, lp_left, lp_right, workspace, hit_left=None,
                      hit_right=None, stream=None, right_stream=None):
    """Left LP shaded, right LP warped from it (uncovered texels ray-cast);
    workspace: a device tensor of at least rep_workspace_bytes(layout) bytes.
    right_stream: optional stream for the ray casting of the uncovered
    texels (the right buffers are then complete in its order)."""
    _check(load().vafr_shade_lp_rep(scene.handle, C.byref(cam_left), C.byref(cam_right), gz, C.byref(sh),
                                    layout.handle, _dptr(lp_left), _dptr(lp_right), _dptr(hit_left),
                                    _dptr(hit_right), _dptr(workspace),
                                    workspace.numel() * workspace.element_size(), _stream(stream),
                                    None if right_stream is None else _stream(right_stream)))


def vafr_shade_lp_rep_noalloc(scene, cam_left, cam_right, gz, sh, layout, lp_left, lp_right, hit_left=None,
                              hit_right=None, stream=None):
    """vafr_shade_lp_rep with the library's static workspace (allocates
    nothing; the layout must already be resident on the device)."""
    _check(load().vafr_shade_lp_rep_noalloc(scene.handle, C.byref(cam_left), C.byref(cam_right), gz, C.byref(sh),
                                            layout.handle, _dptr(lp_left), _dptr(lp_right), _dptr(hit_left),
                                            _dptr(hit_right), _stream(stream)))


def vafr_fxaa_lp(layout, lp_in, lp_out, stream=None):
    _check(load().vafr_fxaa_lp(layout.handle, _dptr(lp_in), _dptr(lp_out), _stream(stream)))


def vafr_reconstruct(layout, gz, lp_rgba, img_rgba, stream=None):
    _check(load().vafr_reconstruct(layout.handle, gz, _dptr(lp_rgba), _dptr(img_rgba), _stream(stream)))


def lmfr_reconstruct(layout, gz, lp_rgba, img_rgba, stream=None):
    _check(load().lmfr_reconstruct(layout.handle, gz, _dptr(lp_rgba), _dptr(img_rgba), _stream(stream)))


def lafr_reconstruct(layout, gz, lp_rgba, img_rgba, stream=None):
    _check(load().lafr_reconstruct(layout.handle, gz, _dptr(lp_rgba), _dptr(img_rgba), _stream(stream)))


def full_shade(scene, cam, disp, sh, img_rgba, hit_id=None, stream=None):
    _check(load().full_shade(scene.handle, C.byref(cam), C.byref(disp), C.byref(sh), _dptr(img_rgba),
                             _dptr(hit_id), _stream(stream)))


def vafr_count_work(scene, cam, gz, sh, layout, counters, stream=None):
    """counters: int64 device tensor of 4 (primary rays, shadow rays, node
    visits, triangle tests), accumulated."""
    _check(load().vafr_count_work(scene.handle, C.byref(cam), gz, C.byref(sh), layout.handle, _dptr(counters),
                                  _stream(stream)))



def view(kind, scene, cam, gz, sh, layout=None, disp=None, lp_rgba=None, hit_id=None, img_rgba=None):
    """A vafr_view; buffers are torch tensors (or None).  The returned
    structure keeps raw pointers: keep the tensors alive while it is used."""
    w = vafr_view()
    w.kind = int(kind)
    w.scene = scene.handle
    w.layout = layout.handle if layout is not None else None
    if disp is not None:
        w.display = disp
    w.camera = cam
    w.gaze = gz
    w.shading = sh
    w.lp_rgba_dev = None if lp_rgba is None else lp_rgba.data_ptr()
    w.hit_id_dev = None if hit_id is None else hit_id.data_ptr()
    w.img_rgba_dev = None if img_rgba is None else img_rgba.data_ptr()
    return w


class Batch:
    """Owns a vafr_batch (one traversal + one reconstruction launch per frame)."""

    def __init__(self, max_views, trace_block=128, recon_rows=4, use_graph=True):
        cfg = vafr_batch_config(int(trace_block), int(recon_rows), 1 if use_graph else 0)
        h = C.c_void_p()
        _check(load().vafr_batch_create(int(max_views), C.byref(cfg), C.byref(h)))
        self._h = h

    def run(self, views, stream=None):
        arr = (vafr_view * len(views))(*views)
        _check(load().vafr_batch_run(self._h, arr, len(views), _stream(stream)))

    def autotune(self, views, reps=3, stream=None):
        arr = (vafr_view * len(views))(*views)
        c = vafr_batch_config()
        _check(load().vafr_batch_autotune(self._h, arr, len(views), int(reps), _stream(stream), C.byref(c)))
        return {"trace_block": c.trace_block, "recon_rows": c.recon_rows, "use_graph": c.use_graph}

    def config(self):
        c = vafr_batch_config()
        _check(load().vafr_batch_get_config(self._h, C.byref(c)))
        return {"trace_block": c.trace_block, "recon_rows": c.recon_rows, "use_graph": c.use_graph}

    def set_config(self, trace_block, recon_rows, use_graph):
        c = vafr_batch_config(int(trace_block), int(recon_rows), 1 if use_graph else 0)
        _check(load().vafr_batch_set_config(self._h, C.byref(c)))

    def set_profiling(self, on=True):
        _check(load().vafr_batch_set_profiling(self._h, 1 if on else 0))

    def stage_ms(self):
        """Mean (upload, traversal, reconstruction) ms and the frame count
        since profiling was switched on."""
        a = (C.c_float * 3)()
        n = C.c_int64()
        _check(load().vafr_batch_stage_ms(self._h, a, C.byref(n)))
        return tuple(a), n.value

    def close(self):
        if self._h:
            load().vafr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Owns a vafr_server: request loop with HBM-budget admission and
    continuous batching (or its simulated executor when simulate=True).
    Launches default to plain kernel launches (use_graph=False): a served
    launch carries milliseconds of device work, so graph replay saves little,
    while every new mix of requests is a new launch shape whose graph would
    be instantiated on the dispatcher thread."""

    def __init__(self, max_views_per_launch=16, max_inflight=3, n_streams=2, max_queue=64,
                 hbm_budget_bytes=64 << 30, trace_block=128, recon_rows=4, use_graph=False, simulate=False,
                 sim_ms_per_launch=0.05, sim_ms_per_mray=0.5, sim_ms_per_mpix=0.002, frame_budget_ms=0.0,
                 latest_only=False, watchdog_ms=0.0):
        cfg = vafr_server_config()
        cfg.max_views_per_launch = int(max_views_per_launch)
        cfg.max_inflight = int(max_inflight)
        cfg.n_streams = int(n_streams)
        cfg.max_queue = int(max_queue)
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.batch = vafr_batch_config(int(trace_block), int(recon_rows), 1 if use_graph else 0)
        cfg.simulate = 1 if simulate else 0
        cfg.sim_ms_per_launch = float(sim_ms_per_launch)
        cfg.sim_ms_per_mray = float(sim_ms_per_mray)
        cfg.sim_ms_per_mpix = float(sim_ms_per_mpix)
        cfg.frame_budget_ms = float(frame_budget_ms)
        cfg.latest_only = 1 if latest_only else 0
        cfg.watchdog_ms = float(watchdog_ms)
        h = C.c_void_p()
        _check(load().vafr_server_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._keep = []

    def add_headset(self, scene, layout, cam_left, cam_right, sh):
        hs = vafr_headset()
        hs.scene = None if scene is None else scene.handle
        hs.layout = layout.handle
        hs.camera[0] = cam_left
        hs.camera[1] = cam_right
        hs.shading = sh
        i = C.c_int32()
        _check(load().vafr_server_add_headset(self._h, C.byref(hs), C.byref(i)))
        self._keep += [scene, layout]
        return i.value

    def submit(self, headset, frame, gz, deadline_ms=0.0, tag=0):
        """True if queued, False if refused (queue full)."""
        r = vafr_request(int(headset), int(frame), gz, float(deadline_ms), int(tag))
        rc = load().vafr_server_submit(self._h, C.byref(r))
        if rc == VAFR_E_BUDGET:
            return False
        _check(rc)
        return True

    def poll(self, max_results=256):
        arr = (vafr_result * max_results)()
        n = C.c_int32()
        _check(load().vafr_server_poll(self._h, arr, max_results, C.byref(n)))
        out = []
        for r in arr[:n.value]:
            out.append({"tag": r.user_tag, "headset": r.headset, "frame": r.frame, "status": r.status,
                        "slot": r.slot, "submit_ms": r.submit_ms, "launch_ms": r.launch_ms, "done_ms": r.done_ms,
                        "img": (r.img_rgba_dev[0], r.img_rgba_dev[1]), "lp": (r.lp_rgba_dev[0], r.lp_rgba_dev[1])})
        return out

    def release(self, slot):
        _check(load().vafr_server_release(self._h, int(slot)))

    def wait_idle(self, timeout_ms=10000):
        _check(load().vafr_server_wait_idle(self._h, int(timeout_ms)))

    def stats(self):
        st = vafr_server_stats()
        _check(load().vafr_server_get_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in vafr_server_stats._fields_}

    def close(self):
        if self._h:
            load().vafr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip = None


def copy_from_device(dst, src_ptr, nbytes=None):
    """Copy nbytes from a raw device pointer (e.g. a served result) into the
    torch tensor dst (device-to-device hipMemcpy)."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    n = dst.numel() * dst.element_size() if nbytes is None else int(nbytes)
    rc = _hip.hipMemcpy(C.c_void_p(dst.data_ptr()), C.c_void_p(src_ptr), n, 3)
    if rc != 0:
        raise VafrError(VAFR_E_HIP, f"hipMemcpy failed ({rc})")
