"""CPU oracle for the VaFR hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow reference written from the paper ("Visual Acuity Consistent
Foveated Rendering towards Retinal Resolution", Zhang, Gai, Li, arXiv
2503.23410).  The arithmetic lives in ``vafr_oracle.c`` (plain C, FP64
mapping, FP32 watertight ray/triangle test, its own BVH); this module only
builds it with gcc and marshals numpy arrays through ctypes.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
the two share no code.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vafr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a separately built copy (e.g. a sanitizer build) may be named instead
_LIB_OVERRIDE = os.environ.get("VAFR_ORACLE_LIB")

DEFAULT_ECC = (0.0, 10.0, 20.0, 30.0, 60.0)   # Sec. 3.3 pivots (degrees)
DEFAULT_CPD = (40.0, 10.0, 6.0, 5.0, 4.0)     # Sec. 3.3 acuity at the pivots
DEFAULT_EMAX = 60.0                           # Sec. 3.2.2 maximum eccentricity

_lib = None


def build() -> str:
    """Compile the oracle with gcc (no fused multiply-add unless written)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=c11",
           "-D_DEFAULT_SOURCE", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            _lib = C.CDLL(_LIB_OVERRIDE)
            _declare(_lib)
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_P = C.c_void_p
_I32 = C.c_int32
_I64 = C.c_int64
_D = C.c_double


def _declare(L):
    sig = {
        "or_set_threads": (None, [C.c_int]),
        "or_get_threads": (C.c_int, []),
        "or_acuity_size": (C.c_int, []),
        "or_acuity_init": (C.c_int, [_P, C.c_int, _P, _P]),
        "or_acuity_set_aniso": (C.c_int, [_P, C.c_int, _P, _P]),
        "or_fxaa_lp": (None, [C.c_int32, _P, _P, _P, _P, C.c_int64, _P]),
        "or_warp_triangles": (C.c_int64, [C.c_int32, _P, _P, _P, _P]),
        "or_rep_warp": (None, [C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
        "or_delta": (_D, [_P, _D]),
        "or_acuity_capped": (C.c_int, [C.c_int, _P, _P, _D, _P, _P, C.c_int]),
        "or_omega": (_D, [_P, _D]),
        "or_u": (_D, [_P, _D]),
        "or_e_of_u": (_D, [_P, _D]),
        "or_l": (_D, [_P, _D]),
        "or_v": (_D, [_P, _D, _D]),
        "or_u_many": (None, [_P, _P, _I64, _P]),
        "or_e_many": (None, [_P, _P, _I64, _P]),
        "or_l_many": (None, [_P, _P, _I64, _P]),
        "or_omega_many": (None, [_P, _P, _I64, _P]),
        "or_vafr_layout_dims": (C.c_int, [_P, _D, _P, _P]),
        "or_vafr_layout_fill": (C.c_int, [_P, _D, _I32, _P, _P, _P, _P]),
        "or_film_pitch": (None, [_I32, _I32, _D, _D, _P]),
        "or_gaze_film": (None, [_I32, _I32, _P, _D, _D, _P]),
        "or_vafr_forward": (None, [_P, _I32, _I32, _P, _P, _I64, _P, _P, _P, _P, _P]),
        "or_vafr_inverse": (None, [_P, _I32, _I32, _P, _P, _I64, _P, _P, _P]),
        "or_vafr_rays": (None, [_P, _P, _I64, _P, _P, _P, _P]),
        "or_full_rays": (None, [_I32, _I32, _P, _P, _I64, _P, _P, _P]),
        "or_lmfr_dims": (None, [_I32, _I32, _D, _P, _P]),
        "or_lmfr_L": (_D, [_I32, _I32, _D, _D]),
        "or_lmfr_rays": (None, [_I32, _I32, _P, _D, _D, _I32, _I32, _D, _P, _I64, _P, _P, _P]),
        "or_lmfr_forward": (None, [_I32, _I32, _D, _D, _I32, _I32, _D, _I64, _P, _P, _P]),
        "or_watertight_many": (None, [_I64, _P, _P, _P, _P, _P, _P]),
        "or_scene_create": (_P, [_P, _I64, _P, _I64, C.c_int]),
        "or_scene_destroy": (None, [_P]),
        "or_scene_nodes": (_I64, [_P]),
        "or_scene_depth": (C.c_int, [_P]),
        "or_trace_closest": (None, [_P, _I64, _P, _P, _P, _P, _P]),
        "or_trace_any": (None, [_P, _I64, _P, _P, _P, _P]),
        "or_albedo_many": (None, [_I64, _P, _P]),
        "or_shade_rays": (None, [_P, _I64, _P, _P, _P, _P, _P, _P]),
        "or_rng01": (C.c_float, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]),
        "or_shade_path_rays": (None, [_P, _I64, _P, _P, _P, _P, C.c_uint64, C.c_uint32, C.c_uint32,
                                      _I32, _P, _P, _P]),
        "or_vafr_reconstruct": (None, [_P, _I32, _P, _P, _P, _I32, _I32, _P, _P, _P, _I64, _P, _P, _P]),
        "or_vafr_taps": (None, [_P, _I32, _P, _P, _I32, _I32, _P, _P, _P, _I64, _P]),
        "or_lmfr_reconstruct": (None, [_I32, _I32, _D, _D, _I32, _I32, _D, _P, _P, _I64, _P, _P, _P]),
        "or_lafr_consts": (C.c_int, [_I32, _I32, _P, _D, _D, _D, _D, _P]),
        "or_lafr_u": (None, [_P, _D, _I64, _P, _P]),
        "or_lafr_z": (None, [_P, _D, _I64, _P, _P]),
        "or_lafr_rays": (C.c_int, [_I32, _I32, _P, _D, _D, _I32, _I32, _D, _D, _D, _P, _I64, _P, _P, _P]),
        "or_lafr_forward": (C.c_int, [_I32, _I32, _P, _D, _D, _I32, _I32, _D, _D, _D, _I64, _P, _P, _P]),
        "or_lafr_reconstruct": (C.c_int, [_I32, _I32, _P, _D, _D, _I32, _I32, _D, _D, _D, _P, _P, _I64, _P, _P,
                                          _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


# --------------------------------------------------------------------------
# Acuity model and layout
# --------------------------------------------------------------------------

class Acuity:
    """Piecewise-linear MAR through acuity pivots (Sec. 3.3, Eq. (12))."""

    def __init__(self, ecc=DEFAULT_ECC, cpd=DEFAULT_CPD, aniso=None):
        """aniso: optional (ecc, delta) table of the tangential-to-radial
        shading-rate ratio Delta(e) of Eq. (19)."""
        L = lib()
        self._buf = C.create_string_buffer(L.or_acuity_size())
        self.ecc = _arr(ecc, np.float64)
        self.cpd = _arr(cpd, np.float64)
        rc = L.or_acuity_init(self._buf, len(self.ecc), _ptr(self.ecc), _ptr(self.cpd))
        if rc != 0:
            raise ValueError("invalid acuity pivots")
        if aniso is not None:
            self.aniso_e = _arr(aniso[0], np.float64)
            self.aniso_d = _arr(aniso[1], np.float64)
            if L.or_acuity_set_aniso(self._buf, len(self.aniso_e), _ptr(self.aniso_e), _ptr(self.aniso_d)) != 0:
                raise ValueError("invalid anisotropy table")

    @property
    def ptr(self):
        return C.cast(self._buf, C.c_void_p)

    def _many(self, fn, x):
        x = _arr(np.atleast_1d(x), np.float64)
        out = np.empty_like(x)
        fn(self.ptr, _ptr(x), x.size, _ptr(out))
        return out

    def u(self, e):
        return self._many(lib().or_u_many, e)

    def e_of_u(self, u):
        return self._many(lib().or_e_many, u)

    def l(self, e):  # noqa: E743 - the paper's symbol
        return self._many(lib().or_l_many, e)

    def omega(self, e):
        return self._many(lib().or_omega_many, e)

    def v(self, e, theta):
        return float(lib().or_v(self.ptr, float(e), float(theta)))

    def delta(self, e):
        return np.array([lib().or_delta(self.ptr, float(x)) for x in np.atleast_1d(e)])


def acuity_capped(cap, ecc=DEFAULT_ECC, cpd=DEFAULT_CPD):
    """Pivots of the device-adapted curve f_cap(e) = min(f(e), cap) (Sec. 3.3)."""
    ecc = _arr(ecc, np.float64)
    cpd = _arr(cpd, np.float64)
    eo = np.empty(2 * len(ecc), np.float64)
    co = np.empty(2 * len(ecc), np.float64)
    n = lib().or_acuity_capped(len(ecc), _ptr(ecc), _ptr(cpd), float(cap), _ptr(eo), _ptr(co), len(eo))
    if n < 0:
        raise ValueError("invalid curve or cap")
    return eo[:n].copy(), co[:n].copy()


class Layout:
    """The constant-size VaFR LP layout (Sec. 3.2.2) and its FP32 tables."""

    def __init__(self, acuity: Acuity | None = None, e_max: float = DEFAULT_EMAX):
        L = lib()
        self.acuity = acuity or Acuity()
        self.e_max = float(e_max)
        nc = C.c_int32()
        nt = C.c_int64()
        L.or_vafr_layout_dims(self.acuity.ptr, self.e_max, C.byref(nc), C.byref(nt))
        self.n_cols = nc.value
        self.n_texels = nt.value
        self.n_rows = np.empty(self.n_cols, np.int32)
        self.col_off = np.empty(self.n_cols + 1, np.int64)
        self.dxy = np.empty(2 * self.n_texels, np.float32)
        self.col_e = np.empty(self.n_cols, np.float64)
        L.or_vafr_layout_fill(self.acuity.ptr, self.e_max, self.n_cols, _ptr(self.n_rows), _ptr(self.col_off),
                              _ptr(self.dxy), _ptr(self.col_e))


def film_pitch(W, H, fov_x=100.0, fov_y=100.0):
    p = np.empty(2, np.float64)
    lib().or_film_pitch(int(W), int(H), float(fov_x), float(fov_y), _ptr(p))
    return p


def gaze_film(W, H, p, gx, gy):
    G = np.empty(2, np.float64)
    p = _arr(p, np.float64)
    lib().or_gaze_film(int(W), int(H), _ptr(p), float(gx), float(gy), _ptr(G))
    return G


def vafr_forward(acuity, W, H, p, G, xy):
    xy = _arr(xy, np.float64).reshape(-1, 2)
    n = xy.shape[0]
    u, v, e, th = (np.empty(n) for _ in range(4))
    p = _arr(p, np.float64)
    G = _arr(G, np.float64)
    lib().or_vafr_forward(acuity.ptr, int(W), int(H), _ptr(p), _ptr(G), n, _ptr(xy), _ptr(u), _ptr(v),
                          _ptr(e), _ptr(th))
    return u, v, e, th


def vafr_inverse(acuity, W, H, p, G, u, v):
    u = _arr(u, np.float64)
    v = _arr(v, np.float64)
    xy = np.empty((u.size, 2))
    p = _arr(p, np.float64)
    G = _arr(G, np.float64)
    lib().or_vafr_inverse(acuity.ptr, int(W), int(H), _ptr(p), _ptr(G), u.size, _ptr(u), _ptr(v), _ptr(xy))
    return xy


# --------------------------------------------------------------------------
# Rays
# --------------------------------------------------------------------------

def _cam(cam):
    c = _arr(cam, np.float32).reshape(-1)
    assert c.size == 12, "camera = eye, right, up, forward (12 floats)"
    return c


def vafr_rays(layout: Layout, idx, G, cam):
    idx = _arr(idx, np.int64)
    org = np.empty((idx.size, 3), np.float32)
    d = np.empty((idx.size, 3), np.float32)
    G = _arr(G, np.float64)
    c = _cam(cam)
    lib().or_vafr_rays(_ptr(layout.dxy), _ptr(idx), idx.size, _ptr(G), _ptr(c), _ptr(org), _ptr(d))
    return org, d


def full_rays(W, H, p, pix, cam):
    pix = _arr(pix, np.int64)
    org = np.empty((pix.size, 3), np.float32)
    d = np.empty((pix.size, 3), np.float32)
    p = _arr(p, np.float64)
    c = _cam(cam)
    lib().or_full_rays(int(W), int(H), _ptr(p), _ptr(pix), pix.size, _ptr(c), _ptr(org), _ptr(d))
    return org, d


def lmfr_dims(W, H, delta=1.8):
    w = C.c_int32()
    h = C.c_int32()
    lib().or_lmfr_dims(int(W), int(H), float(delta), C.byref(w), C.byref(h))
    return w.value, h.value


def lmfr_L(W, H, gx, gy):
    return float(lib().or_lmfr_L(int(W), int(H), float(gx), float(gy)))


def lmfr_rays(W, H, p, gx, gy, w, h, alpha, idx, cam):
    idx = _arr(idx, np.int64)
    org = np.empty((idx.size, 3), np.float32)
    d = np.empty((idx.size, 3), np.float32)
    p = _arr(p, np.float64)
    c = _cam(cam)
    lib().or_lmfr_rays(int(W), int(H), _ptr(p), float(gx), float(gy), int(w), int(h), float(alpha), _ptr(idx),
                       idx.size, _ptr(c), _ptr(org), _ptr(d))
    return org, d


def lmfr_forward(W, H, gx, gy, w, h, alpha, xy):
    xy = _arr(xy, np.float64).reshape(-1, 2)
    u = np.empty(xy.shape[0])
    v = np.empty(xy.shape[0])
    lib().or_lmfr_forward(int(W), int(H), float(gx), float(gy), int(w), int(h), float(alpha), xy.shape[0],
                          _ptr(xy), _ptr(u), _ptr(v))
    return u, v


# LaFR (Sec. 4.1 Eq. (15)): a is LMFR's kernel exponent in the
# buffer-to-screen direction (1/4); alpha and beta as printed for LaFR.
LAFR_A = 0.25
LAFR_ALPHA = 0.85
LAFR_BETA = 0.7


def lafr_consts(W, H, p, gx, gy, a=LAFR_A, alpha=LAFR_ALPHA):
    """(ln L, Z_ef, Fa, U_ef) of Eq. (15) for one gaze; raises ValueError
    where the kernel is undefined."""
    out = np.empty(4)
    p = _arr(p, np.float64)
    rc = lib().or_lafr_consts(int(W), int(H), _ptr(p), float(gx), float(gy), float(a), float(alpha), _ptr(out))
    if rc:
        raise ValueError(f"LaFR kernel undefined: Z_ef={out[1]!r}, Fa={out[2]!r}")
    return out


def lafr_u(consts, z, beta=LAFR_BETA):
    """u / w of Eq. (15) at log ratios z."""
    c = _arr(consts, np.float64)
    z = _arr(z, np.float64)
    u = np.empty(z.size)
    lib().or_lafr_u(_ptr(c), float(beta), z.size, _ptr(z), _ptr(u))
    return u


def lafr_z(consts, t, beta=LAFR_BETA):
    """Inverse of Eq. (15): log ratio z at normalised abscissae t = u / w."""
    c = _arr(consts, np.float64)
    t = _arr(t, np.float64)
    z = np.empty(t.size)
    lib().or_lafr_z(_ptr(c), float(beta), t.size, _ptr(t), _ptr(z))
    return z


def lafr_rays(W, H, p, gx, gy, w, h, idx, cam, a=LAFR_A, alpha=LAFR_ALPHA, beta=LAFR_BETA):
    idx = _arr(idx, np.int64)
    org = np.empty((idx.size, 3), np.float32)
    d = np.empty((idx.size, 3), np.float32)
    p = _arr(p, np.float64)
    c = _cam(cam)
    rc = lib().or_lafr_rays(int(W), int(H), _ptr(p), float(gx), float(gy), int(w), int(h), float(a), float(alpha),
                            float(beta), _ptr(idx), idx.size, _ptr(c), _ptr(org), _ptr(d))
    if rc:
        raise ValueError("LaFR kernel undefined for this display and gaze")
    return org, d


def lafr_forward(W, H, p, gx, gy, w, h, xy, a=LAFR_A, alpha=LAFR_ALPHA, beta=LAFR_BETA):
    xy = _arr(xy, np.float64).reshape(-1, 2)
    u = np.empty(xy.shape[0])
    v = np.empty(xy.shape[0])
    p = _arr(p, np.float64)
    rc = lib().or_lafr_forward(int(W), int(H), _ptr(p), float(gx), float(gy), int(w), int(h), float(a),
                               float(alpha), float(beta), xy.shape[0], _ptr(xy), _ptr(u), _ptr(v))
    if rc:
        raise ValueError("LaFR kernel undefined for this display and gaze")
    return u, v


def watertight_many(org, d, tri9):
    org = _arr(org, np.float32).reshape(-1, 3)
    d = _arr(d, np.float32).reshape(-1, 3)
    tri9 = _arr(tri9, np.float32).reshape(-1, 9)
    n = org.shape[0]
    hit = np.empty(n, np.int32)
    t = np.empty(n, np.float32)
    m = np.empty(n, np.float64)
    lib().or_watertight_many(n, _ptr(org), _ptr(d), _ptr(tri9), _ptr(hit), _ptr(t), _ptr(m))
    return hit.astype(bool), t, m


def albedo(ids):
    ids = _arr(ids, np.int32)
    out = np.empty((ids.size, 3), np.float32)
    lib().or_albedo_many(ids.size, _ptr(ids), _ptr(out))
    return out


def rng01(seed, frame, view, texel, slot):
    return float(lib().or_rng01(int(seed), int(frame), int(view), int(texel), int(slot)))


# --------------------------------------------------------------------------
# Scene, tracing and shading
# --------------------------------------------------------------------------

def shading_params(light_dir=(0.3, 1.0, -0.5), light_rgb=(1.0, 1.0, 1.0), ambient=(0.1, 0.1, 0.1),
                   background=(0.05, 0.05, 0.08), shadow=True):
    """sh = {light_dir, light_rgb, ambient, background, shadow}; defaults are
    the shading reading of Sec. 6.1.  The light direction is an FP32 input
    normalised in FP64 (squares summed as (x x + y y) + z z, each component
    divided by the root) and rounded to FP32."""
    x, y, z = (float(c) for c in np.float32(light_dir))
    n = math.sqrt((x * x + y * y) + z * z)
    ld = [x / n, y / n, z / n]
    return np.concatenate([ld, light_rgb, ambient, background, [1.0 if shadow else 0.0]]).astype(np.float32)


class Scene:
    """Triangle soup plus (optionally) the oracle's own BVH."""

    def __init__(self, verts, tris, use_bvh=True):
        self.verts = _arr(verts, np.float32).reshape(-1, 3)
        self.tris = _arr(tris, np.int32).reshape(-1, 3)
        self._h = lib().or_scene_create(_ptr(self.verts), self.verts.shape[0], _ptr(self.tris),
                                        self.tris.shape[0], 1 if use_bvh else 0)
        if not self._h:
            raise ValueError("triangle index out of range")

    def close(self):
        if self._h:
            lib().or_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_nodes(self):
        return int(lib().or_scene_nodes(self._h))

    @property
    def depth(self):
        return int(lib().or_scene_depth(self._h))

    def closest(self, org, d):
        org = _arr(org, np.float32).reshape(-1, 3)
        d = _arr(d, np.float32).reshape(-1, 3)
        n = org.shape[0]
        ids = np.empty(n, np.int32)
        t = np.empty(n, np.float32)
        fl = np.empty(n, np.uint8)
        lib().or_trace_closest(self._h, n, _ptr(org), _ptr(d), _ptr(ids), _ptr(t), _ptr(fl))
        return ids, t, fl

    def any(self, org, d):
        org = _arr(org, np.float32).reshape(-1, 3)
        d = _arr(d, np.float32).reshape(-1, 3)
        n = org.shape[0]
        occ = np.empty(n, np.uint8)
        fl = np.empty(n, np.uint8)
        lib().or_trace_any(self._h, n, _ptr(org), _ptr(d), _ptr(occ), _ptr(fl))
        return occ.astype(bool), fl

    def shade(self, org, d, sh):
        org = _arr(org, np.float32).reshape(-1, 3)
        d = _arr(d, np.float32).reshape(-1, 3)
        sh = _arr(sh, np.float32)
        n = org.shape[0]
        rgba = np.empty((n, 4), np.float32)
        ids = np.empty(n, np.int32)
        fl = np.empty(n, np.uint8)
        lib().or_shade_rays(self._h, n, _ptr(org), _ptr(d), _ptr(sh), _ptr(rgba), _ptr(ids), _ptr(fl))
        return rgba, ids, fl

    def shade_path(self, org, d, idx, sh, seed, frame, view, bounces):
        org = _arr(org, np.float32).reshape(-1, 3)
        d = _arr(d, np.float32).reshape(-1, 3)
        idx = _arr(idx, np.int64)
        sh = _arr(sh, np.float32)
        n = org.shape[0]
        rgba = np.empty((n, 4), np.float32)
        ids = np.empty(n, np.int32)
        fl = np.empty(n, np.uint8)
        lib().or_shade_path_rays(self._h, n, _ptr(org), _ptr(d), _ptr(idx), _ptr(sh), int(seed), int(frame),
                                 int(view), int(bounces), _ptr(rgba), _ptr(ids), _ptr(fl))
        return rgba, ids, fl


# --------------------------------------------------------------------------
# Reconstruction
# --------------------------------------------------------------------------

def vafr_reconstruct(layout: Layout, lp, W, H, p, G, pix, tflag=None):
    lp = _arr(lp, np.float32).reshape(-1, 4)
    assert lp.shape[0] == layout.n_texels
    pix = _arr(pix, np.int64)
    out = np.empty((pix.size, 4), np.float32)
    pf = np.empty(pix.size, np.uint8)
    p = _arr(p, np.float64)
    G = _arr(G, np.float64)
    tf = None if tflag is None else _arr(tflag, np.uint8)
    lib().or_vafr_reconstruct(layout.acuity.ptr, layout.n_cols, _ptr(layout.n_rows), _ptr(layout.col_off),
                              _ptr(lp), int(W), int(H), _ptr(p), _ptr(G), _ptr(pix), pix.size, _ptr(out),
                              _ptr(tf), _ptr(pf))
    return out, pf.astype(bool)


def vafr_taps(layout: Layout, W, H, p, G, pix):
    """(n, 4) texel indices each display pixel reads: column i0's two rows,
    then column i1's (the reconstruction's footprint)."""
    pix = _arr(pix, np.int64)
    taps = np.empty((pix.size, 4), np.int64)
    p = _arr(p, np.float64)
    G = _arr(G, np.float64)
    lib().or_vafr_taps(layout.acuity.ptr, layout.n_cols, _ptr(layout.n_rows), _ptr(layout.col_off), int(W), int(H),
                       _ptr(p), _ptr(G), _ptr(pix), pix.size, _ptr(taps))
    return taps


def lmfr_reconstruct(W, H, gx, gy, w, h, alpha, lp, pix, tflag=None):
    lp = _arr(lp, np.float32).reshape(-1, 4)
    assert lp.shape[0] == w * h
    pix = _arr(pix, np.int64)
    out = np.empty((pix.size, 4), np.float32)
    pf = np.empty(pix.size, np.uint8)
    tf = None if tflag is None else _arr(tflag, np.uint8)
    lib().or_lmfr_reconstruct(int(W), int(H), float(gx), float(gy), int(w), int(h), float(alpha), _ptr(lp),
                              _ptr(pix), pix.size, _ptr(out), _ptr(tf), _ptr(pf))
    return out, pf.astype(bool)


def lafr_reconstruct(W, H, p, gx, gy, w, h, lp, pix, tflag=None, a=LAFR_A, alpha=LAFR_ALPHA, beta=LAFR_BETA):
    lp = _arr(lp, np.float32).reshape(-1, 4)
    assert lp.shape[0] == w * h
    pix = _arr(pix, np.int64)
    out = np.empty((pix.size, 4), np.float32)
    pf = np.empty(pix.size, np.uint8)
    tf = None if tflag is None else _arr(tflag, np.uint8)
    p = _arr(p, np.float64)
    rc = lib().or_lafr_reconstruct(int(W), int(H), _ptr(p), float(gx), float(gy), int(w), int(h), float(a),
                                   float(alpha), float(beta), _ptr(lp), _ptr(pix), pix.size, _ptr(out), _ptr(tf),
                                   _ptr(pf))
    if rc:
        raise ValueError("LaFR kernel undefined for this display and gaze")
    return out, pf.astype(bool)


# --------------------------------------------------------------------------
# Whole-step helpers (shade an LP buffer / a display) used by tests & bench
# --------------------------------------------------------------------------

def shade_vafr_texels(scene: Scene, layout: Layout, idx, W, H, fov, gaze, cam, sh):
    p = film_pitch(W, H, *fov)
    G = gaze_film(W, H, p, *gaze)
    org, d = vafr_rays(layout, idx, G, cam)
    return scene.shade(org, d, sh)


def shade_full_pixels(scene: Scene, pix, W, H, fov, cam, sh):
    p = film_pitch(W, H, *fov)
    org, d = full_rays(W, H, p, pix, cam)
    return scene.shade(org, d, sh)


def shade_lmfr_texels(scene: Scene, idx, W, H, fov, gaze, w, h, alpha, cam, sh):
    p = film_pitch(W, H, *fov)
    org, d = lmfr_rays(W, H, p, gaze[0], gaze[1], w, h, alpha, idx, cam)
    return scene.shade(org, d, sh)


def shade_lafr_texels(scene: Scene, idx, W, H, fov, gaze, w, h, cam, sh, a=LAFR_A, alpha=LAFR_ALPHA,
                      beta=LAFR_BETA):
    p = film_pitch(W, H, *fov)
    org, d = lafr_rays(W, H, p, gaze[0], gaze[1], w, h, idx, cam, a, alpha, beta)
    return scene.shade(org, d, sh)


def fxaa_lp(layout: Layout, lp, idx=None):
    """FXAA-style anti-aliasing inside the LP buffer (Sec. 3.4) for texels
    idx (all by default): RGBA per listed texel."""
    lp = _arr(lp, np.float32).reshape(-1, 4)
    idx = np.arange(layout.n_texels, dtype=np.int64) if idx is None else _arr(idx, np.int64)
    out = np.empty((idx.size, 4), np.float32)
    lib().or_fxaa_lp(layout.n_cols, _ptr(layout.n_rows), _ptr(layout.col_off), _ptr(lp), _ptr(idx), idx.size,
                     _ptr(out))
    return out


def warp_triangles(layout: Layout):
    """The grid triangles of forward grid warping (Sec. 5.1): (vertices
    (m, 3) texel indices: previous, x, other; ids (m,))."""
    m = int(lib().or_warp_triangles(layout.n_cols, _ptr(layout.n_rows), _ptr(layout.col_off), None, None))
    v = np.empty((m, 3), np.int64)
    ids = np.empty(m, np.int64)
    lib().or_warp_triangles(layout.n_cols, _ptr(layout.n_rows), _ptr(layout.col_off), _ptr(v), _ptr(ids))
    return v, ids


def rep_lp(scene: Scene, layout: Layout, W, H, fov, gaze, cam_left, cam_right, sh, depth=None, parts=False):
    """Binocular reprojection (Sec. 5.1, VaFR_Rep) by forward grid warping:
    the left LP buffer is shaded; its texels' hit points, as a grid of
    triangles, are warped into the right eye's LP grid (nearest surface
    wins, colours interpolated); right texels no triangle covers are ray
    cast.  Returns (left rgba, right rgba, tri, flags, right ids):
    tri[r] = winning grid triangle of right texel r, or -1 where it was ray
    cast; flags mark texels that may legitimately differ.  depth: optional
    float32 array that receives each warped texel's interpolated depth.
    parts=True appends a dict of the flags' sources: "left" (near-tie left
    rays, per left texel), "warp" (right texels inside the widened box of a
    warp triangle that uses a flagged left texel) and "holes" (near-tie rays
    among the ray-cast right texels, per right texel)."""
    idx = np.arange(layout.n_texels, dtype=np.int64)
    p = film_pitch(W, H, *fov)
    G = gaze_film(W, H, p, *gaze)
    org, d = vafr_rays(layout, idx, G, cam_left)
    left, lid, lfl = scene.shade(org, d, sh)
    ids, t, _ = scene.closest(org, d)
    n = layout.n_texels
    right = np.zeros((n, 4), np.float32)
    rid = np.full(n, -1, np.int32)
    tri = np.empty(n, np.int64)
    flag = np.empty(n, np.uint8)
    lfl8 = np.ascontiguousarray(lfl, np.uint8)
    lib().or_rep_warp(layout.n_cols, _ptr(layout.n_rows), _ptr(layout.col_off), _ptr(layout.dxy), _ptr(G),
                      _ptr(org), _ptr(d), _ptr(t), _ptr(_arr(ids, np.int32)), _ptr(lfl8), _ptr(_arr(left, np.float32)),
                      _ptr(_cam(cam_right)), _ptr(right), _ptr(rid), _ptr(tri), _ptr(depth), _ptr(flag))
    rfl = flag.astype(bool)
    hfl = np.zeros(n, bool)
    holes = np.nonzero(tri < 0)[0]
    if holes.size:
        h_rgba, h_id, h_fl = shade_vafr_texels(scene, layout, holes, W, H, fov, gaze, cam_right, sh)
        right[holes] = h_rgba
        rid[holes] = h_id
        hfl[holes] = h_fl.astype(bool)
        rfl |= hfl
    if parts:
        return left, right, tri, rfl, rid, {"left": lfl.astype(bool), "warp": flag.astype(bool), "holes": hfl}
    return left, right, tri, rfl, rid
