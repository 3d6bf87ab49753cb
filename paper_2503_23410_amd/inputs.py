"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the rendering method: it only draws
scenes (triangle soups, a heightfield with icospheres), cameras, gaze traces,
display-size mixes and random LP buffers from fixed seeds, in numpy.  The
paper's scenes (Bistro, Sun Temple) are not available; these stand in for
them with the triangle counts and structure of the workloads below.
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

FOV = (100.0, 100.0)          # horizontal, vertical field of view in degrees
IPD = 0.064                   # metres (scene units)


def soup_scene(n_tris: int = 4096, seed: int = 0):
    """Triangle soup with vertices uniform in [-1, 1]^3 (ids in draw order)."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1.0, 1.0, (n_tris, 3, 3)).astype(np.float32)
    verts = v.reshape(-1, 3)
    tris = np.arange(3 * n_tris, dtype=np.int32).reshape(-1, 3)
    return verts, tris


def soup_camera():
    """Eye at (0, 0, -3) looking along +z, up +y, right +x."""
    return np.array([0, 0, -3, 1, 0, 0, 0, 1, 0, 0, 0, 1], np.float32)


def _gradient_noise(x, z, freq, rng):
    """One octave of 2-D lattice gradient noise on a grid of sample points."""
    gx0 = math.floor(x.min() * freq) - 1
    gz0 = math.floor(z.min() * freq) - 1
    nx = int(math.ceil(x.max() * freq)) - gx0 + 3
    nz = int(math.ceil(z.max() * freq)) - gz0 + 3
    ang = rng.uniform(0.0, 2.0 * math.pi, (nz, nx))
    gxv, gzv = np.cos(ang), np.sin(ang)
    X = x * freq - gx0
    Z = z * freq - gz0
    ix = np.floor(X).astype(np.int64)
    iz = np.floor(Z).astype(np.int64)
    fx = X - ix
    fz = Z - iz

    def fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    def dot(cx, cz):
        return gxv[iz + cz, ix + cx] * (fx - cx) + gzv[iz + cz, ix + cx] * (fz - cz)

    u, w = fade(fx), fade(fz)
    a = dot(0, 0) * (1 - u) + dot(1, 0) * u
    b = dot(0, 1) * (1 - u) + dot(1, 1) * u
    return a * (1 - w) + b * w


def heightfield(nx: int, nz: int, seed: int, octaves: int = 6, amplitude: float = 0.2,
                base_freq: float = 1.0):
    """Grid heights over x in [-2, 2], z in [-1, 1]: y = -0.6 + fBm, with
    lacunarity 2, gain 0.5 and the peak |fBm| scaled to `amplitude`."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(-2.0, 2.0, nx + 1)
    zs = np.linspace(-1.0, 1.0, nz + 1)
    X, Z = np.meshgrid(xs, zs)           # (nz+1, nx+1)
    h = np.zeros_like(X)
    amp, freq = 1.0, base_freq
    for _ in range(octaves):
        h += amp * _gradient_noise(X, Z, freq, rng)
        amp *= 0.5
        freq *= 2.0
    h *= amplitude / np.abs(h).max()
    return xs, zs, -0.6 + h


def icosphere(subdiv: int = 2):
    """Unit icosphere with outward winding: 20 * 4**subdiv triangles."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), np.array(faces, np.int64)


def terrain_scene(nx: int, nz: int, n_spheres: int, seed: int):
    """Heightfield of nx x nz cells (2 triangles per cell) plus n_spheres
    subdivision-2 icospheres (320 triangles each) with radii U[0.02, 0.1],
    centres uniform over the footprint, resting on the surface."""
    rng = np.random.default_rng(seed)
    xs, zs, H = heightfield(nx, nz, seed=int(rng.integers(1 << 31)))
    X, Z = np.meshgrid(xs, zs)
    hv = np.stack([X, H, Z], axis=-1).reshape(-1, 3)
    iz, ix = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    a = (iz * (nx + 1) + ix).reshape(-1)
    b = a + 1
    c = a + (nx + 1)
    d = c + 1
    ht = np.empty((nz * nx * 2, 3), np.int64)
    ht[0::2] = np.stack([a, c, b], 1)
    ht[1::2] = np.stack([b, c, d], 1)
    sv, sf = icosphere(2)
    r = rng.uniform(0.02, 0.1, n_spheres)
    cx = rng.uniform(-2.0, 2.0, n_spheres)
    cz = rng.uniform(-1.0, 1.0, n_spheres)
    # ground height under each centre: bilinear in the grid
    gx = (cx + 2.0) / 4.0 * nx
    gz = (cz + 1.0) / 2.0 * nz
    i0 = np.clip(np.floor(gx).astype(np.int64), 0, nx - 1)
    j0 = np.clip(np.floor(gz).astype(np.int64), 0, nz - 1)
    fx, fz = gx - i0, gz - j0
    h00, h10 = H[j0, i0], H[j0, i0 + 1]
    h01, h11 = H[j0 + 1, i0], H[j0 + 1, i0 + 1]
    gy = (h00 * (1 - fx) + h10 * fx) * (1 - fz) + (h01 * (1 - fx) + h11 * fx) * fz
    cy = gy + r
    verts = [hv]
    tris = [ht]
    base = hv.shape[0]
    for s in range(n_spheres):
        verts.append(sv * r[s] + np.array([cx[s], cy[s], cz[s]]))
        tris.append(sf + base)
        base += sv.shape[0]
    return np.concatenate(verts).astype(np.float32), np.concatenate(tris).astype(np.int32)


def terrain_camera(eye_offset: float = 0.0):
    """Camera over the terrain: eye (-1.2, 0, 0) looking along +x, pitched 60
    degrees down (about 94% of full-resolution primary rays hit the terrain
    at 100 x 100 degrees), shifted along its right axis by eye_offset."""
    pitch = math.radians(60.0)
    fwd = np.array([math.cos(pitch), -math.sin(pitch), 0.0])
    right = np.array([0.0, 0.0, -1.0])
    up = np.cross(fwd, right)
    eye = np.array([-1.2, 0.0, 0.0]) + eye_offset * right
    return np.concatenate([eye, right, up, fwd]).astype(np.float32)


def binocular_cameras(ipd: float = IPD):
    """Parallel left/right cameras at eye -/+ ipd/2 along the right axis."""
    return terrain_camera(-0.5 * ipd), terrain_camera(+0.5 * ipd)


# ---------------------------------------------------------------------------
# Gaze
# ---------------------------------------------------------------------------

def _angles_to_pixels(a_deg, b_deg, W, H, fov=FOV):
    """Film-plane angles (horizontal, vertical) of the gaze -> display pixels."""
    px = 2.0 * math.tan(math.radians(fov[0]) / 2.0) / W
    py = 2.0 * math.tan(math.radians(fov[1]) / 2.0) / H
    x = W / 2.0 + np.tan(np.radians(a_deg)) / px
    y = H / 2.0 + np.tan(np.radians(b_deg)) / py
    return x, y


def uniform_gaze(n: int, W: int, H: int, seed: int, half_range_deg: float = 30.0, fov=FOV):
    """Gaze points whose angles are uniform in the central +-30 degrees."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-half_range_deg, half_range_deg, n)
    b = rng.uniform(-half_range_deg, half_range_deg, n)
    x, y = _angles_to_pixels(a, b, W, H, fov)
    return np.stack([x, y], 1)


def gaze_trace(n_frames: int, W: int, H: int, seed: int, rate_hz: float = 90.0,
               half_range_deg: float = 30.0, fov=FOV):
    """Fixation/saccade gaze trace sampled at rate_hz.

    Fixations last U[200, 400] ms; saccades have amplitude U[2, 20] degrees,
    direction U[0, 360) degrees and duration 2.2 ms/deg + 21 ms (main-sequence
    approximation), with linear motion; the gaze angle is reflected to stay
    within +-half_range_deg per axis.  Returns (n_frames, 2) pixel coords.
    """
    rng = np.random.default_rng(seed)
    dt = 1000.0 / rate_hz
    t_end = n_frames * dt
    events = []                     # (t0, t1, a0, b0, a1, b1)
    t, a, b = 0.0, 0.0, 0.0
    while t < t_end + 1000.0:
        fix = rng.uniform(200.0, 400.0)
        events.append((t, t + fix, a, b, a, b))
        t += fix
        amp = rng.uniform(2.0, 20.0)
        ang = math.radians(rng.uniform(0.0, 360.0))
        dur = 2.2 * amp + 21.0
        a1, b1 = a + amp * math.cos(ang), b + amp * math.sin(ang)

        def reflect(q):
            lim = half_range_deg
            while abs(q) > lim:
                q = (2 * lim - q) if q > lim else (-2 * lim - q)
            return q

        a1, b1 = reflect(a1), reflect(b1)
        events.append((t, t + dur, a, b, a1, b1))
        t += dur
        a, b = a1, b1
    out = np.empty((n_frames, 2))
    k = 0
    for f in range(n_frames):
        tf = f * dt
        while events[k][1] <= tf:
            k += 1
        t0, t1, a0, b0, a1, b1 = events[k]
        s = (tf - t0) / (t1 - t0)
        out[f] = (a0 + s * (a1 - a0), b0 + s * (b1 - b0))
    x, y = _angles_to_pixels(out[:, 0], out[:, 1], W, H, fov)
    return np.stack([x, y], 1)


# ---------------------------------------------------------------------------
# Batched views and LP test buffers
# ---------------------------------------------------------------------------

DISPLAY_SIZES = ((1280, 720), (1920, 1080), (3840, 2160), (7680, 4320))


def batch_views(n_views: int = 16, seed: int = 4):
    """Display sizes drawn from DISPLAY_SIZES and an independent gaze per
    view (uniform in the central +-30 degrees)."""
    rng = np.random.default_rng(seed)
    sizes = [DISPLAY_SIZES[int(i)] for i in rng.integers(0, len(DISPLAY_SIZES), n_views)]
    gazes = []
    for v, (W, H) in enumerate(sizes):
        gazes.append(uniform_gaze(1, W, H, seed=seed * 1000 + v)[0])
    return sizes, np.array(gazes)


def random_lp(n_texels: int, seed: int):
    """RGBA texels uniform in [0, 1) (alpha too), FP32."""
    rng = np.random.default_rng(seed)
    return rng.random((n_texels, 4), dtype=np.float32)


SCENES = {
    # name: (generator kwargs) -- triangle counts in the comments
    "soup4k": dict(kind="soup", n_tris=4096, seed=0),                      # 4,096
    "terrain1m": dict(kind="terrain", nx=1024, nz=512, n_spheres=256, seed=2),   # 1,130,496
    "terrain4m": dict(kind="terrain", nx=2048, nz=1024, n_spheres=1024, seed=3),  # 4,521,984
}


def make_scene(name: str):
    cfg = dict(SCENES[name])
    kind = cfg.pop("kind")
    if kind == "soup":
        return soup_scene(**cfg)
    return terrain_scene(**cfg)
