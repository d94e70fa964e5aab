"""Seeded synthetic scenes, cameras and target images.

This module only draws inputs. It holds none of the rasterizer's arithmetic
(no rotation-from-quaternion, no projection, no compositing), so that the
HIP path and the FP64 oracle can both be fed from it without sharing any of
the method's code.

Every array is drawn in float64 from ``numpy.random.Generator(PCG64(seed))``
and cast once to float32, the precision the library takes at its boundary.

Layouts (structure of arrays, component-major planes, float32):

* ``means``     [3, N]  world-space centres (x, y, z planes)
* ``quats``     [4, N]  rotation quaternions in (w, x, y, z) order, unit
  length in float64 before the cast (the method does not renormalise)
* ``scales``    [3, N]  linear per-axis scales s (drawn as exp of a normal)
* ``colors``    [3, N]  RGB in [0, 1]
* ``opacities`` [N]     o in (0, 1) (drawn as a logistic of a normal)

A camera is a world-to-camera rigid transform (R_cw, t_cw), pinhole
intrinsics (fx, fy, cx, cy), an image size and near/far planes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

DEFAULT_NEAR = 0.01
DEFAULT_FAR = 1.0e10


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Camera:
    R: np.ndarray            # [3, 3] float32, world -> camera rotation (row-major)
    t: np.ndarray            # [3] float32, world -> camera translation
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = DEFAULT_NEAR
    far: float = DEFAULT_FAR
    scene: int = 0           # index of the scene this camera views

    def __post_init__(self):
        self.R = np.asarray(self.R, dtype=np.float32).reshape(3, 3)
        self.t = np.asarray(self.t, dtype=np.float32).reshape(3)
        for name in ("fx", "fy", "cx", "cy", "near", "far"):
            setattr(self, name, float(np.float32(getattr(self, name))))
        self.width = int(self.width)
        self.height = int(self.height)

    @property
    def tiles_x(self) -> int:
        return (self.width + 15) // 16

    @property
    def tiles_y(self) -> int:
        return (self.height + 15) // 16

    @property
    def n_tiles(self) -> int:
        return self.tiles_x * self.tiles_y

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


@dataclass
class Workload:
    name: str
    scenes: List[dict]
    cameras: List[Camera]
    targets: List[np.ndarray] = field(default_factory=list)   # per camera [3, H, W] float32
    seed: int = 0

    @property
    def n_gaussians(self) -> int:
        return sum(s["means"].shape[1] for s in self.scenes)

    @property
    def n_projected(self) -> int:
        return sum(self.scenes[c.scene]["means"].shape[1] for c in self.cameras)

    @property
    def n_pixels(self) -> int:
        return sum(c.n_pixels for c in self.cameras)

    @property
    def n_tiles(self) -> int:
        return sum(c.n_tiles for c in self.cameras)


# --------------------------------------------------------------------------- draws

def random_unit_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Haar-random proper rotation via QR of a Gaussian matrix."""
    a = rng.standard_normal((3, 3))
    qm, r = np.linalg.qr(a)
    qm = qm * np.sign(np.diag(r))[None, :]
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


def _logistic(x: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-x))


def _finish_scene(rng, means, log_scale_mu, log_scale_sd, opac_sd) -> dict:
    n = means.shape[1]
    quats = random_unit_quats(rng, n)
    scales = np.exp(rng.normal(log_scale_mu, log_scale_sd, size=(3, n)))
    colors = rng.uniform(0.0, 1.0, size=(3, n))
    opac = _logistic(rng.normal(0.0, opac_sd, size=n))
    return {
        "means": np.ascontiguousarray(means, dtype=np.float32),
        "quats": np.ascontiguousarray(quats, dtype=np.float32),
        "scales": np.ascontiguousarray(scales, dtype=np.float32),
        "colors": np.ascontiguousarray(colors, dtype=np.float32),
        "opacities": np.ascontiguousarray(opac, dtype=np.float32),
    }


def _split_sizes(n: int, k: int) -> np.ndarray:
    sizes = np.full(k, n // k, dtype=np.int64)
    sizes[: n % k] += 1
    return sizes


def scene_uniform_slab(rng, n, xy=1.0, z=(2.0, 6.0), log_scale=(-3.0, 0.5), opac_sd=1.0) -> dict:
    means = np.stack([
        rng.uniform(-xy, xy, n),
        rng.uniform(-xy, xy, n),
        rng.uniform(z[0], z[1], n),
    ])
    return _finish_scene(rng, means, log_scale[0], log_scale[1], opac_sd)


def scene_frustum_clusters(rng, n, n_clusters=16, sigma=0.3, z=(2.0, 10.0), spread=0.4,
                           log_scale=(-4.0, 0.7), opac_sd=1.5) -> dict:
    """Isotropic clusters whose centres sit inside a pinhole frustum of half-angle atan(0.5)."""
    cz = rng.uniform(z[0], z[1], n_clusters)
    cxy = cz[None, :] * rng.uniform(-spread, spread, size=(2, n_clusters))
    centres = np.concatenate([cxy, cz[None, :]], axis=0)
    parts = []
    for k, m in enumerate(_split_sizes(n, n_clusters)):
        parts.append(centres[:, k:k + 1] + sigma * rng.standard_normal((3, m)))
    return _finish_scene(rng, np.concatenate(parts, axis=1), log_scale[0], log_scale[1], opac_sd)


def scene_box_clusters(rng, n, half=10.0, n_clusters=64, sigma_range=(0.3, 3.0),
                       log_scale=(-5.0, 1.0), opac_sd=2.0) -> dict:
    """Anisotropic clusters filling the cube [-half, half]^3; out-of-box draws are redrawn."""
    centres = rng.uniform(-half, half, size=(3, n_clusters))
    parts = []
    for k, m in enumerate(_split_sizes(n, n_clusters)):
        rot = random_rotation(rng)
        sig = np.exp(rng.uniform(np.log(sigma_range[0]), np.log(sigma_range[1]), 3))
        pts = np.empty((3, m))
        todo = np.arange(m)
        while todo.size:
            z = rng.standard_normal((3, todo.size))
            p = centres[:, k:k + 1] + rot @ (sig[:, None] * z)
            pts[:, todo] = p
            bad = np.any(np.abs(p) > half, axis=0)
            todo = todo[bad]
        parts.append(pts)
    return _finish_scene(rng, np.concatenate(parts, axis=1), log_scale[0], log_scale[1], opac_sd)


def look_at(position, target, down=(0.0, -1.0, 0.0)):
    """World->camera (R_cw, t_cw) for a camera at ``position`` whose +z axis looks at ``target``.

    Camera axes: +z forward, +y towards ``down`` (image rows grow downwards), +x = y cross z.
    """
    pos = np.asarray(position, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - pos
    fwd /= np.linalg.norm(fwd)
    x = np.cross(np.asarray(down, dtype=np.float64), fwd)
    x /= np.linalg.norm(x)
    y = np.cross(fwd, x)
    R = np.stack([x, y, fwd])            # rows are the camera axes in world coordinates
    t = -R @ pos
    return R, t


def _targets(rng, cams):
    return [rng.uniform(0.0, 1.0, size=(3, c.height, c.width)).astype(np.float32) for c in cams]


# ------------------------------------------------------------------------ configurations

CONFIG_NAMES = {
    1: "c1: 1k Gaussians, 64x64",
    2: "c2: 100k Gaussians, 512x512",
    3: "c3: 1M Gaussians, 1920x1080",
    4: "c4: 3M Gaussians, 16 orbit cameras 1280x720",
    5: "c5: 8 scenes log-U[50k,2M], 32 cameras of mixed size",
}


def make_config(idx: int, seed: int | None = None, n_override: int | None = None) -> Workload:
    """Build synthetic workload ``idx`` (1..5); the default seed is the config number."""
    seed = idx if seed is None else seed
    rng = rng_for(seed)
    if idx == 1:
        n = n_override or 1000
        scene = scene_uniform_slab(rng, n)
        cams = [Camera(np.eye(3), np.zeros(3), 64, 64, 32, 32, 64, 64)]
        return Workload(CONFIG_NAMES[1], [scene], cams, _targets(rng, cams), seed)
    if idx == 2:
        n = n_override or 100_000
        scene = scene_frustum_clusters(rng, n)
        cams = [Camera(np.eye(3), np.zeros(3), 512, 512, 256, 256, 512, 512)]
        return Workload(CONFIG_NAMES[2], [scene], cams, _targets(rng, cams), seed)
    if idx == 3:
        n = n_override or 1_000_000
        scene = scene_box_clusters(rng, n)
        cams = [Camera(np.eye(3), (0.0, 0.0, 13.0), 1100, 1100, 960, 540, 1920, 1080)]
        return Workload(CONFIG_NAMES[3], [scene], cams, _targets(rng, cams), seed)
    if idx == 4:
        n = n_override or 3_000_000
        scene = scene_box_clusters(rng, n)
        f = 1100.0 * 1280.0 / 1920.0
        cams = []
        for k in range(16):
            a = 2.0 * np.pi * k / 16
            R, t = look_at((8.0 * np.cos(a), 0.0, 8.0 * np.sin(a)), (0.0, 0.0, 0.0))
            cams.append(Camera(R, t, f, f, 640, 360, 1280, 720))
        return Workload(CONFIG_NAMES[4], [scene], cams, _targets(rng, cams), seed)
    if idx == 5:
        sizes = [(256, 256), (512, 512), (1280, 720), (1920, 1080)]
        scenes, cams = [], []
        for s in range(8):
            lo, hi = np.log(5.0e4), np.log(2.0e6)
            n = n_override or int(round(np.exp(rng.uniform(lo, hi))))
            scenes.append(scene_box_clusters(rng, n))
            for k in range(4):
                a = 0.5 * np.pi * k
                R, t = look_at((13.0 * np.cos(a), 0.0, 13.0 * np.sin(a)), (0.0, 0.0, 0.0))
                w, h = sizes[int(rng.integers(0, 4))]
                f = 1100.0 * w / 1920.0
                cams.append(Camera(R, t, f, f, w / 2, h / 2, w, h, scene=s))
        return Workload(CONFIG_NAMES[5], scenes, cams, _targets(rng, cams), seed)
    raise ValueError(f"unknown config {idx}")


def tiny_scene(seed: int, n: int = 16, width: int = 64, height: int = 48, f: float = 60.0,
               log_scale=(-1.6, 0.4), opac_sd=1.0, z=(2.0, 5.0), spread=0.5) -> Workload:
    """A small random scene in front of one camera, for checks that need brute force or FD."""
    rng = rng_for(seed)
    zz = rng.uniform(z[0], z[1], n)
    xy = zz[None, :] * rng.uniform(-spread, spread, size=(2, n))
    means = np.concatenate([xy, zz[None, :]], axis=0)
    scene = _finish_scene(rng, means, log_scale[0], log_scale[1], opac_sd)
    cam = Camera(np.eye(3), np.zeros(3), f, f * 1.1, width / 2 - 0.3, height / 2 + 0.2, width, height)
    return Workload(f"tiny{seed}", [scene], [cam], _targets(rng, [cam]), seed)


def tilted_camera_scene(seed: int, n: int = 16, width: int = 64, height: int = 48) -> Workload:
    """Like :func:`tiny_scene` but seen through a rotated, translated camera."""
    rng = rng_for(seed)
    base = tiny_scene(seed, n, width, height)
    R, t = look_at((0.4, -0.3, -0.5), (0.05, 0.02, 3.5))
    # small random extra rotation about the view axis keeps every Gaussian in view
    c, s = np.cos(0.2), np.sin(0.2)
    Rz = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    R = Rz @ R
    t = Rz @ t
    cam = Camera(R, t, 60.0, 66.0, width / 2 - 0.3, height / 2 + 0.2, width, height)
    base.cameras = [cam]
    base.targets = _targets(rng, [cam])
    return base
