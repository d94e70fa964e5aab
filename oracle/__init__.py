"""CPU FP64 oracle of the differentiable tile rasterizer of 3D Gaussians.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package. The product path (the HIP
library and its Python binding) never imports, links or calls it, and it never
imports the product path. The only thing both sides share is the seeded input
generator module, which holds none of the method's arithmetic.

The arithmetic lives in ``gs_oracle.c`` (plain C, double precision, written
from the paper's equations; see its header for the readings it takes). This
module marshals NumPy arrays in and out and strings the per-camera steps
together:

    project -> bin_and_sort -> tile_ranges -> rasterize_fwd      (Sec. 2)
    rasterize_bwd -> project_bwd                                 (Sec. 3)

``brute`` holds an independent global-sort renderer used to pin the tiling.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ERRATA_R11 = 1
ERRATA_EQ23_W = 2
ERRATA_DELTA = 4
ERRATA_EQ28_ONLY = 8

F32 = np.float32


def build(force: bool = True) -> str:
    """Compile gs_oracle.c into liboracle.so with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("W", ctypes.c_int64), ("H", ctypes.c_int64),
                ("near_plane", ctypes.c_double), ("far_plane", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("T_min", ctypes.c_double), ("margin_alpha", ctypes.c_double),
                ("margin_T", ctypes.c_double), ("margin_clamp", ctypes.c_double),
                ("round_interface", ctypes.c_int32), ("errata", ctypes.c_int32),
                ("n_threads", ctypes.c_int32), ("normalize_quats", ctypes.c_int32),
                ("background", ctypes.c_double * 3), ("box_lambda_max", ctypes.c_int32), ("pad2", ctypes.c_int32),
                ("round_T", ctypes.c_double)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_project.restype = _I64
        L.orc_project.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
        L.orc_bin_and_sort.restype = None
        L.orc_bin_and_sort.argtypes = [_I64, _P, _P, _P, _I64, _I64, _I64, _P, _P]
        L.orc_tile_ranges.restype = None
        L.orc_tile_ranges.argtypes = [_I64, _P, _I64, _I64, _P]
        L.orc_rasterize_fwd.restype = None
        L.orc_rasterize_fwd.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _I64, _I64, _P, _P, _P, _P, _P, _P]
        L.orc_rasterize_bwd.restype = None
        L.orc_rasterize_bwd.argtypes = [_I64, _P, _P, _P, _P, _I64, _P, _P, _I64, _I64, _P, _P, _P, _P,
                                        ctypes.c_int, _P, _P, _P, _P]
        L.orc_project_bwd.restype = None
        L.orc_project_bwd.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
        L.orc_quat_to_rot.restype = None
        L.orc_quat_to_rot.argtypes = [_P, ctypes.c_int, _P]
        L.orc_cov3d.restype = None
        L.orc_cov3d.argtypes = [_P, _P, ctypes.c_int, _P, _P, _P]
        L.orc_conic_grad_to_cov2d.restype = None
        L.orc_conic_grad_to_cov2d.argtypes = [_P, _P, _P]
        L.orc_project_state.restype = ctypes.c_int
        L.orc_project_state.argtypes = [_P, _P, _P, _P, _P, _P]
        L.orc_rasterize_tiles.restype = ctypes.c_double
        L.orc_rasterize_tiles.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _I64, _I64, _P, _I64, _P, _P, _P, _P, _P, _P]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ------------------------------------------------------------------------- parameters

@dataclass
class Params:
    """Compositing thresholds. ``standard()`` mirrors the float32 values the HIP path uses."""
    alpha_min: float = 0.0
    alpha_max: float = 1.0
    T_min: float = 0.0
    margin_alpha: float = 0.0
    margin_T: float = 0.0
    margin_clamp: float = 0.0
    round_interface: bool = True
    errata: int = 0
    n_threads: int = 0
    background: tuple = (0.0, 0.0, 0.0)   # colour seen through T_final; zero in the paper
    normalize_quats: bool = False         # R(q / |q|); the paper takes q as given
    box_lambda_max: bool = False          # square 3-sigma box from lambda_max (tight box otherwise)
    round_T: float = 0.0                  # rounding bound of one float32 update of T (near-tie flags)

    @staticmethod
    def standard(**kw) -> "Params":
        base = dict(alpha_min=float(F32(1.0 / 255.0)), alpha_max=float(F32(0.99)), T_min=float(F32(1e-4)))
        base.update(kw)
        return Params(**base)

    @staticmethod
    def literal(**kw) -> "Params":
        base = dict(alpha_min=0.0, alpha_max=1.0, T_min=0.0)
        base.update(kw)
        return Params(**base)

    def c(self) -> _Params:
        return _Params(self.alpha_min, self.alpha_max, self.T_min, self.margin_alpha, self.margin_T,
                       self.margin_clamp, int(bool(self.round_interface)), int(self.errata),
                       int(self.n_threads), int(bool(self.normalize_quats)),
                       (ctypes.c_double * 3)(*[float(x) for x in self.background]),
                       int(bool(self.box_lambda_max)), 0, float(self.round_T))


def camera_struct(cam) -> _Camera:
    """Any object with R, t, fx, fy, cx, cy, width, height, near, far attributes."""
    c = _Camera()
    R = np.asarray(cam.R, dtype=np.float64).reshape(9)
    t = np.asarray(cam.t, dtype=np.float64).reshape(3)
    for i in range(9):
        c.R[i] = float(R[i])
    for i in range(3):
        c.t[i] = float(t[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.W, c.H = int(cam.width), int(cam.height)
    c.near_plane, c.far_plane = float(cam.near), float(cam.far)
    return c


def tiles_of(cam):
    tx = (int(cam.width) + 15) // 16
    ty = (int(cam.height) + 15) // 16
    return tx, ty


# ------------------------------------------------------------------------------ steps

def quat_to_rot(q, errata: int = 0) -> np.ndarray:
    q = _f64(q).reshape(4)
    R = np.zeros(9)
    lib().orc_quat_to_rot(_ptr(q), errata, _ptr(R))
    return R.reshape(3, 3)


def cov3d(q, s, errata: int = 0):
    q, s = _f64(q).reshape(4), _f64(s).reshape(3)
    R, M, S = np.zeros(9), np.zeros(9), np.zeros(9)
    lib().orc_cov3d(_ptr(q), _ptr(s), errata, _ptr(R), _ptr(M), _ptr(S))
    return S.reshape(3, 3)


def conic_grad_to_cov2d(Y, G) -> np.ndarray:
    Y, G = _f64(Y).reshape(4), _f64(G).reshape(4)
    out = np.zeros(4)
    lib().orc_conic_grad_to_cov2d(_ptr(Y), _ptr(G), _ptr(out))
    return out.reshape(2, 2)


def project_state(mu, q, s, cam, params: Params | None = None) -> dict:
    """Intermediate quantities of one projection (for invariant tests)."""
    params = params or Params.literal(round_interface=False)
    mu, q, s = _f64(mu).reshape(3), _f64(q).reshape(4), _f64(s).reshape(3)
    out = np.zeros(64)
    cs, ps = camera_struct(cam), params.c()
    ok = lib().orc_project_state(_ptr(mu), _ptr(q), _ptr(s), ctypes.byref(cs), ctypes.byref(ps), _ptr(out))
    return {
        "visible": bool(ok), "R": out[0:9].reshape(3, 3), "Sigma": out[9:18].reshape(3, 3),
        "t": out[18:22], "tp": out[22:26], "J": out[26:32].reshape(2, 3),
        "cov2d": out[32:36].reshape(2, 2), "Y": out[36:40].reshape(2, 2), "mean2d": out[40:42],
        "depth": out[42], "rect": out[43:47].astype(np.int64), "tiles": int(out[47]), "det": out[48],
    }


def project(scene: dict, cam, params: Params) -> dict:
    means, quats, scales = _f64(scene["means"]), _f64(scene["quats"]), _f64(scene["scales"])
    N = means.shape[1]
    out = {
        "mean2d": np.zeros((2, N)), "conic": np.zeros((3, N)), "depth": np.zeros(N),
        "rect": np.zeros((4, N), dtype=np.int32), "tiles": np.zeros(N, dtype=np.int32),
    }
    cs, ps = camera_struct(cam), params.c()
    out["visible"] = lib().orc_project(N, _ptr(means), _ptr(quats), _ptr(scales), ctypes.byref(cs),
                                       ctypes.byref(ps), _ptr(out["mean2d"]), _ptr(out["conic"]),
                                       _ptr(out["depth"]), _ptr(out["rect"]), _ptr(out["tiles"]))
    return out


def bin_and_sort(proj: dict, cam, tile_offset: int = 0) -> dict:
    N = proj["depth"].shape[0]
    K = int(proj["tiles"].astype(np.int64).sum())
    keys = np.zeros(max(K, 1), dtype=np.uint64)
    ids = np.zeros(max(K, 1), dtype=np.int32)
    tx, ty = tiles_of(cam)
    lib().orc_bin_and_sort(N, _ptr(proj["rect"]), _ptr(proj["depth"]), _ptr(proj["tiles"]), tx,
                           tile_offset, K, _ptr(keys), _ptr(ids))
    keys, ids = keys[:K], ids[:K]
    ranges = np.zeros((tx * ty, 2), dtype=np.int64)
    lib().orc_tile_ranges(K, _ptr(keys) if K else None, tx * ty, tile_offset, _ptr(ranges))
    return {"K": K, "keys": keys, "ids": ids, "ranges": ranges}


def splats_from_2d(mean2d, conic, depth, valid, cam, params: Params) -> dict:
    """The per-stage rasterizer input (Sec. 2.2 without the projection): the 3-sigma tile box
    of each slot from given mu' [2, N], Y [3, N] = (Y00, Y01, Y11) and depth [N], with
    Sigma' = Y^-1 formed in float64 from the given values (the box rule of the projection,
    including its lambda_max option). Slots with valid 0, a Y that is not positive definite
    or a box off the image are culled (tiles 0). Returns a projection-like dict."""
    m = _f64(mean2d)
    Y = _f64(conic)
    d = _f64(depth)
    N = m.shape[1]
    TX, TY = tiles_of(cam)
    rect = np.zeros((4, N), dtype=np.int32)
    tiles = np.zeros(N, dtype=np.int32)
    for n in range(N):
        y00, y01, y11 = Y[0, n], Y[1, n], Y[2, n]
        det = y00 * y11 - y01 * y01
        if not valid[n] or not np.isfinite(det) or not det > 0.0 or not y00 > 0.0 or not y11 > 0.0:
            continue
        if not (np.isfinite(d[n]) and d[n] > 0.0):      # not a depth key: culled
            continue
        c00, c01, c11 = y11 / det, -y01 / det, y00 / det
        if not (np.isfinite(c00) and np.isfinite(c01) and np.isfinite(c11) and np.isfinite(m[0, n])
                and np.isfinite(m[1, n])):
            continue
        ex, ey = 3.0 * np.sqrt(c00), 3.0 * np.sqrt(c11)
        if params.box_lambda_max:
            h = (c00 - c11) / 2.0
            ex = ey = 3.0 * np.sqrt((c00 + c11) / 2.0 + np.sqrt(h * h + c01 * c01))
        x0, x1 = np.floor((m[0, n] - ex) / 16.0), np.floor((m[0, n] + ex) / 16.0)
        y0, y1 = np.floor((m[1, n] - ey) / 16.0), np.floor((m[1, n] + ey) / 16.0)
        if not (x1 >= 0 and y1 >= 0 and x0 <= TX - 1 and y0 <= TY - 1):
            continue
        r = (max(x0, 0), max(y0, 0), min(x1, TX - 1), min(y1, TY - 1))
        rect[:, n] = r
        tiles[n] = int((r[2] - r[0] + 1) * (r[3] - r[1] + 1))
    return {"mean2d": m, "conic": Y, "depth": d, "rect": rect, "tiles": tiles}


def rasterize_fwd(proj: dict, colors, opac, bins: dict, cam, params: Params) -> dict:
    colors, opac = _f64(colors), _f64(opac)
    N = opac.shape[0]
    W, H = int(cam.width), int(cam.height)
    out = {"C": np.zeros((3, H, W)), "T_final": np.zeros((H, W)),
           "last": np.zeros((H, W), dtype=np.int32), "visited": np.zeros((H, W), dtype=np.int32),
           "flags": np.zeros((H, W), dtype=np.int32)}
    ids = bins["ids"] if bins["K"] else np.zeros(1, dtype=np.int32)
    ps = params.c()
    lib().orc_rasterize_fwd(N, _ptr(proj["mean2d"]), _ptr(proj["conic"]), _ptr(colors), _ptr(opac),
                            _ptr(ids), _ptr(bins["ranges"]), W, H, ctypes.byref(ps), _ptr(out["C"]),
                            _ptr(out["T_final"]), _ptr(out["last"]), _ptr(out["visited"]),
                            _ptr(out["flags"]))
    return out


def rasterize_tiles(mean2d, conic, colors, opac, ids, ranges, cam, params: Params, tiles, target=None) -> dict:
    """eq. (7) on the tiles ``tiles`` (tile indices of ``cam``) only, each with its list
    ids[ranges[t, 0]:ranges[t, 1]] into the given per-splat arrays. Returns C [3, n, 16, 16],
    T_final, last, flags [n, 16, 16] (pixels past the image edge hold zeros) and, with a
    target [3, H*W] (or [3, H, W]), loss = sum over the tiles' pixels of (C - target)^2."""
    mean2d, conic, colors, opac = _f64(mean2d), _f64(conic), _f64(colors), _f64(opac)
    ids = np.ascontiguousarray(ids, dtype=np.int32) if len(ids) else np.zeros(1, np.int32)
    ranges = np.ascontiguousarray(ranges, dtype=np.int64)
    sel = np.ascontiguousarray(tiles, dtype=np.int64)
    n = sel.size
    W, H = int(cam.width), int(cam.height)
    out = {"C": np.zeros((3, n, 16, 16)), "T_final": np.zeros((n, 16, 16)),
           "last": np.zeros((n, 16, 16), np.int32), "flags": np.zeros((n, 16, 16), np.int32)}
    tgt = None if target is None else _f64(np.asarray(target).reshape(3, -1))
    ps = params.c()
    out["loss"] = lib().orc_rasterize_tiles(opac.shape[0], _ptr(mean2d), _ptr(conic), _ptr(colors), _ptr(opac),
                                            _ptr(ids), _ptr(ranges), W, H, ctypes.byref(ps), n,
                                            _ptr(sel) if n else None, _ptr(tgt) if tgt is not None else None,
                                            _ptr(out["C"]), _ptr(out["T_final"]), _ptr(out["last"]),
                                            _ptr(out["flags"]))
    return out


def rasterize_bwd(proj: dict, colors, opac, bins: dict, cam, params: Params, dL_dC, fwd: dict,
                  form: int = 0) -> dict:
    colors, opac = _f64(colors), _f64(opac)
    dL_dC = _f64(dL_dC)
    N = opac.shape[0]
    W, H = int(cam.width), int(cam.height)
    g = {"mean2d": np.zeros((2, N)), "conic": np.zeros((3, N)), "colors": np.zeros((3, N)),
         "opacities": np.zeros(N)}
    ids = bins["ids"] if bins["K"] else np.zeros(1, dtype=np.int32)
    ps = params.c()
    lib().orc_rasterize_bwd(N, _ptr(_f64(proj["mean2d"])), _ptr(_f64(proj["conic"])), _ptr(colors), _ptr(opac),
                            bins["K"], _ptr(ids), _ptr(bins["ranges"]), W, H, ctypes.byref(ps),
                            _ptr(dL_dC), _ptr(_f64(fwd["T_final"])),
                            _ptr(np.ascontiguousarray(fwd["last"], dtype=np.int32)), form,
                            _ptr(g["mean2d"]), _ptr(g["conic"]), _ptr(g["colors"]), _ptr(g["opacities"]))
    return g


def project_bwd(scene: dict, cam, params: Params, dmean2d, dconic, with_pose: bool = False) -> dict:
    means, quats, scales = _f64(scene["means"]), _f64(scene["quats"]), _f64(scene["scales"])
    N = means.shape[1]
    g = {"means": np.zeros((3, N)), "scales": np.zeros((3, N)), "quats": np.zeros((4, N))}
    dT = np.zeros(16) if with_pose else None
    cs, ps = camera_struct(cam), params.c()
    lib().orc_project_bwd(N, _ptr(means), _ptr(quats), _ptr(scales), ctypes.byref(cs), ctypes.byref(ps),
                          _ptr(_f64(dmean2d)), _ptr(_f64(dconic)), _ptr(g["means"]), _ptr(g["scales"]),
                          _ptr(g["quats"]), _ptr(dT) if dT is not None else None)
    if with_pose:
        g["Tcw"] = dT.reshape(4, 4)
    return g


# --------------------------------------------------------------------------- pipelines

def render(scene: dict, cam, params: Params, tile_offset: int = 0) -> dict:
    """Forward pass of one camera: projection, binning, sort, ranges, compositing."""
    proj = project(scene, cam, params)
    bins = bin_and_sort(proj, cam, tile_offset)
    fwd = rasterize_fwd(proj, scene["colors"], scene["opacities"], bins, cam, params)
    return {"proj": proj, "bins": bins, **fwd}


def render_backward(scene: dict, cam, params: Params, dL_dC, state: dict | None = None, form: int = 0,
                    with_pose: bool = False) -> dict:
    """Gradients of sum(dL_dC * C) with respect to every Gaussian parameter (one camera)."""
    state = state or render(scene, cam, params)
    g2 = rasterize_bwd(state["proj"], scene["colors"], scene["opacities"], state["bins"], cam, params,
                       dL_dC, state, form)
    g3 = project_bwd(scene, cam, params, g2["mean2d"], g2["conic"], with_pose=with_pose)
    out = {"means": g3["means"], "scales": g3["scales"], "quats": g3["quats"],
           "colors": g2["colors"], "opacities": g2["opacities"],
           "mean2d": g2["mean2d"], "conic": g2["conic"]}
    if with_pose:
        out["Tcw"] = g3["Tcw"]
    return out


def loss_l2(C: np.ndarray, target: np.ndarray) -> tuple[float, np.ndarray]:
    """L = sum (C - target)^2 and dL/dC = 2 (C - target)."""
    d = C - np.asarray(target, dtype=np.float64)
    return float(np.sum(d * d)), 2.0 * d


def max_threads() -> int:
    return int(lib().orc_max_threads())
