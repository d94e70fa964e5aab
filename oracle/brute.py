"""Independent NumPy implementations used to pin the C oracle (test infrastructure).

* ``project`` -- the projection of Sec. 2.1 written a second way: the camera-frame
  covariance W = R_cw Sigma R_cw^T first, then Sigma' = J W J^T; R from the
  Hamilton product q (0, v) q*; mu' from the pinhole form f t/t_z + c + 1/2 that
  eq. (2) reduces to once P of eq. (1) is substituted.
* ``render`` -- compositing of Sec. 2.2 with one global depth order instead of
  per-tile lists: every pixel walks all Gaussians whose 3-sigma tile box covers
  the pixel's tile, sorted by (float32 depth, index). Vectorised over pixels.

Neither function shares code with ``gs_oracle.c``.
"""
from __future__ import annotations

import numpy as np


def hamilton(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Quaternion product, (w, x, y, z) order, broadcasting over trailing axes."""
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ])


def rotation_hamilton(q: np.ndarray) -> np.ndarray:
    """R with R v = q (0, v) q* for unit q; q is [4] or [4, N]; returns [3, 3] or [N, 3, 3]."""
    q = np.asarray(q, dtype=np.float64)
    single = q.ndim == 1
    q = q.reshape(4, -1)
    conj = q * np.array([1.0, -1.0, -1.0, -1.0])[:, None]
    cols = []
    for e in np.eye(3):
        v = np.zeros_like(q)
        v[1:] = e[:, None]
        cols.append(hamilton(hamilton(q, v), conj)[1:])      # [3, N]
    R = np.stack(cols, axis=-1)                               # [3, N, 3] (row, n, col)
    R = np.transpose(R, (1, 0, 2))
    return R[0] if single else R


def project(scene: dict, cam) -> dict:
    means = np.asarray(scene["means"], dtype=np.float64)
    q = np.asarray(scene["quats"], dtype=np.float64)
    s = np.asarray(scene["scales"], dtype=np.float64)
    N = means.shape[1]
    R = rotation_hamilton(q / np.linalg.norm(q, axis=0, keepdims=True))   # [N,3,3]
    Sigma = np.einsum("nij,nj,nkj->nik", R, s.T ** 2, R)
    Rcw = np.asarray(cam.R, dtype=np.float64).reshape(3, 3)
    tcw = np.asarray(cam.t, dtype=np.float64).reshape(3)
    t = (Rcw @ means).T + tcw                                           # [N,3]
    Wc = np.einsum("ij,njk,lk->nil", Rcw, Sigma, Rcw)
    tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
    J = np.zeros((N, 2, 3))
    J[:, 0, 0] = cam.fx / tz
    J[:, 0, 2] = -cam.fx * tx / tz ** 2
    J[:, 1, 1] = cam.fy / tz
    J[:, 1, 2] = -cam.fy * ty / tz ** 2
    cov2d = np.einsum("nij,njk,nlk->nil", J, Wc, J)
    mean2d = np.stack([cam.fx * tx / tz + cam.cx + 0.5, cam.fy * ty / tz + cam.cy + 0.5])
    conic = np.linalg.inv(cov2d)
    ex = 3.0 * np.sqrt(cov2d[:, 0, 0])
    ey = 3.0 * np.sqrt(cov2d[:, 1, 1])
    return {"mean2d": mean2d, "cov2d": cov2d, "conic": conic, "depth": tz,
            "box": np.stack([mean2d[0] - ex, mean2d[1] - ey, mean2d[0] + ex, mean2d[1] + ey])}


def tile_box_covers(rect: np.ndarray, tiles: np.ndarray, n: int, tx: np.ndarray, ty: np.ndarray):
    if tiles[n] <= 0:
        return np.zeros(tx.shape, dtype=bool)
    return (tx >= rect[0, n]) & (tx <= rect[2, n]) & (ty >= rect[1, n]) & (ty <= rect[3, n])


def render(mean2d, conic, depth, rect, tiles, colors, opac, width: int, height: int,
           alpha_min: float, alpha_max: float, T_min: float, background=(0.0, 0.0, 0.0)) -> dict:
    """Global-depth-order compositing; conic is [3, N] = (Y00, Y01, Y11). The background
    colour is seen through what is left of each pixel (T_final)."""
    jj, ii = np.meshgrid(np.arange(width), np.arange(height))
    px, py = jj + 0.5, ii + 0.5
    tx, ty = jj // 16, ii // 16
    N = depth.shape[0]
    order = np.lexsort((np.arange(N), depth.astype(np.float32)))
    T = np.ones((height, width))
    C = np.zeros((3, height, width))
    done = np.zeros((height, width), dtype=bool)
    count = np.zeros((height, width), dtype=np.int64)   # position in the pixel's own list
    last = np.zeros((height, width), dtype=np.int64)
    for n in order:
        inc = tile_box_covers(rect, tiles, n, tx, ty)
        if not inc.any():
            continue
        dx = mean2d[0, n] - px
        dy = mean2d[1, n] - py
        sig = 0.5 * (conic[0, n] * dx * dx + 2.0 * conic[1, n] * dx * dy + conic[2, n] * dy * dy)
        a = np.minimum(alpha_max, opac[n] * np.exp(-sig))
        live = inc & ~done
        count = count + inc
        keep = live & ~(a < alpha_min)
        Tn = T * (1.0 - a)
        stop = keep & (Tn < T_min)
        done |= stop
        keep &= ~stop
        for ch in range(3):
            C[ch] = np.where(keep, C[ch] + colors[ch, n] * a * T, C[ch])
        T = np.where(keep, Tn, T)
        last = np.where(keep, count, last)
    for ch in range(3):
        C[ch] = C[ch] + T * background[ch]
    return {"C": C, "T_final": T, "last": last}
