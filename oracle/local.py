"""Local re-rendering of one Gaussian's neighbourhood, for finite differences and sampled
gradients at full scene size (test infrastructure, like the rest of ``oracle``).

A Gaussian enters only the lists of the tiles its 3-sigma box covers (Sec. 2.2), so a
change of its parameters changes only the pixels of those tiles. The loss
L = sum over pixels and channels of (C - target)^2 can therefore be differenced over the
tiles of the Gaussian's box alone (old and new box, each widened by one tile), which keeps
central differences free of cancellation against the loss of the whole image. For each
camera of the Gaussian's scene:

* the scene is projected once (``oracle.project``); the perturbed Gaussian is projected
  again on its own;
* each tile of the region gets its list from the other Gaussians whose boxes cover it, in
  the order of Sec. 2.2 (float32 depth, then index), with the perturbed Gaussian inserted
  at its own key if its new box covers the tile;
* the tiles are composited with ``oracle.rasterize_tiles`` (the oracle's per-pixel loop of
  eq. 7).

The analytic gradient of the same local loss comes from ``oracle.rasterize_bwd`` over the
region's tiles and ``oracle.project_bwd`` of the one Gaussian (Sec. 3), summed over the
scene's cameras.

Nothing here is shared with, or calls, the HIP path.
"""
from __future__ import annotations

import numpy as np

import oracle

PARAM_NAMES = ("mean_x", "mean_y", "mean_z", "quat_w", "quat_x", "quat_y", "quat_z",
               "scale_x", "scale_y", "scale_z", "color_r", "color_g", "color_b", "opacity")
PLANES = (("means", 3), ("quats", 4), ("scales", 3), ("colors", 3), ("opacities", 1))


class Discontinuous(Exception):
    """A perturbation moved the Gaussian's box out of the region (a tile or cull decision
    changed inside the step)."""


def _depth_keys(depth: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(depth, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.int64)


class LocalScene:
    """One scene (float64 planes), the cameras that view it and their targets [3, H, W]."""

    def __init__(self, scene: dict, cams, targets, params: oracle.Params, pad: int = 1):
        self.scene = {k: np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for k, v in scene.items()}
        self.N = self.scene["opacities"].shape[-1]
        self.cams = list(cams)
        self.targets = [np.asarray(t, dtype=np.float64).reshape(3, -1) for t in targets]
        self.prm = params
        self.pad = pad
        self.proj = [oracle.project(self.scene, c, params) for c in self.cams]
        self.keys = [_depth_keys(p["depth"]) for p in self.proj]
        self._cand = {}

    # -------------------------------------------------------------------- parameters
    def theta(self, g: int) -> np.ndarray:
        """The 14 parameters of Gaussian g: mean, quaternion (w, x, y, z), scale, colour, opacity."""
        return np.concatenate([self.scene[k][..., g].reshape(-1) for k, _ in PLANES])

    @staticmethod
    def _one(theta: np.ndarray) -> dict:
        out, o = {}, 0
        for k, n in PLANES:
            v = np.asarray(theta[o:o + n], dtype=np.float64)
            out[k] = v.reshape(n, 1) if k != "opacities" else v.reshape(1)
            o += n
        return out

    def _project_one(self, theta, c: int) -> dict:
        return oracle.project(self._one(theta), self.cams[c], self.prm)

    # ------------------------------------------------------------------------ region
    def region(self, g: int, c: int):
        """(x0, y0, x1, y1) tiles: g's box in camera c widened by `pad` tiles, or None if g
        is culled there."""
        p = self.proj[c]
        if p["tiles"][g] <= 0:
            return None
        cam = self.cams[c]
        r = p["rect"][:, g]
        return (max(int(r[0]) - self.pad, 0), max(int(r[1]) - self.pad, 0),
                min(int(r[2]) + self.pad, cam.tiles_x - 1), min(int(r[3]) + self.pad, cam.tiles_y - 1))

    def region_tiles(self, g: int, c: int) -> np.ndarray:
        reg = self.region(g, c)
        if reg is None:
            return np.zeros(0, np.int64)
        tx = self.cams[c].tiles_x
        ys, xs = np.meshgrid(np.arange(reg[1], reg[3] + 1), np.arange(reg[0], reg[2] + 1), indexing="ij")
        return (ys * tx + xs).reshape(-1).astype(np.int64)

    def _candidates(self, g: int, c: int):
        """Visible Gaussians other than g whose boxes meet the region, in list order."""
        key = (g, c)
        if key not in self._cand:
            reg = self.region(g, c)
            p = self.proj[c]
            r = p["rect"]
            m = ((p["tiles"] > 0) & (r[0] <= reg[2]) & (r[2] >= reg[0]) & (r[1] <= reg[3]) & (r[3] >= reg[1]))
            m[g] = False
            idx = np.nonzero(m)[0]
            order = np.lexsort((idx, self.keys[c][idx]))
            self._cand[key] = idx[order]
        return self._cand[key]

    def _local_arrays(self, g: int, c: int, pg: dict):
        """Per-splat arrays of the candidates (local index 0..n-1) and of g (local index n),
        and each region tile's list as local indices."""
        cand = self._candidates(g, c)
        p = self.proj[c]
        n = cand.size
        cat = lambda a, b: np.ascontiguousarray(np.concatenate([a, b], axis=-1))
        mean2d = cat(p["mean2d"][:, cand], pg["mean2d"])
        conic = cat(p["conic"][:, cand], pg["conic"])
        colors = cat(self.scene["colors"][:, cand], np.zeros((3, 1)))
        opac = cat(self.scene["opacities"][cand], np.zeros(1))
        return cand, n, mean2d, conic, colors, opac

    def _lists(self, g: int, c: int, tiles: np.ndarray, pg: dict, cand: np.ndarray):
        cam = self.cams[c]
        tx = cam.tiles_x
        r = self.proj[c]["rect"][:, cand]
        ck = self.keys[c][cand]
        gk = int(_depth_keys(pg["depth"])[0])
        gr = pg["rect"][:, 0]
        gvis = pg["tiles"][0] > 0
        ranges = np.zeros((cam.tiles_x * cam.tiles_y, 2), np.int64)
        ids = []
        pos = 0
        n = cand.size
        for t in tiles:
            ty, txx = divmod(int(t), tx)
            cov = np.nonzero((r[0] <= txx) & (r[2] >= txx) & (r[1] <= ty) & (r[3] >= ty))[0]
            lst = list(cov)
            if gvis and gr[0] <= txx <= gr[2] and gr[1] <= ty <= gr[3]:
                # insert g at its (key, index) place among the covering candidates
                at = int(np.searchsorted(ck[cov] * (self.N + 1) + cand[cov], gk * (self.N + 1) + g))
                lst.insert(at, n)
            ranges[t] = (pos, pos + len(lst))
            ids.extend(lst)
            pos += len(lst)
        return np.asarray(ids, np.int32), ranges

    def _check_inside(self, g: int, c: int, pg: dict):
        reg = self.region(g, c)
        vis = pg["tiles"][0] > 0
        if reg is None:
            if vis:
                raise Discontinuous(f"Gaussian {g} becomes visible in camera {c}")
            return False
        if not vis:
            raise Discontinuous(f"Gaussian {g} is culled in camera {c}")
        r = pg["rect"][:, 0]
        if r[0] < reg[0] or r[1] < reg[1] or r[2] > reg[2] or r[3] > reg[3]:
            raise Discontinuous(f"Gaussian {g}'s box leaves the region in camera {c}")
        return True

    # --------------------------------------------------------------------- renders
    def render(self, g: int, c: int, theta=None) -> dict:
        """The region of camera c rendered with g's parameters theta (default: its own)."""
        theta = self.theta(g) if theta is None else np.asarray(theta, np.float64)
        pg = self._project_one(theta, c)
        if not self._check_inside(g, c, pg):
            return None
        tiles = self.region_tiles(g, c)
        cand, n, mean2d, conic, colors, opac = self._local_arrays(g, c, pg)
        one = self._one(theta)
        colors[:, n] = one["colors"][:, 0]
        opac[n] = one["opacities"][0]
        ids, ranges = self._lists(g, c, tiles, pg, cand)
        out = oracle.rasterize_tiles(mean2d, conic, colors, opac, ids, ranges, self.cams[c], self.prm, tiles,
                                     target=self.targets[c])
        out.update(tiles=tiles, ids=ids, ranges=ranges, mean2d=mean2d, conic=conic, colors=colors, opac=opac,
                   n=n, pg=pg)
        return out

    def loss(self, g: int, theta) -> float:
        """Sum over the scene's cameras of the L2 loss over g's region tiles."""
        total = 0.0
        for c in range(len(self.cams)):
            out = self.render(g, c, theta)
            if out is not None:
                total += out["loss"]
        return total

    def flagged_pixels(self, g: int) -> int:
        """Near-tie pixels (self.prm's margins) in g's regions over all cameras."""
        n = 0
        for c in range(len(self.cams)):
            out = self.render(g, c)
            if out is not None:
                n += int((out["flags"] != 0).sum())
        return n

    def grad(self, g: int) -> np.ndarray:
        """Analytic gradient (Sec. 3) of the local loss with respect to g's 14 parameters."""
        total = np.zeros(14)
        for c in range(len(self.cams)):
            out = self.render(g, c)
            if out is None:
                continue
            cam = self.cams[c]
            W, H = cam.width, cam.height
            tx = cam.tiles_x
            # full-image state with the region's pixels filled in (other tiles have empty lists)
            C = np.zeros((3, H, W))
            T = np.ones((H, W))
            last = np.zeros((H, W), np.int32)
            for s, t in enumerate(out["tiles"]):
                ty, txx = divmod(int(t), tx)
                r0, c0 = ty * 16, txx * 16
                h, w = min(16, H - r0), min(16, W - c0)
                C[:, r0:r0 + h, c0:c0 + w] = out["C"][:, s, :h, :w]
                T[r0:r0 + h, c0:c0 + w] = out["T_final"][s, :h, :w]
                last[r0:r0 + h, c0:c0 + w] = out["last"][s, :h, :w]
            inside = np.zeros((H, W), bool)
            for t in out["tiles"]:
                ty, txx = divmod(int(t), tx)
                inside[ty * 16:(ty + 1) * 16, txx * 16:(txx + 1) * 16] = True
            dL = 2.0 * (C - self.targets[c].reshape(3, H, W))
            dL[:, ~inside] = 0.0
            proj = {"mean2d": out["mean2d"], "conic": out["conic"]}
            bins = {"K": int(out["ids"].size), "ids": out["ids"], "ranges": out["ranges"]}
            g2 = oracle.rasterize_bwd(proj, out["colors"], out["opac"], bins, cam, self.prm, dL,
                                      {"T_final": T, "last": last})
            n = out["n"]
            one = self._one(self.theta(g))
            g3 = oracle.project_bwd(one, cam, self.prm, g2["mean2d"][:, n:n + 1], g2["conic"][:, n:n + 1])
            total += np.concatenate([g3["means"][:, 0], g3["quats"][:, 0], g3["scales"][:, 0],
                                     g2["colors"][:, n], [g2["opacities"][n]]])
        return total

    def fd(self, g: int, i: int, h: float) -> float:
        """Central difference of the local loss in parameter i with step h."""
        th = self.theta(g)
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        return (self.loss(g, tp) - self.loss(g, tm)) / (2.0 * h)


def steps(theta: np.ndarray, rel: float = 1e-5) -> np.ndarray:
    """Central-difference steps for the 14 parameters of one Gaussian: rel times the
    parameter's magnitude (at least rel) for the quaternion, colour and opacity, rel times
    each scale for the scales, and 1e-3 of the smallest scale for the mean, whose loss
    curvature grows as the inverse square of the Gaussian's size."""
    theta = np.asarray(theta, np.float64)
    h = rel * np.maximum(np.abs(theta), 1.0)
    h[7:10] = rel * np.abs(theta[7:10])
    h[0:3] = 1e-3 * np.abs(theta[7:10]).min()
    return h
