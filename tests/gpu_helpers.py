"""Shared helpers for the GPU parity tests: run the HIP path and the FP64 oracle on the
same seeded workload and return comparable NumPy arrays."""
from __future__ import annotations

import numpy as np

import oracle

# Near-tie margins for the oracle's decision flags. The float32 kernel computes
# alpha = exp2(log2 o + q(Delta)) with |q| <= ~12 in the range where alpha >= 1/255, so
# its relative alpha error stays below ~2e-6; T after n factors carries n such errors
# plus rounding. A pixel whose skip/termination/clamp decision sits within these
# margins of the threshold may legitimately go either way and is excluded (counted).
MARGIN_ALPHA = 1e-5     # relative to alpha_min
MARGIN_T = 1e-3         # relative to T_min
MARGIN_CLAMP = 2e-5     # absolute, around alpha_max

IMAGE_ATOL = 1e-5
GRAD_REL = 1e-3


def oracle_params(**kw):
    return oracle.Params.standard(margin_alpha=MARGIN_ALPHA, margin_T=MARGIN_T, margin_clamp=MARGIN_CLAMP, **kw)


def gpu_forward(wl, keep_visited=True, capacity=None):
    import torch
    from paper_2312_02121_amd import pipeline
    g = pipeline.GaussianSet(wl.scenes)
    cams = pipeline.CameraSet(wl.cameras, g.sizes)
    r = pipeline.Rasterizer(cams, capacity=capacity, keep_visited=keep_visited)
    st = r.forward(g)
    torch.cuda.synchronize()
    return r, st


def splat_arrays(r):
    P = r.cams.n_splats
    rec = r.splats.rec[: P * 12].view(P, 12).cpu().numpy()
    return {
        "mean2d": rec[:, 0:2].T.copy(), "conic": rec[:, 2:5].T.copy(), "opacity": rec[:, 5].copy(),
        "color": rec[:, 6:9].T.copy(), "depth": r.splats.depth[:P].cpu().numpy(),
        "rect": r.splats.rect[: 4 * P].view(P, 4).cpu().numpy().T.copy(),
        "tiles": r.splats.tiles[:P].cpu().numpy(), "src": rec[:, 10].view(np.int32).copy(),
        "cam": rec[:, 11].view(np.int32).copy(),
    }


def bins_arrays(r, K):
    return {"keys": r.bins.keys[:K].cpu().numpy().view(np.uint64), "ids": r.bins.ids[:K].cpu().numpy(),
            "ranges": r.bins.ranges[: 2 * r.cams.n_tiles].view(-1, 2).cpu().numpy()}


def camera_images(r, st, k):
    cams = r.cams
    out = {"C": cams.unpack(st.image, k).cpu().numpy()}
    for name in ("T_final", "last", "visited"):
        t = getattr(st, name)
        if t is not None:
            out[name] = cams.unpack(t.view(1, -1), k)[0].cpu().numpy()
    return out


def oracle_camera(wl, k, prm=None):
    cam = wl.cameras[k]
    scene = wl.scenes[cam.scene]
    prm = prm or oracle_params()
    return oracle.render(scene, cam, prm), scene, cam, prm


def rel_err(a, b):
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))


def elementwise_ok(a, b, rel=GRAD_REL):
    """|a - b| <= rel (|b| + rms(b)) everywhere."""
    rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
    return bool(np.all(np.abs(a - b) <= rel * (np.abs(b) + rms) + 1e-30))


def worst_element(a, b):
    """(index, gpu, ref, normalised error) of the element furthest from the elementwise bar."""
    rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
    r = np.abs(a - b) / (np.abs(b) + rms + 1e-30)
    i = np.unravel_index(int(np.argmax(r)), r.shape)
    return tuple(int(x) for x in i), float(a[i]), float(b[i]), float(r[i])


def tile_offsets(wl):
    offs, t = [], 0
    for c in wl.cameras:
        offs.append(t)
        t += c.n_tiles
    return offs
