"""Shared helpers for the GPU parity tests: run the HIP path and the FP64 oracle on the
same seeded workload and return comparable NumPy arrays."""
from __future__ import annotations

import numpy as np

import oracle

# Near-tie margins for the oracle's decision flags. The float32 kernel evaluates
# alpha = exp2(e) with e = log2 o - sigma log2(e) formed in float64 and rounded to float32
# once; for alpha >= 1/255, |e| <= 8, so the rounding moves alpha by at most 8 * 2^-24 * ln 2
# (3.3e-7) relative, and exp2 adds about one ulp: MARGIN_ALPHA leaves a factor of four over
# that. T after n factors carries, per factor, alpha / (1 - alpha) times the alpha error
# plus two roundings; the oracle adds that bound up along the walk on top of MARGIN_T.
# A pixel whose skip, termination or clamp decision lies inside these margins may
# legitimately go either way: it is excluded from comparison and counted.
MARGIN_ALPHA = 2e-6     # relative to alpha_min
MARGIN_T = 1e-5         # relative to T_min, plus the accumulated float32 bound
MARGIN_CLAMP = 2e-6     # absolute, around alpha_max

IMAGE_ATOL = 1e-5
GRAD_REL = 1e-3


def oracle_params(**kw):
    return oracle.Params.standard(margin_alpha=MARGIN_ALPHA, margin_T=MARGIN_T, margin_clamp=MARGIN_CLAMP, **kw)


def gpu_forward(wl, keep_visited=True, capacity=None, params=None, normalize_quats=False, box_lambda_max=False):
    import torch
    from paper_2312_02121_amd import pipeline
    g = pipeline.GaussianSet(wl.scenes, normalize_quats=normalize_quats, box_lambda_max=box_lambda_max)
    cams = pipeline.CameraSet(wl.cameras, g.sizes)
    r = pipeline.Rasterizer(cams, params, capacity=capacity, keep_visited=keep_visited, keep_records=True)
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


def check_projection(wl, r, views=None, prm=None):
    """Splat fields of every camera (or of `views`) bit-exact against the oracle's projection."""
    s = splat_arrays(r)
    for k in (range(len(wl.cameras)) if views is None else views):
        cam = wl.cameras[k]
        off = int(r.cams.host[k]["proj_offset"])
        n = int(r.cams.host[k]["gauss_count"])
        o = oracle.project(wl.scenes[cam.scene], cam, prm or oracle_params())
        sl = slice(off, off + n)
        assert np.array_equal(s["tiles"][sl], o["tiles"]), "tiles_touched"
        vis = o["tiles"] > 0
        assert np.array_equal(s["rect"][:, sl][:, vis], o["rect"][:, vis]), "rect"
        assert np.array_equal(s["mean2d"][:, sl][:, vis].astype(np.float64), o["mean2d"][:, vis]), "mean2d"
        assert np.array_equal(s["conic"][:, sl][:, vis].astype(np.float64), o["conic"][:, vis]), "conic"
        assert np.array_equal(s["depth"][sl][vis].astype(np.float64), o["depth"][vis]), "depth"
        sc = wl.scenes[cam.scene]
        assert np.array_equal(s["opacity"][sl][vis], sc["opacities"][vis])
        assert np.array_equal(s["color"][:, sl][:, vis], sc["colors"][:, vis])
        assert np.array_equal(s["src"][sl][vis], np.nonzero(vis)[0] + (sum(wl.scenes[j]["opacities"].shape[0]
                                                                          for j in range(cam.scene))))
