"""Shared helpers for the GPU parity tests: run the HIP path and the FP64 oracle on the
same seeded workload and return comparable NumPy arrays."""
from __future__ import annotations

import numpy as np

import oracle

# Near-tie margins for the oracle's decision flags: error bounds of the float32 kernel.
# The kernel evaluates alpha = exp2(e) with e = log2 o - sigma log2(e) formed in float64 and
# rounded to float32 once. For alpha >= 1/255, |e| < 8, so that rounding moves e by at most
# 2^-22 and alpha by at most ln 2 * 2^-22 = 1.65e-7 relative; v_exp_f32 adds at most one ulp
# (2^-23 = 1.19e-7 relative; measured on the MI355X over all 1.09e9 float32 inputs in
# [-8, 0]: at most 0.78 ulp, 8.5e-8 relative). MARGIN_ALPHA = 3e-7 bounds the sum (2.6e-7). The forward updates T with one
# fused multiply-add, T - T alpha, so each factor adds one rounding (ROUND_T = 2^-24) besides
# the alpha error carried through (1 - alpha); a clamped alpha is alpha_max exactly. The oracle
# adds these bounds up along each pixel's walk. A pixel whose skip, termination or clamp
# decision lies inside them may legitimately go either way: it is excluded from image
# comparison and receives zero upstream gradient on both sides.
MARGIN_ALPHA = 3e-7     # relative to alpha_min (and to each alpha, in the T bound)
MARGIN_T = 1e-7         # base of the T band, relative to T_min
ROUND_T = 2.0 ** -24    # one rounding per factor of T
MARGIN_CLAMP = 3e-7     # absolute, around alpha_max
FLAG_RATE = 1e-4        # at most this fraction of a view's pixels may be flagged


def flag_budget(pixels: int) -> int:
    """Flagged pixels allowed in a view of `pixels` pixels: FLAG_RATE of them, and at least
    two (a single pixel is already more than 1e-4 of an image below 10 000 pixels)."""
    return max(2, int(FLAG_RATE * pixels))


IMAGE_ATOL = 1e-5
GRAD_REL = 1e-3


def oracle_params(**kw):
    return oracle.Params.standard(margin_alpha=MARGIN_ALPHA, margin_T=MARGIN_T, margin_clamp=MARGIN_CLAMP,
                                  round_T=ROUND_T, **kw)


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


HEADER, BUCKETS, N_BUCKETS = 64, 8, 16   # work-list layout: header words, bucket counts


def same_work_list(x, y):
    """Work lists are equal up to the order of items inside a length bucket (which blocks
    fill concurrently): the header and every bucket's set of items agree."""
    assert np.array_equal(x[:HEADER], y[:HEADER])
    n = int(x[0])
    assert np.array_equal(x[HEADER + n:], y[HEADER + n:])
    at = HEADER
    for k in range(N_BUCKETS):
        c = int(x[BUCKETS + k])
        assert np.array_equal(np.sort(x[at:at + c]), np.sort(y[at:at + c])), k
        at += c
    assert at == HEADER + n
