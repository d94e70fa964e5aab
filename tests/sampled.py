"""Seeded sampling of Gaussians for gradient checks at full scene size (tests only).

Both the CPU finite-difference pin and the GPU parity test walk the same seeded order:
per scene, a permutation of the Gaussians that some camera of the scene sees, keeping
those with a nonzero gradient of the L2 loss (a Gaussian that no pixel composites has
nothing to check). Everything here runs the oracle only.
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle import local


def local_scenes(wl, params: oracle.Params, pad: int = 0):
    """One oracle.local.LocalScene per scene of the workload, with its cameras and targets."""
    out = []
    for s in range(len(wl.scenes)):
        ks = [k for k, c in enumerate(wl.cameras) if c.scene == s]
        out.append(local.LocalScene(wl.scenes[s], [wl.cameras[k] for k in ks], [wl.targets[k] for k in ks],
                                    params, pad=pad))
    return out


def candidates(ls: local.LocalScene, seed: int, limit: int = 400):
    """Seeded order of the Gaussians that some camera of the scene sees."""
    vis = np.nonzero(np.any([p["tiles"] > 0 for p in ls.proj], axis=0))[0]
    return [int(g) for g in np.random.default_rng(seed).permutation(vis)[:limit]]


def per_type_rms(values: np.ndarray) -> np.ndarray:
    """values [n, 14]: rms over the sample of each parameter type (mean, quaternion, scale,
    colour, opacity), broadcast back to the 14 columns."""
    out = np.zeros(14)
    for a, b in ((0, 3), (3, 7), (7, 10), (10, 13), (13, 14)):
        out[a:b] = np.sqrt(np.mean(values[:, a:b] ** 2))
    return out


def fd_scene(wl, s: int, per_scene: int, seed: int):
    """(analytic [n, 14], central differences at h [n, 14], discontinuous, zero-gradient)
    for the first `per_scene` Gaussians of scene s's seeded order with a nonzero gradient and
    a continuous loss (steps h and h/10 of oracle.local.steps agree within 10%); FP64, no
    interface rounding, one thread."""
    prm = oracle.Params.standard(round_interface=False, n_threads=1)
    ks = [k for k, c in enumerate(wl.cameras) if c.scene == s]
    ls = local.LocalScene(wl.scenes[s], [wl.cameras[k] for k in ks], [wl.targets[k] for k in ks], prm, pad=0)
    an_all, fd_all = [], []
    disc = zero = 0
    for g in candidates(ls, seed):
        if len(an_all) == per_scene:
            break
        an = ls.grad(g)
        if not np.abs(an).max() > 0.0:
            zero += 1
            continue
        hs = local.steps(ls.theta(g))
        try:
            f1 = np.array([ls.fd(g, i, hs[i]) for i in range(14)])
            f2 = np.array([ls.fd(g, i, hs[i] / 10) for i in range(14)])
        except local.Discontinuous:
            disc += 1
            continue
        if np.abs(f1 - f2).max() > 0.1 * np.abs(an).max():
            disc += 1
            continue
        an_all.append(an)
        fd_all.append(f1)
    return np.array(an_all).reshape(-1, 14), np.array(fd_all).reshape(-1, 14), disc, zero
