"""torch.autograd binding of the rasterizer.

``RasterizeGaussians`` runs the C-ABI forward (gs_project, gs_bin_and_sort,
gs_rasterize_fwd) and, in backward, gs_rasterize_bwd and gs_project_bwd. Between the two
passes it keeps only what the forward already wrote for the backward: the splat records,
the sorted tile lists, T_final and `last` per pixel. The backward recomputes sigma and
alpha of every Gaussian-pixel pair and recovers T by division (Sec. 3.1); no per-pair
state is stored.

``render`` is the user-facing wrapper: it takes parameter tensors and a list of cameras
and returns one [3, H, W] image per camera.
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import abi, pipeline

_capacity_hint: dict = {}


class RasterizeGaussians(torch.autograd.Function):
    """Differentiable map (means, quats, scales, colors, opacities) -> packed image [3, n_pixels]."""

    @staticmethod
    def forward(ctx, means, quats, scales, colors, opacities, cams: pipeline.CameraSet,
                params: abi.GsParams, sizes: tuple, normalize_quats: bool = False):
        g = pipeline.GaussianSet.from_tensors(means.detach().contiguous(), quats.detach().contiguous(),
                                              scales.detach().contiguous(), colors.detach().contiguous(),
                                              opacities.detach().contiguous(), sizes, normalize_quats)
        key = (cams.n_splats, cams.n_tiles)
        r = pipeline.Rasterizer(cams, params, capacity=_capacity_hint.get(key))
        st = r.forward(g)
        _capacity_hint[key] = max(r.capacity, int(st.K * 1.1) + 1024)
        ctx.state = st
        ctx.rasterizer = r
        ctx.gaussians = g
        return st.image.clone()

    @staticmethod
    def backward(ctx, dL_dimage):
        r, st = ctx.rasterizer, ctx.state
        grads = r.backward(st, dL_dimage.contiguous())
        ctx.state = ctx.rasterizer = ctx.gaussians = None
        return (grads["means"], grads["quats"], grads["scales"], grads["colors"], grads["opacities"],
                None, None, None, None)


def render(means: torch.Tensor, quats: torch.Tensor, scales: torch.Tensor, colors: torch.Tensor,
           opacities: torch.Tensor, cameras: Sequence, scene_sizes: Sequence[int] | None = None,
           params: abi.GsParams | None = None, normalize_quats: bool = False) -> list[torch.Tensor]:
    """Renders every camera; returns [3, H, W] images that are differentiable in all five inputs.
    params: thresholds and background (pipeline.make_params); normalize_quats: use q / |q|.

    means [3, N], quats [4, N] (w, x, y, z), scales [3, N], colors [3, N], opacities [N], float32 on
    the GPU. Several scenes may be concatenated along N (scene_sizes); each camera's ``scene``
    attribute selects its scene.
    """
    sizes = tuple(scene_sizes) if scene_sizes is not None else (int(opacities.shape[-1]),)
    cams = pipeline.CameraSet(cameras, sizes, device=means.device)
    params = params or pipeline.make_params()
    packed = RasterizeGaussians.apply(means, quats, scales, colors, opacities, cams, params, sizes, normalize_quats)
    return [cams.unpack(packed, k) for k in range(cams.n_cams)]
