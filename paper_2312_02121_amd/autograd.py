"""torch.autograd binding of the rasterizer.

``RasterizeGaussians`` runs the C-ABI forward (gs_project, gs_bin_and_sort,
gs_rasterize_fwd) and, in backward, gs_rasterize_bwd and gs_project_bwd. Between the two
passes it keeps only what the forward already wrote for the backward: the splat records,
the sorted tile lists, T_final and `last` per pixel. The backward recomputes sigma and
alpha of every Gaussian-pixel pair and recovers T by division (Sec. 3.1); no per-pair
state is stored.

``render`` is the user-facing wrapper: it takes parameter tensors and a list of cameras
and returns one [3, H, W] image per camera.

``l2_loss`` is the training form for the L2 image loss L = sum (C - target)^2 over a batch
of cameras: ``RasterizeL2Loss`` runs projection, binning, the fused forward + dL/dC +
backward launch and the projection backward in its forward (one HIP-graph replay of a
step whose buffers are kept between calls), returns L, and hands the stored gradients,
scaled by the incoming dL_out, to autograd in its backward. No call synchronises the host:
the list length is read back asynchronously and the capacity regrown at the next call, and
a step whose list overflowed returns a NaN loss.

The per-stage form splits the same map at the 2D splats: ``ProjectGaussians`` (Sec. 2.1:
means, quats, scales -> mu', Y, with gs_project and gs_project_bwd) and ``RasterizeSplats``
(Sec. 2.2: mu', Y, colours, opacities -> image, with gs_splats_from_2d, the sort and the
rasterizer; its backward gives dL/dmu' and dL/dY, Sec. 3.1). The 2D splats are ordinary
tensors between the two, so they can be inspected, hooked or modified. ``render_stages``
chains them.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
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
        r = pipeline.Rasterizer(cams, params, capacity=_capacity_hint.get(key), write_keys=False)
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


class ProjectGaussians(torch.autograd.Function):
    """(means, quats, scales) -> mu' [2, P], Y [3, P], plus depth [P] and valid [P] (not
    differentiable). P = sum over cameras of the scene size; a culled slot has valid 0. mu' and
    Y hold the projection's float32 values in float64 tensors, so that their gradients reach
    gs_project_bwd in float64 (dL/dSigma' = -Y dL/dY Y amplifies any rounding of dL/dY)."""

    @staticmethod
    def forward(ctx, means, quats, scales, colors, opacities, cams: pipeline.CameraSet, sizes: tuple,
                normalize_quats: bool = False):
        g = pipeline.GaussianSet.from_tensors(means.detach().contiguous(), quats.detach().contiguous(),
                                              scales.detach().contiguous(), colors.detach().contiguous(),
                                              opacities.detach().contiguous(), sizes, normalize_quats)
        r = pipeline.Rasterizer(cams, capacity=1024, keep_records=True)
        r.project(g)
        P = cams.n_splats
        rec = r.splats.rec[: P * 12].view(P, 12)
        mean2d = rec[:, 0:2].t().to(torch.float64).contiguous()
        conic = rec[:, 2:5].t().to(torch.float64).contiguous()
        depth = r.splats.depth[:P].clone()
        valid = (r.splats.tiles[:P] > 0).to(torch.int32)
        ctx.rasterizer, ctx.gaussians = r, g
        ctx.mark_non_differentiable(depth, valid)
        return mean2d, conic, depth, valid

    @staticmethod
    def backward(ctx, d_mean2d, d_conic, _d_depth, _d_valid):
        r, g = ctx.rasterizer, ctx.gaussians
        cams, P = r.cams, r.cams.n_splats
        dev = r.device
        dm = (d_mean2d if d_mean2d is not None else torch.zeros(2, P, device=dev)).to(torch.float64).contiguous()
        dc = (d_conic if d_conic is not None else torch.zeros(3, P, device=dev)).to(torch.float64).contiguous()
        out = {k: torch.zeros(rows, g.n, device=dev) for k, rows in (("means", 3), ("scales", 3), ("quats", 4))}
        stream = pipeline.current_stream()
        abi.gs_project_bwd(g.struct(), cams.ptr, cams.n_cams, r.splats.struct(P), P, dm.data_ptr(), dc.data_ptr(),
                           out["means"].data_ptr(), out["scales"].data_ptr(), out["quats"].data_ptr(), None, stream)
        ctx.rasterizer = ctx.gaussians = None
        return out["means"], out["quats"], out["scales"], None, None, None, None, None


class RasterizeSplats(torch.autograd.Function):
    """(mu' [2, P], Y [3, P], colours [3, N], opacities [N]; depth and valid per slot) ->
    packed image [3, n_pixels]. mu' and Y are rounded to float32 for the kernels; the backward
    returns dL/dmu' and dL/dY (computed in float64) in their dtype, and dL/dc, dL/do."""

    @staticmethod
    def forward(ctx, mean2d, conic, colors, opacities, depth, valid, cams: pipeline.CameraSet,
                params: abi.GsParams, sizes: tuple, box_lambda_max: bool = False):
        n = int(opacities.shape[-1])
        dummy = torch.zeros(4, n, device=colors.device)
        g = pipeline.GaussianSet.from_tensors(dummy[:3], dummy, dummy[:3], colors.detach().contiguous(),
                                              opacities.detach().contiguous(), sizes)
        g.box_lambda_max = bool(box_lambda_max)
        key = (cams.n_splats, cams.n_tiles, "2d")
        r = pipeline.Rasterizer(cams, params, capacity=_capacity_hint.get(key), write_keys=False)
        st = r.forward_2d(g, mean2d.detach().to(torch.float32).contiguous(),
                          conic.detach().to(torch.float32).contiguous(), depth.contiguous(), valid.contiguous())
        _capacity_hint[key] = max(r.capacity, int(st.K * 1.1) + 1024)
        ctx.state, ctx.rasterizer = st, r
        ctx.dtypes = (mean2d.dtype, conic.dtype)
        return st.image.clone()

    @staticmethod
    def backward(ctx, dL_dimage):
        gr = ctx.rasterizer.backward_2d(ctx.state, dL_dimage)
        P = ctx.rasterizer.cams.n_splats
        ctx.state = ctx.rasterizer = None
        return (gr["mean2d"][:, :P].to(ctx.dtypes[0]), gr["conic"][:, :P].to(ctx.dtypes[1]), gr["colors"],
                gr["opacities"], None, None, None, None, None, None)


def render_stages(means, quats, scales, colors, opacities, cameras: Sequence, scene_sizes=None,
                  params: abi.GsParams | None = None, normalize_quats: bool = False, splat_hook=None):
    """``render`` through the two stages; ``splat_hook(mean2d, conic)`` may return modified
    (mean2d, conic) tensors (differentiable) that the rasterizer then uses."""
    sizes = tuple(scene_sizes) if scene_sizes is not None else (int(opacities.shape[-1]),)
    cams = pipeline.CameraSet(cameras, sizes, device=means.device)
    params = params or pipeline.make_params()
    mean2d, conic, depth, valid = ProjectGaussians.apply(means, quats, scales, colors, opacities, cams, sizes,
                                                         normalize_quats)
    if splat_hook is not None:
        mean2d, conic = splat_hook(mean2d, conic)
    packed = RasterizeSplats.apply(mean2d, conic, colors, opacities, depth, valid, cams, params, sizes)
    return [cams.unpack(packed, k) for k in range(cams.n_cams)]


# ------------------------------------------------------------------ fused L2 training form

class _L2Step:
    """A fused TrainStep over fixed parameter, target and camera buffers, captured in a HIP
    graph, with the list length read back without blocking."""

    def __init__(self, g: pipeline.GaussianSet, cams: pipeline.CameraSet, targets: torch.Tensor,
                 params: abi.GsParams, capacity: int | None):
        self.g, self.cams, self.targets, self.params = g, cams, targets, params
        self.step = pipeline.TrainStep(g, cams, targets, params, capacity=capacity, mode="fused", keep_image=False)
        self.graph = pipeline.GraphStep(self.step)
        self.host_counters = torch.zeros(2, dtype=torch.int64, pin_memory=True)
        self.done = None

    def run(self):
        self.graph()
        self.host_counters.copy_(self.step.r.bins.counters, non_blocking=True)
        self.done = torch.cuda.Event()
        self.done.record()

    def previous_counts(self):
        """(K, flags) of the last completed replay, or None while it is still running."""
        if self.done is None or not self.done.query():
            return None
        return int(self.host_counters[0]), int(self.host_counters[1])


_l2_steps: dict = {}


def _camera_key(cameras) -> tuple:
    return tuple((np.asarray(c.R, dtype=np.float64).tobytes(), np.asarray(c.t, dtype=np.float64).tobytes(),
                  float(c.fx), float(c.fy), float(c.cx), float(c.cy), int(c.width), int(c.height), float(c.near),
                  float(c.far), int(getattr(c, "scene", 0))) for c in cameras)


class RasterizeL2Loss(torch.autograd.Function):
    """(means, quats, scales, colors, opacities) -> L = sum over cameras, pixels and channels of
    (C - target)^2, with the whole backward computed in the forward's fused launch."""

    @staticmethod
    def forward(ctx, means, quats, scales, colors, opacities, holder: _L2Step):
        holder.run()
        grads = holder.step.grads
        # copies: the step's buffers are rewritten by the next call, which may come before
        # this backward
        ctx.grads = tuple(grads[k].clone() for k in ("means", "quats", "scales", "colors", "opacities"))
        return grads["loss"].clone().view(())

    @staticmethod
    def backward(ctx, dL_out):
        out = tuple(g.mul_(dL_out) for g in ctx.grads)
        ctx.grads = None
        return out + (None,)


def l2_loss(means: torch.Tensor, quats: torch.Tensor, scales: torch.Tensor, colors: torch.Tensor,
            opacities: torch.Tensor, cameras: Sequence, targets: torch.Tensor,
            scene_sizes: Sequence[int] | None = None, params: abi.GsParams | None = None,
            normalize_quats: bool = False) -> torch.Tensor:
    """Differentiable L2 image loss over a batch of cameras: targets [3, n_pixels] packed in
    camera order (each camera's [3, H, W] target flattened and concatenated along pixels).

    The parameter and target tensors are used in place (not copied): the captured step keeps
    their addresses and is rebuilt when an address, a shape, a camera or the parameters
    change. An optimiser that updates the parameters in place keeps the cached step.
    A NaN loss means the step's tile list overflowed its capacity; the capacity is regrown
    and the next call is valid."""
    sizes = tuple(scene_sizes) if scene_sizes is not None else (int(opacities.shape[-1]),)
    params = params or pipeline.make_params()
    ts = (means, quats, scales, colors, opacities)
    for t in ts + (targets,):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError("l2_loss: parameters and targets must be contiguous float32 device tensors")
    key = (tuple(t.data_ptr() for t in ts), tuple(tuple(t.shape) for t in ts), targets.data_ptr(),
           tuple(targets.shape), sizes, _camera_key(cameras), bytes(params), bool(normalize_quats))
    holder = _l2_steps.get(key)
    if holder is not None:
        prev = holder.previous_counts()
        if prev is not None and (prev[1] & 1 or prev[0] * 1.1 > holder.step.r.capacity):
            # the last step overflowed, or came close: rebuild with room for its K
            holder = _L2Step(holder.g, holder.cams, targets, params, int(prev[0] * 1.25) + 1024)
            _l2_steps[key] = holder
        elif prev is not None and prev[1] & 2:
            pipeline.check_sort_flag(prev[1])
    if holder is None:
        if len(_l2_steps) >= 4:
            _l2_steps.pop(next(iter(_l2_steps)))
        g = pipeline.GaussianSet.from_tensors(*[t.detach() for t in ts], sizes, normalize_quats)
        cams = pipeline.CameraSet(cameras, sizes, device=means.device)
        holder = _L2Step(g, cams, targets, params, None)
        _l2_steps[key] = holder
    return RasterizeL2Loss.apply(means, quats, scales, colors, opacities, holder)
