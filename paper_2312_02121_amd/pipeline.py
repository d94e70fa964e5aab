"""Host-side orchestration of the five C-ABI calls.

PyTorch supplies device memory and the stream; every computation runs in the HIP
library. The classes here pack cameras into the device ``gs_camera`` array, hold the
Gaussian planes, size the intermediate buffers, and call

    gs_project -> gs_bin_and_sort -> gs_rasterize_fwd            (forward)
    gs_rasterize_bwd -> gs_project_bwd                          (backward)

The tile-intersection count K is only known on the device. The forward passes a
capacity; if gs_bin_and_sort reports overflow (its device flag), the buffers are
regrown to K and binning is redone. A fixed-capacity caller (a captured graph) reads
the flag after the fact instead.
"""
from __future__ import annotations

import ctypes

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

from . import abi

STANDARD_PARAMS = dict(alpha_min=1.0 / 255.0, alpha_max=0.99, T_min=1e-4)


def make_params(alpha_min: float = STANDARD_PARAMS["alpha_min"], alpha_max: float = STANDARD_PARAMS["alpha_max"],
                T_min: float = STANDARD_PARAMS["T_min"], background=(0.0, 0.0, 0.0)) -> abi.GsParams:
    """Compositing parameters: the thresholds (standard mode by default; literal mode is
    alpha_min = 0, alpha_max = 1, T_min = 0, the image formation of eq. 7 as printed) and
    the RGB background seen through T_final (zero: the paper's image formation)."""
    bg = (ctypes.c_float * 3)(*[float(np.float32(x)) for x in background])
    return abi.GsParams(float(np.float32(alpha_min)), float(np.float32(alpha_max)), float(np.float32(T_min)), bg, 0)


def check_sort_flag(flag: int):
    """gs_bin_and_sort sets bit 2 of counters[1] when a look-back wait of its sort gave up (or
    its counts disagree), bit 4 for a camera wider than 8192 tiles."""
    if flag & 2:
        raise RuntimeError("gs_bin_and_sort: the single-pass sort's look-back did not complete; the list is invalid")
    if flag & 4:
        raise RuntimeError("gs_bin_and_sort: a camera is wider than 8192 tiles (131072 pixels); nothing was listed")


def current_stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


class CameraSet:
    """A batch of cameras, each viewing one scene, packed into the device gs_camera array.

    ``cameras`` are objects with R, t, fx, fy, cx, cy, width, height, near, far and
    ``scene`` (index into ``scene_sizes``, the Gaussian count of each scene).
    """

    def __init__(self, cameras: Sequence, scene_sizes: Sequence[int], device="cuda"):
        n = len(cameras)
        if n < 1:
            raise ValueError("need at least one camera")
        scene_off = np.concatenate([[0], np.cumsum(np.asarray(scene_sizes, dtype=np.int64))])
        arr = np.zeros(n, dtype=abi.CAMERA_DTYPE)
        proj = pix = tile = 0
        for k, c in enumerate(cameras):
            s = int(getattr(c, "scene", 0))
            W, H = int(c.width), int(c.height)
            if W < 1 or H < 1:
                raise ValueError("camera size must be positive")
            arr[k]["R"] = np.asarray(c.R, dtype=np.float32).reshape(9)
            arr[k]["t"] = np.asarray(c.t, dtype=np.float32).reshape(3)
            arr[k]["fx"], arr[k]["fy"], arr[k]["cx"], arr[k]["cy"] = c.fx, c.fy, c.cx, c.cy
            arr[k]["width"], arr[k]["height"] = W, H
            arr[k]["near_plane"], arr[k]["far_plane"] = c.near, c.far
            arr[k]["gauss_offset"] = scene_off[s]
            arr[k]["gauss_count"] = scene_sizes[s]
            arr[k]["proj_offset"] = proj
            arr[k]["pixel_offset"] = pix
            arr[k]["tile_offset"] = tile
            tx, ty = (W + 15) // 16, (H + 15) // 16
            arr[k]["tiles_x"], arr[k]["tiles_y"] = tx, ty
            proj += int(scene_sizes[s])
            pix += W * H
            tile += tx * ty
        if tile > 0x7FFFFFFF:
            raise ValueError("too many tiles for 32-bit tile ids")
        self.cameras = list(cameras)
        self.host = arr
        self.n_cams = n
        self.n_splats = proj
        self.n_pixels = pix
        self.n_tiles = tile
        self.device = torch.device(device)
        self.dev = torch.from_numpy(arr.view(np.uint8).copy()).to(self.device)

    @property
    def ptr(self) -> int:
        return self.dev.data_ptr()

    def image_slice(self, k: int):
        """(pixel_offset, height, width) of camera k inside the packed image planes."""
        c = self.host[k]
        return int(c["pixel_offset"]), int(c["height"]), int(c["width"])

    def unpack(self, planes: torch.Tensor, k: int) -> torch.Tensor:
        """[C, n_pixels] packed planes -> [C, H, W] view of camera k."""
        off, H, W = self.image_slice(k)
        return planes[:, off:off + H * W].view(planes.shape[0], H, W)


class GaussianSet:
    """Concatenated Gaussian planes of one or more scenes, float32 on the device."""

    KEYS = ("means", "quats", "scales", "colors", "opacities")

    def __init__(self, scenes: Sequence[dict] | dict, device="cuda", requires_grad: bool = False,
                 normalize_quats: bool = False, box_lambda_max: bool = False):
        if isinstance(scenes, dict):
            scenes = [scenes]
        # normalize_quats: the projection uses q / |q| and its backward differentiates through it;
        # box_lambda_max: square 3-sigma boxes from the largest eigenvalue of Sigma'
        self.normalize_quats = bool(normalize_quats)
        self.box_lambda_max = bool(box_lambda_max)
        self.sizes = [int(s["opacities"].shape[-1]) for s in scenes]
        self.n = sum(self.sizes)
        self.t = {}
        for k in self.KEYS:
            parts = [torch.as_tensor(np.asarray(s[k]), dtype=torch.float32) for s in scenes]
            self.t[k] = torch.cat(parts, dim=-1).contiguous().to(device).requires_grad_(requires_grad)

    @staticmethod
    def from_tensors(means, quats, scales, colors, opacities, sizes=None, normalize_quats: bool = False) -> "GaussianSet":
        obj = GaussianSet.__new__(GaussianSet)
        obj.normalize_quats = bool(normalize_quats)
        obj.box_lambda_max = False
        obj.t = {"means": means, "quats": quats, "scales": scales, "colors": colors, "opacities": opacities}
        obj.n = int(opacities.shape[-1])
        obj.sizes = list(sizes) if sizes is not None else [obj.n]
        return obj

    def struct(self) -> abi.GsGaussians:
        t = self.t
        for k in self.KEYS:
            if not (t[k].is_contiguous() and t[k].dtype == torch.float32 and t[k].is_cuda):
                raise ValueError(f"{k} must be a contiguous float32 device tensor")
        return abi.GsGaussians(_ptr(t["means"]), _ptr(t["quats"]), _ptr(t["scales"]), _ptr(t["colors"]),
                               _ptr(t["opacities"]), self.n,
                               (abi.GS_NORMALIZE_QUATS if self.normalize_quats else 0) |
                               (abi.GS_BOX_LAMBDA_MAX if getattr(self, "box_lambda_max", False) else 0))


@dataclass
class Splats:
    rec: torch.Tensor | None
    raster: torch.Tensor
    depth: torch.Tensor
    rect: torch.Tensor
    tiles: torch.Tensor

    @staticmethod
    def alloc(P: int, device, records: bool = False) -> "Splats":
        """records: also keep gs_project's 12-float records (an optional output that no later
        step reads; tests compare it with the oracle's projection)."""
        P1 = max(P, 1)
        return Splats(torch.empty(P1 * abi.REC_FLOATS, dtype=torch.float32, device=device) if records else None,
                      torch.empty(P1 * abi.RASTER_FLOATS, dtype=torch.float32, device=device),
                      torch.empty(P1, dtype=torch.float32, device=device),
                      torch.empty(P1 * 4, dtype=torch.int32, device=device),
                      torch.empty(P1, dtype=torch.int32, device=device))

    def struct(self, P: int) -> abi.GsSplats:
        return abi.GsSplats(_ptr(self.rec), _ptr(self.raster), _ptr(self.depth), _ptr(self.rect), _ptr(self.tiles),
                            P)


@dataclass
class Bins:
    keys: torch.Tensor
    ids: torch.Tensor
    ranges: torch.Tensor
    schedule: torch.Tensor
    counters: torch.Tensor
    workspace: torch.Tensor
    capacity: int
    n_tiles: int

    @staticmethod
    def alloc(P: int, capacity: int, n_tiles: int, device) -> "Bins":
        capacity = int(min(max(capacity, 1), 0x7FFFFFFF))
        ws = abi.gs_bin_and_sort_workspace_size(P, capacity, n_tiles)
        return Bins(torch.empty(capacity, dtype=torch.int64, device=device),
                    torch.empty(capacity, dtype=torch.int32, device=device),
                    torch.empty(2 * max(n_tiles, 1), dtype=torch.int32, device=device),
                    torch.zeros(abi.gs_schedule_size(n_tiles), dtype=torch.int32, device=device),
                    torch.zeros(2, dtype=torch.int64, device=device),
                    torch.empty(max(ws, 1), dtype=torch.uint8, device=device), capacity, n_tiles)

    def struct(self, flags: int = 0) -> abi.GsBins:
        return abi.GsBins(_ptr(self.keys), _ptr(self.ids), _ptr(self.ranges), _ptr(self.schedule),
                          _ptr(self.counters), self.capacity, self.n_tiles, flags)


@dataclass
class ForwardState:
    gaussians: GaussianSet
    cams: CameraSet
    params: abi.GsParams
    splats: Splats
    bins: Bins
    image: torch.Tensor        # [3, n_pixels]
    T_final: torch.Tensor      # [n_pixels]
    last: torch.Tensor         # [n_pixels] int32
    visited: Optional[torch.Tensor] = None
    K: int = -1
    extra: dict = field(default_factory=dict)


class Rasterizer:
    """Reusable buffers for one (GaussianSet layout, CameraSet) pair."""

    def __init__(self, cams: CameraSet, params: abi.GsParams | None = None, capacity: int | None = None,
                 keep_visited: bool = False, keep_records: bool = False, write_keys: bool = True):
        self.cams = cams
        # the sorted 64-bit keys are written only on request: the rasterizer reads ids and ranges
        self.write_keys = write_keys
        self.params = params or make_params()
        self.device = cams.device
        P = cams.n_splats
        self.splats = Splats.alloc(P, self.device, keep_records)
        self.capacity = int(capacity) if capacity else max(4 * P, 1024)
        self.bins = Bins.alloc(P, self.capacity, cams.n_tiles, self.device)
        npx = cams.n_pixels
        self.image = torch.empty(3, npx, dtype=torch.float32, device=self.device)
        self.T_final = torch.empty(npx, dtype=torch.float32, device=self.device)
        self.last = torch.empty(npx, dtype=torch.int32, device=self.device)
        self.visited = torch.empty(npx, dtype=torch.int32, device=self.device) if keep_visited else None

    # ---------------------------------------------------------------- forward pieces
    def project(self, g: GaussianSet, stream: int | None = None):
        stream = current_stream() if stream is None else stream
        P = self.cams.n_splats
        abi.gs_project(g.struct(), self.cams.ptr, self.cams.n_cams, P, self.splats.struct(P), stream)

    def bin_and_sort(self, stream: int | None = None):
        stream = current_stream() if stream is None else stream
        P = self.cams.n_splats
        b = self.bins
        abi.gs_bin_and_sort(self.splats.struct(P), P, self.cams.ptr, self.cams.n_cams,
                            b.struct(0 if self.write_keys else abi.GS_BINS_NO_KEYS),
                            _ptr(b.workspace), b.workspace.numel(), stream)

    def rasterize_fwd(self, stream: int | None = None):
        stream = current_stream() if stream is None else stream
        P = self.cams.n_splats
        abi.gs_rasterize_fwd(self.splats.struct(P), self.bins.struct(), self.cams.ptr, self.cams.n_cams,
                             self.params, self.cams.n_pixels, _ptr(self.image), _ptr(self.T_final), _ptr(self.last),
                             _ptr(self.visited), stream)

    def read_count(self) -> tuple[int, bool]:
        """(K, overflowed). Raises if the sort reported an internal failure (flag bit 2)."""
        c = self.bins.counters.cpu()
        check_sort_flag(int(c[1]))
        return int(c[0]), bool(int(c[1]) & 1)

    def forward(self, g: GaussianSet, check_overflow: bool = True) -> ForwardState:
        self.project(g)
        self.bin_and_sort()
        K = -1
        if check_overflow:
            K, over = self.read_count()
            if over:
                self.capacity = int(K * 1.25) + 1024
                self.bins = Bins.alloc(self.cams.n_splats, self.capacity, self.cams.n_tiles, self.device)
                self.bin_and_sort()
                K, over = self.read_count()
                assert not over
        self.rasterize_fwd()
        return ForwardState(g, self.cams, self.params, self.splats, self.bins, self.image, self.T_final,
                            self.last, self.visited, K)

    def forward_2d(self, g: GaussianSet, mean2d: torch.Tensor, conic: torch.Tensor, depth: torch.Tensor,
                   valid: torch.Tensor) -> ForwardState:
        """Per-stage forward: splats from given mu' [2, P], Y [3, P], depth [P] and valid [P]
        (gs_splats_from_2d) instead of the projection, then bin, sort and rasterize."""
        P = self.cams.n_splats
        for name, t, shape, dt in (("mean2d", mean2d, (2, P), torch.float32), ("conic", conic, (3, P), torch.float32),
                                   ("depth", depth, (P,), torch.float32), ("valid", valid, (P,), torch.int32)):
            if tuple(t.shape) != shape or t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous {dt} device tensor of shape {shape}")
        abi.gs_splats_from_2d(g.struct(), self.cams.ptr, self.cams.n_cams, P, _ptr(mean2d), _ptr(conic), _ptr(depth),
                              _ptr(valid), self.splats.struct(P), current_stream())
        self.bin_and_sort()
        K, over = self.read_count()
        if over:
            self.capacity = int(K * 1.25) + 1024
            self.bins = Bins.alloc(P, self.capacity, self.cams.n_tiles, self.device)
            self.bin_and_sort()
            K, over = self.read_count()
            assert not over
        self.rasterize_fwd()
        return ForwardState(g, self.cams, self.params, self.splats, self.bins, self.image, self.T_final,
                            self.last, self.visited, K)

    def backward_2d(self, state: ForwardState, dL_dimage: torch.Tensor, stream: int | None = None) -> dict:
        """Rasterizer backward only: dL/dmu' [2, P] and dL/dY [3, P] (float64) per slot,
        dL/dc and dL/do per scene Gaussian."""
        stream = current_stream() if stream is None else stream
        g, cams, P = state.gaussians, self.cams, self.cams.n_splats
        dev = self.device
        dL_dimage = dL_dimage.contiguous().to(torch.float32)
        grads = {"mean2d": torch.zeros(2, max(P, 1), dtype=torch.float64, device=dev),
                 "conic": torch.zeros(3, max(P, 1), dtype=torch.float64, device=dev),
                 "colors": torch.zeros(3, g.n, device=dev), "opacities": torch.zeros(g.n, device=dev)}
        abi.gs_rasterize_bwd(state.splats.struct(P), P, state.bins.struct(), cams.ptr, cams.n_cams, state.params,
                             cams.n_pixels, _ptr(dL_dimage), _ptr(state.T_final), _ptr(state.last),
                             _ptr(grads["mean2d"]), _ptr(grads["conic"]), g.n, _ptr(grads["colors"]),
                             _ptr(grads["opacities"]), stream)
        return grads

    # ---------------------------------------------------------------------- backward
    def backward(self, state: ForwardState, dL_dimage: torch.Tensor, with_pose: bool = False,
                 stream: int | None = None) -> dict:
        stream = current_stream() if stream is None else stream
        g, cams, P = state.gaussians, self.cams, self.cams.n_splats
        dev = self.device
        dL_dimage = dL_dimage.contiguous().to(torch.float32)
        grads = {
            "mean2d": torch.empty(2, max(P, 1), dtype=torch.float64, device=dev),
            "conic": torch.empty(3, max(P, 1), dtype=torch.float64, device=dev),
            "colors": torch.empty(3, g.n, device=dev), "opacities": torch.empty(g.n, device=dev),
            "means": torch.empty(3, g.n, device=dev), "scales": torch.empty(3, g.n, device=dev),
            "quats": torch.empty(4, g.n, device=dev),
        }
        if with_pose:
            grads["campose"] = torch.empty(cams.n_cams, 12, device=dev)
        for t in grads.values():
            abi.gs_zero(t.data_ptr(), t.numel() * t.element_size(), stream)
        sp = state.splats.struct(P)
        abi.gs_rasterize_bwd(sp, P, state.bins.struct(), cams.ptr, cams.n_cams, state.params, cams.n_pixels,
                             _ptr(dL_dimage), _ptr(state.T_final), _ptr(state.last), _ptr(grads["mean2d"]),
                             _ptr(grads["conic"]), g.n, _ptr(grads["colors"]), _ptr(grads["opacities"]), stream)
        abi.gs_project_bwd(g.struct(), cams.ptr, cams.n_cams, sp, P, _ptr(grads["mean2d"]), _ptr(grads["conic"]),
                           _ptr(grads["means"]), _ptr(grads["scales"]), _ptr(grads["quats"]),
                           _ptr(grads.get("campose")), stream)
        return grads


class TrainStep:
    """One step of fwd + L2 loss gradient + bwd over a fixed camera set, with every
    buffer preallocated, so the step allocates nothing and can be timed or captured.

    mode "separate": project, bin_and_sort, rasterize_fwd, l2_grad, zero, rasterize_bwd,
                     project_bwd (the image, T and last round-trip through HBM)
    mode "fused":    project, bin_and_sort, zero, fused (fwd + L2 + bwd per work item),
                     project_bwd
    """

    STAGE_SETS = {
        "separate": ("project", "bin_and_sort", "rasterize_fwd", "l2_grad", "zero_grads", "rasterize_bwd",
                     "project_bwd"),
        "fused": ("project", "bin_and_sort", "zero_grads", "fused", "project_bwd"),
    }

    def __init__(self, g: GaussianSet, cams: CameraSet, targets: torch.Tensor, params: abi.GsParams | None = None,
                 capacity: int | None = None, capacity_margin: float = 1.25, mode: str = "separate",
                 keep_image: bool = True, scene_grads: "TrainStep | None" = None, keep_records: bool = False,
                 keep_keys: bool = False):
        self.g, self.cams, self.mode = g, cams, mode
        self.STAGES = self.STAGE_SETS[mode]
        self.r = Rasterizer(cams, params, capacity=capacity, keep_visited=True, keep_records=keep_records,
                            write_keys=keep_keys)
        self.targets = targets.contiguous().view(3, -1).to(torch.float32)
        assert self.targets.shape[1] == cams.n_pixels
        st = self.r.forward(g)                      # sizes the list capacity
        if capacity is None and st.K * capacity_margin > self.r.capacity:
            self.r.capacity = int(st.K * capacity_margin) + 1024
            self.r.bins = Bins.alloc(cams.n_splats, self.r.capacity, cams.n_tiles, cams.device)
            st = self.r.forward(g)
        self.K = st.K
        torch.cuda.synchronize()
        self.E_fwd = int(self.r.visited.sum())     # pairs whose alpha the forward evaluates
        self.E_bwd = int(self.r.last.sum())        # pairs the backward walks
        self.r.visited = None                      # the timed step does not write it
        P, n = cams.n_splats, g.n
        # per-slot gradients (this camera set only) and per-scene gradients, which another
        # step may own: then this step accumulates into them and does not zero them
        P1 = max(P, 1)
        slot = {"mean2d": (2, P1), "conic": (3, P1)}
        scene = {"colors": (3, n), "opacities": (n,), "means": (3, n), "scales": (3, n), "quats": (4, n),
                 "loss": (1,)}
        numel = lambda sh: int(np.prod(sh))
        n_slot = sum(numel(v) for v in slot.values())
        n_scene = sum(numel(v) for v in scene.values())
        self.owns_scene_grads = scene_grads is None
        # one allocation for both parts when this step owns the scene gradients, so that a
        # single fill zeroes them
        slot_bytes = n_slot * 8
        scene_at = (slot_bytes + 255) // 256 * 256
        total = scene_at + n_scene * 4 if self.owns_scene_grads else slot_bytes
        self.grad_bytes = torch.empty(total, dtype=torch.uint8, device=cams.device)
        self.slot_flat = self.grad_bytes[:slot_bytes].view(torch.float64)
        self.grads, o = {}, 0
        for k, sh in slot.items():
            self.grads[k] = self.slot_flat[o:o + numel(sh)].view(sh)
            o += numel(sh)
        if scene_grads is None:
            self.scene_flat = self.grad_bytes[scene_at:].view(torch.float32)
            o = 0
            for k, sh in scene.items():
                self.grads[k] = self.scene_flat[o:o + numel(sh)].view(sh)
                o += numel(sh)
        else:
            self.scene_flat = scene_grads.scene_flat
            for k in scene:
                self.grads[k] = scene_grads.grads[k]
        self.dL = torch.empty(3, cams.n_pixels, dtype=torch.float32, device=cams.device)
        self.keep_image = keep_image

    @property
    def loss(self) -> torch.Tensor:
        return self.grads["loss"]

    def run_stage(self, name: str, stream: int):
        r, cams, g, P = self.r, self.cams, self.g, self.cams.n_splats
        gr = self.grads
        if name == "project":
            r.project(g, stream)
        elif name == "bin_and_sort":
            r.bin_and_sort(stream)
        elif name == "rasterize_fwd":
            r.rasterize_fwd(stream)
        elif name == "l2_grad":
            abi.gs_l2_grad(r.image.data_ptr(), self.targets.data_ptr(), r.image.numel(), self.dL.data_ptr(), stream)
        elif name == "zero_grads":
            # every slot's gradients, with the scene gradients in the same fill when this step
            # owns them (one allocation). Clearing only the listed slots writes as many lines
            # where most 128-byte lines hold a listed slot, and its scattered partial-line
            # writes are slower when the views see most of their scene.
            if self.owns_scene_grads:
                abi.gs_zero(self.grad_bytes.data_ptr(), self.grad_bytes.numel(), stream)
            else:
                abi.gs_zero(self.slot_flat.data_ptr(), self.slot_flat.numel() * 8, stream)
        elif name == "rasterize_bwd":
            abi.gs_rasterize_bwd(r.splats.struct(P), P, r.bins.struct(), cams.ptr, cams.n_cams, r.params,
                                 cams.n_pixels, self.dL.data_ptr(), r.T_final.data_ptr(), r.last.data_ptr(),
                                 gr["mean2d"].data_ptr(), gr["conic"].data_ptr(), g.n, gr["colors"].data_ptr(),
                                 gr["opacities"].data_ptr(), stream)
        elif name == "fused":
            abi.gs_rasterize_fused_l2(r.splats.struct(P), P, r.bins.struct(), cams.ptr, cams.n_cams, r.params,
                                      cams.n_pixels, self.targets.data_ptr(),
                                      r.image.data_ptr() if self.keep_image else None, gr["loss"].data_ptr(),
                                      gr["mean2d"].data_ptr(), gr["conic"].data_ptr(), g.n,
                                      gr["colors"].data_ptr(), gr["opacities"].data_ptr(), stream)
        elif name == "project_bwd":
            abi.gs_project_bwd(g.struct(), cams.ptr, cams.n_cams, r.splats.struct(P), P, gr["mean2d"].data_ptr(),
                               gr["conic"].data_ptr(), gr["means"].data_ptr(), gr["scales"].data_ptr(),
                               gr["quats"].data_ptr(), None, stream)
        else:
            raise KeyError(name)

    def __call__(self, stream: int | None = None, events: list | None = None):
        stream = current_stream() if stream is None else stream
        for i, name in enumerate(self.STAGES):
            if events is not None:
                events[i].record()
            self.run_stage(name, stream)
        if events is not None:
            events[len(self.STAGES)].record()

    def overflowed(self) -> bool:
        flag = int(self.r.bins.counters[1].item())
        check_sort_flag(flag)
        return bool(flag & 1)


class GraphStep:
    """A TrainStep captured once into a HIP graph (gs_graph_* of the C ABI) and replayed.

    Capture runs on a private stream of default priority; replays go to the caller's
    stream. Buffers named by the graph belong to the wrapped TrainStep and stay alive with it.
    """

    def __init__(self, step: TrainStep):
        self.step = step
        self.stream = torch.cuda.Stream()
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        with torch.cuda.stream(self.stream):
            step(stream=self.stream.cuda_stream)          # warm the path outside capture
            self.stream.synchronize()
            abi.gs_graph_begin(self.stream.cuda_stream)
            try:
                step(stream=self.stream.cuda_stream)
            finally:
                self.graph = abi.gs_graph_end(self.stream.cuda_stream)
        cur.wait_stream(self.stream)

    def __call__(self, stream: int | None = None):
        abi.gs_graph_launch(self.graph, current_stream() if stream is None else stream)

    def __del__(self):
        g = getattr(self, "graph", None)
        if g:
            try:
                abi.gs_graph_destroy(g)
            except Exception:
                pass
            self.graph = None


class PerViewSteps:
    """The same step run one camera at a time (one CameraSet per view), no graph: the
    one-view-per-launch baseline for the batched form."""

    def __init__(self, g: GaussianSet, cameras: Sequence, targets: Sequence[torch.Tensor],
                 params: abi.GsParams | None = None, mode: str = "separate"):
        self.steps = []
        for c, t in zip(cameras, targets):
            cs = CameraSet([c], g.sizes)
            first = self.steps[0] if self.steps else None
            self.steps.append(TrainStep(g, cs, t, params, mode=mode, scene_grads=first))
        self.E_fwd = sum(s.E_fwd for s in self.steps)
        self.E_bwd = sum(s.E_bwd for s in self.steps)
        self.K = sum(s.K for s in self.steps)
        self.grads = self.steps[0].grads

    def __call__(self, stream: int | None = None):
        for s in self.steps:
            s(stream)

    def overflowed(self) -> bool:
        return any(s.overflowed() for s in self.steps)
