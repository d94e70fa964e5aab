"""ctypes binding of libgsplat_mi355x.so: struct mirrors and one wrapper per C entry point.

The wrappers only marshal arguments (device pointers as integers, descriptor structs
by reference) and turn a non-zero gs_status into :class:`GsError`. Every step of the
rasterizer runs in the HIP library; there is no CPU fallback. If the library has not
been built, :func:`lib` raises, loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsplat_mi355x.so")

GS_OK, GS_ERR_INVALID, GS_ERR_CAPACITY, GS_ERR_HIP, GS_ERR_DEVICE = 0, -1, -2, -3, -4
REC_FLOATS = 12
RASTER_FLOATS = 16
TILE = 16

EXPORTED = (
    "gs_device_check", "gs_last_hip_error", "gs_last_error_message", "gs_version", "gs_zero", "gs_abi_layout",
    "gs_project", "gs_schedule_size", "gs_bin_and_sort_workspace_size", "gs_bin_and_sort", "gs_rasterize_fwd", "gs_rasterize_bwd",
    "gs_project_bwd", "gs_l2_grad", "gs_rasterize_fused_l2", "gs_graph_begin", "gs_graph_end", "gs_graph_launch",
    "gs_graph_destroy", "gs_set_tuning", "gs_get_tuning", "gs_splats_from_2d", "gs_bin_and_sort_static",
    "gs_set_sort_wait_limit", "gs_set_work_counter", "gs_zero_listed_slot_grads",
)

DEFAULT_SORT_WAIT_LIMIT = 1 << 20

# bytes of the library's static workspace of gs_bin_and_sort_static (GS_STATIC_WORKSPACE_BYTES)
STATIC_WORKSPACE_BYTES = 64 << 20


class GsError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str, hip: int):
        super().__init__(f"{fn} failed: status {code} ({msg}); hip error {hip}")
        self.code, self.hip = code, hip


# ------------------------------------------------------------------------ struct mirrors

CAMERA_DTYPE = np.dtype([
    ("R", "<f4", (9,)), ("t", "<f4", (3,)), ("fx", "<f4"), ("fy", "<f4"), ("cx", "<f4"), ("cy", "<f4"),
    ("width", "<i4"), ("height", "<i4"), ("near_plane", "<f4"), ("far_plane", "<f4"),
    ("gauss_offset", "<i8"), ("gauss_count", "<i8"), ("proj_offset", "<i8"), ("pixel_offset", "<i8"),
    ("tile_offset", "<i4"), ("tiles_x", "<i4"), ("tiles_y", "<i4"), ("reserved", "<i4"),
])
assert CAMERA_DTYPE.itemsize == 128


class GsGaussians(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("quats", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("colors", ctypes.c_void_p), ("opacities", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


GS_BINS_NO_KEYS = 1           # gs_bins.flags: the sort does not write the 64-bit keys
GS_NORMALIZE_QUATS = 1
GS_BOX_LAMBDA_MAX = 2


class GsSplats(ctypes.Structure):
    _fields_ = [("rec", ctypes.c_void_p), ("raster", ctypes.c_void_p), ("depth", ctypes.c_void_p),
                ("rect", ctypes.c_void_p), ("tiles_touched", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


class GsParams(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float), ("T_min", ctypes.c_float),
                ("background", ctypes.c_float * 3), ("reserved", ctypes.c_int32)]


class GsTuning(ctypes.Structure):
    _fields_ = [("split_len", ctypes.c_int32), ("split_parts", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("split_priority", ctypes.c_int32), ("generate_entries", ctypes.c_int32),
                ("item_grab", ctypes.c_int32), ("prio_len", ctypes.c_int32),
                ("bwd_segs", ctypes.c_int32), ("atomic_lanes", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("big_tiles", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class GsBins(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("ids", ctypes.c_void_p), ("ranges", ctypes.c_void_p),
                ("schedule", ctypes.c_void_p), ("counters", ctypes.c_void_p), ("capacity", ctypes.c_int64),
                ("n_tiles", ctypes.c_int32), ("flags", ctypes.c_int32)]


def expected_layout() -> list[int]:
    """The values gs_abi_layout must report for these mirrors."""
    f = CAMERA_DTYPE.fields
    return [CAMERA_DTYPE.itemsize, f["width"][1], f["near_plane"][1], f["gauss_offset"][1], f["pixel_offset"][1],
            f["tile_offset"][1], f["tiles_y"][1],
            ctypes.sizeof(GsGaussians), GsGaussians.n.offset,
            ctypes.sizeof(GsSplats), GsSplats.capacity.offset,
            ctypes.sizeof(GsParams), ctypes.sizeof(GsBins), GsBins.capacity.offset, GsBins.n_tiles.offset,
            ctypes.sizeof(GsTuning), GsTuning.bwd_segs.offset, GsTuning.atomic_lanes.offset, GsTuning.batch.offset,
            GsTuning.big_tiles.offset]


# --------------------------------------------------------------------------- loading

_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


def lib():
    """Loads the HIP library (built in-tree by paper_2312_02121_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_02121_amd.build` "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "gs_device_check": (ctypes.c_int, []),
        "gs_last_hip_error": (ctypes.c_int, []),
        "gs_last_error_message": (ctypes.c_char_p, []),
        "gs_version": (ctypes.c_int, []),
        "gs_zero": (ctypes.c_int, [_P, ctypes.c_size_t, _P]),
        "gs_abi_layout": (ctypes.c_int, [_P, ctypes.c_int]),
        "gs_project": (ctypes.c_int, [_P, _P, _I32, _I64, _P, _P]),
        "gs_splats_from_2d": (ctypes.c_int, [_P, _P, _I32, _I64, _P, _P, _P, _P, _P, _P]),
        "gs_bin_and_sort_workspace_size": (ctypes.c_size_t, [_I64, _I64, _I32]),
        "gs_schedule_size": (ctypes.c_int64, [_I32]),
        "gs_bin_and_sort": (ctypes.c_int, [_P, _I64, _P, _I32, _P, _P, ctypes.c_size_t, _P]),
        "gs_bin_and_sort_static": (ctypes.c_int, [_P, _I64, _P, _I32, _P, _P]),
        "gs_set_sort_wait_limit": (ctypes.c_int, [_I32]),
        "gs_set_work_counter": (ctypes.c_int, [_P]),
        "gs_zero_listed_slot_grads": (ctypes.c_int, [_P, _I64, _P, _P, _P]),
        "gs_rasterize_fwd": (ctypes.c_int, [_P, _P, _P, _I32, _P, _I64, _P, _P, _P, _P, _P]),
        "gs_rasterize_bwd": (ctypes.c_int, [_P, _I64, _P, _P, _I32, _P, _I64, _P, _P, _P, _P, _P, _I64, _P, _P, _P]),
        "gs_project_bwd": (ctypes.c_int, [_P, _P, _I32, _P, _I64, _P, _P, _P, _P, _P, _P, _P]),
        "gs_l2_grad": (ctypes.c_int, [_P, _P, _I64, _P, _P]),
        "gs_rasterize_fused_l2": (ctypes.c_int, [_P, _I64, _P, _P, _I32, _P, _I64, _P, _P, _P, _P, _P, _I64, _P, _P,
                                                 _P]),
        "gs_graph_begin": (ctypes.c_int, [_P]),
        "gs_graph_end": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_void_p)]),
        "gs_graph_launch": (ctypes.c_int, [_P, _P]),
        "gs_graph_destroy": (ctypes.c_int, [_P]),
        "gs_set_tuning": (ctypes.c_int, [_P]),
        "gs_get_tuning": (ctypes.c_int, [_P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(fn: str, rc: int):
    if rc != GS_OK:
        L = lib()
        raise GsError(fn, rc, L.gs_last_error_message().decode(), L.gs_last_hip_error())


def _ref(x):
    return ctypes.byref(x) if x is not None else None


# -------------------------------------------------------------------------- wrappers

def gs_device_check() -> int:
    return lib().gs_device_check()


def gs_abi_layout() -> list[int]:
    out = (ctypes.c_int64 * 64)()
    n = lib().gs_abi_layout(out, 64)
    return list(out[:n])


def gs_zero(ptr: int, nbytes: int, stream: int):
    _check("gs_zero", lib().gs_zero(ptr, nbytes, stream))


def gs_project(g: GsGaussians, cams_ptr: int, n_cams: int, n_splats: int, splats: GsSplats, stream: int):
    _check("gs_project", lib().gs_project(_ref(g), cams_ptr, n_cams, n_splats, _ref(splats), stream))


def gs_splats_from_2d(g: GsGaussians, cams_ptr: int, n_cams: int, n_splats: int, mean2d: int, conic: int,
                      depth: int, valid: int, splats: GsSplats, stream: int):
    _check("gs_splats_from_2d", lib().gs_splats_from_2d(_ref(g), cams_ptr, n_cams, n_splats, mean2d, conic, depth,
                                                        valid, _ref(splats), stream))


def gs_schedule_size(n_tiles: int) -> int:
    return int(lib().gs_schedule_size(n_tiles))


def gs_bin_and_sort_workspace_size(n_splats: int, capacity: int, n_tiles: int) -> int:
    return int(lib().gs_bin_and_sort_workspace_size(n_splats, capacity, n_tiles))


def gs_bin_and_sort(splats: GsSplats, n_splats: int, cams_ptr: int, n_cams: int, bins: GsBins, ws_ptr: int,
                    ws_bytes: int, stream: int):
    _check("gs_bin_and_sort", lib().gs_bin_and_sort(_ref(splats), n_splats, cams_ptr, n_cams, _ref(bins), ws_ptr,
                                                    ws_bytes, stream))


def gs_set_sort_wait_limit(polls: int):
    _check("gs_set_sort_wait_limit", lib().gs_set_sort_wait_limit(polls))


def gs_zero_listed_slot_grads(splats: GsSplats, n_splats: int, dmean2d: int, dconic: int, stream: int):
    _check("gs_zero_listed_slot_grads", lib().gs_zero_listed_slot_grads(_ref(splats), n_splats, dmean2d, dconic,
                                                                        stream))


def gs_set_work_counter(ptr: int | None):
    _check("gs_set_work_counter", lib().gs_set_work_counter(ptr))


def gs_bin_and_sort_static(splats: GsSplats, n_splats: int, cams_ptr: int, n_cams: int, bins: GsBins, stream: int):
    _check("gs_bin_and_sort_static", lib().gs_bin_and_sort_static(_ref(splats), n_splats, cams_ptr, n_cams,
                                                                  _ref(bins), stream))


def gs_rasterize_fwd(splats: GsSplats, bins: GsBins, cams_ptr: int, n_cams: int, prm: GsParams, n_pixels: int,
                     image: int, T_final: int, last: int, visited: int | None, stream: int):
    _check("gs_rasterize_fwd", lib().gs_rasterize_fwd(_ref(splats), _ref(bins), cams_ptr, n_cams, _ref(prm), n_pixels,
                                                      image, T_final, last, visited, stream))


def gs_rasterize_bwd(splats: GsSplats, n_splats: int, bins: GsBins, cams_ptr: int, n_cams: int, prm: GsParams,
                     n_pixels: int, dL_dimage: int, T_final: int, last: int, d_mean2d: int, d_conic: int,
                     n_gaussians: int, d_colors: int, d_opac: int, stream: int):
    _check("gs_rasterize_bwd", lib().gs_rasterize_bwd(_ref(splats), n_splats, _ref(bins), cams_ptr, n_cams, _ref(prm),
                                                      n_pixels, dL_dimage, T_final, last, d_mean2d, d_conic,
                                                      n_gaussians, d_colors, d_opac, stream))


def gs_project_bwd(g: GsGaussians, cams_ptr: int, n_cams: int, splats: GsSplats, n_splats: int, d_mean2d: int,
                   d_conic: int, d_means: int, d_scales: int, d_quats: int, d_campose: int | None, stream: int):
    _check("gs_project_bwd", lib().gs_project_bwd(_ref(g), cams_ptr, n_cams, _ref(splats), n_splats, d_mean2d, d_conic,
                                                  d_means, d_scales, d_quats, d_campose, stream))


def gs_l2_grad(image: int, target: int, n: int, dL_dimage: int, stream: int):
    _check("gs_l2_grad", lib().gs_l2_grad(image, target, n, dL_dimage, stream))


def gs_rasterize_fused_l2(splats: GsSplats, n_splats: int, bins: GsBins, cams_ptr: int, n_cams: int, prm: GsParams,
                          n_pixels: int, target: int, image: int | None, loss: int | None, d_mean2d: int, d_conic: int,
                          n_gaussians: int, d_colors: int, d_opac: int, stream: int):
    _check("gs_rasterize_fused_l2", lib().gs_rasterize_fused_l2(_ref(splats), n_splats, _ref(bins), cams_ptr, n_cams,
                                                                _ref(prm), n_pixels, target, image, loss, d_mean2d,
                                                                d_conic, n_gaussians, d_colors, d_opac, stream))


def gs_graph_begin(stream: int):
    _check("gs_graph_begin", lib().gs_graph_begin(stream))


def gs_graph_end(stream: int) -> int:
    out = ctypes.c_void_p()
    _check("gs_graph_end", lib().gs_graph_end(stream, ctypes.byref(out)))
    return out.value


def gs_graph_launch(graph: int, stream: int):
    _check("gs_graph_launch", lib().gs_graph_launch(graph, stream))


def gs_graph_destroy(graph: int):
    _check("gs_graph_destroy", lib().gs_graph_destroy(graph))


def gs_set_tuning(t: GsTuning):
    _check("gs_set_tuning", lib().gs_set_tuning(ctypes.byref(t)))


def gs_get_tuning() -> GsTuning:
    t = GsTuning()
    _check("gs_get_tuning", lib().gs_get_tuning(ctypes.byref(t)))
    return t
