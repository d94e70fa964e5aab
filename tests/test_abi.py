"""The C-ABI library loads, exports every symbol the header declares, and the Python
struct mirrors match the C layout. No device is touched."""
import os
import re

import pytest

from paper_2312_02121_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsplat_mi355x.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|size_t|const char \*)\s*\*?\s*(gs_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(abi.LIB_PATH):
        from paper_2312_02121_amd import build
        build.build()
    return abi.lib()


def test_header_declares_the_five_steps():
    names = declared_functions()
    for fn in ("gs_project", "gs_bin_and_sort", "gs_rasterize_fwd", "gs_rasterize_bwd", "gs_project_bwd"):
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for fn in names:
        assert hasattr(lib, fn), fn
    assert set(abi.EXPORTED) <= set(names)


def test_struct_mirrors_match_c_layout(lib):
    assert abi.gs_abi_layout() == abi.expected_layout()


def test_workspace_size_is_host_only(lib):
    a = abi.gs_bin_and_sort_workspace_size(1000, 4000, 16)
    b = abi.gs_bin_and_sort_workspace_size(1000, 8000, 16)
    assert 0 < a < b
    assert abi.gs_bin_and_sort_workspace_size(-1, 10, 1) == 0


def test_invalid_arguments_are_rejected_without_a_device(lib):
    # null descriptors fail validation before any HIP call
    assert lib.gs_project(None, None, 1, 10, None, None) == abi.GS_ERR_INVALID
    assert b"gs_project" in lib.gs_last_error_message()
    assert lib.gs_bin_and_sort(None, 0, None, 1, None, None, 0, None) == abi.GS_ERR_INVALID
    assert lib.gs_bin_and_sort_static(None, 0, None, 1, None, None) == abi.GS_ERR_INVALID
    assert lib.gs_rasterize_fwd(None, None, None, 1, None, 0, None, None, None, None, None) == abi.GS_ERR_INVALID
    prm = abi.GsParams(0.0, 1.5, 0.0)          # alpha_max above 1: no valid compositing
    sp = abi.GsSplats(rec=64, raster=64, depth=64, rect=64, tiles_touched=64, capacity=10)
    bins = abi.GsBins(keys=64, ids=64, ranges=64, schedule=64, counters=64, capacity=10, n_tiles=1)
    rc = lib.gs_rasterize_bwd(abi._ref(sp), 10, abi._ref(bins), 16, 1, abi._ref(prm), 4, 16, 16, 16, 16, 16, 10, 16,
                              16, None)
    assert rc == abi.GS_ERR_INVALID
    assert b"alpha_max" in lib.gs_last_error_message()
    # a workspace that is large enough but not 256-byte aligned
    ws = abi.gs_bin_and_sort_workspace_size(10, 10, 1)
    rc = lib.gs_bin_and_sort(abi._ref(sp), 10, 64, 1, abi._ref(bins), 4096 + 8, ws, None)
    assert rc == abi.GS_ERR_INVALID
    assert b"aligned" in lib.gs_last_error_message()
    # flag bits other than GS_BINS_NO_KEYS
    bad = abi.GsBins(keys=64, ids=64, ranges=64, schedule=64, counters=64, capacity=10, n_tiles=1, flags=2)
    rc = lib.gs_bin_and_sort(abi._ref(sp), 10, 64, 1, abi._ref(bad), 4096, ws, None)
    assert rc == abi.GS_ERR_INVALID
    assert b"flags" in lib.gs_last_error_message()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(abi, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(abi, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        abi.lib()


def test_tuning_is_validated_and_round_trips(lib):
    before = abi.gs_get_tuning().as_dict()
    assert before == {"split_len": 256, "split_parts": 4, "waves_per_cu": 32, "split_priority": 1, "generate_entries": 0,
                      "item_grab": 1, "prio_len": 0, "bwd_segs": 1, "atomic_lanes": 4, "batch": 64, "big_tiles": 0}
    for bad in ({"split_len": 0}, {"split_parts": 3}, {"waves_per_cu": 2}, {"waves_per_cu": 65},
                {"generate_entries": 2}, {"item_grab": 0}, {"item_grab": 17}, {"prio_len": -1}, {"bwd_segs": 3},
                {"atomic_lanes": 0}, {"atomic_lanes": 65}, {"batch": 128}, {"batch": 48}, {"big_tiles": 15},
                {"big_tiles": -1}):
        t = abi.GsTuning(**{**before, **bad})
        with pytest.raises(abi.GsError):
            abi.gs_set_tuning(t)
        assert abi.gs_get_tuning().as_dict() == before
    want = {"split_len": 1024, "split_parts": 2, "waves_per_cu": 16, "split_priority": 0, "generate_entries": 1,
            "item_grab": 4, "prio_len": 512, "bwd_segs": 4, "atomic_lanes": 64, "batch": 32, "big_tiles": 16}
    abi.gs_set_tuning(abi.GsTuning(**want))
    try:
        assert abi.gs_get_tuning().as_dict() == want
    finally:
        abi.gs_set_tuning(abi.GsTuning(**before))
