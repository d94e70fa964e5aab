"""HIP path against the FP64 oracle, element by element, on seeded synthetic inputs.

Bars: splat fields, tile lists and sort order bit-exact; image within 1e-5 abs;
gradients within 1e-3 relative (per tensor norm and elementwise against
|g*| + rms(g*)). Pixels whose float decisions sit within the stated margins of a
threshold are excluded and counted (gpu_helpers.MARGIN_*), and receive zero upstream
gradient on both sides so that the backward comparison is exact in its inputs.
"""
import numpy as np
import pytest

import oracle
from paper_2312_02121_amd import synth

from gpu_helpers import (IMAGE_ATOL, GRAD_REL, bins_arrays, camera_images, elementwise_ok, flag_budget,
                         gpu_forward, oracle_camera, oracle_params, rel_err, splat_arrays, tile_offsets,
                         worst_element, check_projection, same_work_list)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _workloads():
    return {
        "c1": synth.make_config(1),
        "tiny_tilted": synth.tilted_camera_scene(40, n=200, width=70, height=45),
        "c2_20k": synth.make_config(2, n_override=20_000),
        "dense_small": synth.tiny_scene(41, n=600, width=100, height=77, log_scale=(-1.5, 0.6), opac_sd=2.5),
        # 257 x 125 tiles: more than one LDS band of the per-tile length count
        "wide_4k": synth.tiny_scene(42, n=500, width=4100, height=2000, f=2000.0, log_scale=(-2.0, 0.8)),
        # 16 orbit views inside the scene: splats near a camera cover most of its tiles
        "c4_20k": synth.make_config(4, n_override=20_000),
        # 12 x 10 tiles, up to ~790 small entries per tile (more than the merge walk stages in
        # LDS at once) under ~125 splats of more than 16 tiles
        "dense_wrap": synth.tiny_scene(44, n=12_000, width=192, height=160, f=150.0, log_scale=(-3.0, 0.6),
                                       spread=0.45),
    }


WL = None


def wl_cache():
    global WL
    if WL is None:
        WL = _workloads()
    return WL


@pytest.mark.parametrize("name", ["c1", "tiny_tilted", "c2_20k", "dense_small"])
def test_projection_bit_exact(name):
    _print_case("projection", wl=name)
    wl = wl_cache()[name]
    r, st = gpu_forward(wl)
    check_projection(wl, r)


@pytest.mark.parametrize("generate", [0, 1])
@pytest.mark.parametrize("name", ["c1", "tiny_tilted", "c2_20k", "dense_small", "wide_4k"])
def test_bins_bit_exact(name, generate):
    """Both first tile-sort passes (emitted list, or entries generated inside the pass)."""
    _print_case("bins", wl=name, generate_entries=generate)
    from paper_2312_02121_amd import autotune
    wl = wl_cache()[name]
    autotune.apply({**autotune.default_tuning(), "generate_entries": generate})
    try:
        r, st = gpu_forward(wl)
    finally:
        autotune.apply(autotune.default_tuning())
    toffs = tile_offsets(wl)
    okeys, oids, oranges = [], [], []
    for k, cam in enumerate(wl.cameras):
        o = oracle.project(wl.scenes[cam.scene], cam, oracle_params())
        b = oracle.bin_and_sort(o, cam, tile_offset=toffs[k])
        poff = int(r.cams.host[k]["proj_offset"])
        okeys.append(b["keys"])
        oids.append(b["ids"] + poff)
        oranges.append(np.where(b["ranges"][:, 1:] > b["ranges"][:, :1], b["ranges"] + sum(map(len, okeys[:-1])), 0))
    okeys, oids = np.concatenate(okeys), np.concatenate(oids)
    assert st.K == okeys.size
    g = bins_arrays(r, st.K)
    assert np.array_equal(g["keys"], okeys)
    assert np.array_equal(g["ids"], oids.astype(np.int32))
    assert np.array_equal(g["ranges"], np.concatenate(oranges).astype(np.int32))


def _oracle_list(wl, r):
    toffs = tile_offsets(wl)
    okeys, oids, oranges = [], [], []
    for k, cam in enumerate(wl.cameras):
        o = oracle.project(wl.scenes[cam.scene], cam, oracle_params())
        b = oracle.bin_and_sort(o, cam, tile_offset=toffs[k])
        poff = int(r.cams.host[k]["proj_offset"])
        okeys.append(b["keys"])
        oids.append(b["ids"] + poff)
        oranges.append(np.where(b["ranges"][:, 1:] > b["ranges"][:, :1], b["ranges"] + sum(map(len, okeys[:-1])), 0))
    return np.concatenate(okeys), np.concatenate(oids).astype(np.int32), np.concatenate(oranges).astype(np.int32)


@pytest.mark.parametrize("big_tiles", [16, 64, 1024])
@pytest.mark.parametrize("name", ["c1", "tiny_tilted", "c2_20k", "dense_small", "wide_4k", "c4_20k", "dense_wrap"])
def test_bins_bit_exact_with_merge(name, big_tiles):
    """Splats with more than big_tiles tiles listed by the per-tile merge instead of the tile
    sort: keys, ids and ranges bit-exact, and the image as the oracle's."""
    from paper_2312_02121_amd import autotune
    wl = wl_cache()[name]
    autotune.apply({**autotune.default_tuning(), "big_tiles": big_tiles})
    try:
        r, st = gpu_forward(wl)
    finally:
        autotune.apply(autotune.default_tuning())
    okeys, oids, oranges = _oracle_list(wl, r)
    tiles = r.splats.tiles[: r.cams.n_splats].cpu().numpy()
    n_big = int((tiles > big_tiles).sum())
    _print_case("bins_merge", wl=name, big_tiles=big_tiles, big_splats=n_big,
                big_entries=int(tiles[tiles > big_tiles].sum()), K=okeys.size)
    assert st.K == okeys.size
    g = bins_arrays(r, st.K)
    assert np.array_equal(g["keys"], okeys)
    assert np.array_equal(g["ids"], oids)
    assert np.array_equal(g["ranges"], oranges)
    if name in ("c1", "dense_small"):
        _forward_compare(wl, r, st)


def test_merge_overflow_and_give_up_build_no_list():
    """With the merge: a capacity below K reports overflow and builds nothing (buffers filled
    with garbage first); a forced give-up of the sort's look-back reports flag 2 and builds
    nothing; a regrown call builds the oracle's list."""
    _print_case("merge_overflow", wl="c4_20k")
    from paper_2312_02121_amd import abi, autotune, pipeline
    wl = wl_cache()["c4_20k"]
    g = pipeline.GaussianSet(wl.scenes)
    cams = pipeline.CameraSet(wl.cameras, g.sizes)
    autotune.apply({**autotune.default_tuning(), "big_tiles": 16})
    try:
        r = pipeline.Rasterizer(cams, capacity=4096)
        r.project(g)
        b = r.bins
        for t in (b.keys, b.ids, b.ranges, b.workspace):
            t.view(torch.uint8).fill_(0x7F)
        r.bin_and_sort()
        torch.cuda.synchronize()
        K, over = r.read_count()
        assert over and K > 4096
        assert int(b.ranges.abs().max()) == 0
        st = r.forward(g)                         # regrows and builds the full list
        torch.cuda.synchronize()
        okeys, oids, oranges = _oracle_list(wl, r)
        assert st.K == K == okeys.size
        assert np.array_equal(bins_arrays(r, st.K)["ids"], oids)
        abi.gs_set_sort_wait_limit(-1)
        try:
            r.bin_and_sort()
            torch.cuda.synchronize()
        finally:
            abi.gs_set_sort_wait_limit(abi.DEFAULT_SORT_WAIT_LIMIT)
        assert int(r.bins.counters[1]) & 2
        assert int(r.bins.ranges.abs().max()) == 0
    finally:
        autotune.apply(autotune.default_tuning())


def _forward_compare(wl, r, st, prm=None, check_last=True):
    flagged_total, pixels = 0, 0
    for k in range(len(wl.cameras)):
        orc, scene, cam, prm = oracle_camera(wl, k, prm)
        g = camera_images(r, st, k)
        ok = orc["flags"] == 0
        flagged_total += int((~ok).sum())
        pixels += ok.size
        assert (~ok).sum() <= flag_budget(ok.size), f"cam {k}: {int((~ok).sum())} near-tie pixels of {ok.size}"
        err = np.abs(g["C"] - orc["C"])[:, ok]
        assert err.max(initial=0.0) <= IMAGE_ATOL, f"cam {k}: image err {err.max()}"
        assert np.abs(g["T_final"] - orc["T_final"])[ok].max(initial=0.0) <= IMAGE_ATOL
        if check_last:
            assert np.array_equal(g["last"][ok], orc["last"][ok])
        assert np.array_equal(g["visited"][ok], orc["visited"][ok])
    return flagged_total, pixels


@pytest.mark.parametrize("name", ["c1", "tiny_tilted", "c2_20k", "dense_small"])
def test_forward_image(name):
    _print_case("forward", wl=name)
    wl = wl_cache()[name]
    r, st = gpu_forward(wl)
    flagged, pixels = _forward_compare(wl, r, st)
    print(f"flagged pixels {flagged} / {pixels} ({flagged / pixels:.2e})")
    assert flagged <= flag_budget(pixels)


@pytest.mark.parametrize("tuning", [{}, {"split_len": 32, "split_parts": 4}, {"split_len": 32, "split_parts": 2}])
@pytest.mark.parametrize("name", ["tiny_tilted", "c2_20k", "dense_small"])
def test_skipped_records_change_nothing(name, tuning):
    """The walks leave out records that cannot reach alpha_min at the pixels still active
    (their rectangle, the exact largest exponent over it). The forward that counts visits
    keeps every record, so the two forwards must agree bit for bit on image, T_final and
    last, for whole tiles and for halves and quarters of split tiles."""
    _print_case("skip_exact", wl=name, **tuning)
    from paper_2312_02121_amd import autotune
    wl = wl_cache()[name]
    autotune.apply({**autotune.default_tuning(), **tuning})
    try:
        r_all, _ = gpu_forward(wl, keep_visited=True)
        r_skip, _ = gpu_forward(wl, keep_visited=False)
    finally:
        autotune.apply(autotune.default_tuning())
    assert r_skip.visited is None and r_all.visited is not None
    assert torch.equal(r_skip.image, r_all.image)
    assert torch.equal(r_skip.T_final, r_all.T_final)
    assert torch.equal(r_skip.last, r_all.last)


def _backward_compare(wl, r, st, seed=0, with_pose=False, prm=None):
    rng = np.random.default_rng(seed)
    cams = r.cams
    g_img = np.zeros((3, cams.n_pixels), dtype=np.float32)
    og = {k: np.zeros_like(v, dtype=np.float64) for k, v in wl.scenes[0].items()}
    ograds = [{key: np.zeros(np.asarray(s[key]).shape) for key in ("means", "quats", "scales", "colors", "opacities")}
              for s in wl.scenes]
    oprm = prm
    for k, cam in enumerate(wl.cameras):
        orc, scene, _, prm = oracle_camera(wl, k, oprm)
        g = rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)
        g[:, orc["flags"] != 0] = 0.0
        off = int(cams.host[k]["pixel_offset"])
        g_img[:, off:off + cam.width * cam.height] = g.reshape(3, -1)
        og = oracle.render_backward(scene, cam, prm, g.astype(np.float64), state=orc)
        for key in ograds[cam.scene]:
            ograds[cam.scene][key] += og[key]
    grads = r.backward(st, torch.from_numpy(g_img).cuda(), with_pose=with_pose)
    torch.cuda.synchronize()
    out = {}
    for key in ("means", "quats", "scales", "colors", "opacities"):
        gpu = grads[key].cpu().numpy().astype(np.float64)
        ref = np.concatenate([o[key] for o in ograds], axis=-1)
        out[key] = (rel_err(gpu, ref), elementwise_ok(gpu, ref))
        if not out[key][1]:
            print(f"worst {key}: {worst_element(gpu, ref)}", flush=True)
    for key in ("mean2d", "conic"):
        if key in grads:
            print(f"{key} grads computed on the GPU: shape {tuple(grads[key].shape)}")
    return out


@pytest.mark.parametrize("name", ["c1", "tiny_tilted", "c2_20k", "dense_small"])
def test_backward_gradients(name):
    _print_case("backward", wl=name)
    wl = wl_cache()[name]
    r, st = gpu_forward(wl)
    res = _backward_compare(wl, r, st)
    print(res)
    for key, (rel, elem) in res.items():
        assert rel <= GRAD_REL, (key, rel)
        assert elem, key



BG = (0.3, -0.2, 0.8)


@pytest.mark.parametrize("name", ["tiny_tilted", "c2_20k"])
def test_background_forward_and_backward(name):
    """The background variant (C + T_final bg; bg in the colour behind every entry) against
    the oracle with the same background, forward and backward."""
    _print_case("background", wl=name)
    from paper_2312_02121_amd import pipeline
    wl = wl_cache()[name]
    r, st = gpu_forward(wl, params=pipeline.make_params(background=BG))
    prm = oracle_params(background=BG)
    flagged, pixels = _forward_compare(wl, r, st, prm=prm)
    assert flagged <= flag_budget(pixels)
    res = _backward_compare(wl, r, st, prm=prm)
    print(res)
    for key, (rel, elem) in res.items():
        assert rel <= GRAD_REL, (key, rel)
        assert elem, key


@pytest.mark.parametrize("name", ["tiny_tilted", "c2_20k"])
def test_normalized_quats_projection_image_and_gradients(name):
    """Quaternion normalisation (R(q / |q|)) on non-unit quaternions: the projection stays
    bit-exact against the oracle with the same option, the image and every gradient (dL/dq
    through the normalisation) within the bars."""
    import copy
    _print_case("normalize_quats", wl=name)
    base = wl_cache()[name]
    wl = copy.copy(base)
    rng = np.random.default_rng(5)
    wl.scenes = [dict(sc, quats=(sc["quats"] * rng.uniform(0.5, 2.0, sc["quats"].shape[1])).astype(np.float32))
                 for sc in base.scenes]
    wl.scenes[0]["quats"][:, 0] = 0.0            # no direction: culled on both sides
    r, st = gpu_forward(wl, normalize_quats=True)
    prm = oracle_params(normalize_quats=True)
    check_projection(wl, r, prm=prm)
    flagged, pixels = _forward_compare(wl, r, st, prm=prm)
    assert flagged <= flag_budget(pixels)
    res = _backward_compare(wl, r, st, prm=prm)
    print(res)
    for key, (rel, elem) in res.items():
        assert rel <= GRAD_REL, (key, rel)
        assert elem, key


@pytest.mark.parametrize("name", ["tiny_tilted", "c2_20k"])
def test_lambda_max_box_projection_lists_image_and_gradients(name):
    """Square 3-sigma boxes from lambda_max: projection (rect, tile counts) and tile lists
    bit-exact against the oracle with the same option, image and gradients within the bars."""
    _print_case("box_lambda_max", wl=name)
    wl = wl_cache()[name]
    r, st = gpu_forward(wl, box_lambda_max=True)
    prm = oracle_params(box_lambda_max=True)
    check_projection(wl, r, prm=prm)
    toffs = tile_offsets(wl)
    K = 0
    for k, cam in enumerate(wl.cameras):
        K += oracle.bin_and_sort(oracle.project(wl.scenes[cam.scene], cam, prm), cam, tile_offset=toffs[k])["K"]
    assert st.K == K
    flagged, pixels = _forward_compare(wl, r, st, prm=prm)
    assert flagged <= flag_budget(pixels)
    res = _backward_compare(wl, r, st, prm=prm)
    print(res)
    for key, (rel, elem) in res.items():
        assert rel <= GRAD_REL, (key, rel)
        assert elem, key

def test_multi_scene_multi_camera():
    _print_case("multi", wl="c5_small")
    wl = synth.make_config(5, n_override=3000)
    # keep the test small: shrink every camera to at most 256 x 256
    for k, c in enumerate(wl.cameras):
        s = min(1.0, 256.0 / max(c.width, c.height))
        w, h = max(1, int(c.width * s)), max(1, int(c.height * s))
        # rebuild so that every camera value is rounded to float32 exactly as the GPU receives it
        wl.cameras[k] = synth.Camera(c.R, c.t, c.fx * s, c.fy * s, w / 2, h / 2, w, h, c.near, c.far, c.scene)
    r, st = gpu_forward(wl)
    check_projection(wl, r)
    flagged, pixels = _forward_compare(wl, r, st)
    assert flagged <= flag_budget(pixels)
    res = _backward_compare(wl, r, st, seed=3)
    for key, (rel, elem) in res.items():
        assert rel <= GRAD_REL, (key, rel)
        assert elem, key


def test_capacity_overflow_regrows():
    _print_case("overflow", wl="c1")
    wl = synth.make_config(1)
    r, st = gpu_forward(wl, capacity=16)
    assert r.bins.capacity > 16
    r2, st2 = gpu_forward(wl)
    assert st.K == st2.K
    assert torch.equal(st.image, st2.image)


def test_overflow_builds_no_list():
    """A list capacity below K: the call reports overflow, leaves every tile range empty and
    writes nothing from the unsorted buffers, which are filled with garbage first (a first
    pass that sorted only the entries below the capacity once left slots of its output
    unwritten, and the next pass gathered depth through them)."""
    _print_case("overflow_garbage", wl="c2_20k")
    from paper_2312_02121_amd import abi, pipeline
    wl = wl_cache()["c2_20k"]
    g = pipeline.GaussianSet(wl.scenes)
    cams = pipeline.CameraSet(wl.cameras, g.sizes)
    r = pipeline.Rasterizer(cams, capacity=4096)
    r.project(g)
    b = r.bins
    for t in (b.keys, b.ids, b.ranges, b.workspace):
        t.view(torch.uint8).fill_(0x7F)
    abi.gs_bin_and_sort(r.splats.struct(cams.n_splats), cams.n_splats, cams.ptr, cams.n_cams, b.struct(),
                        b.workspace.data_ptr(), b.workspace.numel(), pipeline.current_stream())
    r.rasterize_fwd()
    torch.cuda.synchronize()
    K, over = r.read_count()
    assert over and K > 4096
    assert int(b.ranges.abs().max()) == 0
    assert float(r.image.abs().max()) == 0.0
    st = r.forward(g)                         # regrows and builds the full list
    assert st.K == K and not r.read_count()[1]


def test_deterministic_lists_and_image():
    _print_case("determinism", wl="c2_20k")
    wl = wl_cache()["c2_20k"]
    r, st = gpu_forward(wl)
    keys, img = r.bins.keys[: st.K].clone(), st.image.clone()
    r2, st2 = gpu_forward(wl)
    assert torch.equal(keys, r2.bins.keys[: st2.K]) and torch.equal(img, st2.image)


def test_projection_record_is_optional():
    # without gs_project's 12-float record (rec = NULL) the list and the image are the same
    _print_case("optional record", wl="c2_20k")
    from paper_2312_02121_amd import pipeline
    wl = wl_cache()["c2_20k"]
    r, st = gpu_forward(wl)
    g = pipeline.GaussianSet(wl.scenes)
    r2 = pipeline.Rasterizer(pipeline.CameraSet(wl.cameras, g.sizes), keep_records=False)
    assert r2.splats.rec is None
    st2 = r2.forward(g)
    torch.cuda.synchronize()
    assert st2.K == st.K
    assert torch.equal(r.bins.keys[: st.K], r2.bins.keys[: st2.K]) and torch.equal(st.image, st2.image)


@pytest.mark.parametrize("name", ["tiny_tilted", "c2_20k", "c4_20k"])
@pytest.mark.parametrize("generate", [0, 1, "merge"])
def test_sorted_keys_are_optional(name, generate):
    """With GS_BINS_NO_KEYS the sort writes no 64-bit keys; the ids, ranges, count, work list
    and image are those of a call that writes them (one tile pass for the tiny scene, two at
    512x512; entries emitted or generated inside the first pass)."""
    _print_case("no_keys", wl=name, generate=generate)
    from paper_2312_02121_amd import autotune, pipeline
    wl = wl_cache()[name]
    g = pipeline.GaussianSet(wl.scenes)
    knob = {"big_tiles": 16} if generate == "merge" else {"generate_entries": generate}
    autotune.apply({**autotune.default_tuning(), **knob})
    try:
        out = []
        for write_keys in (True, False):
            r = pipeline.Rasterizer(pipeline.CameraSet(wl.cameras, g.sizes), write_keys=write_keys)
            st = r.forward(g)
            torch.cuda.synchronize()
            out.append((r, st))
    finally:
        autotune.apply(autotune.default_tuning())
    (r1, s1), (r2, s2) = out
    assert s1.K == s2.K > 0
    K = s1.K
    for name_ in ("ids", "ranges", "counters"):
        assert torch.equal(getattr(r1.bins, name_)[:K] if name_ == "ids" else getattr(r1.bins, name_),
                           getattr(r2.bins, name_)[:K] if name_ == "ids" else getattr(r2.bins, name_)), name_
    same_work_list(r1.bins.schedule.cpu().numpy(), r2.bins.schedule.cpu().numpy())
    assert torch.equal(s1.image, s2.image)
    # the keys the first call wrote are the oracle's
    toffs = tile_offsets(wl)
    keys = [oracle.bin_and_sort(oracle.project(wl.scenes[c.scene], c, oracle_params()), c,
                                tile_offset=toffs[k])["keys"] for k, c in enumerate(wl.cameras)]
    assert np.array_equal(r1.bins.keys[:K].cpu().numpy().view(np.uint64), np.concatenate(keys))


def test_near_plane_behind_the_camera():
    """With a near plane at or behind the camera the projection still culls t_z <= 0 (depth
    keys are float bits of t_z): splat fields and lists bit-exact against the oracle."""
    _print_case("near_behind", wl="tiny")
    wl = synth.tiny_scene(44, n=300, width=64, height=48)
    rng = np.random.default_rng(1)
    wl.scenes[0]["means"][2] = rng.uniform(-3.0, 4.0, 300).astype(np.float32)
    for c in wl.cameras:
        c.near = -1.0
    r, st = gpu_forward(wl)
    check_projection(wl, r)
    o = oracle.project(wl.scenes[0], wl.cameras[0], oracle_params())
    assert (o["tiles"][wl.scenes[0]["means"][2] <= 0] == 0).all()
    b = oracle.bin_and_sort(o, wl.cameras[0])
    g = bins_arrays(r, st.K)
    assert st.K == b["K"] and np.array_equal(g["keys"], b["keys"]) and np.array_equal(g["ids"], b["ids"])


def test_edge_cases():
    _print_case("edges", wl="edge")
    # everything behind the camera or outside the image: K = 0, empty image
    wl = synth.tiny_scene(42, n=50)
    wl.scenes[0]["means"][2] = -1.0
    r, st = gpu_forward(wl)
    assert st.K == 0
    assert float(st.image.abs().max()) == 0.0 and float(st.T_final.min()) == 1.0
    # one huge Gaussian over a ragged image (partial tiles on both axes), one tiny one
    wl = synth.tiny_scene(43, n=2, width=37, height=23)
    wl.scenes[0]["scales"][:, 0] = 5.0
    wl.scenes[0]["scales"][:, 1] = 1e-3
    r, st = gpu_forward(wl)
    check_projection(wl, r)
    flagged, pixels = _forward_compare(wl, r, st)
    assert flagged <= flag_budget(pixels)
    res = _backward_compare(wl, r, st, seed=5)
    for key, (rel, elem) in res.items():
        assert rel <= GRAD_REL, (key, rel)
        assert elem, key


def test_sort_give_up_path_reports_and_builds_no_list():
    """The single-pass sort's look-back waits are bounded; when one gives up the call must set
    flag 2, build no list (every range empty) and the binding must raise. The host forces that
    path with a negative wait limit (every look-back gives up at once, every kernel ends
    normally), then restores the limit and the same buffers build the full list again."""
    _print_case("sort_give_up", wl="c2_20k")
    from paper_2312_02121_amd import abi, pipeline
    wl = wl_cache()["c2_20k"]
    g = pipeline.GaussianSet(wl.scenes)
    cams = pipeline.CameraSet(wl.cameras, g.sizes)
    r = pipeline.Rasterizer(cams)
    ref = r.forward(g)
    torch.cuda.synchronize()
    K = ref.K
    try:
        abi.gs_set_sort_wait_limit(-1)
        with pytest.raises(RuntimeError, match="look-back"):
            r.forward(g)
        torch.cuda.synchronize()
        assert int(r.bins.counters[1]) & 2
        assert int(r.bins.ranges.abs().max()) == 0
    finally:
        abi.gs_set_sort_wait_limit(abi.DEFAULT_SORT_WAIT_LIMIT)
    st = r.forward(g)
    torch.cuda.synchronize()
    assert st.K == K and int(r.bins.counters[1]) == 0


@pytest.mark.parametrize("name", ["c1", "tiny_tilted", "dense_small"])
def test_literal_mode_forward_and_backward(name):
    """The image formation of eq. (7) as printed -- alpha_min = 0, alpha_max = 1, T_min = 0:
    every entry of a tile's list composites at every pixel of the tile, no clamp, no skip,
    no early stop -- against the oracle's literal mode (pinned on the CPU by closed forms and
    central differences), forward and backward (T recovered by the division of eq. 17)."""
    _print_case("literal", wl=name)
    from gpu_helpers import MARGIN_ALPHA, MARGIN_CLAMP, MARGIN_T, ROUND_T
    from paper_2312_02121_amd import pipeline
    wl = wl_cache()[name]
    r, st = gpu_forward(wl, params=pipeline.make_params(alpha_min=0.0, alpha_max=1.0, T_min=0.0))
    prm = oracle.Params.literal(margin_alpha=MARGIN_ALPHA, margin_T=MARGIN_T, margin_clamp=MARGIN_CLAMP,
                                round_T=ROUND_T)
    # `last` (one past the last composited entry, where the backward starts) is not compared:
    # with alpha_min = 0 every entry composites, and the kernel's count stops at the last one
    # whose float32 alpha is above 0 (later ones underflow to exactly 0 and change nothing)
    flagged, pixels = _forward_compare(wl, r, st, prm=prm, check_last=False)
    print(f"flagged pixels {flagged} / {pixels}")
    res = _backward_compare(wl, r, st, prm=prm)
    print(res)
    for key, (rel, elem) in res.items():
        assert rel <= GRAD_REL, (key, rel)
        assert elem, key


def test_literal_mode_fused_equals_separate():
    _print_case("literal_fused", wl="c1")
    from paper_2312_02121_amd import pipeline
    from test_gpu_batched import build, grads_np, assert_grads_close
    wl = synth.make_config(1)
    prm = pipeline.make_params(alpha_min=0.0, alpha_max=1.0, T_min=0.0)
    _, _, _, sep = build(wl, "separate", params=prm)
    _, _, _, fus = build(wl, "fused", params=prm)
    sep()
    fus()
    torch.cuda.synchronize()
    assert torch.equal(sep.r.image, fus.r.image)
    assert_grads_close(grads_np(fus), grads_np(sep))
