"""gs_bin_and_sort_static -- the binning entry point that allocates nothing and uses the
library's static per-GPU workspace -- against gs_bin_and_sort with a caller workspace: the
same list, ranges, work list and counters, bit for bit, on two calls in a row, the second
with a smaller input (the static array keeps the first call's contents). A call that needs
more than the static workspace is refused before anything is launched."""
import numpy as np
import pytest

from paper_2312_02121_amd import synth

from gpu_helpers import same_work_list

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _state(b, K):
    return {"keys": b.keys[:K].clone(), "ids": b.ids[:K].clone(), "ranges": b.ranges.clone(),
            "schedule": b.schedule.clone(), "counters": b.counters.clone()}


def _both(wl):
    from paper_2312_02121_amd import abi, pipeline
    g = pipeline.GaussianSet(wl.scenes)
    cams = pipeline.CameraSet(wl.cameras, g.sizes)
    r = pipeline.Rasterizer(cams)
    st = r.forward(g)                      # projects, and sizes the list capacity
    torch.cuda.synchronize()
    P, cap = cams.n_splats, r.bins.capacity
    assert abi.gs_bin_and_sort_workspace_size(P, cap, cams.n_tiles) <= abi.STATIC_WORKSPACE_BYTES
    stream = pipeline.current_stream()
    ref = pipeline.Bins.alloc(P, cap, cams.n_tiles, r.device)
    abi.gs_bin_and_sort(r.splats.struct(P), P, cams.ptr, cams.n_cams, ref.struct(), ref.workspace.data_ptr(),
                        ref.workspace.numel(), stream)
    out = pipeline.Bins.alloc(P, cap, cams.n_tiles, r.device)
    out.workspace = torch.empty(0, dtype=torch.uint8, device=r.device)   # not used
    out.keys.fill_(-1)
    out.ids.fill_(-1)
    abi.gs_bin_and_sort_static(r.splats.struct(P), P, cams.ptr, cams.n_cams, out.struct(), stream)
    torch.cuda.synchronize()
    K = int(ref.counters[0])
    assert K == st.K and int(ref.counters[1]) == 0
    a, b = _state(ref, K), _state(out, K)
    for name in ("keys", "ids", "ranges", "counters"):
        assert torch.equal(a[name], b[name]), name
    same_work_list(a["schedule"].cpu().numpy(), b["schedule"].cpu().numpy())
    return r, P, cams


def test_static_workspace_matches_caller_workspace_twice():
    print("[case] no_alloc wl=c3 then c2_20k", flush=True)
    _both(synth.make_config(3))                       # ~41 MB of the static workspace
    print("[case] no_alloc second call, smaller", flush=True)
    r, P, cams = _both(synth.make_config(2, n_override=20_000))

    # a call that needs more than the static workspace is refused on the host
    from paper_2312_02121_amd import abi, pipeline
    big = pipeline.Bins.alloc(P, 1024, cams.n_tiles, r.device)
    s = big.struct()
    s.capacity = 1 << 30
    with pytest.raises(abi.GsError) as e:
        abi.gs_bin_and_sort_static(r.splats.struct(P), P, cams.ptr, cams.n_cams, s, pipeline.current_stream())
    assert e.value.code == abi.GS_ERR_CAPACITY
