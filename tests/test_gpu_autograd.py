"""torch.autograd.Function over the C ABI: gradients against the FP64 oracle and against
finite differences of the GPU forward itself; camera-pose gradients against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2312_02121_amd import synth

from gpu_helpers import GRAD_REL, elementwise_ok, oracle_params, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS = ("means", "quats", "scales", "colors", "opacities")


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def params_of(wl, requires_grad=True):
    s = wl.scenes[0]
    return [torch.tensor(np.asarray(s[k]), device="cuda", requires_grad=requires_grad) for k in KEYS]


@pytest.mark.parametrize("name", ["c1", "tilted"])
def test_autograd_matches_oracle(name):
    _print_case("autograd", wl=name)
    from paper_2312_02121_amd.autograd import render
    wl = synth.make_config(1) if name == "c1" else synth.tilted_camera_scene(50, n=120, width=70, height=45)
    cam = wl.cameras[0]
    prm = oracle_params()
    orc = oracle.render(wl.scenes[0], cam, prm)
    ok = orc["flags"] == 0
    w = np.random.default_rng(1).standard_normal((3, cam.height, cam.width))
    w[:, ~ok] = 0.0
    ps = params_of(wl)
    img = render(*ps, [cam])[0]
    assert np.abs(img.detach().cpu().numpy() - orc["C"])[:, ok].max() <= 1e-5
    loss = (img * torch.from_numpy(w).float().cuda()).sum()
    loss.backward()
    ref = oracle.render_backward(wl.scenes[0], cam, prm, w, state=orc)
    for k, p in zip(KEYS, ps):
        got = p.grad.detach().cpu().numpy().astype(np.float64)
        assert rel_err(got, ref[k]) <= GRAD_REL, (k, rel_err(got, ref[k]))
        assert elementwise_ok(got, ref[k]), k


def test_autograd_finite_differences():
    """Central differences of the GPU forward on the parameters with the largest gradients.

    The forward is float32, so the step must be large (1e-3 relative); a step that moves a
    3-sigma box across a tile edge or an alpha across a threshold makes the loss jump, so each
    sample is taken with three steps (h, h/2, h/4) and kept only when all three agree within
    2%; the analytic gradient is then compared with the smallest step."""
    _print_case("autograd_fd", wl="tiny")
    from paper_2312_02121_amd.autograd import render
    wl = synth.tilted_camera_scene(51, n=12, width=64, height=48)
    cam = wl.cameras[0]
    w = torch.from_numpy(np.random.default_rng(2).standard_normal((3, cam.height, cam.width))).cuda()
    ps = params_of(wl)
    loss = (render(*ps, [cam])[0] * w.float()).sum()
    loss.backward()

    def fd_at(p, idx, h):
        vals = []
        for sgn in (1, -1):
            q = p.detach().clone()
            q.view(-1)[idx] += sgn * h
            args = [x.detach() if x is not p else q for x in ps]
            with torch.no_grad():
                vals.append(float((render(*args, [cam])[0].double() * w).sum()))
        return (vals[0] - vals[1]) / (2 * h)

    checked = skipped = 0
    for p in ps:
        g = p.grad.detach()
        for idx in torch.topk(g.flatten().abs(), 8).indices.tolist():
            h = 1e-3 * max(abs(float(p.detach().flatten()[idx])), 0.1)
            f = [fd_at(p, idx, h / m) for m in (1, 2, 4)]
            scale = max(abs(f[-1]), 1e-2)
            if max(f) - min(f) > 0.02 * scale:
                skipped += 1
                continue
            an = float(g.flatten()[idx])
            assert abs(f[-1] - an) <= 3e-2 * abs(an) + 1e-2, (idx, f, an)
            checked += 1
    print(f"FD samples checked {checked}, discontinuous {skipped}")
    assert checked >= 20


def test_camera_pose_gradient_matches_oracle():
    _print_case("pose", wl="tilted")
    from paper_2312_02121_amd import pipeline
    wl = synth.tilted_camera_scene(52, n=80, width=64, height=48)
    cam = wl.cameras[0]
    prm = oracle_params()
    orc = oracle.render(wl.scenes[0], cam, prm)
    w = np.random.default_rng(3).standard_normal((3, cam.height, cam.width))
    w[:, orc["flags"] != 0] = 0.0
    ref = oracle.render_backward(wl.scenes[0], cam, prm, w, state=orc, with_pose=True)["Tcw"][:3]
    g = pipeline.GaussianSet(wl.scenes)
    cams = pipeline.CameraSet(wl.cameras, g.sizes)
    r = pipeline.Rasterizer(cams)
    st = r.forward(g)
    grads = r.backward(st, torch.from_numpy(w.reshape(3, -1)).float().cuda(), with_pose=True)
    got = grads["campose"][0].view(3, 4).cpu().numpy().astype(np.float64)
    assert rel_err(got, ref) <= GRAD_REL, (got, ref)
    assert elementwise_ok(got, ref), (got, ref)


def test_camera_pose_gradient_many_cameras():
    """eq. (28) with the R_cw term, reduced per camera, for a batch of 32 cameras over 8
    scenes (each camera's pose gradient sums over the Gaussians it sees): every camera's 3x4
    block against the oracle, norm and elementwise bars over the whole batch."""
    _print_case("pose", wl="c5_small")
    from paper_2312_02121_amd import pipeline
    from test_gpu_batched import small_c5
    wl = small_c5()
    prm = oracle_params()
    g = pipeline.GaussianSet(wl.scenes)
    cams = pipeline.CameraSet(wl.cameras, g.sizes)
    rng = np.random.default_rng(4)
    w_img = np.zeros((3, cams.n_pixels), np.float32)
    ref = np.zeros((len(wl.cameras), 3, 4))
    for k, cam in enumerate(wl.cameras):
        orc = oracle.render(wl.scenes[cam.scene], cam, prm)
        w = rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)
        w[:, orc["flags"] != 0] = 0.0
        off, H, W = cams.image_slice(k)
        w_img[:, off:off + H * W] = w.reshape(3, -1)
        ref[k] = oracle.render_backward(wl.scenes[cam.scene], cam, prm, w.astype(np.float64), state=orc,
                                        with_pose=True)["Tcw"][:3]
    r = pipeline.Rasterizer(cams)
    st = r.forward(g)
    grads = r.backward(st, torch.from_numpy(w_img).cuda(), with_pose=True)
    got = grads["campose"].view(-1, 3, 4).cpu().numpy().astype(np.float64)
    e = rel_err(got, ref)
    print(f"camera-pose gradients of {len(wl.cameras)} cameras: rel err {e:.2e}")
    assert e <= GRAD_REL, e
    assert elementwise_ok(got, ref)
