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


@pytest.mark.parametrize("name", ["c1", "tilted", "c5_small"])
def test_l2_loss_function_matches_oracle(name):
    """The fused training form (autograd.l2_loss: one graph replay of project, sort, fused
    forward + dL/dC + backward, project_bwd) against the oracle: the loss and every gradient,
    over one camera or a batch of 32 cameras of 8 scenes, on repeated calls; near-tie pixels
    get the GPU's own image as target (dL/dC exactly 0 there) and zero dL/dC in the oracle."""
    _print_case("l2_loss", wl=name)
    from paper_2312_02121_amd import pipeline
    from paper_2312_02121_amd.autograd import l2_loss
    from test_gpu_batched import small_c5
    wl = {"c1": lambda: synth.make_config(1),
          "tilted": lambda: synth.tilted_camera_scene(50, n=120, width=70, height=45), "c5_small": small_c5}[name]()
    prm = oracle_params()
    sizes = [s["opacities"].shape[0] for s in wl.scenes]
    ps = [torch.tensor(np.concatenate([np.asarray(s[k]) for s in wl.scenes], axis=-1), device="cuda",
                       requires_grad=True) for k in KEYS]
    cams = pipeline.CameraSet(wl.cameras, sizes)
    # the GPU image, for the near-tie pixels' targets
    from paper_2312_02121_amd.autograd import render
    with torch.no_grad():
        imgs = render(*[p.detach() for p in ps], wl.cameras, scene_sizes=sizes)
    tgt = np.concatenate([t.reshape(3, -1) for t in wl.targets], axis=1).astype(np.float32)
    ref = {k: [np.zeros(np.asarray(s[k]).shape) for s in wl.scenes] for k in KEYS}
    loss_ref = 0.0
    for k, cam in enumerate(wl.cameras):
        orc = oracle.render(wl.scenes[cam.scene], cam, prm)
        fl = orc["flags"] != 0
        off, H, W = cams.image_slice(k)
        t = tgt[:, off:off + H * W].reshape(3, H, W)
        t[:, fl] = imgs[k].cpu().numpy()[:, fl]
        l, dL = oracle.loss_l2(orc["C"], t)
        dL[:, fl] = 0.0
        loss_ref += l
        og = oracle.render_backward(wl.scenes[cam.scene], cam, prm, dL, state=orc)
        for key in KEYS:
            ref[key][cam.scene] += og[key]
    target = torch.from_numpy(tgt).cuda()
    for rep in range(3):
        for p in ps:
            p.grad = None
        loss = l2_loss(*ps, wl.cameras, target, scene_sizes=sizes)
        loss.backward()
        torch.cuda.synchronize()
        assert abs(float(loss) - loss_ref) <= 1e-5 * loss_ref, (rep, float(loss), loss_ref)
        for k, p in zip(KEYS, ps):
            got = p.grad.detach().cpu().numpy().astype(np.float64)
            r = np.concatenate(ref[k], axis=-1)
            assert rel_err(got, r) <= GRAD_REL, (rep, k, rel_err(got, r))
            assert elementwise_ok(got, r), (rep, k)


def test_l2_loss_overflow_gives_nan_then_regrows():
    """A list that outgrows the captured step's capacity: that call's loss is NaN (the fused
    launch sees the overflow flag) without any host synchronisation, and the next call, after
    the step has finished, regrows the list and is valid again."""
    _print_case("l2_overflow", wl="c1")
    from paper_2312_02121_amd.autograd import l2_loss
    wl = synth.make_config(1)
    ps = [torch.tensor(np.asarray(wl.scenes[0][k]), device="cuda", requires_grad=True) for k in KEYS]
    target = torch.from_numpy(wl.targets[0].reshape(3, -1)).cuda()
    first = float(l2_loss(*ps, wl.cameras, target))
    assert np.isfinite(first)
    with torch.no_grad():
        ps[2].mul_(8.0)              # scales x8: every box covers far more tiles
    torch.cuda.synchronize()
    assert np.isnan(float(l2_loss(*ps, wl.cameras, target)))
    torch.cuda.synchronize()
    grown = l2_loss(*ps, wl.cameras, target)
    grown.backward()
    assert np.isfinite(float(grown)) and float(grown) != first
