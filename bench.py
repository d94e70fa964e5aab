#!/usr/bin/env python3
"""Benchmark of the differentiable tile rasterizer on one MI355X.

A step is one pass of the whole hot path over the 1M-Gaussian, 1920x1080 workload
(64 anisotropic clusters filling a 20 m box seen from 3 m outside it):
    project -> bin_and_sort -> rasterize_fwd -> L2 loss gradient -> rasterize_bwd -> project_bwd
with every input resident in HBM before the timed region. The metric is Gaussian-pixel
evaluations per second: E = sum over pixels of the list entries whose alpha the forward
evaluates (the backward re-walks the composited ones), divided by the step time.

Prints ONE JSON line on stdout (progress goes to stderr).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd Gaussian-pixel evals/s and ms/view at 1M Gaussians 1080p; batched vs per-view"
# fp32 VALU lane-operations/s: 256 CUs x 4 SIMDs x 32 lanes per clock x 2.4 GHz = 78.6 T, i.e. the
# published 157.3 TFLOP/s fp32 vector peak with an FMA counted as one operation (gfx950 issues a
# non-packed wave64 fp32 instruction every 2 clocks per SIMD)
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# algorithmic VALU lane-operations per Gaussian-pixel pair (exp2 and rcp count 4)
SLOTS_FWD = 21
SLOTS_BWD = 46


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# What the fused kernel's code and launch depend on: its source, the shared device header, the
# C-ABI header and the recorded launch tuning. A change to any of them makes the committed
# traffic summary stale.
FUSED_KERNEL_INPUTS = ("paper_2312_02121_amd/csrc/raster.hip", "paper_2312_02121_amd/csrc/common.h",
                       "include/gsplat_mi355x.h", "paper_2312_02121_amd/tuned.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in FUSED_KERNEL_INPUTS:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(rel.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str, launches_per_step: int = 1):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, if taken on this source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_c3_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(wl, E_fwd: int, repeats: int = 3):
    import numpy as np
    import oracle
    cam, scene = wl.cameras[0], wl.scenes[0]
    prm = oracle.Params.standard()
    target = wl.targets[0].astype(np.float64)
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        pr = oracle.project(scene, cam, prm)
        b = oracle.bin_and_sort(pr, cam)
        f = oracle.rasterize_fwd(pr, scene["colors"], scene["opacities"], b, cam, prm)
        _, dL = oracle.loss_l2(f["C"], target)
        g2 = oracle.rasterize_bwd(pr, scene["colors"], scene["opacities"], b, cam, prm, dL, f)
        oracle.project_bwd(scene, cam, prm, g2["mean2d"], g2["conic"])
        times.append(time.perf_counter() - t0)
        log(f"oracle step {times[-1]:.2f} s")
    t = float(np.median(times))
    return {"value": E_fwd / t, "unit": "evals/s", "cores": oracle.max_threads(), "cpu": cpu_model(), "kind": "oracle",
            "sample": f"the whole 1M-Gaussian 1920x1080 step (FP64 oracle, OpenMP), median of {repeats} runs",
            "seconds_per_step": t}


def oracle_step_seconds(wl, threads: int) -> tuple:
    """(seconds, E) of one whole training step of the FP64 oracle over every view of the
    workload: projection, binning and sort, forward, L2 gradient, backward, projection
    backward, summed over the views; `threads` OpenMP threads."""
    import numpy as np
    import oracle
    prm = oracle.Params.standard(n_threads=threads)
    t0 = time.perf_counter()
    E = 0
    for k, cam in enumerate(wl.cameras):
        scene = wl.scenes[cam.scene]
        pr = oracle.project(scene, cam, prm)
        b = oracle.bin_and_sort(pr, cam)
        f = oracle.rasterize_fwd(pr, scene["colors"], scene["opacities"], b, cam, prm)
        _, dL = oracle.loss_l2(f["C"], wl.targets[k].astype(np.float64))
        g2 = oracle.rasterize_bwd(pr, scene["colors"], scene["opacities"], b, cam, prm, dL, f)
        oracle.project_bwd(scene, cam, prm, g2["mean2d"], g2["conic"])
        E += int(f["visited"].sum())
    return time.perf_counter() - t0, E


def oracle_legs() -> dict:
    """The oracle timed on this host beyond the bounded baseline: every workload once on all
    cores (c1-c3 median of three), and c1, c2 on one core."""
    import numpy as np
    import oracle
    from paper_2312_02121_amd import synth
    allc = oracle.max_threads()
    out = {"cpu": cpu_model(), "threads_all": allc}
    for cfg in (1, 2, 3, 4, 5):
        wl = synth.make_config(cfg)
        runs = [oracle_step_seconds(wl, allc) for _ in range(3 if cfg <= 3 else 1)]
        t = float(np.median([r[0] for r in runs]))
        E = runs[0][1]
        out[f"c{cfg}"] = {"threads": allc, "seconds_per_step": t, "evals_per_s": E / t,
                          "ms_per_view": 1e3 * t / len(wl.cameras), "E_fwd": E, "views": len(wl.cameras)}
        log(f"oracle c{cfg} on {allc} threads: {t:.2f} s/step")
        if cfg <= 2:
            t1, E1 = oracle_step_seconds(wl, 1)
            out[f"c{cfg}_single_core"] = {"threads": 1, "seconds_per_step": t1, "evals_per_s": E1 / t1}
            log(f"oracle c{cfg} on 1 thread: {t1:.2f} s/step")
    return out


def time_steps(fn, steps: int, warmup: int) -> float:
    """Mean ms per call over `steps` calls after `warmup`, events around the whole region."""
    return time_steps_detail(fn, steps, warmup)[0]


def time_steps_detail(fn, steps: int, warmup: int):
    """(mean ms per call over the whole region, [ms of each call]); an event between calls."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for k in range(steps):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    return ev[0].elapsed_time(ev[steps]) / steps, per


def stage_times(step, steps: int, warmup: int) -> dict:
    """Mean ms of each stage of an eager step, from events between the stages on the launch
    stream."""
    import numpy as np
    import torch
    n_st = len(step.STAGES)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(n_st + 1)] for _ in range(steps)]
    for k in range(steps):
        step(events=evs[k])
    torch.cuda.synchronize()
    return {name: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(steps)]))
            for i, name in enumerate(step.STAGES)}


def executed_pairs(step) -> tuple:
    """(forward, backward) Gaussian-pixel pairs the rasterizer kernels execute in one step:
    list slots walked x pixels of the wave (gs_set_work_counter), one eager step."""
    import torch
    from paper_2312_02121_amd import abi
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    abi.gs_set_work_counter(cnt.data_ptr())
    try:
        step()
        torch.cuda.synchronize()
    finally:
        abi.gs_set_work_counter(None)
    return int(cnt[0]), int(cnt[1])


def roofline_of(stage_ms: dict, E_fwd: int, E_bwd: int, executed=None) -> dict:
    """VALU roofline of the dominant rasterizer kernel: algorithmic lane-operations per launch
    (21 per forward pair, 46 per backward pair, pairs of the method: E_fwd, E_bwd) over its
    time; alongside, the same price on the pairs the kernel executes."""
    work = {"rasterize_fwd": SLOTS_FWD * E_fwd, "rasterize_bwd": SLOTS_BWD * E_bwd,
            "fused": SLOTS_FWD * E_fwd + SLOTS_BWD * E_bwd}
    dom = max((s for s in work if s in stage_ms), key=lambda s: stage_ms[s])
    achieved = work[dom] / (stage_ms[dom] * 1e-3) / 1e12
    kname = {"rasterize_fwd": "raster_fwd_kernel", "rasterize_bwd": "raster_bwd_kernel",
             "fused": "raster_fused_kernel"}[dom]
    out = {"bound": "alu", "kernel": kname, "kernel_ms": stage_ms[dom], "achieved": achieved,
           "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS,
           "slots_per_pair": {"fwd": SLOTS_FWD, "bwd": SLOTS_BWD}, "E_fwd": E_fwd, "E_bwd": E_bwd}
    if executed is not None and dom == "fused":
        xf, xb = executed
        ach_x = (SLOTS_FWD * xf + SLOTS_BWD * xb) / (stage_ms[dom] * 1e-3) / 1e12
        out["executed_pairs"] = {"fwd": xf, "bwd": xb}
        out["frac_executed"] = ach_x / VALU_PEAK_TOPS
    return out


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def e_dense(step) -> int:
    """Sum over tiles of list length x image pixels in the tile (every pair of the lists)."""
    import numpy as np
    rg = step.r.bins.ranges[: 2 * step.cams.n_tiles].view(-1, 2).cpu().numpy().astype(np.int64)
    length = rg[:, 1] - rg[:, 0]
    total = 0
    for c in step.cams.host:
        w, h, toff, tx = int(c["width"]), int(c["height"]), int(c["tile_offset"]), int(c["tiles_x"])
        ty = (h + 15) // 16
        px = np.minimum(16, w - 16 * np.arange(tx))[None, :] * np.minimum(16, h - 16 * np.arange(ty))[:, None]
        total += int((length[toff: toff + tx * ty].reshape(ty, tx) * px).sum())
    return total


def batched_vs_per_view(cfg: int, steps: int, warmup: int, tune: bool) -> dict:
    """One fused persistent launch sequence over every camera, captured in a HIP graph, against
    the same kernels run one view per launch sequence with no graph (speedup), and against the
    conventional per-view pipeline with separate forward, loss-gradient and backward launches
    (speedup_vs_separate). Each form gets its own autotuned launch tuning (the search runs
    before the timed region)."""
    import numpy as np
    import torch
    from paper_2312_02121_amd import autotune, pipeline, synth
    wl = synth.make_config(cfg)
    g = pipeline.GaussianSet(wl.scenes)
    cams = pipeline.CameraSet(wl.cameras, g.sizes)
    tgt = torch.from_numpy(np.concatenate([t.reshape(3, -1) for t in wl.targets], axis=1)).cuda()
    step = pipeline.TrainStep(g, cams, tgt, mode="fused", keep_image=False)
    tb = autotune.tune(step, cache_path=autotune.DEFAULT_CACHE) if tune else None
    st_ms = stage_times(step, steps, warmup)
    executed = executed_pairs(step)
    graph = pipeline.GraphStep(step)
    ms_b = time_steps(graph, steps, warmup)
    if step.overflowed():
        raise SystemExit(f"config {cfg}: list overflow in the captured step")
    E, K = step.E_fwd, step.K
    roof = roofline_of(st_ms, step.E_fwd, step.E_bwd, executed)
    del graph, step
    torch.cuda.empty_cache()
    targets = [torch.from_numpy(t.reshape(3, -1)).cuda() for t in wl.targets]
    per_view_ms, per_view_tuning = {}, {}
    for mode in ("fused", "separate"):
        per_view = pipeline.PerViewSteps(g, wl.cameras, targets, mode=mode)
        tv = (autotune.tune_callable(autotune.per_view_key(mode, g, cams, K), per_view,
                                     cache_path=autotune.DEFAULT_CACHE) if tune else None)
        per_view_ms[mode] = time_steps(per_view, steps, warmup)
        per_view_tuning[mode] = tv["tuning"] if tv else None
        del per_view
        torch.cuda.empty_cache()
    autotune.apply(autotune.default_tuning())
    ms_v, ms_s = per_view_ms["fused"], per_view_ms["separate"]
    log(f"config {cfg}: batched {ms_b:.3f} ms, per-view {ms_v:.3f} ms (separate launches {ms_s:.3f} ms)")
    return {"workload": wl.name, "views": cams.n_cams, "n_gaussians": g.n, "E_fwd": E, "E_bwd": roof["E_bwd"],
            "K": K, "stages_ms": st_ms, "roofline": roof,
            "batched_ms_per_step": ms_b, "per_view_ms_per_step": ms_v,
            "batched_evals_per_s": E / (ms_b * 1e-3), "per_view_evals_per_s": E / (ms_v * 1e-3),
            "speedup": ms_v / ms_b, "batched_ms_per_view": ms_b / cams.n_cams,
            "per_view_separate_ms_per_step": ms_s, "speedup_vs_separate": ms_s / ms_b,
            "batched_tuning": tb["tuning"] if tb else None, "per_view_tuning": per_view_tuning["fused"],
            "per_view_separate_tuning": per_view_tuning["separate"]}


def autograd_steps(wl):
    """One training step through torch.autograd: the fused L2 form (autograd.l2_loss, a
    torch.autograd.Function) and loss.backward(), gradients landing in the parameters' .grad;
    and, for comparison, the image form (autograd.render, separate forward and backward
    kernels) with the L2 loss in torch."""
    import numpy as np
    import torch
    from paper_2312_02121_amd.autograd import l2_loss, render
    sizes = [s["opacities"].shape[0] for s in wl.scenes]
    ps = [torch.tensor(np.concatenate([np.asarray(s[k]) for s in wl.scenes], axis=-1), device="cuda",
                       requires_grad=True) for k in ("means", "quats", "scales", "colors", "opacities")]
    tgt = torch.from_numpy(np.concatenate([t.reshape(3, -1) for t in wl.targets], axis=1)).cuda()

    def fused():
        for p in ps:
            p.grad = None                 # an optimiser's zero_grad(set_to_none=True)
        l2_loss(*ps, wl.cameras, tgt, scene_sizes=sizes).backward()

    tgt_img = [torch.from_numpy(t).cuda() for t in wl.targets]

    def image():
        for p in ps:
            p.grad = None
        imgs = render(*ps, wl.cameras, scene_sizes=sizes)
        sum(((i - t) ** 2).sum() for i, t in zip(imgs, tgt_img)).backward()
    return fused, image


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--mode", choices=("fused", "separate"), default="fused")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-autograd", action="store_true")
    ap.add_argument("--oracle-legs", action="store_true",
                    help="only time the FP64 oracle: every workload on all host cores, c1 and c2 on one core "
                         "(minutes of CPU time; prints one JSON object)")
    ap.add_argument("--no-tune", action="store_true", help="keep the library's default launch tuning")
    ap.add_argument("--tuning", type=str, default=None,
                    help="JSON launch tuning to apply instead of searching (profiling runs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB three times (a known-size kernel "
                         "for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE readings)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the rasterizer is built and measured on a single MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    if args.oracle_legs:
        print(json.dumps({"oracle_legs": oracle_legs()}), flush=True)
        return

    import numpy as np
    import torch

    from paper_2312_02121_amd import abi, autotune, pipeline, synth

    torch.cuda.set_device(0)
    if abi.gs_device_check() != abi.GS_OK:
        raise SystemExit("not a gfx950 device")
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 launches reading and writing {args.copy_calibration_mib} MiB each")
        del src, dst
    wl = synth.make_config(args.config)
    g = pipeline.GaussianSet(wl.scenes)
    cams = pipeline.CameraSet(wl.cameras, g.sizes)
    targets = torch.from_numpy(np.concatenate([t.reshape(3, -1) for t in wl.targets], axis=1)).cuda()
    step = pipeline.TrainStep(g, cams, targets, mode=args.mode)
    log(f"K={step.K} E_fwd={step.E_fwd} E_bwd={step.E_bwd} P={cams.n_splats} pixels={cams.n_pixels}")
    tuned = None
    if args.tuning:
        autotune.apply({**autotune.default_tuning(), **json.loads(args.tuning)})
    elif not args.no_tune:
        # launch tuning for this workload: recorded in the package's tuning cache, else
        # searched, before anything is timed
        tuned = autotune.tune(step, cache_path=autotune.DEFAULT_CACHE)
        log(f"autotuned {tuned['tuning']}: {tuned['default_ms']:.4f} -> {tuned['ms']:.4f} ms "
            f"({tuned['evaluated']} candidates, {tuned['seconds']:.1f} s, cached {tuned['cached']})")

    # per-stage times (eager launches, events between stages on the launch stream)
    stage_ms = stage_times(step, args.steps, args.warmup)
    log("stages (ms): " + " ".join(f"{k}={v:.4f}" for k, v in stage_ms.items()))
    executed = executed_pairs(step) if args.mode == "fused" else None

    # the timed step: the whole path, captured once in a HIP graph and replayed
    runner = step if args.no_graph else pipeline.GraphStep(step)
    ms_step, per_step = time_steps_detail(runner, args.steps, args.warmup)
    if step.overflowed():
        raise SystemExit("intersection list overflowed its capacity during the timed steps")
    log(f"step {ms_step:.4f} ms ({'eager' if args.no_graph else 'graph'})")

    roofline = roofline_of(stage_ms, step.E_fwd, step.E_bwd, executed)
    roofline["traffic"] = traffic_from_profiles(roofline["kernel"])

    views = cams.n_cams
    line = {
        "metric": METRIC, "value": step.E_fwd / (ms_step * 1e-3), "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "n_gaussians": g.n, "views": views, "width": int(cams.host[0]["width"]),
                   "height": int(cams.host[0]["height"]), "K": step.K, "E_fwd": step.E_fwd, "E_bwd": step.E_bwd,
                   "E_dense": e_dense(step), "ms_per_view": ms_step / views, "mode": args.mode,
                   "graph": not args.no_graph,
                   "parallelism": "single-gpu", "tuning": autotune.current()},
        "step_ms_median_p10_p90": [float(np.median(per_step)), float(np.percentile(per_step, 10)),
                                   float(np.percentile(per_step, 90))],
        "stages_ms": stage_ms,
        "roofline": roofline,
        "autotune": None if tuned is None else {k: tuned[k] for k in ("default_ms", "ms", "evaluated", "seconds",
                                                                     "cached")},
    }
    del runner
    if not args.no_autograd:
        fused, image = autograd_steps(wl)
        line["autograd_ms_per_step"] = time_steps(fused, args.steps, args.warmup)
        line["autograd_image_form_ms_per_step"] = time_steps(image, max(3, args.steps // 4), 2)
        log(f"autograd: fused L2 form {line['autograd_ms_per_step']:.4f} ms/step, image form "
            f"{line['autograd_image_form_ms_per_step']:.3f} ms/step")
    if not args.no_batched:
        del step
        torch.cuda.empty_cache()
        line["batched"] = {f"c{c}": batched_vs_per_view(c, max(3, args.steps // 4), 2, not args.no_tune)
                           for c in (4, 5)}
    if not args.no_cpu_baseline and args.config in (1, 2, 3):
        line["cpu_baseline"] = cpu_baseline(wl, line["config"]["E_fwd"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
