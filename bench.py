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
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12     # fp32 VALU lane-ops/s, non-packed: 39.3 T
HBM_PEAK_GBS = 8000.0
# algorithmic VALU lane-operations per Gaussian-pixel pair (exp2 and rcp count 4)
SLOTS_FWD = 21
SLOTS_BWD = 46
KERNEL_OF_STAGE = {"rasterize_fwd": "raster_fwd_kernel", "rasterize_bwd": "raster_bwd_kernel"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2312_02121_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + fh.read())
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
    return {"value": E_fwd / t, "unit": "evals/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"the whole 1M-Gaussian 1920x1080 step (FP64 oracle, OpenMP), median of {repeats} runs",
            "seconds_per_step": t}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the rasterizer is built and measured on a single MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2312_02121_amd import abi, pipeline, synth

    torch.cuda.set_device(0)
    if abi.gs_device_check() != abi.GS_OK:
        raise SystemExit("not a gfx950 device")
    wl = synth.make_config(args.config)
    g = pipeline.GaussianSet(wl.scenes)
    cams = pipeline.CameraSet(wl.cameras, g.sizes)
    targets = torch.from_numpy(np.concatenate([t.reshape(3, -1) for t in wl.targets], axis=1)).cuda()
    step = pipeline.TrainStep(g, cams, targets)
    log(f"K={step.K} E_fwd={step.E_fwd} E_bwd={step.E_bwd} P={cams.n_splats} pixels={cams.n_pixels}")

    n_st = len(step.STAGES)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(n_st + 1)] for _ in range(args.steps)]
    t_start, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for k in range(args.steps):
        step(events=evs[k])
    t_end.record()
    torch.cuda.synchronize()
    if step.overflowed():
        raise SystemExit("intersection list overflowed its capacity during the timed steps")
    total_ms = t_start.elapsed_time(t_end)
    ms_step = total_ms / args.steps
    stage_ms = {name: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(args.steps)]))
                for i, name in enumerate(step.STAGES)}
    log("stages (ms): " + " ".join(f"{k}={v:.4f}" for k, v in stage_ms.items()))

    work = {"rasterize_fwd": SLOTS_FWD * step.E_fwd, "rasterize_bwd": SLOTS_BWD * step.E_bwd}
    dom = max(work, key=lambda s: stage_ms[s])
    achieved = work[dom] / (stage_ms[dom] * 1e-3) / 1e12
    traffic = traffic_from_profiles(KERNEL_OF_STAGE[dom])
    roofline = {"bound": "alu", "kernel": KERNEL_OF_STAGE[dom], "achieved": achieved, "peak": VALU_PEAK_TOPS,
                "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic,
                "other": {s: (work[s] / (stage_ms[s] * 1e-3) / 1e12) / VALU_PEAK_TOPS for s in work}}

    views = cams.n_cams
    line = {
        "metric": METRIC, "value": step.E_fwd / (ms_step * 1e-3), "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "n_gaussians": g.n, "views": views, "width": int(cams.host[0]["width"]),
                   "height": int(cams.host[0]["height"]), "K": step.K, "E_fwd": step.E_fwd, "E_bwd": step.E_bwd,
                   "ms_per_view": ms_step / views, "parallelism": "single-gpu"},
        "stages_ms": stage_ms,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline and args.config in (1, 2, 3):
        line["cpu_baseline"] = cpu_baseline(wl, step.E_fwd)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
