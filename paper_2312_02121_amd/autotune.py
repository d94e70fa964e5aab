"""Autotuner of the rasterizer's launch tuning (gs_tuning) for one batch of cameras.

The work list, the sort and the persistent launch have eight knobs (see gs_tuning in the
C header): the list length at which a tile is split, the number of parts (16x8 halves or
16x4 quarters), the persistent grid size in waves per compute unit, whether a wave raises
its priority on split items, whether the first tile-sort pass generates the list entries
itself, how many work items a wave takes per atomic on the work counter, and the list
length from which a wave raises its priority on an unsplit tile, and the number of list
segments a split tile's backward is walked in by the fused kernel. None of them changes a
result beyond the rounding order of gradient sums, only the time.

``tune`` times a full training step (project, bin and sort, fused forward + loss +
backward, project_bwd) captured in a HIP graph under each candidate and keeps the fastest.
The search is a coordinate descent from the best of the library default and a few seeds
(SEEDS): one knob at a time over its values (KNOBS; item_grab stays at 1), keeping the best
value before moving to the next knob, up to three rounds; each candidate is timed as the
best of three runs. Results are
cached in a JSON file keyed by a signature of the workload (cameras, resolutions, Gaussian
count, and the list length rounded to a power of two), so a later process with the same
kind of batch applies the recorded tuning without searching; ``python -m
paper_2312_02121_amd.autotune`` records the benchmark workloads.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Callable

import torch

from . import abi

KNOBS = {
    "split_len": (128, 256, 512, 1024, 1 << 30),
    "split_parts": (2, 4),
    "waves_per_cu": (16, 32),
    "split_priority": (0, 1),
    "generate_entries": (0, 1),
    "prio_len": (0, 96, 128, 192, 256, 512),
    "bwd_segs": (1, 2, 4),
    "atomic_lanes": (2, 4, 8),
    "batch": (32, 64),
    "big_tiles": (0, 256, 1024),
}
# item_grab is left at 1: taking several items per atomic put consecutive long items (the
# head of the longest-first list) on one wave and made the 1M-Gaussian and the 32-view
# steps 2-6x slower, with no gain at 16 views (measured on MI355X).


# Starting points besides the default: knobs that only pay off together (finer splitting
# needs the longest walks cut into backward segments and prioritised), which a search that
# moves one knob at a time does not reach from the default.
SEEDS = (
    {"split_len": 512, "split_parts": 4, "split_priority": 1, "prio_len": 256, "bwd_segs": 2},
    {"split_len": 1024, "split_parts": 4, "split_priority": 1, "bwd_segs": 2},
)


def default_tuning() -> dict:
    return {"split_len": 256, "split_parts": 4, "waves_per_cu": 32, "split_priority": 1, "generate_entries": 0,
            "item_grab": 1, "prio_len": 0, "bwd_segs": 1, "atomic_lanes": 4, "batch": 64, "big_tiles": 0}


def apply(t: dict):
    """Sets the tuning; knobs missing from t (e.g. a tuning recorded before a knob existed)
    take their default."""
    abi.gs_set_tuning(abi.GsTuning(**{k: int(v) for k, v in {**default_tuning(), **t}.items()}))


def current() -> dict:
    return abi.gs_get_tuning().as_dict()


def signature_of(g, cams, K: int) -> str:
    """Workload key: camera count, sizes, Gaussians, splats and log2 of the list length."""
    sizes = sorted({(int(c["width"]), int(c["height"])) for c in cams.host})
    return json.dumps({"views": int(cams.n_cams), "sizes": sizes, "gaussians": int(g.n),
                       "splats": int(cams.n_splats), "log2K": int(round(math.log2(max(K, 1))))},
                      sort_keys=True)


def signature(step) -> str:
    return signature_of(step.g, step.cams, step.K)


def per_view_key(mode: str, g, cams, K: int) -> str:
    """Cache key of the one-view-per-launch form (PerViewSteps) of a batched workload: the
    fused kernels per view, or the conventional separate forward and backward launches."""
    return ("per_view:" if mode == "separate" else f"per_view_{mode}:") + signature_of(g, cams, K)


def _time_graph(step, steps: int, warmup: int, repeats: int = 3) -> float:
    """Mean ms per replay of the step captured as a graph: the best of `repeats` runs of
    `steps` replays (run-to-run noise on a shared GPU is one-sided)."""
    from .pipeline import GraphStep
    graph = GraphStep(step)
    for _ in range(warmup):
        graph()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(repeats):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            graph()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) / steps)
    if step.overflowed():
        raise RuntimeError("list capacity overflow while tuning")
    del graph
    return best


def time_eager(fn, steps: int, warmup: int) -> float:
    """Mean ms per call of fn() over `steps` calls after `warmup`."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def search(measure: Callable[[], float], rounds: int = 3, log: Callable[[str], None] | None = None) -> dict:
    """Coordinate descent over KNOBS from the default; measure() times the workload under
    the tuning currently applied. Applies and returns the best."""
    t0 = time.perf_counter()
    seen: dict = {}

    def run(t: dict) -> float:
        k = tuple(sorted(t.items()))
        if k not in seen:
            apply(t)
            seen[k] = measure()
            if log:
                log(f"tuning {t}: {seen[k]:.4f} ms")
        return seen[k]

    best = default_tuning()
    default_ms = best_ms = run(best)
    for seed in SEEDS:
        cand = {**default_tuning(), **seed}
        ms = run(cand)
        if ms < best_ms:
            best, best_ms = cand, ms
    for _ in range(rounds):
        improved = False
        for knob, values in KNOBS.items():
            for v in values:
                if v == best[knob]:
                    continue
                cand = {**best, knob: v}
                ms = run(cand)
                if ms < best_ms * 0.995:
                    best, best_ms, improved = cand, ms, True
        if not improved:
            break
    apply(best)
    return {"tuning": best, "ms": best_ms, "default_ms": default_ms, "evaluated": len(seen),
            "seconds": time.perf_counter() - t0}


DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def _load(cache_path: str | None) -> dict:
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            return json.load(fh)
    return {}


def _store(cache_path: str, cache: dict):
    os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
    with open(cache_path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)


def tune(step, steps: int = 10, warmup: int = 2, rounds: int = 3, cache_path: str | None = None,
         update_cache: bool = False, log: Callable[[str], None] | None = None) -> dict:
    """Finds the fastest tuning for `step` (a pipeline.TrainStep, timed as a captured graph),
    applies it and returns {"tuning", "ms", "default_ms", "evaluated", "seconds", "cached"}.
    A tuning cached under the step's signature in `cache_path` is applied without a search;
    with update_cache a fresh search result is written back."""
    key = signature(step)
    cache = _load(cache_path)
    if key in cache:
        apply(cache[key]["tuning"])
        return {**cache[key], "cached": True}
    res = search(lambda: _time_graph(step, steps, warmup), rounds=rounds, log=log)
    if cache_path and update_cache:
        cache[key] = res
        _store(cache_path, cache)
    return {**res, "cached": False}


def tune_callable(key: str, fn, steps: int = 2, warmup: int = 1, cache_path: str | None = None,
                  update_cache: bool = False, log: Callable[[str], None] | None = None) -> dict:
    """As tune, for any callable step (timed eagerly), cached under `key`."""
    cache = _load(cache_path)
    if key in cache:
        apply(cache[key]["tuning"])
        return {**cache[key], "cached": True}
    res = search(lambda: time_eager(fn, steps, warmup), log=log)
    if cache_path and update_cache:
        cache[key] = res
        _store(cache_path, cache)
    return {**res, "cached": False}


def main():
    """Searches the launch tuning of the benchmark workloads on this GPU and records it in
    the cache (default: tuned.json beside this file), for the batched step and, with
    --per-view, for the one-view-per-launch form."""
    import argparse

    import numpy as np

    from . import pipeline, synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", type=int, nargs="+", default=[3, 4, 5])
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--per-view", action="store_true")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    for cfg in args.configs:
        wl = synth.make_config(cfg)
        g = pipeline.GaussianSet(wl.scenes)
        cams = pipeline.CameraSet(wl.cameras, g.sizes)
        tgt = torch.from_numpy(np.concatenate([t.reshape(3, -1) for t in wl.targets], axis=1)).cuda()
        apply(default_tuning())
        step = pipeline.TrainStep(g, cams, tgt, mode="fused", keep_image=False)
        key = signature(step)
        cache = _load(args.out)
        cache.pop(key, None)
        _store(args.out, cache)
        res = tune(step, cache_path=args.out, update_cache=True, log=print)
        print(f"c{cfg}: {res['tuning']} {res['default_ms']:.4f} -> {res['ms']:.4f} ms", flush=True)
        if args.per_view:
            K = step.K
            del step
            torch.cuda.empty_cache()
            targets = [torch.from_numpy(t.reshape(3, -1)).cuda() for t in wl.targets]
            for mode in ("fused", "separate"):
                per_view = pipeline.PerViewSteps(g, wl.cameras, targets, mode=mode)
                pkey = per_view_key(mode, g, cams, K)
                cache = _load(args.out)
                cache.pop(pkey, None)
                _store(args.out, cache)
                res = tune_callable(pkey, per_view, cache_path=args.out, update_cache=True, log=print)
                print(f"c{cfg} per view ({mode}): {res['tuning']} {res['default_ms']:.4f} -> {res['ms']:.4f} ms",
                      flush=True)
                del per_view
        torch.cuda.empty_cache()
    apply(default_tuning())


if __name__ == "__main__":
    main()
