"""Autotuner for the launch shape of the batched form (and the plain kernels).

The paper sets threads per block, number of blocks and registers by hand for
every portability layer and reports that library defaults cost about 30 %
(Sec. 5, NVIDIA GPU results).  Here the search is automatic: every candidate configuration is
timed with HIP events on the caller's sample (after a warm-up), and the
fastest is returned and cached in a JSON file keyed by the workload's shape,
so that later runs reuse it.

Search space
  batched form:  block in {64, 128, 256} x tracks_per_thread in {1, 2} x
                 schedule in {dynamic, static} x waves_mult in {1, 2} x
                 state layout in {AoS, SoA, AoSoA-64}
  plain form:    block in {64, 128, 256} x layout in {SoA, AoS, AoSoA-64}
"""
from __future__ import annotations

import itertools
import json
import os
import time

from . import kf as K

BATCHED_SPACE = {
    "block": (64, 128, 256),
    "tpt": (1, 2),
    "schedule": (K.SCHED_DYNAMIC, K.SCHED_STATIC),
    "waves_mult": (1, 2),
    "layout": ("aos", "soa", "aosoa64"),
}
# plain step: block size x the layouts, AoSoA with 16 to 128 tracks per block
PLAIN_SPACE = {"block": (64, 128, 256), "layout": ("soa", "aos", "aosoa16", "aosoa32", "aosoa64", "aosoa128")}

LAYOUTS = {"aos": K.AOS, "soa": K.SOA, "aosoa16": K.aosoa(16), "aosoa32": K.aosoa(32), "aosoa64": K.aosoa(64),
           "aosoa128": K.aosoa(128)}


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "paper_2409_09228_amd", "tune.json")


def candidates(space: dict):
    keys = list(space)
    for vals in itertools.product(*(space[k] for k in keys)):
        yield dict(zip(keys, vals))


def shape_key(form: str, sample: dict, flags: int) -> str:
    import numpy as np
    nl = np.asarray(sample["nlay"])
    geom = np.asarray(sample["geom"])
    return (f"{form}:n={len(nl)}:L={sample['hit_pos'].shape[0]}:sum_layers={int(nl.sum())}:"
            f"cyl={int((geom != 0).sum())}:flags={flags}")


def load_cache(path: str | None = None) -> dict:
    path = path or default_cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str | None = None) -> None:
    path = path or default_cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(fn, reps: int, stream) -> float:
    import torch
    t_w = time.perf_counter()
    while time.perf_counter() - t_w < 0.05:
        fn()
        torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_batched(sample: dict, flags: int = 0, reps: int = 10, space: dict | None = None,
                 cache_path: str | None = None, use_cache: bool = True) -> dict:
    """Best batched configuration for this sample; returns
    {"config": {...}, "ms": t, "tried": [(config, ms), ...]}."""
    import torch
    key = shape_key("batched", sample, flags)
    cache = load_cache(cache_path) if use_cache else {}
    if use_cache and key in cache:
        return cache[key]
    stream = torch.cuda.current_stream()
    staged = {}
    tried = []
    for c in candidates(space or BATCHED_SPACE):
        if c["layout"] not in staged:
            staged[c["layout"]] = K.stage_batched(sample, LAYOUTS[c["layout"]])
        st = staged[c["layout"]]
        outs = (torch.empty_like(st["par"]), torch.empty_like(st["cov"]))
        chi2 = torch.empty(st["n"], device="cuda")
        status = torch.empty(st["n"], dtype=torch.int32, device="cuda")
        launch = K.BatchedLauncher(st, outs, chi2, status, flags=flags,
                                   tune=(c["block"], c["tpt"], c["schedule"], c["waves_mult"]), stream=stream)
        tried.append((c, _time(launch, reps, stream)))
        K.release_graphs()
    best = min(tried, key=lambda x: x[1])
    res = {"config": best[0], "ms": best[1], "tried": tried}
    if use_cache:
        cache[key] = res
        save_cache(cache, cache_path)
    return res


def tune_plain(sample: dict, flags: int = 0, reps: int = 10, space: dict | None = None,
               cache_path: str | None = None, use_cache: bool = True) -> dict:
    """Best plain-kernel configuration (single-geometry sample)."""
    import torch
    key = shape_key("plain", sample, flags)
    cache = load_cache(cache_path) if use_cache else {}
    if use_cache and key in cache:
        return cache[key]
    stream = torch.cuda.current_stream()
    staged = {}
    tried = []
    geom = int(sample["geom"][0])
    for c in candidates(space or PLAIN_SPACE):
        if c["layout"] not in staged:
            staged[c["layout"]] = K.stage_sample(sample, LAYOUTS[c["layout"]])
        st = staged[c["layout"]]
        outs = (torch.empty_like(st["par"]), torch.empty_like(st["cov"]))
        launch = K.StepLauncher(geom, st["par"], st["cov"], st["hit_pos"], st["hit_cov"], st["layers"], st["bz"],
                                st["n"], out=outs, chi2=torch.empty(st["n"], device="cuda"),
                                status=torch.empty(st["n"], dtype=torch.int32, device="cuda"), nlay=st["nlay"],
                                layout=st["layout"], flags=flags, tune=(c["block"], 1), stream=stream)
        tried.append((c, _time(launch, reps, stream)))
    best = min(tried, key=lambda x: x[1])
    res = {"config": best[0], "ms": best[1], "tried": tried}
    if use_cache:
        cache[key] = res
        save_cache(cache, cache_path)
    return res
