#!/usr/bin/env python3
"""Throughput of the batched Kalman-filter step on one MI355X.

One step = one launch of the whole step (propagate + Kalman update through
every layer of every track) over the 100-event x 9600-track plane sample
(960,000 tracks x 20 planes = 19.2M track-layer updates), inputs resident in
HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--layout soa|aosoaB]
                    [--flags 0|1|3] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "track-layer updates/sec (propagate+Kalman) FP32 at 1 GPU; % of HBM/VALU roofline"
DEFAULT_WORKLOAD = "p2z_100x9600"
P2R_WORKLOAD = "p2r_100x9600"
P2R_LAYOUT = "aos"  # the barrel step's fastest layout (the autotuner's pick on the barrel sample)
HBM_PEAK_GBS = 8000.0
# kf_propagate_update_batched's launch shape when none is given (block,
# tracks per thread, schedule, grid multiple), as include/kf.h states it
BATCHED_DEFAULT_SHAPE = (128, 1, 1, 2)
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6

# Mean Newton steps of the barrel crossing search per update on the barrel
# sample (the search stops a lane once its step is below 1e-5 of the path,
# at most five steps); tests/test_bench.py checks it against the oracle's
# single-precision search on sampled tracks of that workload.
NEWTON_STEPS_P2R = 2.17
# Algorithmic cost of one track-layer update (counted from the method's
# formulation step by step, FMA = 2 flops, each sin/cos/reciprocal/sqrt =
# 1 flop).  p2r: 729 flops outside the search's steps plus 27 per step.
FLOPS_PER_UPDATE = {0: 391.0, 1: round(729.0 + 27.0 * NEWTON_STEPS_P2R, 1)}
# The VALU side of the roofline charges each transcendental at its cost in
# FP32 instructions -- a sin/cos pair 40 flops, a reciprocal, division or
# square root 20: p2z has 3 sin/cos pairs and 1 reciprocal per update
# (391 - 7 + 3 x 40 + 20 = 524); p2r 3 pairs and 3 reciprocals or square
# roots outside the steps and one of each per step (900 + 84 per step).  The
# binding roofline is the one of the two (HBM bytes, charged VALU flops) with
# the larger fraction of its published peak.
FLOPS_CHARGED_PER_UPDATE = {0: 524.0, 1: round(900.0 + 84.0 * NEWTON_STEPS_P2R, 1)}
FP32_PEAK_NONPACKED_TFLOPS = 78.6  # 256 CU x 64 lanes x 2 flops (FMA) x 2.4 GHz
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2409_09228_amd", "csrc")


# the sources the plain step kernel is compiled from
STEP_SOURCES = ("kf_step.hip", "kf_track.h", "kf_device.h", "kf_lanes.h", "kf_internal.h")


def kernel_source_digest() -> str:
    """sha256 over the step kernel's sources and build flags: counter figures
    are only valid for the code they were taken on."""
    import hashlib
    from paper_2409_09228_amd import build as B
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    h.update(" ".join(f for f in B.FLAGS if not f.startswith("-I")).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, layout: str, flags: int):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources for this configuration; else None."""
    path = os.path.join(PROFILES, f"kf_step_{workload}_{layout}_traffic.md")
    if flags != 0 or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_digest():
        return None
    try:
        return int(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None
# Bytes that must move per track (parameters + covariance in and out, chi2,
# status) and per layer (hit position + hit covariance), float32.
TRACK_BYTES = (6 + 21) * 4 * 2 + 4 + 4
LAYER_BYTES = (3 + 6) * 4


def parse_layout(s: str):
    from paper_2409_09228_amd import kf as K
    if s == "soa":
        return K.SOA
    if s == "aos":
        return K.AOS
    if s.startswith("aosoa"):
        return K.aosoa(int(s[5:]))
    raise SystemExit(f"unknown layout {s}")


def cpu_identity() -> dict:
    """The host CPU as /proc/cpuinfo and lscpu name it (vendor, family,
    model and stepping numbers as well: a virtualised host may shorten the
    model string)."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                if info:
                    break
                continue
            k, v = (x.strip() for x in line.split(":", 1))
            if k in ("vendor_id", "cpu family", "model", "model name", "stepping") and k not in info:
                info[k] = v
            if k == "flags" and "flags" not in info:
                fl = v.split()
                info["flags"] = " ".join(f for f in ("avx2", "fma", "avx512f") if f in fl)
    except OSError:
        pass
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
                info["lscpu " + k.strip()] = v.strip()
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(sample, n_tracks: int, min_seconds: float = 10.0, build: str = ""):
    """The FP64 oracle on the first n_tracks of the same sample with all host
    cores, repeated until at least min_seconds of wall time (a bounded
    sample of the workload); then one thread on a twentieth of it for about
    a tenth of that time."""
    import oracle as O
    from paper_2409_09228_amd import synth as S
    idx = np.arange(min(n_tracks, sample["par"].shape[0]))
    sub = S.subset(sample, idx)
    upd = int(sub["nlay"].sum())
    threads = len(os.sched_getaffinity(0))
    passes = []
    t0 = time.perf_counter()
    while not passes or time.perf_counter() - t0 < min_seconds:
        tp = time.perf_counter()
        O.run_sample(sub, nthreads=threads)
        passes.append(time.perf_counter() - tp)
    reps = len(passes)
    dt = time.perf_counter() - t0
    med = float(np.median(passes))
    one = S.subset(sample, idx[: max(1, len(idx) // 20)])
    u1 = int(one["nlay"].sum())
    r1 = 0
    t1 = time.perf_counter()
    while r1 == 0 or time.perf_counter() - t1 < min_seconds / 10:
        O.run_sample(one, nthreads=1)
        r1 += 1
    d1 = time.perf_counter() - t1
    ident = cpu_identity()
    return {"value": upd / med, "unit": "track-layer updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": ident.get("lscpu Model name") or ident.get("model name", ""),
            "cpu": ident, "build": build,
            "sample": f"first {len(idx)} tracks ({upd} track-layer updates) of the same sample, FP64, OpenMP "
                      f"over tracks; median of {reps} passes ({dt:.1f} s wall in all)",
            "mean_value": upd * reps / dt,
            "single_thread_value": u1 * r1 / d1,
            "single_thread_sample": f"first {one['par'].shape[0]} tracks ({u1} updates), 1 thread, "
                                    f"{r1} passes in {d1:.1f} s"}


# floors of the floored relative parameter error: cm, cm, cm, 1/GeV, rad, rad
PAR_FLOOR = np.array([1.0, 1.0, 1.0, 0.1, 1.0, 1.0])
PAR_NAMES = ("x", "y", "z", "kappa", "phi", "theta")


def _sym6(P21):
    out = np.zeros(P21.shape[:-1] + (6, 6))
    k = 0
    for i in range(6):
        for j in range(i + 1):
            out[..., i, j] = out[..., j, i] = P21[..., k]
            k += 1
    return out


def output_errors(ref, got, geom: int) -> dict:
    """Per-output error of `got` against the FP64 reference `ref` (both
    (par [n,6], cov [n,21], chi2 [n], status [n])): the floored relative
    error of each parameter, |d p| / max(|p|, floor), floors (1 cm, 1 cm,
    1 cm, 0.1 /GeV, 1 rad, 1 rad), phi compared modulo 2 pi; the largest
    parameter error in units of its standard deviation; the covariance in
    correlation units |d C_ij| / sqrt(C_ii C_jj) (on planes without the z row,
    which is zero on both sides; on cylinders x and y normalised by the
    transverse variance, since the radial direction has none); the relative
    error of each diagonal element, unfloored; chi2 relative (floored at 1);
    and the status words that differ."""
    po, co, c2, st = ref
    qo, qc, q2, qs = got
    d = qo - po
    d[:, 4] = np.angle(np.exp(1j * d[:, 4]))
    P, Q = _sym6(co), _sym6(qc)
    v = np.diagonal(P, axis1=-2, axis2=-1).copy()
    if geom == 1:
        v[:, 0] = v[:, 1] = v[:, 0] + v[:, 1]
    keep = [0, 1, 3, 4, 5] if geom == 0 else list(range(6))
    norm = np.sqrt(v[:, :, None] * v[:, None, :])
    if geom == 0:
        norm[:, 2, :] = np.inf
        norm[:, :, 2] = np.inf
    dg = np.abs(np.diagonal(Q - P, axis1=-2, axis2=-1))[:, keep] / np.diagonal(P, axis1=-2, axis2=-1)[:, keep]
    fl = (np.abs(d) / np.maximum(np.abs(po), PAR_FLOOR)).max(0)
    out = {name: float(f"{fl[i]:.3g}") for i, name in enumerate(PAR_NAMES)}
    out["par_sigma"] = float(f"{(np.abs(d[:, keep]) / np.sqrt(v[:, keep])).max():.3g}")
    out["cov_corr"] = float(f"{(np.abs(Q - P) / norm).max():.3g}")
    out["cov_diag_rel_raw"] = float(f"{dg.max():.3g}")
    out["chi2_rel"] = float(f"{(np.abs(q2 - c2) / np.maximum(c2, 1.0)).max():.3g}")
    out["status_mismatch"] = int(np.sum(st != qs))
    return out


def precision_errors(sample, res, n_sample: int = 20000) -> dict:
    """The GPU's results for precision flags 0 (FP32), 1 (FP64 inverse and
    gain) and 3 (FP64 inverse, gain and Joseph update) on the full workload,
    launched as timed, against the FP64 oracle on n_sample evenly spaced
    tracks (the last one included).  The oracle takes the plain update for
    flags 0 and 1, the Joseph form for flag 3."""
    import torch
    import oracle as O
    from paper_2409_09228_amd import kf as K
    from paper_2409_09228_amd import synth as S
    n = sample["par"].shape[0]
    idx = np.unique(np.linspace(0, n - 1, min(n_sample, n)).astype(np.int64))
    sub = S.subset(sample, idx)
    geom = int(sample["geom"][0])
    st = res["staged"]
    out = {"tracks_compared": int(len(idx)), "workload": res["config"]["workload"],
           "reference": "FP64 oracle (plain update for flags 0 and 1, Joseph form for flag 3)"}
    refs = {}
    for flags in (0, 1, 3):
        joseph = bool(flags & 2)
        if joseph not in refs:
            refs[joseph] = O.run_sample(sub, joseph=joseph)
        po, co, c2, ss = res["outputs"]
        launch = K.StepLauncher(geom, st["par"], st["cov"], st["hit_pos"], st["hit_cov"], st["layers"], st["bz"],
                                st["n"], out=(po, co), chi2=c2, status=ss, nlay=st["nlay"], layout=st["layout"],
                                flags=flags, tune=res["tune"], stream=torch.cuda.current_stream())
        launch()
        torch.cuda.synchronize()
        p, c = K.results_to_logical(st, po, co)
        got = (p[idx], c[idx], c2.cpu().numpy().astype(np.float64)[idx], ss.cpu().numpy()[idx])
        out[f"flags_{flags}"] = output_errors(refs[joseph], got, geom)
    return out


def oracle_leg(sample, args, head, r_sample=None, r=None) -> dict:
    """Everything bench.py does with the FP64 oracle, on the host: the CPU
    baseline (the oracle built for this host with -O3 -march=native, timed on
    a bounded part of the workload) and the per-output precision error of the
    GPU's results on sampled tracks."""
    import tempfile
    import oracle as O
    build = "g++ " + " ".join(O.CXXFLAGS) + " -march=native"
    try:
        tmp = tempfile.mkdtemp(prefix="kf_oracle_")
        O.use_native_build(tmp)
    except Exception as e:  # noqa: BLE001 -- the in-tree build still times the oracle
        build = "g++ " + " ".join(O.CXXFLAGS) + f" (in-tree build; -march=native failed: {e})"
    leg = {"cpu_baseline": cpu_baseline(sample, args.cpu_tracks, args.cpu_seconds, build)}
    pe = {"p2z" if int(sample["geom"][0]) == 0 else "p2r": precision_errors(sample, head)}
    if r is not None:
        pe["p2r"] = precision_errors(r_sample, r)
    leg["precision_error"] = pe
    return leg


def plain_roofline(geom: int, n: int, updates: int, ms_step: float, workload: str, layout: str, flags: int,
                   streamed: bool) -> dict:
    """Both fractions of the plain step over one launch: HBM (algorithmic
    bytes) and VALU (algorithmic flops, transcendentals charged); the larger
    one binds."""
    flops = FLOPS_PER_UPDATE[geom] * updates
    flops_c = FLOPS_CHARGED_PER_UPDATE[geom] * updates
    bytes_ = TRACK_BYTES * n + LAYER_BYTES * updates
    sec = ms_step / 1e3
    hbm = bytes_ / sec / 1e9
    tfl = flops / sec / 1e12
    tfl_c = flops_c / sec / 1e12
    fr_hbm = hbm / HBM_PEAK_GBS
    fr_valu = tfl_c / FP32_PEAK_TFLOPS
    if fr_hbm >= fr_valu:
        roof = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(fr_hbm, 4), "traffic": None}
    else:
        roof = {"bound": "alu", "achieved": round(tfl_c, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(fr_valu, 4), "traffic": None}
    roof["intensity_flop_per_byte"] = round(flops / bytes_, 2)
    roof["ridge_flop_per_byte"] = round(FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9), 2)
    traffic = measured_traffic(workload, layout, flags)
    if traffic is not None:
        roof["traffic"] = traffic
    roof["flops_per_update"] = FLOPS_PER_UPDATE[geom]
    roof["flops_per_update_transcendentals_charged"] = FLOPS_CHARGED_PER_UPDATE[geom]
    roof["valu_achieved_TFLOPs_charged"] = round(tfl_c, 3)
    roof["valu_frac_charged"] = round(fr_valu, 4)
    roof["valu_frac_charged_of_nonpacked_peak"] = round(tfl_c / FP32_PEAK_NONPACKED_TFLOPS, 4)
    roof["alu_achieved_TFLOPs"] = round(tfl, 3)
    roof["alu_frac"] = round(tfl / FP32_PEAK_TFLOPS, 4)
    roof["frac_of_nonpacked_fp32_peak"] = round(tfl / FP32_PEAK_NONPACKED_TFLOPS, 4)
    roof["hbm_algorithmic_bytes_per_launch"] = int(bytes_)
    roof["hbm_achieved_GBs"] = round(hbm, 1)
    roof["hbm_frac"] = round(fr_hbm, 4)
    roof["kernel"] = "kf_step_kernel<%d,%d,%s,%s>" % (geom, {0: 0, 1: 1, 3: 2}.get(flags, 0), layout,
                                                   "streamed" if streamed else "counted")
    roof["kernel_source_sha256"] = kernel_source_digest()
    return roof


def time_plain(sample, workload: str, layout_name: str, flags: int, steps: int, warmup: int, tune) -> dict:
    """One plain step per launch over the whole sample, inputs resident in
    HBM: W warm-up launches, then back-to-back launches for at least 500 ms
    more (clocks settle; nothing idles the GPU before the timed region),
    then `steps` launches between two events on the launch stream."""
    import torch
    from paper_2409_09228_amd import kf as K
    layout = parse_layout(layout_name)
    geom = int(sample["geom"][0])
    st = K.stage_sample(sample, layout)
    n = st["n"]
    updates = int(sample["nlay"].sum())
    par_out = torch.empty_like(st["par"])
    cov_out = torch.empty_like(st["cov"])
    chi2 = torch.empty(n, dtype=torch.float32, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    step = K.StepLauncher(geom, st["par"], st["cov"], st["hit_pos"], st["hit_cov"], st["layers"], st["bz"], n,
                          out=(par_out, cov_out), chi2=chi2, status=status, nlay=st["nlay"], layout=layout,
                          flags=flags, tune=tune, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for _ in range(warmup):
        step()
    warm = warmup
    torch.cuda.synchronize()
    t_w = time.perf_counter()
    while time.perf_counter() - t_w < 0.5:
        for _ in range(20):
            step()
        warm += 20
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_step = ms / steps
    ok = int(((status & 0xFF) == 0).sum().item())
    # diagnostics only (not used above): per-launch spread, events between launches
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(min(steps, 50) + 1)]
    ev[0].record(stream)
    for j in range(len(ev) - 1):
        step()
        ev[j + 1].record(stream)
    ev[-1].synchronize()
    per = sorted(ev[j].elapsed_time(ev[j + 1]) for j in range(len(ev) - 1))
    L = int(sample["hit_pos"].shape[0])
    config = {"workload": workload, "tracks": n, "layers": L, "updates_per_step": updates,
              "nominal_updates_per_step": n * L, "layout": layout_name, "precision_flags": flags,
              "tracks_per_s": round(n * steps / (ms / 1e3), 1), "ok_tracks": ok,
              "warmup_launches": warm,
              "warmup_note": "the W launches asked for, then back-to-back launches for >= 0.5 s more",
              "host_wall_s": round(wall, 4), "launch_ms_mean": round(ms_step, 4),
              "per_launch_events_ms": {"median": round(per[len(per) // 2], 4), "min": round(per[0], 4),
                                       "max": round(per[-1], 4),
                                       "note": "diagnostic: each launch between its own pair of events, "
                                               "which adds a gap per launch; the timed figure is "
                                               "launch_ms_mean (back-to-back launches)"}}
    return {"value": updates * steps / (ms / 1e3), "ms_step": ms_step, "config": config,
            "roofline": plain_roofline(geom, n, updates, ms_step, workload, layout_name, flags, st["nlay"] is None),
            "staged": st, "outputs": (par_out, cov_out, chi2, status), "tune": tune}


def time_launches(fn, steps: int, stream):
    """Mean per-call GPU time (ms) of `fn` over `steps` back-to-back calls,
    directly after >= 500 ms of warm-up calls."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t_w = time.perf_counter()
    while time.perf_counter() - t_w < 0.5:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_batched(args, sample):
    """Mixed geometry, uneven layer counts: the persistent graph-replayed
    launch against one plain launch per (geometry, layer count) bucket."""
    import torch
    from paper_2409_09228_amd import kf as K
    from paper_2409_09228_amd import synth as S
    stream = torch.cuda.current_stream()
    tuned = None
    if args.autotune:
        from paper_2409_09228_amd import tune as T
        t0 = time.perf_counter()
        res = T.tune_batched(sample, flags=args.flags, use_cache=False)
        c = res["config"]
        tuned = {"config": c, "search_s": round(time.perf_counter() - t0, 1), "candidates": len(res["tried"]),
                 "worst_ms": round(max(t for _, t in res["tried"]), 4)}
        args.block, args.tpt, args.sched, args.waves_mult, args.layout = (c["block"], c["tpt"], c["schedule"],
                                                                          c["waves_mult"], c["layout"])
    # the batched form's default state layout is AoS (one record per track,
    # gathered by item); an explicit --layout or the autotuner's choice wins
    layout_name = args.layout if args.layout != "soa" or args.autotune else "aos"
    layout = parse_layout(layout_name)
    st = K.stage_batched(sample, layout)
    n = st["n"]
    updates = int(sample["nlay"].sum())
    par_out, cov_out = torch.empty_like(st["par"]), torch.empty_like(st["cov"])
    chi2 = torch.empty(n, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    # no launch shape given: the library's default (tune = NULL)
    shape = None
    if any(v is not None for v in (args.block, args.tpt, args.sched, args.waves_mult)):
        shape = (args.block or BATCHED_DEFAULT_SHAPE[0], args.tpt or BATCHED_DEFAULT_SHAPE[1],
                 BATCHED_DEFAULT_SHAPE[2] if args.sched is None else args.sched,
                 args.waves_mult or BATCHED_DEFAULT_SHAPE[3])
    launch = K.BatchedLauncher(st, (par_out, cov_out), chi2, status, flags=args.flags, tune=shape, stream=stream)
    ms = time_launches(launch, args.steps, stream)
    ok = int(((status & 0xFF) == 0).sum().item())
    # baseline: one launch of the plain kernel per (geometry, layer count) bucket
    launches = []
    if args.no_baseline:
        ms_b = float("nan")
    for g in ((0, 1) if not args.no_baseline else ()):
        for nl in range(int(sample["nlay"].max()) + 1):
            idx = np.nonzero((sample["geom"] == g) & (sample["nlay"] == nl))[0]
            if len(idx) == 0 or nl == 0:
                continue
            sub = S.subset(sample, idx)
            sub["hit_pos"] = sub["hit_pos"][:nl]
            sub["hit_cov"] = sub["hit_cov"][:nl]
            sb = K.stage_sample(sub, K.SOA)
            outs = (torch.empty_like(sb["par"]), torch.empty_like(sb["cov"]))
            launches.append(K.StepLauncher(g, sb["par"], sb["cov"], sb["hit_pos"], sb["hit_cov"], sb["layers"],
                                           sb["bz"], sb["n"], out=outs, chi2=torch.empty(sb["n"], device="cuda"),
                                           status=torch.empty(sb["n"], dtype=torch.int32, device="cuda"),
                                           flags=args.flags, stream=stream))

    def per_bucket():
        for f in launches:
            f()

    if launches:
        ms_b = time_launches(per_bucket, max(1, args.steps // 4), stream)
    # roofline of the whole call (planning included): algorithmic bytes are the
    # hits (36 B per update) and per track the state in and out, chi2, status,
    # layer count, geometry and hit offset (216 + 8 + 4 + 1 + 8 B); flops per
    # update by geometry, transcendentals charged
    sec = ms / 1e3
    nl = np.asarray(sample["nlay"], np.int64)
    g = np.asarray(sample["geom"])
    bytes_ = LAYER_BYTES * updates + (216 + 8 + 4 + 1 + 8) * n
    flops_c = float(sum(FLOPS_CHARGED_PER_UPDATE[k] * nl[g == k].sum() for k in (0, 1)))
    fr_hbm = bytes_ / sec / 1e9 / HBM_PEAK_GBS
    fr_valu = flops_c / sec / 1e12 / FP32_PEAK_TFLOPS
    if fr_hbm >= fr_valu:
        roof = {"bound": "hbm", "achieved": round(bytes_ / sec / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(fr_hbm, 4), "traffic": None}
    else:
        roof = {"bound": "alu", "achieved": round(flops_c / sec / 1e12, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(fr_valu, 4), "traffic": None}
    roof.update(hbm_frac=round(fr_hbm, 4), valu_frac_charged=round(fr_valu, 4),
                hbm_algorithmic_bytes_per_launch=int(bytes_), kernel="kf_batched_kernel (+ 3 planning kernels)")
    return {
        "metric": METRIC,
        "value": round(updates / (ms / 1e3), 1),
        "unit": "track-layer updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.flags == 0 else "f32+f64", "data": "synthetic",
        "config": {"workload": args.workload, "form": "persistent batched launch, hipGraph replay",
                   "tracks": n, "updates_per_step": updates, "state_layout": layout_name,
                   "launch_shape": "library default" if shape is None else "given",
                   "block": (shape or BATCHED_DEFAULT_SHAPE)[0], "tracks_per_thread": (shape or BATCHED_DEFAULT_SHAPE)[1],
                   "schedule": (shape or BATCHED_DEFAULT_SHAPE)[2], "waves_mult": (shape or BATCHED_DEFAULT_SHAPE)[3],
                   "ok_tracks": ok,
                   "per_bucket_launches": len(launches), "per_bucket_ms": round(ms_b, 4),
                   "per_bucket_updates_per_s": round(updates / (ms_b / 1e3), 1),
                   "speedup_vs_per_bucket": round(ms_b / ms, 3), "autotune": tuned},
        "roofline": roof,
    }


def bench_adjoint(args, sample):
    """Forward + hand-written backward of sum chi2 (planes or cylinders, the
    sample's geometry): checkpoints of every layer, of every 2nd/4th/8th
    layer (recomputing inside a segment), and recomputation from the seed."""
    import torch
    from paper_2409_09228_amd import kf as K
    stream = torch.cuda.current_stream()
    layout = parse_layout(args.layout)
    st = K.stage_sample(sample, layout)
    geom = int(st["geom"])
    n, L = st["n"], st["L"]
    updates = int(sample["nlay"].sum())
    outs = (torch.empty_like(st["par"]), torch.empty_like(st["cov"]))
    chi2 = torch.empty(n, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    w = torch.ones(n, device="cuda")
    fwd = K.StepLauncher(geom, st["par"], st["cov"], st["hit_pos"], st["hit_cov"], st["layers"], st["bz"], n,
                         out=outs, chi2=chi2, status=status, nlay=st["nlay"], layout=layout, stream=stream)
    steps = max(3, args.steps // 4)
    ms = {"forward_plain": time_launches(fwd, steps, stream)}
    totals, ck_bytes = {}, {}
    for every in (1, 2, 4, 8):
        ck = K.checkpoint_buffer(n, L, layout, every=every)
        fwd_ck = K.StepLauncher(geom, st["par"], st["cov"], st["hit_pos"], st["hit_cov"], st["layers"], st["bz"], n,
                                out=outs, chi2=chi2, status=status, nlay=st["nlay"], layout=layout, ckpt=ck,
                                ckpt_every=every, stream=stream)
        fwd_ck()
        torch.cuda.synchronize()

        def bwd_ck(ck=ck, every=every):
            K.chi2_backward(st, status, w, ckpt=ck, ckpt_every=every, stream=stream)

        ms[f"forward_checkpoint_every{every}"] = time_launches(fwd_ck, steps, stream)
        ms[f"backward_checkpoint_every{every}"] = time_launches(bwd_ck, steps, stream)
        totals[f"checkpoint_every{every}"] = ms[f"forward_checkpoint_every{every}"] + ms[f"backward_checkpoint_every{every}"]
        ck_bytes[f"checkpoint_every{every}"] = int(ck.numel() * 4)
        del ck, fwd_ck

    def bwd_re():
        K.chi2_backward(st, status, w, ckpt=None, stream=stream)

    ms["backward_recompute"] = time_launches(bwd_re, max(2, steps // 4), stream)
    totals["recompute"] = ms["forward_plain"] + ms["backward_recompute"]
    ck_bytes["recompute"] = 0
    best = min(totals, key=totals.get)
    # the backward kernel of the best configuration against HBM: what it must
    # read (checkpoint slots, or the seed; hits; status; dL/dchi2) and write
    # (dL/dm per layer, dL/dp0) once
    every = int(best[len("checkpoint_every"):]) if best.startswith("checkpoint_every") else 0
    # checkpoint slots of the layers each track applied: ceil(n_i / every)
    nl = np.asarray(sample["nlay"], np.int64)
    slots = int((-(-nl // every)).sum()) if every else 0
    bwd_bytes = (slots * 27 * 4 + n * ((0 if every else 27 * 4) + 4 + 4 + 6 * 4)
                 + updates * (LAYER_BYTES + 3 * 4))
    bwd_ms = ms[f"backward_checkpoint_every{every}" if every else "backward_recompute"]
    bwd_gbs = bwd_bytes / (bwd_ms / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(bwd_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(bwd_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "kf_adjoint_kernel<%d>" % geom, "hbm_algorithmic_bytes_per_launch": int(bwd_bytes),
                "valu_frac_charged": None,
                "note": "the backward's flops have no algorithmic count; HBM fraction only"}
    return {
        "metric": METRIC + " -- forward + adjoint of sum chi2",
        "value": round(updates / (totals[best] / 1e3), 1),
        "unit": "track-layer updates/s (forward + backward)",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(totals[best], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "form": "adjoint", "tracks": n, "updates_per_step": updates,
                   "layout": args.layout, "best": best, "ms": {k: round(v, 4) for k, v in ms.items()},
                   "fwd_bwd_ms": {k: round(v, 4) for k, v in totals.items()}, "checkpoint_bytes": ck_bytes},
        "roofline": roofline,
    }


def bench_host(args, sample):
    """Host-resident (pinned) arrays, transfers included: kf_propagate_update_host
    streams chunks of tracks through the GPU, copies overlapping kernels.  Each
    call is synchronous, so the host clock times it; the device-resident launch
    of the same sample is timed alongside."""
    import torch
    from paper_2409_09228_amd import kf as K
    layout = parse_layout(args.layout)
    geom = int(sample["geom"][0])
    n = sample["par"].shape[0]
    L = sample["hit_pos"].shape[0]
    updates = int(sample["nlay"].sum())
    host = K.stage_host(sample, layout)
    out = (torch.empty_like(host["par"], pin_memory=True), torch.empty_like(host["cov"], pin_memory=True))

    def call():
        K.propagate_update_host(host, chunk=args.chunk, n_streams=args.streams, out=out)

    t_w = time.perf_counter()
    while time.perf_counter() - t_w < 1.0:
        call()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        call()
    sec = (time.perf_counter() - t0) / args.steps
    link = (TRACK_BYTES * n + LAYER_BYTES * n * L) / sec  # bytes over the host link per second
    dev = K.stage_sample(sample, layout)
    po, co = torch.empty_like(dev["par"]), torch.empty_like(dev["cov"])
    c2 = torch.empty(n, device="cuda")
    ss = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    launch = K.StepLauncher(geom, dev["par"], dev["cov"], dev["hit_pos"], dev["hit_cov"], dev["layers"], dev["bz"],
                            n, out=(po, co), chi2=c2, status=ss, nlay=dev["nlay"], layout=layout, stream=stream)
    kernel_ms = time_launches(launch, 20, stream)
    return {
        "metric": METRIC + " -- host-resident arrays, transfers included",
        "value": round(updates / sec, 1), "unit": "track-layer updates/s (with host-device copies)",
        "n_gpus": 1, "steps": args.steps, "warmup": "1 s", "ms_per_step": round(sec * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "form": "host pipeline", "tracks": n, "updates_per_step": updates,
                   "layout": args.layout, "chunk_tracks": args.chunk or 131072, "streams": args.streams or 3,
                   "tracks_per_s": round(n / sec, 1), "host_link_GBs": round(link / 1e9, 2),
                   "device_resident_ms": round(kernel_ms, 4),
                   "transfer_over_kernel": round(sec * 1e3 / kernel_ms, 2)},
    }


def bench_f64(args, sample):
    """The full-FP64 form (arrays, constants and arithmetic in double) on the
    same sample, device-resident, timed like the plain form."""
    import torch
    from paper_2409_09228_amd import kf as K
    layout = parse_layout(args.layout)
    geom = int(sample["geom"][0])
    n = sample["par"].shape[0]
    updates = int(sample["nlay"].sum())
    st = K.stage_sample_f64(sample, layout)
    stream = torch.cuda.current_stream()
    launch = K.StepLauncherF64(st, flags=args.flags & 2, tune=(args.block or 256, 1), stream=stream)
    for _ in range(args.warmup):
        launch()
    ms_step = time_launches(launch, args.steps, stream)
    sec = ms_step / 1e3
    flops = FLOPS_PER_UPDATE[geom] * updates
    flops_c = FLOPS_CHARGED_PER_UPDATE[geom] * updates
    bytes_ = 2 * (TRACK_BYTES * n + LAYER_BYTES * updates)  # every array in 8-byte words
    hbm = bytes_ / sec / 1e9
    tfl = flops / sec / 1e12
    tfl_c = flops_c / sec / 1e12
    intensity = flops / bytes_
    ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    # the larger fraction binds: HBM bytes or VALU flops (transcendentals
    # charged) against the FP64 vector peak
    if hbm / HBM_PEAK_GBS >= tfl_c / FP64_PEAK_TFLOPS:
        roof = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm / HBM_PEAK_GBS, 4), "traffic": None}
    else:
        roof = {"bound": "alu", "achieved": round(tfl_c, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tfl_c / FP64_PEAK_TFLOPS, 4), "traffic": None}
    roof["valu_frac_fp64_charged"] = round(tfl_c / FP64_PEAK_TFLOPS, 4)
    roof.update(intensity_flop_per_byte=round(intensity, 2), ridge_flop_per_byte=round(ridge, 2),
                alu_achieved_TFLOPs=round(tfl, 3), alu_frac_fp64=round(tfl / FP64_PEAK_TFLOPS, 4),
                hbm_achieved_GBs=round(hbm, 1), hbm_frac=round(hbm / HBM_PEAK_GBS, 4),
                hbm_algorithmic_bytes_per_launch=int(bytes_),
                kernel="kf_step_kernel_f64<%d,%d,%s>" % (geom, 2 if args.flags & 2 else 0, args.layout))
    ok = int(((launch.status & 0xFF) == 0).sum().item())
    return {
        "metric": METRIC + " -- full FP64 form",
        "value": round(updates / sec, 1), "unit": "track-layer updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "form": "full FP64", "tracks": n, "updates_per_step": updates,
                   "layout": args.layout, "joseph": bool(args.flags & 2), "block": args.block or 256, "ok_tracks": ok},
        "roofline": roof,
    }


def bench_smooth(args, sample):
    """Filter with per-layer checkpoints, then the RTS smoother writing the
    smoothed states over the checkpoints (in place); the smoother's launch is
    what is timed and bounded, the whole fit alongside."""
    import torch
    from paper_2409_09228_amd import kf as K
    layout = parse_layout(args.layout)
    geom = int(sample["geom"][0])
    n = sample["par"].shape[0]
    L = sample["hit_pos"].shape[0]
    updates = int(sample["nlay"].sum())
    st = K.stage_sample(sample, layout)
    stream = torch.cuda.current_stream()
    ck = K.checkpoint_buffer(n, L, layout, "cuda")
    po, co = torch.empty_like(st["par"]), torch.empty_like(st["cov"])
    c2 = torch.empty(n, device="cuda")
    ss = torch.empty(n, dtype=torch.int32, device="cuda")
    fwd = K.StepLauncher(geom, st["par"], st["cov"], st["hit_pos"], st["hit_cov"], st["layers"], st["bz"], n,
                         out=(po, co), chi2=c2, status=ss, nlay=st["nlay"], layout=layout, ckpt=ck, ckpt_every=1,
                         tune=(args.block or 256, 1), stream=stream)
    out = K.checkpoint_buffer(n, L, layout, "cuda")
    sm = K.SmoothLauncher(st, ck, po, co, ss, out=out, tune=(args.block or 256, 1), stream=stream)
    fwd()
    for _ in range(args.warmup):
        sm()
    ms_smooth = time_launches(sm, args.steps, stream)

    def fit():
        fwd()
        sm()
    ms_fit = time_launches(fit, max(args.steps // 2, 1), stream)
    ms_fwd = time_launches(fwd, max(args.steps // 2, 1), stream)
    done = int((ss >> 16).sum().item())
    # algorithmic bytes of the smoother: per applied layer the filtered
    # parameters (24 B, layers 0 .. done-2) and the smoothed state (108 B);
    # per track the final state (108 B) and the status word (4 B)
    bytes_ = 108 * done + 24 * (done - n) + (108 + 4) * n
    sec = ms_smooth / 1e3
    hbm = bytes_ / sec / 1e9
    roof = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(hbm / HBM_PEAK_GBS, 4), "traffic": None,
            "hbm_algorithmic_bytes_per_launch": int(bytes_), "kernel": "kf_smooth_kernel<%d,%s>" % (geom, args.layout)}
    return {
        "metric": METRIC + " -- RTS smoother (smoothed track-layer states/s)",
        "value": round(done / sec, 1), "unit": "smoothed track-layer states/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_smooth, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "form": "filter with checkpoints + RTS smoother", "tracks": n,
                   "updates_per_step": updates, "smoothed_states": done, "layout": args.layout,
                   "filter_with_checkpoints_ms": round(ms_fwd, 4), "fit_and_smooth_ms": round(ms_fit, 4),
                   "fit_and_smooth_tracks_per_s": round(n / (ms_fit / 1e3), 1)},
        "roofline": roof,
    }


def bench_gate(args, sample):
    """The filter with hit selection: n_cand candidates per layer (the
    track's hit and decoys at spread x the hit resolution), chi-square gate
    30; device-resident, timed like the plain form."""
    import torch
    from paper_2409_09228_amd import kf as K
    from paper_2409_09228_amd import synth as S
    layout = parse_layout(args.layout)
    geom = int(sample["geom"][0])
    n = sample["par"].shape[0]
    M = args.cand
    mh = S.multi_hit(sample, M, spread=args.spread)
    st = K.stage_sample(sample, layout)
    cands = K.stage_candidates(st, mh)
    del mh
    stream = torch.cuda.current_stream()
    run = K.GateLauncher(st, cands, args.gate, tune=(args.block or 256, 1), stream=stream)
    for _ in range(args.warmup):
        run()
    ms = time_launches(run, args.steps, stream)
    done = int((run.status >> 16).sum().item())
    ch = run.chosen
    L = st["L"]
    proc = torch.arange(L, device="cuda")[:, None] < (run.status >> 16)[None, :]
    holes = int(((ch == -1) & proc).sum().item())
    sec = ms / 1e3
    # algorithmic bytes: per processed layer M candidates (36 B each) and the
    # choice (4 B); per track the state in and out (216 B), nlay, chi2, status
    bytes_ = done * (36 * M + 4) + n * (216 + 12)
    flops = done * (FLOPS_PER_UPDATE[geom] + 44 * M)
    hbm = bytes_ / sec / 1e9
    roof = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(hbm / HBM_PEAK_GBS, 4), "traffic": None, "hbm_algorithmic_bytes_per_launch": int(bytes_),
            "intensity_flop_per_byte": round(flops / bytes_, 2), "alu_achieved_TFLOPs": round(flops / sec / 1e12, 3),
            "kernel": "kf_gate_kernel<%d,%s>" % (geom, args.layout)}
    return {
        "metric": METRIC + " -- hit selection among candidates (track-layer steps/s)",
        "value": round(done / sec, 1), "unit": "track-layer steps/s (propagate + select + update)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "form": "hit selection", "tracks": n, "layers_processed": done,
                   "candidates_per_layer": M, "decoy_spread_sigma": args.spread, "chi2_gate": args.gate,
                   "hole_fraction": round(holes / max(done, 1), 4), "layout": args.layout,
                   "candidates_per_s": round(done * M / sec, 1)},
        "roofline": roof,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--layout", default="soa")
    ap.add_argument("--flags", type=int, default=0)
    ap.add_argument("--block", type=int, default=None,
                    help="threads per block (default 256; the batched form: the library's default shape)")
    ap.add_argument("--tpt", type=int, default=None, help="tracks per thread (default 1)")
    ap.add_argument("--sched", type=int, default=None, help="batched form: 0 dynamic queue, 1 static round-robin")
    ap.add_argument("--waves-mult", type=int, default=None, help="batched form: grid in units of resident blocks")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle leg (CPU baseline and per-output precision error)")
    ap.add_argument("--no-p2r", action="store_true",
                    help="default workload: skip the barrel (p2r_100x9600) line beside it")
    ap.add_argument("--no-baseline", action="store_true", help="batched form: skip the per-bucket launches")
    ap.add_argument("--autotune", action="store_true",
                    help="batched and plain forms: search the launch shape and layout first, then time the winner")
    ap.add_argument("--form", default="auto", choices=["auto", "plain", "batched", "adjoint", "host", "f64", "smooth", "gate"],
                    help="auto: batched for mixed-geometry workloads, plain otherwise; host: host-resident "
                         "arrays, transfers included; f64: the full-FP64 form; smooth: filter + RTS smoother; gate: hit selection")
    ap.add_argument("--chunk", type=int, default=0, help="host form: tracks per chunk (0: library default)")
    ap.add_argument("--streams", type=int, default=0, help="host form: HIP streams (0: library default)")
    ap.add_argument("--cand", type=int, default=8, help="gate form: candidate hits per layer")
    ap.add_argument("--spread", type=float, default=10.0, help="gate form: decoy spread in hit sigmas")
    ap.add_argument("--gate", type=float, default=30.0, help="gate form: chi-square gate")
    ap.add_argument("--cpu-tracks", type=int, default=960000)
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="wall time of the CPU-baseline leg")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 1 GiB device buffer --steps times (calibrates the HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU only: tracks are independent and the step has no cross-GPU "
              "work; run it with --gpus 1", file=sys.stderr)
        return 2

    import torch
    from paper_2409_09228_amd import kf as K
    from paper_2409_09228_amd import synth as S

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read_per_call": src.numel() * 4,
                          "copy_probe_bytes_written_per_call": dst.numel() * 4, "calls": args.steps}))
        return 0
    K.lib()
    sample = S.generate(args.workload)
    mixed = sample["geom"].min() != sample["geom"].max()
    if args.form == "adjoint":
        print(json.dumps(bench_adjoint(args, sample)), flush=True)
        return 0
    if args.form == "host":
        print(json.dumps(bench_host(args, sample)), flush=True)
        return 0
    if args.form == "f64":
        print(json.dumps(bench_f64(args, sample)), flush=True)
        return 0
    if args.form == "smooth":
        print(json.dumps(bench_smooth(args, sample)), flush=True)
        return 0
    if args.form == "gate":
        print(json.dumps(bench_gate(args, sample)), flush=True)
        return 0
    if args.form == "batched" or (args.form == "auto" and mixed):
        print(json.dumps(bench_batched(args, sample)), flush=True)
        return 0
    if mixed:
        raise SystemExit("the plain form needs a single-geometry workload")
    tuned = None
    if args.autotune:
        # block size and layout timed on this sample before the benchmark
        from paper_2409_09228_amd import tune as T
        t0 = time.perf_counter()
        res = T.tune_plain(sample, flags=args.flags, use_cache=False)
        c = res["config"]
        args.block, args.layout = c["block"], c["layout"]
        tuned = {"config": c, "search_s": round(time.perf_counter() - t0, 1), "candidates": len(res["tried"]),
                 "worst_ms": round(max(t for _, t in res["tried"]), 4)}
    args.block, args.tpt = args.block or 256, args.tpt or 1
    head = time_plain(sample, args.workload, args.layout, args.flags, args.steps, args.warmup,
                      (args.block, args.tpt))
    out = {
        "metric": METRIC,
        "value": round(head["value"], 1),
        "unit": "track-layer updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.flags == 0 else "f32+f64",
        "data": "synthetic",
        "config": dict(head["config"], block=args.block, tracks_per_thread=args.tpt, autotune=tuned),
        "roofline": head["roofline"],
    }
    # the barrel form beside the headline plane form: same launch shape, same
    # timing procedure, its own roofline; in AoS records, its fastest layout
    # (each lane's hit is one contiguous record; the autotuner's pick), with
    # the headline's layout timed beside it
    if not args.no_p2r and args.workload == DEFAULT_WORKLOAD and args.flags == 0:
        r_sample = S.generate(P2R_WORKLOAD)
        r_layout = P2R_LAYOUT if args.layout == "soa" else args.layout
        r = time_plain(r_sample, P2R_WORKLOAD, r_layout, 0, args.steps, args.warmup, (args.block, args.tpt))
        out["p2r"] = {"workload": P2R_WORKLOAD, "value": round(r["value"], 1), "unit": "track-layer updates/s",
                      "ms_per_step": round(r["ms_step"], 4), "config": r["config"], "roofline": r["roofline"]}
        if r_layout != args.layout:
            rh = time_plain(r_sample, P2R_WORKLOAD, args.layout, 0, args.steps, args.warmup, (args.block, args.tpt))
            out["p2r"]["in_headline_layout"] = {"layout": args.layout, "ms_per_step": round(rh["ms_step"], 4),
                                                "value": round(rh["value"], 1),
                                                "roofline_frac": rh["roofline"]["frac"]}
            del rh
    else:
        r_sample, r = None, None
    if not args.no_cpu:
        # the oracle leg: the FP64 oracle timed on the host's cores, and its
        # results on sampled tracks against the GPU's (per-output error)
        leg = oracle_leg(sample, args, head, r_sample, r)
        out["cpu_baseline"] = leg["cpu_baseline"]
        out["precision_error"] = leg["precision_error"]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
