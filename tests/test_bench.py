"""Host-side pieces of bench.py (no GPU): the one-GPU guard, the CPU-baseline
record, the counter-summary lookup and the algorithmic cost constants."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
from paper_2409_09228_amd import synth as S  # noqa: E402


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_cpu_baseline_record():
    s = S.subset(S.generate("p2z_1x8192", n_events=1), np.arange(400))
    r = bench.cpu_baseline(s, 400, min_seconds=0.2)
    assert r["kind"] == "oracle" and r["unit"] == "track-layer updates/s"
    assert r["value"] > 0 and r["single_thread_value"] > 0 and r["cores"] >= 1
    assert "400 tracks" in r["sample"]


def test_traffic_lookup_only_for_matching_summaries():
    # the precision form and layouts without a summary never borrow a figure
    assert bench.measured_traffic("p2z_100x9600", "soa", 3) is None
    assert bench.measured_traffic("p2z_100x9600", "aosoa16", 0) is None
    t = bench.measured_traffic("p2z_100x9600", "soa", 0)
    assert t is None or t > 0


def test_algorithmic_bytes_per_update():
    # per track: state in and out (2 x 27 floats), chi2 and status; per layer:
    # hit position (3) and covariance (6); p2z with 20 layers -> 47.2 B/update
    assert bench.TRACK_BYTES == 224 and bench.LAYER_BYTES == 36
    assert abs((bench.TRACK_BYTES / 20 + bench.LAYER_BYTES) - 47.2) < 1e-9
    assert bench.FLOPS_CHARGED_PER_UPDATE[0] > bench.FLOPS_PER_UPDATE[0]
    assert bench.FLOPS_CHARGED_PER_UPDATE[1] > bench.FLOPS_PER_UPDATE[1]


def test_output_errors_report_each_output():
    """A known perturbation of an FP64 result shows up in its own entry of
    the per-output report and nowhere else."""
    import oracle as O
    s = S.subset(S.generate("p2z_1x8192", n_events=1), np.arange(300))
    ref = O.run_sample(s)
    got = [x.copy() for x in ref]
    got[0][:, 3] += 2e-7                     # kappa: 2e-7 over the smallest |kappa| (>= the 0.1 floor)
    got[0][:, 4] += 2 * np.pi                # phi modulo 2 pi: no error
    e = bench.output_errors(ref, tuple(got), 0)
    want = 2e-7 / np.abs(ref[0][:, 3]).min()
    assert abs(e["kappa"] - want) < 5e-3 * want and e["phi"] < 1e-12   # reported to 3 digits
    assert e["x"] == e["y"] == e["z"] == e["theta"] == 0.0
    assert e["cov_corr"] == 0.0 and e["chi2_rel"] == 0.0 and e["status_mismatch"] == 0
    got[2] = got[2] * (1 + 1e-4)
    assert abs(bench.output_errors(ref, tuple(got), 0)["chi2_rel"] - 1e-4) < 2e-5


def test_cpu_identity_is_a_dict():
    info = bench.cpu_identity()
    assert isinstance(info, dict)


def test_newton_step_count_matches_the_oracles_search():
    """The barrel flop count charges NEWTON_STEPS_P2R search steps per update:
    the mean number of steps the oracle's single-precision search takes on
    the barrel sample, from the states the FP64 filter enters each layer with
    (1500 sampled tracks, every layer they apply), within 4 %."""
    import oracle as O
    s = S.generate("p2r_100x9600")
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(s["par"].shape[0], 1500, replace=False))
    sub = S.subset(s, idx)
    rec = O.filter_record(1, sub["par"], sub["cov"], sub["hit_pos"], sub["hit_cov"], sub["layer_r"],
                          float(sub["bz"]), nlay=sub["nlay"])
    steps = []
    for i in range(len(idx)):
        for k in range(int(sub["nlay"][i])):
            p = sub["par"][i] if k == 0 else rec["filt_p"][k - 1, i]
            steps.append(O.newton_r(p, sub["layer_r"][k], float(sub["bz"]), steps=True)[2])
    steps = np.asarray(steps)
    assert steps.min() >= 1 and steps.max() <= 5
    assert abs(steps.mean() - bench.NEWTON_STEPS_P2R) <= 0.04 * bench.NEWTON_STEPS_P2R, steps.mean()
    assert bench.FLOPS_PER_UPDATE[1] == round(729.0 + 27.0 * bench.NEWTON_STEPS_P2R, 1)
