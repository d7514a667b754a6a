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
