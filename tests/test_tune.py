"""The autotuner: search space, cache round trip (CPU), and one tuning run on
the GPU whose winner gives the same results as the default launch."""
import numpy as np
import pytest

from paper_2409_09228_amd import synth as S
from paper_2409_09228_amd import tune as T


def test_search_space_is_complete():
    c = list(T.candidates(T.BATCHED_SPACE))
    assert len(c) == 3 * 2 * 2 * 2 * 3
    assert {"block": 64, "tpt": 2, "schedule": 1, "waves_mult": 2, "layout": "aosoa64"} in c
    plain = list(T.candidates(T.PLAIN_SPACE))
    assert len(plain) == 3 * 6
    assert {c["layout"] for c in plain} == {"soa", "aos", "aosoa16", "aosoa32", "aosoa64", "aosoa128"}
    assert all(c["layout"] in T.LAYOUTS for c in plain)


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "t.json")
    assert T.load_cache(path) == {}
    T.save_cache({"k": {"config": {"block": 64}, "ms": 1.0}}, path)
    assert T.load_cache(path)["k"]["config"]["block"] == 64


def test_shape_key_distinguishes_workloads():
    a = S.subset(S.generate("uneven_250k"), np.arange(1000))
    b = S.subset(S.generate("uneven_250k"), np.arange(1001))
    assert T.shape_key("batched", a, 0) != T.shape_key("batched", b, 0)
    assert T.shape_key("batched", a, 0) != T.shape_key("batched", a, 3)


@pytest.mark.gpu
def test_tuning_run_on_gpu(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_2409_09228_amd import kf as K
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    sub = S.subset(S.generate("uneven_250k"), np.arange(20000))
    space = {"block": (64, 256), "tpt": (1, 2), "schedule": (0, 1), "waves_mult": (1,), "layout": ("aos", "soa")}
    res = T.tune_batched(sub, reps=3, space=space, cache_path=str(tmp_path / "t.json"))
    assert len(res["tried"]) == 16 and res["ms"] > 0
    c = res["config"]
    assert T.tune_batched(sub, space=space, cache_path=str(tmp_path / "t.json"))["config"] == c  # cached
    st = K.stage_batched(sub, T.LAYOUTS[c["layout"]])
    a = K.run_batched(st)
    b = K.run_batched(st, tune=(c["block"], c["tpt"], c["schedule"], c["waves_mult"]))
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.gpu
def test_plain_tuning_run_on_gpu(tmp_path):
    """tune_plain times block size x layout on the sample, caches the pick,
    and the picked configuration gives the default's results bit for bit
    (each track's arithmetic does not depend on the layout or block)."""
    torch = pytest.importorskip("torch")
    from paper_2409_09228_amd import kf as K
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    sub = S.subset(S.generate("p2r_100x9600", n_events=1), np.arange(5000))
    space = {"block": (64, 256), "layout": ("soa", "aos", "aosoa64")}
    path = str(tmp_path / "t.json")
    res = T.tune_plain(sub, reps=3, space=space, cache_path=path)
    assert len(res["tried"]) == 6 and res["ms"] > 0
    c = res["config"]
    assert T.tune_plain(sub, space=space, cache_path=path)["config"] == c  # cached
    st0 = K.stage_sample(sub, K.SOA)
    st1 = K.stage_sample(sub, T.LAYOUTS[c["layout"]])
    a = K.run_staged(st0)
    b = K.run_staged(st1, tune=(c["block"], 1))
    torch.cuda.synchronize()
    for x, y in zip(K.results_to_logical(st0, a[0], a[1]), K.results_to_logical(st1, b[0], b[1])):
        np.testing.assert_array_equal(x, y)
    assert torch.equal(a[2], b[2]) and torch.equal(a[3], b[3])
