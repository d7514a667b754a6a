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
    assert len(list(T.candidates(T.PLAIN_SPACE))) == 9


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
