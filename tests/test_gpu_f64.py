"""The full-FP64 form (kf_propagate_update_z_f64 / _r_f64) against the FP64
oracle: the same algorithm in the same precision, so the two differ only by
operation order and by the kernel's series for helix angles below 1/2.
Gates (tests/parity.py metrics): see F64_TOL below."""
import numpy as np
import pytest

import oracle as O
from paper_2409_09228_amd import synth as S
from parity import assert_within, half_turning_angles, metrics

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# FP64 gates.  Largest differences measured over the tests below (both
# geometries, all layouts, Joseph, 64 planes): parameters 4.1e-13 floored
# relative and 3.0e-10 in sigma units, covariance 7.0e-13 correlation
# units, chi-square 3.3e-11 relative.  Each gate is 30-200x that, and at
# least five decades under the FP32 gates (1e-4 .. 5e-3), which a float
# step anywhere in the kernel would show.
F64_TOL = dict(par_floor=1e-10, par_sigma=1e-8, cov_corr=1e-10, chi2_rel=1e-9)


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2409_09228_amd import kf as K
    K.lib()
    return K


def _layout(kf, name):
    return {"soa": kf.SOA, "aos": kf.AOS, "aosoa64": kf.aosoa(64), "aosoa16": kf.aosoa(16)}[name]


def _run(kf, s, layout="soa", flags=0, tune=None):
    st = kf.stage_sample_f64(s, _layout(kf, layout))
    return kf.run_f64(st, flags=flags, tune=tune)


@pytest.mark.parametrize("layout", ["soa", "aos", "aosoa64", "aosoa16"])
def test_p2z_f64(kf, layout):
    s = S.generate("p2z_1x8192")
    got = _run(kf, s, layout)
    m = metrics(O.run_sample(s), got, 0)
    print(layout, m)
    assert_within(m, F64_TOL, f"p2z f64 {layout}")
    assert np.all(got[3] == 20 << 16)


@pytest.mark.parametrize("layout", ["soa", "aos", "aosoa64"])
def test_p2r_f64(kf, layout):
    s = S.generate("p2r_100x9600", n_events=1)
    got = _run(kf, s, layout)
    m = metrics(O.run_sample(s), got, 1)
    print(layout, m)
    assert_within(m, F64_TOL, f"p2r f64 {layout}")
    np.testing.assert_array_equal(got[3] >> 16, s["nlay"])


@pytest.mark.parametrize("name,geom", [("p2z_1x8192", 0), ("p2r_100x9600", 1)])
def test_joseph_f64(kf, name, geom):
    s = S.generate(name, n_events=1)
    got = _run(kf, s, flags=2)
    m = metrics(O.run_sample(s, joseph=True), got, geom)
    print(name, m)
    assert_within(m, F64_TOL, f"{name} Joseph f64")


def test_f64_is_closer_than_f32(kf):
    """The point of the form: on 64 planes the FP64 kernel stays at the FP64
    gates while the FP32 build of the oracle drifts orders of magnitude
    further."""
    w = S.Workload("p2z_64", "z", 1, 512, 64, seed_index=9)
    s = S.generate(w)
    ref = O.run_sample(s)
    m = metrics(ref, _run(kf, s), 0)
    f32 = metrics(ref, O.run_sample(s, precision="f32"), 0)
    print(m, f32)
    assert_within(m, F64_TOL, "64 layers f64")
    assert m["cov_corr"] * 1e3 < f32["cov_corr"]


@pytest.mark.parametrize("tune", [(64, 1), (128, 1)])
def test_launch_shapes_agree_bitwise(kf, tune):
    s = S.subset(S.generate("p2z_1x8192"), np.arange(3001))
    a = _run(kf, s)
    b = _run(kf, s, tune=tune)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("n", [1, 63, 65, 1000])
def test_ragged_tails_match_soa(kf, n):
    s = S.subset(S.generate("p2z_1x8192"), np.arange(n))
    a = _run(kf, s)
    for lay in ("aosoa16", "aosoa64", "aos"):
        b = _run(kf, s, lay)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_edge_statuses_f64(kf):
    """NaN hit, non-positive-definite S, non-finite input and out-of-range
    per-track layer counts give the oracle's status words."""
    s = S.subset(S.generate("p2z_1x8192"), np.arange(128))
    for k in ("hit_pos", "hit_cov", "par", "nlay"):
        s[k] = s[k].copy()
    s["hit_pos"][5, 2, 1] = np.nan
    s["hit_cov"][9, 4] = O.pack_sym(-np.eye(3))
    s["hit_cov"][0, 5] = np.inf
    s["par"][6, 3] = np.inf
    s["nlay"][7] = 0
    s["nlay"][8] = 1000
    s["nlay"][9] = -3
    s["nlay"][10] = 7
    got = _run(kf, s)
    ref = O.run_sample(s)
    np.testing.assert_array_equal(got[3], ref[3])
    ok = ((ref[3] & 0xFF) == 0) & np.all(np.isfinite(ref[0]), 1)
    assert_within(metrics(ref, got, 0, mask=ok), F64_TOL, "edge f64")


def test_p2r_no_crossing_f64(kf):
    r = S.generate("p2r_100x9600", n_events=1)
    idx = np.nonzero(r["nlay"] < 10)[0][:200]
    s = S.subset(r, idx)
    s["par"] = s["truth"].copy()
    pts = np.stack([S.truth_cross_cylinder(s["truth"], rk, r["bz"]) for rk in r["layer_r"]])
    s["hit_pos"] = np.where(np.isfinite(pts), pts, 0.0)
    s["nlay"] = np.full(len(idx), 20, np.int32)
    got = _run(kf, s)
    ref = O.run_sample(s)
    np.testing.assert_array_equal(got[3], ref[3])
    assert np.all((ref[3] & 0xFF) == O.ST_NO_CROSSING)


@pytest.mark.parametrize("name,geom", [("p2z_100x9600", 0), ("p2r_100x9600", 1)])
def test_full_size_sampled_f64(kf, name, geom):
    """The full 960,000-track samples in the benchmark's launch shape; 300
    sampled tracks, the last one included, against the FP64 oracle."""
    s = S.generate(name)
    n = s["par"].shape[0]
    got = _run(kf, s)
    rng = np.random.default_rng(29)
    idx = np.sort(rng.choice(n, 300, replace=False))
    idx[-1] = n - 1
    ref = O.run_sample(S.subset(s, idx))
    m = metrics(ref, tuple(x[idx] for x in got), geom)
    print(name, m)
    assert_within(m, F64_TOL, f"{name} f64 full size")
    np.testing.assert_array_equal(got[3] >> 16, s["nlay"])


@pytest.mark.parametrize("geom", ["z", "r"])
def test_strongly_curved_tracks_f64(kf, geom):
    """Helices turning by up to a radian or more between surfaces (the
    strongly curved samples of synth.curled): updates with a half turning
    angle |u| >= 1/2 take the library's sin and cos and the closed forms in
    place of the series; the same gates as everywhere in FP64."""
    g = 0 if geom == "z" else 1
    s = S.curled(geom)
    layers = s["layer_z"] if g == 0 else s["layer_r"]
    rec = O.filter_record(g, s["par"], s["cov"], s["hit_pos"], s["hit_cov"], layers, s["bz"], nlay=s["nlay"])
    u = half_turning_angles(s, rec)
    assert (u >= 0.5).mean() > 0.05 and u.max() > 0.8
    got = _run(kf, s)
    m = metrics(O.run_sample(s), got, g)
    print(geom, m)
    assert_within(m, F64_TOL, f"strongly curved {geom} f64")
