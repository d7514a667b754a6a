"""Pins for the oracle's FP32 builds.

The oracle's template is also instantiated in float: ``run(precision="f32")``,
``grad_chi2(precision="f32")`` and the float paths of ``filter_record`` and
``gate_run``.  They are test infrastructure twice removed: they never decide
parity, they only tighten the GPU gates on the 20-layer samples and loosen
them for longer inputs by a bounded factor (tests/parity.py).  A slip in
them that is specific to float (a constant rounded wrongly, a series
switched at the wrong argument, a float intermediate that should not be
one) shows up as an error against the FP64 build far from what single
precision costs on this workload.  So they are pinned:

* against an independent FP32-versus-FP64 calibration of the 8192-track
  plane workload (x, y ~ N(0, 0.01 cm), z = 0, q/pT = +-U(0.5, 5), theta in
  [0.4, 1.2], 20 planes at 10 + 5k cm, Bz = 3.8 T): a NumPy evaluation of
  the same method in float32 and float64, written before the oracle and
  sharing no code with it, gave the per-output maxima in CALIBRATION.  Each
  FP32-oracle figure must fall within a factor 3 of it either way -- below
  would mean the build does not really run in float, above that it loses
  precision it should not;
* by the structural identities between the float paths (the recording
  filter and the one-candidate selection are the plain filter, bit for bit);
* the gradient by the closed form of its last layer and a band against the
  FP64 reference gradient.
"""
import numpy as np
import pytest

import oracle as O
from paper_2409_09228_amd import synth as S
from parity import metrics

# Independent NumPy FP32-vs-FP64 calibration of the 8192-track plane workload:
# floored-relative maxima per parameter (x, y, kappa, phi, theta), the
# largest parameter error in sigma units, the covariance's correlation-
# normalised maximum, chi2's relative maximum and the largest relative
# difference of a sample mean.
CALIBRATION = {"x": 3.0e-5, "y": 3.4e-5, "kappa": 2.9e-6, "phi": 7.6e-7, "theta": 3.0e-7,
               "par_sigma": 2.4e-2, "cov_corr": 1.9e-4, "chi2_rel": 8.7e-4, "means": 5.7e-7}
BAND = 3.0


@pytest.fixture(scope="module")
def c1():
    s = S.generate("p2z_1x8192")
    ref = O.run_sample(s)
    f32 = tuple(np.asarray(x) for x in O.run_sample(s, precision="f32"))
    return s, ref, f32


def _in_band(got, want, what):
    assert want / BAND <= got <= want * BAND, f"{what}: {got:.3g} outside [{want / BAND:.3g}, {want * BAND:.3g}]"


def test_fp32_filter_matches_the_independent_calibration(c1):
    s, ref, f32 = c1
    m = metrics(ref, f32, 0)
    assert m["status_mismatch"] == 0
    each = m["par_floor_each"]
    for j, name in ((0, "x"), (1, "y"), (3, "kappa"), (4, "phi"), (5, "theta")):
        _in_band(each[j], CALIBRATION[name], name)
    assert each[2] == 0.0     # z lands on the plane exactly in both builds
    for k in ("par_sigma", "cov_corr", "chi2_rel"):
        _in_band(m[k], CALIBRATION[k], k)
    means = []
    for a, b in ((ref[0], f32[0]), (ref[2][:, None], f32[2][:, None])):
        ma, mb = a.mean(0), b.astype(np.float64).mean(0)
        means.append(np.max(np.abs(ma - mb) / np.maximum(np.abs(ma), 1.0)))
    assert max(means) <= CALIBRATION["means"] * BAND


def test_fp32_builds_agree_with_each_other(c1):
    """The recording filter (smoother input) and the one-candidate hit
    selection without a gate are the plain filter: in float as in double,
    bit for bit."""
    s, _, f32 = c1
    sub = S.subset(s, np.arange(256))
    base = O.run_sample(sub, precision="f32")
    rec = O.filter_record(0, sub["par"], sub["cov"], sub["hit_pos"], sub["hit_cov"], sub["layer_z"], sub["bz"],
                          nlay=sub["nlay"], precision="f32")
    np.testing.assert_array_equal(rec["status"], base[3])
    np.testing.assert_array_equal(rec["filt_p"][-1], base[0].astype(np.float64))
    np.testing.assert_array_equal(rec["chi2"], base[2].astype(np.float64))
    mh = {"cand_pos": sub["hit_pos"][:, :, None, :], "cand_cov": sub["hit_cov"][:, :, None, :]}
    g = O.gate_sample(sub, mh, np.inf, precision="f32")
    np.testing.assert_array_equal(g["status"], base[3])
    np.testing.assert_array_equal(g["par"], base[0].astype(np.float64))
    np.testing.assert_array_equal(g["cov"], base[1].astype(np.float64))


def test_fp32_paths_on_cylinders_are_float_but_bounded():
    """No independent calibration exists for the barrel.  There the float
    build must keep every status word, and where its closed-form crossing is
    well conditioned -- |q/pT| >= 1.5/GeV, radius of curvature <= 59 cm --
    it must be a float evaluation (errors well above FP64 rounding) inside
    the fixed FP32 gates of tests/parity.py.  At large radii the centre's
    distance from the axis and the radius nearly cancel in float, and the
    error grows as 1/|q/pT|: there (and only there) it exceeds those gates,
    which is why cylinder gates never take more than CEILING from it."""
    from parity import TOL_F32
    s = S.generate("p2r_100x9600", n_events=1)
    ref = O.run_sample(s)
    f32 = tuple(np.asarray(x) for x in O.run_sample(s, precision="f32"))
    assert metrics(ref, f32, 1)["status_mismatch"] == 0
    k = np.abs(s["par"][:, 3])
    m = metrics(ref, f32, 1, mask=k >= 1.5)
    for key, v in TOL_F32.items():
        assert 1e-7 < m[key] <= v, (key, m[key])
    lo = metrics(ref, f32, 1, mask=k < 0.6)
    assert lo["chi2_rel"] > 3 * m["chi2_rel"] and lo["par_sigma"] > 3 * m["par_sigma"]


def _col_err(got, ref, axis):
    """Element-wise |diff| floored at the RMS of its column over tracks."""
    rms = np.sqrt(np.mean(ref ** 2, axis=axis, keepdims=True))
    return (np.abs(got - ref) / np.maximum(np.abs(ref), rms)).max()


def test_fp32_gradient_is_a_float_evaluation_of_the_reference():
    """The float gradient against the FP64 dual-number gradient: errors of
    float size (1e-5 .. 1e-2 of each column's scale: the residual m - q is a
    0.01 cm difference of positions of tens of cm, so float rounding of the
    positions, ~4e-6 cm, is ~1e-3 of it), and on the last layer the closed
    form 2 S^-1 r evaluated from the float filter's own state before it."""
    s = S.subset(S.generate("p2z_64x9600", n_events=1), np.arange(256))
    args = (0, s["par"], s["cov"], s["hit_pos"], s["hit_cov"], s["layer_z"], s["bz"])
    rh, rp = O.grad_chi2(*args, nlay=s["nlay"])
    fh, fp = O.grad_chi2(*args, nlay=s["nlay"], precision="f32")
    for got, ref, ax in ((fh, rh, 1), (fp, rp, 0)):
        e = _col_err(got, ref, ax)
        assert 1e-5 < e < 1e-2, e
    L = s["hit_pos"].shape[0]
    n = s["par"].shape[0]
    po, co, _, _ = O.run_sample(dict(s, nlay=np.full(n, L - 1, np.int32)), precision="f32")
    ref_last = np.zeros((n, 3))
    for i in range(n):
        pt, F, _ = O.propagate(0, po[i].astype(np.float64), s["layer_z"][-1], s["bz"])
        Pt = F @ O.unpack_sym(co[i].astype(np.float64)) @ F.T
        Sm = Pt[:3, :3] + O.unpack_sym(s["hit_cov"][-1, i])
        ref_last[i] = 2 * np.linalg.solve(Sm, s["hit_pos"][-1, i] - pt[:3])
    # the closed form from the float state reproduces the float gradient's
    # last layer more closely than the FP64 gradient does
    e_own = _col_err(fh[-1], ref_last, 0)
    e_ref = _col_err(fh[-1], rh[-1], 0)
    assert e_own < 2e-3 and e_own < e_ref, (e_own, e_ref)
