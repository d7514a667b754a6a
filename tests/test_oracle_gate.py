"""Pins of the oracle's hit selection (filter with several candidate hits per
layer) against facts outside its own code:

* one candidate (the track's hit) and no gate: the one-hit filter, bit for bit;
* the chi-square of the track's own hit follows the chi-square law of the
  measured directions: 3 on planes (mean 3, median 2.366), 2 on cylinders
  (hits are smeared along r*phi and z only: mean 2, median 1.386);
* a candidate exactly at the predicted point has chi-square 0 and is chosen;
* with no usable candidate every layer is a hole: the state is the helix
  propagation alone and the chi-square stays 0;
* the choice is the smallest chi-square within the gate, whatever the order
  of the candidates; following the oracle's own choices reproduces it.
Choosing the largest chi-square, leaving the hit covariance out of S, or
measuring against the state before propagation each fail one of them."""
import numpy as np
import pytest

import oracle as O
from paper_2409_09228_amd import synth as S


@pytest.fixture(scope="module")
def samples():
    return {"z": S.subset(S.generate("p2z_1x8192"), np.arange(2000)),
            "r": S.subset(S.generate("p2r_100x9600", n_events=1), np.arange(2000))}


def _valid(r):
    L = r["chosen"].shape[0]
    return np.arange(L)[:, None] < (r["status"] >> 16)[None, :]


@pytest.mark.parametrize("name", ["z", "r"])
def test_one_candidate_no_gate_is_the_one_hit_filter(samples, name):
    s = samples[name]
    r = O.gate_sample(s, S.multi_hit(s, 1), np.inf)
    one = O.run_sample(s)
    np.testing.assert_array_equal(r["par"], one[0])
    np.testing.assert_array_equal(r["cov"], one[1])
    np.testing.assert_array_equal(r["chi2"], one[2])
    np.testing.assert_array_equal(r["status"], one[3])
    assert np.all(r["chosen"][_valid(r)] == 0)


@pytest.mark.parametrize("name", ["z", "r"])
def test_joseph_selection(samples, name):
    """The Joseph form of the selected update: with one candidate and no gate
    it is the Joseph one-hit filter bit for bit; with candidates and a gate
    (the same choices forced) it equals the plain form to FP64 rounding."""
    s = samples[name]
    r = O.gate_sample(s, S.multi_hit(s, 1), np.inf, joseph=True)
    one = O.run_sample(s, joseph=True)
    for a, b in zip((r["par"], r["cov"], r["chi2"], r["status"]), one):
        np.testing.assert_array_equal(a, b)
    mh = S.multi_hit(s, 8, spread=10.0)
    plain = O.gate_sample(s, mh, 30.0)
    L = plain["chosen"].shape[0]
    forced = np.where(_valid(plain), plain["chosen"], -1)
    jos = O.gate_sample(s, mh, 30.0, forced=forced, joseph=True)
    np.testing.assert_array_equal(jos["status"], plain["status"])
    np.testing.assert_allclose(jos["par"], plain["par"], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(jos["chi2"], plain["chi2"], rtol=1e-9, atol=1e-11)
    assert L == s["hit_pos"].shape[0]


@pytest.mark.parametrize("name,dof,median", [("z", 3, 2.36597), ("r", 2, 1.38629)])
def test_chi2_of_the_tracks_own_hit_follows_the_chi2_law(samples, name, dof, median):
    s = samples[name]
    r = O.gate_sample(s, S.multi_hit(s, 1), np.inf)
    c = r["cand_chi2"][..., 0][_valid(r)]
    print(name, c.size, c.mean(), np.median(c))
    # 2000 tracks x up to 20 layers: the mean's standard error is < 0.02
    assert abs(c.mean() - dof) < 0.08
    assert abs(np.median(c) - median) < 0.06


@pytest.mark.parametrize("name", ["z", "r"])
def test_candidate_at_the_predicted_point_is_chosen(samples, name):
    s = S.subset(samples[name], np.arange(200))
    g = int(s["geom"][0])
    layers = s["layer_z"] if g == 0 else s["layer_r"]
    mh = S.multi_hit(s, 4, spread=3.0)
    for i in range(200):
        q, _, fl = O.propagate(g, s["par"][i], layers[0], s["bz"])
        assert fl == 0
        j = (mh["true_index"][0, i] + 1) % 4
        mh["cand_pos"][0, i, j] = q[:3]
    r = O.gate_sample(s, mh, 30.0)
    j0 = (mh["true_index"][0] + 1) % 4
    np.testing.assert_array_equal(r["chosen"][0], j0)
    assert np.all(np.abs(r["cand_chi2"][0, np.arange(200), j0]) < 1e-20)


@pytest.mark.parametrize("name", ["z", "r"])
def test_no_usable_candidate_means_propagation_only(samples, name):
    s = S.subset(samples[name], np.arange(50))
    g = int(s["geom"][0])
    layers = s["layer_z"] if g == 0 else s["layer_r"]
    mh = S.multi_hit(s, 3)
    mh["cand_pos"][..., 0, :] = np.nan          # non-finite
    mh["cand_cov"][..., 1, :] = O.pack_sym(-np.eye(3))   # not positive definite
    mh["cand_pos"][..., 2, :] += 1e3            # far outside the gate
    r = O.gate_sample(s, mh, 30.0)
    assert np.all(r["chosen"][_valid(r)] == -1) and np.all(r["chi2"] == 0)
    for i in range(50):
        p = s["par"][i]
        for k in range(r["status"][i] >> 16):
            p = O.propagate(g, p, layers[k], s["bz"])[0]
        np.testing.assert_allclose(r["par"][i], p, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("name", ["z", "r"])
def test_choice_is_the_smallest_chi2_in_the_gate_in_any_order(samples, name):
    s = samples[name]
    mh = S.multi_hit(s, 8, spread=3.0)
    r = O.gate_sample(s, mh, 30.0)
    v = _valid(r)
    c = np.where(np.isfinite(r["cand_chi2"]) & (r["cand_chi2"] <= 30.0), r["cand_chi2"], np.inf)
    want = np.where(np.isfinite(c.min(-1)), c.argmin(-1), -1)
    np.testing.assert_array_equal(r["chosen"][v], want[v])
    picked = np.where(r["chosen"] >= 0, np.take_along_axis(r["cand_chi2"], np.maximum(r["chosen"], 0)[..., None],
                                                             -1)[..., 0], 0.0)
    np.testing.assert_allclose(r["chi2"], np.where(v, picked, 0.0).sum(0), rtol=1e-12)
    # reversed candidate order: the same hits chosen, the same states
    rev = {"cand_pos": mh["cand_pos"][:, :, ::-1].copy(), "cand_cov": mh["cand_cov"][:, :, ::-1].copy()}
    r2 = O.gate_sample(s, rev, 30.0)
    ch2 = np.where(r2["chosen"] >= 0, 7 - r2["chosen"], -1)
    ties = np.sort(c, -1)[..., 1] == np.sort(c, -1)[..., 0]
    assert np.all((ch2 == r["chosen"])[v & ~ties])
    np.testing.assert_allclose(r2["par"], r["par"], rtol=1e-12, atol=1e-12)
    # following its own choices reproduces the run
    r3 = O.gate_sample(s, mh, 30.0, forced=np.where(v, r["chosen"], -1))
    np.testing.assert_array_equal(r3["par"], r["par"])
    np.testing.assert_array_equal(r3["chosen"][v], r["chosen"][v])
