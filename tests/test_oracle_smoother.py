"""Pins of the oracle's RTS smoother against facts that do not come from the
recursion itself:

* on the last layer a track applied, smoothed = filtered (nothing follows);
* without process noise the state on layer k is a deterministic function of
  the state on layer k + 1, so the smoothed covariance must be the smoothed
  covariance of layer k + 1 carried back through the inverse of the local
  propagation Jacobian -- here obtained by central finite differences of the
  propagation map, not from the Jacobian the recursion used;
* the smoothed states lie on one helix: the smoothed state on layer k + 1,
  propagated back to layer k along the helix (reversed track), lands on the
  smoothed state of layer k up to second order in the smoothing correction;
* smoothing only adds information: C_filtered - C_smoothed is positive
  semi-definite on every layer.
A transposed gain, a gain without C_k, the Jacobian of the wrong step, or the
filtered instead of the predicted state in the correction each break one of
these."""
import numpy as np
import pytest

import oracle as O
from paper_2409_09228_amd import synth as S


@pytest.fixture(scope="module")
def samples():
    z = S.subset(S.generate("p2z_1x8192"), np.arange(300))
    r = S.subset(S.generate("p2r_100x9600", n_events=1), np.arange(300))
    out = {}
    for name, s in (("z", z), ("r", r)):
        g = int(s["geom"][0])
        layers = s["layer_z"] if g == 0 else s["layer_r"]
        sp, sP, st, rec = O.smooth_sample(s)
        out[name] = dict(s=s, g=g, layers=np.asarray(layers, np.float64), sp=sp, sP=O.unpack_sym(sP), st=st,
                         rec=rec)
    return out


def _reverse(p):
    q = np.array(p, np.float64)
    q[3] = -q[3]
    q[4] = q[4] + np.pi
    q[5] = np.pi - q[5]
    return q


def _back(g, p, target, bz):
    """p propagated backwards along its helix to the surface `target`."""
    q, _, fl = O.propagate(g, _reverse(p), target, bz)
    # inward crossings lie outside the method's own search (its straight-line
    # start aims at the far side of the cylinder, so it may raise
    # ST_NEWTON_RESIDUAL); the state returned is the exact crossing either way
    assert fl & ~O.ST_NEWTON_RESIDUAL == 0
    return _reverse(q)


@pytest.mark.parametrize("name", ["z", "r"])
def test_last_layer_is_the_filtered_state(samples, name):
    d = samples[name]
    done = d["st"] >> 16
    for i in range(len(done)):
        k = done[i] - 1
        np.testing.assert_array_equal(d["sp"][k, i], d["rec"]["filt_p"][k, i])
        np.testing.assert_array_equal(d["sP"][k, i], d["rec"]["filt_P"][k, i])
        assert not d["sp"][done[i]:, i].any()


@pytest.mark.parametrize("name", ["z", "r"])
def test_covariance_is_carried_back_by_the_inverse_jacobian(samples, name):
    d = samples[name]
    g, bz, rec = d["g"], float(d["s"]["bz"]), d["rec"]
    done = d["st"] >> 16
    worst = 0.0
    checked = 0
    for i in range(0, 300, 7):
        for k in range(0, done[i] - 1, 3):
            Uk = O.surface_basis(g, rec["pred_p"][k, i])
            Un = O.surface_basis(g, rec["pred_p"][k + 1, i])
            p = rec["filt_p"][k, i]
            F = np.zeros((5, 5))
            for j in range(5):
                h = 1e-6 * max(1.0, abs(p @ Uk[:, j]))
                a = O.propagate(g, p + h * Uk[:, j], d["layers"][k + 1], bz)[0]
                b = O.propagate(g, p - h * Uk[:, j], d["layers"][k + 1], bz)[0]
                F[:, j] = Un.T @ (a - b) / (2 * h)
            G = np.linalg.inv(F)
            Cn = Un.T @ d["sP"][k + 1, i] @ Un
            Ck = Uk.T @ d["sP"][k, i] @ Uk
            want = G @ Cn @ G.T
            sd = np.sqrt(np.diag(want))
            worst = max(worst, float(np.max(np.abs(Ck - want) / np.outer(sd, sd))))
            dp = Uk.T @ (d["sp"][k, i] - p)
            dwant = G @ (Un.T @ (d["sp"][k + 1, i] - rec["pred_p"][k + 1, i]))
            np.testing.assert_allclose(dp, dwant, rtol=1e-5, atol=1e-6 * sd.max())
            checked += 1
    print(name, checked, worst)
    assert checked > 50 and worst < 1e-6


@pytest.mark.parametrize("name,gate", [("z", 0.05), ("r", 0.25)])
def test_smoothed_states_lie_on_one_helix(samples, name, gate):
    """In units of the filtered sigma: the smoothing correction reaches a few
    sigma, the helix residual stays second order (measured 0.014 on planes,
    0.13 on cylinders, where the position along z bends most)."""
    d = samples[name]
    g, bz = d["g"], float(d["s"]["bz"])
    done = d["st"] >> 16
    worst, corr = 0.0, 0.0
    keep = [0, 1, 3, 4, 5] if g == 0 else [2, 3, 4, 5]
    for i in range(0, 300, 5):
        for k in range(done[i] - 1):
            back = _back(g, d["sp"][k + 1, i], d["layers"][k], bz)
            diff = back - d["sp"][k, i]
            diff[4] = np.angle(np.exp(1j * diff[4]))
            sd = np.sqrt(np.maximum(np.diag(d["rec"]["filt_P"][k, i]), 1e-30))
            worst = max(worst, float(np.max(np.abs(diff[keep]) / sd[keep])))
            step = d["sp"][k, i] - d["rec"]["filt_p"][k, i]
            corr = max(corr, float(np.max(np.abs(step[keep]) / sd[keep])))
    print(name, worst, corr)
    assert corr > 2.0 and worst < gate


@pytest.mark.parametrize("name", ["z", "r"])
def test_smoothing_only_adds_information(samples, name):
    d = samples[name]
    done = d["st"] >> 16
    for i in range(300):
        for k in range(done[i]):
            # on the surface's own coordinates (along the normal both are zero
            # up to rounding)
            U = O.surface_basis(d["g"], d["rec"]["pred_p"][k, i])
            Cf = U.T @ d["rec"]["filt_P"][k, i] @ U
            D = Cf - U.T @ d["sP"][k, i] @ U
            s = np.sqrt(np.diag(Cf))
            ev = np.linalg.eigvalsh(D / np.outer(s, s))
            assert ev.min() > -1e-9, (name, i, k, ev)


def test_failed_tracks_are_smoothed_over_the_layers_they_applied():
    s = S.subset(S.generate("p2z_1x8192"), np.arange(40))
    s["hit_cov"] = s["hit_cov"].copy()
    s["hit_cov"][6, 3] = O.pack_sym(-np.eye(3))
    sp, sP, st, rec = O.smooth_sample(s)
    assert st[3] == (O.ST_NOT_PD | (6 << 16))
    assert not sp[6:, 3].any()
    np.testing.assert_array_equal(sp[5, 3], rec["filt_p"][5, 3])
    assert np.any(sp[0, 3] != rec["filt_p"][0, 3])
