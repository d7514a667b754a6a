"""GPU parity of the RTS smoother (kf_smooth) against the oracle's smoother.

Two comparisons: (1) the whole fit -- the FP32 filter with checkpoints, then
the smoother -- against the FP64 oracle's filter and smoother; (2) the
smoother alone, fed the oracle's own filtered states (rounded to float), so
that only the smoother's arithmetic differs.  Metrics and FP32 gates as for
the filter (tests/parity.py), applied to every (layer, track) state the
smoother writes."""
import numpy as np
import pytest

import oracle as O
from paper_2409_09228_amd import synth as S
from parity import TOL_F32, TOL_SMOOTH_FIT, assert_within, metrics

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2409_09228_amd import kf as K
    K.lib()
    return K


def _layout(kf, name):
    return {"soa": kf.SOA, "aos": kf.AOS, "aosoa64": kf.aosoa(64), "aosoa16": kf.aosoa(16)}[name]


def _stack(sm_p, sm_P, done):
    """(layer, track) pairs the smoother writes -> flat arrays for metrics()."""
    L, n = sm_p.shape[:2]
    k, i = np.nonzero(np.arange(L)[:, None] < done[None, :])
    m = len(k)
    return (sm_p[k, i], sm_P[k, i], np.zeros(m), np.full(m, 1 << 16, np.int64))


def _oracle_smooth(s):
    sp, sP, st, rec = O.smooth_sample(s)
    return sp, sP, st, rec


def _gpu_fit(kf, s, layout="soa", in_place=False, tune=None):
    """Filter + smoother; slots a track did not apply are returned as NaN."""
    st = kf.stage_sample(s, _layout(kf, layout))
    po, co, c2, ss, sm = kf.fit_smooth(st, in_place=in_place, tune=tune)
    torch.cuda.synchronize()
    gp, gP = kf.smoothed_to_logical(st, sm)
    gst = ss.cpu().numpy()
    unused = np.arange(st["L"])[:, None] >= (gst >> 16)[None, :]
    gp[unused] = np.nan
    gP[unused] = np.nan
    return st, gp, gP, gst


@pytest.mark.parametrize("name,layout", [("p2z_1x8192", "soa"), ("p2z_1x8192", "aos"), ("p2z_1x8192", "aosoa64"),
                                         ("p2r_100x9600", "soa"), ("p2r_100x9600", "aosoa16")])
def test_fit_and_smooth_against_oracle(kf, name, layout):
    s = S.generate(name, n_events=1)
    g = int(s["geom"][0])
    sp, sP, ost, _ = _oracle_smooth(s)
    st, gp, gP, gst = _gpu_fit(kf, s, layout)
    np.testing.assert_array_equal(gst, ost)
    done = ost >> 16
    m = metrics(_stack(sp, sP, done), _stack(gp, gP, done), g)
    print(name, layout, m)
    assert_within(m, TOL_SMOOTH_FIT, f"smoothed {name} {layout}")


@pytest.mark.parametrize("name", ["p2z_1x8192", "p2r_100x9600"])
def test_smoother_alone_on_the_oracles_filtered_states(kf, name):
    """Checkpoints, final state and statuses from the FP64 oracle's filter:
    the GPU smoother's own error."""
    s = S.generate(name, n_events=1)
    g = int(s["geom"][0])
    sp, sP, ost, rec = _oracle_smooth(s)
    L, n = rec["filt_p"].shape[:2]
    done = ost >> 16
    ck = np.zeros((L, n, 27))
    ck[0, :, :6] = s["par"]
    ck[0, :, 6:] = s["cov"]
    ck[1:, :, :6] = rec["filt_p"][:-1]
    ck[1:, :, 6:] = O.pack_sym(rec["filt_P"][:-1])
    idx = np.arange(n)
    last = np.maximum(done - 1, 0)
    par_out = rec["filt_p"][last, idx]
    cov_out = O.pack_sym(rec["filt_P"][last, idx])
    # on the GPU a plane's z row is exactly zero; the oracle's is ~1e-22
    if g == 0:
        Z = np.zeros((6, 6), bool)
        Z[2, :] = Z[:, 2] = True
        zpk = O.pack_sym(Z.astype(float)).astype(bool)
        ck[1:, :, 6:][..., zpk] = 0.0
        cov_out[:, zpk] = 0.0
    lay = kf.SOA
    st = {"n": n, "L": L, "layout": lay, "geom": g, "bz": float(s["bz"]),
          "layers": np.asarray(s["layer_z"] if g == 0 else s["layer_r"], np.float32)}
    up = lambda a, E, Lx: torch.from_numpy(kf.to_layout_np(np.asarray(a, np.float32), lay)).cuda()
    ck_t = up(ck, 27, L)
    po_t = up(par_out, 6, 1)
    co_t = up(cov_out, 21, 1)
    ss_t = torch.from_numpy(ost.astype(np.int32)).cuda()
    sm = kf.smooth(st, ck_t, po_t, co_t, ss_t)
    torch.cuda.synchronize()
    gp, gP = kf.smoothed_to_logical(st, sm)
    m = metrics(_stack(sp, sP, done), _stack(gp, gP, done), g)
    print(name, m)
    assert_within(m, TOL_F32, f"smoother alone {name}")


@pytest.mark.parametrize("name", ["p2z_1x8192", "p2r_100x9600"])
def test_in_place_and_layouts_agree_bitwise(kf, name):
    s = S.subset(S.generate(name, n_events=1), np.arange(3001))
    _, a_p, a_P, _ = _gpu_fit(kf, s, "soa")
    for layout, in_place in (("soa", True), ("aos", False), ("aosoa64", True), ("aosoa16", False)):
        _, b_p, b_P, _ = _gpu_fit(kf, s, layout, in_place=in_place)
        np.testing.assert_array_equal(a_p, b_p)  # NaN (slots not written) compare equal
        np.testing.assert_array_equal(a_P, b_P)
    _, c_p, c_P, _ = _gpu_fit(kf, s, "soa", tune=(64, 1))
    np.testing.assert_array_equal(a_p, c_p)


def test_short_failed_and_empty_tracks(kf):
    """Tracks with 0 or 1 layers, a failure part-way and per-track layer
    counts: smoothed over exactly the layers applied (the other slots hold
    unspecified values: element-major layouts are written in whole rows).
    In AoS the other slots are not written."""
    s = S.subset(S.generate("p2z_1x8192"), np.arange(200))
    for k in ("hit_cov", "nlay"):
        s[k] = s[k].copy()
    s["hit_cov"][6, 3] = O.pack_sym(-np.eye(3))   # fails at layer 6
    s["nlay"][4] = 0
    s["nlay"][5] = 1
    s["nlay"][7] = 9
    sp, sP, ost, _ = _oracle_smooth(s)
    for lay in (kf.SOA, kf.AOS):
        st = kf.stage_sample(s, lay)
        po, co, c2, ss = kf.propagate_update(0, st["par"], st["cov"], st["hit_pos"], st["hit_cov"], st["layers"],
                                             st["bz"], st["n"], nlay=st["nlay"], layout=lay,
                                             ckpt=(ck := kf.checkpoint_buffer(st["n"], st["L"], lay, "cuda")))
        out = torch.full_like(ck, 12345.0)
        kf.smooth(st, ck, po, co, ss, out=out)
        torch.cuda.synchronize()
        gst = ss.cpu().numpy()
        np.testing.assert_array_equal(gst, ost)
        gp, gP = kf.smoothed_to_logical(st, out)
        done = ost >> 16
        if lay == kf.AOS:
            for i in range(200):
                assert np.all(gp[done[i]:, i] == 12345.0) and np.all(gP[done[i]:, i] == 12345.0)
        assert done[4] == 0 and done[5] == 1 and done[3] == 6 and done[7] == 9
        m = metrics(_stack(sp, sP, done), _stack(gp, gP, done), 0)
        assert_within(m, TOL_SMOOTH_FIT, "short and failed tracks")


@pytest.mark.parametrize("name,geom", [("p2z_100x9600", 0), ("p2r_100x9600", 1)])
def test_full_size_sampled(kf, name, geom):
    """The full 960k-track sample in the benchmark's launch shape (in place);
    the oracle smooths 2000 sampled tracks."""
    s = S.generate(name)
    n = s["par"].shape[0]
    st = kf.stage_sample(s, kf.SOA)
    po, co, c2, ss, sm = kf.fit_smooth(st, in_place=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    idx = np.sort(rng.choice(n, 2000, replace=False))
    idx[-1] = n - 1
    sp, sP, ost, _ = _oracle_smooth(S.subset(s, idx))
    gp, gP = kf.smoothed_to_logical(st, sm)
    done = ost >> 16
    np.testing.assert_array_equal(ss.cpu().numpy()[idx], ost)
    m = metrics(_stack(sp, sP, done), _stack(gp[:, idx], gP[:, idx], done), geom)
    print(name, m)
    assert_within(m, TOL_SMOOTH_FIT, name)


@pytest.mark.parametrize("geom", ["z", "r"])
def test_64bit_addressing_matches_32bit(kf, geom):
    """640,000 tracks x 64 layers put the filter and the smoother in their
    64-bit address form; the first 20,000 tracks on their own take the 32-bit
    buffer form.  Same arithmetic: the smoothed states agree bit for bit."""
    w = S.Workload(f"p2{geom}_64x640k", geom, 64, 10000, 64, seed_index=9)
    s = S.generate(w)
    m = 20000
    assert s["par"].shape[0] * 64 * 27 * 4 >= 1 << 32

    def run(sample):
        st = kf.stage_sample(sample, kf.SOA)
        po, co, c2, ss, sm = kf.fit_smooth(st, in_place=True)
        torch.cuda.synchronize()
        L, n = st["L"], st["n"]
        return sm.reshape(L, 27, n)[:, :, :m], ss[:m]

    big, sb = run(s)
    small, ss = run(S.subset(s, np.arange(m)))
    assert torch.equal(sb, ss)
    written = torch.arange(64, device="cuda")[:, None] < (ss >> 16)[None, :]
    for e in range(27):
        assert torch.equal(big[:, e][written], small[:, e][written])
