"""GPU parity of the filter with hit selection (kf_propagate_gate_update).

Which candidate wins is decided in FP32 on the GPU and in FP64 by the
oracle, so near-ties may go either way.  The comparison therefore (1) checks
that every GPU choice is a valid one -- along the GPU's own sequence of
choices, replayed by the oracle in FP64, the chosen candidate's chi-square
is within the gate and within FP32 reach of the smallest, and a hole means
no candidate is clearly inside the gate -- and (2) compares the GPU's states
with that replay.  FP32 reach: the filter's FP32 states are within 0.1
sigma of FP64 (its parity gate), which moves a chi-square x by up to
2 * 0.1 * sqrt(x) + 0.01 x.  States: tracks with at most 3 holes are held
to the filter's FP32 gates.  Tracks with more ("lost" tracks) carry their
covariance unupdated over long paths; the next update then subtracts a
prior many times larger than its result, and the plain FP32 covariance
update cancels catastrophically (the FP32 build of the oracle is off by up
to 1.3 in correlation units there).  In the FP32 form they are held to
twice the fixed gates or 4x what the FP32 oracle makes of the same replay,
whichever is more: two FP32 evaluation orders of an ill-conditioned
subtraction agree in magnitude only, so no fixed gate applies.  The
precision form (FP64 inverse, gain and Joseph update) removes the
cancellation: there tracks with at most 3 holes are held to the
precision-form gates and lost ones to twice the FP32 gates (their
covariance is still carried over the holes by the FP32 transport, whose
F C F^T cancels as the correlations grow).  Tracks that fail are compared
by status only.
The fraction of decisions that differ from the oracle's own is reported and
bounded."""
import numpy as np
import pytest

import oracle as O
from paper_2409_09228_amd import synth as S
from parity import TOL_F32, TOL_PRECISION, assert_within, metrics

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GATE = 30.0


def _reach(x):
    return 0.2 * np.sqrt(np.abs(x)) + 0.01 * np.abs(x) + 1e-3


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2409_09228_amd import kf as K
    K.lib()
    return K


def _layout(kf, name):
    return {"soa": kf.SOA, "aos": kf.AOS, "aosoa64": kf.aosoa(64), "aosoa16": kf.aosoa(16)}[name]


def _gpu(kf, s, mh, layout="soa", gate=GATE, tune=None, flags=0):
    st = kf.stage_sample(s, _layout(kf, layout))
    cands = kf.stage_candidates(st, mh)
    run = kf.GateLauncher(st, cands, gate, tune=tune, flags=flags)
    run()
    torch.cuda.synchronize()
    p, c = kf.results_to_logical(st, run.par_out, run.cov_out)
    return (p, c, run.chi2.cpu().numpy().astype(np.float64), run.status.cpu().numpy(), run.chosen.cpu().numpy())


def _check(kf, s, mh, got, gate=GATE, what="", flags=0):
    g = int(s["geom"][0])
    st = got[3]
    L = got[4].shape[0]
    done = st >> 16
    proc = np.arange(L)[:, None] < done[None, :]
    forced = np.where(proc, got[4], -1)
    joseph = bool(flags & 2)
    rep = O.gate_sample(s, mh, gate, forced=forced, joseph=joseph)
    rep32 = O.gate_sample(s, mh, gate, forced=forced, precision="f32")
    own = O.gate_sample(s, mh, gate, joseph=joseph)
    # (1) every choice valid along the replayed path
    c = rep["cand_chi2"]
    cmin = np.min(np.where(np.isfinite(c), c, np.inf), axis=-1)
    ch = got[4]
    pick = np.take_along_axis(c, np.maximum(ch, 0)[..., None], -1)[..., 0]
    ok_pick = (ch >= 0) & np.isfinite(pick) & (pick <= gate + _reach(gate)) & (pick <= cmin + _reach(cmin))
    ok_hole = (ch == -1) & ~(cmin < gate - _reach(gate))
    bad = proc & ~(ok_pick | ok_hole)
    assert not bad.any(), (what, np.argwhere(bad)[:5], ch[bad][:5], pick[bad][:5], cmin[bad][:5])
    np.testing.assert_array_equal(st, rep["status"])
    # (2) states against the replay (tracks that did not fail)
    ok = (rep["status"] & 0xFF) == 0
    holes = np.sum((ch == -1) & proc, axis=0)
    ref = (rep["par"], rep["cov"], rep["chi2"], rep["status"])
    r32 = (rep32["par"], rep32["cov"], rep32["chi2"], rep32["status"])
    good, lost = ok & (holes <= 3), ok & (holes > 3)
    if flags:
        m = metrics(ref, got[:4], g, mask=good)
        print(what, "precision form, tracks", int(good.sum()), "+", int(lost.sum()), "lost:", m)
        assert_within(m, TOL_PRECISION, what)
        if lost.any():
            ml = metrics(ref, got[:4], g, mask=lost)
            print("  lost tracks:", ml)
            assert_within(ml, {k: 2 * v for k, v in TOL_F32.items()}, what + " (lost tracks)")
    else:
        m = metrics(ref, got[:4], g, mask=good)
        print(what, "tracks", int(good.sum()), "+", int(lost.sum()), "lost:", m)
        assert_within(m, TOL_F32, what)
    if lost.any() and not flags:
        ml = metrics(ref, got[:4], g, mask=lost)
        fl = metrics(ref, r32, g, mask=lost)
        print("  lost tracks:", ml, "fp32 oracle:", fl)
        tol = {k: max(2 * v, 4 * fl[k]) for k, v in TOL_F32.items()}
        assert_within(ml, tol, what + " (lost tracks)")
    differ = float(np.mean((own["chosen"] != ch)[proc]))
    print("  decisions differing from the oracle's own:", differ)
    return differ


@pytest.mark.parametrize("name,M,spread", [("p2z_1x8192", 8, 3.0), ("p2z_1x8192", 8, 10.0), ("p2z_1x8192", 16, 30.0),
                                           ("p2r_100x9600", 8, 30.0), ("p2r_100x9600", 4, 10.0)])
def test_gate_against_oracle(kf, name, M, spread):
    s = S.generate(name, n_events=1)
    mh = S.multi_hit(s, M, spread=spread)
    got = _gpu(kf, s, mh)
    differ = _check(kf, s, mh, got, what=f"{name} M={M} spread={spread}")
    assert differ < 0.01


@pytest.mark.parametrize("name,M,spread", [("p2z_1x8192", 8, 10.0), ("p2z_1x8192", 16, 30.0),
                                           ("p2r_100x9600", 8, 30.0), ("p2r_100x9600", 4, 10.0)])
def test_gate_precision_form(kf, name, M, spread):
    """flags = 3: every candidate's S^-1 and chi-square, the gain and the
    Joseph covariance update in FP64, against the FP64 Joseph replay: tracks
    with at most 3 holes at the precision-form gates, lost ones at twice the
    fixed FP32 gates."""
    s = S.generate(name, n_events=1)
    mh = S.multi_hit(s, M, spread=spread)
    got = _gpu(kf, s, mh, flags=3)
    differ = _check(kf, s, mh, got, what=f"{name} M={M} spread={spread} flags=3", flags=3)
    assert differ < 0.01


@pytest.mark.parametrize("name", ["p2z_1x8192", "p2r_100x9600"])
def test_layouts_and_launch_shapes_agree_bitwise(kf, name):
    s = S.subset(S.generate(name, n_events=1), np.arange(3001))
    mh = S.multi_hit(s, 8, spread=10.0)
    a = _gpu(kf, s, mh)
    for lay, tune in (("aos", None), ("aosoa64", None), ("aosoa16", (64, 1)), ("soa", (128, 1))):
        b = _gpu(kf, s, mh, lay, tune=tune)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("name,geom", [("p2z_1x8192", 0), ("p2r_100x9600", 1)])
def test_one_candidate_without_gate_is_the_plain_filter(kf, name, geom):
    s = S.generate(name, n_events=1)
    got = _gpu(kf, s, S.multi_hit(s, 1), gate=float("inf"))
    st = kf.stage_sample(s, kf.SOA)
    po, co, c2, ss = kf.run_staged(st)
    torch.cuda.synchronize()
    p, c = kf.results_to_logical(st, po, co)
    np.testing.assert_array_equal(got[0], p)
    np.testing.assert_array_equal(got[1], c)
    np.testing.assert_array_equal(got[2], c2.cpu().numpy().astype(np.float64))
    np.testing.assert_array_equal(got[3], ss.cpu().numpy())


def test_unusable_candidates_edges_and_failures(kf):
    """Non-finite and non-positive-definite candidates, candidates far
    outside the gate, a non-finite seed and per-track layer counts."""
    s = S.subset(S.generate("p2z_1x8192"), np.arange(300))
    for k in ("par", "nlay"):
        s[k] = s[k].copy()
    mh = S.multi_hit(s, 4, spread=3.0)
    mh["cand_pos"][3, :, 0] = np.nan
    mh["cand_cov"][4, :, 1] = O.pack_sym(-np.eye(3))
    mh["cand_pos"][5, 10:20] += 50.0   # whole layer out of the gate for 10 tracks: holes
    mh["cand_pos"][:, 20] = np.nan     # track 20: no usable candidate anywhere
    s["par"][6, 3] = np.inf
    s["nlay"][7] = 0
    s["nlay"][8] = 3
    s["nlay"][9] = 1000
    got = _gpu(kf, s, mh)
    _check(kf, s, mh, got, what="edges")
    assert np.all(got[4][5, 10:20] == -1) and np.all(got[4][:, 20] == -1) and got[2][20] == 0.0
    assert got[3][6] == O.ST_NONFINITE and got[3][7] == 0 and got[3][8] == 3 << 16


def test_full_size_sampled(kf):
    """960k tracks x 20 planes x 8 candidates in the benchmark's launch
    shape; 2000 sampled tracks replayed by the oracle."""
    s = S.generate("p2z_100x9600")
    n = s["par"].shape[0]
    mh = S.multi_hit(s, 8, spread=10.0)
    got = _gpu(kf, s, mh)
    rng = np.random.default_rng(99)
    idx = np.sort(rng.choice(n, 2000, replace=False))
    idx[-1] = n - 1
    sub = S.subset(s, idx)
    mh_sub = {"cand_pos": mh["cand_pos"][:, idx], "cand_cov": mh["cand_cov"][:, idx]}
    got_sub = tuple(x[idx] for x in got[:4]) + (got[4][:, idx],)
    differ = _check(kf, sub, mh_sub, got_sub, what="full size")
    assert differ < 0.01


def test_streamed_and_counted_forms_agree_bitwise(kf):
    """No per-track layer counts: the candidates stream with the
    non-temporal hint; an explicit array of n_layers takes the default form.
    Same arithmetic, identical results."""
    s = S.subset(S.generate("p2z_1x8192"), np.arange(4000))
    mh = S.multi_hit(s, 8, spread=10.0)
    st = kf.stage_sample(s, kf.SOA)
    assert st["nlay"] is None
    cands = kf.stage_candidates(st, mh)
    a = kf.GateLauncher(st, cands, GATE)
    a()
    full = torch.full((st["n"],), st["L"], dtype=torch.int32, device="cuda")
    b = kf.GateLauncher(dict(st, nlay=full), cands, GATE)
    b()
    torch.cuda.synchronize()
    for x, y in ((a.par_out, b.par_out), (a.cov_out, b.cov_out), (a.chi2, b.chi2), (a.status, b.status),
                 (a.chosen, b.chosen)):
        assert torch.equal(x, y)


def test_64bit_addressing_matches_32bit(kf):
    """640,000 tracks x 64 planes (2 candidates per layer) put the kernel in
    its 64-bit address form; the first 20,000 tracks on their own take the
    32-bit buffer form.  Same arithmetic, same decisions: states, chi2,
    status and the chosen candidates agree bit for bit."""
    w = S.Workload("p2z_64x640k", "z", 64, 10000, 64, seed_index=9)
    s = S.generate(w)
    assert s["par"].shape[0] * 64 * 27 * 4 >= 1 << 32
    mh = S.multi_hit(s, 2, spread=10.0, seed=3)
    m = 20000
    big = _gpu(kf, s, mh)
    sub = S.subset(s, np.arange(m))
    mhs = {k: (v[:, :m] if isinstance(v, np.ndarray) else v) for k, v in mh.items()}
    small = _gpu(kf, sub, mhs)
    for x, y in zip(big[:4], small[:4]):
        np.testing.assert_array_equal(x[:m], y)
    np.testing.assert_array_equal(big[4][:, :m], small[4])
