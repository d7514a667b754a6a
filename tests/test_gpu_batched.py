"""GPU parity of the persistent mixed-geometry batched form
(kf_propagate_update_batched) against the FP64 oracle and against the plain
kernels, including hipGraph replay."""
import numpy as np
import pytest

import oracle as O
from paper_2409_09228_amd import synth as S
from parity import TOL_F32, TOL_PRECISION, assert_within, calibrated, metrics

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2409_09228_amd import kf as K
    K.lib()
    return K


@pytest.fixture(scope="module")
def uneven():
    return S.generate("uneven_250k")


def _logical(K, st, res):
    po, co, c2, ss = res
    torch.cuda.synchronize()
    p, c = K.results_to_logical(st, po, co)
    return p, c, c2.cpu().numpy().astype(np.float64), ss.cpu().numpy()


def _oracle_mixed(sample, joseph=False, precision="f64"):
    n = sample["par"].shape[0]
    out = [np.zeros((n, 6)), np.zeros((n, 21)), np.zeros(n), np.zeros(n, np.int32)]
    for g in (0, 1):
        idx = np.nonzero(sample["geom"] == g)[0]
        if len(idx) == 0:
            continue
        r = O.run_sample(S.subset(sample, idx), geom=g, joseph=joseph, precision=precision)
        for k in range(4):
            out[k][idx] = r[k]
    return tuple(out)


@pytest.mark.parametrize("layout", ["aos", "soa", "aosoa64"])
def test_uneven_250k_matches_oracle(kf, uneven, layout):
    lay = {"aos": kf.AOS, "soa": kf.SOA, "aosoa64": kf.aosoa(64)}[layout]
    st = kf.stage_batched(uneven, lay)
    got = _logical(kf, st, kf.run_batched(st))
    ref = _oracle_mixed(uneven)
    f32 = _oracle_mixed(uneven, precision="f32")
    np.testing.assert_array_equal(got[3] >> 16, uneven["nlay"])
    for g in (0, 1):
        # up to 30 layers: beyond the 20-layer calibration sample, so the gate
        # also admits twice the FP32 oracle's own error on this input
        m = metrics(ref, got, g, mask=uneven["geom"] == g)
        tol = calibrated(TOL_F32, metrics(ref, f32, g, mask=uneven["geom"] == g))
        print(layout, g, m, tol)
        assert_within(m, tol, f"batched {layout} geom {g}")


def test_batched_equals_plain_kernels(kf, uneven):
    """Per track, the persistent kernel computes exactly what the plain kernel
    does: the same device code on the same inputs."""
    sub = S.subset(uneven, np.arange(20000))
    st = kf.stage_batched(sub, kf.AOS)
    got = _logical(kf, st, kf.run_batched(st))
    for g in (0, 1):
        idx = np.nonzero(sub["geom"] == g)[0]
        s1 = S.subset(sub, idx)
        s1["geom"] = np.full(len(idx), g, np.uint8)
        st1 = kf.stage_sample(s1, kf.AOS)
        plain = _logical(kf, st1, kf.run_staged(st1))
        for k in range(4):
            np.testing.assert_array_equal(got[k][idx], plain[k])


def test_graph_replays_match_eager(kf, uneven):
    sub = S.subset(uneven, np.arange(30000))
    st = kf.stage_batched(sub, kf.AOS)
    eager = _logical(kf, st, kf.run_batched(st, flags=kf.KF_F_NO_GRAPH))
    par_out = torch.empty_like(st["par"])
    cov_out = torch.empty_like(st["cov"])
    chi2 = torch.empty(st["n"], device="cuda")
    status = torch.empty(st["n"], dtype=torch.int32, device="cuda")
    launch = kf.BatchedLauncher(st, (par_out, cov_out), chi2, status)
    for rep in range(4):
        # unrelated eager work and a synchronisation between replays
        par_out.fill_(rep + 1.0)
        chi2.zero_()
        status.fill_(-1)
        torch.cuda.synchronize()
        launch()
        got = _logical(kf, st, (par_out, cov_out, chi2, status))
        for k in range(4):
            np.testing.assert_array_equal(got[k], eager[k])
    kf.release_graphs()


@pytest.mark.parametrize("tune", [(64, 1, 0, 1), (128, 2, 0, 1), (256, 2, 1, 1), (64, 1, 0, 2), (256, 1, 1, 4),
                                  (256, 1, 0, 1), (128, 1, 1, 2)])
def test_launch_shapes_give_identical_results(kf, uneven, tune):
    sub = S.subset(uneven, np.arange(10000))
    st = kf.stage_batched(sub, kf.AOS)
    a = _logical(kf, st, kf.run_batched(st))
    b = _logical(kf, st, kf.run_batched(st, tune=tune))
    for k in range(4):
        np.testing.assert_array_equal(a[k], b[k])


def test_batched_precision_form(kf, uneven):
    sub = S.subset(uneven, np.arange(20000))
    st = kf.stage_batched(sub, kf.AOS)
    got = _logical(kf, st, kf.run_batched(st, flags=3))
    ref = _oracle_mixed(sub, joseph=True)
    f32 = _oracle_mixed(sub, joseph=True, precision="f32")
    for g in (0, 1):
        mask = sub["geom"] == g
        tol = calibrated(TOL_PRECISION, metrics(ref, f32, g, mask=mask))
        assert_within(metrics(ref, got, g, mask=mask), tol, f"batched precision geom {g}")


def test_batched_edge_cases(kf, uneven):
    sub = S.subset(uneven, np.arange(300))
    sub["nlay"] = sub["nlay"].copy()
    sub["nlay"][:20] = 0           # nothing to do
    sub["nlay"][20:25] = 1
    sub["hit_pos"] = sub["hit_pos"].copy()
    sub["hit_pos"][2, 40, 0] = np.nan  # a failing layer in the middle of a run
    st = kf.stage_batched(sub, kf.AOS)
    got = _logical(kf, st, kf.run_batched(st))
    ref = _oracle_mixed(sub)
    np.testing.assert_array_equal(got[3], ref[3])
    ok = (ref[3] & 0xFF) == 0
    f32 = _oracle_mixed(sub, precision="f32")
    for g in (0, 1):
        mask = ok & (sub["geom"] == g)
        tol = calibrated(TOL_F32, metrics(ref, f32, g, mask=mask))
        assert_within(metrics(ref, got, g, mask=mask), tol, f"edge geom {g}")
    # one track, and an empty call
    one = S.subset(uneven, np.arange(1))
    st1 = kf.stage_batched(one, kf.AOS)
    g1 = _logical(kf, st1, kf.run_batched(st1))
    r1 = _oracle_mixed(one)
    np.testing.assert_array_equal(g1[3], r1[3])


def test_hit_rows_outside_the_arrays_are_flagged(kf, uneven):
    """A track whose rows would leave [0, n_hits) gets KF_S_BAD_HITS, applies no
    layer and keeps its input state; the other tracks are unaffected."""
    sub = S.subset(uneven, np.arange(500))
    st = kf.stage_batched(sub, kf.AOS)
    ref = _logical(kf, st, kf.run_batched(st))
    n_hits = st["hit_pos"].shape[0]
    off = st["hit_offset"].clone()
    nl = sub["nlay"]
    bad = [int(np.nonzero(nl > 0)[0][0]), int(np.nonzero(nl > 3)[0][-1]), 7]
    off[bad[0]] = -1
    off[bad[1]] = n_hits - int(nl[bad[1]]) + 1   # last row one past the end
    off[bad[2]] = 1 << 40
    st2 = dict(st, hit_offset=off)
    got = _logical(kf, st2, kf.run_batched(st2))
    for i in bad:
        if nl[i] == 0:
            continue
        assert got[3][i] == kf.S_BAD_HITS, (i, got[3][i])
        np.testing.assert_array_equal(got[0][i], sub["par"][i].astype(np.float32))
        assert got[2][i] == 0.0
    keep = np.setdiff1d(np.arange(500), bad)
    for k in range(4):
        np.testing.assert_array_equal(got[k][keep], ref[k][keep])


def test_workspace_too_small_is_rejected(kf, uneven):
    sub = S.subset(uneven, np.arange(1000))
    st = kf.stage_batched(sub, kf.AOS)
    small = torch.empty(100, dtype=torch.uint8, device="cuda")
    with pytest.raises(kf.KFError) as e:
        kf.run_batched(st, workspace=small)
    assert e.value.code == 7


def test_64bit_hit_rows_match_32bit(kf, uneven):
    """Ragged hit arrays of 180M rows (4.32 GB of covariances, past the 4 GiB
    a 32-bit buffer offset reaches) put the persistent kernel in its 64-bit
    address form.  20,000 tracks whose rows sit at the end of those arrays
    (the rows before them zero) give, bit for bit, what the same tracks give
    with their rows in arrays of their own (the 32-bit form)."""
    sub = S.subset(uneven, np.arange(20000))
    st = kf.stage_batched(sub, kf.AOS)
    small = _logical(kf, st, kf.run_batched(st))
    H = st["hit_pos"].shape[0]
    rows = 180_000_000
    assert rows * 24 >= 1 << 32 and rows > H
    start = rows - H
    hp = torch.zeros(rows, 3, device="cuda")
    hc = torch.zeros(rows, 6, device="cuda")
    hp[start:] = st["hit_pos"]
    hc[start:] = st["hit_cov"]
    st2 = dict(st, hit_pos=hp, hit_cov=hc, hit_offset=st["hit_offset"] + start)
    big = _logical(kf, st2, kf.run_batched(st2))
    for k in range(4):
        np.testing.assert_array_equal(big[k], small[k])
    del hp, hc, st2
    kf.release_graphs()
    torch.cuda.empty_cache()
