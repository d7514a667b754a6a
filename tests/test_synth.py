"""The synthetic workloads: determinism, shapes and distributions."""
import numpy as np

from paper_2409_09228_amd import synth as S


def test_deterministic_and_prefix_stable():
    a = S.generate("p2z_100x9600", n_events=2)
    b = S.generate("p2z_100x9600", n_events=2)
    for k in ("par", "cov", "hit_pos", "hit_cov", "nlay", "truth"):
        np.testing.assert_array_equal(a[k], b[k])
    c = S.generate("p2z_100x9600", n_events=1)
    np.testing.assert_array_equal(c["par"], a["par"][:9600])
    np.testing.assert_array_equal(c["hit_pos"], a["hit_pos"][:, :9600])


def test_p2z_distributions():
    s = S.generate("p2z_1x8192")
    t = s["truth"]
    assert t.shape == (8192, 6) and s["hit_pos"].shape == (20, 8192, 3)
    k = np.abs(t[:, 3])
    assert k.min() >= 0.5 and k.max() <= 5.0
    assert 0.45 < np.mean(t[:, 3] > 0) < 0.55
    assert t[:, 5].min() >= 0.4 and t[:, 5].max() <= 1.2
    assert abs(np.std(s["par"][:, 0] - t[:, 0]) - 0.01) < 5e-4
    np.testing.assert_allclose(s["layer_z"], 10 + 5 * np.arange(20))
    # hits lie within a few sigma of their planes
    dz = s["hit_pos"][:, :, 2] - s["layer_z"][:, None]
    assert abs(dz.std() - 0.01) < 3e-4
    assert np.all(s["nlay"] == 20)


def test_p2r_hits_on_cylinders_and_reachability():
    r = S.generate("p2r_100x9600", n_events=1)
    rr = np.hypot(r["hit_pos"][..., 0], r["hit_pos"][..., 1])
    k = np.arange(20)[:, None]
    valid = k < r["nlay"][None, :]
    np.testing.assert_allclose(rr[valid], np.broadcast_to(r["layer_r"][:, None], rr.shape)[valid], rtol=1e-12)
    assert 12.0 < r["nlay"].mean() < 13.6
    rmax = S.truth_max_radius(r["truth"], r["bz"])
    last = r["layer_r"][np.maximum(r["nlay"] - 1, 0)]
    assert np.all(last <= 0.9 * rmax + 1e-9)


def test_uneven_mix():
    u = S.generate("uneven_250k")
    assert u["par"].shape[0] == 250000
    assert np.sum(u["geom"] == 0) == 125000
    z = u["nlay"][u["geom"] == 0]
    assert z.min() == 5 and z.max() == 30
    assert 17.0 < z.mean() < 18.0
    hp, hc, off = S.to_ragged(u["hit_pos"][:, :100], u["hit_cov"][:, :100], u["nlay"][:100])
    assert hp.shape[0] == u["nlay"][:100].sum()
    np.testing.assert_array_equal(hp[off[7] + 3], u["hit_pos"][3, 7])


def test_host_layout_roundtrip():
    """The numpy layout builder of the FP64 form agrees with the offset formula
    of the library's layouts and inverts exactly."""
    from paper_2409_09228_amd import kf as K
    rng = np.random.default_rng(5)
    n, L, E = 100, 3, 7
    x = rng.normal(size=(L, n, E))
    for lay in (K.SOA, K.AOS, K.aosoa(16), K.aosoa(64)):
        f = K.to_layout_np(x, lay)
        np.testing.assert_array_equal(K.from_layout_np(f, E, L, n, lay), x)
        i, l, e = 77, 2, 5
        kind, B = lay
        if kind == K.KF_SOA:
            o = (l * E + e) * n + i
        elif kind == K.KF_AOS:
            o = (l * n + i) * E + e
        else:
            o = (i // B) * (E * L * B) + (i % B) + (l * E + e) * B
        assert f[o] == x[l, i, e]
    y = rng.normal(size=(n, E))
    for lay in (K.SOA, K.AOS, K.aosoa(32)):
        np.testing.assert_array_equal(K.from_layout_np(K.to_layout_np(y, lay), E, 1, n, lay), y)


def test_every_nth_layer_and_curled_samples():
    """every_nth_layer keeps layers 0, step, 2 step, ... with their own hits
    and ceil(nlay / step) layers per track; the strongly curved samples draw
    |q/pT| in their ranges and keep their hits on the surfaces."""
    s = S.subset(S.generate("p2r_100x9600", n_events=1), np.arange(500))
    t = S.every_nth_layer(s, 3)
    assert np.array_equal(t["layer_r"], s["layer_r"][::3])
    assert np.array_equal(t["hit_pos"], s["hit_pos"][::3])
    assert np.array_equal(t["nlay"], -(-s["nlay"] // 3))
    for geom, lo, hi in (("z", 6.0, 9.0), ("r", 4.0, 8.0)):
        c = S.curled(geom)
        k = np.abs(c["truth"][:, 3])
        assert k.min() >= lo and k.max() <= hi
        L = c["hit_pos"].shape[0]
        used = np.arange(L)[:, None] < c["nlay"][None, :]
        if geom == "z":  # smeared along z by 0.01 cm
            dz = c["hit_pos"][..., 2] - c["layer_z"][:, None]
            assert np.abs(dz[used]).max() < 0.1
        else:  # on the cylinders
            r = np.hypot(c["hit_pos"][..., 0], c["hit_pos"][..., 1])
            np.testing.assert_allclose(r[used], np.broadcast_to(c["layer_r"][:, None], r.shape)[used], rtol=1e-12)
            assert np.array_equal(c["layer_r"], 5.0 + 15.0 * np.arange(7))
