"""GPU adjoint of the summed chi-square through barrel cylinders
(kf_chi2_backward, geometry 1) against the FP64 oracle's dual-number
reference gradient (differentiating the exact closed-form crossing; pinned
by finite differences in test_oracle_pins), central finite differences
(h = 1e-4) of the FP64 oracle, the closed form on each track's last layer,
and the torch.autograd.Function.  The tracks' layer counts are the barrel
sample's own (reachable cylinders: 1 to 20, mean 12.8).

Error metric as for the planes (test_gpu_adjoint): element by element,
floored at the RMS over tracks of the reference's column.  Gate TOL_GRAD =
2e-2, twice the planes' 1e-2: the planes' figure comes from one float
rounding of a position of ~50 cm (~4e-6 cm) against the 0.01 cm residual;
barrel hits sit at up to 100 cm (twice the rounding), and the crossing's
position along the cylinder moves by 1/cos of the crossing angle (up to 2.3
at the sample's reach margin) per unit of path-length error.  Measured:
1.1e-2 at most on hits, 3.1e-3 on seed parameters.  (The FP32 build of the
oracle is no yardstick here: its closed-form crossing is ill-conditioned in
float at large radii of curvature.)"""
import numpy as np
import pytest

import oracle as O
from paper_2409_09228_amd import synth as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_GRAD = 2e-2


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2409_09228_amd import kf as K
    K.lib()
    return K


def _col_scale(ref, axis=0):
    return np.sqrt(np.mean(ref ** 2, axis=axis, keepdims=True))


def _err(got, ref, scale=None):
    sc = _col_scale(ref) if scale is None else scale
    return float((np.abs(got - ref) / np.maximum(np.abs(ref), sc)).max())


def _reference(s, w=None):
    rh, rp = O.grad_chi2(1, s["par"], s["cov"], s["hit_pos"], s["hit_cov"], s["layer_r"], s["bz"], w=w,
                         nlay=s["nlay"])
    return rh.transpose(1, 0, 2), rp


def _fwd_bwd(kf, sample, layout=None, checkpoint=True, w=None, every=1):
    layout = kf.SOA if layout is None else layout
    st = kf.stage_sample(sample, layout)
    assert st["geom"] == 1
    n, L = st["n"], st["L"]
    ck = kf.checkpoint_buffer(n, L, layout, every=every) if checkpoint else None
    po, co, c2, ss = kf.run_staged(st, ckpt=ck, ckpt_every=every)
    wt = torch.ones(n, device="cuda") if w is None else torch.from_numpy(w.astype(np.float32)).cuda()
    gh, gp, gc = kf.chi2_backward(st, ss, wt, ckpt=ck, want_cov=True, ckpt_every=every)
    torch.cuda.synchronize()
    if layout[0] == kf.KF_SOA:
        ghl = gh.cpu().numpy().transpose(2, 0, 1)
    elif layout[0] == kf.KF_AOS:
        ghl = gh.cpu().numpy().transpose(1, 0, 2)
    else:
        ghl = kf.unpack(gh, 3, L, n, layout).cpu().numpy().transpose(2, 0, 1)
    gpl = kf.from_layout(gp, 6, n, layout).astype(np.float64)
    return ghl.astype(np.float64), gpl, c2.cpu().numpy(), ss.cpu().numpy(), gc


@pytest.fixture(scope="module")
def barrel():
    return S.generate("p2r_100x9600", n_events=1)


@pytest.mark.parametrize("checkpoint", [True, False])
def test_cylinder_gradient_matches_fp64_reference(kf, barrel, checkpoint):
    s = S.subset(barrel, np.arange(512))
    w = np.random.default_rng(3).uniform(0.5, 2.0, 512)
    gh, gp, _, st, _ = _fwd_bwd(kf, s, checkpoint=checkpoint, w=w)
    np.testing.assert_array_equal(st >> 16, s["nlay"])
    rh, rp = _reference(s, w)
    eh, ep = _err(gh, rh), _err(gp, rp)
    print("cylinders checkpoint", checkpoint, "hit", eh, "par", ep)
    assert eh <= TOL_GRAD and ep <= TOL_GRAD


def test_cylinder_gradient_matches_central_differences_h1e4(kf, barrel):
    """Central differences with h = 1e-4 of the FP64 oracle's chi2: all
    inputs of 16 tracks (seed parameters and every applied hit coordinate)."""
    s = S.subset(barrel, np.arange(16))
    gh, gp, _, _, _ = _fwd_bwd(kf, s)
    h = 1e-4
    L = s["hit_pos"].shape[0]

    def chi(par, hits):
        return O.run(1, par, s["cov"], hits, s["hit_cov"], s["layer_r"], s["bz"], nlay=s["nlay"])[2]

    fp = np.zeros((16, 6))
    for a in range(6):
        e = np.zeros_like(s["par"])
        e[:, a] = h
        fp[:, a] = (chi(s["par"] + e, s["hit_pos"]) - chi(s["par"] - e, s["hit_pos"])) / (2 * h)
    fh = np.zeros((16, L, 3))
    for k in range(L):
        for a in range(3):
            e = np.zeros_like(s["hit_pos"])
            e[k, :, a] = h
            fh[:, k, a] = (chi(s["par"], s["hit_pos"] + e) - chi(s["par"], s["hit_pos"] - e)) / (2 * h)
    print("fd hit", _err(gh, fh), "par", _err(gp, fp))
    assert _err(gh, fh) <= TOL_GRAD and _err(gp, fp) <= TOL_GRAD


def test_cylinder_checkpoints_and_recompute_agree(kf, barrel):
    """Per-layer checkpoints, checkpoints of every 2nd and 4th layer (the
    states inside a segment recomputed) and recomputation from the seed:
    forward results identical, gradients agreeing to FP32 rounding (the
    recomputed segments start from freshly evaluated sin and cos of the
    direction angles) and each meeting the FP64 reference's gate."""
    s = S.subset(barrel, np.arange(1000))
    a = _fwd_bwd(kf, s, every=1)
    rh, rp = _reference(s)
    for every, ck in ((2, True), (4, True), (1, False)):
        b = _fwd_bwd(kf, s, every=every, checkpoint=ck)
        np.testing.assert_array_equal(a[2], b[2])
        np.testing.assert_array_equal(a[3], b[3])
        eh, ep = _err(b[0], rh), _err(b[1], rp)
        print("every", every, "checkpoint", ck, "hit", eh, "par", ep)
        assert eh <= TOL_GRAD and ep <= TOL_GRAD
        assert _err(b[0], a[0], _col_scale(rh)) <= TOL_GRAD and _err(b[1], a[1], _col_scale(rp)) <= TOL_GRAD


@pytest.mark.parametrize("layout", ["aos", "aosoa64"])
def test_cylinder_layouts_agree(kf, barrel, layout):
    s = S.subset(barrel, np.arange(1000))
    a = _fwd_bwd(kf, s)
    lay = kf.AOS if layout == "aos" else kf.aosoa(64)
    b = _fwd_bwd(kf, s, layout=lay)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-6, atol=1e-6 * np.abs(a[0]).max())
    np.testing.assert_allclose(a[1], b[1], rtol=1e-6, atol=1e-6 * np.abs(a[1]).max())


def test_cylinder_last_layer_closed_form(kf, barrel):
    """Nothing downstream depends on a track's last hit: dL/dm = 2 S^-1 r on
    its last applied layer, with S and r from the oracle's state one layer
    earlier."""
    s = S.subset(barrel, np.arange(64))
    gh, _, _, _, _ = _fwd_bwd(kf, s)
    nl = s["nlay"]
    po, co, _, _ = O.run(1, s["par"], s["cov"], s["hit_pos"], s["hit_cov"], s["layer_r"], s["bz"],
                         nlay=np.maximum(nl - 1, 0))
    ref = np.zeros((64, 3))
    got = np.zeros((64, 3))
    for i in range(64):
        k = nl[i] - 1
        pt, F, fl = O.propagate(1, po[i], s["layer_r"][k], s["bz"])
        assert fl == 0
        Pt = F @ O.unpack_sym(co[i]) @ F.T
        Sm = Pt[:3, :3] + O.unpack_sym(s["hit_cov"][k, i])
        ref[i] = 2 * np.linalg.solve(Sm, s["hit_pos"][k, i] - pt[:3])
        got[i] = gh[i, k]
    print("last layer", _err(got, ref))
    assert _err(got, ref) <= TOL_GRAD


def test_cylinder_autograd_function(kf, barrel):
    s = S.subset(barrel, np.arange(300))
    w = np.linspace(0.5, 1.5, 300)
    rh, rp = _reference(s, w)
    st = kf.stage_sample(s)
    par = st["par"].clone().requires_grad_(True)
    hp = st["hit_pos"].clone().requires_grad_(True)
    for ckpt in (True, False, 2):
        chi2 = kf.KFChi2().apply(par, hp, st["cov"], st["hit_cov"], st["layers"], st["bz"], kf.SOA, st["nlay"],
                                 ckpt, 1)
        loss = (chi2 * torch.linspace(0.5, 1.5, 300, device="cuda")).sum()
        par.grad = None
        hp.grad = None
        loss.backward()
        gp = kf.from_soa_tensor(par.grad).astype(np.float64)
        gh = hp.grad.cpu().numpy().transpose(2, 0, 1).astype(np.float64)
        print("autograd", ckpt, _err(gh, rh), _err(gp, rp))
        assert _err(gh, rh) <= TOL_GRAD and _err(gp, rp) <= TOL_GRAD


def test_cylinder_full_size_sampled(kf):
    """The full 960,000-track barrel sample, checkpoints of every 2nd layer:
    gradients of 300 sampled tracks (the last one included) against the FP64
    reference."""
    s = S.generate("p2r_100x9600")
    n = s["par"].shape[0]
    gh, gp, _, st, _ = _fwd_bwd(kf, s, checkpoint=True, every=2)
    assert np.all((st & 0xFF) == 0)
    rng = np.random.default_rng(17)
    idx = np.sort(rng.choice(n, 300, replace=False))
    idx[-1] = n - 1
    rh, rp = _reference(S.subset(s, idx))
    eh, ep = _err(gh[idx], rh), _err(gp[idx], rp)
    print("full size hit", eh, "par", ep)
    assert eh <= TOL_GRAD and ep <= TOL_GRAD
