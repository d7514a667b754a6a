"""Host-resident form (kf_propagate_update_host): chunks streamed through the
GPU on several streams give exactly the results of the device-resident call
on the same inputs -- the same kernels on the same numbers -- for every
layout, chunk size (ragged last chunk included) and stream count."""
import numpy as np
import pytest

from paper_2409_09228_amd import synth as S

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


def _assert_same(kf, dev, got, ref):
    """Bit-for-bit on the tracks (AoSoA padding lanes hold no track and are
    written by neither path)."""
    gp, gc = kf.results_to_logical(dev, got[0].cuda(), got[1].cuda())
    rp, rc = kf.results_to_logical(dev, ref[0], ref[1])
    np.testing.assert_array_equal(gp, rp)
    np.testing.assert_array_equal(gc, rc)
    assert torch.equal(got[2], ref[2].cpu()) and torch.equal(got[3], ref[3].cpu())


@pytest.fixture(scope="module")
def samples():
    z = S.subset(S.generate("p2z_1x8192"), np.arange(5000))
    r = S.subset(S.generate("p2r_100x9600", n_events=1), np.arange(4321))
    return {"z": z, "r": r}


@pytest.mark.parametrize("geom", ["z", "r"])
@pytest.mark.parametrize("layout", ["soa", "aos", "aosoa64", "aosoa16"])
@pytest.mark.parametrize("chunk,streams", [(1000, 3), (777, 2), (0, 1), (64, 4)])
def test_host_pipeline_equals_device_call(kf, samples, geom, layout, chunk, streams):
    s = samples[geom]
    lay = _layout(kf, layout)
    dev = kf.stage_sample(s, lay)
    ref = kf.run_staged(dev)
    torch.cuda.synchronize()
    host = kf.stage_host(s, lay)
    got = kf.propagate_update_host(host, chunk=chunk, n_streams=streams)
    _assert_same(kf, dev, got, ref)


def test_precision_form_and_pageable_memory(kf, samples):
    s = samples["z"]
    dev = kf.stage_sample(s, kf.SOA)
    ref = kf.run_staged(dev, flags=3)
    torch.cuda.synchronize()
    host = kf.stage_host(s, kf.SOA, pinned=False)
    got = kf.propagate_update_host(host, flags=3, chunk=1500, n_streams=2)
    _assert_same(kf, dev, got, ref)


def test_bad_arguments_are_rejected_before_any_copy(kf, samples):
    host = kf.stage_host(samples["z"], kf.SOA)
    with pytest.raises(kf.KFError) as e:
        kf.propagate_update_host(host, n_streams=9)
    assert e.value.code == 2
    with pytest.raises(kf.KFError) as e:
        kf.propagate_update_host(dict(host, geom=2))
    assert e.value.code == 2
    kf.release_host()
