"""Column features and frozen-column steps on the GPU against the oracle."""
import numpy as np
import pytest

from paper_2309_11257_amd import workloads as W
from helpers import EVOLVING, by_id, gpu_tracer, oracle_run, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_11257_amd import _rt
    _rt.lib()
    return _rt


def workloads():
    yield "box", W.make_c1(n_rays=2000)
    yield "jet", W.make_c2(cols=np.arange(0, 16384, 97))
    yield "sphere", W.make_c3(n_rays=60000)


@pytest.mark.parametrize("name", ["box", "jet", "sphere"])
def test_features_fp64_match_oracle(rt, orc, name):
    w = dict(workloads())[name]
    bg, rs, _ = oracle_run(orc, w, 1)
    ref = orc.features(bg, rs)
    tr = gpu_tracer(w, rt.RT_FP64)
    tr.step(w.dt)
    got = tr.features(host=True)
    nz = w.nz
    assert got.shape == ref.shape
    # profiles: the float32 rounding of the inputs
    assert np.array_equal(got[:, :3 * nz], ref[:, :3 * nz].astype(np.float32))
    # moments: double sums in another order, rounded to float32; the height
    # spread (one-pass variance) within its cancellation floor
    g6 = got[:, 3 * nz:].reshape(-1, 8, 6)
    r6 = ref[:, 3 * nz:].reshape(-1, 8, 6)
    assert np.allclose(g6[:, :, :5], r6[:, :, :5].astype(np.float32), rtol=4e-7, atol=0)
    assert np.allclose(g6[:, :, 5], r6[:, :, 5], rtol=1e-6, atol=1e-6 * 100e3)
    assert (r6[:, :, 0] > 0).sum() > 20
    # the device entry point gives the same matrix
    assert np.array_equal(tr.features().cpu().numpy(), got)
    tr.close()


def test_features_fp32_close(rt, orc):
    w = W.make_c3(n_rays=60000)
    bg, rs, _ = oracle_run(orc, w, 1)
    ref = orc.features(bg, rs)
    tr = gpu_tracer(w, rt.RT_FP32)
    tr.step(w.dt)
    got = tr.features(host=True)
    nz = w.nz
    assert rel_l2(got[:, 3 * nz:], ref[:, 3 * nz:]) <= 1e-5
    tr.close()


def test_features_empty_set(rt):
    w = W.make_c1(n_rays=16)
    w.rays["z"][:] = 1e6  # every volume leaves through the top on load
    tr = gpu_tracer(w, rt.RT_FP64)
    X = tr.features(host=True)
    assert np.all(X[:, 3 * w.nz:] == 0)
    tr.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_frozen_columns(rt, orc, precision):
    """Volumes in flagged columns keep their state; the others take the
    ordinary step (bitwise the oracle's in double precision)."""
    w = W.make_c2(cols=np.arange(0, 16384, 131))
    prec = rt.RT_FP64 if precision == "fp64" else rt.RT_FP32
    tr = gpu_tracer(w, prec)
    g0 = by_id(tr.get_rays())
    c0 = tr.get_columns()[np.argsort(tr.get_rays()["id"], kind="stable")]
    mask = np.zeros(w.nx * w.ny, np.uint8)
    mask[::2] = 1
    tr.set_frozen_columns(mask)
    tr.step(w.dt, surrogate=True)
    g1 = by_id(tr.get_rays())
    assert np.array_equal(g0["id"], g1["id"])
    frozen = mask[c0].astype(bool)
    assert frozen.sum() > 100 and (~frozen).sum() > 100
    for f in EVOLVING:
        assert np.array_equal(g1[f][frozen], g0[f][frozen]), f
    if precision == "fp64":
        _, rs, _ = oracle_run(orc, w, 1)
        o = by_id(rs.snapshot())
        for f in EVOLVING:
            assert np.array_equal(g1[f][~frozen], o[f][~frozen]), f
    # all flags clear: identical to a plain step
    tr2 = gpu_tracer(w, prec)
    tr2.set_frozen_columns(None)
    tr2.step(w.dt, surrogate=True)
    tr3 = gpu_tracer(w, prec)
    tr3.step(w.dt)
    a, b = by_id(tr2.get_rays()), by_id(tr3.get_rays())
    for f in EVOLVING:
        assert np.array_equal(a[f], b[f]), f
    for t in (tr, tr2, tr3):
        t.close()


def test_surrogate_flag_needs_flags(rt):
    w = W.make_c1(n_rays=64)
    tr = gpu_tracer(w, rt.RT_FP64)
    with pytest.raises(rt.RTError) as e:
        tr.step(w.dt, surrogate=True)
    assert e.value.code == rt.RT_E_STATE
    tr.close()
