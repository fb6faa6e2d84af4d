"""The boundary's numeric-failure contract: a volume that cannot be carried
on (a non-finite state, a zero wavevector, or a state that overflows during
a step) is deactivated and counted, rt_get_stats reports RT_E_NUMERIC once
with the smallest offending id, and the rest of the set steps exactly as it
does without the offending volumes.  The oracle deactivates the same ids."""
import numpy as np
import pytest

from paper_2309_11257_amd import workloads as W
from helpers import FIELDS, by_id, gpu_tracer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_11257_amd import _rt
    _rt.lib()
    return _rt


def _stats_expect_numeric(rt, tr):
    with pytest.raises(rt.RTError) as e:
        tr.stats()
    assert e.value.code == rt.RT_E_NUMERIC
    return e.value.stats


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bad_volumes_reported_and_rest_unchanged(rt, orc, prec):
    cols = np.sort(np.random.default_rng(71).choice(128 * 128, 200, replace=False))
    w = W.make_c2(cols=cols)
    rays = {k: v.copy() for k, v in w.rays.items()}
    ia, ib, ic = 17, 5, 300  # ids equal slots here
    assert np.array_equal(rays["id"][[ia, ib, ic]], [ia, ib, ic])
    rays["m"][ia] = np.nan                                   # non-finite at load
    rays["k"][ib] = rays["l"][ib] = rays["m"][ib] = 0.0     # K^2 = 0 at load
    rays["m"][ic] = 1e300                                    # K^2 overflows in the step
    P = rt.RT_FP64 if prec == "fp64" else rt.RT_FP32
    tr = gpu_tracer(w, P, rays=rays)
    s = _stats_expect_numeric(rt, tr)
    assert s["first_bad_id"] == ib and s["n_invalid"] == 2
    assert s["n_active"] == rays["x"].size - 2
    s = tr.stats()  # reported once
    assert s["first_bad_id"] == -1 and s["n_invalid"] == 2
    tr.step(w.dt)
    s = _stats_expect_numeric(rt, tr)
    assert s["first_bad_id"] == ic and s["n_invalid"] == 3
    assert tr.stats()["first_bad_id"] == -1

    # the same set without the three volumes, stepped once: identical in
    # double precision.  In single precision a wave whose volumes all stay in
    # its staged stencil box interpolates from the box, and any other wave
    # (here the one holding the overflowing volume) from global memory; the
    # two forms agree to the last bit or two of a cell-relative position
    keep = np.ones(rays["x"].size, bool)
    keep[[ia, ib, ic]] = False
    clean = {k: v[keep] for k, v in w.rays.items()}
    tc = gpu_tracer(w, P, rays=clean)
    tc.step(w.dt)
    g, c = by_id(tr.get_rays()), by_id(tc.get_rays())
    assert np.array_equal(g["id"], c["id"])
    spacing = {"x": w.dx, "y": w.dy, "z": w.dz}
    for f in FIELDS:
        if prec == "fp64":
            assert np.array_equal(g[f], c[f]), f
        elif f in spacing:
            assert (np.abs(g[f] - c[f]) <= 2.0 ** -23 * spacing[f]).all(), f
        else:
            assert (np.abs(g[f] - c[f]) <= 1e-6 * np.abs(c[f])).all(), f
    if prec == "fp64":  # sums over the same set in the same order
        assert tr.stats()["sum_W"] == tc.stats()["sum_W"]

    # the oracle deactivates the same ids
    bg = orc.Background.from_workload(w)
    rs = orc.RaySet(rays)
    t = orc.step(bg, rs, w.dt)
    assert t["n_invalid"] == 3
    assert np.array_equal(np.sort(rs.snapshot()["id"]), g["id"])


def test_numeric_report_survives_split_merge_statistics(rt):
    """rt_split_merge's statistics show the offending id without clearing
    the report; the next rt_get_stats still returns RT_E_NUMERIC."""
    cols = np.sort(np.random.default_rng(72).choice(128 * 128, 50, replace=False))
    w = W.make_c2(cols=cols)
    rays = {k: v.copy() for k, v in w.rays.items()}
    rays["dz"][9] = -1.0  # a non-positive extent
    tr = gpu_tracer(w, rt.RT_FP64, rays=rays)
    sm = tr.split_merge(0.0, 0, rt.RT_SPLIT_ONLY)
    assert sm["first_bad_id"] == 9
    s = _stats_expect_numeric(rt, tr)
    assert s["first_bad_id"] == 9 and s["n_invalid"] == 1
    assert tr.stats()["first_bad_id"] == -1
