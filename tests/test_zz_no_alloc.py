"""The allocation-free host load (rt_set_rays_host_noalloc) against the
ordinary one (rt_set_rays from host memory): the same state, columns,
counters and next step, bit for bit, on two calls in a row on one context
(the second with fewer volumes), with no device allocation requested during
either call.  The first call spans three staging chunks (the last one
ragged)."""
import numpy as np
import pytest

from paper_2309_11257_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_11257_amd import _rt
    _rt.lib()
    return _rt


def _same(a, b):
    assert set(a) == set(b)
    for f in a:
        assert np.array_equal(np.asarray(a[f]), np.asarray(b[f])), f


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_load_matches_set_rays(rt, prec):
    w = W.make_c3(n_rays=300_000, nx=90, ny=45, nz=60)
    p = rt.RT_FP64 if prec == "fp64" else rt.RT_FP32
    chunk = 131072
    first = {k: v.copy() for k, v in w.rays.items()}
    assert 2 * chunk < len(first["id"]) < 3 * chunk
    second = W.subset_rays(w.rays, 1000, seed=5)
    tr = rt.Tracer.for_workload(w, p)
    tr.init_background_from(w)
    for rays in (first, second):
        ref = rt.Tracer.for_workload(w, p)
        ref.init_background_from(w)
        ref.set_rays(rays)
        before = tr.n_alloc_calls
        tr.set_rays_host_noalloc(rays)
        assert tr.n_alloc_calls == before, "the allocation-free load asked for device memory"
        _same(tr.get_rays(), ref.get_rays())
        assert np.array_equal(tr.get_columns(), ref.get_columns())
        assert tr.stats() == ref.stats()
        tr.step(w.dt)
        ref.step(w.dt)
        _same(tr.get_rays(), ref.get_rays())
        assert tr.stats() == ref.stats()
        ref.close()
    # over capacity: refused, the context keeps its set
    big = {k: np.concatenate([v, v]) for k, v in first.items()}
    n_before = tr.stats()["n_active"]
    with pytest.raises(rt.RTError) as e:
        tr.set_rays_host_noalloc(big)
    assert e.value.code == rt.RT_E_CAPACITY
    assert tr.stats()["n_active"] == n_before
    tr.close()


def test_noalloc_load_empty(rt):
    w = W.make_c1(n_rays=16)
    tr = rt.Tracer.for_workload(w, rt.RT_FP64)
    tr.init_background_from(w)
    tr.set_rays_host_noalloc({k: v[:0] for k, v in w.rays.items()})
    assert tr.stats()["n_active"] == 0
    tr.set_rays_host_noalloc(w.rays)
    assert tr.stats()["n_active"] == 16
    tr.close()
