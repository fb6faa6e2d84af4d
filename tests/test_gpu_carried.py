"""The step leaves each volume's px, py, pz and id (and, in double precision,
its wave-action density) in the slot they were loaded into and passes that
slot on with the evolving state.
After any number of steps every reader (rt_get_rays, the removal tallies and
their first invalid id) must still see each volume's own values, and every
operation that rewrites the set (split/merge, launch, a new load) must start
from them."""
import numpy as np
import pytest

from paper_2309_11257_amd import workloads as W
from helpers import FIELDS, by_id, fp32_representable, gpu_tracer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_11257_amd import _rt
    _rt.lib()
    return _rt


def distinct_extents(rays, seed):
    """The rays with px, py, pz different for every volume (so a volume
    reading another's values is seen) and exactly representable in single
    precision."""
    rays = {k: np.array(v, copy=True) for k, v in rays.items()}
    rng = np.random.default_rng(seed)
    for f in ("px", "py", "pz"):
        rays[f] = np.float32(rays[f] * rng.uniform(0.5, 2.0, rays[f].size)).astype(np.float64)
    return rays


def check_own_values(got, loaded):
    """Every volume in `got` carries the px, py, pz it was loaded with."""
    where = {int(v): j for j, v in enumerate(loaded["id"])}
    idx = np.array([where[int(v)] for v in np.asarray(got["id"])])
    for f in ("px", "py", "pz"):
        assert np.array_equal(np.asarray(got[f]), loaded[f][idx]), f
    return idx


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_carried_fields_after_steps(rt, prec):
    """Nine steps over several radix tiles with volumes changing column and
    leaving through the top (removal tallies read the ids through the home
    slots); the wave action of every remaining volume is its own."""
    w = W.make_c3(n_rays=60_000)
    rays = distinct_extents(w.rays, 5)
    tr = gpu_tracer(w, rt.RT_FP32 if prec == "fp32" else rt.RT_FP64, rays=rays)
    W0 = rays["n"] * rays["px"] * rays["py"] * rays["pz"]
    n0 = rays["x"].size
    for s in range(1, 10):
        tr.step(w.dt * 40)
        g = tr.get_rays()
        idx = check_own_values(g, rays)
        Wg = np.asarray(g["n"]) * np.asarray(g["px"]) * np.asarray(g["py"]) * np.asarray(g["pz"])
        assert np.allclose(Wg, W0[idx], rtol=1e-12, atol=0), s
    try:
        st = tr.stats()
    except rt.RTError as e:  # volumes deactivated as non-finite are reported
        st = e.stats
    assert st["n_active"] < n0, "no volume left the set (the tallies read nothing)"
    assert st["n_active"] + sum(st[k] for k in ("n_top", "n_bottom", "n_pole", "n_invalid")) == n0
    tr.close()


def test_split_merge_after_steps_matches_oracle(rt, orc):
    """Steps leave px, py, pz and id at their home slots; a split/merge then
    gathers them back and works on the stepped set exactly as the oracle's
    split and merge of that set do: the same ids, counts, and every field
    within single-precision rounding."""
    w = W.make_c2(cols=np.arange(0, 128 * 128, 331))
    rays = {k: v.copy() for k, v in w.rays.items()}
    rng = np.random.default_rng(94)
    rays["dz"] = rays["dz"] * rng.choice([1.0, 2.5, 5.5], rays["dz"].size)
    rays = fp32_representable(w, rays)
    rays = distinct_extents(rays, 6)
    cap = 8 * rays["x"].size
    tr = gpu_tracer(w, rt.RT_FP32, rays=rays, capacity=cap)
    for _ in range(3):
        tr.step(w.dt)
    stepped = tr.get_rays()
    check_own_values(stepped, rays)
    bg = orc.Background.from_workload(w)
    # the oracle's ray set is in ascending id order (new ids follow it)
    rs = orc.RaySet(by_id(stepped), capacity=cap)
    # new ids continue from the largest id loaded (volumes that left during
    # the steps included)
    to = orc.split(bg, rs, w.split_alpha, next_id=int(rays["id"].max()) + 1)
    mo = orc.merge(bg, rs, 16)
    st = tr.split_merge(w.split_alpha, 16, rt.RT_MERGE)
    assert st["n_split"] == to["n_split"] > 0
    assert st["n_merged"] == mo["n_merged"] > 0
    o, g = by_id(rs.snapshot()), by_id(tr.get_rays())
    assert np.array_equal(o["id"], g["id"])
    for f in FIELDS:
        # a merged volume's W-weighted wavevector can nearly cancel: errors
        # are measured against a twentieth of the field's RMS at least
        sc = np.maximum(np.abs(o[f]), 0.05 * np.sqrt(np.mean(o[f] ** 2)))
        if f in ("x", "y", "z"):
            sc = np.maximum(sc, {"x": w.dx, "y": w.dy, "z": w.dz}[f])
        e = float((np.abs(g[f] - o[f]) / np.maximum(sc, 1e-300)).max())
        assert e <= 2e-6, (f, e)
    # and the set keeps stepping from the gathered fields
    tr.step(w.dt)
    after = by_id(tr.get_rays())
    keep = np.isin(g["id"], after["id"])
    where = {int(v): j for j, v in enumerate(after["id"])}
    j = np.array([where[int(v)] for v in g["id"][keep]])
    for f in ("px", "py", "pz"):
        assert np.array_equal(after[f][j], g[f][keep]), f
    tr.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_launch_and_reload_after_steps(rt, prec):
    """A launch after steps keeps every stepped volume's own px, py, pz; a new
    load after steps starts from the loaded values."""
    cols = np.sort(np.random.default_rng(65).choice(128 * 128, 300, replace=False))
    w = W.make_c2(cols=cols)
    rays = distinct_extents(w.rays, 7)
    flux = np.zeros(w.nx * w.ny)
    flux[cols] = np.random.default_rng(66).uniform(1e-3, 4e-3, cols.size)
    prm = dict(lambda_h=150e3, c_min=2.0, c_max=34.0, c_center=15.0, c_width=10.0, n_speeds=8)
    cap = rays["x"].size + 4 * 4 * prm["n_speeds"] * cols.size
    tr = gpu_tracer(w, rt.RT_FP32 if prec == "fp32" else rt.RT_FP64, rays=rays, capacity=cap)
    for s in range(2):
        tr.step(w.dt)
    before = by_id(tr.get_rays())
    nl = tr.launch(0.5 * w.nz * w.dz, w.dt, flux_col=flux, **prm)
    assert nl > 0
    g = by_id(tr.get_rays())
    old = np.isin(g["id"], before["id"])
    assert np.count_nonzero(old) == before["id"].size
    for f in ("px", "py", "pz"):
        assert np.array_equal(g[f][old], before[f]), f
    tr.step(w.dt)
    tr.step(w.dt)
    g2 = tr.get_rays()
    ids = np.asarray(g2["id"])
    where = {int(v): j for j, v in enumerate(g["id"])}
    idx = np.array([where[int(v)] for v in ids])
    for f in ("px", "py", "pz"):
        assert np.array_equal(np.asarray(g2[f]), g[f][idx]), f
    # a new load after steps
    tr.set_rays(rays)
    check_own_values(tr.get_rays(), rays)
    tr.step(w.dt)
    check_own_values(tr.get_rays(), rays)
    tr.close()
