"""GPU parity of the full flux formulation, the horizontal smoothing and the
wave-action budget (rt_full_fluxes, rt_budget) against the FP64 oracle on
the same seeded inputs, both precisions, with and without smoothing."""
import numpy as np
import pytest

from paper_2309_11257_amd import workloads as W
from helpers import kernel_columns, record_metric, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_11257_amd import _rt
    _rt.lib()
    return _rt


def workload(name):
    if name == "box":
        cols = np.sort(np.random.default_rng(2).choice(128 * 128, 500, replace=False))
        return W.make_c2(cols=cols)
    return W.make_c3(n_rays=120_000)


def per_field_err(got, ref):
    """largest difference of each field relative to that field's largest value"""
    out = []
    for q in range(ref.shape[0]):
        sc = np.abs(ref[q]).max()
        out.append(float(np.abs(got[q] - ref[q]).max() / sc) if sc > 0 else float(np.abs(got[q]).max()))
    return out


@pytest.mark.parametrize("smooth", [False, True])
@pytest.mark.parametrize("name", ["box", "sphere"])
def test_fp64_full_fluxes_and_budget(rt, orc, name, smooth):
    """Every full-flux, buoyancy-flux and budget field within 1e-12 of the
    oracle (relative to the field's largest value), the tendencies and
    propagation terms within 1e-12 relative L2, after three steps."""
    from helpers import gpu_tracer
    w = workload(name)
    bg = orc.Background.from_workload(w)
    rs = orc.RaySet(w.rays)
    tr = gpu_tracer(w, rt.RT_FP64)
    for _ in range(3):
        orc.step(bg, rs, w.dt)
        tr.step(w.dt)
    F = orc.full_fluxes(bg, rs)
    B = orc.budget(bg, rs)
    if smooth:
        F = orc.smooth(bg, F)
        B = orc.smooth(bg, B)
    T = orc.full_tendencies(bg, F)
    Tb = orc.budget_terms(bg, B)
    flux, tend = tr.full_fluxes(smooth=smooth, host=True)
    fields, terms = tr.budget(smooth=smooth, host=True)
    ef, eb = per_field_err(flux, F), per_field_err(fields, B)
    et = [rel_l2(tend[q], T[q]) for q in range(3)]
    etb = [rel_l2(terms[q], Tb[q]) for q in range(2)]
    record_metric(f"fp64_full_fluxes_{name}_{'smooth' if smooth else 'raw'}", flux=max(ef), tend=max(et),
                  budget=max(eb), terms=max(etb))
    assert max(ef) <= 1e-12, ef
    assert max(eb) <= 1e-12, eb
    assert max(et) <= 1e-12, et
    assert max(etb) <= 1e-12, etb
    if name == "sphere":
        assert np.abs(F[4:6]).max() > 0  # rotation: a buoyancy flux and an elastic term
    tr.close()


@pytest.mark.parametrize("name", ["box", "sphere"])
def test_fp32_full_fluxes_and_budget(rt, orc, name):
    """Single precision after one step: fluxes, budget fields, tendencies and
    terms within 1e-5 relative L2 of the oracle, which takes the kernel's
    column for a volume at a cell face."""
    from helpers import gpu_tracer
    w = workload(name)
    bg = orc.Background.from_workload(w)
    rs = orc.RaySet(w.rays)
    orc.step(bg, rs, w.dt)
    tr = gpu_tracer(w, rt.RT_FP32)
    tr.step(w.dt)
    cols, flips = kernel_columns(bg, rs, tr.get_rays(), tr.get_columns())
    assert flips <= 2
    F = orc.smooth(bg, orc.full_fluxes(bg, rs, cols=cols))
    B = orc.smooth(bg, orc.budget(bg, rs, cols=cols))
    T = orc.full_tendencies(bg, F)
    Tb = orc.budget_terms(bg, B)
    flux, tend = tr.full_fluxes(smooth=True, host=True)
    fields, terms = tr.budget(smooth=True, host=True)
    errs = {"flux": max(rel_l2(flux[q], F[q]) for q in range(8) if np.abs(F[q]).max() > 0),
            "tend": max(rel_l2(tend[q], T[q]) for q in range(3)),
            "budget": max(rel_l2(fields[q], B[q]) for q in range(4)),
            "terms": max(rel_l2(terms[q], Tb[q]) for q in range(2))}
    record_metric(f"fp32_full_fluxes_{name}", column_flips=flips, **errs)
    for k, v in errs.items():
        assert v <= 1e-5, (k, v)
    tr.close()


def test_full_fluxes_deterministic_and_pseudo_consistent(rt):
    """Repeated calls give the same bits; with f = 0 the full momentum flux
    equals the pseudo-momentum flux of rt_deposit_flux (bit for bit in the
    fields both deposit the same way) and the buoyancy flux is zero."""
    from helpers import gpu_tracer
    w = W.make_c1(n_rays=2048)
    w.f[:] = 0.0
    tr = gpu_tracer(w, rt.RT_FP64)
    for _ in range(3):
        tr.step(w.dt)
    a, ta = tr.full_fluxes(host=True)
    b, tb = tr.full_fluxes(host=True)
    assert np.array_equal(a, b) and np.array_equal(ta, tb)
    pf, pd = tr.deposit(host=True)
    for q_full, q_pseudo in zip((0, 1, 2, 3, 6, 7), range(6)):
        sc = np.abs(pf[q_pseudo]).max()
        assert np.abs(a[q_full] - pf[q_pseudo]).max() <= 1e-14 * sc
    assert not a[4:6].any()
    assert rel_l2(ta[:2], pd) <= 1e-14
    tr.close()
