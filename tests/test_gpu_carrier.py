"""The deposition after a step takes N^2, f^2 (and Gamma^2) at each carrier
from the values the step wrote with the new state (read from the wave's
stencil box where the step had it) instead of interpolating them again.  It
must give the same fluxes and drag as the deposition that interpolates
(forced by installing the same background again, which invalidates the
step's values), with and without the scale-height correction, on the sphere
and on the box: bit for bit in double precision; in single precision the
box and global-memory forms of one interpolation may round differently by
an ulp (contractions), so there the fluxes agree to 2^-20 of each field's
largest value."""
import numpy as np
import pytest

from paper_2309_11257_amd import workloads as W
from helpers import gpu_tracer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_11257_amd import _rt
    _rt.lib()
    return _rt


def _workload(name, gam):
    if name == "sphere":
        w = W.make_c3(n_rays=60_000)
    else:
        cols = np.sort(np.random.default_rng(5).choice(128 * 128, 400, replace=False))
        w = W.make_c2(cols=cols)
    if gam:
        w.G2 = W.density_gamma2(w)
    return w


@pytest.mark.parametrize("gam", [False, True])
@pytest.mark.parametrize("name", ["sphere", "box"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_carrier_background_from_the_step_equals_interpolated(rt, prec, name, gam):
    w = _workload(name, gam)
    tr = gpu_tracer(w, rt.RT_FP64 if prec == "fp64" else rt.RT_FP32)
    for _ in range(3):
        tr.step(w.dt)
    f_car, d_car = tr.deposit(host=True)
    tr.init_background_from(w)  # the same fields: the step's carrier values no longer count
    f_int, d_int = tr.deposit(host=True)
    assert np.any(f_car != 0.0)
    if prec == "fp64":
        assert np.array_equal(f_car, f_int), np.abs(f_car - f_int).max()
        assert np.array_equal(d_car, d_int)
    else:
        for q in range(f_car.shape[0]):
            sc = np.abs(f_int[q]).max()
            assert np.abs(f_car[q] - f_int[q]).max() <= 2.0 ** -20 * sc, q
        for q in range(d_car.shape[0]):
            sc = np.abs(d_int[q]).max()
            assert np.abs(d_car[q] - d_int[q]).max() <= 2.0 ** -20 * sc, q
    tr.close()
