"""Shared test helpers: run the oracle and the GPU library on the same seeded
inputs and line their outputs up by ray id."""
import numpy as np

FIELDS = ("x", "y", "z", "k", "l", "m", "dx", "dy", "dz", "px", "py", "pz", "n")
EVOLVING = ("x", "y", "z", "k", "l", "m", "dx", "dy", "dz")


def by_id(d):
    o = np.argsort(d["id"], kind="stable")
    return {k: np.asarray(v)[o] for k, v in d.items()}


def oracle_run(orc, w, steps, dt=None, rays=None):
    bg = orc.Background.from_workload(w)
    rs = orc.RaySet(rays if rays is not None else w.rays)
    tallies = []
    for _ in range(steps):
        tallies.append(orc.step(bg, rs, w.dt if dt is None else dt))
    return bg, rs, tallies


def gpu_tracer(w, precision, rays=None, capacity=None):
    from paper_2309_11257_amd import _rt
    tr = _rt.Tracer.for_workload(w, precision, capacity=capacity)
    tr.init_background_from(w)
    tr.set_rays(rays if rays is not None else w.rays)
    return tr


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt((b * b).sum())
    return float(np.sqrt(((a - b) ** 2).sum()) / den) if den > 0 else float(np.sqrt((a * a).sum()))


def assert_flux_close(got, ref, rtol, what=""):
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max()
    assert err <= rtol * max(scale, 1e-300), f"{what}: max abs err {err:.3e} vs scale {scale:.3e}"
