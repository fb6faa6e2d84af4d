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


def oracle_deposit_with_kernel_decisions(orc, bg, rs, gpu_rays, gpu_cols):
    """Oracle fluxes of the oracle's own ray states, with the integer
    decisions (which rays are active, which column each belongs to) taken
    from the kernel's output.  Returns (flux, n_column_flips, n_set_flips)."""
    ids = rs["id"]
    active = rs.active()
    gid = np.asarray(gpu_rays["id"])
    o = np.argsort(gid, kind="stable")
    gs, gc = gid[o], np.asarray(gpu_cols).astype(np.int64)[o]
    if gs.size:
        p = np.clip(np.searchsorted(gs, ids), 0, gs.size - 1)
        found = gs[p] == ids
    else:
        p = np.zeros(ids.size, dtype=np.int64)
        found = np.zeros(ids.size, dtype=bool)
    cols = np.where(found & active, gc[p] if gs.size else -1, -1)
    n_set = int((found != active).sum())
    flips = int(((cols != rs["col"]) & (cols >= 0)).sum())
    save = rs.a["state"][: rs.n].copy()
    rs.a["state"][: rs.n][active & ~found] = orc.INVALID
    flux = orc.deposit(bg, rs, cols=cols)
    rs.a["state"][: rs.n] = save
    return flux, flips, n_set


def fp32_representable(w, rays):
    """The ray set rounded to what the single-precision state can hold
    exactly: wavenumbers, extents and phase-space areas to float32, horizontal
    positions to (cell + float32 offset) and heights to (level + float32
    offset).  Feeding these to both the oracle and the FP32 path isolates the
    error made inside the steps from the rounding of the inputs."""
    f32 = lambda a: np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)
    r = {k: np.array(v, copy=True) for k, v in rays.items()}
    for f in ("k", "l", "m", "dz", "px", "py", "pz"):
        r[f] = f32(r[f])
    gx = (r["x"] - w.x0) / w.dx
    i = np.clip(np.floor(gx), 0, w.nx - 1)
    r["x"] = w.x0 + (i + f32(gx - i)) * w.dx
    gy = (r["y"] - w.y0) / w.dy
    j = np.clip(np.floor(gy), 0, w.ny - 1)
    r["y"] = w.y0 + (j + f32(gy - j)) * w.dy
    gz = r["z"] / w.dz
    kz = np.clip(np.floor(gz), 0, w.nz)
    r["z"] = (kz + f32(gz - kz)) * w.dz
    r["dx"] = f32(r["dx"] / w.dx) * w.dx
    r["dy"] = f32(r["dy"] / w.dy) * w.dy
    return r
