"""Seeded synthetic workloads for the ray-volume tracer.

This module only builds inputs: grids, resolved background fields and initial
ray volumes.  It holds none of the tracer's arithmetic (no dispersion
relation, group velocity, interpolation or flux), so the CPU oracle and the
GPU library can both be fed from it without sharing any of the method.

Every generator is deterministic for a given seed (numpy PCG64).  Ray volumes
are described by

    x, y, z      carrier position (m, or lon rad / lat rad / height m)
    k, l, m      carrier wavevector (rad/m)
    dx, dy, dz   physical extents in coordinate units (m, or rad, rad, m)
    px, py, pz   phase-space areas  (metric extent) x (wavenumber extent),
                 which stay fixed while the volume deforms (Section 3a)
    n            phase-space wave-action density N (constant inside a volume)
    id           unique int64 label

The workload shapes follow the paper's setting: a launch layer of ray volumes
(Section 3c launches at 300 hPa, about 9 km; the convective source launches at
cloud top) with wavelengths of tens to hundreds of kilometres, a latitudinal
background-source profile alpha(phi) with winter/summer fluxes of 8 and
2.4 mPa, and clustered convective sources.  Wave-action amplitudes are set
from a launch flux F as N = F / (k_h dk dl dm * 1 m/s): a synthetic amplitude
with the paper's units of flux, not a physical launch condition.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional

import numpy as np

RAY_FIELDS = ("x", "y", "z", "k", "l", "m", "dx", "dy", "dz", "px", "py", "pz", "n")

CARTESIAN = 0
SPHERICAL = 1

EARTH_RADIUS = 6.371e6
EARTH_OMEGA = 7.292e-5


@dataclass
class Workload:
    name: str
    geometry: int
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    x0: float
    y0: float
    a: float
    U: np.ndarray  # [nz][ny][nx]
    V: np.ndarray
    N2: np.ndarray
    f: np.ndarray  # [ny]
    rho: np.ndarray  # [nz]
    rays: Dict[str, np.ndarray]
    dt: float
    steps: int
    split_alpha: Optional[float] = None
    merge_nmax: Optional[int] = None
    meta: dict = field(default_factory=dict)
    G2: Optional[np.ndarray] = None  # scale-height correction Gamma^2 [nz][ny][nx]; None: Gamma = 0

    @property
    def n_rays(self) -> int:
        return int(self.rays["x"].shape[0])

    @property
    def n_cols(self) -> int:
        return self.nx * self.ny

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    def grid_dict(self) -> dict:
        return dict(geometry=self.geometry, nx=self.nx, ny=self.ny, nz=self.nz,
                    dx=self.dx, dy=self.dy, dz=self.dz, x0=self.x0, y0=self.y0, a=self.a)

    def copy_rays(self) -> Dict[str, np.ndarray]:
        return {k: v.copy() for k, v in self.rays.items()}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _density(zc: np.ndarray) -> np.ndarray:
    # isothermal reference density, 7 km scale height
    return 1.2 * np.exp(-zc / 7.0e3)


def _pack(x, y, z, k, l, m, ex, ey, ez, exm, eym, dk, dl, dm, n) -> Dict[str, np.ndarray]:
    """exm/eym: extents in metres (for the phase-space areas)."""
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    r = dict(x=f64(x), y=f64(y), z=f64(z), k=f64(k), l=f64(l), m=f64(m),
             dx=f64(ex), dy=f64(ey), dz=f64(ez),
             px=f64(exm * dk), py=f64(eym * dl), pz=f64(ez * dm), n=f64(n))
    r["id"] = np.arange(r["x"].shape[0], dtype=np.int64)
    return r


# --------------------------------------------------------------------------
# C1: 16x16x64 periodic box, constant N, tanh shear U(z), 4096 rays at 3 km
# --------------------------------------------------------------------------
def make_c1(seed: int = 1, n_rays: int = 4096) -> Workload:
    nx, ny, nz = 16, 16, 64
    dx = dy = 50.0e3
    dz = 1.0e3
    zc = (np.arange(nz) + 0.5) * dz
    U = np.broadcast_to((20.0 * np.tanh((zc - 20.0e3) / 5.0e3))[:, None, None], (nz, ny, nx)).copy()
    V = np.zeros((nz, ny, nx))
    N2 = np.full((nz, ny, nx), 0.02 * 0.02)
    f = np.full(ny, 1.0e-4)
    g = _rng(seed)
    x = g.uniform(0.0, nx * dx, n_rays)
    y = g.uniform(0.0, ny * dy, n_rays)
    z = np.full(n_rays, 3.0e3)
    lam_h = g.uniform(50.0e3, 500.0e3, n_rays)
    lam_z = g.uniform(2.0e3, 10.0e3, n_rays)
    th = g.uniform(0.0, 2.0 * np.pi, n_rays)
    amp = np.abs(g.standard_normal(n_rays))
    kh = 2.0 * np.pi / lam_h
    k, l = kh * np.cos(th), kh * np.sin(th)
    m = -2.0 * np.pi / lam_z
    dk = dl = 0.1 * kh
    dm = 0.1 * np.abs(m)
    F = 1.0e-3 * amp
    n = F / (kh * dk * dl * dm * 1.0)
    ex = np.full(n_rays, dx)
    ey = np.full(n_rays, dy)
    ez = np.full(n_rays, dz)
    rays = _pack(x, y, z, k, l, m, ex, ey, ez, ex, ey, dk, dl, dm, n)
    return Workload("c1", CARTESIAN, nx, ny, nz, dx, dy, dz, 0.0, 0.0, EARTH_RADIUS,
                    U, V, N2, f, _density(zc), rays, dt=60.0, steps=100)


# --------------------------------------------------------------------------
# C2: 128x128x90 box, zonal jet U(y,z), tropopause jump in N^2, 2M rays as
# 16384 columns x 8 azimuths x 16 phase speeds at 5 km; split + merge
# --------------------------------------------------------------------------
def make_c2(seed: int = 2, cols: Optional[np.ndarray] = None, nx: int = 128, ny: int = 128) -> Workload:
    nz = 90
    dx = dy = 25.0e3
    dz = 0.8e3
    zc = (np.arange(nz) + 0.5) * dz
    yc = (np.arange(ny) + 0.5) * dy
    y0 = 0.5 * ny * dy
    jet = 40.0 * np.exp(-((yc[None, :] - y0) / 800.0e3) ** 2 - ((zc[:, None] - 15.0e3) / 6.0e3) ** 2)
    U = np.broadcast_to(jet[:, :, None], (nz, ny, nx)).copy()
    V = np.zeros((nz, ny, nx))
    N2col = np.where(zc < 12.0e3, 1.0e-4, 4.0e-4)
    N2 = np.broadcast_to(N2col[:, None, None], (nz, ny, nx)).copy()
    f = np.full(ny, 1.0e-4)
    g = _rng(seed)
    ncol = nx * ny
    if cols is None:
        cols = np.arange(ncol)
    cols = np.asarray(cols, dtype=np.int64)
    per = 8 * 16
    nr = cols.size * per
    # per column: 8 azimuths x 16 intrinsic phase speeds
    th = np.tile(np.repeat(np.arange(8) * (np.pi / 4.0), 16), cols.size)
    c_hat = np.tile(np.tile(np.arange(1, 17) * 4.0, 8), cols.size)
    ci = np.repeat(cols % nx, per)
    cj = np.repeat(cols // nx, per)
    ux = g.uniform(0.0, 1.0, nr)
    uy = g.uniform(0.0, 1.0, nr)
    gn = g.standard_normal(nr)
    x = (ci + ux) * dx
    y = (cj + uy) * dy
    z = np.full(nr, 5.0e3)
    kh = np.full(nr, 2.0 * np.pi / 150.0e3)
    k, l = kh * np.cos(th), kh * np.sin(th)
    # launch-layer buoyancy frequency 0.01 s^-1; mid-frequency phase-speed
    # relation |m| = N / c_hat picks the vertical wavenumber of each bin
    m = -0.01 / c_hat
    w = np.exp(-((c_hat - 24.0) / 16.0) ** 2) * np.exp(0.3 * gn)
    wsum = w.reshape(cols.size, per).sum(axis=1)
    F = 2.0e-3 * w / np.repeat(wsum, per)
    dk = dl = 0.1 * kh
    dm = 0.1 * np.abs(m)
    n = F / (kh * dk * dl * dm * 1.0)
    ex = np.full(nr, dx)
    ey = np.full(nr, dy)
    ez = np.full(nr, dz)
    rays = _pack(x, y, z, k, l, m, ex, ey, ez, ex, ey, dk, dl, dm, n)
    return Workload("c2", CARTESIAN, nx, ny, nz, dx, dy, dz, 0.0, 0.0, EARTH_RADIUS,
                    U, V, N2, f, _density(zc), rays, dt=30.0, steps=500,
                    split_alpha=2.0, merge_nmax=64)


# --------------------------------------------------------------------------
# C3 / C5: global 1x1 degree lat-lon, 120 levels to 100 km, f = 2 Omega sin(phi)
# --------------------------------------------------------------------------
def _G(s, w):
    return np.exp(-(s / w) ** 2)


def _S(s):
    return 0.5 * (1.0 + np.tanh(s))


def _n2_profile(z):
    return 1.0e-4 + 3.5e-4 * _S((z - 12.0e3) / 1.0e3) - 1.5e-4 * _S((z - 50.0e3) / 3.0e3)


def _alpha(phi_deg):
    """Latitudinal profile of the background source (Section 3c)."""
    p = np.asarray(phi_deg, dtype=np.float64)
    out = np.zeros_like(p)
    hi = p >= 80.0
    out[hi] = np.minimum(1.0, np.maximum(0.0, 1.0 - (p[hi] - 80.0) / 5.0))
    mid = (p >= 50.0) & (p < 80.0)
    out[mid] = 1.0
    lo = (p >= 20.0) & (p < 50.0)
    out[lo] = 0.5 * (1.0 - np.cos(np.pi * (p[lo] - 20.0) / 30.0))
    return out


def f_sol(phi_deg, F_s=2.4e-3, F_w=8.0e-3):
    return _alpha(phi_deg) * F_s + _alpha(-np.asarray(phi_deg)) * F_w


def _largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    w = np.asarray(weights, dtype=np.float64)
    ideal = w / w.sum() * total
    base = np.floor(ideal).astype(np.int64)
    rem = total - int(base.sum())
    order = np.lexsort((np.arange(w.size), -(ideal - base)))
    base[order[:rem]] += 1
    return base


def make_global(name: str, seed: int, n_rays: int, nx: int = 360, ny: int = 180, nz: int = 120,
                steps: int = 200, dt: float = 20.0) -> Workload:
    dlam = 2.0 * np.pi / nx
    dphi = np.pi / ny
    dz = 100.0e3 / nz
    a = EARTH_RADIUS
    zc = (np.arange(nz) + 0.5) * dz
    phic = -0.5 * np.pi + (np.arange(ny) + 0.5) * dphi
    phid = np.degrees(phic)
    Uy = (30.0 * (_G(phid[None, :] - 30.0, 10.0) + _G(phid[None, :] + 30.0, 10.0)) * _G(zc[:, None] - 12.0e3, 5.0e3)
          + 80.0 * _G(phid[None, :] + 60.0, 12.0) * _G(zc[:, None] - 55.0e3, 15.0e3)
          - 60.0 * _G(phid[None, :] - 40.0, 15.0) * _G(zc[:, None] - 65.0e3, 12.0e3))
    U = np.broadcast_to(Uy[:, :, None], (nz, ny, nx)).copy()
    V = np.zeros((nz, ny, nx))
    N2 = np.broadcast_to(_n2_profile(zc)[:, None, None], (nz, ny, nx)).copy()
    f = 2.0 * EARTH_OMEGA * np.sin(phic)
    g = _rng(seed)

    # convective share: 40 clusters of 9x9 columns at |phi| < 25 deg, 10x the mean
    mean_per_col = n_rays / float(nx * ny)
    per_conv = max(1, int(round(10.0 * mean_per_col)))
    # 40 clusters of 9 x 9 columns on the 1-degree grid; on coarser grids the
    # clusters shrink with the grid so that they still cover 5 % of the columns
    n_clusters, side = 40, max(1, int(round(9 * nx / 360.0)))
    jrows = np.nonzero(np.abs(phid) < 25.0)[0]
    jlo, jhi = int(jrows.min()), int(jrows.max()) - side + 1
    taken = np.zeros((ny, nx), dtype=bool)
    clusters = []
    attempts = 0
    while len(clusters) < n_clusters:
        attempts += 1
        if attempts > 100000:
            raise ValueError("convective clusters do not fit the tropical band of this grid")
        ci = int(g.integers(0, nx))
        cj = int(g.integers(jlo, max(jlo + 1, jhi + 1)))
        ii = (ci + np.arange(side)) % nx
        jj = cj + np.arange(side)
        block = taken[np.ix_(jj, ii)]
        if block.any():
            continue
        taken[np.ix_(jj, ii)] = True
        clusters.append((ii, jj))
    conv_cols = []
    conv_z = []
    for ii, jj in clusters:
        zl = g.uniform(10.0e3, 16.0e3)
        for j in jj:
            for i in ii:
                conv_cols.append(j * nx + i)
                conv_z.append(zl)
    conv_cols = np.array(conv_cols, dtype=np.int64)
    conv_z = np.array(conv_z)
    n_conv = per_conv * conv_cols.size
    if n_conv > n_rays:
        raise ValueError("ray budget too small for the convective clusters")
    n_bg = n_rays - n_conv

    # background share: per-column counts proportional to F_sol(phi)
    wrow = f_sol(phid)
    wcol = np.broadcast_to(wrow[:, None], (ny, nx)).ravel()
    cnt_bg = _largest_remainder(wcol, n_bg)

    parts = []
    # convective rays
    cc = np.repeat(conv_cols, per_conv)
    zl = np.repeat(conv_z, per_conv)
    nr = cc.size
    lam_h = g.uniform(20.0e3, 200.0e3, nr)
    c_hat = g.uniform(5.0, 50.0, nr)
    th = g.uniform(0.0, 2.0 * np.pi, nr)
    amp = np.abs(g.standard_normal(nr))
    Fcol = 5.0e-3
    F = Fcol * amp / np.repeat(amp.reshape(-1, per_conv).sum(axis=1), per_conv)
    parts.append((cc, zl, lam_h, c_hat, th, F))
    # background rays
    bc = np.repeat(np.arange(nx * ny, dtype=np.int64), cnt_bg)
    nr = bc.size
    fj = f[bc // nx]
    lam_h = g.uniform(100.0e3, 1000.0e3, nr)
    kh = 2.0 * np.pi / lam_h
    c_hat = g.uniform(5.0, 60.0, nr)
    bad = kh * c_hat <= 1.05 * np.abs(fj)
    while bad.any():
        c_hat[bad] = g.uniform(5.0, 60.0, int(bad.sum()))
        bad = kh * c_hat <= 1.05 * np.abs(fj)
    rank = np.arange(nr) - np.repeat(np.cumsum(cnt_bg) - cnt_bg, cnt_bg)
    th = (rank % 4) * (np.pi / 2.0)
    Fb = np.repeat(wcol / np.maximum(cnt_bg, 1), cnt_bg)
    parts.append((bc, np.full(nr, 9.0e3), lam_h, c_hat, th, Fb))

    cols = np.concatenate([p[0] for p in parts])
    zl = np.concatenate([p[1] for p in parts])
    lam_h = np.concatenate([p[2] for p in parts])
    c_hat = np.concatenate([p[3] for p in parts])
    th = np.concatenate([p[4] for p in parts])
    F = np.concatenate([p[5] for p in parts])
    order = np.argsort(cols, kind="stable")
    cols, zl, lam_h, c_hat, th, F = (q[order] for q in (cols, zl, lam_h, c_hat, th, F))
    nr = cols.size
    ci, cj = cols % nx, cols // nx
    lam = (ci + g.uniform(0.0, 1.0, nr)) * dlam
    phi = -0.5 * np.pi + (cj + g.uniform(0.0, 1.0, nr)) * dphi
    kh = 2.0 * np.pi / lam_h
    k, l = kh * np.cos(th), kh * np.sin(th)
    m = -np.sqrt(_n2_profile(zl)) / c_hat
    dk = dl = 0.1 * kh
    dm = 0.1 * np.abs(m)
    n = F / (kh * dk * dl * dm * 1.0)
    ex = np.full(nr, dlam)
    ey = np.full(nr, dphi)
    ez = np.full(nr, dz)
    exm = ((a + zl) * np.cos(phi)) * dlam
    eym = (a + zl) * dphi
    rays = _pack(lam, phi, zl, k, l, m, ex, ey, ez, exm, eym, dk, dl, dm, n)
    wl = Workload(name, SPHERICAL, nx, ny, nz, dlam, dphi, dz, 0.0, -0.5 * np.pi, a,
                  U, V, N2, f, _density(zc), rays, dt=dt, steps=steps)
    wl.meta = dict(n_convective=int(n_conv), n_background=int(n_bg),
                   convective_columns=int(conv_cols.size), rays_per_convective_column=int(per_conv))
    return wl


def make_c3(seed: int = 3, n_rays: int = 20_000_000, **kw) -> Workload:
    return make_global("c3", seed, n_rays, **kw)


def make_c5(seed: int = 5, n_rays: int = 50_000_000, **kw) -> Workload:
    kw.setdefault("steps", 100)
    return make_global("c5", seed, n_rays, **kw)


def make_c4(run: int, n_rays: int = 5_000_000, nx: int = 360, ny: int = 180, steps: int = 200) -> Workload:
    """Surrogate training run `run`: the global recipe with seed 4000 + run,
    jet winds scaled by a seeded factor in [0.7, 1.3] and N^2 by one in
    [0.85, 1.15], so that the training backgrounds bracket the global one."""
    w = make_global(f"c4_{run}", 4000 + run, n_rays, nx=nx, ny=ny, steps=steps)
    g = _rng(9000 + run)
    w.U = w.U * g.uniform(0.7, 1.3)
    w.N2 = w.N2 * g.uniform(0.85, 1.15)
    return w


def make(name: str, **kw) -> Workload:
    return {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c5": make_c5}[name](**kw)


# --------------------------------------------------------------------------
# small analytic backgrounds used by the pin tests
# --------------------------------------------------------------------------
def analytic_box(nx=8, ny=8, nz=32, dx=20.0e3, dy=20.0e3, dz=500.0, U=None, V=None, N2=None,
                 f0=1.0e-4, name="box") -> Workload:
    """Cartesian box with fields given as callables of the cell-centre
    coordinates (xc, yc, zc) broadcast to [nz][ny][nx]; no rays."""
    xc = (np.arange(nx) + 0.5) * dx
    yc = (np.arange(ny) + 0.5) * dy
    zc = (np.arange(nz) + 0.5) * dz
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    ev = lambda fn, dflt: (np.broadcast_to(fn(X, Y, Z), (nz, ny, nx)).astype(np.float64).copy()
                           if fn is not None else np.full((nz, ny, nx), dflt))
    return Workload(name, CARTESIAN, nx, ny, nz, dx, dy, dz, 0.0, 0.0, EARTH_RADIUS,
                    ev(U, 0.0), ev(V, 0.0), ev(N2, 1.0e-4), np.full(ny, f0), _density(zc),
                    {f: np.zeros(0) for f in RAY_FIELDS} | {"id": np.zeros(0, np.int64)},
                    dt=60.0, steps=1)


def analytic_sphere(nx=72, ny=36, nz=20, top=40.0e3, U=None, N2=None, rotating=True,
                    name="sphere") -> Workload:
    """Lat-lon shell with fields as callables of (lam, phi, z); no rays."""
    dlam, dphi, dz = 2.0 * np.pi / nx, np.pi / ny, top / nz
    lc = (np.arange(nx) + 0.5) * dlam
    pc = -0.5 * np.pi + (np.arange(ny) + 0.5) * dphi
    zc = (np.arange(nz) + 0.5) * dz
    Z, P, L = np.meshgrid(zc, pc, lc, indexing="ij")
    ev = lambda fn, dflt: (np.broadcast_to(fn(L, P, Z), (nz, ny, nx)).astype(np.float64).copy()
                           if fn is not None else np.full((nz, ny, nx), dflt))
    f = 2.0 * EARTH_OMEGA * np.sin(pc) if rotating else np.zeros(ny)
    return Workload(name, SPHERICAL, nx, ny, nz, dlam, dphi, dz, 0.0, -0.5 * np.pi, EARTH_RADIUS,
                    ev(U, 0.0), np.zeros((nz, ny, nx)), ev(N2, 1.0e-4), f, _density(zc),
                    {f_: np.zeros(0) for f_ in RAY_FIELDS} | {"id": np.zeros(0, np.int64)},
                    dt=60.0, steps=1)


def density_gamma2(w: Workload) -> np.ndarray:
    """Scale-height correction Gamma^2 = 1 / (4 H_rho^2) of the reference
    density, H_rho = -rho / (d rho / dz) by centred differences of the level
    densities (one-sided at the ends), as a [nz][ny][nx] field: the usual
    anelastic value (the paper names the density scale height but gives no
    formula for Gamma)."""
    rho = np.asarray(w.rho, dtype=np.float64)
    drho = np.gradient(rho, w.dz) if w.nz > 1 else np.zeros(1)
    g2 = (0.5 * drho / rho) ** 2
    return np.ascontiguousarray(np.broadcast_to(g2[:, None, None], (w.nz, w.ny, w.nx)), dtype=np.float64)


def varying_gamma2(w: Workload, amp: float) -> np.ndarray:
    """A smooth, everywhere positive Gamma^2 field of size amp that varies in
    all three directions (periodic in x, and in y on the box), for tests that
    must see every Gamma term."""
    xc = (np.arange(w.nx) + 0.5) / w.nx
    yc = (np.arange(w.ny) + 0.5) / w.ny
    zc = (np.arange(w.nz) + 0.5) / w.nz
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    return np.ascontiguousarray(amp * (1.0 + 0.5 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)) * np.exp(-Z),
                                dtype=np.float64)


def rays_from(x, y, z, k, l, m, dx, dy, dz, px, py, pz, n) -> Dict[str, np.ndarray]:
    """Pack explicit arrays (broadcast to a common length) as a ray set."""
    arrs = np.broadcast_arrays(*[np.asarray(v, dtype=np.float64) for v in (x, y, z, k, l, m, dx, dy, dz, px, py, pz, n)])
    r = {f: np.ascontiguousarray(a) for f, a in zip(RAY_FIELDS, arrs)}
    r["id"] = np.arange(arrs[0].shape[0] if arrs[0].ndim else 1, dtype=np.int64)
    if arrs[0].ndim == 0:
        r = {f: v.reshape(1) for f, v in r.items()}
    return r


def subset_rays(rays: Dict[str, np.ndarray], n: int, seed: int = 0) -> Dict[str, np.ndarray]:
    """A deterministic sample of n rays, kept in ascending id order."""
    tot = rays["x"].shape[0]
    if n >= tot:
        return {k: v.copy() for k, v in rays.items()}
    pick = np.sort(_rng(seed).choice(tot, size=n, replace=False))
    return {k: v[pick].copy() for k, v in rays.items()}
