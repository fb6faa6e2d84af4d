"""Pins for the oracle's continuous launch from a ghost layer (Section 3c,
sources: the latitudinal background-source profile, its seasonal cycle,
the launch at every step of the part of the layer that crossed the launch
height, and the discarding of the volumes that cannot propagate).  CPU
only."""
import math
import os

import numpy as np
import pytest

from paper_2309_11257_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
YEAR = 365.25 * 86400.0


def _row_sphere(orc, phi_deg):
    """A one-row spherical grid whose row centre is at phi_deg."""
    dy = math.radians(0.5)
    y0 = math.radians(phi_deg) - 0.5 * dy
    nx, ny, nz = 2, 1, 2
    z = (np.arange(nz) + 0.5) * 1e3
    return orc.Background(W.SPHERICAL, nx, ny, nz, math.pi, dy, 1e3, 0.0, y0, W.EARTH_RADIUS,
                          np.zeros((nz, ny, nx)), np.zeros((nz, ny, nx)), np.full((nz, ny, nx), 1e-4),
                          np.zeros(ny), 1.2 * np.exp(-z / 7e3))


def test_source_profile_and_season_golden(orc):
    """The column launch flux at the northern summer solstice is the
    tabulated F_sol(phi) (8 and 2.4 mPa, Section 3c); half a year later the
    hemispheres swap; a quarter of a year later each latitude gets the mean
    of the two."""
    rows = [list(map(float, ln.split())) for ln in open(os.path.join(GOLDEN, "background_source.txt"))
            if ln.strip() and not ln.startswith("#")]
    table = {phi: fs for phi, _, fs in rows}
    for phi, _, fs in rows:
        bg = _row_sphere(orc, phi)
        p0 = orc.launch_params(9e3, 60.0, t_solstice=0.0)
        p1 = orc.launch_params(9e3, 60.0, t_solstice=0.5 * YEAR)
        p2 = orc.launch_params(9e3, 60.0, t_solstice=0.25 * YEAR)
        assert orc.launch_flux(bg, 0, p0) == pytest.approx(fs, abs=1e-15), phi
        if -phi in table:
            assert orc.launch_flux(bg, 0, p1) == pytest.approx(table[-phi], abs=1e-15), phi
            assert orc.launch_flux(bg, 0, p2) == pytest.approx(0.5 * (fs + table[-phi]), abs=1e-15), phi


def _box(N2=4e-4, f0=1e-4):
    return W.analytic_box(nx=5, ny=4, nz=20, dx=25e3, dy=25e3, dz=1e3, N2=lambda X, Y, Z: 0 * X + N2, f0=f0,
                          U=lambda X, Y, Z: 3.0 + 1e-4 * X)


def _omega(N2, f2, k, l, m):
    return math.sqrt((N2 * (k * k + l * l) + f2 * m * m) / (k * k + l * l + m * m))


def test_launch_carries_the_column_flux(orc):
    """Every propagating bin: omega_hat(k, l, m) = kh c_b, upward (m < 0),
    the volume spans [z_launch, z_launch + cg_z dt] with cg_z the vertical
    group velocity (finite differences of the frequency), and the launched
    pseudo-momentum kh W of a column sums to F_col A dt (all bins
    propagate here); the four directions cancel in sum k W and sum l W;
    ids are consecutive in order of column, direction and phase speed."""
    N2, f0 = 4e-4, 1e-4
    w = _box(N2, f0)
    bg = orc.Background.from_workload(w)
    rng = np.random.default_rng(51)
    flux = rng.uniform(0.5e-3, 3e-3, w.nx * w.ny)
    flux[3] = 0.0  # a column without a source launches nothing
    zl, dt, lam = 9.3e3, 45.0, 200e3
    p = orc.launch_params(zl, dt, lambda_h=lam, c_min=4.0, c_max=44.0, c_center=20.0, c_width=12.0, n_speeds=8,
                          flux_col=flux)
    rs = orc.RaySet({f: np.zeros(0) for f in orc.RAY_FIELDS} | {"id": np.zeros(0, np.int64)},
                    capacity=4 * 8 * w.nx * w.ny)
    t = orc.launch(bg, rs, p, next_id=100)
    n = rs.n
    assert n == 4 * 8 * (w.nx * w.ny - 1) and t["n_launched"] == n
    assert np.array_equal(rs["id"], 100 + np.arange(n))
    kh = 2 * math.pi / lam
    A = w.dx * w.dy
    cols = (np.floor(rs["y"] / w.dy) * w.nx + np.floor(rs["x"] / w.dx)).astype(int)
    assert np.all(np.diff(cols) >= 0) and 3 not in cols
    Wv = rs["n"] * rs["px"] * rs["py"] * rs["pz"]
    assert t["launched_W"] == pytest.approx(Wv.sum(), rel=1e-12, abs=0)
    for c in np.unique(cols):
        sel = cols == c
        assert (kh * Wv[sel]).sum() == pytest.approx(flux[c] * A * dt, rel=1e-12, abs=0)
        assert abs((rs["k"][sel] * Wv[sel]).sum()) <= 1e-12 * kh * Wv[sel].sum()
        assert abs((rs["l"][sel] * Wv[sel]).sum()) <= 1e-12 * kh * Wv[sel].sum()
    cb = 4.0 + (np.arange(8) + 0.5) * 5.0
    for q in range(n):
        k, l, m = rs["k"][q], rs["l"][q], rs["m"][q]
        b = q % 8
        assert m < 0
        assert math.hypot(k, l) == pytest.approx(kh, rel=1e-15, abs=0)
        assert _omega(N2, f0 * f0, k, l, m) == pytest.approx(kh * cb[b], rel=1e-13, abs=0)
        h = 1e-6 * abs(m)
        cgz = (_omega(N2, f0 * f0, k, l, m + h) - _omega(N2, f0 * f0, k, l, m - h)) / (2 * h)
        assert rs["dz"][q] / dt == pytest.approx(cgz, rel=1e-7, abs=0)
        assert rs["z"][q] - 0.5 * rs["dz"][q] == pytest.approx(zl, rel=1e-15, abs=0)
    # directions east, north, west, south in turn for each column
    first = np.arange(0, n, 8)
    d = np.arange(first.size) % 4
    assert np.allclose(rs["k"][first], kh * np.array([1, 0, -1, 0])[d], rtol=0, atol=1e-20)
    assert np.allclose(rs["l"][first], kh * np.array([0, 1, 0, -1])[d], rtol=0, atol=1e-20)


def test_launch_discards_bins_that_cannot_propagate(orc):
    """Phase speeds whose intrinsic frequency lies outside (f, N) are
    reflected in the ghost layer and discarded with their share of the flux;
    capacity shortfall changes nothing."""
    N2, f0 = 1e-4, 1e-4
    w = _box(N2, f0)
    bg = orc.Background.from_workload(w)
    flux = np.full(w.nx * w.ny, 2e-3)
    kinds = set()
    # a long wavelength puts the slow bins below f (inertial), a short one
    # puts the fast bins above N
    for lam, cmin, cmax in ((1000e3, 1.0, 100.0), (100e3, 0.5, 200.0)):
        kh = 2 * math.pi / lam
        nb = 16
        cb = cmin + (np.arange(nb) + 0.5) * (cmax - cmin) / nb
        om = kh * cb
        prop = (om > f0) & (om < math.sqrt(N2))
        assert 0 < prop.sum() < nb
        kinds |= {"inertial"} if (om <= f0).any() else set()
        kinds |= {"fast"} if (om >= math.sqrt(N2)).any() else set()
        wts = np.exp(-(((cb - 50.0) / 40.0) ** 2))
        p = orc.launch_params(8e3, 30.0, lambda_h=lam, c_min=cmin, c_max=cmax, c_center=50.0, c_width=40.0,
                              n_speeds=nb, flux_col=flux)
        rs = orc.RaySet({f: np.zeros(0) for f in orc.RAY_FIELDS} | {"id": np.zeros(0, np.int64)}, capacity=10000)
        orc.launch(bg, rs, p, next_id=0)
        assert rs.n == 4 * int(prop.sum()) * w.nx * w.ny
        assert np.isfinite(rs["m"]).all()
        Wv = rs["n"] * rs["px"] * rs["py"] * rs["pz"]
        tot = (kh * Wv).sum()
        assert tot == pytest.approx(flux.sum() * w.dx * w.dy * 30.0 * wts[prop].sum() / wts.sum(), rel=1e-12, abs=0)
    assert kinds == {"inertial", "fast"}
    small = orc.RaySet({f: np.zeros(0) for f in orc.RAY_FIELDS} | {"id": np.zeros(0, np.int64)}, capacity=rs.n - 1)
    with pytest.raises(RuntimeError):
        orc.launch(bg, small, p, next_id=0)
    assert small.n == 0


def test_launch_on_the_sphere(orc):
    """On the global grid at the solstice: no volumes below 20 degrees or
    above 85 degrees, the launched pseudo-momentum per column equals
    F_sol(phi) times the cell area at the launch height times dt, and the
    phase-space areas use the metric extents at the new volume's height."""
    w = W.make_c3(n_rays=1000, nx=72, ny=36, nz=30)
    bg = orc.Background.from_workload(w)
    p = orc.launch_params(9e3, 20.0, t_solstice=0.0, lambda_h=500e3, c_min=5.0, c_max=45.0, n_speeds=4)
    rs = orc.RaySet({f: np.zeros(0) for f in orc.RAY_FIELDS} | {"id": np.zeros(0, np.int64)}, capacity=100000)
    orc.launch(bg, rs, p, next_id=0)
    phi = np.degrees(rs["y"])
    assert rs.n > 0 and np.abs(phi).min() > 20.0 and np.abs(phi).max() < 85.0
    kh = 2 * math.pi / 500e3
    Wv = rs["n"] * rs["px"] * rs["py"] * rs["pz"]
    rows = np.floor((rs["y"] + 0.5 * math.pi) / w.dy).astype(int)
    cb = 5.0 + (np.arange(4) + 0.5) * 10.0
    wts = np.exp(-(((cb - 25.0) / 15.0) ** 2))
    for j in np.unique(rows):
        sel = (rows == j) & (np.floor(rs["x"] / w.dx).astype(int) == 7)
        phij = -0.5 * math.pi + (j + 0.5) * w.dy
        A = (w.a + 9e3) ** 2 * math.cos(phij) * w.dx * w.dy
        fsol = orc.launch_flux(bg, j, p)
        B = bg.interp(7.5 * w.dx, phij, 9e3)
        om2 = (kh * cb) ** 2
        prop = (om2 > B[12]) & (om2 < B[2])  # slower bins are inertial near the poles
        assert (kh * Wv[sel]).sum() == pytest.approx(fsol * A * 20.0 * wts[prop].sum() / wts.sum(), rel=1e-12, abs=0)
    q = 0
    r = w.a + rs["z"][q]
    assert rs["px"][q] == pytest.approx(r * math.cos(rs["y"][q]) * w.dx * 0.1 * kh, rel=1e-14, abs=0)
    assert rs["py"][q] == pytest.approx(r * w.dy * 0.1 * kh, rel=1e-14, abs=0)
