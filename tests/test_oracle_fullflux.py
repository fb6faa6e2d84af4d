"""Pins for the oracle's full flux formulation, smoothing and wave-action
budget (Section 2b, eq. fluxes:momentum, eq. fluxes:temperature, eq.
fluxes:buoyancy, eq. mean-flow-impact; Appendix B, horizontal flux
smoothing; Section 4, eq. wave-action-budget).

The independent reference for the fluxes is the plane-wave solution of the
linear rotating Boussinesq equations (the polarization relations), solved
numerically here: its phase-averaged Reynolds stresses rho <u_i u_j> and
buoyancy fluxes <u_i b>, for a wave of action A = E / omega_hat, must equal
the oracle's projected fluxes of a volume carrying that action.  CPU only."""
import math

import numpy as np
import pytest

from paper_2309_11257_amd import workloads as W

GRAV = 9.80665


def plane_wave(N2, f, k, l, m, rho):
    """Amplitudes (u, v, w, b) of the linear rotating Boussinesq plane wave
    exp(i(kx + ly + mz - omega t)) on the positive frequency branch, its
    phase-averaged energy density and frequency."""
    om = math.sqrt((N2 * (k * k + l * l) + f * f * m * m) / (k * k + l * l + m * m))
    I = 1j
    # x-momentum, y-momentum, z-momentum, buoyancy, continuity; unknowns u v w b p
    M = np.array([[-I * om, -f, 0, 0, I * k],
                  [f, -I * om, 0, 0, I * l],
                  [0, 0, -I * om, -1, I * m],
                  [0, 0, N2, -I * om, 0],
                  [I * k, I * l, I * m, 0, 0]])
    _, S, Vh = np.linalg.svd(M)
    assert S[-1] < 1e-12 * S[0]  # the dispersion relation makes M singular
    u, v, w, b, _ = Vh[-1].conj()
    E = rho / 4 * (abs(u) ** 2 + abs(v) ** 2 + abs(w) ** 2 + abs(b) ** 2 / N2)
    return (u, v, w, b), E, om


def _avg(a, c):
    return 0.5 * float(np.real(a * np.conj(c)))


@pytest.mark.parametrize("f0", [1.2e-4, -0.9e-4, 0.0])
def test_full_fluxes_equal_polarization_stresses(orc, f0):
    """A volume spanning levels kc and kc+1 exactly (so that both cell means
    and the interface between them see the same density of action) in a
    uniform resting atmosphere: every component of the oracle's full flux
    equals rho <u_i u_j> or <u_i b> of the plane wave with that action."""
    N2 = 3e-4
    w = W.analytic_box(nx=4, ny=4, nz=10, dx=20e3, dy=20e3, dz=1e3, N2=lambda X, Y, Z: 0 * X + N2, f0=f0)
    bg = orc.Background.from_workload(w)
    rng = np.random.default_rng(31 + int(f0 * 1e5))
    kc = 4
    for _ in range(6):
        kh = 2 * np.pi / rng.uniform(50e3, 300e3)
        th = rng.uniform(0, 2 * np.pi)
        k, l = kh * math.cos(th), kh * math.sin(th)
        m = -2 * np.pi / rng.uniform(2e3, 10e3)
        if f0 != 0.0 and math.sqrt((N2 * kh * kh + f0 * f0 * m * m) / (kh * kh + m * m)) < 1.3 * abs(f0):
            continue
        rho = w.rho[kc]
        (u, v, wz, b), E, om = plane_wave(N2, f0, k, l, m, rho)
        A = E / om
        i, j = 1, 2
        vol2 = 2 * w.dx * w.dy * w.dz
        rays = W.rays_from((i + 0.5) * w.dx, (j + 0.5) * w.dy, (kc + 1) * w.dz, k, l, m, w.dx, w.dy, 2 * w.dz,
                           1.0, 1.0, 1.0, A * vol2)
        F = orc.full_fluxes(bg, orc.RaySet(rays))
        expect = {0: rho * _avg(u, u), 1: rho * _avg(u, v), 2: rho * _avg(v, u), 3: rho * _avg(v, v)}
        for q, val in expect.items():
            for lev in (kc, kc + 1):
                assert F[q, lev, j, i] == pytest.approx(val, rel=1e-9, abs=1e-12 * abs(E)), (q, lev)
        # buoyancy flux: rho varies between the two levels, <u b> carries 1/rho
        for lev in (kc, kc + 1):
            (u2, v2, w2, b2), E2, _ = plane_wave(N2, f0, k, l, m, w.rho[lev])
            s = math.sqrt(A * om / E2)  # the same action at this level's density
            scale = s * s * abs(b2) * math.sqrt(abs(u2) ** 2 + abs(v2) ** 2)  # the flux's natural size
            assert F[4, lev, j, i] == pytest.approx(s * s * _avg(u2, b2), rel=1e-9, abs=1e-12 * scale), lev
            assert F[5, lev, j, i] == pytest.approx(s * s * _avg(v2, b2), rel=1e-9, abs=1e-12 * scale), lev
        # vertical fluxes on the interface kc + 1 (its staggered cell lies inside the volume)
        assert F[6, kc + 1, j, i] == pytest.approx(rho * _avg(wz, u), rel=1e-9, abs=0)
        assert F[7, kc + 1, j, i] == pytest.approx(rho * _avg(wz, v), rel=1e-9, abs=0)
        if f0 == 0.0:
            assert not F[4:6].any()


def test_full_reduces_to_pseudo_momentum_without_rotation(orc):
    """With f = 0 the full momentum flux is the pseudo-momentum flux and the
    buoyancy flux vanishes (Appendix A)."""
    w = W.make_c1(n_rays=512)
    w.f[:] = 0.0
    bg = orc.Background.from_workload(w)
    rs = orc.RaySet(w.rays)
    orc.step(bg, rs, w.dt)
    F = orc.full_fluxes(bg, rs)
    Fp = orc.deposit(bg, rs)
    idx = [0, 1, 2, 3, 6, 7]
    for q_full, q_pseudo in zip(idx, range(6)):
        sc = np.abs(Fp[q_pseudo]).max()
        assert np.abs(F[q_full] - Fp[q_pseudo]).max() <= 1e-13 * sc, q_full
    assert not F[4:6].any()


def test_smoothing_weights(orc):
    """3/2/1 weights (centre, edge neighbours, corner neighbours): a unit
    spike spreads as 3/15, 2/15, 1/15; constants are kept; on the periodic
    box the total is kept; on the sphere the first row's spike keeps 3/11
    (the missing row's weights are left out)."""
    box = W.analytic_box(nx=6, ny=5, nz=2)
    bg = orc.Background.from_workload(box)
    F = np.zeros((3, 5, 6))
    F[0, 2, 3] = 1.0
    F[1] = 7.25
    F[2] = np.random.default_rng(3).normal(size=(5, 6))
    S = orc.smooth(bg, F)
    exp = np.zeros((5, 6))
    exp[1:4, 2:5] = np.array([[1, 2, 1], [2, 3, 2], [1, 2, 1]]) / 15.0
    assert np.allclose(S[0], exp, rtol=1e-15, atol=1e-17)
    assert np.allclose(S[1], 7.25, rtol=1e-15)
    assert S[2].sum() == pytest.approx(F[2].sum(), rel=1e-13, abs=0)
    sph = W.analytic_sphere(nx=8, ny=6, nz=2)
    bgs = orc.Background.from_workload(sph)
    G = np.zeros((1, 6, 8))
    G[0, 0, 0] = 1.0
    Sg = orc.smooth(bgs, G)
    assert Sg[0, 0, 0] == pytest.approx(3.0 / 11.0, rel=1e-15, abs=0)
    assert Sg[0, 0, 1] == pytest.approx(2.0 / 11.0, rel=1e-15, abs=0)
    assert Sg[0, 1, 0] == pytest.approx(2.0 / 15.0, rel=1e-15, abs=0)  # row 1 has all its neighbours
    assert Sg[0, 1, 7] == pytest.approx(1.0 / 15.0, rel=1e-15, abs=0)  # periodic corner


def test_tendencies_closed_forms(orc):
    """Elastic term (f/g) e_r x <u'b'> for uniform buoyancy fluxes, the
    buoyancy tendency -div_h <u'b'> for a sinusoidal one, and the momentum
    part equal to the pseudo-momentum drag operator."""
    w = W.analytic_box(nx=16, ny=8, nz=4, dx=10e3, dy=20e3, dz=1e3, f0=1.1e-4)
    w.f = np.linspace(-1e-4, 1.2e-4, w.ny)
    bg = orc.Background.from_workload(w)
    nz, ny, nx = w.nz, w.ny, w.nx
    F = np.zeros((8, nz + 1, ny, nx))
    F[4, :nz] = 0.3
    F[5, :nz] = -0.7
    T = orc.full_tendencies(bg, F)
    fj = w.f[None, :, None]
    assert np.allclose(T[0], -(fj / GRAV) * -0.7, rtol=1e-15, atol=0)
    assert np.allclose(T[1], (fj / GRAV) * 0.3, rtol=1e-15, atol=0)
    assert not T[2].any()
    i = np.arange(nx)
    F[4, :nz] = np.sin(2 * np.pi * i / nx)[None, None, :]
    F[5] = 0.0
    T = orc.full_tendencies(bg, F)
    exp = -(np.cos(2 * np.pi * i / nx) * np.sin(2 * np.pi / nx) / w.dx)[None, None, :]
    assert np.allclose(T[2], np.broadcast_to(exp, T[2].shape), rtol=1e-12, atol=1e-20)
    # momentum part against the pseudo-momentum operator on random fluxes
    rng = np.random.default_rng(4)
    F = rng.normal(size=F.shape)
    F[4:6] = 0.0
    T = orc.full_tendencies(bg, F)
    D = orc.drag(bg, F[[0, 1, 2, 3, 6, 7]])
    assert np.array_equal(T[:2], D)


def brute_budget(orc, w, rays):
    nx, ny, nz, dz = w.nx, w.ny, w.nz, w.dz
    out = np.zeros((4, nz + 1, ny, nx))
    bg = orc.Background.from_workload(w)
    for r in range(rays["x"].shape[0]):
        x, y, z = rays["x"][r], rays["y"][r], rays["z"][r]
        i = min(int(np.floor((x - w.x0) / w.dx)), nx - 1)
        j = min(int(np.floor((y - w.y0) / w.dy)), ny - 1)
        B = bg.interp(x, y, z)
        _, cx, cy, cz = orc.dispersion(B[2], B[12], rays["k"][r], rays["l"][r], rays["m"][r])
        Wr = rays["n"][r] * rays["px"][r] * rays["py"][r] * rays["pz"][r]
        zb, zt = z - rays["dz"][r] / 2, z + rays["dz"][r] / 2
        for kk in range(nz):
            o = max(0.0, min(zt, (kk + 1) * dz) - max(zb, kk * dz))
            vol = w.dx * w.dy * dz
            s = Wr * o / rays["dz"][r] / vol
            out[0, kk, j, i] += s
            out[1, kk, j, i] += (B[0] + cx) * s
            out[2, kk, j, i] += (B[1] + cy) * s
        for kk in range(nz + 1):
            lo, hi = max(0.0, (kk - 0.5) * dz), min(nz * dz, (kk + 0.5) * dz)
            o = max(0.0, min(zt, hi) - max(zb, lo))
            out[3, kk, j, i] += cz * Wr * o / rays["dz"][r] / (w.dx * w.dy * (hi - lo))
    return out


def test_budget_fields_brute_force_and_totals(orc):
    """The budget fields against a per-volume, per-level evaluation of their
    definition; the total action equals the sum of the volumes' W (for
    volumes inside the domain); identical columns give no horizontal term."""
    rng = np.random.default_rng(41)
    w = W.analytic_box(nx=3, ny=3, nz=8, dx=10e3, dy=10e3, dz=1e3,
                       U=lambda X, Y, Z: 5 + 1e-3 * Z, V=lambda X, Y, Z: -2 + 0 * X,
                       N2=lambda X, Y, Z: 1e-4 + 1e-9 * Z, f0=1e-4)
    n = 60
    kh = 2 * np.pi / rng.uniform(20e3, 100e3, n)
    th = rng.uniform(0, 2 * np.pi, n)
    Dz = rng.uniform(200, 2500, n)
    z = rng.uniform(0.5 * Dz, 8e3 - 0.5 * Dz)
    rays = W.rays_from(rng.uniform(0, 30e3, n), rng.uniform(0, 30e3, n), z, kh * np.cos(th), kh * np.sin(th),
                       -2 * np.pi / rng.uniform(1e3, 5e3, n), 10e3, 10e3, Dz, 2.0, 3.0, 0.5, rng.uniform(0.1, 1, n))
    bg = orc.Background.from_workload(w)
    Fb = orc.budget(bg, orc.RaySet(rays))
    ref = brute_budget(orc, w, rays)
    for q in range(4):
        assert np.abs(Fb[q] - ref[q]).max() <= 1e-13 * np.abs(ref[q]).max(), q
    tot = (Fb[0, :w.nz] * w.dx * w.dy * w.dz).sum()
    assert tot == pytest.approx((rays["n"] * rays["px"] * rays["py"] * rays["pz"]).sum(), rel=1e-13, abs=0)
    # identical columns: no horizontal propagation term
    wi = W.make_c1(n_rays=256)
    g = np.arange(256)
    wi.rays["x"][:] = (g % 16 + 0.4) * wi.dx
    wi.rays["y"][:] = (g // 16 + 0.6) * wi.dy
    for fld in ("k", "l", "m", "dz", "px", "py", "pz", "n"):
        wi.rays[fld][:] = wi.rays[fld][0]
    bgi = orc.Background.from_workload(wi)
    Ti = orc.budget_terms(bgi, orc.budget(bgi, orc.RaySet(wi.rays)))
    assert not Ti[0].any()
    assert Ti[1].any()
