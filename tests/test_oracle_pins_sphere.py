"""Pins for the spherical branches of the FP64 oracle: the drag's divergence
on the sphere against closed forms, removal within 0.5 degree of a pole
against the oracle's own great-circle trajectory, and the rotating sphere's
meridional refraction (the (f^2)_phi term of eq. eikonal-sphere 2) against
minus the latitude derivative of the frequency by finite differences.  CPU
only."""
import math

import numpy as np
import pytest

from paper_2309_11257_amd import workloads as W

OMEGA = W.EARTH_OMEGA


# --------------------------------------------------------------------------
# drag on the sphere (eq. mean-flow-impact, divergence in spherical
# coordinates with metric factors in the derivatives)
# --------------------------------------------------------------------------
def test_spherical_drag_closed_form(orc):
    """F_x = sin(lambda), F_y = tan(phi), F_z = s (a + z_kk)^2 have centred
    differences in closed form:
      d_lambda sin at lambda_i over 2 dlambda = cos(lambda_i) sin(dlambda)/dlambda,
      d_phi (cos(phi) tan(phi)) = d_phi sin(phi): centred gives
      cos(phi_j) sin(dphi)/dphi, one-sided at the end rows gives
      (sin(phi_1) - sin(phi_0))/dphi,
      interface difference of (a + z)^2 over dz = 2 r_k with r_k = a + z_k.
    The drag is -(1/rho) of [divx/(r cos phi) + divy/(r cos phi) + divz]."""
    w = W.analytic_sphere(nx=24, ny=18, nz=6, top=30e3, rotating=False)
    bg = orc.Background.from_workload(w)
    nx, ny, nz = w.nx, w.ny, w.nz
    lam = (np.arange(nx) + 0.5) * w.dx
    phi = w.y0 + (np.arange(ny) + 0.5) * w.dy
    zc = (np.arange(nz) + 0.5) * w.dz
    zi = np.arange(nz + 1) * w.dz
    r = w.a + zc
    s = 1e-14
    flux = np.zeros((6, nz + 1, ny, nx))
    flux[0, :nz] = np.sin(lam)[None, None, :]
    flux[4] = (s * (w.a + zi) ** 2)[:, None, None]
    flux[3, :nz] = np.tan(phi)[None, :, None]
    drag = orc.drag(bg, flux)
    rho = w.rho[:, None, None]
    # du: zonal difference of F_x plus the vertical difference of F_zk
    divx = (np.cos(lam) * math.sin(w.dx) / w.dx)[None, None, :] / (r[:, None, None] * np.cos(phi)[None, :, None])
    divz = (2.0 * s * r)[:, None, None]
    exp_u = -(divx + divz) / rho
    # the two terms may nearly cancel: compare against the size of the terms
    scale = (np.abs(divx) + np.abs(divz)) / rho
    assert (np.abs(drag[0] - exp_u) <= 1e-11 * scale).all()
    # dv: meridional difference of cos(phi) F_yl
    dphi = np.empty(ny)
    dphi[1:-1] = np.cos(phi[1:-1]) * math.sin(w.dy) / w.dy
    dphi[0] = (math.sin(phi[1]) - math.sin(phi[0])) / w.dy
    dphi[-1] = (math.sin(phi[-1]) - math.sin(phi[-2])) / w.dy
    exp_v = -(dphi[None, :, None] / (r[:, None, None] * np.cos(phi)[None, :, None])) / rho
    exp_v = np.broadcast_to(exp_v, drag[1].shape)
    assert np.allclose(drag[1], exp_v, rtol=1e-10, atol=0)
    # the interior rows reduce to sin(dphi)/(dphi r): independent of latitude
    inner = drag[1][:, 1:-1, :] * rho
    assert np.allclose(inner, -(math.sin(w.dy) / w.dy) / r[:, None, None], rtol=1e-10, atol=0)


# --------------------------------------------------------------------------
# pole removal (Section 2a: the pole is a coordinate singularity; rays are
# removed within 0.5 degree of it)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("hemisphere", [1.0, -1.0])
def test_pole_removal_step_and_tally(orc, hemisphere):
    """A ray on a meridian (k = 0) in a uniform atmosphere at rest moves
    poleward by about 0.026 degree per 300 s step.  It must stay active on
    every step that ends below 89.5 degrees and be removed on the first
    step that ends at or beyond it; its wave action goes to the removal
    tally once, and the pole count is one."""
    w = W.analytic_sphere(nx=36, ny=180, nz=20, top=40e3, N2=lambda L, P, Z: 0 * L + 4e-4, rotating=False)
    bg = orc.Background.from_workload(w)
    lim = math.radians(89.5)
    l = hemisphere * 2 * np.pi / 100e3
    rays = W.rays_from(1.0, hemisphere * math.radians(89.0), 10e3, 0.0, l, -2 * np.pi / 3e3,
                       1e-4, 1e-4, 100.0, 2.0, 3.0, 5.0, 0.7)
    rs = orc.RaySet(rays)
    Wray = 0.7 * 2.0 * 3.0 * 5.0
    removed_at = None
    ys = []
    for s in range(200):
        t = orc.step(bg, rs, 300.0)
        y = float(rs["y"][0])
        ys.append(y)
        if rs.active()[0]:
            assert abs(y) < lim, (s, math.degrees(y))
            assert t["n_pole"] == 0 and t["removed_W"] == 0.0
        else:
            assert rs["state"][0] == orc.GONE_POLE
            assert abs(y) >= lim, (s, math.degrees(y))
            assert t["n_pole"] == 1
            assert t["removed_W"] == Wray
            removed_at = s
            break
    assert removed_at is not None and removed_at >= 5
    # the ray moved steadily poleward: the last active step ended within
    # one step's advance of the limit, so a threshold a few hundredths of a
    # degree lower or higher would change the step of removal
    adv = abs(ys[-1] - ys[-2])
    assert 0.0 < adv < math.radians(0.05)
    assert lim - abs(ys[-2]) < adv
    # a removed ray stays removed
    t = orc.step(bg, rs, 300.0)
    assert t["n_pole"] == 0 and not rs.active()[0]


# --------------------------------------------------------------------------
# meridional refraction on a rotating sphere (eq. eikonal-sphere 2 with
# Gamma = 0: the (f^2)_phi term)
# --------------------------------------------------------------------------
def _omega_hat(N2, f2, k, l, m):
    kh2 = k * k + l * l
    return math.sqrt((N2 * kh2 + f2 * m * m) / (kh2 + m * m))


def test_sphere_rotating_refraction_matches_latitude_gradient(orc):
    """At rest with uniform N^2 and f = 2 Omega sin(phi), the frequency
    depends on position only through f^2(phi).  For a volume of negligible
    extent the carrier moves with the local group velocity, so the
    wavevector tendencies must be
      kdot_phi = -(1/r) d_phi Omega - k_phi w/r - k_lambda tan(phi) u/r,
      kdot_lambda = -k_lambda w/r + k_lambda tan(phi) v/r,
      kdot_r = k_lambda u/r + k_phi v/r,
    with d_phi Omega by central differences of the analytic frequency and
    (u, v, w) the wavenumber gradient of the frequency by central
    differences.  The grid is fine (0.1 degree rows) so that the row
    interpolation of f^2 and (f^2)_phi is exact to about 1e-6."""
    w = W.analytic_sphere(nx=8, ny=1800, nz=16, top=32e3, N2=lambda L, P, Z: 0 * L + 2e-4, rotating=True)
    bg = orc.Background.from_workload(w)
    N2 = 2e-4
    f2_of = lambda p: (2.0 * OMEGA * math.sin(p)) ** 2
    rng = np.random.default_rng(11)
    seen_f2_term = 0.0
    for _ in range(24):
        lam = rng.uniform(0, 2 * np.pi)
        phi = math.radians(rng.uniform(-70, 70))
        z = rng.uniform(5e3, 25e3)
        kh = 2 * np.pi / rng.uniform(300e3, 3000e3)
        th = rng.uniform(0, 2 * np.pi)
        k, l = kh * math.cos(th), kh * math.sin(th)
        m = -2 * np.pi / rng.uniform(2e3, 20e3)
        f2 = f2_of(phi)
        if _omega_hat(N2, f2, k, l, m) < 1.2 * math.sqrt(f2):
            continue
        r = w.a + z
        F = bg.rhs([lam, phi, z, k, l, m, 1e-9, 1e-9, 1e-3])
        # d_phi Omega, and the group velocity, by central differences
        hp = 1e-6
        dOm = (_omega_hat(N2, f2_of(phi + hp), k, l, m) - _omega_hat(N2, f2_of(phi - hp), k, l, m)) / (2 * hp)
        hk = 1e-6 * kh
        u = (_omega_hat(N2, f2, k + hk, l, m) - _omega_hat(N2, f2, k - hk, l, m)) / (2 * hk)
        v = (_omega_hat(N2, f2, k, l + hk, m) - _omega_hat(N2, f2, k, l - hk, m)) / (2 * hk)
        hm = 1e-6 * abs(m)
        wz = (_omega_hat(N2, f2, k, l, m + hm) - _omega_hat(N2, f2, k, l, m - hm)) / (2 * hm)
        tphi = math.tan(phi)
        exp_l = -dOm / r - l * wz / r - k * tphi * u / r
        exp_k = -k * wz / r + k * tphi * v / r
        exp_m = k * u / r + l * v / r
        scale_l = abs(dOm / r) + abs(l * wz / r) + abs(k * tphi * u / r)
        assert abs(F[4] - exp_l) <= 2e-5 * scale_l, (F[4], exp_l)
        assert abs(F[3] - exp_k) <= 2e-5 * (abs(k * wz / r) + abs(k * tphi * v / r))
        assert abs(F[5] - exp_m) <= 2e-5 * (abs(k * u / r) + abs(l * v / r))
        # carrier rates: angular velocities from the local group velocity
        assert F[0] == pytest.approx(u / (r * math.cos(phi)), rel=2e-5, abs=0)
        assert F[1] == pytest.approx(v / r, rel=2e-5, abs=0)
        assert F[2] == pytest.approx(wz, rel=2e-5, abs=0)
        seen_f2_term = max(seen_f2_term, abs(dOm / r) / scale_l)
    # the (f^2)_phi term carried a sizeable share of kdot_phi somewhere
    assert seen_f2_term > 0.2
