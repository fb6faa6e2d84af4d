"""The oracle's pins must catch the plausible slips they were written for.

Each case plants one mistake in a copy of the oracle's C source (a dropped
metric weight, a dropped or sign-flipped term, a moved threshold), builds it
on the CPU, runs the named pins against the planted build and requires at
least one of them to fail.  The real oracle is untouched and restored after
each case.  CPU only."""
import pytest

import test_oracle_fullflux as X
import test_oracle_gamma as G
import test_oracle_launch as L
import test_oracle_pins as P
import test_oracle_pins_sphere as S
import test_oracle_saturation as T

MUTATIONS = [
    ("launch flux split in two directions instead of four",
     "double Fb = (0.25 * Fc) * (exp(-(s * s)) / sw);",
     "double Fb = (0.5 * Fc) * (exp(-(s * s)) / sw);",
     [L.test_launch_carries_the_column_flux]),
    ("launch keeps bins made evanescent by Gamma",
     "if (!(m2 > 0.0)) continue; /* evanescent: Gamma^2 exceeds m^2 + Gamma^2 */",
     ";",
     [G.test_launch_with_gamma]),
    ("launch ignores Gamma",
     "m2 = ((kh * kh) * (N2 - om2)) / (om2 - f2) - G[0];",
     "m2 = ((kh * kh) * (N2 - om2)) / (om2 - f2);",
     [G.test_launch_with_gamma]),
    ("Gamma dropped from the dispersion relation",
     "double M2 = m * m + G2;",
     "double M2 = m * m;",
     [G.test_dispersion_is_the_gamma_free_relation_at_shifted_m]),
    ("K^2 without Gamma^2 in the dispersion relation",
     "double K2 = kh2 + M2;",
     "double K2 = kh2 + m * m;",
     [G.test_dispersion_is_the_gamma_free_relation_at_shifted_m]),
    ("refraction by Gamma^2 gradients with the wrong sign",
     "qg = -((kh2 * (B[2] - B[12])) / (((2.0 * om) * K2) * K2));",
     "qg = (kh2 * (B[2] - B[12])) / (((2.0 * om) * K2) * K2);",
     [lambda orc: G.test_refraction_by_gamma_gradients_conserves_frequency(orc, "gamma_xz")]),
    ("(f^2)_phi refraction weight without Gamma^2",
     "qf = M2 / ((2.0 * om) * K2);",
     "qf = (m * m) / ((2.0 * om) * K2);",
     [lambda orc: G.test_refraction_by_gamma_gradients_conserves_frequency(orc, "beta")]),
    ("faces evaluated without Gamma",
     "*G2 = g->G2 ? trilin(g, g->G2, &c) : 0.0;",
     "*G2 = 0.0;",
     [G.test_extent_rates_use_gamma_at_the_faces]),
    ("Gamma^2 gradient taken from N^2",
     "g->G2x[c] = ddx(g, g->G2, i, j, k);",
     "g->G2x[c] = ddx(g, g->N2, i, j, k);",
     [G.test_gamma_fields_interpolate_and_differentiate_exactly]),
    ("saturation damping with K^2 without Gamma^2",
     "K2 = (r->k[i] * r->k[i] + r->l[i] * r->l[i]) + (r->m[i] * r->m[i] + G[0]);",
     "K2 = (r->k[i] * r->k[i] + r->l[i] * r->l[i]) + r->m[i] * r->m[i];",
     [G.test_saturation_with_gamma_restores_the_threshold]),
    ("saturation K^2 without Gamma^2",
     "K2 = kh2 + (m2 + G2);",
     "K2 = kh2 + m2;",
     [G.test_saturation_and_deposit_are_gamma_free_at_shifted_m]),
    ("launched volume covers half the crossing",
     "Dz = D[3] * p->dt;",
     "Dz = D[3] * (0.5 * p->dt);",
     [L.test_launch_carries_the_column_flux]),
    ("seasonal cycle with the hemispheres swapped",
     "return 0.5 * (fsol_n * (1.0 + cos(tau)) + fsol_s * (1.0 - cos(tau)));",
     "return 0.5 * (fsol_n * (1.0 - cos(tau)) + fsol_s * (1.0 + cos(tau)));",
     [L.test_source_profile_and_season_golden]),
    ("source ramp between 20 and 50 degrees inverted",
     "if (phi_deg >= 20.0) return 0.5 * (1.0 - cos(ORC_PI * (phi_deg - 20.0) / 30.0));",
     "if (phi_deg >= 20.0) return 0.5 * (1.0 + cos(ORC_PI * (phi_deg - 20.0) / 30.0));",
     [L.test_source_profile_and_season_golden]),
    ("full flux: f^2 term of Fxu with the wrong sign",
     "v[0] = a1 * (D[1] * k) + a2 * (D[2] * l); /* Fxu */",
     "v[0] = a1 * (D[1] * k) - a2 * (D[2] * l); /* Fxu */",
     [lambda orc: X.test_full_fluxes_equal_polarization_stresses(orc, 1.2e-4)]),
    ("full flux: omega^2/(omega^2 - f^2) factor dropped from the vertical flux",
     "v[6] = a1 * (D[3] * k);                   /* Fzu */",
     "v[6] = D[3] * k;                          /* Fzu */",
     [lambda orc: X.test_full_fluxes_equal_polarization_stresses(orc, -0.9e-4)]),
    ("buoyancy flux without 1/rho",
     "for (q = 4; q < 6; q++) flux[(size_t)q * plane + at] += (((v[q] * W) * frac) / vol) / g->rho[kk];",
     "for (q = 4; q < 6; q++) flux[(size_t)q * plane + at] += ((v[q] * W) * frac) / vol;",
     [lambda orc: X.test_full_fluxes_equal_polarization_stresses(orc, 1.2e-4)]),
    ("buoyancy flux with |f| instead of the signed f",
     "fs = rowlin(g->f, &cc);",
     "fs = sqrt(f2);",
     [lambda orc: X.test_full_fluxes_equal_polarization_stresses(orc, -0.9e-4)]),
    ("elastic term with the wrong sign",
     "double el = comp == 0 ? -(fg * flux8[5 * plane + at]) : fg * flux8[4 * plane + at];",
     "double el = comp == 0 ? fg * flux8[5 * plane + at] : -(fg * flux8[4 * plane + at]);",
     [X.test_tendencies_closed_forms]),
    ("smoothing with equal weights",
     "double w = (di == 0 && dj == 0) ? 3.0 : ((di == 0 || dj == 0) ? 2.0 : 1.0);",
     "double w = 1.0;",
     [X.test_smoothing_weights]),
    ("budget flux without the mean wind",
     "v[1] = B[0] + D[1];",
     "v[1] = D[1];",
     [X.test_budget_fields_brute_force_and_totals]),
    ("saturation weight without kh^2",
     "return (m2 * kh2) / (D[0] * K2);",
     "return m2 / (D[0] * K2);",
     [lambda orc: T.test_monochromatic_limit(orc, 1.5)]),
    ("saturation threshold rho instead of rho/2",
     "double ex = P[at] - 0.5 * g->rho[kk];",
     "double ex = P[at] - g->rho[kk];",
     [lambda orc: T.test_monochromatic_limit(orc, 1.5)]),
    ("saturation factor 1 - kappa K^2 dt (factor 2 dropped)",
     "fac = 1.0 - ((2.0 * kbar) * K2) * dt;",
     "fac = 1.0 - (kbar * K2) * dt;",
     [T.test_threshold_restored_in_each_cell]),
    ("saturation factor not held at zero",
     "if (fac < 0.0) fac = 0.0;",
     ";",
     [T.test_density_never_negative_and_dt_independent]),
    ("saturation kappa not weighted by the overlap fraction",
     "kbar += (o / r->dz[i]) * kappa[IDX(g, ci, cj, kk)];",
     "kbar += kappa[IDX(g, ci, cj, kk)];",
     [lambda orc: T.test_saturation_matches_brute_force(orc, "box")]),
    ("spherical drag without the cos(phi) weight of the meridional flux",
     "dphi = (cp * Fy[IDX(g, i, j + 1, k)] - cm * Fy[IDX(g, i, j - 1, k)]) / (2.0 * g->dy);",
     "dphi = (Fy[IDX(g, i, j + 1, k)] - Fy[IDX(g, i, j - 1, k)]) / (2.0 * g->dy);",
     [S.test_spherical_drag_closed_form]),
    ("spherical drag with r = a instead of a + z",
     "double r = g->a + ((double)k + 0.5) * g->dz;\n                    double cj",
     "double r = g->a;\n                    double cj",
     [S.test_spherical_drag_closed_form]),
    ("spherical drag with the zonal term not divided by r cos(phi)",
     "divx = ((Fx[IDX(g, ip, j, k)] - Fx[IDX(g, im, j, k)]) / (2.0 * g->dx)) / rc;",
     "divx = ((Fx[IDX(g, ip, j, k)] - Fx[IDX(g, im, j, k)]) / (2.0 * g->dx)) / r;",
     [S.test_spherical_drag_closed_form]),
    ("meridional refraction without the (f^2)_phi term",
     "gl = ((k * B[4] + l * B[7]) + q * B[10]) + qf * B[13];",
     "gl = (k * B[4] + l * B[7]) + q * B[10];",
     [S.test_sphere_rotating_refraction_matches_latitude_gradient]),
    ("meridional refraction with the (f^2)_phi term's sign flipped",
     "gl = ((k * B[4] + l * B[7]) + q * B[10]) + qf * B[13];",
     "gl = ((k * B[4] + l * B[7]) + q * B[10]) - qf * B[13];",
     [S.test_sphere_rotating_refraction_matches_latitude_gradient]),
    ("meridional metric term k tan(phi) u / r with the wrong sign",
     "F[4] = ((-gl) / r - (l * wc) / r) - ((k * tphi) * uc) / r;",
     "F[4] = ((-gl) / r - (l * wc) / r) + ((k * tphi) * uc) / r;",
     [S.test_sphere_rotating_refraction_matches_latitude_gradient]),
    ("pole removal at 89.4 degrees",
     "if (fabs(Y[1]) >= 89.5 * (3.14159265358979323846 / 180.0)) return ORC_GONE_POLE;",
     "if (fabs(Y[1]) >= 89.4 * (3.14159265358979323846 / 180.0)) return ORC_GONE_POLE;",
     [lambda orc: S.test_pole_removal_step_and_tally(orc, 1.0)]),
    ("pole removal at 89.6 degrees",
     "if (fabs(Y[1]) >= 89.5 * (3.14159265358979323846 / 180.0)) return ORC_GONE_POLE;",
     "if (fabs(Y[1]) >= 89.6 * (3.14159265358979323846 / 180.0)) return ORC_GONE_POLE;",
     [lambda orc: S.test_pole_removal_step_and_tally(orc, -1.0)]),
    ("pole removal that does not tally the wave action",
     "if (r->state[i] != ORC_INVALID) t->removed_W += ray_W(r, i);",
     "if (r->state[i] != ORC_INVALID && r->state[i] != ORC_GONE_POLE) t->removed_W += ray_W(r, i);",
     [lambda orc: S.test_pole_removal_step_and_tally(orc, 1.0)]),
    ("spherical cell area without cos(phi)",
     "return (((r * r) * cos(phi)) * g->dx) * g->dy;",
     "return ((r * r) * g->dx) * g->dy;",
     [lambda orc: P.test_deposit_matches_brute_force(orc, "sphere")]),
]


@pytest.mark.parametrize("case", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_slip(orc, tmp_path, case):
    name, old, new, pins = case
    src = orc.source_text()
    assert src.count(old) == 1, f"the oracle source no longer holds the line this case edits: {old!r}"
    path = orc.build_variant(src.replace(old, new), str(tmp_path / "liborc_variant.so"))
    caught = []
    with orc.using_library(path):
        for pin in pins:
            try:
                pin(orc)
            except AssertionError:
                caught.append(pin)
    assert caught, f"no pin caught the planted slip: {name}"
    # the real oracle still passes the same pins
    for pin in pins:
        pin(orc)
