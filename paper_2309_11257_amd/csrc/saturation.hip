// Spectral saturation (Section 3c, eq. instability-threshold and
// eq. turbulent-diffusivity) for both precisions.
//
//  1. Per cell, the spectrally integrated density perturbation
//       P = sum_j (m^2 kh^2 / (omega_hat K^2)) A_j alpha_j
//     and Q = sum_j P_j K_j^2, where A_j alpha_j for a level is the volume's
//     wave action W_j times its overlap fraction with the level over the cell
//     volume -- the projection of the fluxes, so the per-column deposition
//     machinery forms both sums (two level fields, deterministic).
//  2. kappa = max(0, (P - rho/2) / (2 dt Q)) per cell.
//  3. Every active volume is damped by the overlap-weighted mean of kappa
//     over the levels it covers in its column: N <- N max(0, 1 - 2 kbar K^2 dt)
//     (in single precision the wave action W, which is N times the fixed
//     phase-space areas, takes the factor).
// The double-precision path evaluates every expression in the oracle's order
// (built with -ffp-contract=off).
#include "dev64.h"
#include "f32.h"
#include "deposit_common.h"

// (m^2 kh^2 / (omega_hat K^2)) W / Dz and the same times K^2, per unit height
template <bool GAM>
struct PaySat64 {
    Grid g;
    Bg64P b;
    S64 st;
    double inv_dz;  // unused: the double-precision levels divide
    static constexpr bool EXACT_LEVELS = true;
    static constexpr int NL = 2, NI = 0;
    static constexpr int WAVES = 6;
    __device__ void load(uint32_t s, int col, double &zb, double &zt, double *bv) const
    {
        (void)col;
        const double x = st.x[s], y = st.y[s], z = st.z[s];
        const double k = st.k[s], l = st.l[s], m = st.m[s], Dz = st.dz[s];
        const double W = st.W[s];
        const d64::Axis ay = d64::axis_y(g, y);
        const d64::Cell c = d64::cell_of(g, d64::axis_x(g, x), ay, d64::axis_z(g, z));
        const d64::Corners<1> K(b.A, c, 0);
        const double N2 = TRI64(K, z, c);
        const double f2 = d64::row_lerp(b.f2, ay);
        const double kh2 = k * k + l * l;
        const double m2 = m * m;
        const double M2 = m2 + (GAM ? d64::gam2(b, c) : 0.0);
        const double K2 = kh2 + M2;
        const double om = d64::omega_hat(N2, f2, kh2, M2, K2);
        const double sw = (m2 * kh2) / (om * K2);
        const double a = W / Dz;
        bv[0] = sw * a;
        bv[1] = (sw * K2) * a;
        zb = z - 0.5 * Dz;
        zt = z + 0.5 * Dz;
    }
};

template <bool GAM>
struct PaySat32 {
    G32 g;
    Bg32P b;
    S32 st;
    double zdz;     // level spacing in double
    double inv_dz;  // its reciprocal (level spans)
    static constexpr bool EXACT_LEVELS = false;
    static constexpr int NL = 2, NI = 0;
    static constexpr int WAVES = 6;
    __device__ void load(uint32_t s, int col, double &zb, double &zt, double *bv) const
    {
        const int jc = (int)((uint32_t)col / (uint32_t)g.nx), ic = col - jc * g.nx;
        const int kc = st.lev[s];
        const float zeta = st.zeta[s];
        const float k = st.k[s], l = st.l[s], m = (float)st.m[s];
        const float Dz = st.dz[s];
        float N2, f2;
        f32::n2_f2(g, b, ic, jc, kc, st.xi[s], st.eta[s], zeta, N2, f2);
        const float kh2 = k * k + l * l;
        const float m2 = m * m;
        const float M2 = m2 + (GAM ? f32::gam2_at(g, b, ic, jc, kc, st.xi[s], st.eta[s], zeta) : 0.0f);
        const float K2 = kh2 + M2;
        const float invK2 = f32::rcp(K2);
        const float rom = f32::rsq((N2 * kh2 + f2 * M2) * invK2);  // 1 / omega_hat
        const float sw = m2 * kh2 * rom * invK2;
        const double a = st.W[s] * (double)f32::rcp(Dz);
        bv[0] = (double)sw * a;
        bv[1] = (double)(sw * K2) * a;
        const double zc = ((double)kc + (double)zeta) * zdz;
        zb = zc - 0.5 * (double)Dz;
        zt = zc + 0.5 * (double)Dz;
    }
};

// kappa per cell from the level sums PQ [2][nz+1][ncol] (slot nz unused)
__global__ void k_kappa(Grid g, const double *__restrict__ PQ, const double *__restrict__ rho, double dt,
                        double *__restrict__ kappa)
{
    const int64_t cells = (int64_t)g.nz * g.ncol;
    const int64_t at = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (at >= cells) return;
    const int kk = (int)(at / g.ncol);
    const int64_t plane = (int64_t)(g.nz + 1) * g.ncol;
    const double P = PQ[at], Q = PQ[plane + at];
    const double ex = P - 0.5 * rho[kk];
    kappa[at] = (ex > 0.0 && Q > 0.0) ? ex / ((2.0 * dt) * Q) : 0.0;
}

// overlap-weighted kappa of a volume spanning [zb, zt] in column c, and the
// damping factor for K^2 (held at zero or above)
__device__ inline double sat_factor(const Grid &g, const double *__restrict__ kappa, int c, double zb, double zt,
                                    double Dz, double K2, double dt, bool exact_levels, double inv_dz)
{
    int klo = (int)floor(exact_levels ? zb / g.dz : zb * inv_dz);
    int khi = (int)floor(exact_levels ? zt / g.dz : zt * inv_dz);
    if (klo < 0) klo = 0;
    if (khi > g.nz - 1) khi = g.nz - 1;
    double kbar = 0.0;
    for (int kk = klo; kk <= khi; kk++) {
        const double lo = (double)kk * g.dz, hi = (double)(kk + 1) * g.dz;
        const double o = fmin(zt, hi) - fmax(zb, lo);
        if (!(o > 0.0)) continue;
        kbar += (o / Dz) * kappa[(int64_t)kk * g.ncol + c];
    }
    if (!(kbar > 0.0)) return 1.0;
    const double fac = 1.0 - ((2.0 * kbar) * K2) * dt;
    return fac < 0.0 ? 0.0 : fac;
}

__global__ void k_damp64(Grid g, Bg64P b, S64 st, const uint32_t *__restrict__ perm,
                         const uint32_t *__restrict__ skeys, const DevCounters *__restrict__ dc,
                         const double *__restrict__ kappa, double dt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dc->n_active) return;
    const uint32_t s = perm[i];
    const int c = (int)skeys[i];
    const double z = st.z[s], Dz = st.dz[s];
    const double k = st.k[s], l = st.l[s], m = st.m[s];
    // K^2 includes Gamma^2 at the carrier
    const double K2 = (k * k + l * l) + (m * m + d64::gam2_at(g, b, st.x[s], st.y[s], z));
    const double fac = sat_factor(g, kappa, c, z - 0.5 * Dz, z + 0.5 * Dz, Dz, K2, dt, true, 0.0);
    const uint32_t h = st.home(s);
    if (fac != 1.0) {
        st.n[h] = st.n[h] * fac;
        st.W[s] = ((st.n[h] * st.px[h]) * st.py[h]) * st.pz[h];
    }
}

__global__ void k_damp32(Grid g, f32::G32 g32, Bg32P b, S32 st, const uint32_t *__restrict__ perm,
                         const uint32_t *__restrict__ skeys, const DevCounters *__restrict__ dc,
                         const double *__restrict__ kappa, double dt, double inv_dz)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dc->n_active) return;
    const uint32_t s = perm[i];
    const int c = (int)skeys[i];
    const double zc = ((double)st.lev[s] + (double)st.zeta[s]) * g.dz;
    const double Dz = (double)st.dz[s];
    const float k = st.k[s], l = st.l[s], m = (float)st.m[s];
    const int jc = c / g.nx, ic = c - jc * g.nx;
    const float G2 = f32::gam2_at(g32, b, ic, jc, st.lev[s], st.xi[s], st.eta[s], st.zeta[s]);
    const double K2 = (double)(k * k + l * l + (m * m + G2));
    const double fac = sat_factor(g, kappa, c, zc - 0.5 * Dz, zc + 0.5 * Dz, Dz, K2, dt, false, inv_dz);
    if (fac != 1.0) st.W[s] = st.W[s] * fac;
}

void launch_saturation64(const Grid &g, const Bg64P &b, S64 st, const uint32_t *perm, const uint32_t *skeys,
                         const uint32_t *colstart, const DevCounters *dc, const double *rho, double dt, double *PQ,
                         double *kappa, int64_t bound, hipStream_t s)
{
    if (b.Gm) {
        PaySat64<true> p{g, b, st, 1.0 / g.dz};
        launch_deposit_k(g, p, perm, colstart, PQ, s);
    } else {
        PaySat64<false> p{g, b, st, 1.0 / g.dz};
        launch_deposit_k(g, p, perm, colstart, PQ, s);
    }
    const int64_t cells = (int64_t)g.nz * g.ncol;
    k_kappa<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(g, PQ, rho, dt, kappa);
    if (bound > 0) k_damp64<<<(unsigned)((bound + 255) / 256), 256, 0, s>>>(g, b, st, perm, skeys, dc, kappa, dt);
}

void launch_saturation32(const Grid &g, const Bg32P &b, S32 st, const uint32_t *perm, const uint32_t *skeys,
                         const uint32_t *colstart, const DevCounters *dc, const double *rho, double dt, double *PQ,
                         double *kappa, int64_t bound, hipStream_t s)
{
    if (b.Gm) {
        PaySat32<true> p{f32::make_g32(g), b, st, g.dz, 1.0 / g.dz};
        launch_deposit_k(g, p, perm, colstart, PQ, s);
    } else {
        PaySat32<false> p{f32::make_g32(g), b, st, g.dz, 1.0 / g.dz};
        launch_deposit_k(g, p, perm, colstart, PQ, s);
    }
    const int64_t cells = (int64_t)g.nz * g.ncol;
    k_kappa<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(g, PQ, rho, dt, kappa);
    if (bound > 0)
        k_damp32<<<(unsigned)((bound + 255) / 256), 256, 0, s>>>(g, f32::make_g32(g), b, st, perm, skeys, dc, kappa, dt,
                                                                 1.0 / g.dz);
}
