// Double-precision device arithmetic of the ray-volume step.
//
// The expressions are evaluated in a fixed order with contraction off (the
// translation units that include this header are built with
// -ffp-contract=off), so that on the Cartesian box the results are the
// correctly rounded values of the same operation sequence a plain CPU
// evaluation of the paper's formulas produces: +, -, *, / and sqrt are
// correctly rounded in IEEE double on gfx950, and floor is exact.
#pragma once
#include "rt_internal.h"

namespace d64 {

// Fractional index of a position on a cell-centred axis: g = (p - o)/d - 1/2.
__device__ inline void axis_periodic(double p, double origin, double d, int n, int &i0, int &i1, double &w)
{
    double g = (p - origin) / d - 0.5;
    if (!(fabs(g) < 1.0e15)) {
        i0 = 0;
        i1 = 0;
        w = g - g;
        return;
    }
    double fl = floor(g);
    w = g - fl;
    long long ii = (long long)fl % n;
    if (ii < 0) ii += n;
    i0 = (int)ii;
    i1 = (int)((ii + 1) % n);
}

__device__ inline void axis_clamped(double p, double origin, double d, int n, int &i0, int &i1, double &w)
{
    double g = (p - origin) / d - 0.5;
    if (g != g) {
        i0 = 0;
        i1 = 0;
        w = g;
        return;
    }
    if (g <= 0.0) {
        i0 = 0;
        i1 = 0;
        w = 0.0;
    } else if (g >= (double)(n - 1)) {
        i0 = n - 1;
        i1 = n - 1;
        w = 0.0;
    } else {
        double fl = floor(g);
        i0 = (int)fl;
        i1 = i0 + 1;
        w = g - fl;
    }
}

struct Cell {
    int a00, a10, a01, a11;  // row offsets (j,k) combos: (j0,k0) (j1,k0) (j0,k1) (j1,k1)
    int i0, i1, j0, j1;
    double wx, wy, wz;
};

__device__ inline void locate(const Grid &g, double x, double y, double z, Cell &c)
{
    int k0, k1;
    axis_periodic(x, g.x0, g.dx, g.nx, c.i0, c.i1, c.wx);
    if (g.geometry == RT_CARTESIAN)
        axis_periodic(y, g.y0, g.dy, g.ny, c.j0, c.j1, c.wy);
    else
        axis_clamped(y, g.y0, g.dy, g.ny, c.j0, c.j1, c.wy);
    axis_clamped(z, 0.0, g.dz, g.nz, k0, k1, c.wz);
    c.a00 = (k0 * g.ny + c.j0) * g.nx;
    c.a10 = (k0 * g.ny + c.j1) * g.nx;
    c.a01 = (k1 * g.ny + c.j0) * g.nx;
    c.a11 = (k1 * g.ny + c.j1) * g.nx;
}

// x on the four corner rows, then y, then z
__device__ inline double tri(const double *__restrict__ F, const Cell &c)
{
    double a0 = F[c.a00 + c.i0], a1 = F[c.a00 + c.i1];
    double b0 = F[c.a10 + c.i0], b1 = F[c.a10 + c.i1];
    double d0 = F[c.a01 + c.i0], d1 = F[c.a01 + c.i1];
    double e0 = F[c.a11 + c.i0], e1 = F[c.a11 + c.i1];
    double c00 = a0 + c.wx * (a1 - a0);
    double c10 = b0 + c.wx * (b1 - b0);
    double c01 = d0 + c.wx * (d1 - d0);
    double c11 = e0 + c.wx * (e1 - e0);
    double c0 = c00 + c.wy * (c10 - c00);
    double c1 = c01 + c.wy * (c11 - c01);
    return c0 + c.wz * (c1 - c0);
}

__device__ inline double row(const double *__restrict__ F, const Cell &c)
{
    return F[c.j0] + c.wy * (F[c.j1] - F[c.j0]);
}

// omega_hat^2 = (N^2 kh^2 + f^2 m^2)/K^2 (eq. dispersion, Gamma = 0)
__device__ inline double omega_hat(double N2, double f2, double kh2, double m2, double K2)
{
    return sqrt((N2 * kh2 + f2 * m2) / K2);
}

// Right-hand side of one RK stage.  Y = (x, y, z, k, l, m, Dx, Dy, Dz).
// Carrier wavevector tendency from the centre fields and gradients
// (eq. eikonal-sphere 1-3, Gamma = 0; flat limit on the box); carrier motion
// and extent rates from the group velocities at the opposing face centres
// (Section 3a, Appendix B).
template <bool SPH>
__device__ inline void rhs(const Grid &g, const Bg<double> &b, const double *Y, double *F)
{
    const double x = Y[0], y = Y[1], z = Y[2], k = Y[3], l = Y[4], m = Y[5];
    const double Dx = Y[6], Dy = Y[7], Dz = Y[8];
    const double kh2 = k * k + l * l;
    const double m2 = m * m;
    const double K2 = kh2 + m2;
    const double K4 = K2 * K2;
    Cell c;
    locate(g, x, y, z, c);
    const double N2c = tri(b.N2, c);
    const double f2c = row(b.f2, c);
    const double om = omega_hat(N2c, f2c, kh2, m2, K2);
    const double q = kh2 / ((2.0 * om) * K2);
    const double qf = m2 / ((2.0 * om) * K2);
    const double gk = (k * tri(b.Ux, c) + l * tri(b.Vx, c)) + q * tri(b.N2x, c);
    const double gl = ((k * tri(b.Uy, c) + l * tri(b.Vy, c)) + q * tri(b.N2y, c)) + qf * row(b.f2y, c);
    const double gm = (k * tri(b.Uz, c) + l * tri(b.Vz, c)) + q * tri(b.N2z, c);

    double cxp, cxm, cyp, cym, czp, czm;
    {
        Cell f;
        double N2f, f2f, omf;
        locate(g, x + 0.5 * Dx, y, z, f);
        N2f = tri(b.N2, f);
        f2f = row(b.f2, f);
        omf = omega_hat(N2f, f2f, kh2, m2, K2);
        cxp = tri(b.U, f) + ((k * m2) * (N2f - f2f)) / (omf * K4);
        locate(g, x - 0.5 * Dx, y, z, f);
        N2f = tri(b.N2, f);
        f2f = row(b.f2, f);
        omf = omega_hat(N2f, f2f, kh2, m2, K2);
        cxm = tri(b.U, f) + ((k * m2) * (N2f - f2f)) / (omf * K4);
        locate(g, x, y + 0.5 * Dy, z, f);
        N2f = tri(b.N2, f);
        f2f = row(b.f2, f);
        omf = omega_hat(N2f, f2f, kh2, m2, K2);
        cyp = tri(b.V, f) + ((l * m2) * (N2f - f2f)) / (omf * K4);
        locate(g, x, y - 0.5 * Dy, z, f);
        N2f = tri(b.N2, f);
        f2f = row(b.f2, f);
        omf = omega_hat(N2f, f2f, kh2, m2, K2);
        cym = tri(b.V, f) + ((l * m2) * (N2f - f2f)) / (omf * K4);
        locate(g, x, y, z + 0.5 * Dz, f);
        N2f = tri(b.N2, f);
        f2f = row(b.f2, f);
        omf = omega_hat(N2f, f2f, kh2, m2, K2);
        czp = -(((m * kh2) * (N2f - f2f)) / (omf * K4));
        locate(g, x, y, z - 0.5 * Dz, f);
        N2f = tri(b.N2, f);
        f2f = row(b.f2, f);
        omf = omega_hat(N2f, f2f, kh2, m2, K2);
        czm = -(((m * kh2) * (N2f - f2f)) / (omf * K4));
    }
    if (!SPH) {
        F[0] = 0.5 * (cxp + cxm);
        F[1] = 0.5 * (cyp + cym);
        F[2] = 0.5 * (czp + czm);
        F[3] = -gk;
        F[4] = -gl;
        F[5] = -gm;
        F[6] = cxp - cxm;
        F[7] = cyp - cym;
        F[8] = czp - czm;
    } else {
        const double r = g.a + z;
        const double cphi = cos(y);
        const double tphi = tan(y);
        const double rc = r * cphi;
        const double uc = 0.5 * (cxp + cxm);
        const double vc = 0.5 * (cyp + cym);
        const double wc = 0.5 * (czp + czm);
        F[0] = uc / rc;
        F[1] = vc / r;
        F[2] = wc;
        F[3] = ((-gk) / rc - (k * wc) / r) + ((k * tphi) * vc) / r;
        F[4] = ((-gl) / r - (l * wc) / r) - ((k * tphi) * uc) / r;
        F[5] = ((-gm) + (k * uc) / r) + (l * vc) / r;
        F[6] = (cxp - cxm) / rc;
        F[7] = (cyp - cym) / r;
        F[8] = czp - czm;
    }
}

// Periodic wrap into [origin, origin+L); false if further than one period.
__device__ inline bool wrap(double &p, double origin, double L)
{
    double v = p - origin;
    if (v < 0.0) {
        v = v + L;
        if (v >= L) v = 0.0;
    } else if (v >= L) {
        v = v - L;
    }
    if (!(v >= 0.0 && v < L)) return false;
    p = (origin == 0.0) ? v : v + origin;
    return true;
}

__device__ inline int column_of(const Grid &g, double x, double y)
{
    double fi = floor((x - g.x0) / g.dx);
    double fj = floor((y - g.y0) / g.dy);
    if (fi < 0.0) fi = 0.0;
    if (fi > (double)(g.nx - 1)) fi = (double)(g.nx - 1);
    if (fj < 0.0) fj = 0.0;
    if (fj > (double)(g.ny - 1)) fj = (double)(g.ny - 1);
    return (int)fj * g.nx + (int)fi;
}

// Validity, wrap, removal and column key after an update.  Returns the key:
// the column index, or ncol + reason for a removed volume.
__device__ inline uint32_t post_step(const Grid &g, double *Y)
{
    for (int c = 0; c < 9; c++)
        if (!isfinite(Y[c])) return (uint32_t)(g.ncol + RK_INVALID);
    if (!(Y[6] > 0.0 && Y[7] > 0.0 && Y[8] > 0.0)) return (uint32_t)(g.ncol + RK_INVALID);
    const double K2 = (Y[3] * Y[3] + Y[4] * Y[4]) + Y[5] * Y[5];
    if (K2 == 0.0) return (uint32_t)(g.ncol + RK_INVALID);
    if (!wrap(Y[0], g.x0, g.Lx)) return (uint32_t)(g.ncol + RK_INVALID);
    if (g.geometry == RT_CARTESIAN) {
        if (!wrap(Y[1], g.y0, g.Ly)) return (uint32_t)(g.ncol + RK_INVALID);
    } else {
        if (fabs(Y[1]) >= g.pole) return (uint32_t)(g.ncol + RK_POLE);
    }
    if (Y[2] < 0.0) return (uint32_t)(g.ncol + RK_BOTTOM);
    if (Y[2] > g.Lz) return (uint32_t)(g.ncol + RK_TOP);
    return (uint32_t)column_of(g, Y[0], Y[1]);
}

}  // namespace d64
