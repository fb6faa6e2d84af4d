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

// The eight corners of the interpolation cell: column indices of the four
// (j, i) corners and the two levels, plus the weights.
struct Cell {
    int c00, c01, c10, c11;  // columns (j0,i0) (j0,i1) (j1,i0) (j1,i1), times nz
    int k0, k1;
    double wx, wy, wz;
};

__device__ inline void locate(const Grid &g, double x, double y, double z, Cell &c)
{
    int i0, i1, j0, j1;
    axis_periodic(x, g.x0, g.dx, g.nx, i0, i1, c.wx);
    if (g.geometry == RT_CARTESIAN)
        axis_periodic(y, g.y0, g.dy, g.ny, j0, j1, c.wy);
    else
        axis_clamped(y, g.y0, g.dy, g.ny, j0, j1, c.wy);
    axis_clamped(z, 0.0, g.dz, g.nz, c.k0, c.k1, c.wz);
    c.c00 = (j0 * g.nx + i0) * g.nz;
    c.c01 = (j0 * g.nx + i1) * g.nz;
    c.c10 = (j1 * g.nx + i0) * g.nz;
    c.c11 = (j1 * g.nx + i1) * g.nz;
}

// Trilinear interpolation of a packed 4-vector record, component by
// component: x on the four corner rows, then y, then z.  R = records per cell.
template <int R>
__device__ inline double4 tri4(const double4 *__restrict__ F, const Cell &c, int r)
{
    const double4 a0 = F[(c.c00 + c.k0) * R + r], a1 = F[(c.c01 + c.k0) * R + r];
    const double4 b0 = F[(c.c10 + c.k0) * R + r], b1 = F[(c.c11 + c.k0) * R + r];
    const double4 d0 = F[(c.c00 + c.k1) * R + r], d1 = F[(c.c01 + c.k1) * R + r];
    const double4 e0 = F[(c.c10 + c.k1) * R + r], e1 = F[(c.c11 + c.k1) * R + r];
    double4 o;
#define TRI_(q)                                               \
    {                                                         \
        const double c00 = a0.q + c.wx * (a1.q - a0.q);      \
        const double c10 = b0.q + c.wx * (b1.q - b0.q);      \
        const double c01 = d0.q + c.wx * (d1.q - d0.q);      \
        const double c11 = e0.q + c.wx * (e1.q - e0.q);      \
        const double c0 = c00 + c.wy * (c10 - c00);           \
        const double c1 = c01 + c.wy * (c11 - c01);           \
        o.q = c0 + c.wz * (c1 - c0);                          \
    }
    TRI_(x)
    TRI_(y)
    TRI_(z)
    TRI_(w)
#undef TRI_
    return o;
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
__device__ inline void rhs(const Grid &g, const BgP<double> &b, const double *Y, double *F)
{
    const double x = Y[0], y = Y[1], z = Y[2], k = Y[3], l = Y[4], m = Y[5];
    const double Dx = Y[6], Dy = Y[7], Dz = Y[8];
    const double kh2 = k * k + l * l;
    const double m2 = m * m;
    const double K2 = kh2 + m2;
    const double K4 = K2 * K2;
    Cell c;
    locate(g, x, y, z, c);
    const double4 Ac = tri4<1>(b.A, c, 0);   // U V N2 f2
    const double om = omega_hat(Ac.z, Ac.w, kh2, m2, K2);
    const double q = kh2 / ((2.0 * om) * K2);
    const double qf = m2 / ((2.0 * om) * K2);
    // gradient records one at a time: (Ux Uy Uz Vx) (Vy Vz N2x N2y) (N2z f2y)
    double Ux = 0, Uy = 0, Uz = 0, Vx = 0, Vy = 0, Vz = 0, N2x = 0, N2y = 0, N2z = 0, f2y = 0;
#pragma unroll 1
    for (int r = 0; r < 3; r++) {
        const double4 Gr = tri4<3>(b.G, c, r);
        Ux = r == 0 ? Gr.x : Ux;
        Uy = r == 0 ? Gr.y : Uy;
        Uz = r == 0 ? Gr.z : Uz;
        Vx = r == 0 ? Gr.w : Vx;
        Vy = r == 1 ? Gr.x : Vy;
        Vz = r == 1 ? Gr.y : Vz;
        N2x = r == 1 ? Gr.z : N2x;
        N2y = r == 1 ? Gr.w : N2y;
        N2z = r == 2 ? Gr.x : N2z;
        f2y = r == 2 ? Gr.y : f2y;
    }
    const double gk = (k * Ux + l * Vx) + q * N2x;
    const double gl = ((k * Uy + l * Vy) + q * N2y) + qf * f2y;
    const double gm = (k * Uz + l * Vz) + q * N2z;

    // faces: +x, -x, +y, -y, +z, -z, one at a time (bounded register use)
    double cxp = 0.0, cxm = 0.0, cyp = 0.0, cym = 0.0, czp = 0.0, czm = 0.0;
#pragma unroll 1
    for (int fc = 0; fc < 6; fc++) {
        const int ax = fc >> 1;
        const double sg = (fc & 1) ? -0.5 : 0.5;
        double px = x, py = y, pz = z;
        if (ax == 0)
            px = x + sg * Dx;
        else if (ax == 1)
            py = y + sg * Dy;
        else
            pz = z + sg * Dz;
        Cell f;
        locate(g, px, py, pz, f);
        const double4 Af = tri4<1>(b.A, f, 0);
        const double omf = omega_hat(Af.z, Af.w, kh2, m2, K2);
        const double num = ax == 0 ? k * m2 : (ax == 1 ? l * m2 : m * kh2);
        const double t = (num * (Af.z - Af.w)) / (omf * K4);
        const double v = ax == 0 ? Af.x + t : (ax == 1 ? Af.y + t : -t);
        cxp = fc == 0 ? v : cxp;
        cxm = fc == 1 ? v : cxm;
        cyp = fc == 2 ? v : cyp;
        cym = fc == 3 ? v : cym;
        czp = fc == 4 ? v : czp;
        czm = fc == 5 ? v : czm;
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
