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

// One axis of a trilinear stencil: lower/upper node and the weight of the
// upper one.
struct Axis {
    int i0, i1;
    double w;
};

// Fractional index of a position on a cell-centred axis: g = (p - o)/d - 1/2.
__device__ inline Axis axis_periodic(double p, double origin, double d, int n)
{
    Axis a;
    const double g = (p - origin) / d - 0.5;
    if (!(fabs(g) < 1.0e15)) {
        a.i0 = 0;
        a.i1 = 0;
        a.w = g - g;
        return a;
    }
    const double fl = floor(g);
    a.w = g - fl;
    long long ii = (long long)fl;
    if (ii < 0 || ii >= n) {
        ii %= n;
        if (ii < 0) ii += n;
    }
    a.i0 = (int)ii;
    a.i1 = (ii + 1 == n) ? 0 : (int)ii + 1;
    return a;
}

__device__ inline Axis axis_clamped(double p, double origin, double d, int n)
{
    Axis a;
    const double g = (p - origin) / d - 0.5;
    if (g != g) {
        a.i0 = 0;
        a.i1 = 0;
        a.w = g;
        return a;
    }
    if (g <= 0.0) {
        a.i0 = 0;
        a.i1 = 0;
        a.w = 0.0;
    } else if (g >= (double)(n - 1)) {
        a.i0 = n - 1;
        a.i1 = n - 1;
        a.w = 0.0;
    } else {
        const double fl = floor(g);
        a.i0 = (int)fl;
        a.i1 = a.i0 + 1;
        a.w = g - fl;
    }
    return a;
}

__device__ inline Axis axis_x(const Grid &g, double x) { return axis_periodic(x, g.x0, g.dx, g.nx); }
__device__ inline Axis axis_y(const Grid &g, double y)
{
    return g.geometry == RT_CARTESIAN ? axis_periodic(y, g.y0, g.dy, g.ny) : axis_clamped(y, g.y0, g.dy, g.ny);
}
__device__ inline Axis axis_z(const Grid &g, double z) { return axis_clamped(z, 0.0, g.dz, g.nz); }

// The eight corners of the interpolation cell: column indices of the four
// (j, i) corners and the two levels, plus the weights.
struct Cell {
    int c00, c01, c10, c11;  // columns (j0,i0) (j0,i1) (j1,i0) (j1,i1), times nz
    int k0, k1;
    double wx, wy, wz;
};

// 24-bit products (full rate): a context has fewer than 2^24 columns and at
// most 640 levels, and every product is a cell index below 2^31
__device__ inline int mul24(int a, int b) { return (int)__umul24((uint32_t)a, (uint32_t)b); }
__device__ inline int col_cells(const Grid &g, int j, int i) { return mul24(mul24(j, g.nx) + i, g.nz); }

__device__ inline Cell cell_of(const Grid &g, const Axis &x, const Axis &y, const Axis &z)
{
    Cell c;
    c.c00 = col_cells(g, y.i0, x.i0);
    c.c01 = col_cells(g, y.i0, x.i1);
    c.c10 = col_cells(g, y.i1, x.i0);
    c.c11 = col_cells(g, y.i1, x.i1);
    c.k0 = z.i0;
    c.k1 = z.i1;
    c.wx = x.w;
    c.wy = y.w;
    c.wz = z.w;
    return c;
}

__device__ inline void locate(const Grid &g, double x, double y, double z, Cell &c)
{
    c = cell_of(g, axis_x(g, x), axis_y(g, y), axis_z(g, z));
}

__device__ inline double lerp3(double a0, double a1, double b0, double b1, double d0, double d1, double e0, double e1,
                               const Cell &c)
{
    const double c00 = a0 + c.wx * (a1 - a0);
    const double c10 = b0 + c.wx * (b1 - b0);
    const double c01 = d0 + c.wx * (d1 - d0);
    const double c11 = e0 + c.wx * (e1 - e0);
    const double c0 = c00 + c.wy * (c10 - c00);
    const double c1 = c01 + c.wy * (c11 - c01);
    return c0 + c.wz * (c1 - c0);
}

// the eight corner records of a packed double4 field (R records per cell)
template <int R>
struct Corners {
    double4 a0, a1, b0, b1, d0, d1, e0, e1;
    __device__ inline Corners() {}
    __device__ inline Corners(const double4 *__restrict__ F, const Cell &c, int r) { fill(F, c, r); }
    __device__ inline void fill(const double4 *__restrict__ F, const Cell &c, int r)
    {
        a0 = F[(c.c00 + c.k0) * R + r];
        a1 = F[(c.c01 + c.k0) * R + r];
        b0 = F[(c.c10 + c.k0) * R + r];
        b1 = F[(c.c11 + c.k0) * R + r];
        d0 = F[(c.c00 + c.k1) * R + r];
        d1 = F[(c.c01 + c.k1) * R + r];
        e0 = F[(c.c10 + c.k1) * R + r];
        e1 = F[(c.c11 + c.k1) * R + r];
    }
};
#define TRI64(K, q, c) lerp3(K.a0.q, K.a1.q, K.b0.q, K.b1.q, K.d0.q, K.d1.q, K.e0.q, K.e1.q, c)

// Trilinear interpolation of a packed 4-vector record, component by
// component: x on the four corner rows, then y, then z.  R = records per cell.
template <int R>
__device__ inline double4 tri4(const double4 *__restrict__ F, const Cell &c, int r)
{
    const Corners<R> K(F, c, r);
    double4 o;
    o.x = TRI64(K, x, c);
    o.y = TRI64(K, y, c);
    o.z = TRI64(K, z, c);
    o.w = TRI64(K, w, c);
    return o;
}

// Per-wave stencil box in LDS.  When every volume of a wave lies in one
// column and the wave's levels span at most WB64_LMAX - 6, the wave stages the
// A records of the 5 x 5 columns around it and the gradient records of the
// 3 x 3 columns, for the levels kbase .. kbase + L - 1, and a lookup whose
// corners lie in the box for every lane of the wave reads them from LDS; any
// other lookup reads global memory for the whole wave.  The values are the
// same either way.
#define WB64_LMAX 13
#define WB64_A (25 * WB64_LMAX)
#define WB64_RECS (WB64_A + 18 * WB64_LMAX)
extern __shared__ double4 wb64_lds[];

struct WBox {
    int on;  // wave-uniform
    int ic, jc, kbase, L;
};

struct BCell {
    int r00, r01, r10, r11, k0, k1;
    int on;  // faces: every lane's corners in the box (wave-uniform)
};

__device__ inline int wrapd(int d, int n)
{
    if (d > n / 2)
        d -= n;
    else if (d < -(n / 2))
        d += n;
    return d;
}

template <int R>
__device__ inline void fill_box(Corners<R> &K, int off, const BCell &b)
{
    K.a0 = wb64_lds[off + b.r00 + b.k0];
    K.a1 = wb64_lds[off + b.r01 + b.k0];
    K.b0 = wb64_lds[off + b.r10 + b.k0];
    K.b1 = wb64_lds[off + b.r11 + b.k0];
    K.d0 = wb64_lds[off + b.r00 + b.k1];
    K.d1 = wb64_lds[off + b.r01 + b.k1];
    K.e0 = wb64_lds[off + b.r10 + b.k1];
    K.e1 = wb64_lds[off + b.r11 + b.k1];
}

// f^2 (or its latitude derivative) between rows: equal, bit for bit, to the
// trilinear interpolation of the field replicated along x and z
__device__ inline double row_lerp(const double *__restrict__ f, const Axis &y)
{
    const double a = f[y.i0], b = f[y.i1];
    return a + y.w * (b - a);
}

// omega_hat^2 = (N^2 kh^2 + f^2 M2)/K^2 (eq. dispersion) with M2 = m^2 +
// Gamma^2 and K^2 = kh^2 + M2 (m^2 and kh^2 + m^2 where Gamma = 0)
__device__ inline double omega_hat(double N2, double f2, double kh2, double M2, double K2)
{
    return sqrt((N2 * kh2 + f2 * M2) / K2);
}

// Gamma^2 at a cell's interpolation point, 0 where Gamma = 0 (the branch is
// uniform: the field is there for every volume or for none)
__device__ inline double gam2(const double4 *Gm, const Cell &c)
{
    if (!Gm) return 0.0;
    // the first component of each corner record only
    const double *G = (const double *)Gm;
    return lerp3(G[4 * (c.c00 + c.k0)], G[4 * (c.c01 + c.k0)], G[4 * (c.c10 + c.k0)], G[4 * (c.c11 + c.k0)],
                 G[4 * (c.c00 + c.k1)], G[4 * (c.c01 + c.k1)], G[4 * (c.c10 + c.k1)], G[4 * (c.c11 + c.k1)], c);
}
__device__ inline double gam2(const Bg64P &b, const Cell &c) { return gam2(b.Gm, c); }

__device__ inline double gam2_at(const Grid &g, const Bg64P &b, double x, double y, double z)
{
    if (!b.Gm) return 0.0;
    Cell c;
    locate(g, x, y, z, c);
    return gam2(b, c);
}

// Offsets of a lookup's nodes from the wave's column and lowest staged level
// (the box position), and whether they lie in the 5 x 5 A box; faces replace
// the offsets of one axis
struct BOff {
    int dx0, dx1, dy0, dy1, k0, k1;
};

__device__ inline void box_offsets(const Grid &g, const WBox &w, const Axis &x, const Axis &y, const Axis &z, BOff &o)
{
    o.dx0 = wrapd(x.i0 - w.ic, g.nx);
    o.dx1 = wrapd(x.i1 - w.ic, g.nx);
    o.dy0 = y.i0 - w.jc;
    o.dy1 = y.i1 - w.jc;
    if (g.geometry == RT_CARTESIAN) {
        o.dy0 = wrapd(o.dy0, g.ny);
        o.dy1 = wrapd(o.dy1, g.ny);
    }
    o.k0 = z.i0 - w.kbase;
    o.k1 = z.i1 - w.kbase;
}

// box cell of a lookup in the box of radius RAD (2: A records, 5 x 5 columns;
// 1: gradient records, 3 x 3); on = 1 when the nodes of every lane of the
// wave lie in it (wave-uniform)
template <int RAD>
__device__ inline BCell box_cell(const WBox &w, const BOff &o)
{
    constexpr int side = 2 * RAD + 1;
    BCell b;
    b.r00 = mul24((o.dy0 + RAD) * side + (o.dx0 + RAD), w.L);
    b.r01 = mul24((o.dy0 + RAD) * side + (o.dx1 + RAD), w.L);
    b.r10 = mul24((o.dy1 + RAD) * side + (o.dx0 + RAD), w.L);
    b.r11 = mul24((o.dy1 + RAD) * side + (o.dx1 + RAD), w.L);
    b.k0 = o.k0;
    b.k1 = o.k1;
    const bool in = w.on && abs(o.dx0) <= RAD && abs(o.dx1) <= RAD && abs(o.dy0) <= RAD && abs(o.dy1) <= RAD &&
                    o.k0 >= 0 && o.k1 < w.L;
    b.on = __ballot(!in) == 0ull ? 1 : 0;
    return b;
}

// the A box cell of a face (AX: the face's axis, a its nodes on that axis)
template <int AX>
__device__ inline BCell face_box(const Grid &g, const WBox &w, const BOff &o, const Axis &a)
{
    BOff f = o;
    if (AX == 0) {
        f.dx0 = wrapd(a.i0 - w.ic, g.nx);
        f.dx1 = wrapd(a.i1 - w.ic, g.nx);
    } else if (AX == 1) {
        f.dy0 = a.i0 - w.jc;
        f.dy1 = a.i1 - w.jc;
        if (g.geometry == RT_CARTESIAN) {
            f.dy0 = wrapd(f.dy0, g.ny);
            f.dy1 = wrapd(f.dy1, g.ny);
        }
    } else {
        f.k0 = a.i0 - w.kbase;
        f.k1 = a.i1 - w.kbase;
    }
    return box_cell<2>(w, f);
}

// horizontal (AX = 0: U, AX = 1: V) or vertical (AX = 2) group velocity at
// one face: the wind component along the axis (none vertically) plus the
// intrinsic part, from the face's N^2 and f^2 (Section 3a, Appendix B)
template <int AX, bool GAM>
__device__ inline double face_v(const Grid &g, const WBox &w, const Bg64P &b, const Cell &f, const BCell &bc,
                                double k, double l, double m, double kh2, double m2, double K2, double K4, double f2f)
{
    (void)g;
    double c8[8], n8[8];
    if (bc.on) {
        const double *L = (const double *)wb64_lds;
        const int rr[4] = {bc.r00, bc.r01, bc.r10, bc.r11};
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const int rec = rr[t & 3] + ((t & 4) ? bc.k1 : bc.k0);
            if (AX < 2) c8[t] = L[4 * rec + AX];
            n8[t] = L[4 * rec + 2];
        }
    } else {
        const double *A = (const double *)b.A;
        const int cc[4] = {f.c00, f.c01, f.c10, f.c11};
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const int rec = cc[t & 3] + ((t & 4) ? f.k1 : f.k0);
            if (AX < 2) c8[t] = A[4 * (int64_t)rec + AX];
            n8[t] = A[4 * (int64_t)rec + 2];
        }
    }
    // corner order of lerp3: (j0,i0) (j0,i1) (j1,i0) (j1,i1) at k0, then at k1
    const double N2f = lerp3(n8[0], n8[1], n8[2], n8[3], n8[4], n8[5], n8[6], n8[7], f);
    const double M2f = GAM ? m2 + gam2(b, f) : m2;
    const double K2f = GAM ? kh2 + M2f : K2;
    const double K4f = GAM ? K2f * K2f : K4;
    const double omf = omega_hat(N2f, f2f, kh2, M2f, K2f);
    const double num = AX == 0 ? k * M2f : (AX == 1 ? l * M2f : m * kh2);
    const double t = (num * (N2f - f2f)) / (omf * K4f);
    if (AX == 2) return -t;
    const double wnd = lerp3(c8[0], c8[1], c8[2], c8[3], c8[4], c8[5], c8[6], c8[7], f);
    return wnd + t;
}

// Right-hand side of one RK stage.  Y = (x, y, z, k, l, m, Dx, Dy, Dz).
// Carrier wavevector tendency from the centre fields and gradients
// (eq. eikonal-sphere 1-3; flat limit on the box); carrier motion and extent
// rates from the group velocities at the opposing face centres (Section 3a,
// Appendix B).  A face differs from the centre along one axis, so only that
// axis is located again.  GAM: with the scale-height correction, Gamma^2 at
// the centre and each face and its gradients at the centre (m^2 is replaced
// by M2 = m^2 + Gamma^2 in the frequency and the horizontal group velocity,
// and d omega_hat / d Gamma^2 = -(kh^2 / (2 omega_hat K^2)) (N^2 - f^2)/K^2
// weighs the gradients).
template <bool SPH, bool GAM>
__device__ inline void rhs(const Grid &g, const Bg64P &b, const double *Y, double *F, const WBox &w)
{
    const double x = Y[0], y = Y[1], z = Y[2], k = Y[3], l = Y[4], m = Y[5];
    const double Dx = Y[6], Dy = Y[7], Dz = Y[8];
    const double kh2 = k * k + l * l;
    const double m2 = m * m;
    const Axis ax = axis_x(g, x), ay = axis_y(g, y), az = axis_z(g, z);
    const Cell c = cell_of(g, ax, ay, az);
    BOff bo;
    box_offsets(g, w, ax, ay, az, bo);
    double4 Gc = make_double4(0.0, 0.0, 0.0, 0.0);
    if (GAM) {
        const Corners<1> KG(b.Gm, c, 0);
        Gc.x = TRI64(KG, x, c);
        Gc.y = TRI64(KG, y, c);
        Gc.z = TRI64(KG, z, c);
        Gc.w = TRI64(KG, w, c);
    }
    const double M2 = GAM ? m2 + Gc.x : m2;
    const double K2 = kh2 + M2;
    const double K4 = K2 * K2;
    // centre: N2 and Ux, the last two components of the A records
    double N2c, Ux;
    {
        const BCell bc = box_cell<2>(w, bo);
        double n8[8], u8[8];
        const double *src = bc.on ? (const double *)wb64_lds : (const double *)b.A;
        const int rr[4] = {bc.on ? bc.r00 : c.c00, bc.on ? bc.r01 : c.c01, bc.on ? bc.r10 : c.c10,
                           bc.on ? bc.r11 : c.c11};
        const int kk0 = bc.on ? bc.k0 : c.k0, kk1 = bc.on ? bc.k1 : c.k1;
        if (bc.on) {
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const int rec = rr[t & 3] + ((t & 4) ? kk1 : kk0);
                n8[t] = src[4 * rec + 2];
                u8[t] = src[4 * rec + 3];
            }
        } else {
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const int64_t rec = rr[t & 3] + ((t & 4) ? kk1 : kk0);
                n8[t] = src[4 * rec + 2];
                u8[t] = src[4 * rec + 3];
            }
        }
        N2c = lerp3(n8[0], n8[1], n8[2], n8[3], n8[4], n8[5], n8[6], n8[7], c);
        Ux = lerp3(u8[0], u8[1], u8[2], u8[3], u8[4], u8[5], u8[6], u8[7], c);
    }
    const double f2c = row_lerp(b.f2, ay);
    const double om = omega_hat(N2c, f2c, kh2, M2, K2);
    const double q = kh2 / ((2.0 * om) * K2);
    const double qf = M2 / ((2.0 * om) * K2);
    const double f2y = row_lerp(b.f2y, ay);
    // gradient records one at a time, (Uy Uz Vx Vy) then (Vz N2x N2y N2z),
    // each folded into the refraction sums as soon as it is complete
    double gk = 0.0, gl = 0.0, gm = 0.0;
    {
        const BCell bg = box_cell<1>(w, bo);
        double gk0 = 0.0, gl0 = 0.0, kUz = 0.0;
#pragma unroll 1
        for (int r = 0; r < 2; r++) {
            Corners<2> KG;
            if (bg.on)
                fill_box(KG, WB64_A + r * 9 * WB64_LMAX, bg);
            else
                KG.fill(b.G, c, r);
            const double4 Gr =
                make_double4(TRI64(KG, x, c), TRI64(KG, y, c), TRI64(KG, z, c), TRI64(KG, w, c));
            if (r == 0) {
                gk0 = k * Ux + l * Gr.z;     // k Ux + l Vx
                gl0 = k * Gr.x + l * Gr.w;   // k Uy + l Vy
                kUz = k * Gr.y;
            } else {
                gk = gk0 + q * Gr.y;                  // + q N2x
                gl = (gl0 + q * Gr.z) + qf * f2y;     // + q N2y + qf (f2)_y
                gm = (kUz + l * Gr.x) + q * Gr.w;     // k Uz + l Vz + q N2z
            }
        }
    }
    if (GAM) {
        const double qg = -((kh2 * (N2c - f2c)) / (((2.0 * om) * K2) * K2));
        gk = gk + qg * Gc.y;
        gl = gl + qg * Gc.z;
        gm = gm + qg * Gc.w;
    }

    // faces, one axis at a time and one face at a time (bounded register
    // use): a face differs from the centre along its own axis only, so the
    // centre's nodes of the other two axes (and their cell and box offsets)
    // are kept
    const int X0 = mul24(ax.i0, g.nz), X1 = mul24(ax.i1, g.nz);  // x nodes, in cells
    const int R0 = c.c00 - X0, R1 = c.c10 - X0;                    // y rows, in cells
    double cxp = 0.0, cxm = 0.0, cyp = 0.0, cym = 0.0, czp = 0.0, czm = 0.0;
#pragma unroll 1
    for (int sd = 0; sd < 2; sd++) {
        const double sg = sd ? -0.5 : 0.5;
        const Axis fx = axis_x(g, x + sg * Dx);
        Cell f = c;
        const int F0 = mul24(fx.i0, g.nz), F1 = mul24(fx.i1, g.nz);
        f.c00 = R0 + F0;
        f.c01 = R0 + F1;
        f.c10 = R1 + F0;
        f.c11 = R1 + F1;
        f.wx = fx.w;
        const double v = face_v<0, GAM>(g, w, b, f, face_box<0>(g, w, bo, fx), k, l, m, kh2, m2, K2, K4, f2c);
        cxp = sd == 0 ? v : cxp;
        cxm = sd == 1 ? v : cxm;
    }
#pragma unroll 1
    for (int sd = 0; sd < 2; sd++) {
        const double sg = sd ? -0.5 : 0.5;
        const Axis fy = axis_y(g, y + sg * Dy);
        Cell f = c;
        const int Q0 = mul24(mul24(fy.i0, g.nx), g.nz), Q1 = mul24(mul24(fy.i1, g.nx), g.nz);
        f.c00 = Q0 + X0;
        f.c01 = Q0 + X1;
        f.c10 = Q1 + X0;
        f.c11 = Q1 + X1;
        f.wy = fy.w;
        const double v = face_v<1, GAM>(g, w, b, f, face_box<1>(g, w, bo, fy), k, l, m, kh2, m2, K2, K4,
                                         row_lerp(b.f2, fy));
        cyp = sd == 0 ? v : cyp;
        cym = sd == 1 ? v : cym;
    }
#pragma unroll 1
    for (int sd = 0; sd < 2; sd++) {
        const double sg = sd ? -0.5 : 0.5;
        const Axis fz = axis_z(g, z + sg * Dz);
        Cell f = c;
        f.k0 = fz.i0;
        f.k1 = fz.i1;
        f.wz = fz.w;
        const double v = face_v<2, GAM>(g, w, b, f, face_box<2>(g, w, bo, fz), k, l, m, kh2, m2, K2, K4, f2c);
        czp = sd == 0 ? v : czp;
        czm = sd == 1 ? v : czm;
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
        double sphi, cphi;
        sincos(y, &sphi, &cphi);
        const double tphi = sphi / cphi;
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
