// Single-precision arithmetic of the ray-volume step: grid constants,
// trilinear interpolation in the packed background, the RK stage right-hand
// side, and the periodic renormalisation of cell-relative positions.
//
// FP32 layout.  A horizontal position is held as the index of its column plus
// an offset in cell units, and the height as the index of its level plus an
// offset in level units, so the resolution is a fixed fraction of a cell
// (about 1e-7 cell) everywhere in the domain instead of degrading with the
// distance from the origin; this keeps the column assignment and the
// vertical overlaps of the FP32 path as sharp as the FP64 ones.  Extents
// Dx, Dy are in cell units, Dz in metres.
#pragma once
#include "rt_internal.h"

namespace f32 {

struct G32 {
    int geometry, nx, ny, nz, ncol;
    float dz, inv_dz, Lz, a;
    float inv_dx, inv_dy;  // Cartesian: 1/dx, 1/dy in 1/m; spherical: 1/dlambda, 1/dphi
    float y0, dyr;         // spherical: latitude origin and spacing (rad)
    float pole;
};

__host__ __device__ inline G32 make_g32(const Grid &g)
{
    G32 h;
    h.geometry = g.geometry;
    h.nx = g.nx;
    h.ny = g.ny;
    h.nz = g.nz;
    h.ncol = g.ncol;
    h.dz = (float)g.dz;
    h.inv_dz = (float)(1.0 / g.dz);
    h.Lz = (float)g.Lz;
    h.a = (float)g.a;
    h.inv_dx = (float)(1.0 / g.dx);
    h.inv_dy = (float)(1.0 / g.dy);
    h.y0 = (float)g.y0;
    h.dyr = (float)g.dy;
    h.pole = (float)g.pole;
    return h;
}

// one axis of a trilinear stencil: lower/upper node and the weight of the
// upper one
struct Axis {
    int i0, i1;
    float w;
};

// periodic axis: base cell ic, offset u in cell units
__device__ inline Axis axis_per(int ic, float u, int n)
{
    Axis a;
    const float t = u - 0.5f;
    if (!(fabsf(t) < 1.0e6f)) {
        a.i0 = 0;
        a.i1 = 0;
        a.w = t - t;
        return a;
    }
    const float fl = floorf(t);
    a.w = t - fl;
    int ii = ic + (int)fl;
    if (ii < 0 || ii >= n) {
        ii %= n;
        if (ii < 0) ii += n;
    }
    a.i0 = ii;
    a.i1 = (ii + 1 == n) ? 0 : ii + 1;
    return a;
}

// clamped axis (latitude rows, levels): value held beyond the end centres
__device__ inline Axis axis_clamp(int ic, float u, int n)
{
    Axis a;
    const float t = u - 0.5f;
    if (!(fabsf(t) < 1.0e6f)) {
        a.i0 = 0;
        a.i1 = 0;
        a.w = t - t;
        return a;
    }
    const float fl = floorf(t);
    const int j0 = ic + (int)fl;
    if (j0 < 0) {
        a.i0 = 0;
        a.i1 = 0;
        a.w = 0.0f;
    } else if (j0 >= n - 1) {
        a.i0 = n - 1;
        a.i1 = n - 1;
        a.w = 0.0f;
    } else {
        a.i0 = j0;
        a.i1 = j0 + 1;
        a.w = t - fl;
    }
    return a;
}

__device__ inline Axis axis_y(const G32 &g, int jc, float eta)
{
    return g.geometry == RT_CARTESIAN ? axis_per(jc, eta, g.ny) : axis_clamp(jc, eta, g.ny);
}

struct Cell {
    uint32_t c00, c01, c10, c11;  // columns (j0,i0) (j0,i1) (j1,i0) (j1,i1), times nz
    uint32_t k0, k1;
    float wx, wy, wz;
};

// cell indices use 24-bit multiplies (full rate): every factor is below 2^24
// (columns < 2^24 is checked at context creation) and every product below
// 2^31 (the single-precision path's index limit)
__device__ inline uint32_t col_base(const G32 &g, int j, int i)
{
    return __umul24(__umul24((uint32_t)j, (uint32_t)g.nx) + (uint32_t)i, (uint32_t)g.nz);
}

__device__ inline Cell cell_of(const G32 &g, const Axis &x, const Axis &y, const Axis &z)
{
    Cell c;
    c.c00 = col_base(g, y.i0, x.i0);
    c.c01 = col_base(g, y.i0, x.i1);
    c.c10 = col_base(g, y.i1, x.i0);
    c.c11 = col_base(g, y.i1, x.i1);
    c.k0 = (uint32_t)z.i0;
    c.k1 = (uint32_t)z.i1;
    c.wx = x.w;
    c.wy = y.w;
    c.wz = z.w;
    return c;
}

__device__ inline void locate(const G32 &g, int ic, int jc, int kc, float xi, float eta, float zeta, Cell &c)
{
    c = cell_of(g, axis_per(ic, xi, g.nx), axis_y(g, jc, eta), axis_clamp(kc, zeta, g.nz));
}

__device__ inline float lerp3(float a0, float a1, float b0, float b1, float d0, float d1, float e0, float e1,
                              const Cell &c)
{
    const float c00 = a0 + c.wx * (a1 - a0);
    const float c10 = b0 + c.wx * (b1 - b0);
    const float c01 = d0 + c.wx * (d1 - d0);
    const float c11 = e0 + c.wx * (e1 - e0);
    const float c0 = c00 + c.wy * (c10 - c00);
    const float c1 = c01 + c.wy * (c11 - c01);
    return c0 + c.wz * (c1 - c0);
}

// record at a 32-bit byte offset from a uniform base (the packed arrays are
// below 4 GiB, checked at context creation), so the load takes a scalar base
// and a 32-bit vector offset
__device__ inline float4 rec(const float4 *__restrict__ F, uint32_t index)
{
    return *(const float4 *)((const char *)F + (index << 4));
}

// the eight corner records of a packed float4 field (R records per cell)
template <int R>
struct Corners {
    float4 a0, a1, b0, b1, d0, d1, e0, e1;
    __device__ inline Corners() {}
    __device__ inline Corners(const float4 *__restrict__ F, const Cell &c, int r) { fill(F, c, r); }
    __device__ inline void fill(const float4 *__restrict__ F, const Cell &c, int r)
    {
        const uint32_t rr = (uint32_t)r;
        a0 = rec(F, (c.c00 + c.k0) * R + rr);
        a1 = rec(F, (c.c01 + c.k0) * R + rr);
        b0 = rec(F, (c.c10 + c.k0) * R + rr);
        b1 = rec(F, (c.c11 + c.k0) * R + rr);
        d0 = rec(F, (c.c00 + c.k1) * R + rr);
        d1 = rec(F, (c.c01 + c.k1) * R + rr);
        e0 = rec(F, (c.c10 + c.k1) * R + rr);
        e1 = rec(F, (c.c11 + c.k1) * R + rr);
    }
};
#define TRI_COMP(K, comp, c) \
    lerp3(K.a0.comp, K.a1.comp, K.b0.comp, K.b1.comp, K.d0.comp, K.d1.comp, K.e0.comp, K.e1.comp, c)

template <int R>
__device__ inline float4 tri4(const float4 *__restrict__ F, const Cell &c, int r)
{
    const Corners<R> K(F, c, r);
    float4 o;
    o.x = TRI_COMP(K, x, c);
    o.y = TRI_COMP(K, y, c);
    o.z = TRI_COMP(K, z, c);
    o.w = TRI_COMP(K, w, c);
    return o;
}

// f^2 and its latitude derivative depend on the row only: a linear
// interpolation between rows (equal to the trilinear one of the replicated
// field)
__device__ inline float row_lerp(const float *__restrict__ f, const Axis &y)
{
    // 32-bit byte offsets from the uniform base (rows are non-negative)
    const char *p = (const char *)f;
    const float a = *(const float *)(p + ((uint32_t)y.i0 << 2)), b = *(const float *)(p + ((uint32_t)y.i1 << 2));
    return a + y.w * (b - a);
}

// element idx of an array of 4-byte values, at a 32-bit byte offset from the
// array's uniform base (idx < 2^30)
template <class T>
__device__ inline T at(const T *__restrict__ p, uint32_t idx)
{
    static_assert(sizeof(T) == 4, "4-byte elements");
    return *(const T *)((const char *)p + (idx << 2));
}
template <class T>
__device__ inline void put(T *__restrict__ p, uint32_t idx, T v)
{
    static_assert(sizeof(T) == 4, "4-byte elements");
    *(T *)((char *)p + (idx << 2)) = v;
}

// single-precision reciprocal and reciprocal square root (one rounding each,
// within about one unit in the last place)
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// N2 and f2 at a carrier in the packed single-precision background
__device__ inline void n2_f2(const G32 &g, const Bg32P &b, int ic, int jc, int kc, float xi, float eta, float zeta,
                             float &N2, float &f2)
{
    const Axis ax = axis_per(ic, xi, g.nx), ay = axis_y(g, jc, eta), az = axis_clamp(kc, zeta, g.nz);
    const Cell c = cell_of(g, ax, ay, az);
    const Corners<1> K(b.A, c, 0);
    N2 = TRI_COMP(K, z, c);
    f2 = row_lerp(b.f2, ay);
}

// Gamma^2 at a cell's interpolation point, 0 where Gamma = 0 (a uniform
// branch: the field is there for every volume or for none)
__device__ inline float gam2(const Bg32P &b, const Cell &c)
{
    if (!b.Gm) return 0.0f;
    // the first component of each corner record only (32-bit byte offsets)
    const char *G = (const char *)b.Gm;
    auto at = [&](uint32_t idx) { return *(const float *)(G + (idx << 4)); };
    return lerp3(at(c.c00 + c.k0), at(c.c01 + c.k0), at(c.c10 + c.k0), at(c.c11 + c.k0), at(c.c00 + c.k1),
                 at(c.c01 + c.k1), at(c.c10 + c.k1), at(c.c11 + c.k1), c);
}

__device__ inline float gam2_at(const G32 &g, const Bg32P &b, int ic, int jc, int kc, float xi, float eta,
                                float zeta)
{
    if (!b.Gm) return 0.0f;
    Cell c;
    locate(g, ic, jc, kc, xi, eta, zeta, c);
    return gam2(b, c);
}

// Per-wave stencil box in LDS.  When every volume of a wave lies in one
// column and the wave's levels span at most WB_LMAX - 6, the wave stages the
// A records of the 5 x 5 columns around it for the levels kbase .. kbase +
// L - 1 (the faces' reach), the gradient records of the 3 x 3 columns for
// the narrower window kbase_g .. kbase_g + LG - 1 (the centre's nodes only),
// plus f2 and (f2)_y of the five rows, and interpolates from LDS; a lookup
// that falls outside the box for any lane of the wave goes to global memory
// for the whole wave.  8 160 bytes a wave: 20 waves fit a compute unit's LDS.
#define WB_LMAX 13
#define WB_GMAX (WB_LMAX - 3)
#define WB_A (25 * WB_LMAX)
#define WB_F2 (WB_A + 18 * WB_GMAX)  // five rows of (f2, (f2)_y, 0, 0) after the records
#define WB_RECS (WB_F2 + 5)
// with the scale-height correction the Gamma^2 records of the 5 x 5 columns
// follow, in the A records' layout (13 424 bytes a wave)
#define WB_GM WB_RECS
#define WB_RECS_GAM (WB_RECS + 25 * WB_LMAX)
extern __shared__ float4 wb_lds[];

struct WBox {
    int on;  // wave-uniform
    int ic, jc, kbase, L, base;
    int kbase_g, LG;  // level window of the gradient records
};

__device__ inline int wrapd(int d, int n)
{
    if (d > n / 2) d -= n;
    else if (d < -(n / 2)) d += n;
    return d;
}

// box position of a stencil: the box holds column (ic + d) mod nx at x
// offset d (and the row the global lookup reads at y offset d), so the upper
// x node of a cell is always the next box column and the upper y and z nodes
// the next row and level unless the axis clamps them; one base index and two
// strides (0 or a row, 0 or a level) locate all eight corners.  Layout
// [dy][dx][k] with a column stride of LS records (WB_LMAX for the A records,
// WB_GMAX for the gradient records), levels from kb, L of them.
struct BCell {
    int base, sy, sz;
};

template <int RAD, int LS>
__device__ inline bool box_of(const G32 &g, const WBox &w, int kb, int L, const Axis &x, const Axis &y, const Axis &z,
                              BCell &b)
{
    const int dx0 = wrapd(x.i0 - w.ic, g.nx);
    int dy0 = y.i0 - w.jc;
    if (g.geometry == RT_CARTESIAN) dy0 = wrapd(dy0, g.ny);
    const int ey = y.i1 - y.i0, k0 = z.i0 - kb;  // ey: 0 (clamped) or 1 (or 1 - ny, periodic wrap)
    const int side = 2 * RAD + 1;
    b.base = __mul24((dy0 + RAD) * side + (dx0 + RAD), LS) + k0;
    b.sy = ey != 0 ? side * LS : 0;
    b.sz = z.i1 - z.i0;
    return dx0 >= -RAD && dx0 < RAD && dy0 >= -RAD && dy0 + (ey != 0 ? 1 : 0) <= RAD && k0 >= 0 && k0 + b.sz < L;
}

template <int R, int LS>
__device__ inline void fill_box(Corners<R> &K, int off, const BCell &b)
{
    const int p = off + b.base;
    K.a0 = wb_lds[p];
    K.a1 = wb_lds[p + LS];
    K.b0 = wb_lds[p + b.sy];
    K.b1 = wb_lds[p + b.sy + LS];
    K.d0 = wb_lds[p + b.sz];
    K.d1 = wb_lds[p + b.sz + LS];
    K.e0 = wb_lds[p + b.sy + b.sz];
    K.e1 = wb_lds[p + b.sy + b.sz + LS];
}

// A corners of a cell: from the box when every lane of the wave is inside
__device__ inline void corners_A(const G32 &g, const WBox &w, const Bg32P &b, const Axis &x, const Axis &y,
                                 const Axis &z, const Cell &c, Corners<1> &K)
{
    BCell bc;
    const bool in = w.on && box_of<2, WB_LMAX>(g, w, w.kbase, w.L, x, y, z, bc);
    if (__ballot(!in) == 0ull)
        fill_box<1, WB_LMAX>(K, w.base, bc);
    else
        K.fill(b.A, c, 0);
}

__device__ inline void corners_G(const G32 &g, const WBox &w, const Bg32P &b, const Axis &x, const Axis &y,
                                 const Axis &z, const Cell &c, int r, Corners<2> &K)
{
    BCell bc;
    const bool in = w.on && box_of<1, WB_GMAX>(g, w, w.kbase_g, w.LG, x, y, z, bc);
    if (__ballot(!in) == 0ull)
        fill_box<2, WB_GMAX>(K, w.base + WB_A + r * 9 * WB_GMAX, bc);
    else
        K.fill(b.G, c, r);
}

// Right-hand side from the centre's refraction sums (gk, gl, gm) and the face
// velocities of each axis (sum s and half-difference h of the + and - faces).
template <bool SPH>
__device__ inline void assemble(const G32 &g, int kc, float2 lat, const float *Y, float gk, float gl, float gm,
                                float sx, float hx, float sy, float hy, float sz, float hz, float *F)
{
    const float k = Y[3], l = Y[4];
    if (!SPH) {
        F[0] = 0.5f * sx * g.inv_dx;
        F[1] = 0.5f * sy * g.inv_dy;
        F[2] = 0.5f * sz * g.inv_dz;
        F[3] = -gk;
        F[4] = -gl;
        F[5] = -gm;
        F[6] = 2.0f * hx * g.inv_dx;
        F[7] = 2.0f * hy * g.inv_dy;
        F[8] = 2.0f * hz;
    } else {
        const float r = g.a + ((float)kc + Y[2]) * g.dz;
        const float ir = rcp(r);
        // sin and cos of the latitude from those of the cell's southern edge
        // (lat) and the Taylor series of the offset d = y dphi; up to half a
        // radian the terms kept leave an error far below one ulp
        const float d = Y[1] * g.dyr, d2 = d * d;
        const float sd = d + d * d2 * (-1.0f / 6.0f + d2 * (1.0f / 120.0f + d2 * (-1.0f / 5040.0f + d2 * (1.0f / 362880.0f))));
        const float cd = 1.0f + d2 * (-0.5f + d2 * (1.0f / 24.0f + d2 * (-1.0f / 720.0f + d2 * (1.0f / 40320.0f))));
        const float sphi = lat.x * cd + lat.y * sd;
        const float cphi = lat.y * cd - lat.x * sd;
        const float icphi = rcp(cphi);
        const float tphi = sphi * icphi;
        const float irc = ir * icphi;
        const float uc = 0.5f * sx;
        const float vc = 0.5f * sy;
        const float wc = 0.5f * sz;
        F[0] = uc * irc * g.inv_dx;
        F[1] = vc * ir * g.inv_dy;
        F[2] = wc * g.inv_dz;
        F[3] = -gk * irc - k * wc * ir + k * tphi * vc * ir;
        F[4] = -gl * ir - l * wc * ir - k * tphi * uc * ir;
        F[5] = -gm + k * uc * ir + l * vc * ir;
        F[6] = 2.0f * hx * irc * g.inv_dx;
        F[7] = 2.0f * hy * ir * g.inv_dy;
        F[8] = 2.0f * hz;
    }
}

// ---------------------------------------------------------------------------
// Box-only stage.  When every lookup of every lane of a wave lies in the
// wave's stencil box, the stage works in box coordinates: a horizontal node
// is an offset from the wave's column, so no periodic wrap or row clamp is
// formed (the box holds the wrapped columns and the clamped rows; where a
// row is clamped both nodes hold the same record, and interpolating between
// equal values returns that value), and a lookup is one LDS base index.

// lower node of one axis relative to the base cell and the upper node's
// weight; the offset is clamped to +-1e6 cells (a non-finite offset belongs
// to a state that is removed after the step)
__device__ inline int bnode(float t, float &wgt)
{
    const float tc = fminf(fmaxf(t, -1.0e6f), 1.0e6f);
    const float fl = floorf(tc);
    wgt = tc - fl;
    return (int)fl;
}

// level axis, clamped at the grid's ends: box level of the lower node, step to
// the upper node (0 where clamped) and its weight
__device__ inline int blev(const G32 &g, const WBox &w, int kc, float t, int &sz, float &wgt)
{
    float f;
    const int j0 = kc + bnode(t, f);
    const bool out = j0 < 0 || j0 >= g.nz - 1;
    sz = out ? 0 : 1;
    wgt = out ? 0.0f : f;
    return (j0 < 0 ? 0 : (j0 >= g.nz - 1 ? g.nz - 1 : j0)) - w.kbase;
}

// face positions, written once so that the box test and the stage form the
// same values
__device__ inline float face_t(float c, float sg, float ext) { return fmaf(sg, ext, c) - 0.5f; }

// every lookup of the stage in the box: centre nodes at offsets -1 or 0 (the
// 3 x 3 gradient box), face nodes at -2 .. 1 (the 5 x 5 box), levels inside
// (the centre's in both level windows)
__device__ inline bool box_stage_in(const G32 &g, const WBox &w, int kc, const float *Y)
{
    // horizontal nodes: floor(t) in lo .. hi exactly when lo <= t < hi + 1
    // (false for a NaN); the stage forms the same t
    const float tx = Y[0] - 0.5f, ty = Y[1] - 0.5f;
    const float txp = face_t(Y[0], 0.5f, Y[6]), txm = face_t(Y[0], -0.5f, Y[6]);
    const float typ = face_t(Y[1], 0.5f, Y[7]), tym = face_t(Y[1], -0.5f, Y[7]);
    const bool hor = tx >= -1.0f && tx < 1.0f && ty >= -1.0f && ty < 1.0f && txp >= -2.0f && txp < 2.0f &&
                     txm >= -2.0f && txm < 2.0f && typ >= -2.0f && typ < 2.0f && tym >= -2.0f && tym < 2.0f;
    float t;
    int s0, s1, s2;
    const float sdz = Y[8] * g.inv_dz;
    const int k0 = blev(g, w, kc, Y[2] - 0.5f, s0, t);
    const int kp = blev(g, w, kc, face_t(Y[2], 0.5f, sdz), s1, t);
    const int km = blev(g, w, kc, face_t(Y[2], -0.5f, sdz), s2, t);
    const int kg = k0 + (w.kbase - w.kbase_g);
    return hor && (uint32_t)k0 < (uint32_t)(w.L - s0) && (uint32_t)kp < (uint32_t)(w.L - s1) &&
           (uint32_t)km < (uint32_t)(w.L - s2) && (uint32_t)kg < (uint32_t)(w.LG - s0);
}

// eight corners from LDS: p the lower corner's record, sx/sy/sz the steps to
// the upper nodes (records)
template <int R>
__device__ inline void box_corners(Corners<R> &K, int p, int sxs, int sys, int szs)
{
    K.a0 = wb_lds[p];
    K.a1 = wb_lds[p + sxs];
    K.b0 = wb_lds[p + sys];
    K.b1 = wb_lds[p + sys + sxs];
    K.d0 = wb_lds[p + szs];
    K.d1 = wb_lds[p + szs + sxs];
    K.e0 = wb_lds[p + szs + sys];
    K.e1 = wb_lds[p + szs + sys + sxs];
}

// f2 or (f2)_y (component c of the row records) between box rows r and r + 1
__device__ inline float box_row(int r, float wgt, int c)
{
    const float *f = (const float *)&wb_lds[WB_F2];
    const float a = f[4 * r + c], b = f[4 * r + 4 + c];
    return a + wgt * (b - a);
}

template <bool SPH, bool GAM>
__device__ inline void rhs_box(const G32 &g, int kc, float2 lat, const float *Y, float *F, const WBox &w)
{
    constexpr int SA = 5 * WB_LMAX, SG = 3 * WB_GMAX;  // row steps of the A and gradient boxes
    const float k = Y[3], l = Y[4], m = Y[5];
    const float kh2 = k * k + l * l;
    const float m2 = m * m;
    Cell c;
    int sz;
    const int dx = bnode(Y[0] - 0.5f, c.wx), dy = bnode(Y[1] - 0.5f, c.wy);
    const int kb = blev(g, w, kc, Y[2] - 0.5f, sz, c.wz);
    const int pyz = (dy + 2) * SA + kb;  // A box: row and level of the centre
    // GAM: Gamma^2 and its gradients at the centre (the Gamma^2 records sit
    // in the A records' layout)
    float4 Gc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (GAM) {
        Corners<1> KM;
        box_corners(KM, WB_GM + pyz + (dx + 2) * WB_LMAX, WB_LMAX, SA, sz);
        Gc = make_float4(TRI_COMP(KM, x, c), TRI_COMP(KM, y, c), TRI_COMP(KM, z, c), TRI_COMP(KM, w, c));
    }
    const float M2 = GAM ? m2 + Gc.x : m2;
    const float K2 = kh2 + M2;
    const float invK2 = rcp(K2);
    const float invK4 = invK2 * invK2;
    const float f2c = box_row(dy + 2, c.wy, 0);
    float gk, gl, gm;
    {
        Corners<1> KA;
        box_corners(KA, pyz + (dx + 2) * WB_LMAX, WB_LMAX, SA, sz);
        const float N2c = TRI_COMP(KA, z, c);
        const float rom = rsq((N2c * kh2 + f2c * M2) * invK2);  // 1 / omega_hat
        const float h = 0.5f * invK2 * rom;
        const float q = kh2 * h;
        const float qf = M2 * h;
        gk = k * TRI_COMP(KA, w, c);
        gl = qf * box_row(dy + 2, c.wy, 1);
        gm = 0.0f;
        if (GAM) {
            const float qg = -(q * (N2c - f2c) * invK2);
            gk += qg * Gc.y;
            gl += qg * Gc.z;
            gm += qg * Gc.w;
        }
        const int pg = WB_A + (dy + 1) * SG + (dx + 1) * WB_GMAX + kb + (w.kbase - w.kbase_g);
        // gradient records one at a time (bounded register use)
#pragma unroll 1
        for (int r = 0; r < 2; r++) {
            Corners<2> KG;
            box_corners(KG, pg + r * 9 * WB_GMAX, WB_GMAX, SG, sz);
            const float4 Gr = make_float4(TRI_COMP(KG, x, c), TRI_COMP(KG, y, c), TRI_COMP(KG, z, c), TRI_COMP(KG, w, c));
            if (r == 0) {  // Uy Uz Vx Vy
                gl += k * Gr.x + l * Gr.w;
                gm += k * Gr.y;
                gk += l * Gr.z;
            } else {  // Vz N2x N2y N2z
                gm += l * Gr.x + q * Gr.w;
                gk += q * Gr.y;
                gl += q * Gr.z;
            }
        }
    }
    // a face's M2 = m^2 + Gamma^2 and 1/K^4 (the centre's without Gamma);
    // p: the face's lower corner in the A layout, sxs/szs its steps
    auto face_m2 = [&](int p, int sys, int szs, const Cell &f, float &M2f, float &invK4f) {
        if (GAM) {
            const float4 *G = wb_lds + WB_GM + p;
            const float g2 = lerp3(G[0].x, G[WB_LMAX].x, G[sys].x, G[sys + WB_LMAX].x, G[szs].x, G[szs + WB_LMAX].x,
                                   G[szs + sys].x, G[szs + sys + WB_LMAX].x, f);
            M2f = m2 + g2;
            const float iK2 = rcp(kh2 + M2f);
            invK4f = iK2 * iK2;
        } else {
            M2f = M2;
            invK4f = invK4;
        }
    };
    const float sdz = Y[8] * g.inv_dz;
    float sx = 0.0f, hx = 0.0f, sy = 0.0f, hy = 0.0f, szs = 0.0f, hz = 0.0f;
#pragma unroll 1
    for (int sd = 0; sd < 2; sd++) {
        const float sg = sd ? -0.5f : 0.5f;
        Cell f = c;
        const int d = bnode(face_t(Y[0], sg, Y[6]), f.wx);
        const int p = pyz + (d + 2) * WB_LMAX;
        Corners<1> K;
        box_corners(K, p, WB_LMAX, SA, sz);
        float M2f, invK4f;
        face_m2(p, SA, sz, f, M2f, invK4f);
        const float N2f = TRI_COMP(K, z, f);
        const float romf = rsq((N2f * kh2 + f2c * M2f) * (GAM ? rcp(kh2 + M2f) : invK2));
        const float v = TRI_COMP(K, x, f) + k * M2f * ((N2f - f2c) * invK4f * romf);
        sx += v;
        hx += sg * v;
    }
#pragma unroll 1
    for (int sd = 0; sd < 2; sd++) {
        const float sg = sd ? -0.5f : 0.5f;
        Cell f = c;
        const int d = bnode(face_t(Y[1], sg, Y[7]), f.wy);
        const int p = (d + 2) * SA + (dx + 2) * WB_LMAX + kb;
        Corners<1> K;
        box_corners(K, p, WB_LMAX, SA, sz);
        float M2f, invK4f;
        face_m2(p, SA, sz, f, M2f, invK4f);
        const float N2f = TRI_COMP(K, z, f);
        const float f2f = box_row(d + 2, f.wy, 0);
        const float romf = rsq((N2f * kh2 + f2f * M2f) * (GAM ? rcp(kh2 + M2f) : invK2));
        const float v = TRI_COMP(K, y, f) + l * M2f * ((N2f - f2f) * invK4f * romf);
        sy += v;
        hy += sg * v;
    }
#pragma unroll 1
    for (int sd = 0; sd < 2; sd++) {
        const float sg = sd ? -0.5f : 0.5f;
        Cell f = c;
        int szf;
        const int kf = blev(g, w, kc, face_t(Y[2], sg, sdz), szf, f.wz);
        const int p = (dy + 2) * SA + (dx + 2) * WB_LMAX + kf;
        Corners<1> K;
        box_corners(K, p, WB_LMAX, SA, szf);
        float M2f, invK4f;
        face_m2(p, SA, szf, f, M2f, invK4f);
        const float N2f = TRI_COMP(K, z, f);
        const float romf = rsq((N2f * kh2 + f2c * M2f) * (GAM ? rcp(kh2 + M2f) : invK2));
        const float v = -m * kh2 * ((N2f - f2c) * invK4f * romf);
        szs += v;
        hz += sg * v;
    }
    assemble<SPH>(g, kc, lat, Y, gk, gl, gm, sx, hx, sy, hy, szs, hz, F);
}

// N^2 and f^2 at a volume's carrier (base cell ic, jc, kc and offsets in
// cell and level units): from the wave's stencil box when every lane's nodes
// lie in it (a volume that moved to a neighbouring column included), else
// from global memory.  The box holds the wrapped columns and the clamped
// rows (interpolating between two equal clamped rows returns that row), and
// a clamped level has weight 0 in both forms; the two forms may still round
// differently by an ulp where the compiler contracts them differently.
__device__ inline void n2_f2_carrier(const G32 &g, const Bg32P &b, const WBox &w, int ic, int jc, int kc, float xi,
                                     float eta, float zeta, float &N2, float &f2)
{
    constexpr int SA = 5 * WB_LMAX;
    Cell c;
    int sz;
    int dy0 = jc - w.jc;
    if (g.geometry == RT_CARTESIAN) dy0 = wrapd(dy0, g.ny);
    const int dx = wrapd(ic - w.ic, g.nx) + bnode(xi - 0.5f, c.wx), dy = dy0 + bnode(eta - 0.5f, c.wy);
    const int kb = blev(g, w, kc, zeta - 0.5f, sz, c.wz);
    const bool in = w.on && dx >= -2 && dx <= 1 && dy >= -2 && dy <= 1 && kb >= 0 && kb + sz < w.L;
    if (__ballot(!in) == 0ull) {
        Corners<1> K;
        box_corners(K, (dy + 2) * SA + (dx + 2) * WB_LMAX + kb, WB_LMAX, SA, sz);
        N2 = TRI_COMP(K, z, c);
        f2 = box_row(dy + 2, c.wy, 0);
    } else {
        n2_f2(g, b, ic, jc, kc, xi, eta, zeta, N2, f2);
    }
}

// RK stage right-hand side in cell units: Y = (xi, eta, zeta, k, l, m, Dxi,
// Deta, Dz), offsets relative to the base cell (ic, jc, kc), Dz in metres.
// Centre: 12 fields from three records per corner (U V N2 Ux | Uy Uz Vx Vy |
// Vz N2x N2y N2z) plus f2 and (f2)_y by row.  Faces: (U or V) and N2 from the
// first record; the face differs from the centre along one axis only, so the
// other two axes are reused, and f2 is the centre's except on the y faces.
// GAM: with the scale-height correction (global lookups of the Gamma^2
// records): m^2 -> M2 = m^2 + Gamma^2 in the frequency and the horizontal
// group velocity at the centre and each face, K^2 = kh^2 + M2, and the
// Gamma^2 gradients weighed by d omega_hat / d Gamma^2 =
// -(kh^2 / (2 omega_hat K^2)) (N^2 - f^2) / K^2.
template <bool SPH, bool GAM>
__device__ inline void rhs(const G32 &g, const Bg32P &b, int ic, int jc, int kc, float2 lat, const float *Y,
                           float *F, const WBox &w)
{
    const float xi = Y[0], eta = Y[1], zeta = Y[2], k = Y[3], l = Y[4], m = Y[5];
    const float kh2 = k * k + l * l;
    const float m2 = m * m;
    const Axis ax = axis_per(ic, xi, g.nx), ay = axis_y(g, jc, eta), az = axis_clamp(kc, zeta, g.nz);
    const Cell c = cell_of(g, ax, ay, az);
    float4 Gc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (GAM) Gc = tri4<1>(b.Gm, c, 0);
    const float M2 = GAM ? m2 + Gc.x : m2;
    const float K2 = kh2 + M2;
    const float invK2 = rcp(K2);
    const float invK4 = invK2 * invK2;
    const float f2c = row_lerp(b.f2, ay);
    float gk, gl, gm, N2c;
    {
        Corners<1> KA;
        corners_A(g, w, b, ax, ay, az, c, KA);
        float4 A0;  // U V N2 Ux
        A0.x = TRI_COMP(KA, x, c);
        A0.y = TRI_COMP(KA, y, c);
        A0.z = TRI_COMP(KA, z, c);
        A0.w = TRI_COMP(KA, w, c);
        N2c = A0.z;
        const float rom = rsq((N2c * kh2 + f2c * M2) * invK2);  // 1 / omega_hat
        const float h = 0.5f * invK2 * rom;
        const float q = kh2 * h;
        const float qf = M2 * h;
        gk = k * A0.w;
        gl = qf * row_lerp(b.f2y, ay);
        gm = 0.0f;
        if (GAM) {
            const float qg = -(q * (N2c - f2c) * invK2);
            gk += qg * Gc.y;
            gl += qg * Gc.z;
            gm += qg * Gc.w;
        }
        // gradient records one at a time (bounded register use)
#pragma unroll 1
        for (int r = 0; r < 2; r++) {
            Corners<2> KG;
            corners_G(g, w, b, ax, ay, az, c, r, KG);
            float4 Gr;
            Gr.x = TRI_COMP(KG, x, c);
            Gr.y = TRI_COMP(KG, y, c);
            Gr.z = TRI_COMP(KG, z, c);
            Gr.w = TRI_COMP(KG, w, c);
            if (r == 0) {  // Uy Uz Vx Vy
                gl += k * Gr.x + l * Gr.w;
                gm += k * Gr.y;
                gk += l * Gr.z;
            } else {  // Vz N2x N2y N2z
                gm += l * Gr.x + q * Gr.w;
                gk += q * Gr.y;
                gl += q * Gr.z;
            }
        }
    }
    // faces +x, -x, +y, -y, +z, -z, one at a time (bounded register use)
    const float sdz = Y[8] * g.inv_dz;
    float cxp = 0.0f, cxm = 0.0f, cyp = 0.0f, cym = 0.0f, czp = 0.0f, czm = 0.0f;
#pragma unroll 1
    for (int fc = 0; fc < 6; fc++) {
        const int axn = fc >> 1;
        const float sg = (fc & 1) ? -0.5f : 0.5f;
        Axis fx = ax, fy = ay, fz = az;
        if (axn == 0)
            fx = axis_per(ic, xi + sg * Y[6], g.nx);
        else if (axn == 1)
            fy = axis_y(g, jc, eta + sg * Y[7]);
        else
            fz = axis_clamp(kc, zeta + sg * sdz, g.nz);
        const Cell f = cell_of(g, fx, fy, fz);
        Corners<1> K;
        corners_A(g, w, b, fx, fy, fz, f, K);
        // wind component along the face normal: U on x faces, V on y faces
        const bool useU = axn == 0;
        const float wnd = lerp3(useU ? K.a0.x : K.a0.y, useU ? K.a1.x : K.a1.y, useU ? K.b0.x : K.b0.y,
                                useU ? K.b1.x : K.b1.y, useU ? K.d0.x : K.d0.y, useU ? K.d1.x : K.d1.y,
                                useU ? K.e0.x : K.e0.y, useU ? K.e1.x : K.e1.y, f);
        const float N2f = TRI_COMP(K, z, f);
        const float f2f = axn == 1 ? row_lerp(b.f2, fy) : f2c;
        const float M2f = GAM ? m2 + gam2(b, f) : M2;
        const float invK2f = GAM ? rcp(kh2 + M2f) : invK2;
        const float invK4f = GAM ? invK2f * invK2f : invK4;
        const float romf = rsq((N2f * kh2 + f2f * M2f) * invK2f);
        const float sc = (N2f - f2f) * invK4f * romf;
        const float v = axn == 0 ? wnd + k * M2f * sc : (axn == 1 ? wnd + l * M2f * sc : -m * kh2 * sc);
        cxp = fc == 0 ? v : cxp;
        cxm = fc == 1 ? v : cxm;
        cyp = fc == 2 ? v : cyp;
        cym = fc == 3 ? v : cym;
        czp = fc == 4 ? v : czp;
        czm = fc == 5 ? v : czm;
    }
    assemble<SPH>(g, kc, lat, Y, gk, gl, gm, cxp + cxm, 0.5f * (cxp - cxm), cyp + cym, 0.5f * (cyp - cym), czp + czm,
                  0.5f * (czp - czm), F);
}

// move a periodic (cell, offset) pair back to offset in [0, 1)
__device__ inline void renorm_periodic(int &ic, float &u, int n)
{
    const float fl = floorf(u);
    int ii = ic + (int)fl;
    u = u - fl;
    if (u >= 1.0f) {
        u = 0.0f;
        ii += 1;
    }
    if (ii < 0 || ii >= n) {
        ii %= n;
        if (ii < 0) ii += n;
    }
    ic = ii;
}

}  // namespace f32

using f32::G32;
