// Single-precision kernels: RK3 step on the FP32 state, load/store between the
// double-precision interface and the FP32 layout, removal tallies,
// diagnostics and the deposition payload.
//
// FP32 layout.  A horizontal position is held as the index of its column plus
// an offset in cell units, and the height as the index of its level plus an
// offset in level units, so the resolution is a fixed fraction of a cell
// (about 1e-7 cell) everywhere in the domain instead of degrading with the
// distance from the origin; this keeps the column assignment and the
// vertical overlaps of the FP32 path as sharp as the FP64 ones.  Extents
// Dx, Dy are in cell units, Dz in metres.  The
// wave action W = N Px Py Pz is formed once in double at load and kept in
// double, and every flux sum is accumulated in double.
#include "dev64.h"
#include "deposit_common.h"
#include "features_common.h"

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
    __device__ inline Corners(const float4 *__restrict__ F, const Cell &c, int r)
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
    const float a = f[y.i0], b = f[y.i1];
    return a + y.w * (b - a);
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

// RK stage right-hand side in cell units: Y = (xi, eta, zeta, k, l, m, Dxi,
// Deta, Dz), offsets relative to the base cell (ic, jc, kc), Dz in metres.
// Centre: 12 fields from three records per corner (U V N2 Ux | Uy Uz Vx Vy |
// Vz N2x N2y N2z) plus f2 and (f2)_y by row.  Faces: (U or V) and N2 from the
// first record; the face differs from the centre along one axis only, so the
// other two axes are reused, and f2 is the centre's except on the y faces.
template <bool SPH>
__device__ inline void rhs(const G32 &g, const Bg32P &b, int ic, int jc, int kc, float phi0, const float *Y, float *F)
{
    const float xi = Y[0], eta = Y[1], zeta = Y[2], k = Y[3], l = Y[4], m = Y[5];
    const float kh2 = k * k + l * l;
    const float m2 = m * m;
    const float K2 = kh2 + m2;
    const float invK2 = rcp(K2);
    const float invK4 = invK2 * invK2;
    const Axis ax = axis_per(ic, xi, g.nx), ay = axis_y(g, jc, eta), az = axis_clamp(kc, zeta, g.nz);
    const Cell c = cell_of(g, ax, ay, az);
    const float f2c = row_lerp(b.f2, ay);
    float gk, gl, gm, N2c;
    {
        const float4 A0 = tri4<1>(b.A, c, 0);  // U V N2 Ux
        N2c = A0.z;
        const float rom = rsq((N2c * kh2 + f2c * m2) * invK2);  // 1 / omega_hat
        const float h = 0.5f * invK2 * rom;
        const float q = kh2 * h;
        const float qf = m2 * h;
        gk = k * A0.w;
        gl = qf * row_lerp(b.f2y, ay);
        gm = 0.0f;
        // gradient records one at a time (bounded register use)
#pragma unroll 1
        for (int r = 0; r < 2; r++) {
            const float4 Gr = tri4<2>(b.G, c, r);
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
        const Corners<1> K(b.A, f, 0);
        // wind component along the face normal: U on x faces, V on y faces
        const bool useU = axn == 0;
        const float wnd = lerp3(useU ? K.a0.x : K.a0.y, useU ? K.a1.x : K.a1.y, useU ? K.b0.x : K.b0.y,
                                useU ? K.b1.x : K.b1.y, useU ? K.d0.x : K.d0.y, useU ? K.d1.x : K.d1.y,
                                useU ? K.e0.x : K.e0.y, useU ? K.e1.x : K.e1.y, f);
        const float N2f = TRI_COMP(K, z, f);
        const float f2f = axn == 1 ? row_lerp(b.f2, fy) : f2c;
        const float romf = rsq((N2f * kh2 + f2f * m2) * invK2);
        const float sc = (N2f - f2f) * invK4 * romf;
        const float v = axn == 0 ? wnd + k * m2 * sc : (axn == 1 ? wnd + l * m2 * sc : -m * kh2 * sc);
        cxp = fc == 0 ? v : cxp;
        cxm = fc == 1 ? v : cxm;
        cyp = fc == 2 ? v : cyp;
        cym = fc == 3 ? v : cym;
        czp = fc == 4 ? v : czp;
        czm = fc == 5 ? v : czm;
    }
    if (!SPH) {
        F[0] = 0.5f * (cxp + cxm) * g.inv_dx;
        F[1] = 0.5f * (cyp + cym) * g.inv_dy;
        F[2] = 0.5f * (czp + czm) * g.inv_dz;
        F[3] = -gk;
        F[4] = -gl;
        F[5] = -gm;
        F[6] = (cxp - cxm) * g.inv_dx;
        F[7] = (cyp - cym) * g.inv_dy;
        F[8] = czp - czm;
    } else {
        const float r = g.a + ((float)kc + zeta) * g.dz;
        const float ir = rcp(r);
        float sphi, cphi;
        sincosf(phi0 + eta * g.dyr, &sphi, &cphi);
        const float icphi = rcp(cphi);
        const float tphi = sphi * icphi;
        const float irc = ir * icphi;
        const float uc = 0.5f * (cxp + cxm);
        const float vc = 0.5f * (cyp + cym);
        const float wc = 0.5f * (czp + czm);
        F[0] = uc * irc * g.inv_dx;
        F[1] = vc * ir * g.inv_dy;
        F[2] = wc * g.inv_dz;
        F[3] = -gk * irc - k * wc * ir + k * tphi * vc * ir;
        F[4] = -gl * ir - l * wc * ir - k * tphi * uc * ir;
        F[5] = -gm + k * uc * ir + l * vc * ir;
        F[6] = (cxp - cxm) * irc * g.inv_dx;
        F[7] = (cyp - cym) * ir * g.inv_dy;
        F[8] = czp - czm;
    }
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

template <bool SPH>
__global__ __launch_bounds__(256, 5) void k_step32(G32 g, Bg32P b, S32 src, S32 dst, const uint32_t *__restrict__ perm,
                                                   uint32_t *__restrict__ key_out, const DevCounters *__restrict__ dc,
                                                   float dt, const uint8_t *__restrict__ frozen,
                                                   const uint32_t *__restrict__ skeys)
{
    const int64_t i = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= dc->n_active) return;
    const uint32_t s = perm[i];
    const uint32_t col = src.col[s];
    int ic = (int)(col % (uint32_t)g.nx), jc = (int)(col / (uint32_t)g.nx);
    const int kc0 = src.lev[s];
    float Y[9] = {src.xi[s], src.eta[s], src.zeta[s], src.k[s], src.l[s], src.m[s], src.dxi[s], src.deta[s], src.dz[s]};
    float Q[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    float F[9];
    const float A[3] = {0.0f, -5.0f / 9.0f, -153.0f / 128.0f};
    const float B[3] = {1.0f / 3.0f, 15.0f / 16.0f, 8.0f / 15.0f};
    const float phi0 = g.y0 + (float)jc * g.dyr;
    // volumes in columns handed to the surrogate keep their state this step
    const int nst = (frozen && frozen[skeys[i]]) ? 0 : 3;
#pragma unroll 1
    for (int st = 0; st < nst; st++) {
        f32::rhs<SPH>(g, b, ic, jc, kc0, phi0, Y, F);
#pragma unroll
        for (int c = 0; c < 9; c++) {
            Q[c] = A[st] * Q[c] + dt * F[c];
            Y[c] = Y[c] + B[st] * Q[c];
        }
    }
    // post-step: validity, wrap, removal, column key
    uint32_t key;
    int kc = kc0;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 9; c++) ok = ok && isfinite(Y[c]);
    ok = ok && Y[6] > 0.0f && Y[7] > 0.0f && Y[8] > 0.0f && (Y[3] * Y[3] + Y[4] * Y[4] + Y[5] * Y[5]) > 0.0f;
    ok = ok && fabsf(Y[0]) < 1.0e6f && fabsf(Y[1]) < 1.0e6f && fabsf(Y[2]) < 1.0e6f;
    if (!ok) {
        key = (uint32_t)(g.ncol + RK_INVALID);
    } else {
        f32::renorm_periodic(ic, Y[0], g.nx);
        key = 0;
        if (SPH) {
            const float phi = phi0 + Y[1] * g.dyr;
            if (fabsf(phi) >= g.pole) key = (uint32_t)(g.ncol + RK_POLE);
            const float fl = floorf(Y[1]);
            int jj = jc + (int)fl;
            Y[1] = Y[1] - fl;
            if (Y[1] >= 1.0f) {
                Y[1] = 0.0f;
                jj += 1;
            }
            if (jj < 0) {
                jj = 0;
                Y[1] = 0.0f;
            }
            if (jj > g.ny - 1) {
                jj = g.ny - 1;
                Y[1] = 0.999999940395f;
            }
            jc = jj;
        } else {
            f32::renorm_periodic(jc, Y[1], g.ny);
        }
        {
            // level index + offset in [0, 1)
            const float fl = floorf(Y[2]);
            kc = kc0 + (int)fl;
            Y[2] = Y[2] - fl;
            if (Y[2] >= 1.0f) {
                Y[2] = 0.0f;
                kc += 1;
            }
        }
        if (key == 0) {
            if (kc < 0)
                key = (uint32_t)(g.ncol + RK_BOTTOM);
            else if (kc > g.nz || (kc == g.nz && Y[2] > 0.0f))
                key = (uint32_t)(g.ncol + RK_TOP);
            else
                key = (uint32_t)(jc * g.nx + ic);
        }
    }
    dst.col[i] = (uint32_t)(jc * g.nx + ic);
    dst.lev[i] = kc;
    dst.xi[i] = Y[0];
    dst.eta[i] = Y[1];
    dst.zeta[i] = Y[2];
    dst.k[i] = Y[3];
    dst.l[i] = Y[4];
    dst.m[i] = Y[5];
    dst.dxi[i] = Y[6];
    dst.deta[i] = Y[7];
    dst.dz[i] = Y[8];
    dst.px[i] = src.px[s];
    dst.py[i] = src.py[s];
    dst.pz[i] = src.pz[s];
    dst.W[i] = src.W[s];
    dst.id[i] = src.id[s];
    key_out[i] = key;
}

void launch_step32(const Grid &g, const Bg32P &b, S32 src, S32 dst, const uint32_t *perm, uint32_t *key_out,
                   const DevCounters *dc, int64_t bound, double dt, const uint8_t *frozen, const uint32_t *skeys,
                   hipStream_t s)
{
    if (bound <= 0) return;
    const unsigned nb = (unsigned)((bound + 255) / 256);
    const G32 h = f32::make_g32(g);
    if (g.geometry == RT_SPHERICAL)
        k_step32<true><<<nb, 256, 0, s>>>(h, b, src, dst, perm, key_out, dc, (float)dt, frozen, skeys);
    else
        k_step32<false><<<nb, 256, 0, s>>>(h, b, src, dst, perm, key_out, dc, (float)dt, frozen, skeys);
}

// ---------------------------------------------------------------------------
// packed single-precision background: A = (U, V, N2, Ux),
// G = (Uy, Uz, Vx, Vy), (Vz, N2x, N2y, N2z) at index col*nz + k
// ---------------------------------------------------------------------------
__global__ void k_pack32(Grid g, Bg<double> b, float4 *A, float4 *G)
{
    const int64_t cells = (int64_t)g.ncol * g.nz;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cells) return;
    const int64_t col = e / g.nz, k = e % g.nz;
    const int64_t s = k * g.ncol + col;
    A[e] = make_float4((float)b.U[s], (float)b.V[s], (float)b.N2[s], (float)b.Ux[s]);
    G[2 * e] = make_float4((float)b.Uy[s], (float)b.Uz[s], (float)b.Vx[s], (float)b.Vy[s]);
    G[2 * e + 1] = make_float4((float)b.Vz[s], (float)b.N2x[s], (float)b.N2y[s], (float)b.N2z[s]);
}

void launch_pack32(const Grid &g, const Bg<double> &b, float4 *A, float4 *G, hipStream_t s)
{
    const int64_t cells = (int64_t)g.ncol * g.nz;
    k_pack32<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(g, b, A, G);
}

// ---------------------------------------------------------------------------
// conversions
// ---------------------------------------------------------------------------
__global__ void k_round32(const double *in, float *out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

void launch_round32(const double *in, float *out, int64_t n, hipStream_t s)
{
    if (n > 0) k_round32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(in, out, n);
}

__global__ void k_load32(Grid g, rt_rays in, int64_t n, S32 d, uint32_t *key)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double Y[9] = {in.x[i], in.y[i], in.z[i], in.k[i], in.l[i], in.m[i], in.dx[i], in.dy[i], in.dz[i]};
    const uint32_t kk = d64::post_step(g, Y);
    uint32_t col = 0;
    float xi = 0.0f, eta = 0.0f;
    if (kk < (uint32_t)g.ncol) {
        col = kk;
        const int ic = (int)(col % (uint32_t)g.nx), jc = (int)(col / (uint32_t)g.nx);
        xi = (float)((Y[0] - g.x0) / g.dx - (double)ic);
        eta = (float)((Y[1] - g.y0) / g.dy - (double)jc);
        if (xi >= 1.0f) xi = 0.99999994f;
        if (eta >= 1.0f) eta = 0.99999994f;
    }
    // height as level index + offset in level units
    const double gz = Y[2] / g.dz;
    double fk = floor(gz);
    if (!(fk >= 0.0)) fk = 0.0;
    if (fk > (double)g.nz) fk = (double)g.nz;
    float zeta = (float)(gz - fk);
    if (zeta >= 1.0f) zeta = 0.99999994f;
    d.col[i] = col;
    d.lev[i] = (int32_t)fk;
    d.xi[i] = xi;
    d.eta[i] = eta;
    d.zeta[i] = zeta;
    d.k[i] = (float)Y[3];
    d.l[i] = (float)Y[4];
    d.m[i] = (float)Y[5];
    d.dxi[i] = (float)(Y[6] / g.dx);
    d.deta[i] = (float)(Y[7] / g.dy);
    d.dz[i] = (float)Y[8];
    d.px[i] = (float)in.px[i];
    d.py[i] = (float)in.py[i];
    d.pz[i] = (float)in.pz[i];
    d.W[i] = ((in.n[i] * in.px[i]) * in.py[i]) * in.pz[i];
    d.id[i] = in.id[i];
    key[i] = kk;
}

void launch_load32(const Grid &g, const rt_rays &in, int64_t n, S32 dst, uint32_t *key, hipStream_t s)
{
    if (n > 0) k_load32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g, in, n, dst, key);
}

__global__ void k_store32(Grid g, S32 st, const uint32_t *perm, const DevCounters *dc, rt_rays o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dc->n_active) return;
    const uint32_t s = perm[i];
    const uint32_t col = st.col[s];
    const int ic = (int)(col % (uint32_t)g.nx), jc = (int)(col / (uint32_t)g.nx);
    o.x[i] = g.x0 + ((double)ic + (double)st.xi[s]) * g.dx;
    o.y[i] = g.y0 + ((double)jc + (double)st.eta[s]) * g.dy;
    o.z[i] = ((double)st.lev[s] + (double)st.zeta[s]) * g.dz;
    o.k[i] = st.k[s];
    o.l[i] = st.l[s];
    o.m[i] = st.m[s];
    o.dx[i] = (double)st.dxi[s] * g.dx;
    o.dy[i] = (double)st.deta[s] * g.dy;
    o.dz[i] = st.dz[s];
    const double px = st.px[s], py = st.py[s], pz = st.pz[s];
    o.px[i] = px;
    o.py[i] = py;
    o.pz[i] = pz;
    o.n[i] = st.W[s] / ((px * py) * pz);
    o.id[i] = st.id[s];
}

void launch_store32(const Grid &g, S32 src, const uint32_t *perm, const DevCounters *dc, rt_rays out, int64_t bound,
                    hipStream_t s)
{
    if (bound > 0) k_store32<<<(unsigned)((bound + 255) / 256), 256, 0, s>>>(g, src, perm, dc, out);
}

// ---------------------------------------------------------------------------
// tallies and diagnostics (deterministic, see kern64.hip)
// ---------------------------------------------------------------------------
__global__ void k_tally32(Grid g, S32 st, const uint32_t *perm, const uint32_t *skeys, DevCounters *dc)
{
    __shared__ double sw[256];
    __shared__ int cnt[RK_NREASON];
    const int tid = threadIdx.x;
    if (tid < RK_NREASON) cnt[tid] = 0;
    __syncthreads();
    const int64_t a = dc->n_active, e = dc->n_sorted;
    double w = 0.0;
    for (int64_t i = a + tid; i < e; i += 256) {
        const int reason = (int)(skeys[i] - (uint32_t)g.ncol);
        if (reason >= 0 && reason < RK_NREASON) atomicAdd(&cnt[reason], 1);
        if (reason != RK_INVALID && reason != RK_MERGED) w += st.W[perm[i]];
    }
    sw[tid] = w;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) sw[tid] += sw[tid + off];
        __syncthreads();
    }
    if (tid == 0) dc->removed_W += sw[0];
    if (tid < RK_NREASON) dc->removed[tid] += cnt[tid];
}

void launch_tally32(const Grid &g, S32 st, const uint32_t *perm, const uint32_t *skeys, DevCounters *dc, double *red,
                    hipStream_t s)
{
    (void)red;
    k_tally32<<<1, 256, 0, s>>>(g, st, perm, skeys, dc);
}

__global__ void k_stats32_part(S32 st, const uint32_t *perm, const DevCounters *dc, double *part)
{
    __shared__ double sh[4][256];
    const int tid = threadIdx.x;
    const int64_t n = dc->n_active;
    const int64_t i = (int64_t)blockIdx.x * 256 + tid;
    double v[4] = {0, 0, 0, 0};
    if (i < n) {
        const uint32_t s = perm[i];
        const double W = st.W[s];
        v[0] = W;
        v[1] = (double)st.k[s] * W;
        v[2] = (double)st.l[s] * W;
        v[3] = (double)st.m[s] * W;
    }
    for (int q = 0; q < 4; q++) sh[q][tid] = v[q];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off)
            for (int q = 0; q < 4; q++) sh[q][tid] += sh[q][tid + off];
        __syncthreads();
    }
    if (tid < 4) part[4 + (int64_t)blockIdx.x * 4 + tid] = sh[tid][0];
}

__global__ void k_stats32_final(double *part, int64_t nblocks)
{
    __shared__ double sh[4][256];
    const int tid = threadIdx.x;
    double v[4] = {0, 0, 0, 0};
    for (int64_t b = tid; b < nblocks; b += 256)
        for (int q = 0; q < 4; q++) v[q] += part[4 + b * 4 + q];
    for (int q = 0; q < 4; q++) sh[q][tid] = v[q];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off)
            for (int q = 0; q < 4; q++) sh[q][tid] += sh[q][tid + off];
        __syncthreads();
    }
    if (tid < 4) part[tid] = sh[tid][0];
}

void launch_stats32(S32 st, const uint32_t *perm, const DevCounters *dc, double *red, int64_t bound, hipStream_t s)
{
    const int64_t nb = bound > 0 ? (bound + 255) / 256 : 0;
    if (nb > 0) k_stats32_part<<<(unsigned)nb, 256, 0, s>>>(st, perm, dc, red);
    k_stats32_final<<<1, 256, 0, s>>>(red, nb);
}

// ---------------------------------------------------------------------------
// deposition payload: single-precision dispersion at the carrier, wave action
// and the flux densities in double
// ---------------------------------------------------------------------------
struct Pay32 {
    G32 g;
    Bg32P b;
    S32 st;
    double zdz;  // level spacing in double
    __device__ void load(uint32_t s, double &zb, double &zt, double *bv) const
    {
        const uint32_t col = st.col[s];
        const int ic = (int)(col % (uint32_t)g.nx), jc = (int)(col / (uint32_t)g.nx);
        const int kc = st.lev[s];
        const float zeta = st.zeta[s];
        const float k = st.k[s], l = st.l[s], m = st.m[s];
        const float Dz = st.dz[s];
        float N2, f2;
        f32::n2_f2(g, b, ic, jc, kc, st.xi[s], st.eta[s], zeta, N2, f2);
        const float kh2 = k * k + l * l;
        const float m2 = m * m;
        const float K2 = kh2 + m2;
        const float om = sqrtf((N2 * kh2 + f2 * m2) / K2);
        const float sc = (N2 - f2) / (K2 * K2) / om;
        const double cx = (double)(k * m2 * sc);
        const double cy = (double)(l * m2 * sc);
        const double cz = (double)(-m * kh2 * sc);
        const double sW = st.W[s] / (double)Dz;
        const double kd = k, ld = l;
        bv[0] = (cx * kd) * sW;
        bv[1] = (cx * ld) * sW;
        bv[2] = (cy * kd) * sW;
        bv[3] = (cy * ld) * sW;
        bv[4] = (cz * kd) * sW;
        bv[5] = (cz * ld) * sW;
        const double zc = ((double)kc + (double)zeta) * zdz;
        zb = zc - 0.5 * (double)Dz;
        zt = zc + 0.5 * (double)Dz;
    }
    // spectral state, wave action and intrinsic vertical group velocity at
    // the carrier (surrogate features)
    __device__ void spec(uint32_t s, double &kd, double &ld, double &md, double &W, double &cgz, double &z) const
    {
        const uint32_t col = st.col[s];
        const int ic = (int)(col % (uint32_t)g.nx), jc = (int)(col / (uint32_t)g.nx);
        float N2, f2;
        f32::n2_f2(g, b, ic, jc, st.lev[s], st.xi[s], st.eta[s], st.zeta[s], N2, f2);
        const float k = st.k[s], l = st.l[s], m = st.m[s];
        const float kh2 = k * k + l * l;
        const float m2 = m * m;
        const float K2 = kh2 + m2;
        const float om = sqrtf((N2 * kh2 + f2 * m2) / K2);
        const float sc = (N2 - f2) / (K2 * K2) / om;
        kd = k;
        ld = l;
        md = m;
        W = st.W[s];
        cgz = (double)(-m * kh2 * sc);
        z = ((double)st.lev[s] + (double)st.zeta[s]) * zdz;
    }
    __device__ void profile(int col, int k, double &u, double &v, double &n2) const
    {
        const float4 a = b.A[(int64_t)col * g.nz + k];
        u = a.x;
        v = a.y;
        n2 = a.z;
    }
};

void launch_deposit32(const Grid &g, const Bg32P &b, S32 st, const uint32_t *perm, const uint32_t *colstart,
                      double *flux, hipStream_t s)
{
    Pay32 p{f32::make_g32(g), b, st, g.dz};
    launch_deposit_k(g, p, perm, colstart, flux, s);
}

void launch_features32(const Grid &g, const Bg32P &b, S32 st, const uint32_t *perm, const uint32_t *colstart,
                       float *X, hipStream_t s)
{
    Pay32 p{f32::make_g32(g), b, st, g.dz};
    k_features<Pay32><<<(unsigned)((g.ncol + 3) / 4), 256, 0, s>>>(g, p, perm, colstart, X);
}
