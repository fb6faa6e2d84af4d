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

// periodic axis: base cell ic, offset u in cell units
__device__ inline void axis_per(int ic, float u, int n, int &i0, int &i1, float &w)
{
    const float t = u - 0.5f;
    if (!(fabsf(t) < 1.0e6f)) {
        i0 = 0;
        i1 = 0;
        w = t - t;
        return;
    }
    const float fl = floorf(t);
    w = t - fl;
    int ii = ic + (int)fl;
    if (ii < 0 || ii >= n) {
        ii %= n;
        if (ii < 0) ii += n;
    }
    i0 = ii;
    i1 = (ii + 1 == n) ? 0 : ii + 1;
}

// clamped axis (latitude rows, levels): value held beyond the end centres
__device__ inline void axis_clamp(int ic, float u, int n, int &i0, int &i1, float &w)
{
    const float t = u - 0.5f;
    if (!(fabsf(t) < 1.0e6f)) {
        i0 = 0;
        i1 = 0;
        w = t - t;
        return;
    }
    const float fl = floorf(t);
    const int j0 = ic + (int)fl;
    if (j0 < 0) {
        i0 = 0;
        i1 = 0;
        w = 0.0f;
    } else if (j0 >= n - 1) {
        i0 = n - 1;
        i1 = n - 1;
        w = 0.0f;
    } else {
        i0 = j0;
        i1 = j0 + 1;
        w = t - fl;
    }
}

struct Cell {
    int c00, c01, c10, c11;  // columns (j0,i0) (j0,i1) (j1,i0) (j1,i1), times nz
    int k0, k1;
    float wx, wy, wz;
};

__device__ inline void locate(const G32 &g, int ic, int jc, int kc, float xi, float eta, float zeta, Cell &c)
{
    int i0, i1, j0, j1;
    axis_per(ic, xi, g.nx, i0, i1, c.wx);
    if (g.geometry == RT_CARTESIAN)
        axis_per(jc, eta, g.ny, j0, j1, c.wy);
    else
        axis_clamp(jc, eta, g.ny, j0, j1, c.wy);
    axis_clamp(kc, zeta, g.nz, c.k0, c.k1, c.wz);
    c.c00 = (j0 * g.nx + i0) * g.nz;
    c.c01 = (j0 * g.nx + i1) * g.nz;
    c.c10 = (j1 * g.nx + i0) * g.nz;
    c.c11 = (j1 * g.nx + i1) * g.nz;
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

// trilinear interpolation of a packed float4 record (R records per cell)
template <int R>
__device__ inline float4 tri4(const float4 *__restrict__ F, const Cell &c, int r)
{
    const float4 a0 = F[(c.c00 + c.k0) * R + r], a1 = F[(c.c01 + c.k0) * R + r];
    const float4 b0 = F[(c.c10 + c.k0) * R + r], b1 = F[(c.c11 + c.k0) * R + r];
    const float4 d0 = F[(c.c00 + c.k1) * R + r], d1 = F[(c.c01 + c.k1) * R + r];
    const float4 e0 = F[(c.c10 + c.k1) * R + r], e1 = F[(c.c11 + c.k1) * R + r];
    float4 o;
    o.x = lerp3(a0.x, a1.x, b0.x, b1.x, d0.x, d1.x, e0.x, e1.x, c);
    o.y = lerp3(a0.y, a1.y, b0.y, b1.y, d0.y, d1.y, e0.y, e1.y, c);
    o.z = lerp3(a0.z, a1.z, b0.z, b1.z, d0.z, d1.z, e0.z, e1.z, c);
    o.w = lerp3(a0.w, a1.w, b0.w, b1.w, d0.w, d1.w, e0.w, e1.w, c);
    return o;
}

// group velocity component along one axis at a face: background wind (if
// any) plus the intrinsic part from the dispersion relation
__device__ inline float face_cg(const BgP<float> &b, const Cell &f, int axis, float k, float l, float m, float kh2,
                                float m2, float invK2, float invK4)
{
    const float4 A = tri4<1>(b.A, f, 0);
    const float om = sqrtf((A.z * kh2 + A.w * m2) * invK2);
    const float s = (A.z - A.w) * invK4 / om;
    if (axis == 0) return A.x + k * m2 * s;
    if (axis == 1) return A.y + l * m2 * s;
    return -m * kh2 * s;
}

// RK stage right-hand side in cell units: Y = (xi, eta, zeta, k, l, m, Dxi,
// Deta, Dz), offsets relative to the base cell (ic, jc, kc), Dz in metres
template <bool SPH>
__device__ inline void rhs(const G32 &g, const BgP<float> &b, int ic, int jc, int kc, float phi0, const float *Y,
                           float *F)
{
    const float xi = Y[0], eta = Y[1], zeta = Y[2], k = Y[3], l = Y[4], m = Y[5];
    const float kh2 = k * k + l * l;
    const float m2 = m * m;
    const float K2 = kh2 + m2;
    const float invK2 = 1.0f / K2;
    const float invK4 = invK2 * invK2;
    Cell c;
    locate(g, ic, jc, kc, xi, eta, zeta, c);
    const float4 Ac = tri4<1>(b.A, c, 0);  // U V N2 f2
    const float om = sqrtf((Ac.z * kh2 + Ac.w * m2) * invK2);
    const float h = 0.5f * invK2 / om;
    const float q = kh2 * h;
    const float qf = m2 * h;
    // gradient records one at a time: (Ux Uy Uz Vx) (Vy Vz N2x N2y) (N2z f2y)
    float gk = 0.0f, gl = 0.0f, gm = 0.0f;
#pragma unroll 1
    for (int r = 0; r < 3; r++) {
        const float4 Gr = tri4<3>(b.G, c, r);
        // r=0: k*Ux -> gk, k*Uy -> gl, k*Uz -> gm, l*Vx -> gk
        // r=1: l*Vy -> gl, l*Vz -> gm, q*N2x -> gk, q*N2y -> gl
        // r=2: q*N2z -> gm, qf*f2y -> gl
        if (r == 0) {
            gk += k * Gr.x + l * Gr.w;
            gl += k * Gr.y;
            gm += k * Gr.z;
        } else if (r == 1) {
            gl += l * Gr.x + q * Gr.w;
            gm += l * Gr.y;
            gk += q * Gr.z;
        } else {
            gm += q * Gr.x;
            gl += qf * Gr.y;
        }
    }
    // faces +x, -x, +y, -y, +z, -z, one at a time (bounded register use)
    float cxp = 0.0f, cxm = 0.0f, cyp = 0.0f, cym = 0.0f, czp = 0.0f, czm = 0.0f;
#pragma unroll 1
    for (int fc = 0; fc < 6; fc++) {
        const int ax = fc >> 1;
        const float sg = (fc & 1) ? -0.5f : 0.5f;
        float px = xi, py = eta, pz = zeta;
        if (ax == 0)
            px += sg * Y[6];
        else if (ax == 1)
            py += sg * Y[7];
        else
            pz += sg * (Y[8] * g.inv_dz);
        Cell f;
        locate(g, ic, jc, kc, px, py, pz, f);
        const float4 A = tri4<1>(b.A, f, 0);
        const float omf = sqrtf((A.z * kh2 + A.w * m2) * invK2);
        const float sc = (A.z - A.w) * invK4 / omf;
        const float v = ax == 0 ? A.x + k * m2 * sc : (ax == 1 ? A.y + l * m2 * sc : -m * kh2 * sc);
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
        const float ir = 1.0f / r;
        float sphi, cphi;
        sincosf(phi0 + eta * g.dyr, &sphi, &cphi);
        const float tphi = sphi / cphi;
        const float irc = ir / cphi;
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
__global__ __launch_bounds__(256, 2) void k_step32(G32 g, BgP<float> b, S32 src, S32 dst, const uint32_t *__restrict__ perm,
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

void launch_step32(const Grid &g, const BgP<float> &b, S32 src, S32 dst, const uint32_t *perm, uint32_t *key_out,
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
    BgP<float> b;
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
        f32::Cell c;
        f32::locate(g, ic, jc, kc, st.xi[s], st.eta[s], zeta, c);
        const float4 Ac = f32::tri4<1>(b.A, c, 0);
        const float N2 = Ac.z;
        const float f2 = Ac.w;
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
        f32::Cell c;
        f32::locate(g, ic, jc, st.lev[s], st.xi[s], st.eta[s], st.zeta[s], c);
        const float4 Ac = f32::tri4<1>(b.A, c, 0);
        const float k = st.k[s], l = st.l[s], m = st.m[s];
        const float kh2 = k * k + l * l;
        const float m2 = m * m;
        const float K2 = kh2 + m2;
        const float om = sqrtf((Ac.z * kh2 + Ac.w * m2) / K2);
        const float sc = (Ac.z - Ac.w) / (K2 * K2) / om;
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

void launch_deposit32(const Grid &g, const BgP<float> &b, S32 st, const uint32_t *perm, const uint32_t *colstart,
                      double *flux, hipStream_t s)
{
    Pay32 p{f32::make_g32(g), b, st, g.dz};
    k_deposit<Pay32><<<(unsigned)g.ncol, 256, deposit_smem(g), s>>>(g, p, perm, colstart, flux);
}

void launch_features32(const Grid &g, const BgP<float> &b, S32 st, const uint32_t *perm, const uint32_t *colstart,
                       float *X, hipStream_t s)
{
    Pay32 p{f32::make_g32(g), b, st, g.dz};
    k_features<Pay32><<<(unsigned)g.ncol, 256, 0, s>>>(g, p, perm, colstart, X);
}
