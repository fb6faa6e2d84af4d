// Single-precision RK3 step of every active ray volume (Appendix B:
// Williamson's low-storage third-order scheme; Section 3a), followed by the
// post-step wrap, removal and column key.  One thread per volume, volumes
// read through the previous sort's permutation and written in sorted order.
// Each wave takes up to 64 consecutive volumes of one column (a column of n
// volumes has ceil(n / 64) waves of its own, from the wave table built with
// the column offsets), so every wave first stages the background stencil its volumes
// share into LDS (see f32.h); its interpolations then read LDS.
#include "f32.h"

// one wave per workgroup: a workgroup's slot and stencil box are released as
// soon as its wave ends, whatever the other waves' loads
#define STEP_BLOCK 64

template <bool SPH, bool GAM>
__global__ __launch_bounds__(STEP_BLOCK, GAM ? 4 : 5) void k_step32(G32 g, Bg32P b, S32 src, S32 dst,
                                                          const uint32_t *__restrict__ perm,
                                                          uint32_t *__restrict__ key_out,
                                                          const uint32_t *__restrict__ colstart,
                                                          const uint32_t *__restrict__ wcol, float dt,
                                                          const uint8_t *__restrict__ frozen,
                                                          const uint32_t *__restrict__ skeys)
{
    // this wave's column and its chunk of the column's sorted positions (the
    // grid is an upper bound of the waves; waves past the last column's and
    // the gaps between columns exit here).  32-bit volume indices (the
    // single-precision path holds fewer than 2^30 volumes): 4-byte fields are
    // read and written at 32-bit byte offsets from their uniform bases, which
    // keeps one register per index live
    const uint32_t wv = (uint32_t)xcd_block(gridDim.x);
    if (wv >= (uint32_t)g.ncol + colstart[g.ncol] / 64u) return;
    const uint32_t cw = wcol[wv];
    if (cw == 0xffffffffu) return;
    const uint32_t i = colstart[cw] + 64u * (wv - cw - colstart[cw] / 64u) + threadIdx.x;
    // stage the stencil box shared by the wave's volumes (all lanes take part:
    // the wave-wide reductions need every lane)
    const bool valid = i < colstart[cw + 1];
    const uint32_t s = valid ? f32::at(perm, i) : 0u;
    // every volume of the wave lies in column cw (a volume's stored column is
    // its sort key)
    const int kc0 = valid ? f32::at(src.lev, s) : 0;
    // the state's loads are in flight during the staging; m is carried in
    // double (md) and rounded to single precision for each stage's arithmetic
    float Y[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double md = 0.0;
    if (valid) {
        Y[0] = f32::at(src.xi, s);
        Y[1] = f32::at(src.eta, s);
        Y[2] = f32::at(src.zeta, s);
        Y[3] = f32::at(src.k, s);
        Y[4] = f32::at(src.l, s);
        md = src.m[s];
        Y[5] = (float)md;
        Y[6] = f32::at(src.dxi, s);
        Y[7] = f32::at(src.deta, s);
        Y[8] = f32::at(src.dz, s);
    }
    f32::WBox w;
    {
        const int lane = threadIdx.x & 63;
        const int kmn = wave_min_i(valid ? kc0 : 0x7fffffff), kmx = wave_max_i(valid ? kc0 : -1);
        w.base = 0;
        w.ic = (int)(cw % (uint32_t)g.nx);
        w.jc = (int)(cw / (uint32_t)g.nx);
        // levels: margins of two levels below and three above the wave's
        // range hold the faces of most volumes (a lookup outside the box
        // reads global memory)
        w.kbase = max(0, kmn - 2);
        w.L = min(g.nz - 1, kmx + 3) - w.kbase + 1;
        // the gradient records serve the centre only: one level either side
        w.kbase_g = max(0, kmn - 1);
        w.LG = min(g.nz - 1, kmx + 1) - w.kbase_g + 1;
        // one wrap corrects a column or row index when the grid has at least two
        w.on = w.L <= WB_LMAX && w.LG <= WB_GMAX && g.nx >= 2 && (g.geometry != RT_CARTESIAN || g.ny >= 2);
        if (w.on) {
            // a lane keeps one box column (and gradient record) and a phase
            // of its levels: A records by 50 lanes (25 columns x 2 phases,
            // levels ph, ph + 2, ...), gradient records by 54 lanes (9
            // columns x 2 records x 3 phases, levels ph, ph + 3, ...); the
            // column is located once, the levels are constant offsets, and
            // all loads are issued before the LDS writes
            constexpr int NA = (WB_LMAX + 1) / 2, NG = (WB_GMAX + 2) / 3;
            const int ca = lane % 25, pa = lane / 25;  // pa: 0, 1 (2 idle)
            const int gg = lane % 18, pg = lane / 18;  // pg: 0 .. 2 (3 idle)
            const int rg = gg / 9, cg = gg % 9;
            int ia = w.ic + ca % 5 - 2, ja = w.jc + ca / 5 - 2;
            int ig = w.ic + cg % 3 - 1, jg = w.jc + cg / 3 - 1;
            ia += ia < 0 ? g.nx : 0;
            ia -= ia >= g.nx ? g.nx : 0;
            ig += ig < 0 ? g.nx : 0;
            ig -= ig >= g.nx ? g.nx : 0;
            if (g.geometry == RT_CARTESIAN) {
                ja += ja < 0 ? g.ny : 0;
                ja -= ja >= g.ny ? g.ny : 0;
                jg += jg < 0 ? g.ny : 0;
                jg -= jg >= g.ny ? g.ny : 0;
            } else {
                ja = min(max(ja, 0), g.ny - 1);
                jg = min(max(jg, 0), g.ny - 1);
            }
            const uint32_t ka = f32::col_base(g, ja, ia) + (uint32_t)(w.kbase + pa);
            const uint32_t kg = (f32::col_base(g, jg, ig) + (uint32_t)(w.kbase_g + pg)) * 2u + (uint32_t)rg;
            float4 va[NA], vg[NG];
#pragma unroll
            for (int t = 0; t < NA; t++)
                if (pa < 2 && pa + 2 * t < w.L) va[t] = f32::rec(b.A, ka + 2u * t);
#pragma unroll
            for (int t = 0; t < NG; t++)
                if (pg < 3 && pg + 3 * t < w.LG) vg[t] = f32::rec(b.G, kg + 6u * t);
#pragma unroll
            for (int t = 0; t < NA; t++)
                if (pa < 2 && pa + 2 * t < w.L) f32::wb_lds[ca * WB_LMAX + pa + 2 * t] = va[t];
            if (GAM) {
                // the Gamma^2 records of the same cells, in the same layout
                float4 vm[NA];
#pragma unroll
                for (int t = 0; t < NA; t++)
                    if (pa < 2 && pa + 2 * t < w.L) vm[t] = f32::rec(b.Gm, ka + 2u * t);
#pragma unroll
                for (int t = 0; t < NA; t++)
                    if (pa < 2 && pa + 2 * t < w.L) f32::wb_lds[WB_GM + ca * WB_LMAX + pa + 2 * t] = vm[t];
            }
#pragma unroll
            for (int t = 0; t < NG; t++)
                if (pg < 3 && pg + 3 * t < w.LG) f32::wb_lds[WB_A + rg * 9 * WB_GMAX + cg * WB_GMAX + pg + 3 * t] = vg[t];
            // f2 and (f2)_y of the five box rows
            if (lane < 5) {
                int jj = w.jc + lane - 2;
                if (g.geometry == RT_CARTESIAN) {
                    jj += jj < 0 ? g.ny : 0;
                    jj -= jj >= g.ny ? g.ny : 0;
                } else {
                    jj = min(max(jj, 0), g.ny - 1);
                }
                f32::wb_lds[WB_F2 + lane] = make_float4(b.f2[jj], b.f2y[jj], 0.0f, 0.0f);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    if (!valid) return;
    int ic = w.ic, jc = w.jc;
    float Q[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    float F[9];
    const float A[3] = {0.0f, -5.0f / 9.0f, -153.0f / 128.0f};
    const float B[3] = {1.0f / 3.0f, 15.0f / 16.0f, 8.0f / 15.0f};
    const float phi0 = g.y0 + (float)jc * g.dyr;
    float2 lat = make_float2(0.0f, 1.0f);
    if (SPH) sincosf(phi0, &lat.x, &lat.y);
    // volumes in columns handed to the surrogate keep their state this step
    const int nst = (frozen && frozen[f32::at(skeys, i)]) ? 0 : 3;
#pragma unroll 1
    for (int st = 0; st < nst; st++) {
        // a stage whose lookups all lie in the box, for every lane, runs the
        // box-only form; otherwise each lookup tests the box itself
        if (w.on && __ballot(!f32::box_stage_in(g, w, kc0, Y)) == 0ull)
            f32::rhs_box<SPH, GAM>(g, kc0, lat, Y, F, w);
        else
            f32::rhs<SPH, GAM>(g, b, ic, jc, kc0, lat, Y, F, w);
#pragma unroll
        for (int c = 0; c < 9; c++) {
            Q[c] = A[st] * Q[c] + dt * F[c];
            if (c == 5) {
                // the running sum of m in double: its single-precision
                // rounding at every stage would cost the drag more accuracy
                // than everything else in the step together
                md = md + (double)(B[st] * Q[5]);
                Y[5] = (float)md;
            } else {
                Y[c] = Y[c] + B[st] * Q[c];
            }
        }
    }
    // the wave action is carried with the state (the deposition streams it);
    // px, py, pz and id stay at their home slot, which is passed on; the
    // column of an active volume is its key
    const double cW = src.W[s];
    const uint32_t chm = src.hm ? f32::at(src.hm, s) : s;
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
    // the carrier background of the new state, for the deposition
    if (key < (uint32_t)g.ncol) {
        float cn2, cf2;
        f32::n2_f2_carrier(g, b, w, ic, jc, kc, Y[0], Y[1], Y[2], cn2, cf2);
        f32::put(dst.cn2, i, cn2);
        f32::put(dst.cf2, i, cf2);
        if (GAM) f32::put(dst.cg2, i, f32::gam2_at(g, b, ic, jc, kc, Y[0], Y[1], Y[2]));
    }
    f32::put(dst.lev, i, kc);
    f32::put(dst.xi, i, Y[0]);
    f32::put(dst.eta, i, Y[1]);
    f32::put(dst.zeta, i, Y[2]);
    f32::put(dst.k, i, Y[3]);
    f32::put(dst.l, i, Y[4]);
    dst.m[i] = md;
    f32::put(dst.dxi, i, Y[6]);
    f32::put(dst.deta, i, Y[7]);
    f32::put(dst.dz, i, Y[8]);
    dst.W[i] = cW;
    f32::put(dst.hm, i, chm);
    f32::put(key_out, i, key);
}

void launch_step32(const Grid &g, const Bg32P &b, S32 src, S32 dst, const uint32_t *perm, uint32_t *key_out,
                   const uint32_t *colstart, const uint32_t *wcol, int64_t bound, double dt,
                   const uint8_t *frozen, const uint32_t *skeys, hipStream_t s)
{
    if (bound <= 0) return;
    const unsigned nb = (unsigned)wave_table_len(bound, g.ncol);  // an upper bound of the waves
    const G32 h = f32::make_g32(g);
    const bool sph = g.geometry == RT_SPHERICAL, gam = b.Gm != nullptr;
    const size_t lds = (size_t)(gam ? WB_RECS_GAM : WB_RECS) * sizeof(float4);  // the wave's stencil box
    if (sph && gam)
        k_step32<true, true><<<nb, STEP_BLOCK, lds, s>>>(h, b, src, dst, perm, key_out, colstart, wcol, (float)dt,
                                                         frozen, skeys);
    else if (sph)
        k_step32<true, false><<<nb, STEP_BLOCK, lds, s>>>(h, b, src, dst, perm, key_out, colstart, wcol, (float)dt,
                                                          frozen, skeys);
    else if (gam)
        k_step32<false, true><<<nb, STEP_BLOCK, lds, s>>>(h, b, src, dst, perm, key_out, colstart, wcol, (float)dt,
                                                          frozen, skeys);
    else
        k_step32<false, false><<<nb, STEP_BLOCK, lds, s>>>(h, b, src, dst, perm, key_out, colstart, wcol,
                                                           (float)dt, frozen, skeys);
}
