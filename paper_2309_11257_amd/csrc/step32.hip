// Single-precision RK3 step of every active ray volume (Appendix B:
// Williamson's low-storage third-order scheme; Section 3a), followed by the
// post-step wrap, removal and column key.  One thread per volume, volumes
// read through the previous sort's permutation and written in sorted order.
// A wave whose volumes share one column first stages the background stencil
// they all use into LDS (see f32.h); its interpolations then read LDS.
#include "f32.h"

// one wave per workgroup: a workgroup's slot and stencil box are released as
// soon as its wave ends, whatever the other waves' loads
#define STEP_BLOCK 64

template <bool SPH>
__global__ __launch_bounds__(STEP_BLOCK, 5) void k_step32(G32 g, Bg32P b, S32 src, S32 dst,
                                                          const uint32_t *__restrict__ perm,
                                                          uint32_t *__restrict__ key_out,
                                                          const DevCounters *__restrict__ dc, float dt,
                                                          const uint8_t *__restrict__ frozen,
                                                          const uint32_t *__restrict__ skeys)
{
    const int64_t i = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
    // stage the stencil box shared by the wave's volumes (all lanes take part:
    // the wave-wide reductions need every lane)
    const bool valid = i < dc->n_active;
    const uint32_t s = valid ? perm[i] : 0u;
    const uint32_t col = valid ? src.col[s] : 0xffffffffu;
    const int kc0 = valid ? src.lev[s] : 0;
    f32::WBox w;
    {
        const int lane = threadIdx.x & 63;
        const uint32_t c0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)col);
        const bool uni = __ballot(valid && col != c0) == 0ull && c0 != 0xffffffffu;
        const int kmn = wave_min_i(valid ? kc0 : 0x7fffffff), kmx = wave_max_i(valid ? kc0 : -1);
        w.base = 0;
        w.ic = (int)(c0 % (uint32_t)g.nx);
        w.jc = (int)(c0 / (uint32_t)g.nx);
        // levels: margins of two levels below and three above the wave's
        // range hold the faces of most volumes (a lookup outside the box
        // reads global memory)
        w.kbase = max(0, kmn - 2);
        w.L = min(g.nz - 1, kmx + 3) - w.kbase + 1;
        // one wrap corrects a column or row index when the grid has at least two
        w.on = uni && w.L <= WB_LMAX && g.nx >= 2 && (g.geometry != RT_CARTESIAN || g.ny >= 2);
        if (w.on) {
            // a lane issues all of its loads before its LDS writes; t / L as
            // (t * ceil(2^16 / L)) >> 16, exact for t < 512 and L <= 26
            constexpr int NA = (25 * WB_LMAX + 63) / 64, NG = (18 * WB_LMAX + 63) / 64;
            const int nA = 25 * w.L, nG = 18 * w.L, L9 = 9 * w.L;
            const uint32_t mL = (65536u + (uint32_t)w.L - 1u) / (uint32_t)w.L;
            float4 va[NA], vg[NG];
#pragma unroll
            for (int it = 0; it < NA; it++) {
                const int e = lane + 64 * it;
                if (e < nA) {
                    const int bxy = (int)(((uint32_t)e * mL) >> 16), kk = e - bxy * w.L;
                    int ii = w.ic + bxy % 5 - 2, jj = w.jc + bxy / 5 - 2;
                    ii += ii < 0 ? g.nx : 0;
                    ii -= ii >= g.nx ? g.nx : 0;
                    if (g.geometry == RT_CARTESIAN) {
                        jj += jj < 0 ? g.ny : 0;
                        jj -= jj >= g.ny ? g.ny : 0;
                    } else {
                        jj = min(max(jj, 0), g.ny - 1);
                    }
                    va[it] = f32::rec(b.A, f32::col_base(g, jj, ii) + (uint32_t)(w.kbase + kk));
                }
            }
#pragma unroll
            for (int it = 0; it < NG; it++) {
                const int e = lane + 64 * it;
                if (e < nG) {
                    const int r = e >= L9 ? 1 : 0, t = e - r * L9;
                    const int bxy = (int)(((uint32_t)t * mL) >> 16), kk = t - bxy * w.L;
                    int ii = w.ic + bxy % 3 - 1, jj = w.jc + bxy / 3 - 1;
                    ii += ii < 0 ? g.nx : 0;
                    ii -= ii >= g.nx ? g.nx : 0;
                    if (g.geometry == RT_CARTESIAN) {
                        jj += jj < 0 ? g.ny : 0;
                        jj -= jj >= g.ny ? g.ny : 0;
                    } else {
                        jj = min(max(jj, 0), g.ny - 1);
                    }
                    vg[it] = f32::rec(b.G, (f32::col_base(g, jj, ii) + (uint32_t)(w.kbase + kk)) * 2u + (uint32_t)r);
                }
            }
#pragma unroll
            for (int it = 0; it < NA; it++) {
                const int e = lane + 64 * it;
                if (e < nA) {
                    const int bxy = (int)(((uint32_t)e * mL) >> 16), kk = e - bxy * w.L;
                    f32::wb_lds[w.base + bxy * WB_LMAX + kk] = va[it];
                }
            }
#pragma unroll
            for (int it = 0; it < NG; it++) {
                const int e = lane + 64 * it;
                if (e < nG) {
                    const int r = e >= L9 ? 1 : 0, tt = e - r * L9;
                    const int bxy = (int)(((uint32_t)tt * mL) >> 16), kk = tt - bxy * w.L;
                    f32::wb_lds[w.base + WB_A + r * 9 * WB_LMAX + bxy * WB_LMAX + kk] = vg[it];
                }
            }
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
    int ic = (int)(col % (uint32_t)g.nx), jc = (int)(col / (uint32_t)g.nx);
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
        // a stage whose lookups all lie in the box, for every lane, runs the
        // box-only form; otherwise each lookup tests the box itself
        if (w.on && __ballot(!f32::box_stage_in(g, w, kc0, Y)) == 0ull)
            f32::rhs_box<SPH>(g, kc0, phi0, Y, F, w);
        else
            f32::rhs<SPH>(g, b, ic, jc, kc0, phi0, Y, F, w);
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
    const unsigned nb = (unsigned)((bound + STEP_BLOCK - 1) / STEP_BLOCK);
    const G32 h = f32::make_g32(g);
    const size_t lds = (size_t)WB_RECS * sizeof(float4);  // the wave's stencil box
    if (g.geometry == RT_SPHERICAL)
        k_step32<true><<<nb, STEP_BLOCK, lds, s>>>(h, b, src, dst, perm, key_out, dc, (float)dt, frozen, skeys);
    else
        k_step32<false><<<nb, STEP_BLOCK, lds, s>>>(h, b, src, dst, perm, key_out, dc, (float)dt, frozen, skeys);
}
