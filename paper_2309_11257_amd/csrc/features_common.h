// Per-column surrogate features, shared by both precisions.
//
// One wave per column (four columns per 256-thread workgroup), as in the
// deposition: the column's ray volumes (sorted order) are taken 64 at a time,
// one per lane; their sectors and moment terms go through the wave's LDS to
// the 48 lanes that own one (sector, moment) sum each, which add them in the
// sorted order, so the result does not depend on scheduling.  The profile
// part copies U, V, N2 of the column from the packed background.
// Per sector: sum W, sum |cg_z| k_h W, W-weighted means of log10 k_h,
// log10 |m| and z, W-weighted standard deviation of z.
#pragma once
#include "rt_internal.h"

// tan(pi/8): sector boundaries lie at 22.5 + 45 n degrees of the horizontal
// wavevector's azimuth; the test compares |l| with t|k| and |k| with t|l|
__device__ inline int azimuth_sector(double k, double l)
{
    const double t = 0.41421356237309503;
    const double ak = fabs(k), al = fabs(l);
    if (al <= t * ak) return k > 0.0 ? 0 : 4;
    if (ak <= t * al) return l > 0.0 ? 2 : 6;
    if (k > 0.0) return l > 0.0 ? 1 : 7;
    return l > 0.0 ? 3 : 5;
}

// P::spec(slot, k, l, m, W, cgz, z); P::profile(col, k) -> (U, V, N2)
template <class P>
__global__ __launch_bounds__(256) void k_features(Grid g, P pl, const uint32_t *__restrict__ perm,
                                                  const uint32_t *__restrict__ colstart, float *__restrict__ X)
{
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= g.ncol) return;  // whole wave
    const int nf = 3 * g.nz + 48;
    for (int k = lane; k < g.nz; k += 64) {
        double u, v, n2;
        pl.profile(c, k, u, v, n2);
        X[(int64_t)c * nf + k] = (float)u;
        X[(int64_t)c * nf + g.nz + k] = (float)v;
        X[(int64_t)c * nf + 2 * g.nz + k] = (float)n2;
    }
    // moments: per chunk of 64 volumes each lane forms one volume's sector and
    // six values in the wave's LDS, then lane 6 t + q (t < 8 sectors, q < 6
    // moments) adds moment q of sector t over the chunk's volumes in their
    // sorted order -- a fixed order, and one accumulator per lane
    __shared__ double fv[4][6][64];
    __shared__ int fsec[4][64];
    const int wave = threadIdx.x >> 6;
    const int my_t = lane / 6, my_q = lane - 6 * (lane / 6);
    double acc = 0.0;
    const uint32_t s0 = colstart[c], s1 = colstart[c + 1];
    for (uint32_t base = s0; base < s1; base += 64) {
        const uint32_t r = base + (uint32_t)lane;
        int sec = -1;
        double v[6] = {0, 0, 0, 0, 0, 0};
        if (r < s1) {
            double k, l, m, W, cgz, z;
            pl.spec(perm[r], k, l, m, W, cgz, z);
            const double kh = sqrt(k * k + l * l);
            v[0] = W;
            v[1] = (fabs(cgz) * kh) * W;
            v[2] = W * log10(kh);
            v[3] = W * log10(fabs(m));
            v[4] = W * z;
            v[5] = (W * z) * z;
            sec = azimuth_sector(k, l);
        }
#pragma unroll
        for (int q = 0; q < 6; q++) fv[wave][q][lane] = v[q];
        fsec[wave][lane] = sec;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int cnt = (int)min(64u, s1 - base);
        if (lane < 48)
            for (int j = 0; j < cnt; j++) acc += fsec[wave][j] == my_t ? fv[wave][my_q][j] : 0.0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    // lane s < 8 gathers sector s's six sums from lanes 6 s .. 6 s + 5
    double pq[6];
#pragma unroll
    for (int q = 0; q < 6; q++) pq[q] = __shfl(acc, min(6 * lane + q, 63), 64);
    if (lane < 8) {  // lane s writes sector s
        const double *p = pq;
        float o[6] = {(float)p[0], (float)p[1], 0.0f, 0.0f, 0.0f, 0.0f};
        if (p[0] > 0.0) {
            const double zm = p[4] / p[0];
            const double var = p[5] / p[0] - zm * zm;
            o[2] = (float)(p[2] / p[0]);
            o[3] = (float)(p[3] / p[0]);
            o[4] = (float)zm;
            o[5] = (float)(var > 0.0 ? sqrt(var) : 0.0);
        }
#pragma unroll
        for (int q = 0; q < 6; q++) X[(int64_t)c * nf + 3 * g.nz + 6 * lane + q] = o[q];
    }
}
