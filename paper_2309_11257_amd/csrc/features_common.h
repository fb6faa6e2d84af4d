// Per-column surrogate features, shared by both precisions.
//
// One wave per column (four columns per 256-thread workgroup), as in the
// deposition: the column's ray volumes (sorted order) are dealt to the lanes
// round-robin; each lane keeps its 8 sectors x 6 moments in registers
// (selected without indexing, so nothing spills), and the wave combines them
// by a fixed butterfly, so the result does not depend on scheduling.  The
// profile part copies U, V, N2 of the column from the packed background.
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
    double acc[48];
#pragma unroll
    for (int q = 0; q < 48; q++) acc[q] = 0.0;
    const uint32_t s0 = colstart[c], s1 = colstart[c + 1];
    for (uint32_t r = s0 + (uint32_t)lane; r < s1; r += 64) {
        double k, l, m, W, cgz, z;
        pl.spec(perm[r], k, l, m, W, cgz, z);
        const double kh = sqrt(k * k + l * l);
        const double v[6] = {W, (fabs(cgz) * kh) * W, W * log10(kh), W * log10(fabs(m)), W * z, (W * z) * z};
        const int sec = azimuth_sector(k, l);
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const bool hit = t == sec;
#pragma unroll
            for (int q = 0; q < 6; q++) acc[6 * t + q] += hit ? v[q] : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < 48; q++)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off, 64);
    if (lane < 8) {  // lane s writes sector s
        double p[6];
#pragma unroll
        for (int q = 0; q < 6; q++) {
            p[q] = acc[q];
#pragma unroll
            for (int t = 1; t < 8; t++) p[q] = lane == t ? acc[6 * t + q] : p[q];
        }
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
