// Per-column surrogate features, shared by both precisions.
//
// One 256-thread workgroup per column, as in the deposition: the column's ray
// volumes (sorted order) are dealt to the threads round-robin; each thread
// keeps its 8 sectors x 4 moments in registers (selected without indexing,
// so nothing spills), and the workgroup combines them in a fixed order
// (wave butterflies, then the four waves in turn), so the result does not
// depend on scheduling.  The profile part copies U, V, N2 of the column from
// the packed background.  Per sector: sum W, sum |cg_z| k_h W, W-weighted
// means of log10 k_h, log10 |m| and z, W-weighted standard deviation of z.
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
    __shared__ double part[4][48];
    const int c = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nf = 3 * g.nz + 48;
    for (int k = tid; k < g.nz; k += 256) {
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
    for (uint32_t r = s0 + (uint32_t)tid; r < s1; r += 256) {
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
    for (int q = 0; q < 48; q++) {
        double v = acc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) part[wave][q] = v;
    }
    __syncthreads();
    if (tid < 48) {
        const double tot = ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
        part[0][tid] = tot;  // each thread rewrites only its own entry after reading it
    }
    __syncthreads();
    if (tid < 8) {
        const double *p = &part[0][6 * tid];
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
        for (int q = 0; q < 6; q++) X[(int64_t)c * nf + 3 * g.nz + 6 * tid + q] = o[q];
    }
}
