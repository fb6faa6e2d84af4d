// Per-column surrogate features, shared by both precisions.
//
// One 256-thread workgroup per column, as in the deposition: the column's ray
// volumes (sorted order) are dealt to the threads round-robin; each thread
// keeps its 8 sectors x 4 moments in registers (selected without indexing,
// so nothing spills), and the workgroup combines them in a fixed order
// (wave butterflies, then the four waves in turn), so the result does not
// depend on scheduling.  The profile part copies U, V, N2 of the column from
// the packed background.
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

// P::spec(slot, k, l, m, W, cgz); P::profile(col, k) -> (U, V, N2)
template <class P>
__global__ __launch_bounds__(256) void k_features(Grid g, P pl, const uint32_t *__restrict__ perm,
                                                  const uint32_t *__restrict__ colstart, float *__restrict__ X)
{
    __shared__ double part[4][32];
    const int c = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nf = 3 * g.nz + 32;
    for (int k = tid; k < g.nz; k += 256) {
        double u, v, n2;
        pl.profile(c, k, u, v, n2);
        X[(int64_t)c * nf + k] = (float)u;
        X[(int64_t)c * nf + g.nz + k] = (float)v;
        X[(int64_t)c * nf + 2 * g.nz + k] = (float)n2;
    }
    double acc[32];
#pragma unroll
    for (int q = 0; q < 32; q++) acc[q] = 0.0;
    const uint32_t s0 = colstart[c], s1 = colstart[c + 1];
    for (uint32_t r = s0 + (uint32_t)tid; r < s1; r += 256) {
        double k, l, m, W, cgz;
        pl.spec(perm[r], k, l, m, W, cgz);
        const double kh = sqrt(k * k + l * l);
        const double v0 = W, v1 = (fabs(cgz) * kh) * W, v2 = W * log10(kh), v3 = W * log10(fabs(m));
        const int sec = azimuth_sector(k, l);
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const bool hit = t == sec;
            acc[4 * t + 0] += hit ? v0 : 0.0;
            acc[4 * t + 1] += hit ? v1 : 0.0;
            acc[4 * t + 2] += hit ? v2 : 0.0;
            acc[4 * t + 3] += hit ? v3 : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < 32; q++) {
        double v = acc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) part[wave][q] = v;
    }
    __syncthreads();
    if (tid < 32) {
        const double tot = ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
        part[0][tid] = tot;  // each thread rewrites only its own entry after reading it
    }
    __syncthreads();
    if (tid < 32) {
        const int sec = tid >> 2, q = tid & 3;
        const double w = part[0][4 * sec];
        double out = part[0][tid];
        if (q >= 2) out = w > 0.0 ? out / w : 0.0;
        X[(int64_t)c * nf + 3 * g.nz + tid] = (float)out;
    }
}
