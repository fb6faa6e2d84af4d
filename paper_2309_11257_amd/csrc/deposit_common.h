// Per-column flux deposition shared by both precisions.
//
// Ray volumes arrive grouped by column (radix sort on the column key).  One
// 256-thread workgroup owns one column and walks its volumes in chunks of 256
// in sorted order.  Within a chunk every contribution is converted to an
// integer in a fixed-point format chosen from the chunk's largest
// contribution (2^52 units for that value) and added into an int64 profile in
// LDS; integer addition is associative, so the chunk total does not depend on
// the order in which lanes arrive.  Chunk totals are added to a double
// profile in chunk order.  The result is therefore bitwise reproducible from
// run to run, with no floating-point atomics, and each contribution is
// rounded once at the level of the chunk maximum's last bit -- the accuracy of
// an ordinary double sum.
#pragma once
#include "rt_internal.h"

// P::load(slot, zb, zt, bv[6]) fills the vertical span of the volume and its
// six flux densities per unit height: (cgx k, cgx l, cgy k, cgy l, cgz k,
// cgz l) * W / Dz.
template <class P>
__global__ __launch_bounds__(256) void k_deposit(Grid g, P pl, const uint32_t *__restrict__ perm,
                                                 const uint32_t *__restrict__ colstart, double *__restrict__ flux)
{
    extern __shared__ unsigned long long dep_smem[];
    const int nzp = g.nz + 1;
    unsigned long long *acc = dep_smem;          // [6][nzp]
    double *prof = (double *)(dep_smem + 6 * nzp);  // [6][nzp]
    __shared__ double wmax[4][6];
    __shared__ int sexp[6];
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < 6 * nzp; e += 256) {
        acc[e] = 0ull;
        prof[e] = 0.0;
    }
    const uint32_t s0 = colstart[c], s1 = colstart[c + 1];
    __syncthreads();
    for (uint32_t base = s0; base < s1; base += 256) {
        const uint32_t r = base + (uint32_t)tid;
        const bool valid = r < s1;
        double zb = 0.0, zt = 0.0, bv[6] = {0, 0, 0, 0, 0, 0};
        if (valid) pl.load(perm[r], zb, zt, bv);
        const double h = valid ? fmin(zt - zb, g.dz) : 0.0;
        double mv[6];
#pragma unroll
        for (int q = 0; q < 6; q++) mv[q] = fabs(bv[q]) * h;
#pragma unroll
        for (int q = 0; q < 6; q++)
            for (int off = 32; off > 0; off >>= 1) mv[q] = fmax(mv[q], __shfl_xor(mv[q], off, 64));
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < 6; q++) wmax[wave][q] = mv[q];
        __syncthreads();
        if (tid < 6) {
            double m = fmax(fmax(wmax[0][tid], wmax[1][tid]), fmax(wmax[2][tid], wmax[3][tid]));
            int e = 0;
            if (m > 0.0 && m < 1.0e300) {
                frexp(m, &e);
                sexp[tid] = 52 - e;
            } else {
                sexp[tid] = 0;
            }
        }
        __syncthreads();
        if (valid) {
            int sx[6];
#pragma unroll
            for (int q = 0; q < 6; q++) sx[q] = sexp[q];
            int klo = (int)floor(zb / g.dz), khi = (int)floor(zt / g.dz);
            if (klo < 0) klo = 0;
            if (khi > g.nz - 1) khi = g.nz - 1;
            for (int kk = klo; kk <= khi; kk++) {
                const double lo = (double)kk * g.dz, hi = (double)(kk + 1) * g.dz;
                const double o = fmin(zt, hi) - fmax(zb, lo);
                if (!(o > 0.0)) continue;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const long long v = llrint(ldexp(bv[q] * o, sx[q]));
                    if (v) atomicAdd(&acc[q * nzp + kk], (unsigned long long)v);
                }
            }
            klo = (int)floor(zb / g.dz + 0.5);
            khi = (int)floor(zt / g.dz + 0.5);
            if (klo < 0) klo = 0;
            if (khi > g.nz) khi = g.nz;
            for (int kk = klo; kk <= khi; kk++) {
                double lo = ((double)kk - 0.5) * g.dz, hi = ((double)kk + 0.5) * g.dz;
                if (lo < 0.0) lo = 0.0;
                if (hi > g.Lz) hi = g.Lz;
                const double o = fmin(zt, hi) - fmax(zb, lo);
                if (!(o > 0.0)) continue;
#pragma unroll
                for (int q = 4; q < 6; q++) {
                    const long long v = llrint(ldexp(bv[q] * o, sx[q]));
                    if (v) atomicAdd(&acc[q * nzp + kk], (unsigned long long)v);
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < 6 * nzp; e += 256) {
            const long long v = (long long)acc[e];
            if (v) {
                prof[e] += ldexp((double)v, -sexp[e / nzp]);
                acc[e] = 0ull;
            }
        }
        __syncthreads();
    }
    // divide by the cell volume (levels) or staggered-cell volume (interfaces)
    const int ci = c % g.nx, cj = c / g.nx;
    double area_h = g.dx * g.dy, cphi = 1.0;
    if (g.geometry == RT_SPHERICAL) cphi = cos(g.y0 + ((double)cj + 0.5) * g.dy);
    (void)ci;
    for (int e = tid; e < 6 * nzp; e += 256) {
        const int q = e / nzp, kk = e % nzp;
        double val;
        if (q < 4) {
            if (kk == g.nz) {
                val = 0.0;
            } else {
                double area = area_h;
                if (g.geometry == RT_SPHERICAL) {
                    const double rr = g.a + ((double)kk + 0.5) * g.dz;
                    area = (((rr * rr) * cphi) * g.dx) * g.dy;
                }
                val = prof[e] / (area * g.dz);
            }
        } else {
            double lo = ((double)kk - 0.5) * g.dz, hi = ((double)kk + 0.5) * g.dz;
            if (lo < 0.0) lo = 0.0;
            if (hi > g.Lz) hi = g.Lz;
            double area = area_h;
            if (g.geometry == RT_SPHERICAL) {
                const double rr = g.a + (double)kk * g.dz;
                area = (((rr * rr) * cphi) * g.dx) * g.dy;
            }
            val = prof[e] / (area * (hi - lo));
        }
        flux[((size_t)q * nzp + kk) * (size_t)g.ncol + c] = val;
    }
}

inline size_t deposit_smem(const Grid &g) { return (size_t)12 * (size_t)(g.nz + 1) * 8; }
